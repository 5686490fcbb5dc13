"""MI355X-native P-ABC-SMC with Beta-distributed step sizes (arXiv 2106.15508).

The compute path is the HIP library ``libabcsmc_hip.so`` (built from
``csrc/``) behind the C ABI declared in ``include/abcsmc.h``.  Import
``paper_2106_15508_amd.abcsmc`` for the binding; ``workloads`` holds the
synthetic workload definitions and loads nothing native.
"""

__all__ = ["abcsmc", "workloads"]
