"""The allocation-free network forward (abcsmc_mlp_forward_noalloc, for
callers that cannot allocate device memory) against the allocating entry
point abcsmc_mlp_forward: bit-identical outputs on two calls in a row, the
second with fewer rows and another network (so nothing of the first call's
bfloat16 copy may survive), nothing written past n, and argument errors
reported before any work is enqueued."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _params(seed):
    from oracle import mlp_ref as M
    p = M.init(seed).copy()
    rng = np.random.default_rng(seed)
    for b in ("b1", "b2", "b3", "b4"):
        a0, a1 = M.offsets()[b]
        p[a0:a1] = rng.normal(0, 0.1, a1 - a0).astype(np.float32)
    return p


def test_noalloc_forward_matches_allocating_forward():
    import torch
    from oracle import mlp_ref as M
    from paper_2106_15508_amd import abcsmc as A

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    for call, (n, seed) in enumerate(((5000, 21), (300, 22))):
        print(f"noalloc forward call {call}: n={n} seed={seed}", flush=True)
        p = _params(seed)
        x = np.random.default_rng(100 + seed).uniform(-1, 1, (n, 8)).astype(np.float32)
        P = torch.from_numpy(p).to(dev)
        X = torch.from_numpy(x).to(dev)
        O = torch.full((n + 64, 3), float("nan"), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        A.mlp_forward_noalloc(P.data_ptr(), n, X.data_ptr(), O.data_ptr(), stream.cuda_stream)
        torch.cuda.synchronize()
        got = O.cpu().numpy()
        want = A.mlp_forward(p, x)
        assert np.array_equal(got[:n].view(np.uint32), want.view(np.uint32)), call
        assert np.all(np.isnan(got[n:])), call
        # the same bar as the allocating forward against the bf16-emulating oracle
        if n <= 300:
            emu, _ = M.forward_bf16(p, x)
            scale = max(1.0, float(np.max(np.abs(emu))))
            assert np.max(np.abs(got[:n] - emu)) <= 2e-3 * scale


def test_noalloc_forward_rejects_bad_arguments():
    import torch
    from paper_2106_15508_amd import abcsmc as A

    dev = torch.device("cuda:0")
    P = torch.zeros(A.mlp_param_count(), dtype=torch.float32, device=dev)
    X = torch.zeros((8, 8), dtype=torch.float32, device=dev)
    O = torch.zeros((8, 3), dtype=torch.float32, device=dev)
    for n in (0, -1, 65537):
        with pytest.raises(A.AbcsmcError) as e:
            A.mlp_forward_noalloc(P.data_ptr(), n, X.data_ptr(), O.data_ptr(), 0)
        assert e.value.code == A.EINVAL and "65536" in str(e.value)
    with pytest.raises(A.AbcsmcError) as e:
        A.mlp_forward_noalloc(0, 8, X.data_ptr(), O.data_ptr(), 0)
    assert e.value.code == A.EINVAL
    torch.cuda.synchronize()
