// predict.h -- arguments of the posterior predictive simulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace abcsmc {

// Stream round of the predictive simulations (the observations use 0xFFFF).
constexpr uint32_t kPredictRound = 0xFFFE;

struct PredictArgs {
    Model m;                 // T = prediction horizon
    const double* u;         // n x 8 unit-cube particles
    int64_t n;
    uint32_t round;          // stream round of the predictive simulations
    double* series;          // (T + 1) x 3 x n
    const double* quant;     // n_quant levels in [0, 1]
    int32_t n_quant;
    double* bands;           // (T + 1) x 3 x n_quant
};

void launch_predict(const PredictArgs& a, hipStream_t s);

}  // namespace abcsmc
