// Internal launch interface of the learned CTU time predictor kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "trs.h"

namespace trs {

constexpr int kMlpIn = TRS_MLP_IN, kMlpHid = TRS_MLP_HIDDEN;

hipError_t launch_mlp_inputs(int W, int H, int cs, int w, int h, const uint32_t *tex,
                             const uint32_t *var, const uint32_t *mean, const uint32_t *prev,
                             float *x, hipStream_t s);
hipError_t launch_mlp_forward(const trs_mlp &m, const trs_mlp_norm &nm, const float *x, long long n,
                              float *y, float *z1, float *z2, hipStream_t s);
long long mlp_chunk(long long n);
size_t mlp_backward_workspace(long long n);
hipError_t launch_mlp_backward(const trs_mlp &m, const trs_mlp_norm &nm, const float *x,
                               const float *z1, const float *z2, const float *dy, long long n,
                               const trs_mlp_grads &g, char *ws, hipStream_t s);
hipError_t launch_mlp_cost(long long n, const float *y, const float *x, const trs_mlp_norm &nm,
                           const uint32_t *tex, const uint32_t *prev, trs_blend b, uint32_t *cost,
                           uint32_t *n_fallback, hipStream_t s);

}  // namespace trs
