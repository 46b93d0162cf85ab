// Launchers of the learned-indicator kernels (implemented in ccz4_mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ccz4_layout.hpp"

namespace ccz4 {

constexpr int MLP_NIN = 81, MLP_NH = 64, MLP_NOUT = 3, MLP_NPARAM = 9603;
// floats per row of the optional gradient trace: x (81), a1 (64), a2 (64), d3 (3), d2 (64), d1 (64)
constexpr int MLP_TRACE = MLP_NIN + 4 * MLP_NH + MLP_NOUT;

int32_t mlp_tiles(int64_t n);
// the library's own gradient partials (ccz4_mlp_grad_noalloc): room for this many 64-row tiles
constexpr int MLP_SCRATCH_TILES = 64;
// device address of the partials array on the current device (taken once per device)
hipError_t mlp_scratch(float **out);
hipError_t launch_features(const double *Q, const double *HM, const PatchGeom *geom, int32_t npatch, float *feat,
                           hipStream_t st);
hipError_t launch_mlp_forward(const float *prm, const float *norm, const float *feat, int64_t n, float *logits,
                              hipStream_t st);
hipError_t launch_mlp_grad(const float *prm, const float *norm, const float *feat, const int8_t *tags, int64_t n,
                           float *work, float *trace, float *grad, float *loss, hipStream_t st);
hipError_t launch_mlp_adam(float *prm, float *m, float *v, const float *grad, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t st);
hipError_t launch_tag_learned(const float *logits, const int8_t *plain, const PatchGeom *geom, const int32_t *sib,
                              int32_t npatch, float conf, int32_t max_level, int8_t *pre, int8_t *tags,
                              hipStream_t st);

}  // namespace ccz4
