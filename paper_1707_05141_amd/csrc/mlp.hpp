// Rank-prediction network: sizes, descriptors and launchers.
#pragma once

#include <hip/hip_runtime.h>

namespace bsvd {

constexpr int MLP_IN = 16;
constexpr int MLP_H = 64;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;  // 5313
constexpr int MLP_SCRATCH = 1 + 4 * MLP_H;  // per-sample backward scratch (floats)
constexpr int PROBE_COLS = 16;              // columns of the probe sketch
constexpr int PROBE_COL0 = 1 << 20;         // counter column of its first sample

// Features of one block from the R factor of its probe sketch.
struct FeatDesc {
    const double *R;
    const double *xsq;  // ||A||_F^2 as (hi, lo) pairs over ntile row tiles
    int ldr, k, m, n, out, ntile;
};

hipError_t launch_mlp_forward(const float *params, int n, const float *X, float *y, hipStream_t st);
hipError_t launch_mlp_loss_grad(const float *params, int n, const float *X, const float *T, const int *idx,
                                float *scratch, float *lt, float *grad, float *loss, hipStream_t st);
hipError_t launch_mlp_adam(float *p, float *m1, float *m2, const float *g, float lr, int step, hipStream_t st);
hipError_t launch_mlp_init(float *p, unsigned long long seed, hipStream_t st);
hipError_t launch_features(const FeatDesc *d, int count, float *feats, hipStream_t st);

}  // namespace bsvd
