// Rank-prediction network: 16 -> 64 -> 64 -> 1, ReLU hidden layers, FP32, MSE loss, Adam.
//
// Parameter vector (5313 floats): W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3 (output-major).
//   mlp_forward_kernel    one thread per sample; the weights are staged in LDS (21 KB)
//   mlp_backward_kernel   one thread per sample: forward, then the per-sample deltas of both hidden
//                         layers and of the output, written to a scratch buffer
//   mlp_grad_kernel       one thread per parameter: the mini-batch gradient as a sum over samples in
//                         sample order (deterministic, no atomics)
//   mlp_adam_kernel       one thread per parameter (Kingma & Ba, ICLR 2015)
//   features_kernel       the 16 probe features of a block from the R factor of its probe sketch

#include "common.hpp"
#include "mlp.hpp"
#include "dpp.hpp"

namespace bsvd {

constexpr int IN = MLP_IN, H = MLP_H;
constexpr int OW1 = 0, OB1 = H * IN, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;

__device__ __forceinline__ void mlp_fwd(const float *p, const float *x, float *a1, float *a2, float &y) {
#pragma unroll 4
    for (int o = 0; o < H; ++o) {
        float s = p[OB1 + o];
#pragma unroll
        for (int i = 0; i < IN; ++i) s = fmaf(p[OW1 + o * IN + i], x[i], s);
        a1[o] = s;
    }
#pragma unroll 4
    for (int o = 0; o < H; ++o) {
        float s = p[OB2 + o];
        for (int i = 0; i < H; ++i) s = fmaf(p[OW2 + o * H + i], fmaxf(a1[i], 0.0f), s);
        a2[o] = s;
    }
    float s = p[OB3];
    for (int i = 0; i < H; ++i) s = fmaf(p[OW3 + i], fmaxf(a2[i], 0.0f), s);
    y = s;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ params, int n,
                                                          const float *__restrict__ X, float *__restrict__ y) {
    __shared__ float p[MLP_NPARAM];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += 256) p[i] = params[i];
    __syncthreads();
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float x[IN], a1[H], a2[H], out;
#pragma unroll
    for (int i = 0; i < IN; ++i) x[i] = X[(size_t)s * IN + i];
    mlp_fwd(p, x, a1, a2, out);
    y[s] = out;
}

// Per-sample backward of L = (1/N) sum (f - t)^2: writes dy (1), delta2 (64), delta1 (64), and the
// post-ReLU activations h1 (64), h2 (64) of the sample into scratch[s][257]; loss terms into lt[s].
__global__ __launch_bounds__(256) void mlp_backward_kernel(const float *__restrict__ params, int n, float inv_n,
                                                           const float *__restrict__ X, const float *__restrict__ T,
                                                           const int *__restrict__ idx, float *__restrict__ scratch,
                                                           float *__restrict__ lt) {
    __shared__ float p[MLP_NPARAM];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += 256) p[i] = params[i];
    __syncthreads();
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int src = idx ? idx[s] : s;
    float x[IN], a1[H], a2[H], out;
#pragma unroll
    for (int i = 0; i < IN; ++i) x[i] = X[(size_t)src * IN + i];
    mlp_fwd(p, x, a1, a2, out);
    const float r = out - T[src];
    lt[s] = r * r;
    const float dy = 2.0f * r * inv_n;
    float *sc = scratch + (size_t)s * MLP_SCRATCH;
    sc[0] = dy;
    float d2[H];
    for (int i = 0; i < H; ++i) {
        d2[i] = a2[i] > 0.0f ? dy * p[OW3 + i] : 0.0f;
        sc[1 + i] = d2[i];
        sc[1 + 3 * H + i] = fmaxf(a2[i], 0.0f);
    }
    for (int i = 0; i < H; ++i) {
        float d = 0.0f;
        for (int o = 0; o < H; ++o) d = fmaf(p[OW2 + o * H + i], d2[o], d);
        sc[1 + H + i] = a1[i] > 0.0f ? d : 0.0f;
        sc[1 + 2 * H + i] = fmaxf(a1[i], 0.0f);
    }
}

// grad[param] = sum over samples (in order) of that sample's contribution.
__global__ __launch_bounds__(256) void mlp_grad_kernel(int n, const float *__restrict__ X, const int *__restrict__ idx,
                                                       const float *__restrict__ scratch, float *__restrict__ grad) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= MLP_NPARAM) return;
    float g = 0.0f;
    if (q < OB1) {  // W1[o][i] += delta1[o] x[i]
        const int o = q / IN, i = q - (q / IN) * IN;
        for (int s = 0; s < n; ++s) {
            const int src = idx ? idx[s] : s;
            g = fmaf(scratch[(size_t)s * MLP_SCRATCH + 1 + H + o], X[(size_t)src * IN + i], g);
        }
    } else if (q < OW2) {  // b1[o] += delta1[o]
        const int o = q - OB1;
        for (int s = 0; s < n; ++s) g += scratch[(size_t)s * MLP_SCRATCH + 1 + H + o];
    } else if (q < OB2) {  // W2[o][i] += delta2[o] h1[i]
        const int o = (q - OW2) / H, i = (q - OW2) - ((q - OW2) / H) * H;
        for (int s = 0; s < n; ++s) {
            const float *sc = scratch + (size_t)s * MLP_SCRATCH;
            g = fmaf(sc[1 + o], sc[1 + 2 * H + i], g);
        }
    } else if (q < OW3) {  // b2[o] += delta2[o]
        const int o = q - OB2;
        for (int s = 0; s < n; ++s) g += scratch[(size_t)s * MLP_SCRATCH + 1 + o];
    } else if (q < OB3) {  // W3[i] += dy h2[i]
        const int i = q - OW3;
        for (int s = 0; s < n; ++s) {
            const float *sc = scratch + (size_t)s * MLP_SCRATCH;
            g = fmaf(sc[0], sc[1 + 3 * H + i], g);
        }
    } else {  // b3 += dy
        for (int s = 0; s < n; ++s) g += scratch[(size_t)s * MLP_SCRATCH];
    }
    grad[q] = g;
}

__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ p, float *__restrict__ m1,
                                                       float *__restrict__ m2, const float *__restrict__ g, float lr,
                                                       float b1, float b2, float eps, float bc1, float bc2) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= MLP_NPARAM) return;
    const float gq = g[q];
    const float a = b1 * m1[q] + (1.0f - b1) * gq;
    const float b = b2 * m2[q] + (1.0f - b2) * gq * gq;
    m1[q] = a;
    m2[q] = b;
    p[q] -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
}

// Sum of the per-sample loss terms in fixed order (single workgroup).
__global__ __launch_bounds__(256) void mlp_loss_kernel(int n, const float *__restrict__ lt, float *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += (double)lt[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(red[0] / (double)n);
}

// Probe features of block b from the k x k upper triangle R of its probe sketch (ld ldr):
//   f0 = log2(m) / 9, f1 = log2(n) / 9,
//   f(1 + i) = max(log10(|R_ii| / |R_00|), -20) / 16 for i = 1 .. 13 (-20/16 where i >= k or R_00 = 0),
//   f15 = log2(k ||A||_F^2 / s1^2) / 8 with s1 = ||R v|| after 64 power steps on R^T R from
//         v = (1, ..., 1) / sqrt(k) (0 if ||A||_F or s1 is 0): the stable rank of A seen through the
//         probe, which keeps growing where the 16 diagonal entries no longer resolve a slow decay.
// Sixteen lanes per block (four blocks per wave): lane i keeps row i and column i of R in registers,
// so each power step is two triangular products whose other operand (v, then w = R v) comes from
// the group's lanes by shuffles, and the norm is a DPP group sum. The products run over j in
// ascending order as in the plain loops (zero entries outside the triangle add nothing).
__global__ __launch_bounds__(64) void features_kernel(const FeatDesc *__restrict__ d, int count,
                                                      float *__restrict__ feats) {
    constexpr int K = PROBE_COLS;
    static_assert(K == 16, "one DPP row of lanes per block");
    const int lane = threadIdx.x;
    const int grp = lane >> 4, i = lane & 15, base = lane & ~15;
    const int b = blockIdx.x * 4 + grp;
    const bool act = b < count;
    FeatDesc D{};
    if (act) D = d[b];
    const int k = act ? D.k : 0;
    double rrow[K], rcol[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        rrow[j] = (i < k && j >= i && j < k) ? D.R[i + (size_t)j * D.ldr] : 0.0;
        rcol[j] = (i < k && j <= i) ? D.R[j + (size_t)i * D.ldr] : 0.0;
    }
    double v = (i < k) ? 1.0 / sqrt((double)k) : 0.0;
    for (int it = 0; it < 64 && k > 0; ++it) {
        double w = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) w += rrow[j] * __shfl(v, base + j, 64);
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) s += rcol[j] * __shfl(w, base + j, 64);
        const double nz = sqrt(group_sum<16>(s * s));
        if (!(nz > 0.0)) break;  // the same in every lane of the group
        v = s / nz;
    }
    double w = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) w += rrow[j] * __shfl(v, base + j, 64);
    const double s1 = group_sum<16>(w * w);
    if (!act) return;
    float *f = feats + (size_t)D.out * MLP_IN;
    if (i == 0) {
        f[0] = (float)(log2((double)D.m) / 9.0);
        f[1] = (float)(log2((double)D.n) / 9.0);
        double a2 = 0.0;
        for (int t = 0; t < D.ntile; ++t) a2 += D.xsq[2 * t] + D.xsq[2 * t + 1];
        f[MLP_IN - 1] = (a2 > 0.0 && s1 > 0.0) ? (float)(log2((double)k * a2 / s1) / 8.0) : 0.0f;
    } else if (i < MLP_IN - 2) {
        double val = -20.0;
        const double r0 = fabs(D.R[0]);
        if (i < k && r0 > 0.0) {
            const double ri = fabs(D.R[i + (size_t)i * D.ldr]);
            val = ri > 0.0 ? fmax(log10(ri / r0), -20.0) : -20.0;
        }
        f[1 + i] = (float)(val / 16.0);
    }
}

__global__ void mlp_init_kernel(float *__restrict__ p, unsigned long long seed) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= MLP_NPARAM) return;
    // He-uniform weights (bound sqrt(6 / fan_in)), zero biases; uniform from a 32-bit hash of (seed, q)
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(q + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const float u = ((float)(z >> 40) + 0.5f) * (1.0f / 16777216.0f) * 2.0f - 1.0f;
    float bound = 0.0f;
    if (q < OB1) bound = sqrtf(6.0f / IN);
    else if (q >= OW2 && q < OB2) bound = sqrtf(6.0f / H);
    else if (q >= OW3 && q < OB3) bound = sqrtf(6.0f / H);
    p[q] = bound * u;
}

// ---------------------------------------------------------------------------------------------
static inline int nb256(int n) { return (n + 255) / 256; }

hipError_t launch_mlp_forward(const float *params, int n, const float *X, float *y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(nb256(n)), dim3(256), 0, st, params, n, X, y);
    return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float *params, int n, const float *X, const float *T, const int *idx,
                                float *scratch, float *lt, float *grad, float *loss, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(nb256(n)), dim3(256), 0, st, params, n, 1.0f / (float)n, X, T, idx,
                       scratch, lt);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nb256(MLP_NPARAM)), dim3(256), 0, st, n, X, idx, scratch, grad);
    if (loss) hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, st, n, lt, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *p, float *m1, float *m2, const float *g, float lr, int step, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.0f - powf(b1, (float)step), bc2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3(nb256(MLP_NPARAM)), dim3(256), 0, st, p, m1, m2, g, lr, b1, b2, 1e-8f,
                       bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float *p, unsigned long long seed, hipStream_t st) {
    hipLaunchKernelGGL(mlp_init_kernel, dim3(nb256(MLP_NPARAM)), dim3(256), 0, st, p, seed);
    return hipGetLastError();
}

hipError_t launch_features(const FeatDesc *d, int count, float *feats, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(features_kernel, dim3((count + 3) / 4), dim3(64), 0, st, d, count, feats);
    return hipGetLastError();
}

}  // namespace bsvd
