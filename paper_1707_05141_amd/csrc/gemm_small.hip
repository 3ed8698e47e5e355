// Batched small GEMM C = A B (column-major, A M x K, B K x N, K, N <= 64) for back-transforms such
// as U = Q U_R (Section 6.2) and U = Q U_R, V = Q_B V_R (Section 7.1, Algorithm 4).
//
// One 256-thread workgroup per instance: B is staged in LDS, each thread produces rows r, r + 256,
// ... of C for all N columns in register chunks of 16 columns. Reads of A are coalesced along the
// rows of each column.

#include "common.hpp"

namespace bsvd {

template <typename T, int KMAX>
__global__ __launch_bounds__(256) void gemm_small_kernel(const GemmDesc *__restrict__ descs, const int *__restrict__ list) {
    __shared__ T sB[KMAX * 64];
    const GemmDesc D = descs[list[blockIdx.x]];
    const int t = threadIdx.x;
    const int M = D.M, N = D.N, K = D.K;
    const T *A = static_cast<const T *>(D.A);
    const T *B = static_cast<const T *>(D.B);
    T *C = static_cast<T *>(D.C);
    for (int idx = t; idx < K * N; idx += 256) {
        const int c = idx / K, k = idx - c * K;
        sB[k + c * KMAX] = B[k + (size_t)c * D.ldb];
    }
    __syncthreads();
    for (int r = t; r < M; r += 256) {
        for (int c0 = 0; c0 < N; c0 += 16) {
            T acc[16];
#pragma unroll
            for (int cc = 0; cc < 16; ++cc) acc[cc] = T(0);
            for (int k = 0; k < K; ++k) {
                const T a = A[r + (size_t)k * D.lda];
#pragma unroll
                for (int cc = 0; cc < 16; ++cc) acc[cc] = fma(a, sB[k + (c0 + cc) * KMAX], acc[cc]);
            }
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
                if (c0 + cc < N) C[r + (size_t)(c0 + cc) * D.ldc] = acc[cc];
        }
    }
}

hipError_t launch_gemm_small(int dtype, const GemmDesc *d, const int *list, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    if (dtype == 0)
        hipLaunchKernelGGL((gemm_small_kernel<double, 64>), dim3(count), dim3(256), 0, st, d, list);
    else
        hipLaunchKernelGGL((gemm_small_kernel<float, 64>), dim3(count), dim3(256), 0, st, d, list);
    return hipGetLastError();
}

}  // namespace bsvd
