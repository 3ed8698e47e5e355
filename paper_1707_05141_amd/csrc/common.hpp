// Internal declarations shared by the host dispatcher and the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsvd {

// Per-instance descriptor of a batched_svd call, uploaded to the device workspace.
// The working matrix is A (trans = 0) or A^T (trans = 1) so that it is M x N with M >= N.
struct SvdDesc {
    const void *A;
    void *S;
    void *U;
    void *V;
    int m, n, lda, ldu, ldv;
    int trans;
    int M, N;
};

// Per-instance info codes (see bsvd.h).
enum { INFO_OK = 0, INFO_SWEEPS = 1, INFO_RANKCAP = 2, INFO_NONFINITE = 3 };

// Launchers (defined in the .hip files).
hipError_t launch_jacobi_wave(int dtype, int mmax, int np, const SvdDesc *d, const int *list, int count,
                              double tol, int max_sweeps, int *sweeps, int *info, hipStream_t st);
bool jacobi_wave_supported(int dtype, int M, int N, int *mmax, int *np);

}  // namespace bsvd
