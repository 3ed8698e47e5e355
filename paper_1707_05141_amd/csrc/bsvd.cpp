// Host side of the C ABI: context, workspace, argument validation, planning and dispatch.
#include "../../include/bsvd.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "common.hpp"
#include "ctx.hpp"

using namespace bsvd;

namespace bsvd {

int Ctx::fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
}

int Ctx::hip_fail(hipError_t e, const char *what) {
    return fail(BSVD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int Ctx::ensure_device(size_t bytes) {
    if (bytes <= dws_size) return BSVD_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (dws) hipFree(dws);
    dws = nullptr;
    dws_size = 0;
    size_t want = bytes + bytes / 4 + (1u << 20);
    e = hipMalloc(&dws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(BSVD_ENOMEM, "device workspace of %zu bytes: %s", want, hipGetErrorString(e));
    }
    dws_size = want;
    return BSVD_OK;
}

int Ctx::ensure_host(size_t bytes) {
    hipError_t e;
    if (staged_pending) {
        e = hipEventSynchronize(staged);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        staged_pending = false;
    }
    if (bytes <= hws_size) return BSVD_OK;
    if (hws) hipHostFree(hws);
    hws = nullptr;
    hws_size = 0;
    size_t want = bytes + bytes / 4 + (1u << 16);
    e = hipHostMalloc(&hws, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(BSVD_ENOMEM, "pinned staging of %zu bytes: %s", want, hipGetErrorString(e));
    }
    hws_size = want;
    return BSVD_OK;
}

int Ctx::upload(size_t bytes) {
    if (bytes == 0) return BSVD_OK;
    hipError_t e = hipMemcpyAsync(dws, hws, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(descriptors)");
    e = hipEventRecord(staged, stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    staged_pending = true;
    return BSVD_OK;
}

}  // namespace bsvd

extern "C" {

const char *bsvd_version(void) { return "bsvd 0.1 (gfx950)"; }

int bsvd_create(bsvd_ctx **out, int device, void *stream) {
    if (!out) return BSVD_EARG;
    *out = nullptr;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return BSVD_EHIP;
    Ctx *c = new Ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete c;
        return BSVD_EHIP;
    }
    *out = reinterpret_cast<bsvd_ctx *>(c);
    return BSVD_OK;
}

void bsvd_destroy(bsvd_ctx *ctx) {
    if (!ctx) return;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    if (c->dws) hipFree(c->dws);
    if (c->hws) hipHostFree(c->hws);
    hipEventDestroy(c->staged);
    delete c;
}

const char *bsvd_last_error(const bsvd_ctx *ctx) {
    if (!ctx) return "null context";
    return reinterpret_cast<const Ctx *>(ctx)->err.c_str();
}

int bsvd_sync(bsvd_ctx *ctx) {
    if (!ctx) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "hipStreamSynchronize");
    return BSVD_OK;
}

int batched_svd(bsvd_ctx *ctx, int dtype, int batch, const int *m, const int *n, const void *const *A,
                const int *lda, void *const *S, void *const *U, const int *ldu, void *const *V, const int *ldv,
                double tol, int max_sweeps, int *sweeps, int *info, unsigned flags) {
    if (!ctx) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    if (dtype != BSVD_F64 && dtype != BSVD_F32) return c->fail(BSVD_EARG, "dtype %d is not BSVD_F64/BSVD_F32", dtype);
    if (batch < 0) return c->fail(BSVD_EARG, "batch = %d < 0", batch);
    if (batch == 0) return BSVD_OK;
    if (!m || !n || !A || !lda || !S) return c->fail(BSVD_EARG, "m, n, A, lda and S must be non-NULL");
    if (U && !ldu) return c->fail(BSVD_EARG, "U given without ldu");
    if (V && !ldv) return c->fail(BSVD_EARG, "V given without ldv");
    if (tol <= 0.0) tol = (dtype == BSVD_F64) ? 1e-15 : 1e-6;
    if (max_sweeps <= 0) max_sweeps = 60;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");

    // Validate and plan: group instances by kernel configuration.
    std::map<std::pair<int, int>, std::vector<int>> bins;
    for (int b = 0; b < batch; ++b) {
        if (m[b] < 1) return c->fail(BSVD_EARG, "instance %d: m = %d < 1", b, m[b]);
        if (n[b] < 1) return c->fail(BSVD_EARG, "instance %d: n = %d < 1", b, n[b]);
        if (lda[b] < m[b]) return c->fail(BSVD_EARG, "instance %d: lda = %d < m = %d", b, lda[b], m[b]);
        if (!A[b]) return c->fail(BSVD_EARG, "instance %d: A is NULL", b);
        if (!S[b]) return c->fail(BSVD_EARG, "instance %d: S is NULL", b);
        if (U && U[b] && ldu[b] < m[b]) return c->fail(BSVD_EARG, "instance %d: ldu = %d < m = %d", b, ldu[b], m[b]);
        if (V && V[b] && ldv[b] < n[b]) return c->fail(BSVD_EARG, "instance %d: ldv = %d < n = %d", b, ldv[b], n[b]);
        const int M = m[b] >= n[b] ? m[b] : n[b];
        const int N = m[b] >= n[b] ? n[b] : m[b];
        int mmax = 0, np = 0;
        if (flags & (BSVD_SVD_FORCE_LDS | BSVD_SVD_FORCE_BLOCK | BSVD_SVD_QR_FIRST))
            return c->fail(BSVD_EUNSUP, "instance %d: requested kernel path is not available", b);
        if (!jacobi_wave_supported(dtype, M, N, &mmax, &np))
            return c->fail(BSVD_EUNSUP, "instance %d: %d x %d has no Jacobi kernel", b, m[b], n[b]);
        bins[{mmax, np}].push_back(b);
    }

    const size_t desc_bytes = sizeof(SvdDesc) * (size_t)batch;
    const size_t list_off = (desc_bytes + 255) & ~(size_t)255;
    const size_t total = list_off + sizeof(int) * (size_t)batch;
    int rc = c->ensure_device(total);
    if (rc) return rc;
    rc = c->ensure_host(total);
    if (rc) return rc;

    SvdDesc *hd = reinterpret_cast<SvdDesc *>(c->hws);
    for (int b = 0; b < batch; ++b) {
        SvdDesc &d = hd[b];
        d.A = A[b];
        d.S = S[b];
        d.U = U ? U[b] : nullptr;
        d.V = V ? V[b] : nullptr;
        d.m = m[b];
        d.n = n[b];
        d.lda = lda[b];
        d.ldu = (U && U[b]) ? ldu[b] : 0;
        d.ldv = (V && V[b]) ? ldv[b] : 0;
        d.trans = m[b] < n[b] ? 1 : 0;
        d.M = d.trans ? n[b] : m[b];
        d.N = d.trans ? m[b] : n[b];
    }
    int *hl = reinterpret_cast<int *>(static_cast<char *>(c->hws) + list_off);
    std::vector<std::pair<std::pair<int, int>, std::pair<int, int>>> launches;  // key -> (offset, count)
    int off = 0;
    for (auto &kv : bins) {
        launches.push_back({kv.first, {off, (int)kv.second.size()}});
        for (int b : kv.second) hl[off++] = b;
    }
    rc = c->upload(total);
    if (rc) return rc;

    const SvdDesc *dd = reinterpret_cast<const SvdDesc *>(c->dws);
    const int *dl = reinterpret_cast<const int *>(static_cast<char *>(c->dws) + list_off);
    for (auto &L : launches) {
        e = launch_jacobi_wave(dtype, L.first.first, L.first.second, dd, dl + L.second.first, L.second.second, tol,
                               max_sweeps, sweeps, info, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "jacobi_wave launch");
    }
    return BSVD_OK;
}

}  // extern "C"
