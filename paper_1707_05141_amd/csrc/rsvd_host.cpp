// Host orchestration of batched_rsvd: randomized SVD (Section 7.1, Algorithm 4) with an adaptive
// range finder and an exact a-posteriori check, for a batch of instances of different shapes.
//
// Every stage is one launch per kernel configuration over all instances that take part in it
// (size-binned tiles, no per-instance launches). The data-dependent part -- how many sample blocks
// each instance needs -- is driven from the host: after each growth round and each check the
// per-instance decisions are read back (one synchronisation), and the next round's descriptors are
// built for the instances still growing.
//
// Per instance (all FP64, column-major, in the context's workspace):
//   Q   m x cap   orthonormal basis of the sampled range, grown block by block
//   Y   m x cap   current sample block Y = A Omega, then its projection
//   Om  n x bmax  Gaussian block, row-major
//   H   cap x 8   Q^T Y for the two classical Gram-Schmidt passes
//   Bt  n x cap   B^T = A^T Q
//   QB  n x cap, RB cap x cap  QR of B^T
//   UR, VR cap x cap, sig cap  SVD of R_B^T by one-sided Jacobi (rotating the rows of R_B)
// with cap = min(m, n, 64).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/bsvd.h"
#include "common.hpp"
#include "ctx.hpp"
#include "plan.hpp"
#include "rsvd.hpp"
#include "mlp.hpp"

using namespace bsvd;

namespace {

constexpr int CAPMAX = 64;
constexpr int GROW_BLK = 8;
constexpr double SAFETY = 2.0;

inline int nmax_for(int x) { return x <= 8 ? 8 : (x <= 16 ? 16 : (x <= 32 ? 32 : 64)); }
inline int cdiv(int a, int b) { return (a + b - 1) / b; }

struct Inst {
    int m, n, lda, cap, ell, ell0, maxr;
    size_t oQ, oY, oOm, oH, oBt, oQB, oRB, oUR, oVR, oSig, oXsq, oCsq, oBsq;
};

// Sequential packer of one round's descriptors into the pinned staging buffer; device addresses
// are those the block will have after upload_to(doff).
struct Packer {
    char *h;
    char *d;
    size_t cap;
    size_t off = 0;
    bool overflow = false;
    template <typename T>
    T *put(size_t count, T **dev) {
        off = (off + 255) & ~(size_t)255;
        const size_t bytes = sizeof(T) * (count ? count : 1);
        if (off + bytes > cap) {
            overflow = true;
            *dev = nullptr;
            return nullptr;
        }
        T *hp = reinterpret_cast<T *>(h + off);
        *dev = reinterpret_cast<T *>(d + off);
        off += bytes;
        return hp;
    }
};

struct MMGroup {
    std::vector<MMDesc> desc;
    std::vector<int> tiles_per;  // tiles of each descriptor
};

struct QLaunch {
    QKey key;
    const int *list;
    int count;
    double bytes, flops;
};

}  // namespace

// Probe features of every instance: Y = A Omega_p (PROBE_COLS Gaussian columns at counter column
// PROBE_COL0), R = qr(Y), features from diag(R). Omp (n x kp row-major), Y (m x kp) and R (kp x kp,
// ld ldr) are per-instance scratch given as device pointers. Enqueued on the context's stream.
struct ProbeBufs {
    double *Om, *Y, *R;
    int ldr;
};

static int probe_features(Ctx *c, int batch, const int *m, const int *n, const void *const *A, const int *lda,
                          const std::vector<ProbeBufs> &pb, unsigned long long seed, float *feats, size_t desc_cap) {
    Packer p;
    int rc = c->ensure_host(desc_cap);
    if (rc) return rc;
    p.h = static_cast<char *>(c->hws);
    p.d = static_cast<char *>(c->dws);
    p.cap = desc_cap;
    RngDesc *drd;
    RngDesc *hrd = p.put<RngDesc>(batch, &drd);
    FeatDesc *dfd;
    FeatDesc *hfd = p.put<FeatDesc>(batch, &dfd);
    if (!hrd || !hfd) return c->fail(BSVD_EHIP, "internal: descriptor region overflow");
    std::vector<int2> rt;
    std::map<int, MMGroup> sk;
    std::vector<QrDesc> qv;
    std::map<QKey, std::vector<int>> qbins;
    std::map<int, std::pair<double, double>> skcost;  // per NMAX: algorithmic bytes, flops
    for (int b = 0; b < batch; ++b) {
        const int kp = std::min(PROBE_COLS, std::min(m[b], n[b]));
        hrd[b] = RngDesc{pb[b].Om, n[b], kp, PROBE_COL0, kp, b, 0};
        for (int t = 0; t < cdiv(n[b] * kp, 256); ++t) rt.push_back(make_int2(b, t));
        MMDesc d;
        d.X = static_cast<const double *>(A[b]); d.Y = pb[b].Om; d.C = pb[b].Y; d.xsq = nullptr; d.csq = nullptr;
        d.alpha = 1.0; d.beta = 0.0; d.M = m[b]; d.N = kp; d.K = n[b]; d.ldx = lda[b]; d.ldy = kp; d.ldc = m[b];
        d.ytrans = 1;
        sk[nmax_for(kp)].desc.push_back(d);
        sk[nmax_for(kp)].tiles_per.push_back(cdiv(m[b], 64));
        QrDesc q;
        q.A = pb[b].Y; q.m = m[b]; q.n = kp; q.lda = m[b]; q.trans = 0; q.Q = nullptr; q.ldq = 0; q.R = pb[b].R;
        q.ldr = pb[b].ldr;
        qv.push_back(q);
        QKey k;
        if (!qr_config(m[b], kp, &k.nb, &k.seg, &k.kr)) return c->fail(BSVD_EUNSUP, "instance %d: probe QR", b);
        qbins[k].push_back(b);
        hfd[b] = FeatDesc{pb[b].R, pb[b].ldr, kp, m[b], n[b], b};
        skcost[nmax_for(kp)].first += 8.0 * ((double)m[b] * n[b] + (double)(m[b] + n[b]) * kp);
        skcost[nmax_for(kp)].second += 2.0 * (double)m[b] * n[b] * kp;
    }
    int2 *drt;
    int2 *hrt = p.put<int2>(rt.size(), &drt);
    if (hrt) std::copy(rt.begin(), rt.end(), hrt);
    QrDesc *dq;
    QrDesc *hq = p.put<QrDesc>(qv.size(), &dq);
    if (hq) std::copy(qv.begin(), qv.end(), hq);
    std::vector<QLaunch> ql;
    for (auto &kv : qbins) {
        int *dl;
        int *hl = p.put<int>(kv.second.size(), &dl);
        if (!hl) break;
        std::copy(kv.second.begin(), kv.second.end(), hl);
        double by = 0.0, fl = 0.0;
        for (int b : kv.second) {
            const double M = m[b], N = std::min(PROBE_COLS, std::min(m[b], n[b]));
            fl += 2.0 * M * N * N - 2.0 * N * N * N / 3.0;  // factorisation only, R kept
            by += 8.0 * (M * N + N * N);
        }
        ql.push_back(QLaunch{kv.first, dl, (int)kv.second.size(), by, fl});
    }
    std::vector<std::pair<MMDesc *, std::pair<int2 *, int>>> mm;
    std::vector<int> mmn;
    for (auto &kv : sk) {
        MMDesc *dd;
        MMDesc *hd = p.put<MMDesc>(kv.second.desc.size(), &dd);
        int nt = 0;
        for (int t : kv.second.tiles_per) nt += t;
        int2 *dt;
        int2 *ht = p.put<int2>(nt, &dt);
        if (!hd || !ht) break;
        int k = 0;
        for (size_t i = 0; i < kv.second.desc.size(); ++i) {
            hd[i] = kv.second.desc[i];
            for (int t = 0; t < kv.second.tiles_per[i]; ++t) ht[k++] = make_int2((int)i, t);
        }
        mm.push_back({dd, {dt, nt}});
        mmn.push_back(kv.first);
    }
    if (p.overflow) return c->fail(BSVD_EHIP, "internal: descriptor region overflow");
    if ((rc = c->upload_to(0, p.off))) return rc;
    int pi = c->prof_begin(BSVD_STAGE_RNG, "rng_kernel");
    hipError_t e = launch_rng(drd, drt, (int)rt.size(), seed, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "rng launch");
    c->prof_end(pi, 0.0, 0.0);
    for (size_t i = 0; i < mm.size(); ++i) {
        pi = c->prof ? c->prof_begin(BSVD_STAGE_SKETCH, kname_gemm(0, mmn[i]).c_str()) : -1;
        e = launch_gemm_nn(mmn[i], mm[i].first, mm[i].second.first, mm[i].second.second, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "probe sketch launch");
        c->prof_end(pi, skcost[mmn[i]].first, skcost[mmn[i]].second);
    }
    for (auto &L : ql) {
        pi = c->prof ? c->prof_begin(BSVD_STAGE_QR, kname_qr(0, L.key).c_str()) : -1;
        e = launch_qr(0, L.key.nb, L.key.seg, L.key.kr, dq, L.list, L.count, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "probe qr launch");
        c->prof_end(pi, L.bytes, L.flops);
    }
    pi = c->prof_begin(BSVD_STAGE_SMALL, "features_kernel");
    e = launch_features(dfd, batch, feats, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "features launch");
    c->prof_end(pi, 0.0, 0.0);
    return BSVD_OK;
}

extern "C" int bsvd_rank_features(bsvd_ctx *ctx, int batch, const int *m, const int *n, const void *const *A,
                                  const int *lda, unsigned long long seed, float *feats) {
    if (!ctx) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    if (batch < 0) return c->fail(BSVD_EARG, "batch = %d < 0", batch);
    if (batch == 0) return BSVD_OK;
    if (!m || !n || !A || !lda || !feats) return c->fail(BSVD_EARG, "m, n, A, lda and feats must be non-NULL");
    size_t dsz = 1u << 16;
    for (int b = 0; b < batch; ++b) {
        if (m[b] < 1 || n[b] < 1 || m[b] > 512 || n[b] > 512 || lda[b] < m[b] || !A[b])
            return c->fail(BSVD_EARG, "instance %d: bad shape / lda / pointer", b);
        dsz += 1024 + 8 * (size_t)cdiv(n[b] * PROBE_COLS, 256) + 16 * (size_t)cdiv(m[b], 64);
    }
    dsz = (dsz + 4095) & ~(size_t)4095;
    Arena ar;
    ar.off = dsz;
    std::vector<ProbeBufs> pb(batch);
    std::vector<size_t> o(3 * (size_t)batch);
    for (int b = 0; b < batch; ++b) {
        o[3 * b] = ar.alloc(8 * (size_t)n[b] * PROBE_COLS);
        o[3 * b + 1] = ar.alloc(8 * (size_t)m[b] * PROBE_COLS);
        o[3 * b + 2] = ar.alloc(8 * (size_t)PROBE_COLS * PROBE_COLS);
    }
    int rc = c->ensure_device(ar.off);
    if (rc) return rc;
    char *db = static_cast<char *>(c->dws);
    for (int b = 0; b < batch; ++b)
        pb[b] = ProbeBufs{reinterpret_cast<double *>(db + o[3 * b]), reinterpret_cast<double *>(db + o[3 * b + 1]),
                          reinterpret_cast<double *>(db + o[3 * b + 2]), PROBE_COLS};
    return probe_features(c, batch, m, n, A, lda, pb, seed, feats, dsz);
}

extern "C" int batched_rsvd(bsvd_ctx *ctx, int batch, const int *m, const int *n, const void *const *A,
                            const int *lda, const double *eps, const int *max_rank, void *const *S, void *const *U,
                            const int *ldu, void *const *V, const int *ldv, int *rank, double *err_est, int *info,
                            unsigned long long seed, unsigned flags, const int *ell0, int *samples) {
    if (!ctx) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    if (batch < 0) return c->fail(BSVD_EARG, "batch = %d < 0", batch);
    if (batch == 0) return BSVD_OK;
    if (!m || !n || !A || !lda || !max_rank || !S) return c->fail(BSVD_EARG, "m, n, A, lda, max_rank and S must be non-NULL");
    if (U && !ldu) return c->fail(BSVD_EARG, "U given without ldu");
    if (V && !ldv) return c->fail(BSVD_EARG, "V given without ldv");
    if ((flags & BSVD_RSVD_FIXED) && !ell0) return c->fail(BSVD_EARG, "BSVD_RSVD_FIXED needs ell0");
    if ((flags & BSVD_RSVD_LEARNED) && (ell0 || (flags & BSVD_RSVD_FIXED)))
        return c->fail(BSVD_EARG, "BSVD_RSVD_LEARNED chooses ell0 itself (pass ell0 = NULL, no FIXED)");
    if ((flags & BSVD_RSVD_LEARNED) && !c->model) return c->fail(BSVD_EARG, "BSVD_RSVD_LEARNED needs a rank model");
    if (flags & ~(unsigned)(BSVD_RSVD_FIXED | BSVD_RSVD_LEARNED | BSVD_RSVD_MIXED))
        return c->fail(BSVD_EUNSUP, "flags 0x%x not supported", flags);
    const bool learned = (flags & BSVD_RSVD_LEARNED) != 0;
    const bool mixed = (flags & BSVD_RSVD_MIXED) != 0;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");

    // ---- validation and workspace layout ---------------------------------------------------
    std::vector<Inst> I(batch);
    size_t dsz = 1u << 16;  // descriptor region bound
    for (int b = 0; b < batch; ++b) {
        if (m[b] < 1) return c->fail(BSVD_EARG, "instance %d: m = %d < 1", b, m[b]);
        if (n[b] < 1) return c->fail(BSVD_EARG, "instance %d: n = %d < 1", b, n[b]);
        if (m[b] > 512 || n[b] > 512)
            return c->fail(BSVD_EUNSUP, "instance %d: %d x %d exceeds the 512 x 512 limit", b, m[b], n[b]);
        if (lda[b] < m[b]) return c->fail(BSVD_EARG, "instance %d: lda = %d < m = %d", b, lda[b], m[b]);
        if (!A[b]) return c->fail(BSVD_EARG, "instance %d: A is NULL", b);
        if (!S[b]) return c->fail(BSVD_EARG, "instance %d: S is NULL", b);
        if (max_rank[b] < 1) return c->fail(BSVD_EARG, "instance %d: max_rank = %d < 1", b, max_rank[b]);
        if (U && U[b] && ldu[b] < m[b]) return c->fail(BSVD_EARG, "instance %d: ldu = %d < m = %d", b, ldu[b], m[b]);
        if (V && V[b] && ldv[b] < n[b]) return c->fail(BSVD_EARG, "instance %d: ldv = %d < n = %d", b, ldv[b], n[b]);
        if (eps && !(eps[b] > 0.0 && eps[b] < 1.0))
            return c->fail(BSVD_EARG, "instance %d: eps = %g not in (0, 1)", b, eps[b]);
        Inst &q = I[b];
        q.m = m[b];
        q.n = n[b];
        q.lda = lda[b];
        q.cap = std::min(std::min(m[b], n[b]), CAPMAX);
        q.ell = 0;
        q.ell0 = ell0 ? std::min(std::max(ell0[b], 0), q.cap) : 0;
        if ((flags & BSVD_RSVD_FIXED) && q.ell0 < 1) return c->fail(BSVD_EARG, "instance %d: ell0 < 1 with FIXED", b);
        q.maxr = max_rank[b];
        if (learned) q.ell0 = q.cap;  // the learned count is at most cap: size buffers for it
        const int bmax = std::max(std::max(GROW_BLK, q.ell0), PROBE_COLS);
        dsz += 4096 + 8 * (size_t)cdiv(q.n * bmax, 256) + 96 * (size_t)cdiv(q.m, 64) + 96 * (size_t)cdiv(q.n, 64);
    }
    dsz = (dsz + 4095) & ~(size_t)4095;
    Arena ar;
    ar.off = dsz;
    const size_t oState = ar.alloc(sizeof(RsvdState) * (size_t)batch);
    const size_t oJinfo = ar.alloc(sizeof(int) * (size_t)batch);
    const size_t oJsweeps = ar.alloc(sizeof(int) * (size_t)batch);
    const size_t oFlags = ar.alloc(sizeof(int) * (size_t)batch);
    const size_t oRankc = ar.alloc(sizeof(int) * (size_t)batch);
    const size_t oFeat = ar.alloc(sizeof(float) * MLP_IN * (size_t)batch);
    const size_t oPred = ar.alloc(sizeof(float) * (size_t)batch);
    const size_t oCap = ar.alloc(sizeof(int) * (size_t)batch);
    for (int b = 0; b < batch; ++b) {
        Inst &q = I[b];
        const size_t M = q.m, N = q.n, C = q.cap;
        const size_t bmax = std::max(std::max(GROW_BLK, q.ell0), PROBE_COLS);
        q.oQ = ar.alloc(8 * M * C);
        q.oY = ar.alloc(8 * M * C);
        q.oOm = ar.alloc(8 * N * bmax);
        q.oH = ar.alloc(8 * C * GROW_BLK);
        q.oBt = ar.alloc(8 * N * C);
        q.oQB = ar.alloc(8 * N * C);
        q.oRB = ar.alloc(8 * C * C);
        q.oUR = ar.alloc(8 * C * C);
        q.oVR = ar.alloc(8 * C * C);
        q.oSig = ar.alloc(8 * C);
        q.oXsq = ar.alloc(8 * (size_t)cdiv(q.m, 64));
        q.oCsq = ar.alloc(8 * (size_t)cdiv(q.m, 64));
        q.oBsq = ar.alloc(8 * (size_t)cdiv(q.n, 64));
    }
    int rc = c->ensure_device(ar.off);
    if (rc) return rc;
    rc = c->ensure_host(std::max(dsz, sizeof(RsvdState) * (size_t)batch));
    if (rc) return rc;
    rc = c->ensure_readback(2 * sizeof(int) * (size_t)batch);
    if (rc) return rc;
    char *db = static_cast<char *>(c->dws);
    RsvdState *dstate = reinterpret_cast<RsvdState *>(db + oState);
    int *djinfo = reinterpret_cast<int *>(db + oJinfo);
    int *djsweeps = reinterpret_cast<int *>(db + oJsweeps);
    int *dflags = reinterpret_cast<int *>(db + oFlags);
    int *drankc = reinterpret_cast<int *>(db + oRankc);
    const int *rb = static_cast<const int *>(c->rb);

    {
        RsvdState *hs = static_cast<RsvdState *>(c->hws);
        for (int b = 0; b < batch; ++b) {
            const Inst &q = I[b];
            RsvdState &s = hs[b];
            std::memset(&s, 0, sizeof s);
            s.A = static_cast<const double *>(A[b]);
            s.xsq = reinterpret_cast<double *>(db + q.oXsq);
            s.csq = reinterpret_cast<double *>(db + q.oCsq);
            s.bsq = reinterpret_cast<double *>(db + q.oBsq);
            s.sig = reinterpret_cast<double *>(db + q.oSig);
            s.Sout = static_cast<double *>(S[b]);
            s.eps = eps ? eps[b] : 1e-6;
            s.safety = SAFETY;
            s.m = q.m;
            s.n = q.n;
            s.lda = q.lda;
            s.cap = q.cap;
            s.max_rank = q.maxr;
            s.ntile_m = cdiv(q.m, 64);
            s.ntile_n = cdiv(q.n, 64);
        }
        rc = c->upload_to(oState, sizeof(RsvdState) * (size_t)batch);
        if (rc) return rc;
    }
    auto dptr = [&](size_t off) { return reinterpret_cast<double *>(db + off); };
    auto new_packer = [&](Packer &p) -> int {
        int r = c->ensure_host(dsz);
        if (r) return r;
        p.h = static_cast<char *>(c->hws);
        p.d = db;
        p.cap = dsz;
        p.off = 0;
        p.overflow = false;
        return BSVD_OK;
    };
    auto commit = [&](Packer &p) -> int {
        if (p.overflow) return c->fail(BSVD_EHIP, "internal: descriptor region overflow");
        return c->upload_to(0, p.off);
    };
    auto readback = [&](int count) -> int {
        if (count <= 0) return BSVD_OK;
        hipError_t ee = hipMemcpyAsync(c->rb, dflags, sizeof(int) * (size_t)count, hipMemcpyDeviceToHost, c->stream);
        if (ee != hipSuccess) return c->hip_fail(ee, "hipMemcpyAsync(flags)");
        ee = hipStreamSynchronize(c->stream);
        if (ee != hipSuccess) return c->hip_fail(ee, "hipStreamSynchronize");
        return BSVD_OK;
    };
    // Pack a set of GEMM descriptors grouped by NMAX together with their tile lists and launch them.
    struct Pending {
        int nmax;
        int tn;  // 0 nn, 1 tn, 2 nn with FP32 arithmetic
        MMDesc *d;
        int2 *tiles;
        int ntiles;
        double bytes, flops;  // algorithmic: operands read once, result written once
    };
    auto pack_mm = [&](Packer &p, std::map<int, MMGroup> &groups, int tn, std::vector<Pending> &out) {
        for (auto &kv : groups) {
            MMGroup &g = kv.second;
            if (g.desc.empty()) continue;
            MMDesc *dd;
            MMDesc *hd = p.put<MMDesc>(g.desc.size(), &dd);
            int nt = 0;
            for (int t : g.tiles_per) nt += t;
            int2 *dt;
            int2 *ht = p.put<int2>((size_t)nt, &dt);
            if (!hd || !ht) return;
            int k = 0;
            double by = 0.0, fl = 0.0;
            for (size_t i = 0; i < g.desc.size(); ++i) {
                const MMDesc &md = g.desc[i];
                hd[i] = md;
                for (int t = 0; t < g.tiles_per[i]; ++t) ht[k++] = make_int2((int)i, t);
                const double M = md.M, N = md.N, K = md.K;
                fl += 2.0 * M * N * K;
                if (tn == 1)  // C (K x N) = X^T Y
                    by += 8.0 * (M * K + M * N + K * N);
                else  // C (M x N) = alpha X Y + beta C; the FP32 variant reads Y as FP32
                    by += 8.0 * M * K + (tn == 2 ? 4.0 : 8.0) * K * N + 8.0 * M * N * (md.beta != 0.0 ? 2.0 : 1.0);
            }
            out.push_back(Pending{kv.first, tn, dd, dt, nt, by, fl});
        }
    };
    auto launch_mm = [&](const std::vector<Pending> &v, int stage) -> int {
        for (const Pending &pd : v) {
            const int pi = c->prof ? c->prof_begin(stage, kname_gemm(pd.tn, pd.nmax).c_str()) : -1;
            hipError_t ee = pd.tn == 1   ? launch_gemm_tn(pd.nmax, pd.d, pd.tiles, pd.ntiles, c->stream)
                            : pd.tn == 2 ? launch_gemm_nn_f32(pd.nmax, pd.d, pd.tiles, pd.ntiles, c->stream)
                                         : launch_gemm_nn(pd.nmax, pd.d, pd.tiles, pd.ntiles, c->stream);
            if (ee != hipSuccess) return c->hip_fail(ee, "gemm launch");
            c->prof_end(pi, pd.bytes, pd.flops);
        }
        return BSVD_OK;
    };
    auto mm_nn = [&](const double *X, int ldx, const double *Y, int ldy, int ytrans, double *C, int ldc, int M,
                     int N, int K, double alpha, double beta, double *xsq, double *csq) {
        MMDesc d;
        d.X = X; d.Y = Y; d.C = C; d.xsq = xsq; d.csq = csq; d.alpha = alpha; d.beta = beta;
        d.M = M; d.N = N; d.K = K; d.ldx = ldx; d.ldy = ldy; d.ldc = ldc; d.ytrans = ytrans;
        return d;
    };
    // QR launches grouped by kernel configuration, with their algorithmic cost: Householder
    // factorisation and formation of the thin Q (2 (2 m n^2 - 2 n^3 / 3) flops); A read, Q written,
    // R written when asked for
    auto pack_qr = [&](Packer &p, const std::vector<QrDesc> &qv, std::vector<QLaunch> &out, QrDesc **dq) -> int {
        std::map<QKey, std::vector<int>> bins;
        for (size_t i = 0; i < qv.size(); ++i) {
            QKey k;
            if (!qr_config(qv[i].m, qv[i].n, &k.nb, &k.seg, &k.kr)) return BSVD_EUNSUP;
            bins[k].push_back((int)i);
        }
        QrDesc *hq = p.put<QrDesc>(qv.size(), dq);
        if (!hq) return BSVD_OK;
        for (size_t i = 0; i < qv.size(); ++i) hq[i] = qv[i];
        for (auto &kv : bins) {
            int *dl;
            int *hl = p.put<int>(kv.second.size(), &dl);
            if (!hl) return BSVD_OK;
            double by = 0.0, fl = 0.0;
            for (size_t i = 0; i < kv.second.size(); ++i) {
                hl[i] = kv.second[i];
                const QrDesc &q = qv[kv.second[i]];
                const double M = q.m, N = q.n;
                fl += 2.0 * (2.0 * M * N * N - 2.0 * N * N * N / 3.0);
                by += 8.0 * (M * N + (q.Q ? M * N : 0.0) + (q.R ? N * N : 0.0));
            }
            out.push_back(QLaunch{kv.first, dl, (int)kv.second.size(), by, fl});
        }
        return BSVD_OK;
    };
    auto launch_qrs = [&](QrDesc *dq, const std::vector<QLaunch> &v) -> int {
        for (auto &L : v) {
            const int pi = c->prof ? c->prof_begin(BSVD_STAGE_QR, kname_qr(0, L.key).c_str()) : -1;
            hipError_t ee = launch_qr(0, L.key.nb, L.key.seg, L.key.kr, dq, L.list, L.count, c->stream);
            if (ee != hipSuccess) return c->hip_fail(ee, "qr launch");
            c->prof_end(pi, L.bytes, L.flops);
        }
        return BSVD_OK;
    };

    // ---- learned initial sample count: probe features -> network -> ell0 ----------------------
    if (learned) {
        std::vector<ProbeBufs> pb(batch);
        for (int b = 0; b < batch; ++b) pb[b] = ProbeBufs{dptr(I[b].oOm), dptr(I[b].oY), dptr(I[b].oRB), I[b].cap};
        float *dfeat = reinterpret_cast<float *>(db + oFeat);
        float *dpred = reinterpret_cast<float *>(db + oPred);
        int *dcap = reinterpret_cast<int *>(db + oCap);
        if ((rc = probe_features(c, batch, m, n, A, lda, pb, seed, dfeat, dsz))) return rc;
        if ((rc = c->ensure_host(dsz))) return rc;
        int *hc = static_cast<int *>(c->hws);
        for (int b = 0; b < batch; ++b) hc[b] = I[b].cap;
        if ((rc = c->upload_to(oCap, sizeof(int) * (size_t)batch))) return rc;
        int pi = c->prof_begin(BSVD_STAGE_SMALL);  // forward network + ell0: two launches
        e = launch_mlp_forward(static_cast<const float *>(c->model), batch, dfeat, dpred, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "mlp forward launch");
        e = launch_ell0(dpred, dcap, batch, c->rank_margin, dflags, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "ell0 launch");
        c->prof_end(pi, 0.0, 0.0);
        if ((rc = readback(batch))) return rc;
        for (int b = 0; b < batch; ++b) I[b].ell0 = rb[b];
    }

    // ---- phase A: initial block of ell0 samples (Algorithm 4 as printed) -------------------
    std::vector<int> grow, pend_check, finished;
    {
        std::vector<int> init;
        for (int b = 0; b < batch; ++b) (I[b].ell0 > 0 ? init : grow).push_back(b);
        if (!init.empty()) {
            Packer p;
            if ((rc = new_packer(p))) return rc;
            RngDesc *drd;
            RngDesc *hrd = p.put<RngDesc>(init.size(), &drd);
            std::vector<int2> rt;
            std::map<int, MMGroup> sk;
            std::vector<QrDesc> qv;
            GrowItem *dgi;
            GrowItem *hgi = p.put<GrowItem>(init.size(), &dgi);
            if (!hrd || !hgi) return commit(p);
            for (size_t i = 0; i < init.size(); ++i) {
                const int b = init[i];
                Inst &q = I[b];
                hrd[i] = RngDesc{dptr(q.oOm), q.n, q.ell0, 0, q.ell0, b, mixed ? 1 : 0};
                for (int t = 0; t < cdiv(q.n * q.ell0, 256); ++t) rt.push_back(make_int2((int)i, t));
                MMGroup &g = sk[nmax_for(q.ell0)];
                g.desc.push_back(mm_nn(static_cast<const double *>(A[b]), q.lda, dptr(q.oOm), q.ell0, 1, dptr(q.oY),
                                       q.m, q.m, q.ell0, q.n, 1.0, 0.0, dptr(q.oXsq), nullptr));
                g.tiles_per.push_back(cdiv(q.m, 64));
                QrDesc qd;
                qd.A = dptr(q.oY); qd.m = q.m; qd.n = q.ell0; qd.lda = q.m; qd.trans = 0;
                qd.Q = dptr(q.oQ); qd.ldq = q.m; qd.R = nullptr; qd.ldr = 0;
                qv.push_back(qd);
                hgi[i] = GrowItem{b, q.ell0, 1, 0};
                q.ell = q.ell0;
            }
            double rgb = 0;
            for (int b : init) rgb += (mixed ? 4.0 : 8.0) * I[b].n * (double)I[b].ell0;
            int2 *drt;
            int2 *hrt = p.put<int2>(rt.size(), &drt);
            if (hrt) std::copy(rt.begin(), rt.end(), hrt);
            std::vector<Pending> mm;
            pack_mm(p, sk, mixed ? 2 : 0, mm);
            QrDesc *dq;
            std::vector<QLaunch> ql;
            if ((rc = pack_qr(p, qv, ql, &dq))) return c->fail(rc, "internal: no QR kernel for the initial block");
            if ((rc = commit(p))) return rc;
            int pi = c->prof_begin(BSVD_STAGE_RNG, "rng_kernel");
            e = launch_rng(drd, drt, (int)rt.size(), seed, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "rng launch");
            c->prof_end(pi, rgb, 0.0);
            if ((rc = launch_mm(mm, BSVD_STAGE_SKETCH))) return rc;
            if ((rc = launch_qrs(dq, ql))) return rc;
            pi = c->prof_begin(BSVD_STAGE_SMALL, "init_norm_kernel");
            e = launch_init_norm(dstate, dgi, (int)init.size(), c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "init launch");
            c->prof_end(pi, 0.0, 0.0);
            pend_check = init;
        }
    }

    // ---- phases B/C: growth rounds and exact checks ----------------------------------------
    while (!grow.empty() || !pend_check.empty()) {
        if (!grow.empty()) {
            Packer p;
            if ((rc = new_packer(p))) return rc;
            const int G = (int)grow.size();
            RngDesc *drd;
            RngDesc *hrd = p.put<RngDesc>(G, &drd);
            GrowItem *dgi;
            GrowItem *hgi = p.put<GrowItem>(G, &dgi);
            if (!hrd || !hgi) return commit(p);
            std::vector<int2> rt;
            std::map<int, MMGroup> sk, tn1, nn1, tn2, nn2;
            std::vector<QrDesc> qv;
            double rgb = 0;
            for (int i = 0; i < G; ++i) {
                const int b = grow[i];
                Inst &q = I[b];
                const int blk = std::min(GROW_BLK, q.cap - q.ell);
                const int first = q.ell == 0;
                rgb += (mixed ? 4.0 : 8.0) * q.n * (double)blk;
                hrd[i] = RngDesc{dptr(q.oOm), q.n, blk, q.ell, blk, b, mixed ? 1 : 0};
                for (int t = 0; t < cdiv(q.n * blk, 256); ++t) rt.push_back(make_int2(i, t));
                MMGroup &g = sk[8];
                g.desc.push_back(mm_nn(static_cast<const double *>(A[b]), q.lda, dptr(q.oOm), blk, 1, dptr(q.oY), q.m,
                                       q.m, blk, q.n, 1.0, 0.0, first ? dptr(q.oXsq) : nullptr,
                                       first ? dptr(q.oCsq) : nullptr));
                g.tiles_per.push_back(cdiv(q.m, 64));
                if (!first) {
                    // two classical Gram-Schmidt passes: H = Q^T Y, Y -= Q H
                    for (int pass = 0; pass < 2; ++pass) {
                        MMGroup &gt = (pass ? tn2 : tn1)[8];
                        gt.desc.push_back(mm_nn(dptr(q.oQ), q.m, dptr(q.oY), q.m, 0, dptr(q.oH), q.cap, q.m, blk, q.ell,
                                                1.0, 0.0, nullptr, nullptr));
                        gt.tiles_per.push_back(1);
                        MMGroup &gn = (pass ? nn2 : nn1)[8];
                        gn.desc.push_back(mm_nn(dptr(q.oQ), q.m, dptr(q.oH), q.cap, 0, dptr(q.oY), q.m, q.m, blk, q.ell,
                                                -1.0, 1.0, nullptr, pass ? dptr(q.oCsq) : nullptr));
                        gn.tiles_per.push_back(cdiv(q.m, 64));
                    }
                }
                QrDesc qd;
                qd.A = dptr(q.oY); qd.m = q.m; qd.n = blk; qd.lda = q.m; qd.trans = 0;
                qd.Q = dptr(q.oQ) + (size_t)q.ell * q.m; qd.ldq = q.m; qd.R = nullptr; qd.ldr = 0;
                qv.push_back(qd);
                hgi[i] = GrowItem{b, blk, first, 0};
                q.ell += blk;
            }
            int2 *drt;
            int2 *hrt = p.put<int2>(rt.size(), &drt);
            if (hrt) std::copy(rt.begin(), rt.end(), hrt);
            std::vector<Pending> msk, mt1, mn1, mt2, mn2;
            pack_mm(p, sk, mixed ? 2 : 0, msk);
            pack_mm(p, tn1, 1, mt1);
            pack_mm(p, nn1, 0, mn1);
            pack_mm(p, tn2, 1, mt2);
            pack_mm(p, nn2, 0, mn2);
            QrDesc *dq;
            std::vector<QLaunch> ql;
            if ((rc = pack_qr(p, qv, ql, &dq))) return c->fail(rc, "internal: no QR kernel for a sample block");
            if ((rc = commit(p))) return rc;
            int pi = c->prof_begin(BSVD_STAGE_RNG, "rng_kernel");
            e = launch_rng(drd, drt, (int)rt.size(), seed, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "rng launch");
            c->prof_end(pi, rgb, 0.0);
            if ((rc = launch_mm(msk, BSVD_STAGE_SKETCH))) return rc;
            if ((rc = launch_mm(mt1, BSVD_STAGE_CGS)) || (rc = launch_mm(mn1, BSVD_STAGE_CGS)) ||
                (rc = launch_mm(mt2, BSVD_STAGE_CGS)) || (rc = launch_mm(mn2, BSVD_STAGE_CGS)))
                return rc;
            if ((rc = launch_qrs(dq, ql))) return rc;
            pi = c->prof_begin(BSVD_STAGE_SMALL, "grow_decide_kernel");
            e = launch_grow_decide(dstate, dgi, G, dflags, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "decide launch");
            c->prof_end(pi, 0.0, 0.0);
            if ((rc = readback(G))) return rc;
            std::vector<int> still;
            for (int i = 0; i < G; ++i) (rb[i] ? pend_check : still).push_back(grow[i]);
            grow.swap(still);
        }
        if (!pend_check.empty()) {
            Packer p;
            if ((rc = new_packer(p))) return rc;
            const int P = (int)pend_check.size();
            std::map<int, MMGroup> bt;
            for (int i = 0; i < P; ++i) {
                const int b = pend_check[i];
                const Inst &q = I[b];
                MMGroup &g = bt[nmax_for(q.ell)];
                g.desc.push_back(mm_nn(static_cast<const double *>(A[b]), q.lda, dptr(q.oQ), q.m, 0, dptr(q.oBt), q.n,
                                       q.m, q.ell, q.n, 1.0, 0.0, nullptr, dptr(q.oBsq)));
                g.tiles_per.push_back(cdiv(q.n, 64));
            }
            int *dl;
            int *hl = p.put<int>(P, &dl);
            if (!hl) return commit(p);
            std::copy(pend_check.begin(), pend_check.end(), hl);
            std::vector<Pending> mb;
            pack_mm(p, bt, 1, mb);
            if ((rc = commit(p))) return rc;
            if ((rc = launch_mm(mb, BSVD_STAGE_PROJECT))) return rc;
            int pi = c->prof_begin(BSVD_STAGE_SMALL, "check_kernel");
            e = launch_check(dstate, dl, P, dflags, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "check launch");
            c->prof_end(pi, 0.0, 0.0);
            if ((rc = readback(P))) return rc;
            for (int i = 0; i < P; ++i) {
                const int b = pend_check[i];
                if (rb[i] || I[b].ell >= I[b].cap || (flags & BSVD_RSVD_FIXED))
                    finished.push_back(b);
                else
                    grow.push_back(b);
            }
            pend_check.clear();
        }
    }

    // ---- phase D: QR(B^T), Jacobi SVD of R_B^T, truncation -----------------------------------
    std::sort(finished.begin(), finished.end());
    const int F = (int)finished.size();
    {
        Packer p;
        if ((rc = new_packer(p))) return rc;
        std::vector<QrDesc> qv;
        std::map<JKey, std::vector<int>> jb;
        SvdDesc *dsd;
        SvdDesc *hsd = p.put<SvdDesc>(F, &dsd);
        int *dl;
        int *hl = p.put<int>(F, &dl);
        if (!hsd || !hl) return commit(p);
        for (int i = 0; i < F; ++i) {
            const int b = finished[i];
            const Inst &q = I[b];
            QrDesc qd;
            qd.A = dptr(q.oBt); qd.m = q.n; qd.n = q.ell; qd.lda = q.n; qd.trans = 0;
            qd.Q = dptr(q.oQB); qd.ldq = q.n; qd.R = dptr(q.oRB); qd.ldr = q.cap;
            qv.push_back(qd);
            // SVD of R_B^T: rotate the rows of R_B; the kernel sends the normalised columns of the
            // working matrix R_B^T (= U_R) to .V and the accumulated rotations (= V_R) to .U.
            SvdDesc &d = hsd[i];
            d.A = dptr(q.oRB); d.m = q.ell; d.n = q.ell; d.lda = q.cap; d.trans = 1; d.M = q.ell; d.N = q.ell;
            d.S = dptr(q.oSig); d.U = dptr(q.oVR); d.ldu = q.cap; d.V = dptr(q.oUR); d.ldv = q.cap;
            JKey k;
            if (choose_jacobi(0, q.ell, q.ell, 0, &k)) return c->fail(BSVD_EUNSUP, "internal: no Jacobi kernel");
            jb[k].push_back(i);
            hl[i] = b;
        }
        // Jacobi lists index the descriptor array (position i), finalize lists index instances
        std::vector<std::pair<JKey, std::pair<const int *, int>>> jl;
        for (auto &kv : jb) {
            int *djl;
            int *hjl = p.put<int>(kv.second.size(), &djl);
            if (!hjl) return commit(p);
            std::copy(kv.second.begin(), kv.second.end(), hjl);
            jl.push_back({kv.first, {djl, (int)kv.second.size()}});
        }
        QrDesc *dq;
        std::vector<QLaunch> ql;
        if ((rc = pack_qr(p, qv, ql, &dq))) return c->fail(rc, "internal: no QR kernel for B^T");
        if ((rc = commit(p))) return rc;
        // Jacobi: R_B read, U_R and V_R written, sigma written
        std::map<JKey, double> jbytes;
        for (auto &kv : jb)
            for (int i : kv.second) {
                const double l = I[finished[i]].ell;
                jbytes[kv.first] += 8.0 * (3.0 * l * l + l);
            }
        if ((rc = launch_qrs(dq, ql))) return rc;
        int pi;
        // profiled runs also read back the sweeps, to give each Jacobi record its flop count
        std::vector<std::pair<int, const std::vector<int> *>> jrec;
        for (auto &L : jl) {
            // info and sweeps per descriptor position -> djinfo[position], djsweeps[position]
            pi = c->prof ? c->prof_begin(BSVD_STAGE_JACOBI, kname_jacobi(0, L.first).c_str()) : -1;
            if (L.first.kind == JK_WAVE)
                e = launch_jacobi_wave(0, L.first.a, L.first.b, dsd, L.second.first, L.second.second, 1e-15, 60,
                                       djsweeps, djinfo, c->stream);
            else
                e = launch_jacobi_lds(0, L.first.a, L.first.b, dsd, L.second.first, L.second.second, 1e-15, 60,
                                      djsweeps, djinfo, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "jacobi launch");
            c->prof_end(pi, jbytes[L.first], 0.0);
            if (pi >= 0) jrec.push_back({pi, &jb[L.first]});
        }
        pi = c->prof_begin(BSVD_STAGE_SMALL, "finalize_kernel");
        e = launch_finalize(dstate, dl, F, rank, err_est, info, djinfo, drankc, samples, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "finalize launch");
        c->prof_end(pi, 0.0, 0.0);
        e = hipMemcpyAsync(c->rb, drankc, sizeof(int) * (size_t)F, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync(rank)");
        if (!jrec.empty()) {
            e = hipMemcpyAsync(static_cast<int *>(c->rb) + F, djsweeps, sizeof(int) * (size_t)F, hipMemcpyDeviceToHost,
                               c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync(sweeps)");
        }
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "hipStreamSynchronize");
        for (auto &jr : jrec) {
            double fl = 0.0;
            for (int i : *jr.second) fl += jacobi_flops(I[finished[i]].ell, I[finished[i]].ell, rb[F + i]);
            c->recs[jr.first].flops = fl;
        }
    }
    // ---- back-transform U = Q U_R[:, :k], V = Q_B V_R[:, :k] ---------------------------------
    {
        std::vector<int> kk(F);
        for (int i = 0; i < F; ++i) kk[i] = rb[i];
        Packer p;
        if ((rc = new_packer(p))) return rc;
        std::map<int, MMGroup> out;
        for (int i = 0; i < F; ++i) {
            const int b = finished[i];
            const Inst &q = I[b];
            const int k = kk[i];
            if (k <= 0) continue;
            MMGroup &g = out[nmax_for(k)];
            if (U && U[b]) {
                g.desc.push_back(mm_nn(dptr(q.oQ), q.m, dptr(q.oUR), q.cap, 0, static_cast<double *>(U[b]), ldu[b], q.m,
                                       k, q.ell, 1.0, 0.0, nullptr, nullptr));
                g.tiles_per.push_back(cdiv(q.m, 64));
            }
            if (V && V[b]) {
                g.desc.push_back(mm_nn(dptr(q.oQB), q.n, dptr(q.oVR), q.cap, 0, static_cast<double *>(V[b]), ldv[b], q.n,
                                       k, q.ell, 1.0, 0.0, nullptr, nullptr));
                g.tiles_per.push_back(cdiv(q.n, 64));
            }
        }
        std::vector<Pending> mo;
        pack_mm(p, out, 0, mo);
        if ((rc = commit(p))) return rc;
        if ((rc = launch_mm(mo, BSVD_STAGE_OUTPUT))) return rc;
    }
    return BSVD_OK;
}

extern "C" int bsvd_sample_omega(bsvd_ctx *ctx, unsigned long long seed, int inst, int n, int col0, int b, double *out) {
    if (!ctx) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    if (n < 0 || b < 0 || col0 < 0 || inst < 0) return c->fail(BSVD_EARG, "negative size or index");
    if (n == 0 || b == 0) return BSVD_OK;
    if (!out) return c->fail(BSVD_EARG, "out is NULL");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return c->hip_fail(e, "hipSetDevice");
    const int nt = cdiv(n * b, 256);
    Arena up;
    const size_t od = up.alloc(sizeof(RngDesc));
    const size_t ot = up.alloc(sizeof(int2) * (size_t)nt);
    int rc = c->ensure_device(up.off);
    if (rc) return rc;
    rc = c->ensure_host(up.off);
    if (rc) return rc;
    char *hb = static_cast<char *>(c->hws);
    *reinterpret_cast<RngDesc *>(hb + od) = RngDesc{out, n, b, col0, b, inst, 0};
    int2 *ht = reinterpret_cast<int2 *>(hb + ot);
    for (int t = 0; t < nt; ++t) ht[t] = make_int2(0, t);
    if ((rc = c->upload(up.off))) return rc;
    char *db = static_cast<char *>(c->dws);
    e = launch_rng(reinterpret_cast<RngDesc *>(db + od), reinterpret_cast<int2 *>(db + ot), nt, seed, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "rng launch");
    return BSVD_OK;
}
