// Host side of the rank-prediction network: parameters, Adam state and training loop.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <algorithm>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "../../include/bsvd.h"
#include "ctx.hpp"
#include "mlp.hpp"

using namespace bsvd;

namespace bsvd {

int Ctx::ensure_model() {
    if (model) return BSVD_OK;
    hipError_t e = hipMalloc(&model, sizeof(float) * 4 * MLP_NPARAM + 64);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        model = nullptr;
        return fail(BSVD_ENOMEM, "rank model buffers: %s", hipGetErrorString(e));
    }
    e = hipMemsetAsync(model, 0, sizeof(float) * 4 * MLP_NPARAM + 64, stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(model)");
    return BSVD_OK;
}

int Ctx::ensure_mlp_scratch(int n) {
    const size_t need = sizeof(float) * ((size_t)n * MLP_SCRATCH + (size_t)n) + sizeof(int) * (size_t)n + 256;
    if (need <= mlp_scratch_size) return BSVD_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (mlp_scratch) hipFree(mlp_scratch);
    mlp_scratch = nullptr;
    mlp_scratch_size = 0;
    e = hipMalloc(&mlp_scratch, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(BSVD_ENOMEM, "rank model scratch: %s", hipGetErrorString(e));
    }
    mlp_scratch_size = need;
    return BSVD_OK;
}

}  // namespace bsvd

namespace {
float *P_(Ctx *c) { return static_cast<float *>(c->model); }
float *M1_(Ctx *c) { return static_cast<float *>(c->model) + MLP_NPARAM; }
float *M2_(Ctx *c) { return static_cast<float *>(c->model) + 2 * MLP_NPARAM; }
float *G_(Ctx *c) { return static_cast<float *>(c->model) + 3 * MLP_NPARAM; }
float *L_(Ctx *c) { return static_cast<float *>(c->model) + 4 * MLP_NPARAM; }
}  // namespace

extern "C" {

int bsvd_rank_model_nparam(void) { return MLP_NPARAM; }

int bsvd_rank_model_init(bsvd_ctx *ctx, unsigned long long seed) {
    if (!ctx) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    int rc = c->ensure_model();
    if (rc) return rc;
    hipError_t e = hipMemsetAsync(c->model, 0, sizeof(float) * 4 * MLP_NPARAM + 64, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "hipMemsetAsync(model)");
    e = launch_mlp_init(P_(c), seed, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "mlp init launch");
    c->adam_step = 0;
    return BSVD_OK;
}

int bsvd_rank_model_set(bsvd_ctx *ctx, const float *params, float margin) {
    if (!ctx || !params) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    int rc = c->ensure_model();
    if (rc) return rc;
    hipError_t e = hipMemcpy(P_(c), params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice);
    if (e != hipSuccess) return c->hip_fail(e, "hipMemcpy(params)");
    c->rank_margin = margin;
    return BSVD_OK;
}

int bsvd_rank_model_get(bsvd_ctx *ctx, float *params, float *margin) {
    if (!ctx || !params) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    if (!c->model) return c->fail(BSVD_EARG, "no rank model");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "hipStreamSynchronize");
    e = hipMemcpy(params, P_(c), sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return c->hip_fail(e, "hipMemcpy(params)");
    if (margin) *margin = c->rank_margin;
    return BSVD_OK;
}

int bsvd_rank_model_save(bsvd_ctx *ctx, const char *path) {
    if (!ctx || !path) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    std::vector<float> p(MLP_NPARAM);
    float margin = 0.0f;
    int rc = bsvd_rank_model_get(ctx, p.data(), &margin);
    if (rc) return rc;
    FILE *f = fopen(path, "wb");
    if (!f) return c->fail(BSVD_EARG, "cannot write %s", path);
    const char magic[8] = {'B', 'S', 'V', 'D', 'M', 'L', 'P', '1'};
    const int np = MLP_NPARAM;
    bool ok = fwrite(magic, 1, 8, f) == 8 && fwrite(&np, sizeof np, 1, f) == 1 &&
              fwrite(&margin, sizeof margin, 1, f) == 1 && fwrite(p.data(), sizeof(float), MLP_NPARAM, f) == (size_t)MLP_NPARAM;
    fclose(f);
    return ok ? BSVD_OK : c->fail(BSVD_EARG, "short write to %s", path);
}

int bsvd_rank_model_load(bsvd_ctx *ctx, const char *path) {
    if (!ctx || !path) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    FILE *f = fopen(path, "rb");
    if (!f) return c->fail(BSVD_EARG, "cannot open %s", path);
    char magic[8];
    int np = 0;
    float margin = 0.0f;
    std::vector<float> p(MLP_NPARAM);
    bool ok = fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "BSVDMLP1", 8) == 0 && fread(&np, sizeof np, 1, f) == 1 &&
              np == MLP_NPARAM && fread(&margin, sizeof margin, 1, f) == 1 &&
              fread(p.data(), sizeof(float), MLP_NPARAM, f) == (size_t)MLP_NPARAM;
    fclose(f);
    if (!ok) return c->fail(BSVD_EARG, "%s is not a rank-model file", path);
    return bsvd_rank_model_set(ctx, p.data(), margin);
}

int bsvd_rank_model_forward(bsvd_ctx *ctx, int n, const float *X, float *y) {
    if (!ctx || n < 0 || (n > 0 && (!X || !y))) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    if (!c->model) return c->fail(BSVD_EARG, "no rank model (init, set or load one first)");
    hipError_t e = launch_mlp_forward(P_(c), n, X, y, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "mlp forward launch");
    return BSVD_OK;
}

int bsvd_rank_model_loss_grad(bsvd_ctx *ctx, int n, const float *X, const float *T, float *loss, float *grad) {
    if (!ctx || n < 1 || !X || !T) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    if (!c->model) return c->fail(BSVD_EARG, "no rank model");
    int rc = c->ensure_mlp_scratch(n);
    if (rc) return rc;
    float *scr = static_cast<float *>(c->mlp_scratch);
    float *lt = scr + (size_t)n * MLP_SCRATCH;
    hipError_t e = launch_mlp_loss_grad(P_(c), n, X, T, nullptr, scr, lt, grad ? grad : G_(c), L_(c), c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "mlp loss/grad launch");
    if (loss) {
        e = hipMemcpyAsync(loss, L_(c), sizeof(float), hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync(loss)");
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "hipStreamSynchronize");
    }
    return BSVD_OK;
}

int bsvd_rank_model_train(bsvd_ctx *ctx, int n, const float *X, const float *T, int epochs, int batch, float lr,
                          unsigned long long seed, float *final_loss) {
    if (!ctx || n < 1 || !X || !T || epochs < 0 || batch < 1 || !(lr > 0.0f)) return BSVD_EARG;
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    c->err.clear();
    if (!c->model) {
        int rc = bsvd_rank_model_init(ctx, seed);
        if (rc) return rc;
    }
    if (batch > n) batch = n;
    int rc = c->ensure_mlp_scratch(std::max(n, batch));
    if (rc) return rc;
    float *scr = static_cast<float *>(c->mlp_scratch);
    float *lt = scr + (size_t)std::max(n, batch) * MLP_SCRATCH;
    int *didx = reinterpret_cast<int *>(lt + std::max(n, batch));
    // epoch permutations are drawn on the host (seeded) and uploaded through pinned staging
    std::mt19937_64 rng(seed);
    std::vector<int> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    for (int ep = 0; ep < epochs; ++ep) {
        std::shuffle(perm.begin(), perm.end(), rng);
        rc = c->ensure_host(sizeof(int) * (size_t)n);
        if (rc) return rc;
        std::memcpy(c->hws, perm.data(), sizeof(int) * (size_t)n);
        hipError_t e = hipMemcpyAsync(didx, c->hws, sizeof(int) * (size_t)n, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "hipMemcpyAsync(perm)");
        e = hipEventRecord(c->staged, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "hipEventRecord");
        c->staged_pending = true;
        for (int s0 = 0; s0 + batch <= n; s0 += batch) {
            e = launch_mlp_loss_grad(P_(c), batch, X, T, didx + s0, scr, lt, G_(c), nullptr, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "mlp backward launch");
            e = launch_mlp_adam(P_(c), M1_(c), M2_(c), G_(c), lr, ++c->adam_step, c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "mlp adam launch");
        }
    }
    if (final_loss) return bsvd_rank_model_loss_grad(ctx, n, X, T, final_loss, nullptr);
    return BSVD_OK;
}

}  // extern "C"
