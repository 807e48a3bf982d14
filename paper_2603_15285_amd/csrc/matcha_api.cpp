// matcha_api.cpp -- the C ABI of libmatcha (include/matcha.h): argument validation,
// read-only table construction, launch sizing.  Everything numerical runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/matcha.h"
#include "matcha_launch.hpp"

using namespace matcha;

struct matcha_ctx {
    int device = 0;
    int tab_L = -1;  // tables cover l <= tab_L
    float4 *tab = nullptr;
    PairInfo *pinfo = nullptr;
};

namespace {

// Recurrence coefficients of the wedge pair (m, n) (App. A.4; standard three-term relation
// d^{l+1} = a_l (cos b - c_l) d^l - b_l d^{l-1}), in FP64.
double rec_a(int l, int m, int n)
{
    const double l1 = l + 1.0;
    return l1 * (2.0 * l + 1.0) / std::sqrt((l1 * l1 - (double)m * m) * (l1 * l1 - (double)n * n));
}
double rec_b(int l, int m, int n)
{
    if (l == 0) return 0.0;
    const double l1 = l + 1.0;
    return l1 * std::sqrt(((double)l * l - (double)m * m) * ((double)l * l - (double)n * n)) /
           ((double)l * std::sqrt((l1 * l1 - (double)m * m) * (l1 * l1 - (double)n * n)));
}
double rec_c(int l, int m, int n) { return l == 0 ? 0.0 : (double)m * n / ((double)l * (l + 1.0)); }

// Per (l, q) entry: A = abar_{l-1}, AC = abar_{l-1} c_{l-1}, PW = w P_l, PWT = w~ s P_l, with
// P_m = P_{m+1} = 1, P_{l+1} = b_l P_{l-1} and abar_l = a_l P_l / P_{l+1}, so that
// D^l = d^l / P_l obeys D^l = abar_{l-1} (cos b - c_{l-1}) D^{l-1} - D^{l-2}.
// w = 1/2 for the self-conjugate pair (0, 0) (every other term is doubled by its Hermitian
// mirror); w~ = 0 for diagonal pairs whose partner is the pair itself; s = (-1)^{m-n} for
// n >= 0 (d_nm = (-1)^{m-n} d_mn) and 1 for n < 0 (d_{-n,-m} = d_mn).
void build_tables(int Lmax, std::vector<float4> &tab, std::vector<PairInfo> &pinfo)
{
    tab.assign((size_t)wedge_row(Lmax + 1), make_float4(0.f, 0.f, 0.f, 0.f));
    pinfo.assign((size_t)(Lmax + 1) * (Lmax + 1), PairInfo{0, 0, 0.0});
    std::vector<double> P((size_t)Lmax + 2);
    for (int m = 0; m <= Lmax; ++m)
        for (int n = -m; n <= m; ++n) {
            const int q = m * m + m + n;
            pinfo[q].m = m;
            pinfo[q].n = n;
            pinfo[q].lbh2 = 0.5 * (std::lgamma(2.0 * m + 1.0) - std::lgamma(m + n + 1.0) - std::lgamma(m - n + 1.0)) /
                            std::log(2.0);
            const double wt = (m == 0) ? 0.5 : 1.0;
            const double wtt = (n == m || n == -m) ? 0.0 : 1.0;
            const double sg = (n >= 0 && ((m - n) & 1)) ? -1.0 : 1.0;
            P[m] = 1.0;
            P[m + 1] = 1.0;
            for (int l = m + 1; l <= Lmax; ++l) P[l + 1] = rec_b(l, m, n) * P[l - 1];
            for (int l = m; l <= Lmax; ++l) {
                float4 e;
                if (l == m) {
                    e.x = 0.f;
                    e.y = 0.f;
                } else {
                    const double ab = rec_a(l - 1, m, n) * P[l - 1] / P[l];
                    e.x = (float)ab;
                    e.y = (float)(ab * rec_c(l - 1, m, n));
                }
                e.z = (float)(wt * P[l]);
                e.w = (float)(wtt * sg * P[l]);
                tab[(size_t)wedge_row(l) + q] = e;
            }
        }
}

matcha_status ensure_tables(matcha_ctx *ctx, int L)
{
    if (L <= ctx->tab_L) return MATCHA_OK;
    std::vector<float4> tab;
    std::vector<PairInfo> pinfo;
    build_tables(L, tab, pinfo);
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    float4 *dt = nullptr;
    PairInfo *dp = nullptr;
    if (hipMalloc(&dt, tab.size() * sizeof(float4)) != hipSuccess) return MATCHA_ERR_HIP;
    if (hipMalloc(&dp, pinfo.size() * sizeof(PairInfo)) != hipSuccess) {
        (void)hipFree(dt);
        return MATCHA_ERR_HIP;
    }
    if (hipMemcpy(dt, tab.data(), tab.size() * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dp, pinfo.data(), pinfo.size() * sizeof(PairInfo), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dt);
        (void)hipFree(dp);
        return MATCHA_ERR_HIP;
    }
    // the previous (smaller) tables may still be in use by enqueued work
    if (ctx->tab) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->tab);
        (void)hipFree(ctx->pinfo);
    }
    ctx->tab = dt;
    ctx->pinfo = dp;
    ctx->tab_L = L;
    return MATCHA_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Common batch checks; on success minL / maxL / maxR hold the host-side extents.
matcha_status check_batch(const matcha_batch *b, int *minL, int *maxL, int *maxR)
{
    if (!b || b->n_particles < 0) return MATCHA_ERR_INVALID_ARG;
    if (b->n_particles == 0) {
        *minL = *maxL = *maxR = 0;
        return MATCHA_OK;
    }
    if (!b->L_host || !b->R_host || !b->L_dev || !b->R_dev || !b->C_offset) return MATCHA_ERR_INVALID_ARG;
    if (b->L_h < 0 || b->L_h > MATCHA_MAX_L || b->R_h < 1) return MATCHA_ERR_INVALID_ARG;
    int lo = 1 << 30, hi = -1, rh = 0;
    for (int p = 0; p < b->n_particles; ++p) {
        const int L = b->L_host[p], R = b->R_host[p];
        if (L < 0 || L > MATCHA_MAX_L || L > b->L_h || R < 1 || R > b->R_h) return MATCHA_ERR_INVALID_ARG;
        lo = std::min(lo, L);
        hi = std::max(hi, L);
        rh = std::max(rh, R);
    }
    if (b->L_max < hi || b->L_max > MATCHA_MAX_L) return MATCHA_ERR_INVALID_ARG;
    *minL = lo;
    *maxL = hi;
    *maxR = rh;
    return MATCHA_OK;
}

matcha_status launched(hipError_t e) { return e == hipSuccess ? MATCHA_OK : MATCHA_ERR_HIP; }

int march_nc(int Kc) { return Kc <= 32 ? 4 : 8; }

}  // namespace

extern "C" {

matcha_status matcha_create(int device, matcha_ctx **out)
{
    if (!out) return MATCHA_ERR_INVALID_ARG;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return MATCHA_ERR_HIP;
    if (device < 0 || device >= n) return MATCHA_ERR_INVALID_ARG;
    matcha_ctx *c = new (std::nothrow) matcha_ctx();
    if (!c) return MATCHA_ERR_HIP;
    c->device = device;
    *out = c;
    return MATCHA_OK;
}

matcha_status matcha_destroy(matcha_ctx *ctx)
{
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    if (ctx->tab) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->tab);
        (void)hipFree(ctx->pinfo);
    }
    delete ctx;
    return MATCHA_OK;
}

matcha_status matcha_prepare(matcha_ctx *ctx, int32_t L_max, int32_t B, int32_t n_grid)
{
    if (!ctx || L_max < 0 || L_max > MATCHA_MAX_L || B < 0 || B > L_max || n_grid < 0) return MATCHA_ERR_INVALID_ARG;
    return ensure_tables(ctx, L_max);
}

const char *matcha_status_string(matcha_status s)
{
    switch (s) {
    case MATCHA_OK: return "ok";
    case MATCHA_ERR_INVALID_ARG: return "invalid argument";
    case MATCHA_ERR_UNSUPPORTED: return "unsupported configuration";
    case MATCHA_ERR_HIP: return "HIP runtime error";
    case MATCHA_ERR_WORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

int64_t matcha_c_elems(int32_t L)
{
    if (L < 0 || L > MATCHA_MAX_L) return -1;
    return 2 * wedge_row(L + 1);
}

int64_t matcha_f_elems(int32_t L, int32_t R)
{
    if (L < 0 || L > MATCHA_MAX_L || R < 0) return -1;
    return (int64_t)R * (L + 1) * (L + 1);
}

size_t matcha_workspace_size(const matcha_batch *batch, int32_t Kc)
{
    (void)batch;
    (void)Kc;
    return 0;
}

matcha_status matcha_coeff_assemble(matcha_ctx *ctx, const matcha_batch *batch, const void *f, const void *h,
                                    const float *w, float *C, matcha_precision prec, void *stream)
{
    int lo, hi, rmax;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return MATCHA_OK;
    if (!f || !h || !w || !C || !batch->f_offset || !aligned16(C)) return MATCHA_ERR_INVALID_ARG;
    if (prec != MATCHA_FP32) return MATCHA_ERR_UNSUPPORTED;
    if (assemble_smem_bytes(hi, rmax) > 160 * 1024) return MATCHA_ERR_UNSUPPORTED;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    AsmArgs a;
    a.f = static_cast<const float2 *>(f);
    a.f_off = batch->f_offset;
    a.h = static_cast<const float2 *>(h);
    a.w = w;
    a.Lp = batch->L_dev;
    a.Rp = batch->R_dev;
    a.Lh = batch->L_h;
    a.C = reinterpret_cast<float4 *>(C);
    a.C_off = batch->C_offset;
    return launched(launch_assemble_f32(a, batch->n_particles, hi, rmax, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_soft_search(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                 const matcha_soft_cfg *cfg, float *cand, uint32_t *status, void *stream)
{
    int lo, hi, rmax;
    if (!ctx || !cfg) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return MATCHA_OK;
    if (!C || !cand || !status || !aligned16(C) || !aligned16(cand)) return MATCHA_ERR_INVALID_ARG;
    const int B = cfg->B, n = cfg->n_grid, Kc = cfg->Kc;
    if (B < 1 || B > lo || B > 32 || n < 4 || n > 96 || Kc < 1 || Kc > MATCHA_MAX_KC) return MATCHA_ERR_INVALID_ARG;
    if (soft_smem_bytes(n, B) > 160 * 1024) return MATCHA_ERR_UNSUPPORTED;
    st = ensure_tables(ctx, std::max(hi, B));
    if (st != MATCHA_OK) return st;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    SoftArgs a;
    a.C = reinterpret_cast<const float4 *>(C);
    a.C_off = batch->C_offset;
    a.tab = ctx->tab;
    a.pinfo = ctx->pinfo;
    a.B = B;
    a.n = n;
    a.Kc = Kc;
    a.cand = reinterpret_cast<float4 *>(cand);
    a.status = status;
    return launched(launch_soft(a, batch->n_particles, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_march_newton(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                  const matcha_march_cfg *cfg, int32_t Kc, float *cand, float *best,
                                  int32_t *best_idx, uint32_t *status, void *stream)
{
    int lo, hi, rmax;
    if (!ctx || !cfg) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return MATCHA_OK;
    if (!C || !cand || !best || !best_idx || !status || !aligned16(C) || !aligned16(cand) || !aligned16(best))
        return MATCHA_ERR_INVALID_ARG;
    if (Kc < 1 || Kc > MATCHA_MAX_KC || cfg->steps < 0 || cfg->n_levels < 1 || cfg->n_levels > MATCHA_MAX_LEVELS ||
        !cfg->levels || !(cfg->max_step >= 0.0) || lo < 1)
        return MATCHA_ERR_INVALID_ARG;
    for (int j = 0; j < cfg->n_levels; ++j) {
        if (cfg->levels[j] < 1 || cfg->levels[j] > MATCHA_MAX_L) return MATCHA_ERR_INVALID_ARG;
        if (j > 0 && cfg->levels[j] <= cfg->levels[j - 1]) return MATCHA_ERR_INVALID_ARG;
    }
    st = ensure_tables(ctx, hi);
    if (st != MATCHA_OK) return st;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    MarchArgs a;
    std::memset(&a, 0, sizeof a);
    a.C = reinterpret_cast<const float4 *>(C);
    a.C_off = batch->C_offset;
    a.Lp = batch->L_dev;
    a.tab = ctx->tab;
    a.pinfo = ctx->pinfo;
    a.n_levels = cfg->n_levels;
    for (int j = 0; j < cfg->n_levels; ++j) a.levels[j] = cfg->levels[j];
    a.steps = cfg->steps;
    a.max_step = cfg->max_step;
    a.early_stop = cfg->early_stop;
    a.tol_grad = cfg->tol_grad;
    a.tol_step = cfg->tol_step;
    a.tol_rel = cfg->tol_rel;
    a.Kc = Kc;
    a.cand = reinterpret_cast<float4 *>(cand);
    a.best = reinterpret_cast<float4 *>(best);
    a.best_idx = best_idx;
    a.status = status;
    const int nc = march_nc(Kc);
    return launched(launch_march_any(a, batch->n_particles, nc, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_evaluate(matcha_ctx *ctx, const matcha_batch *batch, const float *C, int32_t L_eval,
                              const float *theta, float *out, void *stream)
{
    int lo, hi, rmax;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return MATCHA_OK;
    if (!C || !theta || !out || !aligned16(C) || !aligned16(theta)) return MATCHA_ERR_INVALID_ARG;
    if (L_eval < 0 || L_eval > lo) return MATCHA_ERR_INVALID_ARG;
    st = ensure_tables(ctx, std::max(hi, L_eval));
    if (st != MATCHA_OK) return st;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    EvalArgs a;
    a.C = reinterpret_cast<const float4 *>(C);
    a.C_off = batch->C_offset;
    a.tab = ctx->tab;
    a.pinfo = ctx->pinfo;
    a.L = L_eval;
    a.theta = reinterpret_cast<const float4 *>(theta);
    a.out = out;
    return launched(launch_evaluate(a, batch->n_particles, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_grad_template(matcha_ctx *ctx, const matcha_batch *batch, const float *f, const float *h,
                                   const float *w, const float *best, const float *g, float *grad_h, float *grad_f,
                                   void *ws, size_t ws_bytes, void *stream)
{
    (void)ctx;
    (void)batch;
    (void)f;
    (void)h;
    (void)w;
    (void)best;
    (void)g;
    (void)grad_h;
    (void)grad_f;
    (void)ws;
    (void)ws_bytes;
    (void)stream;
    return MATCHA_ERR_UNSUPPORTED;
}

}  // extern "C"
