// matcha_api.cpp -- the C ABI of libmatcha (include/matcha.h): argument validation,
// read-only table construction, launch sizing.  Everything numerical runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
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
    double2 *tab64 = nullptr;  // (A, AC) of tab in FP64
    PairInfo *pinfo = nullptr;
    matcha_tuning tune{0, 0};
    int grid_B = -1, grid_n = -1;  // the SOFFT node tables below are for (grid_B, grid_n)
    float2 *dgrid = nullptr;
    float *dft = nullptr;           // DFT tables of the SOFFT grid kernel (build_soft_dft)
    float *soft_ws = nullptr;       // SOFFT grid workspace of the eager calls
    size_t soft_ws_bytes = 0;
    int32_t *by_L = nullptr;        // particle order of the eager assembly calls on mixed L_p
    int by_L_cap = 0;
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
void build_tables(int Lmax, std::vector<float4> &tab, std::vector<double2> &tab64, std::vector<PairInfo> &pinfo)
{
    tab.assign((size_t)wedge_row(Lmax + 1), make_float4(0.f, 0.f, 0.f, 0.f));
    tab64.assign((size_t)wedge_row(Lmax + 1), make_double2(0.0, 0.0));
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
                double2 e64 = make_double2(0.0, 0.0);
                if (l == m) {
                    e.x = 0.f;
                    e.y = 0.f;
                } else {
                    const double ab = rec_a(l - 1, m, n) * P[l - 1] / P[l];
                    e64 = make_double2(ab, ab * rec_c(l - 1, m, n));
                    e.x = (float)e64.x;
                    e.y = (float)e64.y;
                }
                tab64[(size_t)wedge_row(l) + q] = e64;
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
    std::vector<double2> tab64;
    std::vector<PairInfo> pinfo;
    build_tables(L, tab, tab64, pinfo);
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    float4 *dt = nullptr;
    double2 *dt64 = nullptr;
    PairInfo *dp = nullptr;
    if (hipMalloc(&dt, tab.size() * sizeof(float4)) != hipSuccess) return MATCHA_ERR_HIP;
    if (hipMalloc(&dt64, tab64.size() * sizeof(double2)) != hipSuccess) {
        (void)hipFree(dt);
        return MATCHA_ERR_HIP;
    }
    if (hipMalloc(&dp, pinfo.size() * sizeof(PairInfo)) != hipSuccess) {
        (void)hipFree(dt);
        (void)hipFree(dt64);
        return MATCHA_ERR_HIP;
    }
    if (hipMemcpy(dt, tab.data(), tab.size() * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dt64, tab64.data(), tab64.size() * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dp, pinfo.data(), pinfo.size() * sizeof(PairInfo), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dt);
        (void)hipFree(dt64);
        (void)hipFree(dp);
        return MATCHA_ERR_HIP;
    }
    // the previous (smaller) tables may still be in use by enqueued work
    if (ctx->tab) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->tab);
        (void)hipFree(ctx->tab64);
        (void)hipFree(ctx->pinfo);
    }
    ctx->tab = dt;
    ctx->tab64 = dt64;
    ctx->pinfo = dp;
    ctx->tab_L = L;
    return MATCHA_OK;
}

// d^l_mn(b_i) at the SOFFT polar nodes b_i = pi (2i+1) / (2n) for every wedge pair and l <= B,
// in FP64 by the three-term recurrence from the edge value
//   d^m_mn(b) = (-1)^{m-n} sqrt(binom(2m, m+n)) cos^{m+n}(b/2) sin^{m-n}(b/2),
// stored per node in the wedge layout as (w d, w~ s d) -- the weights of build_tables.
void build_grid_table(int B, int n, std::vector<float2> &g)
{
    const int64_t rows = wedge_row(B + 1);
    g.assign((size_t)(n * rows), make_float2(0.f, 0.f));
    for (int i = 0; i < n; ++i) {
        const double b = M_PI * (2.0 * i + 1.0) / (2.0 * n);
        const double cb = std::cos(b), ch = std::cos(0.5 * b), sh = std::sin(0.5 * b);
        for (int m = 0; m <= B; ++m)
            for (int nn = -m; nn <= m; ++nn) {
                const int q = m * m + m + nn;
                const double wt = (m == 0) ? 0.5 : 1.0;
                const double wtt = (nn == m || nn == -m) ? 0.0 : 1.0;
                const double sg = (nn >= 0 && ((m - nn) & 1)) ? -1.0 : 1.0;
                const double lb = 0.5 * (std::lgamma(2.0 * m + 1.0) - std::lgamma(m + nn + 1.0) - std::lgamma(m - nn + 1.0));
                double d = std::exp(lb) * std::pow(ch, m + nn) * std::pow(sh, m - nn);
                if ((m - nn) & 1) d = -d;
                double dm = 0.0;
                for (int l = m; l <= B; ++l) {
                    g[(size_t)(i * rows + wedge_row(l) + q)] = make_float2((float)(wt * d), (float)(wtt * sg * d));
                    const double dn = rec_a(l, m, nn) * (cb - rec_c(l, m, nn)) * d - rec_b(l, m, nn) * dm;
                    dm = d;
                    d = dn;
                }
            }
    }
}

matcha_status ensure_grid(matcha_ctx *ctx, int B, int n)
{
    if (ctx->dgrid && ctx->grid_B == B && ctx->grid_n == n) return MATCHA_OK;
    std::vector<float2> g;
    build_grid_table(B, n, g);
    std::vector<float> e(soft_dft_floats(n, B));
    build_soft_dft(B, n, e.data());
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    float2 *d = nullptr;
    float *de = nullptr;
    if (hipMalloc(&d, g.size() * sizeof(float2)) != hipSuccess) return MATCHA_ERR_HIP;
    if (hipMalloc(&de, e.size() * sizeof(float)) != hipSuccess) {
        (void)hipFree(d);
        return MATCHA_ERR_HIP;
    }
    if (hipMemcpy(d, g.data(), g.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(de, e.data(), e.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        (void)hipFree(de);
        return MATCHA_ERR_HIP;
    }
    if (ctx->dgrid) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->dgrid);
        (void)hipFree(ctx->dft);
    }
    ctx->dgrid = d;
    ctx->dft = de;
    ctx->grid_B = B;
    ctx->grid_n = n;
    return MATCHA_OK;
}

// The SOFFT search of a particle keeps in a workspace, between its kernels: the Wigner
// transforms of its n polar nodes ((B+1)(2B+1) complex each), its grid (n^3 floats) and its list
// of maxima keys with their count.  Batches whose workspace would exceed kSoftWsCap run in chunks
// of particles.  Layout of a chunk of pc particles (each region 256-byte aligned): the grids, pc
// lists of kSoftListMax keys, pc counts, the Wigner transforms.
constexpr size_t kSoftWsCap = (size_t)4 << 30;
constexpr size_t kSoftListMax = 1024;  // keys per particle: the larger select workgroup's list

size_t soft_grid_bytes(int n) { return (size_t)n * n * n * sizeof(float); }
size_t soft_s_bytes(int n, int B) { return (size_t)n * (B + 1) * (2 * B + 1) * sizeof(float2); }
size_t soft_particle_bytes(int n, int B)
{
    return soft_grid_bytes(n) + kSoftListMax * sizeof(unsigned long long) + sizeof(uint32_t) + soft_s_bytes(n, B);
}
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SoftChunk {
    size_t grid, list, count, S, total;  // region offsets and total bytes
};

SoftChunk soft_chunk(size_t pc, int n, int B)
{
    SoftChunk c;
    c.grid = 0;
    c.list = align256(pc * soft_grid_bytes(n));
    c.count = c.list + align256(pc * kSoftListMax * sizeof(unsigned long long));
    c.S = c.count + align256(pc * sizeof(uint32_t));
    c.total = c.S + align256(pc * soft_s_bytes(n, B));
    return c;
}

size_t soft_ws_need(int P, int n, int B)
{
    const size_t pc = std::max<size_t>(1, std::min<size_t>((size_t)P, kSoftWsCap / soft_particle_bytes(n, B)));
    return soft_chunk(pc, n, B).total;
}

matcha_status ensure_soft_ws(matcha_ctx *ctx, size_t bytes)
{
    if (ctx->soft_ws_bytes >= bytes) return MATCHA_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    if (ctx->soft_ws) {
        (void)hipDeviceSynchronize();  // earlier searches may still read it
        (void)hipFree(ctx->soft_ws);
        ctx->soft_ws = nullptr;
        ctx->soft_ws_bytes = 0;
    }
    if (hipMalloc(&ctx->soft_ws, bytes) != hipSuccess) {
        ctx->soft_ws = nullptr;
        return MATCHA_ERR_HIP;
    }
    ctx->soft_ws_bytes = bytes;
    return MATCHA_OK;
}

matcha_status ensure_by_L(matcha_ctx *ctx, int P)
{
    if (ctx->by_L_cap >= P) return MATCHA_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    if (ctx->by_L) {
        (void)hipDeviceSynchronize();  // earlier assemblies may still read it
        (void)hipFree(ctx->by_L);
        ctx->by_L = nullptr;
        ctx->by_L_cap = 0;
    }
    if (hipMalloc(&ctx->by_L, sizeof(int32_t) * (size_t)P) != hipSuccess) {
        ctx->by_L = nullptr;
        return MATCHA_ERR_HIP;
    }
    ctx->by_L_cap = P;
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

int march_nc(const matcha_ctx *ctx, int Kc)
{
    int nc = ctx->tune.march_nc;
    if (nc == 0) nc = Kc <= 32 ? 4 : 8;
    while ((Kc + nc - 1) / nc > 8) nc *= 2;
    return nc;
}

// Argument checks of the assembly (the batch itself is checked by check_batch).
matcha_status assemble_check(const matcha_batch *batch, const void *f, const void *h, const float *w, const float *C,
                             matcha_precision prec, int hi, int rmax)
{
    if (!f || !h || !w || !C || !batch->f_offset || !aligned16(C)) return MATCHA_ERR_INVALID_ARG;
    if (prec != MATCHA_FP32 && prec != MATCHA_BF16_FP32ACC) return MATCHA_ERR_UNSUPPORTED;
    // the kernels index within one particle's f and within h with 32-bit offsets
    if ((int64_t)batch->R_h * (batch->L_h + 1) * (batch->L_h + 1) >= INT32_MAX) return MATCHA_ERR_UNSUPPORTED;
    const size_t smem = prec == MATCHA_FP32 ? assemble_smem_bytes(hi, rmax) : assemble_bf16_smem_bytes(hi, rmax);
    if (smem > 160 * 1024) return MATCHA_ERR_UNSUPPORTED;
    return MATCHA_OK;
}

// The assembly launches.  With mixed L_p (lo < hi), by_L ([P] int32) receives the particles in
// the order of decreasing L_p first, so that each degree's rows cover only the particles that
// have it.
matcha_status assemble_ws(matcha_ctx *ctx, const matcha_batch *batch, const void *f, const void *h, const float *w,
                          float *C, matcha_precision prec, int lo, int hi, int rmax, int32_t *by_L, hipStream_t s)
{
    const int P = batch->n_particles;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    int np_l[kMaxL + 1];
    const bool mixed = lo != hi;
    if (mixed) {
        for (int l = 0; l <= hi; ++l) np_l[l] = 0;
        for (int p = 0; p < P; ++p) np_l[batch->L_host[p]] += 1;
        for (int l = hi - 1; l >= 0; --l) np_l[l] += np_l[l + 1];  // particles with L_p >= l
        const hipError_t e = launch_order_by_L(batch->L_dev, P, hi, by_L, s);
        if (e != hipSuccess) return launched(e);
    }
    if (prec == MATCHA_BF16_FP32ACC) {
        AsmBArgs b;
        std::memset(&b, 0, sizeof b);
        b.f = static_cast<const __bf16 *>(f);
        b.f_off = batch->f_offset;
        b.h = static_cast<const __bf16 *>(h);
        b.w = w;
        b.Lp = batch->L_dev;
        b.Rp = batch->R_dev;
        b.Lh = batch->L_h;
        b.C = reinterpret_cast<float4 *>(C);
        b.C_off = batch->C_offset;
        if (mixed) {
            b.by_L = by_L;
            std::memcpy(b.np_l, np_l, sizeof(int) * (size_t)(hi + 1));
        }
        return launched(launch_assemble_bf16(b, P, hi, rmax, s));
    }
    AsmArgs a;
    std::memset(&a, 0, sizeof a);
    a.f = static_cast<const float2 *>(f);
    a.f_off = batch->f_offset;
    a.h = static_cast<const float2 *>(h);
    a.w = w;
    a.Lp = batch->L_dev;
    a.Rp = batch->R_dev;
    a.Lh = batch->L_h;
    a.C = reinterpret_cast<float4 *>(C);
    a.C_off = batch->C_offset;
    if (mixed) {
        a.by_L = by_L;
        std::memcpy(a.np_l, np_l, sizeof(int) * (size_t)(hi + 1));
    }
    return launched(launch_assemble_f32(a, P, hi, rmax, s));
}

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
        (void)hipFree(ctx->tab64);
        (void)hipFree(ctx->pinfo);
    }
    if (ctx->dgrid || ctx->soft_ws || ctx->by_L) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        if (ctx->dgrid) (void)hipFree(ctx->dgrid);
        if (ctx->dft) (void)hipFree(ctx->dft);
        if (ctx->soft_ws) (void)hipFree(ctx->soft_ws);
        if (ctx->by_L) (void)hipFree(ctx->by_L);
    }
    delete ctx;
    return MATCHA_OK;
}

matcha_status matcha_prepare(matcha_ctx *ctx, int32_t L_max, int32_t B, int32_t n_grid)
{
    if (!ctx || L_max < 0 || L_max > MATCHA_MAX_L || B < 0 || B > L_max || n_grid < 0) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = ensure_tables(ctx, L_max);
    if (st != MATCHA_OK || B < 1 || n_grid < 4) return st;
    return ensure_grid(ctx, B, n_grid);
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

matcha_status matcha_set_tuning(matcha_ctx *ctx, const matcha_tuning *t)
{
    if (!ctx || !t) return MATCHA_ERR_INVALID_ARG;
    const int nc = t->march_nc;
    if (nc != 0 && nc != 1 && nc != 2 && nc != 4 && nc != 8) return MATCHA_ERR_INVALID_ARG;
    const int st = t->soft_threads;
    if (st != 0 && st != 256 && st != 512) return MATCHA_ERR_INVALID_ARG;
    ctx->tune = *t;
    return MATCHA_OK;
}

matcha_status matcha_get_tuning(const matcha_ctx *ctx, matcha_tuning *t)
{
    if (!ctx || !t) return MATCHA_ERR_INVALID_ARG;
    *t = ctx->tune;
    return MATCHA_OK;
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
    (void)Kc;
    if (!batch || batch->n_particles <= 0 || !batch->L_host || !batch->R_host) return 0;
    // matcha_grad_template: one complex float32 template-gradient term per particle, laid out like f
    size_t n = 0;
    for (int p = 0; p < batch->n_particles; ++p) {
        const int64_t e = matcha_f_elems(batch->L_host[p], batch->R_host[p]);
        if (e < 0) return 0;
        n += (size_t)e;
    }
    return n * 2 * sizeof(float);
}

matcha_status matcha_coeff_assemble(matcha_ctx *ctx, const matcha_batch *batch, const void *f, const void *h,
                                    const float *w, float *C, matcha_precision prec, void *stream)
{
    int lo, hi, rmax;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return MATCHA_OK;
    st = assemble_check(batch, f, h, w, C, prec, hi, rmax);
    if (st != MATCHA_OK) return st;
    if (lo != hi) {
        st = ensure_by_L(ctx, batch->n_particles);
        if (st != MATCHA_OK) return st;
    }
    return assemble_ws(ctx, batch, f, h, w, C, prec, lo, hi, rmax, ctx->by_L, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// Checks of a SOFFT search; on success *nt is the select kernel's workgroup size.
matcha_status soft_check(matcha_ctx *ctx, const matcha_batch *batch, const float *C, const matcha_soft_cfg *cfg,
                         const float *cand, const uint32_t *status, int *nt)
{
    int lo, hi, rmax;
    if (!ctx || !cfg) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return MATCHA_OK;
    if (!C || !cand || !status || !aligned16(C) || !aligned16(cand)) return MATCHA_ERR_INVALID_ARG;
    const int B = cfg->B, n = cfg->n_grid, Kc = cfg->Kc;
    if (B < 1 || B > lo || B > 32 || n < 4 || n > 96 || Kc < 1 || Kc > MATCHA_MAX_KC) return MATCHA_ERR_INVALID_ARG;
    *nt = ctx->tune.soft_threads ? ctx->tune.soft_threads : 256;
    if (soft_grid_smem_bytes(n, B) > 160 * 1024 || soft_select_smem_bytes(n, *nt) > 160 * 1024)
        return MATCHA_ERR_UNSUPPORTED;
    st = ensure_tables(ctx, std::max(hi, B));
    if (st != MATCHA_OK) return st;
    return ensure_grid(ctx, B, n);
}

// The search proper over a grid workspace ws of ws_bytes (at least one particle's grid).
matcha_status soft_search_ws(matcha_ctx *ctx, const matcha_batch *batch, const float *C, const matcha_soft_cfg *cfg,
                             float *cand, uint32_t *status, int nt, float *ws, size_t ws_bytes, hipStream_t s)
{
    const int P = batch->n_particles, n = cfg->n_grid, B = cfg->B;
    if (!ws || ws_bytes < soft_chunk(1, n, B).total) return MATCHA_ERR_INVALID_ARG;
    size_t pcs = std::min<size_t>((size_t)P, ws_bytes / soft_particle_bytes(n, B));
    while (pcs > 1 && soft_chunk(pcs, n, B).total > ws_bytes) --pcs;
    const int pc = (int)std::max<size_t>(pcs, 1);
    const SoftChunk ch = soft_chunk((size_t)pc, n, B);
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    char *base = reinterpret_cast<char *>(ws);
    SoftArgs a;
    std::memset(&a, 0, sizeof a);
    a.C = reinterpret_cast<const float4 *>(C);
    a.C_off = batch->C_offset;
    a.dgrid = ctx->dgrid;
    a.dft = ctx->dft;
    a.pinfo = ctx->pinfo;
    a.B = B;
    a.n = n;
    a.Kc = cfg->Kc;
    a.grid = reinterpret_cast<float *>(base + ch.grid);
    a.mlist = reinterpret_cast<unsigned long long *>(base + ch.list);
    a.mcount = reinterpret_cast<uint32_t *>(base + ch.count);
    a.S = reinterpret_cast<float2 *>(base + ch.S);
    a.cand = reinterpret_cast<float4 *>(cand);
    a.status = status;
    for (int p0 = 0; p0 < P; p0 += pc) {
        const int cnt = std::min(pc, P - p0);
        a.p0 = p0;
        if (launch_soft_wigner(a, cnt, s) != hipSuccess) return MATCHA_ERR_HIP;
        if (launch_soft_grid(a, cnt, s) != hipSuccess) return MATCHA_ERR_HIP;
        if (launch_soft_select(a, cnt, nt, s) != hipSuccess) return MATCHA_ERR_HIP;
    }
    return MATCHA_OK;
}

}  // namespace

extern "C" {

matcha_status matcha_soft_search(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                 const matcha_soft_cfg *cfg, float *cand, uint32_t *status, void *stream)
{
    int nt = 0;
    matcha_status st = soft_check(ctx, batch, C, cfg, cand, status, &nt);
    if (st != MATCHA_OK || batch->n_particles == 0) return st;
    st = ensure_soft_ws(ctx, soft_ws_need(batch->n_particles, cfg->n_grid, cfg->B));
    if (st != MATCHA_OK) return st;
    return soft_search_ws(ctx, batch, C, cfg, cand, status, nt, ctx->soft_ws, ctx->soft_ws_bytes,
                          static_cast<hipStream_t>(stream));
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
    a.tab64 = ctx->tab64;
    a.fp64_above = cfg->fp64_above > 0 ? cfg->fp64_above : MATCHA_MAX_L;
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
    a.order = batch->order;
    const int nc = march_nc(ctx, Kc);
    const bool f64 = a.fp64_above < hi;  // a level above the threshold: some particle's L_p
    return launched(launch_march_any(a, batch->n_particles, nc, f64, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_evaluate(matcha_ctx *ctx, const matcha_batch *batch, const float *C, int32_t L_eval,
                              int32_t fp64_above, const float *theta, float *out, void *stream)
{
    int lo, hi, rmax;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return MATCHA_OK;
    if (!C || !theta || !out || !aligned16(C) || !aligned16(theta)) return MATCHA_ERR_INVALID_ARG;
    if (L_eval < 0 || L_eval > lo) return MATCHA_ERR_INVALID_ARG;  /* 0: each particle's own L_p */
    st = ensure_tables(ctx, std::max(hi, L_eval));
    if (st != MATCHA_OK) return st;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    EvalArgs a;
    a.C = reinterpret_cast<const float4 *>(C);
    a.C_off = batch->C_offset;
    a.tab = ctx->tab;
    a.tab64 = ctx->tab64;
    a.fp64_above = fp64_above > 0 ? fp64_above : MATCHA_MAX_L;
    a.pinfo = ctx->pinfo;
    a.Lp = batch->L_dev;
    a.L = L_eval;
    a.theta = reinterpret_cast<const float4 *>(theta);
    a.out = out;
    return launched(launch_evaluate(a, batch->n_particles, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_grad_template(matcha_ctx *ctx, const matcha_batch *batch, const float *f, const float *h,
                                   const float *w, const float *best, const float *g, float *grad_h, float *grad_f,
                                   void *ws, size_t ws_bytes, void *stream)
{
    int lo, hi, rmax;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return MATCHA_OK;
    if (!f || !h || !w || !best || !g || !batch->f_offset || !aligned16(best)) return MATCHA_ERR_INVALID_ARG;
    if (!grad_h && !grad_f) return MATCHA_OK;
    if (grad_h && (!ws || ws_bytes < matcha_workspace_size(batch, 0))) return MATCHA_ERR_WORKSPACE;
    if (grad_smem_bytes(hi) > 160 * 1024) return MATCHA_ERR_UNSUPPORTED;
    st = ensure_tables(ctx, hi);
    if (st != MATCHA_OK) return st;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    GradArgs a;
    std::memset(&a, 0, sizeof a);
    a.f = reinterpret_cast<const float2 *>(f);
    a.f_off = batch->f_offset;
    a.h = reinterpret_cast<const float2 *>(h);
    a.w = w;
    a.Lp = batch->L_dev;
    a.Rp = batch->R_dev;
    a.Lh = batch->L_h;
    a.Rh = batch->R_h;
    a.L_max = hi;
    a.P = batch->n_particles;
    a.best = reinterpret_cast<const float4 *>(best);
    a.g = g;
    a.grad_f = reinterpret_cast<float2 *>(grad_f);
    a.grad_h = reinterpret_cast<float2 *>(grad_h);
    a.ws = grad_h ? static_cast<float2 *>(ws) : nullptr;
    a.pinfo = ctx->pinfo;
    a.tab = ctx->tab;
    return launched(launch_grad(a, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_lpt_order(const matcha_batch *batch, const matcha_march_cfg *cfg, int32_t *order_host)
{
    int lo, hi, rmax;
    if (!cfg || !order_host || !cfg->levels || cfg->n_levels < 1) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    const int P = batch->n_particles;
    std::vector<std::pair<double, int>> cost((size_t)P);
    for (int p = 0; p < P; ++p) {
        const int Lp = batch->L_host[p];
        double c = 0.0;
        for (int j = 0; j < cfg->n_levels; ++j)
            if (cfg->levels[j] < Lp) c += (double)wedge_row(cfg->levels[j] + 1);
        c += (double)wedge_row(Lp + 1);
        cost[(size_t)p] = {-c, p};
    }
    std::stable_sort(cost.begin(), cost.end());
    for (int p = 0; p < P; ++p) order_host[p] = cost[(size_t)p].second;
    return MATCHA_OK;
}

struct matcha_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float *soft_ws = nullptr;  // the graph's own SOFFT grid workspace (the context's may be regrown)
    int32_t *by_L = nullptr;   // the graph's own particle order for the assembly (mixed L_p)
    int device = 0;
};

matcha_status matcha_align_graph_create(matcha_ctx *ctx, const matcha_batch *batch, const void *f, const void *h,
                                        const float *w, float *C, matcha_precision prec, const matcha_soft_cfg *soft,
                                        const matcha_march_cfg *march, float *cand, float *best, int32_t *best_idx,
                                        uint32_t *status, matcha_graph **out)
{
    int lo, hi, rmax;
    if (!ctx || !soft || !march || !out) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    // build every table now: nothing may allocate while the stream is being captured
    st = ensure_tables(ctx, std::max(hi, soft->B));
    if (st != MATCHA_OK) return st;
    int nt = 0;
    st = soft_check(ctx, batch, C, soft, cand, status, &nt);
    if (st != MATCHA_OK) return st;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    matcha_graph *g = new (std::nothrow) matcha_graph();
    if (!g) return MATCHA_ERR_HIP;
    g->device = ctx->device;
    const int P = batch->n_particles;
    const size_t ws_bytes = P > 0 ? soft_ws_need(P, soft->n_grid, soft->B) : 0;
    if (P > 0 && hipMalloc(&g->soft_ws, ws_bytes) != hipSuccess) {
        delete g;
        return MATCHA_ERR_HIP;
    }
    auto fail = [&](matcha_status e) {
        if (g->soft_ws) (void)hipFree(g->soft_ws);
        if (g->by_L) (void)hipFree(g->by_L);
        delete g;
        return e;
    };
    if (P > 0 && lo != hi && hipMalloc(&g->by_L, sizeof(int32_t) * (size_t)P) != hipSuccess) return fail(MATCHA_ERR_HIP);
    if (P > 0) {
        st = assemble_check(batch, f, h, w, C, prec, hi, rmax);
        if (st != MATCHA_OK) return fail(st);
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(MATCHA_ERR_HIP);
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail(MATCHA_ERR_HIP);
    }
    if (P > 0) st = assemble_ws(ctx, batch, f, h, w, C, prec, lo, hi, rmax, g->by_L, cs);
    if (st == MATCHA_OK && P > 0) st = soft_search_ws(ctx, batch, C, soft, cand, status, nt, g->soft_ws, ws_bytes, cs);
    if (st == MATCHA_OK) st = matcha_march_newton(ctx, batch, C, march, soft->Kc, cand, best, best_idx, status, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (st != MATCHA_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(st != MATCHA_OK ? st : MATCHA_ERR_HIP);
    }
    if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(MATCHA_ERR_HIP);
    }
    g->graph = graph;
    *out = g;
    return MATCHA_OK;
}

matcha_status matcha_graph_launch(matcha_graph *g, void *stream)
{
    if (!g || !g->exec) return MATCHA_ERR_INVALID_ARG;
    return launched(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_graph_destroy(matcha_graph *g)
{
    if (!g) return MATCHA_ERR_INVALID_ARG;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->soft_ws || g->by_L) {
        (void)hipSetDevice(g->device);
        (void)hipDeviceSynchronize();  // replays may still read them
        if (g->soft_ws) (void)hipFree(g->soft_ws);
        if (g->by_L) (void)hipFree(g->by_L);
    }
    delete g;
    return MATCHA_OK;
}

matcha_status matcha_autotune(matcha_ctx *ctx, const matcha_batch *batch, const float *C, const matcha_soft_cfg *soft,
                              const matcha_march_cfg *march, float *cand, float *best, int32_t *best_idx,
                              uint32_t *status, int32_t reps, matcha_tuning *best_tuning)
{
    if (!ctx || !soft || !march || !best_tuning || reps < 1) return MATCHA_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return MATCHA_ERR_HIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return MATCHA_ERR_HIP;
    }
    const matcha_tuning saved = ctx->tune;
    matcha_status st = MATCHA_OK;
    auto time_it = [&](auto &&run, float *ms) -> matcha_status {
        matcha_status r = run();  // warm-up
        if (r != MATCHA_OK) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return MATCHA_ERR_HIP;
        for (int i = 0; i < reps; ++i)
            if ((r = run()) != MATCHA_OK) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return MATCHA_ERR_HIP;
        return hipEventElapsedTime(ms, e0, e1) == hipSuccess ? MATCHA_OK : MATCHA_ERR_HIP;
    };
    matcha_tuning best_t = saved;
    // SOFFT workgroup size
    float best_ms = 1e30f;
    for (int nt : {256, 512}) {
        ctx->tune.soft_threads = nt;
        float ms = 0.f;
        st = time_it([&] { return matcha_soft_search(ctx, batch, C, soft, cand, status, s); }, &ms);
        if (st == MATCHA_ERR_UNSUPPORTED) {  // this shape does not fit the workgroup's LDS
            st = MATCHA_OK;
            continue;
        }
        if (st != MATCHA_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best_t.soft_threads = nt;
        }
    }
    // march candidates per wave (each trial re-runs the search so that it starts from fresh candidates)
    ctx->tune.soft_threads = best_t.soft_threads;
    best_ms = 1e30f;
    for (int nc : {2, 4, 8}) {
        if (st != MATCHA_OK) break;
        if ((soft->Kc + nc - 1) / nc > 8) continue;
        ctx->tune.march_nc = nc;
        float ms = 0.f;
        st = time_it(
            [&] {
                matcha_status r = matcha_soft_search(ctx, batch, C, soft, cand, status, s);
                return r == MATCHA_OK ? matcha_march_newton(ctx, batch, C, march, soft->Kc, cand, best, best_idx, status, s)
                                      : r;
            },
            &ms);
        if (st == MATCHA_OK && ms < best_ms) {
            best_ms = ms;
            best_t.march_nc = nc;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    ctx->tune = st == MATCHA_OK ? best_t : saved;
    *best_tuning = ctx->tune;
    return st;
}

}  // extern "C"
