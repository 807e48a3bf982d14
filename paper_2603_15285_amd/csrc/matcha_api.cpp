// matcha_api.cpp -- the C ABI of libmatcha (include/matcha.h): argument validation,
// read-only table construction, workspace layout, launch sizing, the tune cache.  Everything
// numerical runs in the kernels.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/matcha.h"
#include "matcha_ball.hpp"
#include "matcha_launch.hpp"

using namespace matcha;

namespace {

// SOFFT node tables of one prepared (B, n) shape.
struct GridTables {
    int B = 0, n = 0;
    float2 *dgrid = nullptr;  // weighted d^l(b_i) per node and wedge pair (build_grid_table)
    float *dft = nullptr;     // DFT tables of the grid kernel (build_soft_dft)
};

// 3-D FFT plans of one prepared (N, batch): real-to-half-complex and back, work area from the caller.
struct FftPlans {
    int N = 0, P = 0;
    hipfftHandle r2c = 0, c2r = 0;
    size_t work = 0;
};

// Ball-harmonic tables of one prepared (N, Lambda) (k_ball.hip).
struct BallTables {
    int N = 0;
    double lam = 0.0;
    BallIndex ix;
    int64_t Vo = 0, Vo_pad = 0;
    int col_off[9] = {0};
    int n_entries = 0;  // Kmax (L+1)^2
    int32_t *oct = nullptr;
    float *T = nullptr;
    BallMapEntry *map = nullptr;
};

}  // namespace

// The workspace of matcha_soft_search_noalloc: one array per device, held until the process ends.
// Host code never uses this name as an address; it uses the per-device pointer from
// hipGetSymbolAddress (noalloc_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[MATCHA_NOALLOC_SCRATCH_BYTES];

struct matcha_ctx {
    int device = 0;
    int n_cu = 0;
    void *scratch = nullptr;  // this device's address of `scratch`
    // recurrence tables for every l <= kMaxL, built by matcha_create
    float4 *tab = nullptr;
    double2 *tab64 = nullptr;  // (A, AC) of tab in FP64
    PairInfo *pinfo = nullptr;
    std::vector<GridTables> grids;  // every prepared (B, n); freed by matcha_destroy only
    std::vector<BallTables> balls;  // every prepared (N, Lambda); freed by matcha_destroy only
    std::vector<FftPlans> ffts;     // every prepared (N, batch); destroyed by matcha_destroy only
    matcha_tuning tune{0, 0, 0, 0, 0};
    std::string tune_path;  // tune cache file, empty: none
    std::map<std::string, matcha_tuning> tune_cache;
    std::string arch;  // device name and compute-unit count, part of every tune cache key
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


const GridTables *find_grid(const matcha_ctx *ctx, int B, int n)
{
    for (const GridTables &g : ctx->grids)
        if (g.B == B && g.n == n) return &g;
    return nullptr;
}

template <typename T>
matcha_status upload(const std::vector<T> &host, T **dev)
{
    *dev = nullptr;
    if (hipMalloc(dev, host.size() * sizeof(T)) != hipSuccess) {
        *dev = nullptr;
        return MATCHA_ERR_HIP;
    }
    if (hipMemcpy(*dev, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(*dev);
        *dev = nullptr;
        return MATCHA_ERR_HIP;
    }
    return MATCHA_OK;
}

void free_tables(matcha_ctx *ctx)
{
    if (ctx->tab) (void)hipFree(ctx->tab);
    if (ctx->tab64) (void)hipFree(ctx->tab64);
    if (ctx->pinfo) (void)hipFree(ctx->pinfo);
    for (GridTables &g : ctx->grids) {
        if (g.dgrid) (void)hipFree(g.dgrid);
        if (g.dft) (void)hipFree(g.dft);
    }
    ctx->grids.clear();
    for (BallTables &b : ctx->balls) {
        if (b.oct) (void)hipFree(b.oct);
        if (b.T) (void)hipFree(b.T);
        if (b.map) (void)hipFree(b.map);
    }
    ctx->balls.clear();
    for (FftPlans &q : ctx->ffts) {
        if (q.r2c) (void)hipfftDestroy(q.r2c);
        if (q.c2r) (void)hipfftDestroy(q.c2r);
    }
    ctx->ffts.clear();
    ctx->tab = nullptr;
    ctx->tab64 = nullptr;
    ctx->pinfo = nullptr;
}

// ---- workspace layouts (every region 256-byte aligned) ----------------------------------
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// The SOFFT search of a particle keeps in the workspace, between its kernels: the Wigner
// transforms of its n polar nodes ((B+1)(2B+1) complex each), its grid (n^3 floats) and its list
// of maxima keys with their count.  A chunk of pc particles lays out: the grids, pc lists of
// kSoftListMax keys, pc counts, the Wigner transforms.  matcha_workspace_size offers one chunk of
// the whole batch up to kSoftWsCap; a smaller workspace runs the batch in more chunks.
constexpr size_t kSoftWsCap = (size_t)4 << 30;
constexpr size_t kSoftListMax = 1024;  // keys per particle: the larger select workgroup's list

size_t soft_grid_bytes(int n) { return (size_t)n * n * n * sizeof(float); }
size_t soft_s_bytes(int n, int B) { return (size_t)n * (B + 1) * (2 * B + 1) * sizeof(float2); }
size_t soft_particle_bytes(int n, int B)
{
    return soft_grid_bytes(n) + kSoftListMax * sizeof(unsigned long long) + sizeof(uint32_t) + soft_s_bytes(n, B);
}

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

// Assembly of mixed L_p: the particle order by decreasing L_p, P int32 at the head of ws.
size_t assemble_ws_need(int P, bool mixed) { return mixed ? sizeof(int32_t) * (size_t)P : 0; }

// The persistent march's work counter at the head of ws.
constexpr size_t kMarchWs = 256;

// Adjoint: P int64 offsets of the particles' template terms (packed by the library, whatever
// f_offset is), the partial sums of the segments of particles (grad_segments of them, each
// R_h (L_h+1)^2 complex float32), then the terms, R_p (L_p+1)^2 complex float32 each.
size_t grad_terms(const matcha_batch *b)
{
    size_t n = 0;
    for (int p = 0; p < b->n_particles; ++p)
        n += (size_t)b->R_host[p] * (size_t)(b->L_host[p] + 1) * (size_t)(b->L_host[p] + 1);
    return n;
}
size_t grad_part_bytes(const matcha_batch *b)
{
    const int64_t E = (int64_t)b->R_h * (b->L_h + 1) * (b->L_h + 1);
    return align256((size_t)grad_segments(E, b->n_particles) * (size_t)E * sizeof(float2));
}
size_t grad_ws_need(const matcha_batch *b)
{
    return align256(sizeof(int64_t) * (size_t)b->n_particles) + grad_part_bytes(b) + grad_terms(b) * sizeof(float2);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Device address of `scratch` on `device` (current), looked up once per device.
matcha_status noalloc_scratch_ptr(int device, void **out)
{
    constexpr int kDevices = 64;
    static std::mutex mu;
    static void *ptr[kDevices] = {};
    if (device < 0 || device >= kDevices) return MATCHA_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MATCHA_ERR_HIP;
        ptr[device] = p;
    }
    *out = ptr[device];
    return MATCHA_OK;
}

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
matcha_status assemble_launch(matcha_ctx *ctx, const matcha_batch *batch, const void *f, const void *h,
                              const float *w, float *C, matcha_precision prec, int lo, int hi, int rmax,
                              int32_t *by_L, hipStream_t s)
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
        b.tiles_per_wave = ctx->tune.asm_tiles;
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
    a.tiles_per_wave = ctx->tune.asm_tiles;
    if (mixed) {
        a.by_L = by_L;
        std::memcpy(a.np_l, np_l, sizeof(int) * (size_t)(hi + 1));
    }
    return launched(launch_assemble_f32(a, P, hi, rmax, s));
}

// The smallest workspace of a search: one particle's share.
size_t soft_ws_min(int n, int B) { return soft_chunk(1, n, B).total; }

// Checks of a SOFFT search, in the order batch, configuration and buffers, workspace, context (so
// that the host-side checks need no device); on success *nt is the select kernel's workgroup size
// and *gt the prepared tables.
matcha_status soft_check(const matcha_ctx *ctx, const matcha_batch *batch, const float *C, const matcha_soft_cfg *cfg,
                         const float *cand, const uint32_t *status, const void *ws, size_t ws_bytes, int *nt,
                         const GridTables **gt)
{
    int lo, hi, rmax;
    if (!cfg) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    const int B = cfg->B, n = cfg->n_grid, Kc = cfg->Kc;
    if (B < 1 || B > 32 || n < 4 || n > 96 || Kc < 1 || Kc > MATCHA_MAX_KC) return MATCHA_ERR_INVALID_ARG;
    if (batch->n_particles == 0) return ctx ? MATCHA_OK : MATCHA_ERR_INVALID_ARG;
    if (!C || !cand || !status || !aligned16(C) || !aligned16(cand) || B > lo) return MATCHA_ERR_INVALID_ARG;
    if (!ws || !aligned16(ws) || ws_bytes < soft_ws_min(n, B)) return MATCHA_ERR_WORKSPACE;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    *nt = ctx->tune.soft_threads ? ctx->tune.soft_threads : 256;
    if (soft_grid_smem_bytes(n, B) > 160 * 1024 || soft_select_smem_bytes(n, *nt) > 160 * 1024)
        return MATCHA_ERR_UNSUPPORTED;
    *gt = find_grid(ctx, B, n);
    return *gt ? MATCHA_OK : MATCHA_ERR_NOT_PREPARED;
}

// The search proper over a workspace of ws_bytes (at least one particle's share).
matcha_status soft_launch(const matcha_ctx *ctx, const matcha_batch *batch, const float *C, const matcha_soft_cfg *cfg,
                          const GridTables *gt, float *cand, uint32_t *status, int nt, void *ws, size_t ws_bytes,
                          hipStream_t s)
{
    const int P = batch->n_particles, n = cfg->n_grid, B = cfg->B;
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
    a.dgrid = gt->dgrid;
    a.dft = gt->dft;
    a.pinfo = ctx->pinfo;
    a.B = B;
    a.n = n;
    a.Kc = cfg->Kc;
    a.grid_nodes = ctx->tune.grid_nodes;
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

// Checks of the march configuration.
matcha_status march_check(const matcha_batch *batch, const matcha_march_cfg *cfg, int32_t Kc, int lo)
{
    if (Kc < 1 || Kc > MATCHA_MAX_KC || cfg->steps < 0 || cfg->n_levels < 1 || cfg->n_levels > MATCHA_MAX_LEVELS ||
        !cfg->levels || !(cfg->max_step >= 0.0) || !(cfg->gd_rate >= 0.0) || lo < 1)
        return MATCHA_ERR_INVALID_ARG;
    if (cfg->C_final && !aligned16(cfg->C_final)) return MATCHA_ERR_INVALID_ARG;
    if (cfg->early_stop && !(cfg->tol_grad >= 0.0 && cfg->tol_step >= 0.0 && cfg->tol_rel >= 0.0))
        return MATCHA_ERR_INVALID_ARG;
    for (int j = 0; j < cfg->n_levels; ++j) {
        if (cfg->levels[j] < 1 || cfg->levels[j] > MATCHA_MAX_L) return MATCHA_ERR_INVALID_ARG;
        if (j > 0 && cfg->levels[j] <= cfg->levels[j - 1]) return MATCHA_ERR_INVALID_ARG;
    }
    (void)batch;
    return MATCHA_OK;
}

// ---- tune cache --------------------------------------------------------------------------
// One line per entry: "<key> <march_nc> <soft_threads>".  The key names the device and every
// input of the timing: the batch's size and band / shell statistics, the search shape and the
// march schedule.
std::string tune_key(const matcha_ctx *ctx, const matcha_batch *b, const matcha_soft_cfg *soft,
                     const matcha_march_cfg *march, matcha_precision prec)
{
    long long sL = 0, sR = 0;
    int lo = 1 << 30, hi = -1, rlo = 1 << 30, rhi = -1;
    for (int p = 0; p < b->n_particles; ++p) {
        sL += b->L_host[p];
        sR += b->R_host[p];
        lo = std::min(lo, b->L_host[p]);
        hi = std::max(hi, b->L_host[p]);
        rlo = std::min(rlo, b->R_host[p]);
        rhi = std::max(rhi, b->R_host[p]);
    }
    std::string k = ctx->arch + "|P" + std::to_string(b->n_particles) + "|L" + std::to_string(lo) + "," +
                    std::to_string(hi) + "," + std::to_string(sL) + "|R" + std::to_string(rlo) + "," +
                    std::to_string(rhi) + "," + std::to_string(sR) + "|ord" + std::to_string(b->order ? 1 : 0) +
                    "|B" + std::to_string(soft->B) + ",n" + std::to_string(soft->n_grid) + ",K" +
                    std::to_string(soft->Kc) + "|lv";
    for (int j = 0; j < march->n_levels; ++j) k += (j ? "," : "") + std::to_string(march->levels[j]);
    k += "|s" + std::to_string(march->steps) + "|f64_" + std::to_string(march->fp64_above) + "|es" +
         std::to_string(march->early_stop) + "|pr" + std::to_string((int)prec) + (march->gd_rate > 0.0 ? "|gd" : "");
    for (char &c : k)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    return k;
}

void tune_cache_load(matcha_ctx *ctx)
{
    FILE *fp = std::fopen(ctx->tune_path.c_str(), "r");
    if (!fp) return;
    char line[4096];
    while (std::fgets(line, sizeof line, fp)) {
        char key[4000];
        matcha_tuning t{0, 0, 0, 0, 0};
        if (std::sscanf(line, "%3999s %d %d %d %d %d", key, &t.march_nc, &t.soft_threads, &t.asm_tiles, &t.grid_nodes,
                        &t.march_persistent) == 6)
            ctx->tune_cache[key] = t;
    }
    std::fclose(fp);
}

bool tune_cache_store(const matcha_ctx *ctx, const std::string &key, const matcha_tuning &t)
{
    if (ctx->tune_path.empty()) return true;
    FILE *fp = std::fopen(ctx->tune_path.c_str(), "a");
    if (!fp) return false;
    std::fprintf(fp, "%s %d %d %d %d %d\n", key.c_str(), t.march_nc, t.soft_threads, t.asm_tiles, t.grid_nodes,
                 t.march_persistent);
    return std::fclose(fp) == 0;
}

const FftPlans *find_fft(const matcha_ctx *ctx, int N, int P)
{
    for (const FftPlans &q : ctx->ffts)
        if (q.N == N && q.P == P) return &q;
    return nullptr;
}

// Refinement offsets per axis for an upsampling factor kappa: +-0.75 voxel around the integer peak.
int ups_points(int kappa) { return 2 * ((3 * kappa + 3) / 4) + 1; }

struct TransWs {
    size_t vol = 0, spec = 0, spec2 = 0, ups = 0, utab = 0, peak = 0, work = 0, total = 0;
};

// Workspace layout of the translation calls for P volumes: rotated templates / correlations
// [P][N^3] float, a spectrum [P][N][N][N/2+1] complex, the refinement partials [P][N][m][m] complex,
// the refinement's phase tables [P][(N/2+1) + N][m] complex, the integer peaks [P] int4, the FFT work
// area; each region 256-byte aligned.  The search also
// keeps a second spectrum (the cross spectrum's copy that the inverse transform consumes).
TransWs trans_ws(int N, int P, int kappa, size_t fft_work)
{
    TransWs w;
    const size_t n3 = (size_t)N * N * N, nh = (size_t)N * N * (N / 2 + 1);
    const int m = ups_points(kappa);
    w.vol = 0;
    w.spec = w.vol + align256(sizeof(float) * n3 * P);
    w.spec2 = w.spec + align256(sizeof(float2) * nh * P);
    w.ups = w.spec2 + align256(sizeof(float2) * nh * P);
    w.utab = w.ups + align256(sizeof(float2) * (size_t)N * m * m * P);
    w.peak = w.utab + align256(sizeof(float2) * (size_t)(N / 2 + 1 + N) * m * P);
    w.work = w.peak + align256(sizeof(int4) * (size_t)P);
    w.total = w.work + align256(fft_work);
    return w;
}

const BallTables *find_ball(const matcha_ctx *ctx, int N, double lam)
{
    for (const BallTables &b : ctx->balls)
        if (b.N == N && b.lam == lam) return &b;
    return nullptr;
}

// The index set of Lambda within what the transform supports (degrees <= MATCHA_BALL_MAX_L).
matcha_status ball_index_checked(double lam, BallIndex &ix)
{
    if (!(lam > 0.0) || !(lam <= MATCHA_BALL_MAX_LAMBDA)) return MATCHA_ERR_INVALID_ARG;
    if (!ball_index(lam, ix)) return MATCHA_ERR_INVALID_ARG;
    if (ix.L > MATCHA_BALL_MAX_L) return MATCHA_ERR_UNSUPPORTED;
    return MATCHA_OK;
}

// Columns of the transform of ix: sum_l |K_l| (2l + 1) (Re for m = 0..l, Im for m = 1..l).
int64_t ball_columns(const BallIndex &ix)
{
    int64_t n = 0;
    for (int l = 0; l <= ix.L; ++l) n += (int64_t)ix.zeros[(size_t)l].size() * (2 * l + 1);
    return n;
}

// Octant voxels of the N^3 grid inside the ball (coordinates >= 0, centre strictly inside).
int64_t ball_octant_voxels(int N)
{
    int64_t V = 0;
    for (int i = N / 2; i < N; ++i)
        for (int j = N / 2; j < N; ++j)
            for (int k = N / 2; k < N; ++k) {
                const double z = -1.0 + (2.0 / N) * (i + 0.5), y = -1.0 + (2.0 / N) * (j + 0.5),
                             x = -1.0 + (2.0 / N) * (k + 0.5);
                V += std::sqrt(x * x + y * y + z * z) < 1.0;
            }
    return V;
}

// Split count and workspace bytes of a transform of P volumes: the symmetrised volumes
// [8][P][Vo_pad] and the partial sums [S][P][ncol], each 256-byte aligned.
int ball_split_count(const matcha_ctx *ctx, const BallTables &t, int P)
{
    return ball_splits(P, ball_col_tiles(t.col_off, nullptr), t.Vo_pad, ctx->n_cu > 0 ? ctx->n_cu : 256);
}

size_t ball_ws_need(const matcha_ctx *ctx, const BallTables &t, int P)
{
    if (P <= 0) return 0;
    const int S = ball_split_count(ctx, t, P);
    return align256(sizeof(float) * 8 * (size_t)P * (size_t)t.Vo_pad) +
           align256(sizeof(float) * (size_t)S * (size_t)P * (size_t)t.col_off[8]);
}

}  // namespace

extern "C" {

matcha_status matcha_create(int device, const char *tune_cache, matcha_ctx **out)
{
    if (!out) return MATCHA_ERR_INVALID_ARG;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return MATCHA_ERR_HIP;
    if (device < 0 || device >= n) return MATCHA_ERR_INVALID_ARG;
    matcha_ctx *c = new (std::nothrow) matcha_ctx();
    if (!c) return MATCHA_ERR_HIP;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return MATCHA_ERR_HIP;
    }
    c->arch = std::string(prop.gcnArchName) + "_cu" + std::to_string(prop.multiProcessorCount);
    c->n_cu = prop.multiProcessorCount;
    if (noalloc_scratch_ptr(device, &c->scratch) != MATCHA_OK) {
        delete c;
        return MATCHA_ERR_HIP;
    }
    std::vector<float4> tab;
    std::vector<double2> tab64;
    std::vector<PairInfo> pinfo;
    build_tables(kMaxL, tab, tab64, pinfo);
    if (upload(tab, &c->tab) != MATCHA_OK || upload(tab64, &c->tab64) != MATCHA_OK ||
        upload(pinfo, &c->pinfo) != MATCHA_OK) {
        free_tables(c);
        delete c;
        return MATCHA_ERR_HIP;
    }
    if (tune_cache && tune_cache[0]) {
        c->tune_path = tune_cache;
        tune_cache_load(c);
    }
    *out = c;
    return MATCHA_OK;
}

matcha_status matcha_destroy(matcha_ctx *ctx)
{
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();  // enqueued work may still read the tables
    free_tables(ctx);
    delete ctx;
    return MATCHA_OK;
}

matcha_status matcha_prepare(matcha_ctx *ctx, int32_t B, int32_t n_grid)
{
    if (!ctx || B < 1 || B > 32 || n_grid < 4 || n_grid > 96) return MATCHA_ERR_INVALID_ARG;
    if (find_grid(ctx, B, n_grid)) return MATCHA_OK;
    std::vector<float2> g;
    build_grid_table(B, n_grid, g);
    std::vector<float> e(soft_dft_floats(n_grid, B));
    build_soft_dft(B, n_grid, e.data());
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    GridTables t;
    t.B = B;
    t.n = n_grid;
    if (upload(g, &t.dgrid) != MATCHA_OK) return MATCHA_ERR_HIP;
    if (upload(e, &t.dft) != MATCHA_OK) {
        (void)hipFree(t.dgrid);
        return MATCHA_ERR_HIP;
    }
    ctx->grids.push_back(t);
    return MATCHA_OK;
}

const char *matcha_status_string(matcha_status s)
{
    switch (s) {
    case MATCHA_OK: return "ok";
    case MATCHA_ERR_INVALID_ARG: return "invalid argument";
    case MATCHA_ERR_UNSUPPORTED: return "unsupported configuration";
    case MATCHA_ERR_HIP: return "HIP runtime error";
    case MATCHA_ERR_WORKSPACE: return "workspace too small";
    case MATCHA_ERR_NOT_PREPARED: return "SOFFT shape not prepared (call matcha_prepare)";
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
    const int at = t->asm_tiles;
    if (at != 0 && at != 1 && at != 2 && at != 4 && at != 8) return MATCHA_ERR_INVALID_ARG;
    const int gn = t->grid_nodes;
    if (gn != 0 && gn != 8 && gn != 16 && gn != 32 && gn != 48 && gn != 64) return MATCHA_ERR_INVALID_ARG;
    if (t->march_persistent != 0 && t->march_persistent != 1) return MATCHA_ERR_INVALID_ARG;
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

size_t matcha_workspace_size(const matcha_ctx *ctx, const matcha_batch *batch, const matcha_soft_cfg *soft,
                             const matcha_march_cfg *march)
{
    (void)ctx;
    (void)march;
    int lo, hi, rmax;
    if (check_batch(batch, &lo, &hi, &rmax) != MATCHA_OK || batch->n_particles == 0) return 0;
    size_t need = std::max(assemble_ws_need(batch->n_particles, lo != hi), kMarchWs);
    if (soft && soft->B >= 1 && soft->n_grid >= 4)
        need = std::max(need, soft_ws_need(batch->n_particles, soft->n_grid, soft->B));
    return need;
}

size_t matcha_grad_workspace_size(const matcha_batch *batch)
{
    int lo, hi, rmax;
    if (check_batch(batch, &lo, &hi, &rmax) != MATCHA_OK || batch->n_particles == 0) return 0;
    return grad_ws_need(batch);
}

matcha_status matcha_c_unpack(int32_t L, const float *C_wedge_host, float *C_byl_host)
{
    if (L < 0 || L > MATCHA_MAX_L || !C_wedge_host || !C_byl_host) return MATCHA_ERR_INVALID_ARG;
    typedef std::complex<float> cf;
    const cf *wv = reinterpret_cast<const cf *>(C_wedge_host);
    cf *out = reinterpret_cast<cf *>(C_byl_host);
    for (int l = 0; l <= L; ++l) {
        const int64_t blk = (int64_t)l * (4 * l * l - 1) / 3, w = 2 * l + 1;
        std::vector<char> set((size_t)(w * w), 0);
        auto put = [&](int m, int n, cf v) {
            out[blk + (m + l) * w + (n + l)] = v;
            set[(size_t)((m + l) * w + (n + l))] = 1;
        };
        for (int m = 0; m <= l; ++m)
            for (int n = -m; n <= m; ++n) {
                const int64_t q = (int64_t)m * m + m + n, at = 2 * (wedge_row(l) + q);
                put(m, n, wv[at]);
                const int pm = n >= 0 ? n : -n, pn = n >= 0 ? m : -m;
                if (pm != m || pn != n) put(pm, pn, wv[at + 1]);
            }
        // the rest by C^l_{-m,-n} = (-1)^{m-n} conj(C^l_mn)
        for (int m = -l; m <= l; ++m)
            for (int n = -l; n <= l; ++n)
                if (!set[(size_t)((m + l) * w + (n + l))]) {
                    const cf v = std::conj(out[blk + (-m + l) * w + (-n + l)]);
                    out[blk + (m + l) * w + (n + l)] = ((m - n) & 1) ? -v : v;
                }
    }
    return MATCHA_OK;
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

matcha_status matcha_coeff_assemble(matcha_ctx *ctx, const matcha_batch *batch, const void *f, const void *h,
                                    const float *w, float *C, matcha_precision prec, void *ws, size_t ws_bytes,
                                    void *stream)
{
    int lo, hi, rmax;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return ctx ? MATCHA_OK : MATCHA_ERR_INVALID_ARG;
    st = assemble_check(batch, f, h, w, C, prec, hi, rmax);
    if (st != MATCHA_OK) return st;
    const size_t need = assemble_ws_need(batch->n_particles, lo != hi);
    if (need && (!ws || ws_bytes < need || !aligned16(ws))) return MATCHA_ERR_WORKSPACE;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    return assemble_launch(ctx, batch, f, h, w, C, prec, lo, hi, rmax, static_cast<int32_t *>(ws),
                           static_cast<hipStream_t>(stream));
}

matcha_status matcha_soft_search(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                 const matcha_soft_cfg *cfg, float *cand, uint32_t *status, void *ws, size_t ws_bytes,
                                 void *stream)
{
    int nt = 0;
    const GridTables *gt = nullptr;
    matcha_status st = soft_check(ctx, batch, C, cfg, cand, status, ws, ws_bytes, &nt, &gt);
    if (st != MATCHA_OK || batch->n_particles == 0) return st;
    return soft_launch(ctx, batch, C, cfg, gt, cand, status, nt, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

matcha_status matcha_soft_search_noalloc(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                         const matcha_soft_cfg *cfg, float *cand, uint32_t *status, void *stream)
{
    if (!ctx || !ctx->scratch) return MATCHA_ERR_INVALID_ARG;
    int nt = 0;
    const GridTables *gt = nullptr;
    matcha_status st = soft_check(ctx, batch, C, cfg, cand, status, ctx->scratch, MATCHA_NOALLOC_SCRATCH_BYTES, &nt,
                                  &gt);
    if (st != MATCHA_OK || batch->n_particles == 0) return st;
    return soft_launch(ctx, batch, C, cfg, gt, cand, status, nt, ctx->scratch, MATCHA_NOALLOC_SCRATCH_BYTES,
                       static_cast<hipStream_t>(stream));
}

matcha_status matcha_march_newton(matcha_ctx *ctx, const matcha_batch *batch, const float *C,
                                  const matcha_march_cfg *cfg, int32_t Kc, float *cand, float *best,
                                  int32_t *best_idx, uint32_t *status, void *ws, size_t ws_bytes, void *stream)
{
    int lo, hi, rmax;
    if (!cfg) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (batch->n_particles == 0) return ctx ? MATCHA_OK : MATCHA_ERR_INVALID_ARG;
    if (!C || !cand || !best || !best_idx || !status || !aligned16(C) || !aligned16(cand) || !aligned16(best))
        return MATCHA_ERR_INVALID_ARG;
    st = march_check(batch, cfg, Kc, lo);
    if (st != MATCHA_OK) return st;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    const bool persist = ctx->tune.march_persistent != 0;
    if (persist && (!ws || !aligned16(ws) || ws_bytes < kMarchWs)) return MATCHA_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    MarchArgs a;
    std::memset(&a, 0, sizeof a);
    a.C = reinterpret_cast<const float4 *>(C);
    a.C_fin = reinterpret_cast<const float4 *>(cfg->C_final);
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
    a.gd_rate = cfg->gd_rate;
    a.Kc = Kc;
    a.cand = reinterpret_cast<float4 *>(cand);
    a.best = reinterpret_cast<float4 *>(best);
    a.best_idx = best_idx;
    a.status = status;
    a.order = batch->order;
    a.queue = persist ? static_cast<int *>(ws) : nullptr;
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
    if (L_eval < 0 || L_eval > lo) return MATCHA_ERR_INVALID_ARG; /* 0: each particle's own L_p */
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
                                   matcha_precision prec, void *ws, size_t ws_bytes, void *stream)
{
    int lo, hi, rmax;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (prec != MATCHA_FP32) return MATCHA_ERR_UNSUPPORTED;
    if (batch->n_particles == 0) return ctx ? MATCHA_OK : MATCHA_ERR_INVALID_ARG;
    if (!f || !h || !w || !best || !g || !batch->f_offset || !aligned16(best)) return MATCHA_ERR_INVALID_ARG;
    if (grad_h && (!ws || !aligned16(ws) || ws_bytes < grad_ws_need(batch))) return MATCHA_ERR_WORKSPACE;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    if (!grad_h && !grad_f) return MATCHA_OK;
    if (grad_smem_bytes(hi) > 160 * 1024) return MATCHA_ERR_UNSUPPORTED;
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
    if (grad_h) {
        char *base = static_cast<char *>(ws);
        const size_t off_bytes = align256(sizeof(int64_t) * (size_t)a.P);
        a.ws_off = reinterpret_cast<int64_t *>(base);
        a.part = reinterpret_cast<float2 *>(base + off_bytes);
        a.ws = reinterpret_cast<float2 *>(base + off_bytes + grad_part_bytes(batch));
    }
    a.pinfo = ctx->pinfo;
    a.tab = ctx->tab;
    return launched(launch_grad(a, static_cast<hipStream_t>(stream)));
}

matcha_status matcha_lowrank_spectrum(matcha_ctx *ctx, const matcha_batch *batch, const float *f, const float *h,
                                      const float *w, double rho, int32_t n_sv, double *sv, int32_t *r_eff,
                                      void *stream)
{
    int lo, hi, rmax;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    if (!(rho > 0.0 && rho < 1.0) || n_sv < 1 || n_sv > 64) return MATCHA_ERR_INVALID_ARG;
    if (batch->n_particles == 0) return ctx ? MATCHA_OK : MATCHA_ERR_INVALID_ARG;
    if (!f || !h || !w || !sv || !r_eff || !batch->f_offset) return MATCHA_ERR_INVALID_ARG;
    if (rmax > MATCHA_LOWRANK_MAX_SHELLS) return MATCHA_ERR_UNSUPPORTED;
    if (!ctx) return MATCHA_ERR_INVALID_ARG;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    LowRankArgs a;
    std::memset(&a, 0, sizeof a);
    a.f = reinterpret_cast<const float2 *>(f);
    a.f_off = batch->f_offset;
    a.h = reinterpret_cast<const float2 *>(h);
    a.w = w;
    a.Lp = batch->L_dev;
    a.Rp = batch->R_dev;
    a.Lh = batch->L_h;
    a.L_max = hi;
    a.R_max = rmax;
    a.P = batch->n_particles;
    a.rho = rho;
    a.sv = sv;
    a.r_eff = r_eff;
    a.n_sv = n_sv;
    return launched(launch_lowrank(a, static_cast<hipStream_t>(stream)));
}

struct matcha_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

matcha_status matcha_align_graph_create(matcha_ctx *ctx, const matcha_batch *batch, const matcha_align_bufs *bufs,
                                        const matcha_soft_cfg *soft, const matcha_march_cfg *march, void *ws,
                                        size_t ws_bytes, matcha_graph **out)
{
    int lo, hi, rmax;
    if (!ctx || !bufs || !soft || !march || !out) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    const bool fin = bufs->f32 || bufs->h32;
    if (fin && (!bufs->f32 || !bufs->h32 || !bufs->C32)) return MATCHA_ERR_INVALID_ARG;
    const int P = batch->n_particles;
    int nt = 0;
    const GridTables *gt = nullptr;
    st = soft_check(ctx, batch, bufs->C, soft, bufs->cand, bufs->status, ws, ws_bytes, &nt, &gt);
    if (st != MATCHA_OK) return st;
    if (P > 0) {
        st = assemble_check(batch, bufs->f, bufs->h, bufs->w, bufs->C, bufs->prec, hi, rmax);
        if (st == MATCHA_OK && fin) st = assemble_check(batch, bufs->f32, bufs->h32, bufs->w, bufs->C32, MATCHA_FP32, hi, rmax);
        if (st != MATCHA_OK) return st;
        if (ws_bytes < std::max(assemble_ws_need(P, lo != hi), kMarchWs)) return MATCHA_ERR_WORKSPACE;
    }
    matcha_march_cfg mc = *march;
    mc.C_final = fin ? bufs->C32 : nullptr;
    if (P > 0) {
        st = march_check(batch, &mc, soft->Kc, lo);
        if (st != MATCHA_OK) return st;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    matcha_graph *g = new (std::nothrow) matcha_graph();
    if (!g) return MATCHA_ERR_HIP;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        delete g;
        return MATCHA_ERR_HIP;
    }
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        delete g;
        return MATCHA_ERR_HIP;
    }
    if (P > 0) {
        st = assemble_launch(ctx, batch, bufs->f, bufs->h, bufs->w, bufs->C, bufs->prec, lo, hi, rmax,
                             static_cast<int32_t *>(ws), cs);
        if (st == MATCHA_OK && fin)
            st = assemble_launch(ctx, batch, bufs->f32, bufs->h32, bufs->w, bufs->C32, MATCHA_FP32, lo, hi, rmax,
                                 static_cast<int32_t *>(ws), cs);
        if (st == MATCHA_OK)
            st = soft_launch(ctx, batch, bufs->C, soft, gt, bufs->cand, bufs->status, nt, ws, ws_bytes, cs);
        if (st == MATCHA_OK)
            st = matcha_march_newton(ctx, batch, bufs->C, &mc, soft->Kc, bufs->cand, bufs->best, bufs->best_idx,
                                     bufs->status, ws, ws_bytes, cs);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (st != MATCHA_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        return st != MATCHA_OK ? st : MATCHA_ERR_HIP;
    }
    if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return MATCHA_ERR_HIP;
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
    delete g;
    return MATCHA_OK;
}

matcha_status matcha_autotune(matcha_ctx *ctx, const matcha_batch *batch, const matcha_align_bufs *bufs,
                              const matcha_soft_cfg *soft, const matcha_march_cfg *march, int32_t reps, void *ws,
                              size_t ws_bytes, matcha_tuning *best_tuning)
{
    int lo, hi, rmax;
    if (!ctx || !bufs || !soft || !march || !best_tuning || reps < 1) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = check_batch(batch, &lo, &hi, &rmax);
    if (st != MATCHA_OK) return st;
    const std::string key = tune_key(ctx, batch, soft, march, bufs->prec);
    const auto hit = ctx->tune_cache.find(key);
    if (hit != ctx->tune_cache.end()) {
        st = matcha_set_tuning(ctx, &hit->second);
        if (st == MATCHA_OK) *best_tuning = ctx->tune;
        return st;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return MATCHA_ERR_HIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return MATCHA_ERR_HIP;
    }
    const matcha_tuning saved = ctx->tune;
    auto time_it = [&](auto &&run, float *ms) -> matcha_status {
        matcha_status r = run();  // warm-up
        if (r != MATCHA_OK) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return MATCHA_ERR_HIP;
        for (int i = 0; i < reps; ++i)
            if ((r = run()) != MATCHA_OK) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return MATCHA_ERR_HIP;
        return hipEventElapsedTime(ms, e0, e1) == hipSuccess ? MATCHA_OK : MATCHA_ERR_HIP;
    };
    // one field at a time: try each value with the others at their best so far; shapes a call
    // cannot take (MATCHA_ERR_UNSUPPORTED) are skipped.  Every value is timed in two interleaved
    // rounds and keeps its faster one, so that the first value tried does not pay for the clocks
    // and caches settling (choices a few tenths of a percent apart are otherwise decided by order).
    constexpr int kRounds = 2;
    matcha_tuning best_t = saved;
    auto tune_field = [&](int32_t matcha_tuning::*field, std::initializer_list<int32_t> values, auto &&run) {
        const std::vector<int32_t> vals(values);
        std::vector<float> ms_of(vals.size(), 1e30f);
        for (int round = 0; round < kRounds; ++round)
            for (size_t i = 0; i < vals.size(); ++i) {
                if (st != MATCHA_OK) return;
                ctx->tune = best_t;
                ctx->tune.*field = vals[i];
                float ms = 0.f;
                st = time_it(run, &ms);
                if (st == MATCHA_ERR_UNSUPPORTED) {
                    st = MATCHA_OK;
                    continue;
                }
                if (st == MATCHA_OK) ms_of[i] = std::min(ms_of[i], ms);
            }
        float best_ms = 1e30f;
        for (size_t i = 0; i < vals.size(); ++i)
            if (ms_of[i] < best_ms) {
                best_ms = ms_of[i];
                best_t.*field = vals[i];
            }
    };
    auto assemble = [&] {
        return matcha_coeff_assemble(ctx, batch, bufs->f, bufs->h, bufs->w, bufs->C, bufs->prec, ws, ws_bytes, s);
    };
    auto search = [&] {
        return matcha_soft_search(ctx, batch, bufs->C, soft, bufs->cand, bufs->status, ws, ws_bytes, s);
    };
    auto search_march = [&] {
        matcha_status r = search();
        return r == MATCHA_OK ? matcha_march_newton(ctx, batch, bufs->C, march, soft->Kc, bufs->cand, bufs->best,
                                                    bufs->best_idx, bufs->status, ws, ws_bytes, s)
                              : r;
    };
    tune_field(&matcha_tuning::asm_tiles, {1, 2, 4, 8}, assemble);
    tune_field(&matcha_tuning::soft_threads, {256, 512}, search);
    tune_field(&matcha_tuning::grid_nodes, {8, 16, 32, 48, 64}, search);
    std::vector<int32_t> ncs;
    for (int nc : {2, 4, 8})
        if ((soft->Kc + nc - 1) / nc <= 8) ncs.push_back(nc);
    // candidates per wave and launch form together (the persistent grid's size depends on both)
    {
        std::vector<float> ms_of(ncs.size() * 2, 1e30f);
        const matcha_tuning base = best_t;
        for (int round = 0; round < kRounds; ++round)
            for (size_t i = 0; i < ncs.size(); ++i)
                for (int32_t pers : {0, 1}) {
                    if (st != MATCHA_OK) break;
                    ctx->tune = base;
                    ctx->tune.march_nc = ncs[i];
                    ctx->tune.march_persistent = pers;
                    float ms = 0.f;
                    st = time_it(search_march, &ms);
                    if (st == MATCHA_OK) ms_of[2 * i + pers] = std::min(ms_of[2 * i + pers], ms);
                }
        float best_ms = 1e30f;
        for (size_t k = 0; k < ms_of.size(); ++k)
            if (ms_of[k] < best_ms) {
                best_ms = ms_of[k];
                best_t.march_nc = ncs[k / 2];
                best_t.march_persistent = (int32_t)(k % 2);
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    ctx->tune = st == MATCHA_OK ? best_t : saved;
    if (st == MATCHA_OK) {
        ctx->tune_cache[key] = ctx->tune;
        (void)tune_cache_store(ctx, key, ctx->tune);  // best effort: the context keeps the result either way
    }
    *best_tuning = ctx->tune;
    return st;
}

// ---- translation search (App. C) -------------------------------------------------------------
matcha_status matcha_fft_prepare(matcha_ctx *ctx, int32_t N, int32_t n_volumes)
{
    if (!ctx || N < 4 || N > MATCHA_TRANSLATE_MAX_N || (N & 1) || n_volumes < 1) return MATCHA_ERR_INVALID_ARG;
    if (find_fft(ctx, N, n_volumes)) return MATCHA_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    FftPlans q;
    q.N = N;
    q.P = n_volumes;
    int n[3] = {N, N, N};
    size_t w1 = 0, w2 = 0;
    bool ok = hipfftCreate(&q.r2c) == HIPFFT_SUCCESS && hipfftSetAutoAllocation(q.r2c, 0) == HIPFFT_SUCCESS &&
              hipfftMakePlanMany(q.r2c, 3, n, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_R2C, n_volumes, &w1) ==
                  HIPFFT_SUCCESS;
    ok = ok && hipfftCreate(&q.c2r) == HIPFFT_SUCCESS && hipfftSetAutoAllocation(q.c2r, 0) == HIPFFT_SUCCESS &&
         hipfftMakePlanMany(q.c2r, 3, n, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_C2R, n_volumes, &w2) == HIPFFT_SUCCESS;
    if (!ok) {
        if (q.r2c) (void)hipfftDestroy(q.r2c);
        if (q.c2r) (void)hipfftDestroy(q.c2r);
        return MATCHA_ERR_HIP;
    }
    q.work = std::max(w1, w2);
    ctx->ffts.push_back(q);
    return MATCHA_OK;
}

size_t matcha_translate_workspace_size(const matcha_ctx *ctx, int32_t N, int32_t n_volumes, int32_t upsample)
{
    if (!ctx || upsample < 1 || upsample > MATCHA_TRANSLATE_MAX_UPSAMPLE) return 0;
    const FftPlans *q = find_fft(ctx, N, n_volumes);
    return q ? trans_ws(N, n_volumes, upsample, q->work).total : 0;
}

namespace {

// Checks shared by the translation calls; *q the prepared plans.
matcha_status trans_check(matcha_ctx *ctx, int N, int P, void *ws, size_t ws_bytes, int kappa, const FftPlans **q)
{
    if (!ctx || N < 4 || N > MATCHA_TRANSLATE_MAX_N || (N & 1) || P < 0) return MATCHA_ERR_INVALID_ARG;
    if (P == 0) return MATCHA_OK;
    *q = find_fft(ctx, N, P);
    if (!*q) return MATCHA_ERR_NOT_PREPARED;
    if (!ws || !aligned16(ws) || ws_bytes < trans_ws(N, P, kappa, (*q)->work).total) return MATCHA_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    return MATCHA_OK;
}

matcha_status fft_exec(hipfftHandle plan, void *work, hipStream_t s, const void *in, void *out, bool forward)
{
    if (hipfftSetWorkArea(plan, work) != HIPFFT_SUCCESS || hipfftSetStream(plan, s) != HIPFFT_SUCCESS)
        return MATCHA_ERR_HIP;
    const hipfftResult r =
        forward ? hipfftExecR2C(plan, static_cast<hipfftReal *>(const_cast<void *>(in)), static_cast<hipfftComplex *>(out))
                : hipfftExecC2R(plan, static_cast<hipfftComplex *>(const_cast<void *>(in)), static_cast<hipfftReal *>(out));
    return r == HIPFFT_SUCCESS ? MATCHA_OK : MATCHA_ERR_HIP;
}

}  // namespace

matcha_status matcha_volume_spectrum(matcha_ctx *ctx, int32_t N, int32_t n_volumes, const float *vol, float *spec,
                                     void *ws, size_t ws_bytes, void *stream)
{
    const FftPlans *q = nullptr;
    if (n_volumes > 0 && (!vol || !spec || !aligned16(spec))) return MATCHA_ERR_INVALID_ARG;
    matcha_status st = trans_check(ctx, N, n_volumes, ws, ws_bytes, 1, &q);
    if (st != MATCHA_OK || n_volumes == 0) return st;
    char *base = static_cast<char *>(ws);
    return fft_exec(q->r2c, base + trans_ws(N, n_volumes, 1, q->work).work, static_cast<hipStream_t>(stream), vol, spec,
                    true);
}

matcha_status matcha_shift_volumes(matcha_ctx *ctx, int32_t N, int32_t n_volumes, const float *spec, const float *shifts,
                                   float *out, void *ws, size_t ws_bytes, void *stream)
{
    const FftPlans *q = nullptr;
    if (n_volumes > 0 && (!spec || !shifts || !out || !aligned16(spec) || !aligned16(shifts)))
        return MATCHA_ERR_INVALID_ARG;
    matcha_status st = trans_check(ctx, N, n_volumes, ws, ws_bytes, 1, &q);
    if (st != MATCHA_OK || n_volumes == 0) return st;
    const TransWs w = trans_ws(N, n_volumes, 1, q->work);
    char *base = static_cast<char *>(ws);
    TransArgs a;
    std::memset(&a, 0, sizeof a);
    a.N = N;
    a.P = n_volumes;
    a.spec_in = reinterpret_cast<const float2 *>(spec);
    a.spec_out = reinterpret_cast<float2 *>(base + w.spec);
    a.shift = reinterpret_cast<const float4 *>(shifts);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    st = launched(launch_phase_shift(a, s));
    if (st != MATCHA_OK) return st;
    return fft_exec(q->c2r, base + w.work, s, a.spec_out, out, false);
}

matcha_status matcha_translation_search(matcha_ctx *ctx, int32_t N, int32_t n_volumes, const float *spec_f,
                                        const float *h, const float *euler, int32_t window, int32_t upsample,
                                        float *shift_out, void *ws, size_t ws_bytes, void *stream)
{
    const FftPlans *q = nullptr;
    if (n_volumes > 0 && (!spec_f || !h || !euler || !shift_out || !aligned16(spec_f) || !aligned16(euler) ||
                          !aligned16(shift_out)))
        return MATCHA_ERR_INVALID_ARG;
    if (window < 0 || upsample < 1 || upsample > MATCHA_TRANSLATE_MAX_UPSAMPLE) return MATCHA_ERR_INVALID_ARG;
    if (n_volumes > 65535) return MATCHA_ERR_UNSUPPORTED;  // one grid row per volume
    matcha_status st = trans_check(ctx, N, n_volumes, ws, ws_bytes, upsample, &q);
    if (st != MATCHA_OK || n_volumes == 0) return st;
    const int m = ups_points(upsample);
    if (upsample_xy_smem(N, m) > 64 * 1024) return MATCHA_ERR_UNSUPPORTED;
    const TransWs w = trans_ws(N, n_volumes, upsample, q->work);
    char *base = static_cast<char *>(ws);
    TransArgs a;
    std::memset(&a, 0, sizeof a);
    a.N = N;
    a.P = n_volumes;
    a.h = h;
    a.euler = reinterpret_cast<const float4 *>(euler);
    a.vol = reinterpret_cast<float *>(base + w.vol);
    a.spec_in = reinterpret_cast<const float2 *>(spec_f);
    a.spec_out = reinterpret_cast<float2 *>(base + w.spec);
    a.spec_aux = reinterpret_cast<float2 *>(base + w.spec2);
    a.window = std::min(window, N / 2);
    a.peak = reinterpret_cast<int4 *>(base + w.peak);
    a.ups = reinterpret_cast<float2 *>(base + w.ups);
    a.ups_tab = reinterpret_cast<float2 *>(base + w.utab);
    a.m = m;
    a.kappa = upsample;
    a.shift_out = reinterpret_cast<float4 *>(shift_out);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    void *work = base + w.work;
    if ((st = launched(launch_rotate_volume(a, s))) != MATCHA_OK) return st;
    if ((st = fft_exec(q->r2c, work, s, a.vol, a.spec_out, true)) != MATCHA_OK) return st;
    if ((st = launched(launch_cross_spectrum(a, s))) != MATCHA_OK) return st;
    if ((st = fft_exec(q->c2r, work, s, a.spec_aux, a.vol, false)) != MATCHA_OK) return st;
    return launched(launch_peak_refine(a, s));
}

// ---- ball-harmonic front end ----------------------------------------------------------------
matcha_status matcha_ball_index(double Lambda, int32_t *L, int32_t *Kmax, int32_t *nk_l, double *zeros)
{
    if (!L || !Kmax) return MATCHA_ERR_INVALID_ARG;
    BallIndex ix;
    const matcha_status st = ball_index_checked(Lambda, ix);
    if (st != MATCHA_OK) return st;
    *L = ix.L;
    *Kmax = ix.Kmax;
    for (int l = 0; l <= ix.L; ++l) {
        const auto &z = ix.zeros[(size_t)l];
        if (nk_l) nk_l[l] = (int32_t)z.size();
        if (zeros)
            for (int k = 0; k < ix.Kmax; ++k) zeros[(size_t)l * ix.Kmax + k] = k < (int)z.size() ? z[(size_t)k] : 0.0;
    }
    return MATCHA_OK;
}

matcha_status matcha_ball_prepare(matcha_ctx *ctx, int32_t N, double Lambda)
{
    if (!ctx || N < 2 || N > MATCHA_BALL_MAX_N) return MATCHA_ERR_INVALID_ARG;
    if (find_ball(ctx, N, Lambda)) return MATCHA_OK;
    BallIndex ix;
    matcha_status st = ball_index_checked(Lambda, ix);
    if (st != MATCHA_OK) return st;
    const int64_t Vo_pad = (ball_octant_voxels(N) + kBallChunk - 1) / kBallChunk * kBallChunk;
    if ((size_t)ball_columns(ix) * (size_t)Vo_pad * sizeof(float) > MATCHA_BALL_MAX_TABLE_BYTES)
        return MATCHA_ERR_UNSUPPORTED;
    BallHostTables h;
    ball_build_tables(N, ix, h);
    BallTables t;
    t.N = N;
    t.lam = Lambda;
    t.Vo = h.Vo;
    t.Vo_pad = h.Vo_pad;
    std::copy(h.col_off, h.col_off + 9, t.col_off);
    t.n_entries = (int)h.map.size();
    t.ix = std::move(ix);
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    st = upload(h.oct, &t.oct);
    if (st == MATCHA_OK) st = upload(h.T, &t.T);
    if (st == MATCHA_OK) st = upload(h.map, &t.map);
    if (st != MATCHA_OK) {
        if (t.oct) (void)hipFree(t.oct);
        if (t.T) (void)hipFree(t.T);
        return st;
    }
    ctx->balls.push_back(std::move(t));
    return MATCHA_OK;
}

size_t matcha_ball_workspace_size(const matcha_ctx *ctx, int32_t N, double Lambda, int32_t n_volumes)
{
    if (!ctx || n_volumes <= 0) return 0;
    const BallTables *t = find_ball(ctx, N, Lambda);
    return t ? ball_ws_need(ctx, *t, n_volumes) : 0;
}

matcha_status matcha_ball_transform(matcha_ctx *ctx, int32_t N, double Lambda, int32_t n_volumes, const float *u,
                                    float *coef, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx || N < 2 || N > MATCHA_BALL_MAX_N || n_volumes < 0) return MATCHA_ERR_INVALID_ARG;
    if (n_volumes == 0) return MATCHA_OK;
    if (!u || !coef || ((uintptr_t)coef & 7u) != 0) return MATCHA_ERR_INVALID_ARG;
    const BallTables *t = find_ball(ctx, N, Lambda);
    if (!t) return MATCHA_ERR_NOT_PREPARED;
    if (!ws || !aligned16(ws) || ws_bytes < ball_ws_need(ctx, *t, n_volumes)) return MATCHA_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return MATCHA_ERR_HIP;
    const int P = n_volumes, S = ball_split_count(ctx, *t, P);
    float *usym = static_cast<float *>(ws);
    float *part = reinterpret_cast<float *>(static_cast<char *>(ws) +
                                            align256(sizeof(float) * 8 * (size_t)P * (size_t)t->Vo_pad));
    BallSymArgs sa{};
    sa.u = u;
    sa.oct = t->oct;
    sa.usym = usym;
    sa.Vo = t->Vo;
    sa.Vo_pad = t->Vo_pad;
    sa.N = N;
    sa.P = P;
    BallGemmArgs ga{};
    ga.usym = usym;
    ga.T = t->T;
    ga.part = part;
    ga.Vo_pad = t->Vo_pad;
    const int64_t chunks = t->Vo_pad / kBallChunk;
    ga.kper = (chunks + S - 1) / S * kBallChunk;
    ga.P = P;
    ga.ncol = t->col_off[8];
    ga.S = S;
    std::copy(t->col_off, t->col_off + 9, ga.col_off);
    BallScatterArgs ca{};
    ca.part = part;
    ca.map = t->map;
    ca.out = coef;
    ca.P = P;
    ca.ncol = ga.ncol;
    ca.S = S;
    ca.n_entries = t->n_entries;
    return launched(launch_ball(sa, ga, ca, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
