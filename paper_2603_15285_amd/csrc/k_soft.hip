// k_soft.hip -- low-bandwidth SOFFT search (Sec. 2.3; Alg. 1, its first two steps).
//
// Two kernels per batch of particles, with the grid in an HBM workspace between them.
//
// k_soft_grid synthesises C_B on the n^3 grid (a_j = 2 pi j / n, b_i = pi (2i+1) / (2n),
// c_k = 2 pi k / n).  A workgroup takes a few polar nodes of one particle; per node it
// forms the Wigner-d transform over l of the coefficients,
//   S_i[m, n] = sum_{l <= B} C^l_mn d^l_mn(b_i)   on the half plane {m > 0} U {m = 0, n >= 0},
// (the wedge recurrence of the march, one step serving a pair and its partner; the d values at
// the nodes come from a table shared by all particles), then the 2-D inverse DFT over (a, c):
// first T[m][k] = sum_n S[m, n] e^{i n c_k}, then g[j][k] = 2 Re sum_m T[m][k] e^{i m a_j}.
//
// k_soft_select takes one particle per workgroup and streams its grid slice by slice through an
// LDS ring of three slices (the next one is prefetched into registers meanwhile); the middle
// slice is tested for local maxima against its 26 neighbours.  Maxima enter an LDS list of
// 64-bit keys (ordered value, inverted linear index) that is sorted and cut to the Kc best now
// and then, so the final ranking is exact whatever order the nodes arrive in.  Once Kc maxima
// are known, the Kc-th best key is a threshold: a node below it is dropped after one compare,
// which is the fate of almost every node of the later slices.
#include "matcha_launch.hpp"

namespace matcha {

// ---------------------------------------------------------------- grid synthesis
constexpr int kGridThreads = 256;

__host__ __device__ inline size_t soft_grid_smem(int n, int B, int G)
{
    const size_t SW = (size_t)(B + 1) * (2 * B + 1), TW = (size_t)(B + 1) * n;
    return sizeof(float2) * (G * SW + G * TW + TW + n);
}

// Polar nodes per workgroup: four when their LDS fits 64 KB (two or more workgroups per CU),
// else fewer.
inline int soft_grid_slices(int n, int B)
{
    for (int G : {4, 2})
        if (soft_grid_smem(n, B, G) <= 64 * 1024) return G;
    return 1;
}

// S_i for the pairs of one task: S[pair] = sum_l C^l_pair dg0^l_pair(b_i), S[partner] = sum_l
// C^l_partner dg1^l_pair(b_i).  Entries (0, n < 0) are never written and stay zero.  Four
// degrees per trip keep eight independent loads in flight.
__device__ inline void wigner_pair(const float4 *__restrict__ Cp, const float2 *__restrict__ dg, const PairInfo &pi,
                                   int q, int B, float2 *S)
{
    const int W = 2 * B + 1;
    const int m = pi.m, n = pi.n;
    float2 u0 = make_float2(0.f, 0.f), u1 = u0;
    int row = (int)wedge_row(m) + q;
    int l = m;
    for (; l + 3 <= B; l += 4) {
        const int r0 = row, r1 = r0 + (l + 1) * (l + 1), r2 = r1 + (l + 2) * (l + 2), r3 = r2 + (l + 3) * (l + 3);
        row = r3 + (l + 4) * (l + 4);
        const float2 d0 = dg[r0], d1 = dg[r1], d2 = dg[r2], d3 = dg[r3];
        const float4 c0 = Cp[r0], c1 = Cp[r1], c2 = Cp[r2], c3 = Cp[r3];
        u0.x = fmaf(c0.x, d0.x, u0.x);
        u0.y = fmaf(c0.y, d0.x, u0.y);
        u1.x = fmaf(c0.z, d0.y, u1.x);
        u1.y = fmaf(c0.w, d0.y, u1.y);
        u0.x = fmaf(c1.x, d1.x, u0.x);
        u0.y = fmaf(c1.y, d1.x, u0.y);
        u1.x = fmaf(c1.z, d1.y, u1.x);
        u1.y = fmaf(c1.w, d1.y, u1.y);
        u0.x = fmaf(c2.x, d2.x, u0.x);
        u0.y = fmaf(c2.y, d2.x, u0.y);
        u1.x = fmaf(c2.z, d2.y, u1.x);
        u1.y = fmaf(c2.w, d2.y, u1.y);
        u0.x = fmaf(c3.x, d3.x, u0.x);
        u0.y = fmaf(c3.y, d3.x, u0.y);
        u1.x = fmaf(c3.z, d3.y, u1.x);
        u1.y = fmaf(c3.w, d3.y, u1.y);
    }
    for (; l <= B; ++l) {
        const float2 d = dg[row];
        const float4 cc = Cp[row];
        row += (l + 1) * (l + 1);
        u0.x = fmaf(cc.x, d.x, u0.x);
        u0.y = fmaf(cc.y, d.x, u0.y);
        u1.x = fmaf(cc.z, d.y, u1.x);
        u1.y = fmaf(cc.w, d.y, u1.y);
    }
    S[m * W + n + B] = u0;
    if (n != m && n != -m) {  // diagonal pairs are their own partners
        const int a2 = n >= 0 ? n : -n, b2 = n >= 0 ? m : -m;
        S[a2 * W + b2 + B] = u1;
    }
}

__global__ void __launch_bounds__(kGridThreads) k_soft_grid(SoftArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int B = a.B, N = a.n, W = 2 * B + 1;
    const int SW = (B + 1) * W, TW = (B + 1) * N;
    const int G = a.gslices;
    const int NG = (N + G - 1) / G;
    const int pl = blockIdx.x / NG, i0 = (blockIdx.x - pl * NG) * G;
    const int ni = min(G, N - i0);
    const int p = a.p0 + pl;
    float2 *S = reinterpret_cast<float2 *>(smem_raw);  // [G][SW]
    float2 *T = S + G * SW;                             // [G][TW]
    float2 *E = T + G * TW;                             // [TW] e^{i m a_j}, then [N] twiddles
    const float2 *tw = E + TW;
    const float4 *Cp = a.C + a.C_off[p] / 2;
    for (int t = threadIdx.x; t < TW + N; t += kGridThreads) E[t] = a.etab[t];
    for (int t = threadIdx.x; t < G * SW; t += kGridThreads) S[t] = make_float2(0.f, 0.f);
    __syncthreads();

    // Wigner-d transforms of the block's nodes
    const int npairs = (B + 1) * (B + 1);
    const int64_t drow = wedge_row(B + 1);
    for (int t = threadIdx.x; t < ni * npairs; t += kGridThreads) {
        const int gi = t / npairs, q = t - gi * npairs;
        wigner_pair(Cp, a.dgrid + (int64_t)(i0 + gi) * drow, a.pinfo[q], q, B, S + gi * SW);
    }
    __syncthreads();

    // first DFT stage, three k per task; the twiddle index (n k) mod N advances incrementally
    {
        constexpr int KB = 3;
        const int NKB = (N + KB - 1) / KB, per = (B + 1) * NKB;
        for (int t = threadIdx.x; t < ni * per; t += kGridThreads) {
            const int gi = t / per, tt = t - gi * per;
            const int m = tt / NKB, kb = tt - m * NKB;
            int k[KB], r[KB];
            float2 acc[KB];
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                k[u] = min(KB * kb + u, N - 1);
                r[u] = (N - (B * k[u]) % N) % N;
                acc[u] = make_float2(0.f, 0.f);
            }
            const float2 *Sm = S + gi * SW + m * W;
            for (int nn = 0; nn < W; ++nn) {
                const float2 sv = Sm[nn];
#pragma unroll
                for (int u = 0; u < KB; ++u) {
                    const float2 e = tw[r[u]];
                    acc[u].x = fmaf(sv.x, e.x, fmaf(-sv.y, e.y, acc[u].x));
                    acc[u].y = fmaf(sv.x, e.y, fmaf(sv.y, e.x, acc[u].y));
                    r[u] += k[u];
                    if (r[u] >= N) r[u] -= N;
                }
            }
            float2 *Tm = T + gi * TW + m * N;
#pragma unroll
            for (int u = 0; u < KB; ++u)
                if (KB * kb + u < N) Tm[KB * kb + u] = acc[u];
        }
    }
    __syncthreads();

    // second stage, a 6 (j) x 2 (k) block per task, straight to the workspace
    {
        constexpr int JB = 6, KB = 2;
        const int NJ = (N + JB - 1) / JB, NK = (N + KB - 1) / KB, per = NJ * NK;
        for (int t = threadIdx.x; t < ni * per; t += kGridThreads) {
            const int gi = t / per, tt = t - gi * per;
            const int jb = tt / NK, kb = tt - jb * NK;
            const int j0 = JB * jb, k0 = KB * kb, k1 = min(k0 + 1, N - 1);
            const float2 *Tg = T + gi * TW;
            float g[JB][KB];
#pragma unroll
            for (int r = 0; r < JB; ++r) g[r][0] = g[r][1] = 0.f;
            for (int m = 0; m <= B; ++m) {
                const float2 x0 = Tg[m * N + k0], x1 = Tg[m * N + k1];
                const float2 *Em = E + m * N;
#pragma unroll
                for (int r = 0; r < JB; ++r) {
                    const float2 e = Em[min(j0 + r, N - 1)];
                    g[r][0] = fmaf(x0.x, e.x, fmaf(-x0.y, e.y, g[r][0]));
                    g[r][1] = fmaf(x1.x, e.x, fmaf(-x1.y, e.y, g[r][1]));
                }
            }
            float *out = a.grid + ((int64_t)pl * N + i0 + gi) * N * N;
#pragma unroll
            for (int r = 0; r < JB; ++r) {
                if (j0 + r < N) {
                    out[(j0 + r) * N + k0] = 2.f * g[r][0];
                    if (k0 + 1 < N) out[(j0 + r) * N + k0 + 1] = 2.f * g[r][1];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- maxima and ranking
constexpr int kSelMaxN = 96;

// Key-list capacity of an NT-thread workgroup: room for the Kc <= 64 kept keys plus one chunk
// of NT offers, which the chunked offer needs.
template <int NT>
constexpr int list_cap() { return 2 * NT; }

// Grid values per thread of one prefetched slice.
template <int NT>
constexpr int sel_per() { return (kSelMaxN * kSelMaxN + NT - 1) / NT; }

// LDS layout, sized per launch from n.
struct SoftSmem {
    unsigned long long *list;  // [list_cap]
    unsigned long long *thresh;
    int *count;
    int *nmax;
    int *overflow;
    float *ring0;              // 3 x [n*n]    grid values of three consecutive slices
    int plane;                 // floats per slice slot (n*n rounded to 16 bytes)
    __device__ float *ring(int s) const { return ring0 + s * plane; }
};

__host__ __device__ inline size_t soft_align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t soft_select_smem(int n, int cap)
{
    return soft_align16(sizeof(unsigned long long) * cap) + 3 * soft_align16(sizeof(float) * n * n);
}

__device__ inline unsigned long long make_key(float v, uint32_t idx)
{
    return ((unsigned long long)ordered_bits(v) << 32) | (unsigned long long)(0xffffffffu - idx);
}

// Bitonic sort of sm.list[0 .. sz) in descending key order; sz is a power of two.
template <int NT>
__device__ void sort_list_desc(SoftSmem &sm, int sz)
{
    for (int k = 2; k <= sz; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < sz; i += NT) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const unsigned long long a = sm.list[i], b = sm.list[ixj];
                    const bool desc = (i & k) == 0;
                    if (desc ? (a < b) : (a > b)) {
                        sm.list[i] = b;
                        sm.list[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Keep the Kc largest keys (count <= list capacity on entry).  With Kc keys kept, the Kc-th is
// the new threshold: a key at or below it can never be ranked.
template <int NT>
__device__ void compact_list(SoftSmem &sm, int Kc)
{
    __syncthreads();
    const int cnt = *sm.count;
    int sz = 2;
    while (sz < cnt) sz <<= 1;
    for (int i = cnt + threadIdx.x; i < sz; i += NT) sm.list[i] = 0ull;
    __syncthreads();
    sort_list_desc<NT>(sm, sz);
    if (threadIdx.x == 0) {
        const int keep = min(cnt, Kc);
        (*sm.count) = keep;
        if (keep == Kc) (*sm.thresh) = sm.list[Kc - 1];
    }
    __syncthreads();
}

// Exact test of the node t of slice i against its 26 neighbours: a neighbour beats it with a
// larger key (ordered value bits, then the smaller linear index).  The wrapped row and column
// offsets are formed once; the index is consulted only on equal value bits.
template <int NT>
__device__ bool beats_all(const SoftArgs &a, const SoftSmem &sm, int i, int t, int pslot, int cslot, int nslot)
{
    const int N = a.n;
    const int j = t / N, k = t - (t / N) * N;
    const int rows[3] = {(j == 0 ? N - 1 : j - 1) * N, j * N, (j == N - 1 ? 0 : j + 1) * N};
    const int cols[3] = {k == 0 ? N - 1 : k - 1, k, k == N - 1 ? 0 : k + 1};
    const uint32_t ov = ordered_bits(sm.ring(cslot)[t]);
    const uint32_t idx = (uint32_t)(i * N * N + t);
#pragma unroll
    for (int di = 0; di < 3; ++di) {
        const int slot = di == 0 ? pslot : (di == 2 ? nslot : cslot);
        if (slot < 0) continue;
        const float *pl = sm.ring(slot);
        const uint32_t base = (uint32_t)((i + di - 1) * N * N);
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int dk = 0; dk < 3; ++dk) {
                if (di == 1 && dj == 1 && dk == 1) continue;
                const int o = rows[dj] + cols[dk];
                const uint32_t ou = ordered_bits(pl[o]);
                if (ou > ov || (ou == ov && base + (uint32_t)o < idx)) return false;
            }
    }
    return true;
}

// Is node t of slice i worth a key?  want_max: a local maximum (counted in nmax); otherwise a
// node that is not one.  Nodes whose value lies below the threshold's are dropped first, then
// (for maxima) nodes below one of their six axis neighbours; only the rest take the exact test.
template <int NT>
__device__ bool offer_node(const SoftArgs &a, const SoftSmem &sm, int i, int t, int pslot, int cslot, int nslot,
                           bool want_max, uint32_t th_hi, unsigned long long &key)
{
    const int N = a.n;
    const float *cur = sm.ring(cslot);
    const float v = cur[t];
    if (ordered_bits(v) < th_hi) return false;
    if (want_max) {
        const int j = t / N, k = t - (t / N) * N;
        const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
        const int km = k == 0 ? N - 1 : k - 1, kp = k == N - 1 ? 0 : k + 1;
        bool pass = v >= cur[jm * N + k] && v >= cur[jp * N + k] && v >= cur[j * N + km] && v >= cur[j * N + kp];
        if (pass && pslot >= 0) pass = v >= sm.ring(pslot)[t];
        if (pass && nslot >= 0) pass = v >= sm.ring(nslot)[t];
        if (!pass || !beats_all<NT>(a, sm, i, t, pslot, cslot, nslot)) return false;
        atomicAdd(sm.nmax, 1);
    } else if (beats_all<NT>(a, sm, i, t, pslot, cslot, nslot)) {
        return false;
    }
    key = make_key(v, (uint32_t)(i * N * N + t));
    return key > (*sm.thresh);
}

// Offer the nodes of slice i (ring slot cslot; neighbour slots pslot / nslot, -1 when the
// slice is absent) to the list, one pass over the slice.  Called between barriers; the list
// state it reads was last changed before the preceding barrier.
template <int NT>
__device__ void offer_pass(const SoftArgs &a, const SoftSmem &sm, int i, int pslot, int cslot, int nslot,
                           bool want_max)
{
    const int NN = a.n * a.n;
    const uint32_t th_hi = (uint32_t)((*sm.thresh) >> 32);
    for (int t = threadIdx.x; t < NN; t += NT) {
        unsigned long long key;
        if (offer_node<NT>(a, sm, i, t, pslot, cslot, nslot, want_max, th_hi, key)) {
            const int slot = atomicAdd(sm.count, 1);
            if (slot < list_cap<NT>())
                sm.list[slot] = key;
            else
                (*sm.overflow) = 1;
        }
    }
}

// After offer_pass and a barrier.  If the slice's keys overflowed the list, they are taken back
// (count and nmax as before the pass) and the slice is offered again in chunks of NT nodes
// with a compaction whenever fewer than NT slots are free (a chunk adds at most NT keys).
// Otherwise the list is cut when it holds twice the ranks, and as soon as the first Kc keys
// are in (that sets the threshold).
template <int NT>
__device__ void offer_finish(const SoftArgs &a, SoftSmem &sm, int i, int pslot, int cslot, int nslot, bool want_max,
                             int count0, int nmax0)
{
    const int NN = a.n * a.n, Kc = a.Kc;
    if (*sm.overflow) {
        __syncthreads();
        if (threadIdx.x == 0) {
            (*sm.count) = count0;
            (*sm.nmax) = nmax0;
            (*sm.overflow) = 0;
        }
        compact_list<NT>(sm, Kc);
        for (int base = 0; base < NN; base += NT) {
            // count is read by every thread between two barriers, so all take the same branch
            const bool full = (*sm.count) > list_cap<NT>() - NT;
            __syncthreads();
            if (full) compact_list<NT>(sm, Kc);
            const int t = base + threadIdx.x;
            const uint32_t th = (uint32_t)((*sm.thresh) >> 32);
            unsigned long long key;
            if (t < NN && offer_node<NT>(a, sm, i, t, pslot, cslot, nslot, want_max, th, key))
                sm.list[atomicAdd(sm.count, 1)] = key;
            __syncthreads();
        }
        return;
    }
    const int cnt = *sm.count;
    if (cnt >= 2 * Kc || (cnt >= Kc && (*sm.thresh) == 0ull)) compact_list<NT>(sm, Kc);
}

// One sweep over the particle's grid; offers maxima (want_max) or non-maxima to the list.
// Slice ic+2 is loaded into registers before slice ic is offered and stored into the ring slot
// of slice ic-1 afterwards.
template <int NT>
__device__ void select_sweep(const SoftArgs &a, SoftSmem &sm, const float *grid, bool want_max)
{
    const int N = a.n, NN = N * N;
    constexpr int PER = sel_per<NT>();
    for (int s = 0; s < 2; ++s)
        for (int t = threadIdx.x; t < NN; t += NT) sm.ring(s)[t] = grid[(int64_t)s * NN + t];
    __syncthreads();
    for (int ic = 0; ic < N; ++ic) {
        // the list is quiet from here until the offer: every thread sees the same state
        const int count0 = *sm.count, nmax0 = *sm.nmax;
        const bool pre = ic + 2 < N;
        float nxt[PER];
        if (pre) {
            const float *src = grid + (int64_t)(ic + 2) * NN;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int t = threadIdx.x + u * NT;
                nxt[u] = t < NN ? src[t] : 0.f;
            }
        }
        const int pslot = ic >= 1 ? (ic - 1) % 3 : -1;
        const int nslot = ic + 1 < N ? (ic + 1) % 3 : -1;
        offer_pass<NT>(a, sm, ic, pslot, ic % 3, nslot, want_max);
        __syncthreads();
        offer_finish<NT>(a, sm, ic, pslot, ic % 3, nslot, want_max, count0, nmax0);
        if (pre) {
            float *dst = sm.ring((ic + 2) % 3);
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int t = threadIdx.x + u * NT;
                if (t < NN) dst[t] = nxt[u];
            }
        }
        __syncthreads();
    }
}

__device__ inline float4 key_to_cand(unsigned long long key, int N)
{
    const uint32_t idx = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
    const float v = unordered_bits((uint32_t)(key >> 32));
    const int i = idx / (N * N), j = (idx / N) % N, k = idx % N;
    return make_float4((float)(kTwoPi * j / N), (float)(kPi * (2.0 * i + 1.0) / (2.0 * N)), (float)(kTwoPi * k / N), v);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_soft_select(SoftArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ unsigned long long s_thresh;
    __shared__ int s_count, s_nmax, s_overflow;
    SoftSmem sm;
    const int N = a.n, Kc = a.Kc;
    sm.list = reinterpret_cast<unsigned long long *>(smem_raw);
    sm.ring0 = reinterpret_cast<float *>(smem_raw + soft_align16(sizeof(unsigned long long) * list_cap<NT>()));
    sm.plane = (int)(soft_align16(sizeof(float) * N * N) / sizeof(float));
    sm.thresh = &s_thresh;
    sm.count = &s_count;
    sm.nmax = &s_nmax;
    sm.overflow = &s_overflow;
    const int pl = blockIdx.x, p = a.p0 + pl;
    const float *grid = a.grid + (int64_t)pl * N * N * N;
    if (threadIdx.x == 0) {
        (*sm.count) = 0;
        (*sm.nmax) = 0;
        (*sm.overflow) = 0;
        (*sm.thresh) = 0ull;
    }
    __syncthreads();
    select_sweep<NT>(a, sm, grid, true);
    compact_list<NT>(sm, Kc);
    const int nmax = (*sm.nmax);
    const int nm = min(nmax, Kc);
    // ranked maxima -> cand[0 .. nm)
    for (int t = threadIdx.x; t < nm; t += NT) a.cand[(int64_t)p * Kc + t] = key_to_cand(sm.list[t], N);
    __syncthreads();
    if (nmax < Kc) {
        // rare: fill with the best nodes that are not local maxima (second sweep)
        if (threadIdx.x == 0) {
            (*sm.count) = 0;
            (*sm.thresh) = 0ull;
        }
        __syncthreads();
        select_sweep<NT>(a, sm, grid, false);
        compact_list<NT>(sm, Kc - nm);
        for (int t = threadIdx.x; t < Kc - nm; t += NT) a.cand[(int64_t)p * Kc + nm + t] = key_to_cand(sm.list[t], N);
    }
    if (threadIdx.x == 0) a.status[p] = nmax < Kc ? 16u : 0u;
}

size_t soft_grid_smem_bytes(int n, int B) { return soft_grid_smem(n, B, 1); }
size_t soft_select_smem_bytes(int n, int threads) { return soft_select_smem(n, 2 * threads); }

hipError_t launch_soft_grid(const SoftArgs &a0, int P, hipStream_t s)
{
    SoftArgs a = a0;
    a.gslices = soft_grid_slices(a.n, a.B);
    const int NG = (a.n + a.gslices - 1) / a.gslices;
    hipLaunchKernelGGL(k_soft_grid, dim3(P * NG), dim3(kGridThreads), soft_grid_smem(a.n, a.B, a.gslices), s, a);
    return hipGetLastError();
}

hipError_t launch_soft_select(const SoftArgs &a, int P, int threads, hipStream_t s)
{
    if (a.n > kSelMaxN) return hipErrorInvalidValue;
    if (threads == 256)
        hipLaunchKernelGGL(k_soft_select<256>, dim3(P), dim3(256), soft_select_smem(a.n, list_cap<256>()), s, a);
    else if (threads == 512)
        hipLaunchKernelGGL(k_soft_select<512>, dim3(P), dim3(512), soft_select_smem(a.n, list_cap<512>()), s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace matcha
