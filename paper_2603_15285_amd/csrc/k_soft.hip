// k_soft.hip -- low-bandwidth SOFFT search (Sec. 2.3; Alg. 1 lines 1-2).
//
// One workgroup per particle sweeps the polar nodes b_i = pi (2i+1) / (2n) in order.
// For each node it forms the Wigner-d transform over l of the coefficients,
//   S_i[m, n] = sum_{l <= B} C^l_mn d^l_mn(b_i)   on the half plane {m > 0} U {m = 0, n >= 0},
// (the wedge recurrence of the march, one step serving a pair and its partner), then the
// 2-D inverse DFT over (a, c) that gives C_B on the n x n slice.  The n^3 grid never
// leaves the chip: three consecutive slices live in an LDS ring, and the middle one is
// tested for local maxima against its 26 neighbours.  Maxima enter an LDS list of 64-bit
// keys (ordered value, inverted linear index) that is sorted and cut to the Kc best now and
// then, so the final ranking is exact whatever order the nodes arrive in.  Once Kc maxima
// are known, the Kc-th best key is a threshold: a node below it is dropped after one
// compare, which is the fate of almost every node of the later slices.
#include "matcha_launch.hpp"

namespace matcha {

// Key-list capacity of an NT-thread workgroup: room for the Kc <= 64 kept keys plus one chunk
// of NT offers, which the chunked offer needs.
template <int NT>
constexpr int list_cap() { return 2 * NT; }


// LDS layout, sized per launch from (n, B).
struct SoftSmem {
    unsigned long long *list;  // [list_cap]
    unsigned long long *thresh;
    int *count;
    int *nmax;
    int *overflow;
    float2 *S;                 // 2 x [(B+1)(2B+1)]   (double buffered)
    float2 *T;                 // 2 x [(B+1) n]       (double buffered)
    float2 *tw;                // [n]          e^{2 pi i t / n}
    float2 *E;                 // [(B+1) n]    e^{i m a_j}
    float *ring0;              // 3 x [n*n]    grid values of three consecutive slices
    int plane;                 // floats per slice slot (n*n rounded to 16 bytes)
    int s_stride, t_stride;    // float2 per S / T buffer
    __device__ float *ring(int s) const { return ring0 + s * plane; }
    __device__ float2 *Sb(int i) const { return S + (i & 1) * s_stride; }
    __device__ float2 *Tb(int i) const { return T + (i & 1) * t_stride; }
};

__host__ __device__ inline size_t soft_align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t soft_smem_size(int n, int B, int cap)
{
    size_t o = soft_align16(sizeof(unsigned long long) * cap);
    o += 2 * soft_align16(sizeof(float2) * (B + 1) * (2 * B + 1));
    o += 2 * soft_align16(sizeof(float2) * (B + 1) * n);
    o += soft_align16(sizeof(float2) * n);
    o += soft_align16(sizeof(float2) * (B + 1) * n);
    o += 3 * soft_align16(sizeof(float) * n * n);
    return o;
}

__device__ inline void soft_bind(SoftSmem &sm, unsigned char *base, int n, int B, int cap)
{
    size_t o = 0;
    sm.list = reinterpret_cast<unsigned long long *>(base + o);
    o += soft_align16(sizeof(unsigned long long) * cap);
    sm.S = reinterpret_cast<float2 *>(base + o);
    sm.s_stride = (int)(soft_align16(sizeof(float2) * (B + 1) * (2 * B + 1)) / sizeof(float2));
    o += 2 * soft_align16(sizeof(float2) * (B + 1) * (2 * B + 1));
    sm.T = reinterpret_cast<float2 *>(base + o);
    sm.t_stride = (int)(soft_align16(sizeof(float2) * (B + 1) * n) / sizeof(float2));
    o += 2 * soft_align16(sizeof(float2) * (B + 1) * n);
    sm.tw = reinterpret_cast<float2 *>(base + o);
    o += soft_align16(sizeof(float2) * n);
    sm.E = reinterpret_cast<float2 *>(base + o);
    o += soft_align16(sizeof(float2) * (B + 1) * n);
    sm.plane = (int)(soft_align16(sizeof(float) * n * n) / sizeof(float));
    sm.ring0 = reinterpret_cast<float *>(base + o);
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

// Wigner-d transform of polar node i into the half-plane array S[m (2B+1) + n + B] (buffer
// i mod 2): S[pair] = sum_l C^l_pair dg0^l_pair(b_i), S[partner] = sum_l C^l_partner dg1^l_pair(b_i),
// with the node's d values (weights folded in) read from the table shared by all particles.
// Entries (0, n < 0) are never written and stay zero.  Four degrees per trip keep eight
// independent loads in flight.
template <int NT>
__device__ void wigner_slice(const SoftArgs &a, const float4 *Cp, const SoftSmem &sm, int i)
{
    const int B = a.B, W = 2 * B + 1;
    const int npairs = (B + 1) * (B + 1);
    const float2 *dg = a.dgrid + (int64_t)i * wedge_row(B + 1);
    float2 *S = sm.Sb(i);
    for (int q = threadIdx.x; q < npairs; q += NT) {
        const PairInfo pi = a.pinfo[q];
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
}

// First stage of the grid slice: T[m][k] = sum_n S[m, n] e^{i n c_k} (buffer i mod 2), three
// k per task; the twiddle index (n k) mod N advances incrementally.
template <int NT>
__device__ void dft_stage1(const SoftArgs &a, const SoftSmem &sm, int i)
{
    const int B = a.B, W = 2 * B + 1, N = a.n;
    constexpr int KB = 3;
    const int NKB = (N + KB - 1) / KB;
    const float2 *S = sm.Sb(i);
    float2 *T = sm.Tb(i);
    for (int t = threadIdx.x; t < (B + 1) * NKB; t += NT) {
        const int m = t / NKB, kb = t - (t / NKB) * NKB;
        int k[KB], r[KB];
        float2 acc[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            k[u] = min(KB * kb + u, N - 1);
            r[u] = (N - (B * k[u]) % N) % N;
            acc[u] = make_float2(0.f, 0.f);
        }
        const float2 *Sm = S + m * W;
        for (int nn = 0; nn < W; ++nn) {
            const float2 sv = Sm[nn];
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const float2 e = sm.tw[r[u]];
                acc[u].x = fmaf(sv.x, e.x, fmaf(-sv.y, e.y, acc[u].x));
                acc[u].y = fmaf(sv.x, e.y, fmaf(sv.y, e.x, acc[u].y));
                r[u] += k[u];
                if (r[u] >= N) r[u] -= N;
            }
        }
#pragma unroll
        for (int u = 0; u < KB; ++u)
            if (KB * kb + u < N) T[m * N + KB * kb + u] = acc[u];
    }
}

// Second stage: g[j][k] = 2 sum_m Re(T[m][k] e^{i m a_j}) into the ring slot, a 6 x 2 block of
// (j, k) per task.
template <int NT>
__device__ void dft_stage2(const SoftArgs &a, const SoftSmem &sm, int i, float *out)
{
    const int B = a.B, N = a.n;
    constexpr int JB = 6, KB = 2;
    const int NJ = (N + JB - 1) / JB, NK = (N + KB - 1) / KB;
    const float2 *T = sm.Tb(i);
    for (int t = threadIdx.x; t < NJ * NK; t += NT) {
        const int jb = t / NK, kb = t - (t / NK) * NK;
        const int j0 = JB * jb, k0 = KB * kb, k1 = min(k0 + 1, N - 1);
        float g[JB][KB];
#pragma unroll
        for (int r = 0; r < JB; ++r) g[r][0] = g[r][1] = 0.f;
        for (int m = 0; m <= B; ++m) {
            const float2 x0 = T[m * N + k0], x1 = T[m * N + k1];
            const float2 *Em = sm.E + m * N;
#pragma unroll
            for (int r = 0; r < JB; ++r) {
                const float2 e = Em[min(j0 + r, N - 1)];
                g[r][0] = fmaf(x0.x, e.x, fmaf(-x0.y, e.y, g[r][0]));
                g[r][1] = fmaf(x1.x, e.x, fmaf(-x1.y, e.y, g[r][1]));
            }
        }
#pragma unroll
        for (int r = 0; r < JB; ++r) {
            if (j0 + r < N) {
                out[(j0 + r) * N + k0] = 2.f * g[r][0];
                if (k0 + 1 < N) out[(j0 + r) * N + k0 + 1] = 2.f * g[r][1];
            }
        }
    }
}

// Exact test of the node t of slice i against its 26 neighbours: (value, smaller index) wins.
template <int NT>
__device__ bool beats_all(const SoftArgs &a, const SoftSmem &sm, int i, int t, int pslot, int cslot, int nslot)
{
    const int N = a.n;
    const int j = t / N, k = t - (t / N) * N;
    const unsigned long long key = make_key(sm.ring(cslot)[t], (uint32_t)(i * N * N + t));
    for (int di = -1; di <= 1; ++di) {
        const int slot = di < 0 ? pslot : (di > 0 ? nslot : cslot);
        if (slot < 0) continue;
        const float *pl = sm.ring(slot);
        for (int dj = -1; dj <= 1; ++dj) {
            const int jj = (j + dj + N) % N;
            for (int dk = -1; dk <= 1; ++dk) {
                if (!di && !dj && !dk) continue;
                const int kk = (k + dk + N) % N;
                if (make_key(pl[jj * N + kk], (uint32_t)((i + di) * N * N + jj * N + kk)) > key) return false;
            }
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

// One sweep over the grid; offers maxima (want_max) or non-maxima to the list.  Two phases per
// polar node, one barrier each:
//   A: Wigner transform of node i+1 (S buffer (i+1) mod 2) and second DFT stage of node i
//      (T buffer i mod 2 -> ring slot i mod 3);
//   B: first DFT stage of node i+1 (S -> T buffer (i+1) mod 2) and the offer of node i-1, whose
//      neighbours i-2 .. i are complete.
template <int NT>
__device__ void soft_sweep(const SoftArgs &a, const float4 *Cp, SoftSmem &sm, bool want_max)
{
    const int N = a.n;
    wigner_slice<NT>(a, Cp, sm, 0);
    __syncthreads();
    dft_stage1<NT>(a, sm, 0);
    __syncthreads();
    for (int i = 0; i <= N; ++i) {
        // the list is quiet from here until phase B's offer: every thread sees the same state
        const int count0 = *sm.count, nmax0 = *sm.nmax;
        if (i < N) {
            if (i + 1 < N) wigner_slice<NT>(a, Cp, sm, i + 1);
            dft_stage2<NT>(a, sm, i, sm.ring(i % 3));
        }
        __syncthreads();
        if (i + 1 < N) dft_stage1<NT>(a, sm, i + 1);
        if (i >= 1) {
            const int ic = i - 1;
            const int pslot = ic >= 1 ? (ic - 1) % 3 : -1;
            const int nslot = ic + 1 < N ? (ic + 1) % 3 : -1;
            offer_pass<NT>(a, sm, ic, pslot, ic % 3, nslot, want_max);
            __syncthreads();
            offer_finish<NT>(a, sm, ic, pslot, ic % 3, nslot, want_max, count0, nmax0);
        } else {
            __syncthreads();
        }
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_soft_search(SoftArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ unsigned long long s_thresh;
    __shared__ int s_count, s_nmax, s_overflow;
    SoftSmem sm;
    soft_bind(sm, smem_raw, a.n, a.B, list_cap<NT>());
    sm.thresh = &s_thresh;
    sm.count = &s_count;
    sm.nmax = &s_nmax;
    sm.overflow = &s_overflow;
    const int p = blockIdx.x;
    const int N = a.n, Kc = a.Kc;
    const float4 *Cp = a.C + a.C_off[p] / 2;
    for (int t = threadIdx.x; t < N; t += NT) {
        float s, c;
        sincosf((float)(kTwoPi * t / N), &s, &c);
        sm.tw[t] = make_float2(c, s);
    }
    for (int t = threadIdx.x; t < (a.B + 1) * N; t += NT) {
        const int m = t / N, j = t - (t / N) * N;
        float s, c;
        sincosf((float)(kTwoPi * ((m * j) % N) / N), &s, &c);
        sm.E[t] = make_float2(c, s);
    }
    for (int t = threadIdx.x; t < 2 * sm.s_stride; t += NT) sm.S[t] = make_float2(0.f, 0.f);
    if (threadIdx.x == 0) {
        (*sm.count) = 0;
        (*sm.nmax) = 0;
        (*sm.overflow) = 0;
        (*sm.thresh) = 0ull;
    }
    __syncthreads();
    soft_sweep<NT>(a, Cp, sm, true);
    compact_list<NT>(sm, Kc);
    const int nmax = (*sm.nmax);
    const int nm = min(nmax, Kc);
    // ranked maxima -> cand[0 .. nm)
    for (int t = threadIdx.x; t < nm; t += NT) {
        const unsigned long long key = sm.list[t];
        const uint32_t idx = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
        const float v = unordered_bits((uint32_t)(key >> 32));
        const int i = idx / (N * N), j = (idx / N) % N, k = idx % N;
        a.cand[(int64_t)p * Kc + t] = make_float4((float)(kTwoPi * j / N), (float)(kPi * (2.0 * i + 1.0) / (2.0 * N)),
                                                  (float)(kTwoPi * k / N), v);
    }
    __syncthreads();
    if (nmax < Kc) {
        // rare: fill with the best nodes that are not local maxima (second sweep)
        if (threadIdx.x == 0) {
            (*sm.count) = 0;
            (*sm.thresh) = 0ull;
        }
        __syncthreads();
        soft_sweep<NT>(a, Cp, sm, false);
        compact_list<NT>(sm, Kc - nm);
        for (int t = threadIdx.x; t < Kc - nm; t += NT) {
            const unsigned long long key = sm.list[t];
            const uint32_t idx = 0xffffffffu - (uint32_t)(key & 0xffffffffull);
            const float v = unordered_bits((uint32_t)(key >> 32));
            const int i = idx / (N * N), j = (idx / N) % N, k = idx % N;
            a.cand[(int64_t)p * Kc + nm + t] = make_float4((float)(kTwoPi * j / N),
                                                           (float)(kPi * (2.0 * i + 1.0) / (2.0 * N)),
                                                           (float)(kTwoPi * k / N), v);
        }
    }
    if (threadIdx.x == 0) a.status[p] = nmax < Kc ? 16u : 0u;
}

size_t soft_smem_bytes(int n, int B, int threads) { return soft_smem_size(n, B, 2 * threads); }

hipError_t launch_soft(const SoftArgs &a, int P, int threads, hipStream_t s)
{
    if (threads == 256)
        hipLaunchKernelGGL(k_soft_search<256>, dim3(P), dim3(256), soft_smem_size(a.n, a.B, list_cap<256>()), s, a);
    else if (threads == 512)
        hipLaunchKernelGGL(k_soft_search<512>, dim3(P), dim3(512), soft_smem_size(a.n, a.B, list_cap<512>()), s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace matcha
