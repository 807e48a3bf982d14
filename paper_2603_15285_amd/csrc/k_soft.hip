// k_soft.hip -- low-bandwidth SOFFT search (Sec. 2.3; Alg. 1 lines 1-2).
//
// One workgroup per particle sweeps the polar nodes b_i = pi (2i+1) / (2n) in order.
// For each node it forms the Wigner-d transform over l of the coefficients,
//   S_i[m, n] = sum_{l <= B} C^l_mn d^l_mn(b_i)   on the half plane {m > 0} U {m = 0, n >= 0},
// (the wedge recurrence of the march, one step serving a pair and its partner), then the
// 2-D inverse DFT over (a, c) that gives C_B on the n x n slice.  The n^3 grid never
// leaves the chip: three consecutive slices live in an LDS ring, and the middle one is
// tested for local maxima against its 26 neighbours.  Maxima enter an LDS list of 64-bit
// keys (ordered value, inverted linear index) that is periodically sorted and cut to the
// Kc best, so the final ranking is exact whatever order the nodes arrive in.
#include "matcha_launch.hpp"

namespace matcha {

constexpr int kListCap = 1024;


// LDS layout, sized per launch from (n, B).
struct SoftSmem {
    unsigned long long *list;  // [kListCap]
    unsigned long long *thresh;
    int *count;
    int *nmax;
    float2 *S;                 // [(B+1)(2B+1)]
    float2 *T;                 // [(B+1) n]
    float2 *tw;                // [n]          e^{2 pi i t / n}
    float2 *E;                 // [(B+1) n]    e^{i m a_j}
    float *ring0;              // 3 x [n*n]    grid values of three consecutive slices
    float *mx90;               // 3 x [n*n]    3x3 in-plane maximum (centre included)
    int plane;                 // floats per slice slot (n*n rounded to 16 bytes)
    __device__ float *ring(int s) const { return ring0 + s * plane; }
    __device__ float *mx9(int s) const { return mx90 + s * plane; }
};

__host__ __device__ inline size_t soft_align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t soft_smem_size(int n, int B)
{
    size_t o = soft_align16(sizeof(unsigned long long) * kListCap);
    o += soft_align16(sizeof(float2) * (B + 1) * (2 * B + 1));
    o += soft_align16(sizeof(float2) * (B + 1) * n);
    o += soft_align16(sizeof(float2) * n);
    o += soft_align16(sizeof(float2) * (B + 1) * n);
    o += 6 * soft_align16(sizeof(float) * n * n);
    return o;
}

__device__ inline void soft_bind(SoftSmem &sm, unsigned char *base, int n, int B)
{
    size_t o = 0;
    sm.list = reinterpret_cast<unsigned long long *>(base + o);
    o += soft_align16(sizeof(unsigned long long) * kListCap);
    sm.S = reinterpret_cast<float2 *>(base + o);
    o += soft_align16(sizeof(float2) * (B + 1) * (2 * B + 1));
    sm.T = reinterpret_cast<float2 *>(base + o);
    o += soft_align16(sizeof(float2) * (B + 1) * n);
    sm.tw = reinterpret_cast<float2 *>(base + o);
    o += soft_align16(sizeof(float2) * n);
    sm.E = reinterpret_cast<float2 *>(base + o);
    o += soft_align16(sizeof(float2) * (B + 1) * n);
    sm.plane = (int)(soft_align16(sizeof(float) * n * n) / sizeof(float));
    sm.ring0 = reinterpret_cast<float *>(base + o);
    o += 3 * soft_align16(sizeof(float) * n * n);
    sm.mx90 = reinterpret_cast<float *>(base + o);
}

__device__ inline unsigned long long make_key(float v, uint32_t idx)
{
    return ((unsigned long long)ordered_bits(v) << 32) | (unsigned long long)(0xffffffffu - idx);
}

// Bitonic sort of sm.list[0..kListCap) in descending key order (empty slots hold 0).
template <int NT>
__device__ void sort_list_desc(SoftSmem &sm)
{
    for (int k = 2; k <= kListCap; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < kListCap; i += NT) {
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

// Keep the Kc largest keys; everything at or below the Kc-th key can never be ranked.
template <int NT>
__device__ void compact_list(SoftSmem &sm, int Kc)
{
    __syncthreads();
    for (int i = (*sm.count) + threadIdx.x; i < kListCap; i += NT) sm.list[i] = 0ull;
    __syncthreads();
    sort_list_desc<NT>(sm);
    if (threadIdx.x == 0) {
        const int keep = min((*sm.count), Kc);
        (*sm.count) = keep;
        if (keep == Kc) (*sm.thresh) = sm.list[Kc - 1];
    }
    __syncthreads();
}

// Wigner-d transform of polar node i into the half-plane array S[m (2B+1) + n + B]:
// S[pair] = sum_l C^l_pair dg0^l_pair(b_i), S[partner] = sum_l C^l_partner dg1^l_pair(b_i), with
// the node's d values (weights folded in) read from the table shared by all particles.
// Entries (0, n < 0) are never written and stay zero.
template <int NT>
__device__ void wigner_slice(const SoftArgs &a, const float4 *Cp, SoftSmem &sm, int i)
{
    const int B = a.B, W = 2 * B + 1;
    const int npairs = (B + 1) * (B + 1);
    const float2 *dg = a.dgrid + (int64_t)i * wedge_row(B + 1);
    for (int q = threadIdx.x; q < npairs; q += NT) {
        const PairInfo pi = a.pinfo[q];
        const int m = pi.m, n = pi.n;
        float2 u0 = make_float2(0.f, 0.f), u1 = u0;
        int row = (int)wedge_row(m);
        for (int l = m; l <= B; ++l) {
            const float2 d = dg[row + q];
            const float4 cc = Cp[row + q];
            row += (l + 1) * (l + 1);
            u0.x = fmaf(cc.x, d.x, u0.x);
            u0.y = fmaf(cc.y, d.x, u0.y);
            u1.x = fmaf(cc.z, d.y, u1.x);
            u1.y = fmaf(cc.w, d.y, u1.y);
        }
        sm.S[m * W + n + B] = u0;
        if (n != m && n != -m) {  // diagonal pairs are their own partners
            const int a2 = n >= 0 ? n : -n, b2 = n >= 0 ? m : -m;
            sm.S[a2 * W + b2 + B] = u1;
        }
    }
    __syncthreads();
}

// grid slice g[j][k] = 2 Re sum_{(m, n) in half plane} S[m, n] e^{i (m a_j + n c_k)}, then the
// 3x3 in-plane maximum of the slice (a and c periodic).
template <int NT>
__device__ void dft_slice(const SoftArgs &a, SoftSmem &sm, float *out, float *m9)
{
    const int B = a.B, W = 2 * B + 1, N = a.n;
    // T[m][k] = sum_n S[m, n] e^{i n c_k}; twiddle index (n k) mod N advanced incrementally
    for (int t = threadIdx.x; t < (B + 1) * N; t += NT) {
        const int m = t / N, k = t - (t / N) * N;
        float2 acc = make_float2(0.f, 0.f);
        int r = (N - (B * k) % N) % N;
        const float2 *Sm = sm.S + m * W;
        for (int nn = 0; nn < W; ++nn) {
            const float2 sv = Sm[nn], e = sm.tw[r];
            acc.x = fmaf(sv.x, e.x, fmaf(-sv.y, e.y, acc.x));
            acc.y = fmaf(sv.x, e.y, fmaf(sv.y, e.x, acc.y));
            r += k;
            if (r >= N) r -= N;
        }
        sm.T[m * N + k] = acc;
    }
    __syncthreads();
    // g[j][k] = 2 sum_m Re(T[m][k] e^{i m a_j}), six rows j per task
    constexpr int JB = 6;
    const int NJ = (N + JB - 1) / JB;
    for (int t = threadIdx.x; t < NJ * N; t += NT) {
        const int jb = t / N, k = t - (t / N) * N;
        const int j0 = JB * jb;
        float g[JB];
#pragma unroll
        for (int r = 0; r < JB; ++r) g[r] = 0.f;
        for (int m = 0; m <= B; ++m) {
            const float2 x = sm.T[m * N + k];
            const float2 *Em = sm.E + m * N;
#pragma unroll
            for (int r = 0; r < JB; ++r) {
                const float2 e = Em[min(j0 + r, N - 1)];
                g[r] = fmaf(x.x, e.x, fmaf(-x.y, e.y, g[r]));
            }
        }
#pragma unroll
        for (int r = 0; r < JB; ++r)
            if (j0 + r < N) out[(j0 + r) * N + k] = 2.f * g[r];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < N * N; t += NT) {
        const int j = t / N, k = t - (t / N) * N;
        const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
        const int km = k == 0 ? N - 1 : k - 1, kp = k == N - 1 ? 0 : k + 1;
        const float *r0 = out + jm * N, *r1 = out + j * N, *r2 = out + jp * N;
        float v = fmaxf(fmaxf(r0[km], r0[k]), r0[kp]);
        v = fmaxf(v, fmaxf(fmaxf(r1[km], r1[k]), r1[kp]));
        v = fmaxf(v, fmaxf(fmaxf(r2[km], r2[k]), r2[kp]));
        m9[t] = v;
    }
    __syncthreads();
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

// Offer the nodes of slice i (ring slot cslot; neighbour slots pslot / nslot, -1 when the
// slice is absent) to the list.  A node can be a local maximum only if its value equals the
// maximum of the three 3x3 in-plane maxima around it; only those nodes take the exact test.
// want_max: offer the local maxima (and count them); otherwise offer every other node.
template <int NT>
__device__ void offer_slice(const SoftArgs &a, SoftSmem &sm, int i, int pslot, int cslot, int nslot, bool want_max)
{
    const int N = a.n;
    const float *cur = sm.ring(cslot);
    for (int base = 0; base < N * N; base += NT) {
        const int t = base + threadIdx.x;
        bool offer = false;
        unsigned long long key = 0ull;
        if (t < N * N) {
            const float v = cur[t];
            float mx = sm.mx9(cslot)[t];
            if (pslot >= 0) mx = fmaxf(mx, sm.mx9(pslot)[t]);
            if (nslot >= 0) mx = fmaxf(mx, sm.mx9(nslot)[t]);
            const bool is_max = (v >= mx) && beats_all<NT>(a, sm, i, t, pslot, cslot, nslot);
            if (want_max && is_max) atomicAdd(sm.nmax, 1);
            offer = want_max ? is_max : !is_max;
            if (offer) {
                key = make_key(v, (uint32_t)(i * N * N + t));
                if (key <= (*sm.thresh)) offer = false;
            }
        }
        if (offer) {
            const int slot = atomicAdd(sm.count, 1);
            sm.list[slot] = key;
        }
        if (!want_max) {
            // every node of a chunk may be offered: keep room for a whole chunk
            __syncthreads();
            if ((*sm.count) > kListCap - NT) compact_list<NT>(sm, a.Kc);
        }
    }
    // local maxima never touch each other in a slice, so one slice adds at most n^2/4 keys
    __syncthreads();
    if ((*sm.count) > kListCap - (N * N + 3) / 4 - NT) compact_list<NT>(sm, a.Kc);
}

// One sweep over the grid; offers maxima (want_max) or non-maxima to the list.
template <int NT>
__device__ void soft_sweep(const SoftArgs &a, const float4 *Cp, SoftSmem &sm, bool want_max)
{
    const int N = a.n;
    for (int i = 0; i <= N; ++i) {
        if (i < N) {
            wigner_slice<NT>(a, Cp, sm, i);
            dft_slice<NT>(a, sm, sm.ring(i % 3), sm.mx9(i % 3));
        }
        if (i >= 1) {
            const int ic = i - 1;
            const int pslot = ic >= 1 ? (ic - 1) % 3 : -1;
            const int nslot = ic + 1 < N ? (ic + 1) % 3 : -1;
            offer_slice<NT>(a, sm, ic, pslot, ic % 3, nslot, want_max);
        }
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_soft_search(SoftArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ unsigned long long s_thresh;
    __shared__ int s_count, s_nmax;
    SoftSmem sm;
    soft_bind(sm, smem_raw, a.n, a.B);
    sm.thresh = &s_thresh;
    sm.count = &s_count;
    sm.nmax = &s_nmax;
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
    for (int t = threadIdx.x; t < (a.B + 1) * (2 * a.B + 1); t += NT) sm.S[t] = make_float2(0.f, 0.f);
    if (threadIdx.x == 0) {
        (*sm.count) = 0;
        (*sm.nmax) = 0;
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

size_t soft_smem_bytes(int n, int B) { return soft_smem_size(n, B); }

hipError_t launch_soft(const SoftArgs &a, int P, int threads, hipStream_t s)
{
    if (threads == 256)
        hipLaunchKernelGGL(k_soft_search<256>, dim3(P), dim3(256), soft_smem_size(a.n, a.B), s, a);
    else if (threads == 512)
        hipLaunchKernelGGL(k_soft_search<512>, dim3(P), dim3(512), soft_smem_size(a.n, a.B), s, a);
    else if (threads == 1024)
        hipLaunchKernelGGL(k_soft_search<1024>, dim3(P), dim3(1024), soft_smem_size(a.n, a.B), s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace matcha
