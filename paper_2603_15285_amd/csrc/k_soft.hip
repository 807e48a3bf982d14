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

constexpr int kSoftThreads = 256;
constexpr int kListCap = 1024;


// LDS layout, sized per launch from (n, B).
struct SoftSmem {
    unsigned long long *list;  // [kListCap]
    unsigned long long *thresh;
    int *count;
    int *nmax;
    float2 *S;                 // [(B+1)(2B+1)]
    float2 *T;                 // [(B+1) n]
    float2 *tw;                // [n]
    float *ring[3];            // [n*n] each
};

__host__ __device__ inline size_t soft_align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t soft_smem_size(int n, int B)
{
    size_t o = soft_align16(sizeof(unsigned long long) * kListCap);
    o += soft_align16(sizeof(float2) * (B + 1) * (2 * B + 1));
    o += soft_align16(sizeof(float2) * (B + 1) * n);
    o += soft_align16(sizeof(float2) * n);
    o += 3 * soft_align16(sizeof(float) * n * n);
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
    for (int r = 0; r < 3; ++r) {
        sm.ring[r] = reinterpret_cast<float *>(base + o);
        o += soft_align16(sizeof(float) * n * n);
    }
}

__device__ inline unsigned long long make_key(float v, uint32_t idx)
{
    return ((unsigned long long)ordered_bits(v) << 32) | (unsigned long long)(0xffffffffu - idx);
}

// Bitonic sort of sm.list[0..kListCap) in descending key order (empty slots hold 0).
__device__ void sort_list_desc(SoftSmem &sm)
{
    for (int k = 2; k <= kListCap; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < kListCap; i += kSoftThreads) {
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
__device__ void compact_list(SoftSmem &sm, int Kc)
{
    __syncthreads();
    for (int i = (*sm.count) + threadIdx.x; i < kListCap; i += kSoftThreads) sm.list[i] = 0ull;
    __syncthreads();
    sort_list_desc(sm);
    if (threadIdx.x == 0) {
        const int keep = min((*sm.count), Kc);
        (*sm.count) = keep;
        if (keep == Kc) (*sm.thresh) = sm.list[Kc - 1];
    }
    __syncthreads();
}

// Wigner-d transform of one polar node into the half-plane array S[(m)(2B+1) + n + B].
__device__ void wigner_slice(const SoftArgs &a, const float4 *Cp, SoftSmem &sm, double b)
{
    const int B = a.B, W = 2 * B + 1;
    for (int i = threadIdx.x; i < (B + 1) * W; i += kSoftThreads) sm.S[i] = make_float2(0.f, 0.f);
    __syncthreads();
    const BetaConst bc = beta_const(b);
    const int npairs = (B + 1) * (B + 1);
    for (int q = threadIdx.x; q < npairs; q += kSoftThreads) {
        const PairInfo pi = a.pinfo[q];
        const int m = pi.m, n = pi.n;
        float s0, s1, s2;
        edge_seed(m, n, pi.lbh2, bc, s0, s1, s2);
        float D = 0.f, Dm = 0.f;
        float2 u0 = make_float2(0.f, 0.f), u1 = u0;
        float pwt = 0.f;
        for (int l = m; l <= B; ++l) {
            const float4 tb = a.tab[wedge_row(l) + q];
            const float4 cc = Cp[wedge_row(l) + q];
            float dn = fmaf(tb.x * bc.cb - tb.y, D, -Dm);
            if (l == m) dn = s0;
            Dm = D;
            D = dn;
            u0.x = fmaf(cc.x * tb.z, dn, u0.x);
            u0.y = fmaf(cc.y * tb.z, dn, u0.y);
            u1.x = fmaf(cc.z * tb.w, dn, u1.x);
            u1.y = fmaf(cc.w * tb.w, dn, u1.y);
            pwt = tb.w;
        }
        sm.S[m * W + n + B] = u0;
        if (pwt != 0.f) {  // not a diagonal pair: the partner is a distinct entry
            const int a2 = n >= 0 ? n : -n, b2 = n >= 0 ? m : -m;
            sm.S[a2 * W + b2 + B] = u1;
        }
    }
    __syncthreads();
}

// grid slice g[j][k] = 2 Re sum_{(m, n) in half plane} S[m, n] e^{i (m a_j + n c_k)}
__device__ void dft_slice(const SoftArgs &a, SoftSmem &sm, float *out)
{
    const int B = a.B, W = 2 * B + 1, N = a.n;
    for (int t = threadIdx.x; t < (B + 1) * N; t += kSoftThreads) {
        const int m = t / N, k = t % N;
        float2 acc = make_float2(0.f, 0.f);
        for (int nn = -B; nn <= B; ++nn) {
            int r = (nn * k) % N;
            if (r < 0) r += N;
            const float2 s = sm.S[m * W + nn + B], e = sm.tw[r];
            acc.x = fmaf(s.x, e.x, fmaf(-s.y, e.y, acc.x));
            acc.y = fmaf(s.x, e.y, fmaf(s.y, e.x, acc.y));
        }
        sm.T[m * N + k] = acc;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < N * N; t += kSoftThreads) {
        const int j = t / N, k = t % N;
        float acc = 0.f;
        for (int m = 0; m <= B; ++m) {
            const int r = (m * j) % N;
            const float2 x = sm.T[m * N + k], e = sm.tw[r];
            acc = fmaf(x.x, e.x, fmaf(-x.y, e.y, acc));
        }
        out[t] = 2.f * acc;
    }
    __syncthreads();
}

// Offer the nodes of slice i (value ring slot ci, neighbours pi / ni, -1 when absent) to the list.
// want_max: offer local maxima (and count them); otherwise offer the other nodes.
__device__ void offer_slice(const SoftArgs &a, SoftSmem &sm, int i, int pslot, int cslot, int nslot, bool want_max)
{
    const int N = a.n;
    const float *cur = sm.ring[cslot];
    for (int base = 0; base < N * N; base += kSoftThreads) {
        const int t = base + threadIdx.x;
        bool offer = false;
        unsigned long long key = 0ull;
        if (t < N * N) {
            const int j = t / N, k = t % N;
            const uint32_t idx = (uint32_t)(i * N * N + t);
            const float v = cur[t];
            key = make_key(v, idx);
            bool is_max = true;
            for (int di = -1; di <= 1 && is_max; ++di) {
                const int slot = di < 0 ? pslot : (di > 0 ? nslot : cslot);
                if (slot < 0) continue;
                const float *pl = sm.ring[slot];
                const int ii = i + di;
                for (int dj = -1; dj <= 1; ++dj) {
                    const int jj = (j + dj + N) % N;
                    for (int dk = -1; dk <= 1; ++dk) {
                        if (!di && !dj && !dk) continue;
                        const int kk = (k + dk + N) % N;
                        const unsigned long long kn = make_key(pl[jj * N + kk], (uint32_t)(ii * N * N + jj * N + kk));
                        if (kn > key) is_max = false;
                    }
                }
            }
            offer = want_max ? is_max : !is_max;
            if (want_max && is_max) atomicAdd(sm.nmax, 1);
            if (offer && key <= (*sm.thresh)) offer = false;
        }
        if (offer) {
            const int slot = atomicAdd(sm.count, 1);
            sm.list[slot] = key;
        }
        __syncthreads();
        if ((*sm.count) > kListCap - kSoftThreads) compact_list(sm, a.Kc);
    }
}

// One sweep over the grid; offers maxima (want_max) or non-maxima to the list.
__device__ void soft_sweep(const SoftArgs &a, const float4 *Cp, SoftSmem &sm, bool want_max)
{
    const int N = a.n;
    for (int i = 0; i <= N; ++i) {
        if (i < N) {
            const double b = kPi * (2.0 * i + 1.0) / (2.0 * N);
            wigner_slice(a, Cp, sm, b);
            dft_slice(a, sm, sm.ring[i % 3]);
        }
        if (i >= 1) {
            const int ic = i - 1;
            const int pslot = ic >= 1 ? (ic - 1) % 3 : -1;
            const int nslot = ic + 1 < N ? (ic + 1) % 3 : -1;
            offer_slice(a, sm, ic, pslot, ic % 3, nslot, want_max);
        }
    }
}

__global__ void __launch_bounds__(kSoftThreads) k_soft_search(SoftArgs a)
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
    for (int t = threadIdx.x; t < N; t += kSoftThreads) {
        float s, c;
        sincosf((float)(kTwoPi * t / N), &s, &c);
        sm.tw[t] = make_float2(c, s);
    }
    if (threadIdx.x == 0) {
        (*sm.count) = 0;
        (*sm.nmax) = 0;
        (*sm.thresh) = 0ull;
    }
    __syncthreads();
    soft_sweep(a, Cp, sm, true);
    compact_list(sm, Kc);
    const int nmax = (*sm.nmax);
    const int nm = min(nmax, Kc);
    // ranked maxima -> cand[0 .. nm)
    for (int t = threadIdx.x; t < nm; t += kSoftThreads) {
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
        soft_sweep(a, Cp, sm, false);
        compact_list(sm, Kc - nm);
        for (int t = threadIdx.x; t < Kc - nm; t += kSoftThreads) {
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

hipError_t launch_soft(const SoftArgs &a, int P, hipStream_t s)
{
    hipLaunchKernelGGL(k_soft_search, dim3(P), dim3(kSoftThreads), soft_smem_size(a.n, a.B), s, a);
    return hipGetLastError();
}

}  // namespace matcha
