// k_soft.hip -- low-bandwidth SOFFT search (Sec. 2.3; Alg. 1, its first two steps).
//
// Four kernels per chunk of particles, with the node transforms, the grid and the maxima lists in
// an HBM workspace between them.
//
// k_soft_wigner forms, for every polar node b_i = pi (2i+1) / (2n) of a particle, the Wigner-d
// transform over l of the coefficients,
//   S_i[m, n] = sum_{l <= B} C^l_mn d^l_mn(b_i)   on the half plane {m > 0} U {m = 0, n >= 0},
// two workgroups per particle (half its nodes each) with its coefficients staged in LDS, one step
// of the sum serving a pair and its partner; the d values at the nodes come from a table shared
// by all particles.
//
// k_soft_grid_reg (small bands, operands in registers) or k_soft_grid (any band, operands in LDS)
// synthesises C_B on the n^3 grid (a_j = 2 pi j / n, c_k = 2 pi k / n) with the 2-D inverse DFT
// over (a, c), each wave taking a few polar nodes of one particle: first
// T[m][k] = sum_n S[m, n] e^{i n c_k}, then g[j][k] = 2 Re sum_m T[m][k] e^{i m a_j}.
//
// k_soft_maxima_q (n a multiple of 4; k_soft_maxima otherwise) takes a particle and a run of
// consecutive polar nodes per workgroup and tests every node for a local maximum against its 26
// neighbours (a subset of the neighbours first, then the exact test); each maximum's 64-bit key
// (ordered value, inverted linear index) is appended to the particle's list in the workspace.
//
// k_soft_rank takes one particle per workgroup, sorts its list and writes the Kc best keys, so
// the ranking is exact whatever order the maxima arrived in.  A particle whose list overflowed,
// or that has fewer than Kc maxima, takes the streaming path instead: its grid goes slice by
// slice through an LDS ring, the maxima enter an LDS key list that is sorted and cut to the Kc
// best now and then, and once Kc maxima are known the Kc-th best key is a threshold below which
// a node is dropped after one compare; a second sweep ranks the best non-maxima when there are
// fewer than Kc maxima.
#include "matcha_launch.hpp"

#include <algorithm>

namespace matcha {

// ---------------------------------------------------------------- grid synthesis
//
// Per polar node the 2-D inverse DFT is two real products on the matrix cores
// (v_mfma_f32_16x16x4_f32: lane i supplies A[i%16][i/16] and B[i/16][i%16] of a 16 x 4 x 16 step
// and holds D rows 4(i/16) .. +3 of column i%16):
//   stage 1  T = S B1:  A = S with (Re, Im) interleaved along K = 2(n+B) + c, B1r / B1i the
//            twiddles of e^{i n c_k} in the matching real form, giving Re T and Im T;
//   stage 2  g = A2 T':  A2[j][2m + c] = 2 cos(m a_j) / -2 sin(m a_j), T'[2m + c][k] = Re / Im T.
// In k_soft_grid, S and T' live in the wave's own LDS; B1 and A2 are host-built tables, in the
// workgroup's LDS or read through the caches.
constexpr int kGridSPW = 3;  // polar nodes per wave

struct GridGeom {
    int MT;   // 16-row tiles of m (B+1 rows)
    int KP;   // stage-1 K, 2(2B+1) padded to a multiple of 4
    int NP;   // k (and j) padded to a multiple of 16
    int KS2;  // stage-2 K steps: ceil(2(B+1) / 4)
    int K2R;  // rows of T' held: the 4 KS2 that stage 2 reads (two per m)
    int TF;   // floats of the DFT tables: B1r, B1i [KP][NP], A2 [NP][4 KS2]
};

__host__ __device__ inline GridGeom grid_geom(int n, int B)
{
    GridGeom g;
    g.MT = (B + 16) / 16;
    g.KP = 4 * ((2 * (2 * B + 1) + 3) / 4);
    g.NP = 16 * ((n + 15) / 16);
    g.KS2 = (2 * (B + 1) + 3) / 4;
    g.K2R = 4 * g.KS2;
    g.TF = 2 * g.KP * g.NP + g.NP * 4 * g.KS2;
    return g;
}

__host__ __device__ inline int grid_wave_floats(const GridGeom &g) { return 16 * g.MT * g.KP + g.K2R * g.NP; }

// LDS of a workgroup of `waves` waves, with the DFT tables in LDS (tab_lds) or read from memory.
__host__ __device__ inline size_t soft_grid_smem(int n, int B, int waves, bool tab_lds)
{
    const GridGeom g = grid_geom(n, B);
    return sizeof(float) * ((size_t)waves * grid_wave_floats(g) + (tab_lds ? (size_t)g.TF : 0));
}

// Launch shape: the tables go to LDS whenever one wave fits beside them; then up to four waves
// while the workgroup stays within 80 KB (two workgroups per CU).  Otherwise the tables are read
// through the caches and up to four waves share 64 KB.
struct GridShape {
    int waves;
    bool tab_lds;
};

inline GridShape soft_grid_shape(int n, int B)
{
    if (soft_grid_smem(n, B, 1, true) <= 160 * 1024) {
        for (int w : {4, 2})
            if (soft_grid_smem(n, B, w, true) <= 80 * 1024) return {w, true};
        return {1, true};
    }
    for (int w : {4, 2})
        if (soft_grid_smem(n, B, w, false) <= 64 * 1024) return {w, false};
    return {1, false};
}

// The two l-sums of one wedge pair at polar node b_i:
// u0 = sum_l C^l_pair dg0^l_pair(b_i), u1 = sum_l C^l_partner dg1^l_pair(b_i).  Four degrees per
// trip keep eight independent loads in flight.
__device__ __forceinline__ void wigner_sums(const float4 *__restrict__ Cp, const float2 *__restrict__ dg, int m, int q, int B,
                                   float2 &u0, float2 &u1)
{
    u0 = make_float2(0.f, 0.f);
    u1 = u0;
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
}

// Wigner-d transform of every polar node of the launch's particles into the half-plane array
// S[m][n + B] of the workspace; the pair's value goes to (m, n), its partner's to (n, m) (n >= 0)
// or (-n, -m) (n < 0).  kWignerSplit workgroups per particle, each taking a run of its nodes in
// whole LDS stages (with 4096 particles, 2 against 1 shortens the last partial round of resident
// workgroups: 279 against 287 us at four nodes per stage; 3, 4 and 6 took 291, 301 and 326 us,
// re-staging C each time).  Three nodes per stage then took 264 us (2, 4 and 6: 286, 279, 288).
// Each stages the particle's coefficients up to band B in LDS once (when they fit, CP_LDS), and
// each thread takes (node, pair) tasks with consecutive threads on consecutive pairs, so the node
// tables are read coalesced.  The entries (0, n < 0), the Hermitian mirrors of (0, -n), are
// written as zero by the (0, 0) pair's task.
constexpr int kWignerThreads = 256;
constexpr int kWignerStage = 3;  // polar nodes staged in LDS at a time
constexpr int kWignerSplit = 2;  // workgroups per particle, each taking a run of its polar nodes

// Polar nodes per workgroup: n split kWignerSplit ways, in whole LDS stages.
__host__ __device__ inline int soft_wigner_span(int n)
{
    const int per = (n + kWignerSplit - 1) / kWignerSplit;
    return (per + kWignerStage - 1) / kWignerStage * kWignerStage;
}

template <bool CP_LDS>
__global__ void __launch_bounds__(kWignerThreads) k_soft_wigner(SoftArgs a)
{
    extern __shared__ __align__(16) float4 cs[];
    const int B = a.B, N = a.n, W = 2 * B + 1;
    const int npairs = (B + 1) * (B + 1);
    const int span = soft_wigner_span(N);
    const int nsplit = (N + span - 1) / span;
    const int pl = blockIdx.x / nsplit, p = a.p0 + pl;
    const int ib = (blockIdx.x - pl * nsplit) * span, ie = min(ib + span, N);  // this workgroup's nodes
    const float4 *Cg = a.C + a.C_off[p] / 2;
    const float4 *Cp = Cg;
    if (CP_LDS) {
        const int rows = (int)wedge_row(B + 1);
        for (int t = threadIdx.x; t < rows; t += kWignerThreads) cs[t] = Cg[t];
        __syncthreads();
        Cp = cs;
    }
    const int64_t drow = wedge_row(B + 1);
    const int SW = (B + 1) * W;
    float2 *Sp = a.S + (int64_t)pl * N * SW;
    if (CP_LDS) {
        // kWignerStage nodes at a time into LDS (every entry of a node's array is written: the
        // partners fill the entries past the wedge), then out as one contiguous run, so the
        // partners' transposed positions never reach memory as scattered 8-byte writes
        float2 *sb = reinterpret_cast<float2 *>(cs + wedge_row(B + 1));
        for (int i0 = ib; i0 < ie; i0 += kWignerStage) {
            const int g = min(kWignerStage, ie - i0);
            for (int t = threadIdx.x; t < g * npairs; t += kWignerThreads) {
                const int il = t / npairs, q = t - (t / npairs) * npairs;
                const PairInfo pi = a.pinfo[q];
                const int m = pi.m, n = pi.n;
                float2 u0, u1;
                wigner_sums(Cp, a.dgrid + (i0 + il) * drow, m, q, B, u0, u1);
                float2 *S = sb + il * SW;
                S[m * W + n + B] = u0;
                if (n != m && n != -m) {  // diagonal pairs are their own partners
                    const int a2 = n >= 0 ? n : -n, b2 = n >= 0 ? m : -m;
                    S[a2 * W + b2 + B] = u1;
                }
                if (q == 0)
                    for (int k = 0; k < B; ++k) S[k] = make_float2(0.f, 0.f);
            }
            __syncthreads();
            float2 *dst = Sp + (int64_t)i0 * SW;
            for (int t = threadIdx.x; t < g * SW; t += kWignerThreads) dst[t] = sb[t];
            __syncthreads();
        }
        return;
    }
    for (int t = ib * npairs + threadIdx.x; t < ie * npairs; t += kWignerThreads) {
        const int i = t / npairs, q = t - (t / npairs) * npairs;
        const PairInfo pi = a.pinfo[q];
        const int m = pi.m, n = pi.n;
        float2 u0, u1;
        wigner_sums(Cp, a.dgrid + i * drow, m, q, B, u0, u1);
        float2 *S = Sp + (int64_t)i * SW;
        S[m * W + n + B] = u0;
        if (n != m && n != -m) {  // diagonal pairs are their own partners
            const int a2 = n >= 0 ? n : -n, b2 = n >= 0 ? m : -m;
            S[a2 * W + b2 + B] = u1;
        }
        if (q == 0)
            for (int k = 0; k < B; ++k) S[k] = make_float2(0.f, 0.f);
    }
}

inline size_t soft_wigner_smem(int B)
{
    return wedge_row(B + 1) * sizeof(float4) + sizeof(float2) * kWignerStage * (size_t)(B + 1) * (2 * B + 1);
}
inline bool soft_wigner_cp_lds(int B) { return soft_wigner_smem(B) <= 64 * 1024; }

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kGridChunk = 8;  // K steps whose operands are loaded before their MFMAs
// float2 values of a node's half-plane array prefetched per lane: all of it while
// (B+1)(2B+1) <= 8 * 64, i.e. B <= 15
constexpr int kGridSReg = 8;

template <bool TAB_LDS>
__global__ void __launch_bounds__(256) k_soft_grid(SoftArgs a)
{
    extern __shared__ __align__(16) float smem_f[];
    const int B = a.B, N = a.n;
    const GridGeom g = grid_geom(N, B);
    const int WB = a.gslices;  // waves per workgroup
    const int SB = WB * kGridSPW;
    const int NG = (N + SB - 1) / SB;
    const int pl = blockIdx.x / NG, ib = (blockIdx.x - pl * NG) * SB;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int col = lane % 16, kq = lane / 16;
    const float *tabs = a.dft;
    float *wbase = smem_f;
    if (TAB_LDS) {
        // the DFT tables, shared by the workgroup's waves (TF is a multiple of 4)
        for (int t = threadIdx.x; t < g.TF / 4; t += blockDim.x)
            reinterpret_cast<float4 *>(smem_f)[t] = reinterpret_cast<const float4 *>(a.dft)[t];
        __syncthreads();
        tabs = smem_f;
        wbase = smem_f + g.TF;
    }
    float *Sf = wbase + wave * grid_wave_floats(g);  // [16 MT][KP]
    float *Tf = Sf + 16 * g.MT * g.KP;              // [K2R][NP]
    const float *B1r = tabs, *B1i = B1r + g.KP * g.NP, *A2 = B1i + g.KP * g.NP;
    const int A2W = 4 * g.KS2;
    if (ib == 0 && threadIdx.x == 0) a.mcount[pl] = 0u;  // the maxima kernel that follows appends from 0
    const int KS1 = g.KP / 4, NT = g.NP / 16;
    // the padding rows and columns of S stay zero; each node overwrites the rest
    for (int t = lane; t < 16 * g.MT * g.KP; t += kWave) Sf[t] = 0.f;
    const int W = 2 * B + 1, SW = (B + 1) * W;
    const float2 *Sb = a.S + (int64_t)pl * N * SW;
    const int i_first = ib + wave * kGridSPW;
    const int i_last = min(i_first + kGridSPW, N) - 1;  // the wave's polar nodes
    // S of a node is read at clamped addresses, all of a lane's loads in flight together; the
    // next node's values are loaded while the current node runs on the matrix cores
    float2 sv[kGridSReg];
    auto load_s = [&](int i) {
        const float2 *Sg = Sb + (int64_t)min(i, N - 1) * SW;
#pragma unroll
        for (int u = 0; u < kGridSReg; ++u) sv[u] = Sg[min(u * kWave + lane, SW - 1)];
    };
    if (i_first < N) load_s(i_first);
    auto put_s = [&](int t, float2 v) {
        const int mm = t / W, nn = t - (t / W) * W;
        Sf[mm * g.KP + 2 * nn] = v.x;
        Sf[mm * g.KP + 2 * nn + 1] = v.y;
    };
    for (int i = i_first; i <= i_last; ++i) {
        // S into the interleaved rows of Sf (the padding stays zero): the prefetched head, then
        // (B > 15) the rest, eight loads in flight per lane
#pragma unroll
        for (int u = 0; u < kGridSReg; ++u)
            if (u * kWave + lane < SW) put_s(u * kWave + lane, sv[u]);
        const float2 *Sg = Sb + (int64_t)i * SW;
        for (int t0 = kGridSReg * kWave; t0 < SW; t0 += 8 * kWave) {
            float2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = Sg[min(t0 + u * kWave + lane, SW - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (t0 + u * kWave + lane < SW) put_s(t0 + u * kWave + lane, v[u]);
        }
        wave_sync();
        if (i < i_last) load_s(i + 1);
        // stage 1: Re T and Im T, rows m, columns k
        for (int tn = 0; tn < NT; ++tn)
            for (int tm = 0; tm < g.MT; ++tm) {
                f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
                for (int s0 = 0; s0 < KS1; s0 += kGridChunk) {
                    float av[kGridChunk], br[kGridChunk], bi[kGridChunk];
#pragma unroll
                    for (int s = 0; s < kGridChunk; ++s) {
                        if (s0 + s < KS1) {
                            const int kk = 4 * (s0 + s) + kq;
                            av[s] = Sf[(16 * tm + col) * g.KP + kk];
                            br[s] = B1r[kk * g.NP + 16 * tn + col];
                            bi[s] = B1i[kk * g.NP + 16 * tn + col];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int s = 0; s < kGridChunk; ++s) {
                        if (s0 + s < KS1) {
                            cr = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], br[s], cr, 0, 0, 0);
                            ci = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bi[s], ci, 0, 0, 0);
                        }
                    }
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = 16 * tm + 4 * kq + v;  // rows past K2R are zero and never read
                    if (2 * m + 1 < g.K2R) {
                        Tf[(2 * m) * g.NP + 16 * tn + col] = cr[v];
                        Tf[(2 * m + 1) * g.NP + 16 * tn + col] = ci[v];
                    }
                }
            }
        wave_sync();
        // stage 2: g[j][k] = sum_K A2[j][K] T'[K][k], straight to the workspace
        float *out = a.grid + ((int64_t)pl * N + i) * N * N;
        for (int tj = 0; tj < NT; ++tj)
            for (int tk = 0; tk < NT; ++tk) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                for (int s0 = 0; s0 < g.KS2; s0 += kGridChunk) {
                    float av[kGridChunk], bv[kGridChunk];
#pragma unroll
                    for (int s = 0; s < kGridChunk; ++s) {
                        if (s0 + s < g.KS2) {
                            const int kk = 4 * (s0 + s) + kq;
                            av[s] = A2[(16 * tj + col) * A2W + kk];
                            bv[s] = Tf[kk * g.NP + 16 * tk + col];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int s = 0; s < kGridChunk; ++s)
                        if (s0 + s < g.KS2) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
                }
                const int k = 16 * tk + col;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = 16 * tj + 4 * kq + v;
                    if (j < N && k < N) out[j * N + k] = acc[v];
                }
            }
        wave_sync();  // the next node overwrites S and T'
    }
}

// ---------------------------------------------------------------- grid synthesis in registers
//
// The same two products for small bands, with no LDS: every operand lives in registers.
//   * The DFT tables are the same for every node and particle: each lane loads its B1r operands
//     (stage 1) and A2 operands (stage 2) once, (B+1) NT + NT (B+2)/2 floats.  B1i's rows are
//     B1r's rows swapped in pairs (2n' <-> 2n'+1, the even ones negated), and the rows of a pair
//     sit in lane rows q and q^1, so each B1i operand is formed just before its use with one
//     v_permlane16_swap (exchanging lane rows 0 <-> 1 and 2 <-> 3) and a sign.
//   * Stage 1's A operand, lane (q, c) taking S[m = c][4 s + q], is loaded straight from the
//     workspace; the next node's is loaded while the current one runs on the matrix cores (two
//     register sets in turn, so no register copy waits for those loads).
//   * Stage 2's B operand is T' = (Re T, Im T) interleaved by row, 2m + c.  Stage 1 leaves lane
//     (q, c) holding rows m = 4q .. 4q+3 of column c; stage 2 wants in lane (q, c), for K step s,
//     row 2s + (q >> 1), part q & 1.  For s = 2r that is register q (of Re T0, Im T0, Re T1,
//     Im T1) of lane row r, for s = 2r + 1 register q of (Re T2, Im T2, Re T3, Im T3): a 4 x 4
//     transpose between the four 16-lane rows, done with two rounds of lane-row swaps
//     (v_permlane32_swap exchanges rows 2-3 of one register with rows 0-1 of another,
//     v_permlane16_swap rows 1 and 3 of one with rows 0 and 2 of another).
// A wave takes a.grid_nodes consecutive nodes (in a particle-major order) on its own; an even count
// (the node loop is unrolled by two), kGridRegNodes by default.
constexpr int kGridRegNodes = 16;

// In-register 4 x 4 transpose across lane rows: x[j] of row r becomes x[r] of row j.
__device__ __forceinline__ void transpose_rows(float (&x)[4])
{
    auto s02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[0]), __float_as_uint(x[2]), false, false);
    auto s13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[1]), __float_as_uint(x[3]), false, false);
    auto s01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
    auto s23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
    x[0] = __uint_as_float(s01[0]);
    x[1] = __uint_as_float(s01[1]);
    x[2] = __uint_as_float(s23[0]);
    x[3] = __uint_as_float(s23[1]);
}

// Stage 1's A operand of node nd (clamped to the launch): S[m = col][4 s + kq], zero outside.
template <int BB>
__device__ __forceinline__ void load_node_s(const SoftArgs &a, int nd, int nodes, int col, int kq, float (&v)[BB + 1])
{
    constexpr int W = 2 * BB + 1, SWF = 2 * W;
    const float *base = reinterpret_cast<const float *>(a.S + (int64_t)min(nd, nodes - 1) * (BB + 1) * W);
    const float mok = col <= BB ? 1.f : 0.f;
    const int row = min(col, BB) * SWF;
#pragma unroll
    for (int s = 0; s <= BB; ++s) {
        const int K = 4 * s + kq;
        v[s] = base[row + min(K, SWF - 1)] * (K < SWF ? mok : 0.f);
    }
}

template <int BB, int NT>
__device__ __forceinline__ void grid_reg_node(const SoftArgs &a, int nd, bool active, int col, int kq,
                                              const float (&br)[NT][BB + 1],
                                              const float (&a2)[NT][(BB + 2) / 2], const float (&s1)[BB + 1])
{
    constexpr int KS1 = BB + 1, KS2 = (BB + 2) / 2;
    if (!active) return;
    const int N = a.n;
    const int pl = nd / N, i = nd - (nd / N) * N;
    if (i == 0 && threadIdx.x % kWave == 0) a.mcount[pl] = 0u;  // the maxima kernel that follows appends from 0
    // stage 1: Re T and Im T, rows m, columns k of each column tile
    f32x4 cr[NT], ci[NT];
#pragma unroll
    for (int tn = 0; tn < NT; ++tn) cr[tn] = ci[tn] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS1; ++s)
#pragma unroll
        for (int tn = 0; tn < NT; ++tn) {
            cr[tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(s1[s], br[tn][s], cr[tn], 0, 0, 0);
            // B1i[2n'][k] = -B1r[2n'+1][k], B1i[2n'+1][k] = B1r[2n'][k]: lane row q takes row q^1
            const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(br[tn][s]), __float_as_uint(br[tn][s]), false, false);
            const float bis = (kq & 1) ? __uint_as_float(sw[0]) : -__uint_as_float(sw[1]);
            ci[tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(s1[s], bis, ci[tn], 0, 0, 0);
        }
    // T' operands of stage 2: b2[tn][s], s = 0 .. 7
    float b2[NT][8];
#pragma unroll
    for (int tn = 0; tn < NT; ++tn) {
        float x[4] = {cr[tn][0], ci[tn][0], cr[tn][1], ci[tn][1]};
        float y[4] = {cr[tn][2], ci[tn][2], cr[tn][3], ci[tn][3]};
        transpose_rows(x);
        transpose_rows(y);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            b2[tn][2 * r] = x[r];
            b2[tn][2 * r + 1] = y[r];
        }
    }
    // stage 2: g[j][k] = sum_K A2[j][K] T'[K][k], straight to the workspace
    float *out = a.grid + (int64_t)nd * N * N;
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
        for (int tk = 0; tk < NT; ++tk) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS2; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[tj][s], b2[tk][s], acc, 0, 0, 0);
            const int k = 16 * tk + col;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * tj + 4 * kq + v;
                if (j < N && k < N) out[j * N + k] = acc[v];
            }
        }
}

template <int BB, int NT>
__global__ void __launch_bounds__(256) k_soft_grid_reg(SoftArgs a)
{
    static_assert(BB + 1 <= 16 && (BB + 2) / 2 <= 8, "one 16-row tile of m, at most 8 stage-2 K steps");
    constexpr int KS1 = BB + 1, KS2 = (BB + 2) / 2, KP = 4 * KS1, NP = 16 * NT, A2W = 4 * KS2;
    const int lane = threadIdx.x % kWave, col = lane % 16, kq = lane / 16;
    const int nodes = a.np * a.n;
    const int nd0 = (blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * a.grid_nodes;
    if (nd0 >= nodes) return;  // no barrier in this kernel
    const int nd1 = min(nd0 + a.grid_nodes, nodes);
    const float *B1r = a.dft, *A2 = a.dft + 2 * KP * NP;
    float br[NT][KS1], a2[NT][KS2];
#pragma unroll
    for (int tn = 0; tn < NT; ++tn) {
#pragma unroll
        for (int s = 0; s < KS1; ++s) {
            br[tn][s] = B1r[(4 * s + kq) * NP + 16 * tn + col];
        }
#pragma unroll
        for (int s = 0; s < KS2; ++s) a2[tn][s] = A2[(16 * tn + col) * A2W + 4 * s + kq];
    }
    float s0[KS1], s1[KS1];
    load_node_s<BB>(a, nd0, nodes, col, kq, s0);
    for (int nd = nd0; nd < nd1; nd += 2) {
        load_node_s<BB>(a, nd + 1, nodes, col, kq, s1);
        grid_reg_node<BB, NT>(a, nd, true, col, kq, br, a2, s0);
        load_node_s<BB>(a, nd + 2, nodes, col, kq, s0);
        grid_reg_node<BB, NT>(a, nd + 1, nd + 1 < nd1, col, kq, br, a2, s1);
    }
}

// The register-resident kernel needs the B+1 rows of m in one 16-row tile and stage 2's K steps
// within the 8 that the transpose forms (B <= 14); it is built for B = 12 on grids of 33 .. 48
// nodes per axis and B = 8 on grids of 17 .. 32.
inline bool soft_grid_reg_shape(int n, int B) { return (B == 12 && n > 32 && n <= 48) || (B == 8 && n > 16 && n <= 32); }

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
__device__ __forceinline__ bool beats_all(const SoftArgs &a, const SoftSmem &sm, int i, int t, int pslot, int cslot,
                                          int nslot)
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

// ---------------------------------------------------------------- parallel maxima
constexpr int kMaxThreads = 256;
constexpr int kMaxSlices = 8;    // polar nodes tested per workgroup, any n
constexpr int kMaxQSlices = 16;  // polar nodes tested per workgroup, n a multiple of 4

__host__ __device__ inline size_t soft_maxima_smem(int n) { return 3 * soft_align16(sizeof(float) * n * n); }
// Candidate queue of the n-multiple-of-4 maxima kernel: n^2 / 2 entries for a run of up to 16
// slices (a band-limited grid has far fewer nodes that top their six axis neighbours).
__host__ __device__ inline int soft_maxima_qcap(int n) { return n * n / 2; }
// two slice planes and the queue
__host__ __device__ inline size_t soft_maxima_q_smem(int n)
{
    return 2 * soft_align16(sizeof(float) * n * n) + soft_align16(sizeof(uint32_t) * soft_maxima_qcap(n));
}

__device__ __forceinline__ void append_maximum(const SoftArgs &a, int pl, float v, uint32_t idx)
{
    const uint32_t slot = atomicAdd(a.mcount + pl, 1u);
    if (slot < (uint32_t)a.mcap) a.mlist[(int64_t)pl * a.mcap + slot] = make_key(v, idx);
}

// Any n: a workgroup streams its slices (plus one neighbour slice on each side) through an LDS
// ring of three; a node whose value is at least the largest of its six axis neighbours (absent
// slices count as -inf) takes the exact test.
__global__ void __launch_bounds__(kMaxThreads) k_soft_maxima(SoftArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int N = a.n, NN = N * N;
    const int NG = (N + kMaxSlices - 1) / kMaxSlices;
    const int pl = blockIdx.x / NG, i0 = (blockIdx.x - pl * NG) * kMaxSlices;
    const int i1 = min(i0 + kMaxSlices, N);  // tests slices i0 .. i1-1
    SoftSmem sm;
    sm.ring0 = reinterpret_cast<float *>(smem_raw);
    sm.plane = (int)(soft_align16(sizeof(float) * NN) / sizeof(float));
    const float *grid = a.grid + (int64_t)pl * N * NN;
    // slice s lives in ring slot s mod 3
    for (int s = max(i0 - 1, 0); s <= min(i0 + 1, N - 1); ++s)
        for (int t = threadIdx.x; t < NN; t += kMaxThreads) sm.ring(s % 3)[t] = grid[(int64_t)s * NN + t];
    __syncthreads();
    for (int ic = i0; ic < i1; ++ic) {
        const int pslot = ic >= 1 ? (ic - 1) % 3 : -1;
        const int cslot = ic % 3;
        const int nslot = ic + 1 < N ? (ic + 1) % 3 : -1;
        const float *cur = sm.ring(cslot);
        for (int t = threadIdx.x; t < NN; t += kMaxThreads) {
            const float v = cur[t];
            const int j = t / N, k = t - (t / N) * N;
            const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
            const int km = k == 0 ? N - 1 : k - 1, kp = k == N - 1 ? 0 : k + 1;
            float mx = fmaxf(fmaxf(cur[jm * N + k], cur[jp * N + k]), fmaxf(cur[j * N + km], cur[j * N + kp]));
            if (pslot >= 0) mx = fmaxf(mx, sm.ring(pslot)[t]);
            if (nslot >= 0) mx = fmaxf(mx, sm.ring(nslot)[t]);
            if (v >= mx && beats_all<kMaxThreads>(a, sm, ic, t, pslot, cslot, nslot))
                append_maximum(a, pl, v, (uint32_t)(ic * NN + t));
        }
        __syncthreads();
        if (ic + 1 < i1 && ic + 2 < N)  // slice ic+2 replaces ic-1
            for (int t = threadIdx.x; t < NN; t += kMaxThreads)
                sm.ring((ic + 2) % 3)[t] = grid[(int64_t)(ic + 2) * NN + t];
        __syncthreads();
    }
}

// Exact test of node t of slice i (value v) against its 26 neighbours, read from the grid in
// memory: a neighbour beats it with a larger key (ordered value bits, then the smaller linear
// index).  Loads take a uniform slice base and a 32-bit byte offset.
__device__ __forceinline__ bool beats_all_mem(const float *grid, int N, int i, int t, float v)
{
    const int NN = N * N;
    const int j = t / N, k = t - (t / N) * N;
    const uint32_t rows[3] = {(uint32_t)((j == 0 ? N - 1 : j - 1) * N), (uint32_t)(j * N),
                              (uint32_t)((j == N - 1 ? 0 : j + 1) * N)};
    const uint32_t cols[3] = {(uint32_t)(k == 0 ? N - 1 : k - 1), (uint32_t)k, (uint32_t)(k == N - 1 ? 0 : k + 1)};
    const uint32_t ov = ordered_bits(v);
    const uint32_t idx = (uint32_t)(i * NN + t);
    bool win = true;
#pragma unroll 1
    for (int di = 0; di < 3; ++di) {
        const int s = i + di - 1;
        if (s < 0 || s >= N) continue;
        const char *pl = reinterpret_cast<const char *>(grid + (int64_t)s * NN);
        float nb[9];
#pragma unroll
        for (int d = 0; d < 9; ++d) nb[d] = *reinterpret_cast<const float *>(pl + 4u * (rows[d / 3] + cols[d % 3]));
        // bitwise operators keep the compares branch-free; the node itself never beats itself
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            const uint32_t o = (uint32_t)(s * NN) + rows[d / 3] + cols[d % 3];
            const uint32_t ou = ordered_bits(nb[d]);
            win &= !((ou > ov) | ((ou == ov) & (o < idx)));
        }
    }
    return win;
}

// One slice's float4 quads of this thread (quad threadIdx.x + u * kMaxThreads), slice s clamped
// to [0, n): unconditional loads at clamped addresses, so that the number in flight is known
// where they are consumed (a load skipped on some path would force a full wait).
template <int PER>
__device__ __forceinline__ void load_quads(const float *grid, int N, int NQ, int s, float4 (&dst)[PER])
{
    const char *base = reinterpret_cast<const char *>(grid + (int64_t)min(max(s, 0), N - 1) * 4 * NQ);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const uint32_t qd = (uint32_t)min((int)threadIdx.x + u * kMaxThreads, NQ - 1);
        dst[u] = *reinterpret_cast<const float4 *>(base + 16u * qd);
    }
}

// n a multiple of 4: each thread owns up to PER float4 quads of a slice and carries them through
// the workgroup's slices with the previous and next slice's quads in registers, so the three-
// slice window costs no LDS.  Only the current slice goes to LDS (double-buffered), for the row
// and column neighbours.  The slice after next is loaded while the current one is tested; the
// four register sets change roles from slice to slice (the slice loop is unrolled by four), so
// no register copy waits for those loads.
//   A node at least the largest of up to 14 of its neighbours (the 6 axis ones, and the
// k-neighbours in the rows above and below and in the previous and next slice where the quad
// holds them, with no further loads) is a candidate: about 3 per local maximum on band-limited
// grids, against 7 with the axis neighbours alone.  Candidates are queued in LDS (linear node index) for the whole run of
// slices and take the exact test in one pass at the end, reading the grid in memory: memory loads are counted in issue order, so an
// exact test between two slices would wait for the prefetched slice too.  A queue that
// overflows (a flat grid, where every node ties with its neighbours) is ignored and every node
// of the run takes the exact test instead.
//   One barrier per slice: the LDS plane written for slice ic was last read for slice ic-2,
// before the barrier of slice ic-1.
struct MaximaQ {
    const float *grid;
    float *lds0;
    uint32_t *queue;
    uint32_t *qcount;
    int N, NN, NQ, QR, plane, i1, qcap;
};

template <int PER>
__device__ __forceinline__ void maxima_q_slice(const MaximaQ &M, int ic, const float4 (&prv)[PER], const float4 (&cur)[PER],
                                               const float4 (&nxt)[PER], float4 (&nn2)[PER])
{
    // Past the run's end (its length not a multiple of four) a step still loads and waits, so
    // that every path issues the same loads, and tests nothing.
    const int N = M.N, QR = M.QR;
    float *lc = M.lds0 + (ic & 1) * M.plane;
    float4 *lc4 = reinterpret_cast<float4 *>(lc);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int qd = threadIdx.x + u * kMaxThreads;
        if (qd < M.NQ) lc4[qd] = cur[u];
    }
    // slice ic+2, needed from slice ic+1 on; past the run's last slice, slice i1 is reloaded
    load_quads<PER>(M.grid, N, M.NQ, min(ic + 2, M.i1), nn2);
    __syncthreads();
    const bool hp = ic >= 1, hn = ic + 1 < N;  // absent slices count as -inf
    const float ninf = -__builtin_huge_valf();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int qd = threadIdx.x + u * kMaxThreads;
        if (qd < M.NQ && ic < M.i1) {
            const int j = qd / QR, kq = qd - (qd / QR) * QR, k0 = 4 * kq;
            const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
            const float4 c = cur[u], up = lc4[jm * QR + kq], dn = lc4[jp * QR + kq];
            const float left = lc[j * N + (k0 == 0 ? N - 1 : k0 - 1)];
            const float right = lc[j * N + (k0 + 4 == N ? 0 : k0 + 4)];
            const float4 pv = hp ? prv[u] : make_float4(ninf, ninf, ninf, ninf);
            const float4 nv = hn ? nxt[u] : make_float4(ninf, ninf, ninf, ninf);
            const float vv[4] = {c.x, c.y, c.z, c.w}, uu[4] = {up.x, up.y, up.z, up.w};
            const float dd[4] = {dn.x, dn.y, dn.z, dn.w};
            const float ll[4] = {left, c.x, c.y, c.z}, rr[4] = {c.y, c.z, c.w, right};
            const float pp[4] = {pv.x, pv.y, pv.z, pv.w}, qq[4] = {nv.x, nv.y, nv.z, nv.w};
            // the 6 axis neighbours, and the k-neighbours in the rows above and below and in the
            // previous and next slice where the quad holds them (a true maximum passes any subset
            // of its 26 neighbours)
            unsigned cand = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float mx = fmaxf(fmaxf(fmaxf(uu[q], dd[q]), fmaxf(ll[q], rr[q])), fmaxf(pp[q], qq[q]));
                if (q > 0) mx = fmaxf(mx, fmaxf(fmaxf(uu[q - 1], dd[q - 1]), fmaxf(pp[q - 1], qq[q - 1])));
                if (q < 3) mx = fmaxf(mx, fmaxf(fmaxf(uu[q + 1], dd[q + 1]), fmaxf(pp[q + 1], qq[q + 1])));
                cand |= (vv[q] >= mx ? 1u : 0u) << q;
            }
            if (cand) {
                uint32_t e = atomicAdd(M.qcount, (uint32_t)__builtin_popcount(cand));
                for (; cand; ++e) {
                    if (e < (uint32_t)M.qcap) M.queue[e] = (uint32_t)(ic * M.NN + j * N + k0 + __builtin_ctz(cand));
                    cand &= cand - 1;
                }
            }
        }
    }
}

template <int PER>
__global__ void __launch_bounds__(kMaxThreads) k_soft_maxima_q(SoftArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ uint32_t qcount;
    MaximaQ M;
    M.N = a.n;
    M.NN = M.N * M.N;
    M.NQ = M.NN / 4;
    M.QR = M.N / 4;
    const int NG = (M.N + kMaxQSlices - 1) / kMaxQSlices;
    const int pl = blockIdx.x / NG;
    const int i0 = (blockIdx.x - pl * NG) * kMaxQSlices;
    M.i1 = min(i0 + kMaxQSlices, M.N);  // tests slices i0 .. i1-1
    M.plane = (int)(soft_align16(sizeof(float) * M.NN) / sizeof(float));
    M.lds0 = reinterpret_cast<float *>(smem_raw);
    M.queue = reinterpret_cast<uint32_t *>(M.lds0 + 2 * M.plane);
    M.qcap = soft_maxima_qcap(M.N);
    M.qcount = &qcount;
    M.grid = a.grid + (int64_t)pl * M.N * M.NN;
    float4 r0[PER], r1[PER], r2[PER], r3[PER];
    load_quads<PER>(M.grid, M.N, M.NQ, i0 - 1, r0);
    load_quads<PER>(M.grid, M.N, M.NQ, i0, r1);
    load_quads<PER>(M.grid, M.N, M.NQ, i0 + 1, r2);
    if (threadIdx.x == 0) qcount = 0u;
    for (int ic = i0; ic < M.i1; ic += 4) {
        maxima_q_slice<PER>(M, ic, r0, r1, r2, r3);
        maxima_q_slice<PER>(M, ic + 1, r1, r2, r3, r0);
        maxima_q_slice<PER>(M, ic + 2, r2, r3, r0, r1);
        maxima_q_slice<PER>(M, ic + 3, r3, r0, r1, r2);
    }
    __syncthreads();
    const uint32_t nc = qcount;
    if (nc <= (uint32_t)M.qcap) {
        for (uint32_t e = threadIdx.x; e < nc; e += kMaxThreads) {
            const uint32_t idx = M.queue[e];
            const int i = (int)(idx / (uint32_t)M.NN), t = (int)(idx - (uint32_t)i * M.NN);
            const float v = M.grid[idx];
            if (beats_all_mem(M.grid, M.N, i, t, v)) append_maximum(a, pl, v, idx);
        }
    } else {
        for (int idx = i0 * M.NN + threadIdx.x; idx < M.i1 * M.NN; idx += kMaxThreads) {
            const int i = idx / M.NN, t = idx - i * M.NN;
            const float v = M.grid[idx];
            if (beats_all_mem(M.grid, M.N, i, t, v)) append_maximum(a, pl, v, (uint32_t)idx);
        }
    }
}

// Quads per thread of the n-multiple-of-4 maxima kernel.
inline int soft_maxima_per(int n)
{
    const int nq = n * n / 4;
    for (int per : {3, 4, 6, 9})
        if (nq <= per * kMaxThreads) return per;
    return 0;
}

// Ranking of one particle's maxima (fast path), or the streaming search when its list
// overflowed or holds fewer than Kc keys.  The list capacity a.mcap equals list_cap<NT>().
template <int NT>
__global__ void __launch_bounds__(NT) k_soft_rank(SoftArgs a)
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
    const uint32_t cnt = a.mcount[pl];
    if (cnt >= (uint32_t)Kc && cnt <= (uint32_t)a.mcap) {
        int sz = 2;
        while (sz < (int)cnt) sz <<= 1;
        const unsigned long long *src = a.mlist + (int64_t)pl * a.mcap;
        for (int t = threadIdx.x; t < sz; t += NT) sm.list[t] = t < (int)cnt ? src[t] : 0ull;
        __syncthreads();
        sort_list_desc<NT>(sm, sz);
        for (int t = threadIdx.x; t < Kc; t += NT) a.cand[(int64_t)p * Kc + t] = key_to_cand(sm.list[t], N);
        if (threadIdx.x == 0) a.status[p] = 0u;
        return;
    }
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
        // fill with the best nodes that are not local maxima (second sweep)
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

size_t soft_grid_smem_bytes(int n, int B)
{
    const GridShape sh = soft_grid_shape(n, B);
    return soft_grid_smem(n, B, sh.waves, sh.tab_lds);
}

size_t soft_select_smem_bytes(int n, int threads)
{
    return std::max(soft_select_smem(n, 2 * threads), soft_maxima_smem(n));
}

hipError_t launch_soft_wigner(const SoftArgs &a, int P, hipStream_t s)
{
    const int span = soft_wigner_span(a.n), wsplit = (a.n + span - 1) / span;
    if (soft_wigner_cp_lds(a.B))
        hipLaunchKernelGGL(k_soft_wigner<true>, dim3(P * wsplit), dim3(kWignerThreads), soft_wigner_smem(a.B), s, a);
    else
        hipLaunchKernelGGL(k_soft_wigner<false>, dim3(P * wsplit), dim3(kWignerThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_soft_grid(const SoftArgs &a0, int P, hipStream_t s)
{
    SoftArgs a = a0;
    a.np = P;
    if (soft_grid_reg_shape(a.n, a.B)) {
        if (a.grid_nodes < 2 || (a.grid_nodes & 1)) a.grid_nodes = kGridRegNodes;
        const int waves = (P * a.n + a.grid_nodes - 1) / a.grid_nodes;
        if (a.B == 12)
            hipLaunchKernelGGL((k_soft_grid_reg<12, 3>), dim3((waves + 3) / 4), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_soft_grid_reg<8, 2>), dim3((waves + 3) / 4), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const GridShape sh = soft_grid_shape(a.n, a.B);
    a.gslices = sh.waves;
    const int SB = a.gslices * kGridSPW;
    const int NG = (a.n + SB - 1) / SB;
    const size_t smem = soft_grid_smem(a.n, a.B, sh.waves, sh.tab_lds);
    if (sh.tab_lds)
        hipLaunchKernelGGL(k_soft_grid<true>, dim3(P * NG), dim3(kWave * a.gslices), smem, s, a);
    else
        hipLaunchKernelGGL(k_soft_grid<false>, dim3(P * NG), dim3(kWave * a.gslices), smem, s, a);
    return hipGetLastError();
}

size_t soft_dft_floats(int n, int B) { return (size_t)grid_geom(n, B).TF; }

// The DFT tables of k_soft_grid for (B, n), in FP64 with each angle reduced exactly as
// (integer mod n) / n, rounded once: B1r, B1i [KP][NP], then A2 [NP][4 KS2]; padding is zero.
void build_soft_dft(int B, int n, float *t)
{
    const GridGeom g = grid_geom(n, B);
    const size_t nf = soft_dft_floats(n, B);
    for (size_t x = 0; x < nf; ++x) t[x] = 0.f;
    float *B1r = t, *B1i = t + (size_t)g.KP * g.NP, *A2 = B1i + (size_t)g.KP * g.NP;
    const int W = 2 * B + 1;
    for (int np = 0; np < W; ++np)
        for (int k = 0; k < n; ++k) {
            const int nn = np - B;
            const int r = (((nn * k) % n) + n) % n;
            const double th = 2.0 * kPi * r / n;
            const double c = cos(th), sn = sin(th);
            B1r[(2 * np) * g.NP + k] = (float)c;
            B1i[(2 * np) * g.NP + k] = (float)sn;
            B1r[(2 * np + 1) * g.NP + k] = (float)(-sn);
            B1i[(2 * np + 1) * g.NP + k] = (float)c;
        }
    const int A2W = 4 * g.KS2;
    for (int j = 0; j < n; ++j)
        for (int m = 0; m <= B; ++m) {
            const double ph = 2.0 * kPi * ((m * j) % n) / n;
            A2[j * A2W + 2 * m] = (float)(2.0 * cos(ph));
            A2[j * A2W + 2 * m + 1] = (float)(-2.0 * sin(ph));
        }
}

hipError_t launch_soft_select(const SoftArgs &a0, int P, int threads, hipStream_t s)
{
    if (a0.n > kSelMaxN || (threads != 256 && threads != 512)) return hipErrorInvalidValue;
    SoftArgs a = a0;
    a.mcap = 2 * threads;  // == list_cap<threads>()
    const int per = a.n % 4 == 0 ? soft_maxima_per(a.n) : 0;
    const int NGq = (a.n + kMaxQSlices - 1) / kMaxQSlices, NG = (a.n + kMaxSlices - 1) / kMaxSlices;
    const size_t qs = soft_maxima_q_smem(a.n);
    if (per == 3)
        hipLaunchKernelGGL(k_soft_maxima_q<3>, dim3(P * NGq), dim3(kMaxThreads), qs, s, a);
    else if (per == 4)
        hipLaunchKernelGGL(k_soft_maxima_q<4>, dim3(P * NGq), dim3(kMaxThreads), qs, s, a);
    else if (per == 6)
        hipLaunchKernelGGL(k_soft_maxima_q<6>, dim3(P * NGq), dim3(kMaxThreads), qs, s, a);
    else if (per == 9)
        hipLaunchKernelGGL(k_soft_maxima_q<9>, dim3(P * NGq), dim3(kMaxThreads), qs, s, a);
    else
        hipLaunchKernelGGL(k_soft_maxima, dim3(P * NG), dim3(kMaxThreads), soft_maxima_smem(a.n), s, a);
    if (threads == 256)
        hipLaunchKernelGGL(k_soft_rank<256>, dim3(P), dim3(256), soft_select_smem(a.n, list_cap<256>()), s, a);
    else
        hipLaunchKernelGGL(k_soft_rank<512>, dim3(P), dim3(512), soft_select_smem(a.n, list_cap<512>()), s, a);
    return hipGetLastError();
}

}  // namespace matcha
