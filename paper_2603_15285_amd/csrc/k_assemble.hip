// k_assemble.hip -- coefficient assembly, eq. sigmalmm (Sec. 2.1, App. A.5):
//   C^l_mn = sum_{r < R_p} w_r f_lm(r) conj(h_ln(r)),  l <= L_p,
// for the half plane m >= 0 of each degree (Hermitian-symmetric inputs), written into the
// wedge layout: the value at (m, n) lands in slot 0 of the wedge pair (m, n) when |n| <= m,
// otherwise in slot 1 (the partner slot) of the pair (n, m) (n > 0) or (-n, -m) (n < 0).
//
// The template h is shared by every particle, so per degree the whole batch is one tall
// product: the rows (p, m), m <= l, of all particles stacked, times the template's (2l+1)
// columns.  In real form, with the shells interleaved (Re, Im) along K = 2R,
//   Cr[row][j] = sum_k A[row][k] Br[k][j],  Ci[row][j] = sum_k A[row][k] Bi[k][j],
//   A[(p,m)][2r] = w_r Re f_lm(r),  A[(p,m)][2r+1] = w_r Im f_lm(r),
//   Br[2r][j] = Re h,  Br[2r+1][j] = Im h,  Bi[2r][j] = -Im h,  Bi[2r+1][j] = Re h,
// on the matrix cores in FP32 (v_mfma_f32_16x16x4_f32: lane i supplies A[i%16][i/16] and
// B[i/16][i%16] of a 16 x 4 x 16 step and holds D rows 4(i/16) .. +3 of column i%16).
//
// A workgroup takes one degree and a run of 16-row tiles of its stacked rows.  It copies the
// template's degree-l row, h_l(r) for all shells, into LDS once; each wave then loads the A
// column of a row tile straight from f (every f value is read once), keeps it in registers
// and sweeps the column tiles with B from LDS.  Rows of one tile may belong to several
// particles, so small degrees still fill the 16-row tiles.  When the band limits differ, the
// rows of degree l cover only the particles with L_p >= l: the particles are taken in the
// order of decreasing L_p (k_order_by_L), of which the first np_l[l] qualify.  Shells
// r >= R_p are masked to zero.  Workgroups of the highest degrees (most column tiles) are
// launched first.
#include "matcha_launch.hpp"

namespace matcha {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kAsmThreads = 256;
constexpr int kAsmWaves = kAsmThreads / kWave;
constexpr int kAsmTilesPerWave = 4;  // default row tiles per wave and workgroup (a.tiles_per_wave)

__device__ inline void store_half_plane(float2 *Cp2, int l, int m, int n, float2 v)
{
    const int64_t row = wedge_row(l);
    if (m == 0 && n < 0) return;  // Hermitian mirror of (0, -n), not stored
    const int an = n >= 0 ? n : -n;
    if (an <= m) {
        const int64_t q = (int64_t)m * m + m + n;
        Cp2[2 * (row + q)] = v;
        if (an == m) Cp2[2 * (row + q) + 1] = v;  // diagonal pair: its own partner
    } else if (n > 0) {
        const int64_t q = (int64_t)n * n + n + m;  // pair (n, m), partner (m, n)
        Cp2[2 * (row + q) + 1] = v;
    } else {
        const int64_t q = (int64_t)an * an + an - m;  // pair (-n, -m), partner (m, n)
        Cp2[2 * (row + q) + 1] = v;
    }
}

// Columns of degree l padded to whole 16-column tiles.
__host__ __device__ inline int asm_cols(int l) { return 16 * ((2 * l + 1 + 15) / 16); }

// MS: K steps (of 2 shells) held in registers at a time; 16 for R <= 32, 32 for R <= 64, so that
// the A column of a row tile is loaded once; with more shells it is reloaded per column tile.
template <int MS>
__global__ void __launch_bounds__(kAsmThreads) k_assemble_f32(AsmArgs a)
{
    extern __shared__ __align__(16) float2 hs[];  // [Rmax][asm_cols(l)]: h_l(r) of the degree
    // the workgroup's degree: blocks of degree Lmax - d start at blk_lo[d]
    int d = 0;
    while ((int)blockIdx.x >= a.blk_lo[d + 1]) ++d;
    const int l = a.Lmax - d, blk = blockIdx.x - a.blk_lo[d];
    const int N = 2 * l + 1, NP = asm_cols(l), ntn = NP / 16;
    const int R = a.Rmax, sh = (a.Lh + 1) * (a.Lh + 1);
    float *ws = reinterpret_cast<float *>(hs + R * NP);  // [Rmax] shell weights
    for (int t = threadIdx.x; t < R * NP; t += kAsmThreads) {
        const int r = t / NP, j = t - (t / NP) * NP;
        hs[t] = j < N ? a.h[r * sh + l * l + j] : make_float2(0.f, 0.f);
    }
    for (int t = threadIdx.x; t < R; t += kAsmThreads) ws[t] = a.w[t];
    __syncthreads();
    const int rows = a.np_l[l] * (l + 1), RT = (rows + 15) / 16;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int col = lane % 16, kq = lane / 16;
    const int par = kq & 1, rsub = kq >> 1;  // K index 4 s + kq = 2 (2 s + rsub) + par
    const int nsteps = (R + 1) / 2;
    const int tpb = kAsmWaves * a.tiles_per_wave;
    for (int it = 0; it < a.tiles_per_wave; ++it) {
        const int rt = blk * tpb + it * kAsmWaves + wave;
        if (rt >= RT) break;
        // the lane's A row
        const int rho = min(16 * rt + col, rows - 1);
        const int pi = rho / (l + 1), m = rho - pi * (l + 1);
        const int p = a.by_L ? a.by_L[pi] : pi;
        const int Lp = a.Lp[p], Rp = a.Rp[p];
        const bool rok = 16 * rt + col < rows && l <= Lp;
        const int sf = (Lp + 1) * (Lp + 1);
        const float2 *fp = a.f + a.f_off[p] + (l <= Lp ? l * l + l + m : 0);  // in the particle's f
        // the lane's output rows: C of their particles and their m (rows past the batch or of
        // particles with L_p < l are not stored)
        float2 *cp[4];
        int mo[4];
        bool ook[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ro = 16 * rt + 4 * kq + v;
            const int pio = min(ro, rows - 1) / (l + 1);
            const int po = a.by_L ? a.by_L[pio] : pio;
            const int Lpo = a.Lp[po];
            mo[v] = ro - pio * (l + 1);
            ook[v] = (ro < rows) & (l <= Lpo);
            cp[v] = reinterpret_cast<float2 *>(a.C + a.C_off[po] / 2);
        }
        float av[MS];
        for (int tn = 0; tn < ntn; ++tn) {
            f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
            for (int s0 = 0; s0 < nsteps; s0 += MS) {
                // A: unconditional loads at clamped (valid, finite) addresses, masked by the
                // shell weight or 0 afterwards, so that all of a chunk's loads are in flight
                // together.  With one chunk the A column is loaded once per row tile.
                if (tn == 0 || nsteps > MS) {
#pragma unroll
                    for (int s = 0; s < MS; ++s) {
                        const int r = 2 * (s0 + s) + rsub;
                        const int rc = min(r, Rp - 1);
                        const float2 v = fp[rc * sf];
                        const float keep = ws[rc] * ((r < Rp && rok) ? 1.f : 0.f);
                        av[s] = (par ? v.y : v.x) * keep;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < MS; ++s) {
                    const float2 hv = hs[min(2 * (s0 + s) + rsub, R - 1) * NP + 16 * tn + col];
                    const float br = par ? hv.y : hv.x;
                    const float bi = par ? hv.x : -hv.y;
                    cr = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], br, cr, 0, 0, 0);
                    ci = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bi, ci, 0, 0, 0);
                }
            }
            const int j = 16 * tn + col;
            if (j < N) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (ook[v]) store_half_plane(cp[v], l, mo[v], j - l, make_float2(cr[v], ci[v]));
            }
        }
    }
}

// Counting sort of the particles by decreasing L_p in one workgroup: a histogram of L_p in LDS,
// the start of each degree's run, then every particle takes the next slot of its run (the
// order within a run is whatever the LDS atomics give; the assembly does not depend on it).
constexpr int kOrderThreads = 1024;
__global__ void __launch_bounds__(kOrderThreads) k_order_by_L(const int32_t *Lp, int P, int Lmax, int32_t *by_L)
{
    __shared__ int cnt[kMaxL + 1], start[kMaxL + 1];
    for (int l = threadIdx.x; l <= Lmax; l += kOrderThreads) cnt[l] = 0;
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += kOrderThreads) atomicAdd(&cnt[min(max(Lp[p], 0), Lmax)], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int l = Lmax; l >= 0; --l) {
            start[l] = s;
            s += cnt[l];
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += kOrderThreads) by_L[atomicAdd(&start[min(max(Lp[p], 0), Lmax)], 1)] = p;
}

hipError_t launch_order_by_L(const int32_t *Lp, int P, int Lmax, int32_t *by_L, hipStream_t s)
{
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_order_by_L, dim3(1), dim3(kOrderThreads), 0, s, Lp, P, Lmax, by_L);
    return hipGetLastError();
}

size_t assemble_smem_bytes(int Lmax, int Rmax)
{
    return sizeof(float2) * (size_t)Rmax * asm_cols(Lmax) + sizeof(float) * (size_t)Rmax;
}

hipError_t launch_assemble_f32(const AsmArgs &a0, int P, int Lmax, int Rmax, hipStream_t s)
{
    AsmArgs a = a0;
    a.P = P;
    a.Lmax = Lmax;
    a.Rmax = Rmax;
    if (a.tiles_per_wave < 1) a.tiles_per_wave = kAsmTilesPerWave;
    const int tpb = kAsmWaves * a.tiles_per_wave;
    int nb = 0;
    for (int d = 0; d <= Lmax; ++d) {
        const int l = Lmax - d;
        if (!a.by_L) a.np_l[l] = P;
        const int64_t rt = ((int64_t)a.np_l[l] * (l + 1) + 15) / 16;
        a.blk_lo[d] = nb;
        nb += (int)((rt + tpb - 1) / tpb);
    }
    a.blk_lo[Lmax + 1] = nb;
    if (nb == 0) return hipSuccess;
    const size_t smem = assemble_smem_bytes(Lmax, Rmax);
    if (Rmax > 32 && Rmax <= 64)
        hipLaunchKernelGGL(k_assemble_f32<32>, dim3(nb), dim3(kAsmThreads), smem, s, a);
    else
        hipLaunchKernelGGL(k_assemble_f32<16>, dim3(nb), dim3(kAsmThreads), smem, s, a);
    return hipGetLastError();
}

}  // namespace matcha
