// k_assemble_bf16.hip -- coefficient assembly (eq. sigmalmm) from BF16 coefficients on the
// matrix cores, FP32 accumulation, FP32 output in the wedge layout.
//
// As in the FP32 kernel, per degree the whole batch is one tall product: the rows (p, m),
// m <= l, of all particles stacked, times the template's (2l+1) columns.  In real form, with
// the shells interleaved (Re, Im) along K = 2R (padded to the 32-wide MFMA step),
//   Cr[row][j] = sum_k A[row][k] Br[k][j],  Ci[row][j] = sum_k A[row][k] Bi[k][j],
//   A[(p,m)][2r] = Re f_lm(r),  A[(p,m)][2r+1] = Im f_lm(r),
//   Br[2r][j] = w_r Re h_lj(r),  Br[2r+1][j] = w_r Im h_lj(r),
//   Bi[2r][j] = -w_r Im h_lj(r), Bi[2r+1][j] = w_r Re h_lj(r),
// with w_r h rounded once more to BF16.  v_mfma_f32_16x16x32_bf16: lane i holds A row i%16, B
// column i%16 and K elements 8(i/16) .. +7 of a 32-wide step (four shells, Re and Im); the
// result lane holds rows 4(i/16) .. +3 of column i%16.
//
// A workgroup takes one degree and a run of 16-row tiles of its stacked rows.  It builds B for
// the degree in LDS once ([column][K], K contiguous, rows padded by 16 bytes); each wave loads
// the A operands of a row tile straight from f (four 4-byte complex values per lane and step;
// every f value is read once), keeps them in registers and sweeps the column tiles.  When the
// band limits differ, the rows of degree l cover only the particles with L_p >= l, taken in
// the order of decreasing L_p; shells r >= R_p are masked to zero.  Workgroups of the highest
// degrees are launched first.
#include "matcha_launch.hpp"

namespace matcha {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kAsmBThreads = 256;
constexpr int kAsmBWaves = kAsmBThreads / kWave;
constexpr int kAsmBMaxSteps = 4;      // 32-wide K steps (16 shells each) held in registers at a time
constexpr int kAsmBTilesPerWave = 4;  // default row tiles per wave and workgroup (a.tiles_per_wave)

__device__ inline void store_half_plane_b(float2 *Cp2, int l, int m, int n, float2 v)
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

__host__ __device__ inline int asmb_cols(int l) { return 16 * ((2 * l + 1 + 15) / 16); }
__host__ __device__ inline int asmb_k(int Rmax) { return 32 * ((2 * Rmax + 31) / 32); }
__host__ __device__ inline int asmb_kstride(int Rmax) { return asmb_k(Rmax) + 8; }  // bf16 per LDS row

__global__ void __launch_bounds__(kAsmBThreads) k_assemble_bf16(AsmBArgs a)
{
    extern __shared__ __align__(16) __bf16 bs[];  // Br, Bi: [asmb_cols(l)][K + 8] each
    int d = 0;
    while ((int)blockIdx.x >= a.blk_lo[d + 1]) ++d;
    const int l = a.Lmax - d, blk = blockIdx.x - a.blk_lo[d];
    const int N = 2 * l + 1, NP = asmb_cols(l), ntn = NP / 16;
    const int R = a.Rmax, K = asmb_k(R), KS = asmb_kstride(R), sh = (a.Lh + 1) * (a.Lh + 1);
    __bf16 *Brs = bs, *Bis = bs + NP * KS;
    for (int t = threadIdx.x; t < NP * (K / 2); t += kAsmBThreads) {
        const int j = t / (K / 2), r = t - (t / (K / 2)) * (K / 2);
        float hr = 0.f, hi = 0.f;
        if (j < N && r < R) {
            const float wr = a.w[r];
            hr = wr * (float)a.h[2 * (r * sh + l * l + j)];
            hi = wr * (float)a.h[2 * (r * sh + l * l + j) + 1];
        }
        Brs[j * KS + 2 * r] = (__bf16)hr;
        Brs[j * KS + 2 * r + 1] = (__bf16)hi;
        Bis[j * KS + 2 * r] = (__bf16)(-hi);
        Bis[j * KS + 2 * r + 1] = (__bf16)hr;
    }
    __syncthreads();
    const int rows = a.np_l[l] * (l + 1), RT = (rows + 15) / 16;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int col = lane % 16, kg = lane / 16;  // K elements 8 kg .. +7: shells 4 kg .. +3 of a step
    const int nk = K / 32;
    const uint32_t *f32 = reinterpret_cast<const uint32_t *>(a.f);  // one complex BF16 value per word
    const int tpb = kAsmBWaves * a.tiles_per_wave;
    for (int it = 0; it < a.tiles_per_wave; ++it) {
        const int rt = blk * tpb + it * kAsmBWaves + wave;
        if (rt >= RT) break;
        const int rho = min(16 * rt + col, rows - 1);
        const int pi = rho / (l + 1), m = rho - pi * (l + 1);
        const int p = a.by_L ? a.by_L[pi] : pi;
        const int Lp = a.Lp[p], Rp = a.Rp[p];
        const bool rok = (16 * rt + col < rows) & (l <= Lp);
        const int sf = (Lp + 1) * (Lp + 1);
        const uint32_t *fp = f32 + a.f_off[p] + (l <= Lp ? l * l + l + m : 0);  // in the particle's f
        float2 *cp[4];
        int mo[4];
        bool ook[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ro = 16 * rt + 4 * kg + v;
            const int pio = min(ro, rows - 1) / (l + 1);
            const int po = a.by_L ? a.by_L[pio] : pio;
            const int Lpo = a.Lp[po];
            mo[v] = ro - pio * (l + 1);
            ook[v] = (ro < rows) & (l <= Lpo);
            cp[v] = reinterpret_cast<float2 *>(a.C + a.C_off[po] / 2);
        }
        bf16x8 av[kAsmBMaxSteps];
        for (int tn = 0; tn < ntn; ++tn) {
            f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < nk; k0 += kAsmBMaxSteps) {
                // A: unconditional loads at clamped addresses, zeroed by a bit mask, so that all
                // of a chunk's loads are in flight together; one chunk when R <= 64
                if (tn == 0 || nk > kAsmBMaxSteps) {
#pragma unroll
                    for (int s = 0; s < kAsmBMaxSteps; ++s) {
                        u32x4 u;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int r = 16 * (k0 + s) + 4 * kg + e;
                            const uint32_t x = fp[min(r, Rp - 1) * sf];
                            u[e] = x & (((r < Rp) & rok) ? 0xffffffffu : 0u);
                        }
                        av[s] = __builtin_bit_cast(bf16x8, u);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < kAsmBMaxSteps; ++s) {
                    if (k0 + s < nk) {
                        const int kk = 32 * (k0 + s) + 8 * kg;
                        const bf16x8 br = *reinterpret_cast<const bf16x8 *>(Brs + (16 * tn + col) * KS + kk);
                        const bf16x8 bi = *reinterpret_cast<const bf16x8 *>(Bis + (16 * tn + col) * KS + kk);
                        cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[s], br, cr, 0, 0, 0);
                        ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[s], bi, ci, 0, 0, 0);
                    }
                }
            }
            const int j = 16 * tn + col;
            if (j < N) {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (ook[v]) store_half_plane_b(cp[v], l, mo[v], j - l, make_float2(cr[v], ci[v]));
            }
        }
    }
}

size_t assemble_bf16_smem_bytes(int Lmax, int Rmax)
{
    return 2 * sizeof(__bf16) * (size_t)asmb_cols(Lmax) * asmb_kstride(Rmax);
}

hipError_t launch_assemble_bf16(const AsmBArgs &a0, int P, int Lmax, int Rmax, hipStream_t s)
{
    AsmBArgs a = a0;
    a.P = P;
    a.Lmax = Lmax;
    a.Rmax = Rmax;
    if (a.tiles_per_wave < 1) a.tiles_per_wave = kAsmBTilesPerWave;
    const int tpb = kAsmBWaves * a.tiles_per_wave;
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
    hipLaunchKernelGGL(k_assemble_bf16, dim3(nb), dim3(kAsmBThreads), assemble_bf16_smem_bytes(Lmax, Rmax), s, a);
    return hipGetLastError();
}

}  // namespace matcha
