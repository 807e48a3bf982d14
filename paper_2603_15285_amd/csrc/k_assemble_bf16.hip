// k_assemble_bf16.hip -- coefficient assembly (eq. sigmalmm) from BF16 coefficients on the
// matrix cores, FP32 accumulation, FP32 output in the wedge layout.
//
// Per degree l the half plane of C^l is a complex product (l+1) x R times R x (2l+1).  As a real
// product with the shells interleaved (Re, Im) along K = 2R:
//   Cr[m][n] = sum_k A[m][k] Br[k][n],  Ci[m][n] = sum_k A[m][k] Bi[k][n],
//   A[m][2r] = Re f_lm(r),  A[m][2r+1] = Im f_lm(r),
//   Br[2r][n] = w_r Re h_ln(r),  Br[2r+1][n] = w_r Im h_ln(r),
//   Bi[2r][n] = -w_r Im h_ln(r), Bi[2r+1][n] = w_r Re h_ln(r).
// A and B are staged in LDS with K contiguous (16 bytes per lane and fragment), and each wave
// computes 16 x 16 output tiles with v_mfma_f32_16x16x32_bf16 (lane i holds A row i%16,
// B column i%16, and K elements 8*(i/16) .. +7; the result lane holds rows 4*(i/16) .. +3 of
// column i%16).
#include "matcha_launch.hpp"

namespace matcha {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kAsmBThreads = 256;

__device__ inline void store_half_plane_b(float2 *Cp2, int l, int m, int n, float2 v)
{
    const int64_t row = wedge_row(l);
    if (m == 0 && n < 0) return;
    const int an = n >= 0 ? n : -n;
    if (an <= m) {
        const int64_t q = (int64_t)m * m + m + n;
        Cp2[2 * (row + q)] = v;
        if (an == m) Cp2[2 * (row + q) + 1] = v;
    } else if (n > 0) {
        const int64_t q = (int64_t)n * n + n + m;
        Cp2[2 * (row + q) + 1] = v;
    } else {
        const int64_t q = (int64_t)an * an + an - m;
        Cp2[2 * (row + q) + 1] = v;
    }
}

__global__ void __launch_bounds__(kAsmBThreads) k_assemble_bf16(AsmBArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int p = blockIdx.x / a.n_chunks, chunk = blockIdx.x % a.n_chunks;
    const int L = a.Lp[p], R = a.Rp[p];
    const int l_lo = a.chunk_lo[chunk], l_hi = min(a.chunk_lo[chunk + 1] - 1, L);
    const int K = 2 * ((R + 15) / 16) * 16;  // K padded to the 32-wide MFMA step
    const int64_t sf = (int64_t)(L + 1) * (L + 1), sh = (int64_t)(a.Lh + 1) * (a.Lh + 1);
    const __bf16 *fp = a.f + 2 * a.f_off[p];
    float2 *Cp2 = reinterpret_cast<float2 *>(a.C + a.C_off[p] / 2);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int l = l_lo; l <= l_hi; ++l) {
        const int M = l + 1, N = 2 * l + 1;
        const int Mp = (M + 15) / 16 * 16, Np = (N + 15) / 16 * 16;
        __bf16 *As = reinterpret_cast<__bf16 *>(smem_raw);  // [Mp][K]
        __bf16 *Brs = As + Mp * K;                            // [Np][K]
        __bf16 *Bis = Brs + Np * K;                           // [Np][K]
        const __bf16 zero = (__bf16)0.f;
        for (int t = threadIdx.x; t < Mp * (K / 2); t += kAsmBThreads) {
            const int m = t / (K / 2), r = t - (t / (K / 2)) * (K / 2);
            __bf16 re = zero, im = zero;
            if (m < M && r < R) {
                re = fp[2 * (r * sf + l * l + l + m)];
                im = fp[2 * (r * sf + l * l + l + m) + 1];
            }
            As[m * K + 2 * r] = re;
            As[m * K + 2 * r + 1] = im;
        }
        for (int t = threadIdx.x; t < Np * (K / 2); t += kAsmBThreads) {
            const int j = t / (K / 2), r = t - (t / (K / 2)) * (K / 2);
            float hr = 0.f, hi = 0.f;
            if (j < N && r < R) {
                const float wr = a.w[r];
                hr = wr * (float)a.h[2 * (r * sh + l * l + j)];
                hi = wr * (float)a.h[2 * (r * sh + l * l + j) + 1];
            }
            Brs[j * K + 2 * r] = (__bf16)hr;
            Brs[j * K + 2 * r + 1] = (__bf16)hi;
            Bis[j * K + 2 * r] = (__bf16)(-hi);
            Bis[j * K + 2 * r + 1] = (__bf16)hr;
        }
        __syncthreads();
        const int tm = Mp / 16, tn = Np / 16;
        for (int tile = wave; tile < tm * tn; tile += kAsmBThreads / kWave) {
            const int im_ = tile / tn, in_ = tile - (tile / tn) * tn;
            f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
            const int arow = 16 * im_ + (lane % 16), bcol = 16 * in_ + (lane % 16);
            for (int k0 = 0; k0 < K; k0 += 32) {
                const int kk = k0 + 8 * (lane / 16);
                const bf16x8 av = *reinterpret_cast<const bf16x8 *>(As + arow * K + kk);
                const bf16x8 br = *reinterpret_cast<const bf16x8 *>(Brs + bcol * K + kk);
                const bf16x8 bi = *reinterpret_cast<const bf16x8 *>(Bis + bcol * K + kk);
                cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, br, cr, 0, 0, 0);
                ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bi, ci, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = 16 * im_ + 4 * (lane / 16) + v, j = bcol;
                if (m < M && j < N) store_half_plane_b(Cp2, l, m, j - l, make_float2(cr[v], ci[v]));
            }
        }
        __syncthreads();
    }
}

size_t assemble_bf16_smem_bytes(int Lmax, int Rmax)
{
    const size_t K = 2 * (size_t)((Rmax + 15) / 16) * 16;
    const size_t Mp = (size_t)((Lmax + 1 + 15) / 16) * 16, Np = (size_t)((2 * Lmax + 1 + 15) / 16) * 16;
    return 2 * K * (Mp + 2 * Np);
}

hipError_t launch_assemble_bf16(const AsmBArgs &a, int P, int Lmax, int Rmax, hipStream_t s)
{
    hipLaunchKernelGGL(k_assemble_bf16, dim3(P * a.n_chunks), dim3(kAsmBThreads), assemble_bf16_smem_bytes(Lmax, Rmax),
                       s, a);
    return hipGetLastError();
}

}  // namespace matcha
