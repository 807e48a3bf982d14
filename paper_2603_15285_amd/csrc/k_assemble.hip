// k_assemble.hip -- coefficient assembly, eq. sigmalmm (Sec. 2.1, App. A.5):
//   C^l_mn = sum_{r < R_p} w_r f_lm(r) conj(h_ln(r)),  l <= L_p,
// for the half plane m >= 0 of each degree (Hermitian-symmetric inputs), written into the
// wedge layout: the value at (m, n) lands in slot 0 of the wedge pair (m, n) when |n| <= m,
// otherwise in slot 1 (the partner slot) of the pair (n, m) (n > 0) or (-n, -m) (n < 0).
//
// Per degree the half plane is the complex product (l+1) x R times R x (2l+1).  In real form,
// with the shells interleaved (Re, Im) along K = 2R,
//   Cr[m][j] = sum_k A[m][k] Br[k][j],  Ci[m][j] = sum_k A[m][k] Bi[k][j],
//   A[m][2r] = Re f,  A[m][2r+1] = Im f,
//   Br[2r][j] = w_r Re h,  Br[2r+1][j] = w_r Im h,  Bi[2r][j] = -w_r Im h,  Bi[2r+1][j] = w_r Re h,
// it runs on the matrix cores in FP32 (v_mfma_f32_16x16x4_f32: lane i supplies A[i%16][i/16]
// and B[i/16][i%16] of a 16 x 4 x 16 step and holds D rows 4(i/16) .. +3 of column i%16).
// Operands come straight from memory: a wave owns a 16-row tile of one degree, keeps its A
// column (one float per K step) in registers, and sweeps the 16-column tiles of B, whose
// template rows are shared by every particle and stay in L2.  The waves of a workgroup take
// the (degree, row tile) units of one particle's degree chunk in turn, with no barrier.
#include "matcha_launch.hpp"

namespace matcha {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kAsmThreads = 256;
constexpr int kAsmMaxSteps = 16;  // K steps (of 2 shells) held in registers at a time

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

__global__ void __launch_bounds__(kAsmThreads) k_assemble_f32(AsmArgs a)
{
    const int p = blockIdx.x / a.n_chunks, chunk = blockIdx.x % a.n_chunks;
    const int L = a.Lp[p], R = a.Rp[p];
    const int l_lo = a.chunk_lo[chunk], l_hi = min(a.chunk_lo[chunk + 1] - 1, L);
    // element offsets within one particle's f and within h fit 32 bits (the library bounds
    // R_h (L_h+1)^2 below 2^31), so loads take a uniform base and a 32-bit per-lane offset
    const int sf = (L + 1) * (L + 1), sh = (a.Lh + 1) * (a.Lh + 1);
    const float2 *fp = a.f + a.f_off[p];
    float2 *Cp2 = reinterpret_cast<float2 *>(a.C + a.C_off[p] / 2);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nwaves = kAsmThreads / kWave;
    const int col = lane % 16, kq = lane / 16;
    const int par = kq & 1, rsub = kq >> 1;  // K index 4 s + kq = 2 (2 s + rsub) + par
    const int nsteps = (R + 1) / 2;
    int u = 0;
    // heaviest degrees first, so the units spread evenly over the waves
    for (int l = l_hi; l >= l_lo; --l) {
        const int ntm = (l + 16) / 16, ntn = (2 * l + 16) / 16;
        const int lrow = l * l;
        for (int tm = 0; tm < ntm; ++tm, ++u) {
            if (u % nwaves != wave) continue;
            const int m = 16 * tm + col;
            const bool mok = m <= l;
            const int mc = min(m, l);
            float av[kAsmMaxSteps], wv[kAsmMaxSteps];
            for (int tn = 0; tn < ntn; ++tn) {
                const int j = 16 * tn + col;
                const bool jok = j < 2 * l + 1;
                const int jc = min(j, 2 * l);
                f32x4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
                for (int s0 = 0; s0 < nsteps; s0 += kAsmMaxSteps) {
                    // Loads are unconditional at clamped (valid, finite) addresses and masked by a
                    // 0/1 factor afterwards, so that all of a chunk's loads are in flight together.
                    // With one chunk (R <= 32) the A column and the weights are loaded once per
                    // tile row.
                    if (tn == 0 || nsteps > kAsmMaxSteps) {
#pragma unroll
                        for (int s = 0; s < kAsmMaxSteps; ++s) {
                            const int r = 2 * (s0 + s) + rsub;
                            const int rc = min(r, R - 1);
                            const float2 v = fp[rc * sf + lrow + l + mc];
                            const float keep = (r < R && mok) ? 1.f : 0.f;
                            av[s] = (par ? v.y : v.x) * keep;
                            wv[s] = a.w[rc] * (r < R ? 1.f : 0.f);
                        }
                    }
                    float2 hv[kAsmMaxSteps];
#pragma unroll
                    for (int s = 0; s < kAsmMaxSteps; ++s)
                        hv[s] = a.h[min(2 * (s0 + s) + rsub, R - 1) * sh + lrow + jc];
                    __builtin_amdgcn_sched_barrier(0);
                    const float jmask = jok ? 1.f : 0.f;
#pragma unroll
                    for (int s = 0; s < kAsmMaxSteps; ++s) {
                        const float wr = wv[s] * jmask;
                        const float br = wr * (par ? hv[s].y : hv[s].x);
                        const float bi = par ? wr * hv[s].x : -(wr * hv[s].y);
                        cr = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], br, cr, 0, 0, 0);
                        ci = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bi, ci, 0, 0, 0);
                    }
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int mo = 16 * tm + 4 * kq + v;
                    if (mo <= l && jok) store_half_plane(Cp2, l, mo, j - l, make_float2(cr[v], ci[v]));
                }
            }
        }
    }
}

size_t assemble_smem_bytes(int, int) { return 0; }

hipError_t launch_assemble_f32(const AsmArgs &a, int P, int, int, hipStream_t s)
{
    hipLaunchKernelGGL(k_assemble_f32, dim3(P * a.n_chunks), dim3(kAsmThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace matcha
