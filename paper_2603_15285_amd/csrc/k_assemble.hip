// k_assemble.hip -- coefficient assembly, eq. sigmalmm (Sec. 2.1, App. A.5):
//   C^l_mn = sum_{r < R_p} w_r f_lm(r) conj(h_ln(r)),  l <= L_p,
// for the half plane m >= 0 of each degree (Hermitian-symmetric inputs), written into the
// wedge layout: the value at (m, n) lands in slot 0 of the wedge pair (m, n) when |n| <= m,
// otherwise in slot 1 (the partner slot) of the pair (n, m) (n > 0) or (-n, -m) (n < 0).
//
// A workgroup takes one particle and a chunk of degrees.  Per degree it stages the m >= 0 rows
// of f and the rows w_r conj(h) in LDS, then each thread forms a 2 (m) x 4 (n) block of the
// (l+1) x (2l+1) product over the shells, so LDS traffic is 1.5 bytes per FMA.
#include "matcha_launch.hpp"

namespace matcha {

constexpr int kAsmThreads = 256;

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
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int p = blockIdx.x / a.n_chunks, chunk = blockIdx.x % a.n_chunks;
    const int L = a.Lp[p], R = a.Rp[p];
    const int l_lo = a.chunk_lo[chunk], l_hi = min(a.chunk_lo[chunk + 1] - 1, L);
    const int64_t sf = (int64_t)(L + 1) * (L + 1), sh = (int64_t)(a.Lh + 1) * (a.Lh + 1);
    const float2 *fp = a.f + a.f_off[p];
    float2 *Cp2 = reinterpret_cast<float2 *>(a.C + a.C_off[p] / 2);
    float2 *Fs = reinterpret_cast<float2 *>(smem_raw);  // [R][l+1]     f_lm(r), m >= 0
    for (int l = l_lo; l <= l_hi; ++l) {
        const int nf = l + 1, nh = 2 * l + 1;
        float2 *Gs = Fs + R * nf;                         // [R][2l+1]   w_r conj(h_ln(r))
        for (int t = threadIdx.x; t < R * nf; t += kAsmThreads) {
            const int r = t / nf, m = t - (t / nf) * nf;
            Fs[t] = fp[r * sf + l * l + l + m];
        }
        for (int t = threadIdx.x; t < R * nh; t += kAsmThreads) {
            const int r = t / nh, j = t - (t / nh) * nh;
            const float2 hv = a.h[r * sh + l * l + j];
            const float wr = a.w[r];
            Gs[t] = make_float2(wr * hv.x, -wr * hv.y);
        }
        __syncthreads();
        const int nmb = (nf + 1) / 2, nnb = (nh + 3) / 4;
        for (int blk = threadIdx.x; blk < nmb * nnb; blk += kAsmThreads) {
            const int mb = blk / nnb, nb = blk - (blk / nnb) * nnb;
            const int m0 = 2 * mb, j0 = 4 * nb;
            const int m1 = min(m0 + 1, l), ja = min(j0 + 1, nh - 1), jb = min(j0 + 2, nh - 1), jc = min(j0 + 3, nh - 1);
            float cr[2][4], ci[2][4];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) cr[x][y] = ci[x][y] = 0.f;
            for (int r = 0; r < R; ++r) {
                const float2 f0 = Fs[r * nf + m0], f1 = Fs[r * nf + m1];
                const float2 *g = Gs + r * nh;
                const float2 gv[4] = {g[j0], g[ja], g[jb], g[jc]};
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    cr[0][y] = fmaf(f0.x, gv[y].x, fmaf(-f0.y, gv[y].y, cr[0][y]));
                    ci[0][y] = fmaf(f0.x, gv[y].y, fmaf(f0.y, gv[y].x, ci[0][y]));
                    cr[1][y] = fmaf(f1.x, gv[y].x, fmaf(-f1.y, gv[y].y, cr[1][y]));
                    ci[1][y] = fmaf(f1.x, gv[y].y, fmaf(f1.y, gv[y].x, ci[1][y]));
                }
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const int m = m0 + x, j = j0 + y;
                    if (m <= l && j < nh) store_half_plane(Cp2, l, m, j - l, make_float2(cr[x][y], ci[x][y]));
                }
        }
        __syncthreads();
    }
}

size_t assemble_smem_bytes(int Lmax, int Rmax)
{
    return sizeof(float2) * (size_t)Rmax * (size_t)(3 * Lmax + 2);
}

hipError_t launch_assemble_f32(const AsmArgs &a, int P, int Lmax, int Rmax, hipStream_t s)
{
    hipLaunchKernelGGL(k_assemble_f32, dim3(P * a.n_chunks), dim3(kAsmThreads), assemble_smem_bytes(Lmax, Rmax), s, a);
    return hipGetLastError();
}

}  // namespace matcha
