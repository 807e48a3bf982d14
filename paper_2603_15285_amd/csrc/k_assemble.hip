// k_assemble.hip -- coefficient assembly, eq. sigmalmm (Sec. 2.1, App. A.5):
//   C^l_mn = sum_{r < R_p} w_r f_lm(r) conj(h_ln(r)),  l <= L_p,
// written in the wedge layout (per l, per wedge pair q: the pair's value and its partner's).
// Only the m >= 0 half of f is read (Hermitian-symmetric inputs); the template rows are
// pre-multiplied by w_r and conjugated while being staged in LDS.
#include "matcha_launch.hpp"

namespace matcha {

constexpr int kAsmThreads = 256;


__global__ void __launch_bounds__(kAsmThreads) k_assemble_f32(AsmArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int p = blockIdx.x;
    const int L = a.Lp[p], R = a.Rp[p];
    const int64_t sf = (int64_t)(L + 1) * (L + 1), sh = (int64_t)(a.Lh + 1) * (a.Lh + 1);
    const float2 *fp = a.f + a.f_off[p];
    float4 *Cp = a.C + a.C_off[p] / 2;
    float2 *Fs = reinterpret_cast<float2 *>(smem_raw);  // [R][l+1]     f_lm(r), m >= 0
    for (int l = 0; l <= L; ++l) {
        const int nf = l + 1, nh = 2 * l + 1;
        float2 *Hs = Fs + R * nf;                         // [R][2l+1]   w_r conj(h_ln(r))
        for (int t = threadIdx.x; t < R * nf; t += kAsmThreads) {
            const int r = t / nf, m = t % nf;
            Fs[t] = fp[r * sf + l * l + l + m];
        }
        for (int t = threadIdx.x; t < R * nh; t += kAsmThreads) {
            const int r = t / nh, j = t % nh;
            const float2 hv = a.h[r * sh + l * l + j];
            const float wr = a.w[r];
            Hs[t] = make_float2(wr * hv.x, -wr * hv.y);
        }
        __syncthreads();
        const int np = (l + 1) * (l + 1);
        for (int q = threadIdx.x; q < np; q += kAsmThreads) {
            const int m = isqrt_dev(q), n = q - m * m - m;
            const int m2 = n >= 0 ? n : -n, n2 = n >= 0 ? m : -m;
            float c0r = 0.f, c0i = 0.f, c1r = 0.f, c1i = 0.f;
            for (int r = 0; r < R; ++r) {
                const float2 x = Fs[r * nf + m], y = Hs[r * nh + n + l];
                const float2 u = Fs[r * nf + m2], v = Hs[r * nh + n2 + l];
                c0r = fmaf(x.x, y.x, fmaf(-x.y, y.y, c0r));
                c0i = fmaf(x.x, y.y, fmaf(x.y, y.x, c0i));
                c1r = fmaf(u.x, v.x, fmaf(-u.y, v.y, c1r));
                c1i = fmaf(u.x, v.y, fmaf(u.y, v.x, c1i));
            }
            Cp[wedge_row(l) + q] = make_float4(c0r, c0i, c1r, c1i);
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
    hipLaunchKernelGGL(k_assemble_f32, dim3(P), dim3(kAsmThreads), assemble_smem_bytes(Lmax, Rmax), s, a);
    return hipGetLastError();
}

}  // namespace matcha
