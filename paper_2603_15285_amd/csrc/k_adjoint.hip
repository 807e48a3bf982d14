// k_adjoint.hip -- adjoint of sum_p g_p C_{L_p}(R_p*) with the rotations held fixed.
//
// With C_L(g) = Re sum C^l_mn conj(D^l_mn(g)) and C^l_mn = sum_r w_r f_lm(r) conj(h_ln(r)), the
// gradients packed as d/dRe + i d/dIm of the full complex arrays are
//   grad_f_p[r][l, m] = g_p w_r sum_n D^l_mn(R_p*) h_ln(r)             (the rotated template)
//   grad_h[r][l, n]   = sum_p g_p w_r sum_m f_p,lm(r) conj(D^l_mn(R_p*)) (back-rotated particles)
// with D^l_mn = e^{-i m a} d^l_mn(b) e^{-i n c} (eq. wigner-D).
//
// One workgroup per particle walks the degrees l = 0..L_p.  The wedge recurrences (one per
// pair, normalised as in the march) advance one degree at a time in registers and write the
// full d^l matrix into LDS through d_mn = (-1)^{m-n} d_nm = d_{-n,-m}; the d tables are
// recomputed here, never stored.  The products with d run over shell chunks staged in LDS.
// The particle's grad_h term goes to a workspace laid out like f; a second kernel sums the
// particles in index order (no floating-point atomics, so the result is deterministic).
#include "matcha_launch.hpp"

namespace matcha {

constexpr int kAdjThreads = 256;
constexpr int kAdjPairsPerThread = (65 * 65 + kAdjThreads - 1) / kAdjThreads;  // L <= 64
constexpr int kAdjShellChunk = 16;

__global__ void __launch_bounds__(kAdjThreads) k_grad_particle(GradArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int p = blockIdx.x;
    const int L = a.Lp[p], R = a.Rp[p];
    const int Lmax = a.L_max;
    float *dm = reinterpret_cast<float *>(smem_raw);                    // [(2Lmax+1)^2]
    float2 *ea = reinterpret_cast<float2 *>(dm + (2 * Lmax + 1) * (2 * Lmax + 1));  // [Lmax+1] e^{i k a}
    float2 *eg = ea + (Lmax + 1);                                        // [Lmax+1] e^{i k c}
    float2 *Hs = eg + (Lmax + 1);                                        // [chunk][2l+1]
    float2 *Fs = Hs + kAdjShellChunk * (2 * Lmax + 1);                   // [chunk][2l+1]

    const float4 th = a.best[p];
    const float gp = a.g[p];
    for (int k = threadIdx.x; k <= L; k += kAdjThreads) {
        const double ta = fmod((double)k * th.x, kTwoPi), tc = fmod((double)k * th.z, kTwoPi);
        float s, c;
        sincosf((float)ta, &s, &c);
        ea[k] = make_float2(c, s);
        sincosf((float)tc, &s, &c);
        eg[k] = make_float2(c, s);
    }
    const BetaConst bc = beta_const((double)th.y);
    float D[kAdjPairsPerThread], Dm[kAdjPairsPerThread];
#pragma unroll
    for (int k = 0; k < kAdjPairsPerThread; ++k) D[k] = Dm[k] = 0.f;

    const int64_t sf = (int64_t)(L + 1) * (L + 1), sh = (int64_t)(a.Lh + 1) * (a.Lh + 1);
    const float2 *fp = a.f + a.f_off[p];
    float2 *gf = a.grad_f ? a.grad_f + a.f_off[p] : nullptr;
    float2 *gw = a.ws ? a.ws + a.f_off[p] : nullptr;

    for (int l = 0; l <= L; ++l) {
        const int w = 2 * l + 1;
        const int np = (l + 1) * (l + 1);
        const int64_t row = wedge_row(l);
        // d^l for every wedge pair, then the four symmetric entries of the full matrix
#pragma unroll
        for (int k = 0; k < kAdjPairsPerThread; ++k) {
            const int q = threadIdx.x + k * kAdjThreads;
            if (q < np) {
                const PairInfo pi = a.pinfo[q];
                const float4 tb = a.tab[row + q];
                float dn;
                if (pi.m == l) {
                    float s1, s2;
                    edge_seed(pi.m, pi.n, pi.lbh2, bc, dn, s1, s2);
                } else {
                    dn = fmaf(fmaf(tb.x, bc.cb, -tb.y), D[k], -Dm[k]);
                }
                Dm[k] = D[k];
                D[k] = dn;
                const float P = q == 0 ? 2.f * tb.z : tb.z;  // the table holds w P_l, w = 1/2 at (0, 0)
                const float d = P * dn;
                const float ds = ((pi.m - pi.n) & 1) ? -d : d;
                const int m = pi.m, n = pi.n;
                dm[(m + l) * w + (n + l)] = d;
                dm[(n + l) * w + (m + l)] = ds;
                dm[(-n + l) * w + (-m + l)] = d;
                dm[(-m + l) * w + (-n + l)] = ds;
            }
        }
        for (int r0 = 0; r0 < R; r0 += kAdjShellChunk) {
            const int rc = min(kAdjShellChunk, R - r0);
            // Hs[r][n] = e^{-i n c} h_ln(r),  Fs[r][m] = e^{i m a} f_lm(r)
            for (int t = threadIdx.x; t < rc * w; t += kAdjThreads) {
                const int r = t / w, j = t - (t / w) * w, k = j - l;
                const float2 hv = a.h[(r0 + r) * sh + l * l + j];
                const float2 fv = fp[(r0 + r) * sf + l * l + j];
                const float2 e1 = k >= 0 ? cconj(eg[k]) : eg[-k];
                const float2 e2 = k >= 0 ? ea[k] : cconj(ea[-k]);
                Hs[t] = cmul(e1, hv);
                Fs[t] = cmul(e2, fv);
            }
            __syncthreads();
            // grad_f: 4 rows m per task;  grad_h term: 4 columns n per task
            const int nb = (w + 3) / 4;
            for (int task = threadIdx.x; task < 2 * rc * nb; task += kAdjThreads) {
                const bool forf = task < rc * nb;
                const int tt = forf ? task : task - rc * nb;
                const int r = tt / nb, b0 = 4 * (tt - (tt / nb) * nb);
                float2 acc[4] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
                if (forf) {
                    for (int j = 0; j < w; ++j) {
                        const float2 u = Hs[r * w + j];
#pragma unroll
                        for (int x = 0; x < 4; ++x) {
                            const float d = dm[min(b0 + x, w - 1) * w + j];
                            acc[x].x = fmaf(d, u.x, acc[x].x);
                            acc[x].y = fmaf(d, u.y, acc[x].y);
                        }
                    }
                } else {
                    for (int i = 0; i < w; ++i) {
                        const float2 u = Fs[r * w + i];
                        const float *drow = dm + i * w;
#pragma unroll
                        for (int x = 0; x < 4; ++x) {
                            const float d = drow[min(b0 + x, w - 1)];
                            acc[x].x = fmaf(d, u.x, acc[x].x);
                            acc[x].y = fmaf(d, u.y, acc[x].y);
                        }
                    }
                }
                const float sc = gp * a.w[r0 + r];
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int j = b0 + x;
                    if (j >= w) break;
                    const int k = j - l;
                    const int64_t idx = (int64_t)(r0 + r) * sf + l * l + j;
                    if (forf) {
                        if (gf) {
                            const float2 e = k >= 0 ? cconj(ea[k]) : ea[-k];  // e^{-i m a}
                            const float2 v = cmul(e, acc[x]);
                            gf[idx] = make_float2(sc * v.x, sc * v.y);
                        }
                    } else if (gw) {
                        const float2 e = k >= 0 ? eg[k] : cconj(eg[-k]);  // e^{i n c}
                        const float2 v = cmul(e, acc[x]);
                        gw[idx] = make_float2(sc * v.x, sc * v.y);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// grad_h[r][lm] = sum over particles in index order of their terms (zero outside a particle's
// shells and degrees).
__global__ void __launch_bounds__(256) k_grad_reduce(GradArgs a)
{
    const int64_t nl = (int64_t)(a.Lh + 1) * (a.Lh + 1);
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nl * a.Rh) return;
    const int r = (int)(e / nl);
    const int lm = (int)(e - (int64_t)r * nl);
    const int l = (int)sqrtf((float)lm + 0.5f);
    float2 s = make_float2(0.f, 0.f);
    for (int p = 0; p < a.P; ++p) {
        const int Lp = a.Lp[p], Rp = a.Rp[p];
        if (r < Rp && l <= Lp) {
            const float2 v = a.ws[a.f_off[p] + (int64_t)r * (Lp + 1) * (Lp + 1) + lm];
            s.x += v.x;
            s.y += v.y;
        }
    }
    a.grad_h[e] = s;
}

size_t grad_smem_bytes(int Lmax)
{
    const size_t w = 2 * (size_t)Lmax + 1;
    return sizeof(float) * w * w + sizeof(float2) * 2 * (Lmax + 1) + sizeof(float2) * 2 * kAdjShellChunk * w;
}

hipError_t launch_grad(const GradArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_particle, dim3(a.P), dim3(kAdjThreads), grad_smem_bytes(a.L_max), s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.grad_h) return e;
    const int64_t n = (int64_t)(a.Lh + 1) * (a.Lh + 1) * a.Rh;
    hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace matcha
