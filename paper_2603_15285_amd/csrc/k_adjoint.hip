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
// recomputed here, never stored.  The products with d run over shell chunks staged in LDS, on
// the matrix cores: per degree and chunk of 16 shells, grad_f is the real product d . Hs^T and
// the grad_h term d^T . Fs^T (v_mfma_f32_16x16x4_f32; lane i supplies A[i%16][i/16] and
// B[i/16][i%16] of a 16 x 4 x 16 step and holds D rows 4(i/16) .. +3 of column i%16), with the
// real and imaginary parts of the staged arrays as two B operands.
// The particle's grad_h term goes to a workspace at packed offsets (computed from L_p and R_p by a
// first kernel, independent of the caller's f_offset); a last kernel sums the particles in index
// order (no floating-point atomics, so the result is deterministic).
#include <algorithm>

#include "matcha_launch.hpp"

namespace matcha {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kAdjThreads = 256;
constexpr int kAdjPairsPerThread = (65 * 65 + kAdjThreads - 1) / kAdjThreads;  // L <= 64
constexpr int kAdjShellChunk = 16;

// 4 waves per SIMD (at most 128 registers): with one workgroup per particle, 4 workgroups per CU
// take 1024 particles in one round.
__global__ void __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) k_grad_particle(GradArgs a)
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
    float2 *gw = a.ws ? a.ws + a.ws_off[p] : nullptr;

    for (int l = 0; l <= L; ++l) {
        const int w = 2 * l + 1;
        const int np = (l + 1) * (l + 1);
        const int64_t row = wedge_row(l);
        // d^l for every wedge pair, then the four symmetric entries of the full matrix
#pragma unroll
        for (int k = 0; k < kAdjPairsPerThread; ++k) {
            if (k * kAdjThreads >= np) break;
            const int q = threadIdx.x + k * kAdjThreads, qc = min(q, np - 1);
            // loads at clamped addresses outside the branch, so that they need not wait in turn
            const PairInfo pi = a.pinfo[qc];
            const float4 tb = a.tab[row + qc];
            if (q < np) {
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
            // Output tiles of 16 rows (m for grad_f, n for the grad_h term) x 16 shells, one per wave
            // at a time.  Operands outside the degree (index >= w) or the chunk (shell >= rc) are
            // read at clamped addresses and zeroed.
            const int MT = (w + 15) / 16, KS = (w + 3) / 4;
            const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
            const int col = lane % 16, kq = lane / 16;
            for (int task = wave; task < 2 * MT; task += kAdjThreads / kWave) {
                const bool forf = task < MT;
                const int t0 = 16 * (forf ? task : task - MT);
                const int ar = min(t0 + col, w - 1);
                const bool aok = t0 + col < w, sok = col < rc;
                const float2 *src = (forf ? Hs : Fs) + min(col, rc - 1) * w;
                f32x4 gre = {0.f, 0.f, 0.f, 0.f}, gim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
                for (int ks = 0; ks < KS; ++ks) {
                    const int k = 4 * ks + kq, kc = min(k, w - 1);
                    const bool kok = k < w;
                    // grad_f: A[m][n] = d_mn, B[n][r] = Hs[r][n];  grad_h: A[n][m] = d_mn, B[m][r] = Fs[r][m]
                    const float av = (aok && kok) ? (forf ? dm[ar * w + kc] : dm[kc * w + ar]) : 0.f;
                    const float2 bv = src[kc];
                    const float bm = (sok && kok) ? 1.f : 0.f;
                    gre = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv.x * bm, gre, 0, 0, 0);
                    gim = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv.y * bm, gim, 0, 0, 0);
                }
                if (sok) {
                    const float sc = gp * a.w[r0 + col];
                    float2 *dst = forf ? gf : gw;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int j = t0 + 4 * kq + v;
                        if (j >= w || !dst) continue;
                        const int k = j - l;
                        // grad_f: e^{-i m a};  grad_h term: e^{i n c}
                        const float2 e = forf ? (k >= 0 ? cconj(ea[k]) : ea[-k]) : (k >= 0 ? eg[k] : cconj(eg[-k]));
                        const float2 val = cmul(e, make_float2(gre[v], gim[v]));
                        dst[(int64_t)(r0 + col) * sf + l * l + j] = make_float2(sc * val.x, sc * val.y);
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ws_off[p] = sum_{q < p} R_q (L_q+1)^2: the packed offsets of the particles' template terms, in one
// workgroup (each thread sums a run of particles, the runs' totals are scanned in LDS, then each
// thread writes its run's offsets).
constexpr int kScanThreads = 1024;
__global__ void __launch_bounds__(kScanThreads) k_term_offsets(const int32_t *Lp, const int32_t *Rp, int P, int64_t *off)
{
    __shared__ int64_t part[kScanThreads];
    const int t = threadIdx.x;
    const int per = (P + kScanThreads - 1) / kScanThreads;
    const int b = min(t * per, P), e = min(b + per, P);
    int64_t s = 0;
    for (int p = b; p < e; ++p) s += (int64_t)Rp[p] * (Lp[p] + 1) * (Lp[p] + 1);
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t o = t > 0 ? part[t - 1] : 0;
    for (int p = b; p < e; ++p) {
        off[p] = o;
        o += (int64_t)Rp[p] * (Lp[p] + 1) * (Lp[p] + 1);
    }
}

// Partial template gradients: segment sg (blockIdx.y) sums the terms of particles
// [sg * seg_len, (sg + 1) * seg_len) in index order into part[sg][r][lm] (zero outside a particle's
// shells and degrees).  Segments give the sum enough workgroups to fill the chip.
__global__ void __launch_bounds__(256) k_grad_reduce(GradArgs a)
{
    const int64_t nl = (int64_t)(a.Lh + 1) * (a.Lh + 1), E = nl * a.Rh;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    const int r = (int)(e / nl);
    const int lm = (int)(e - (int64_t)r * nl);
    const int l = (int)sqrtf((float)lm + 0.5f);
    const int pb = blockIdx.y * a.seg_len, pe = min(pb + a.seg_len, a.P);
    float2 s = make_float2(0.f, 0.f);
    // 16 particles' loads in flight at a time (clamped to a valid address where the particle has
    // no such term), then added in index order
    constexpr int U = 16;
    for (int p0 = pb; p0 < pe; p0 += U) {
        float2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = min(p0 + u, pe - 1);
            const int Lp = a.Lp[p], Rp = a.Rp[p];
            const bool ok = p0 + u < pe && r < Rp && l <= Lp;
            v[u] = a.ws[ok ? a.ws_off[p] + (int64_t)r * (Lp + 1) * (Lp + 1) + lm : 0];
            if (!ok) v[u] = make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s.x += v[u].x;
            s.y += v[u].y;
        }
    }
    a.part[blockIdx.y * E + e] = s;
}

// grad_h[r][lm] = the segments' partial sums added in segment order.
__global__ void __launch_bounds__(256) k_grad_segments(GradArgs a)
{
    const int64_t E = (int64_t)(a.Lh + 1) * (a.Lh + 1) * a.Rh;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    float2 s = make_float2(0.f, 0.f);
    for (int sg = 0; sg < a.n_seg; ++sg) {
        const float2 v = a.part[sg * E + e];
        s.x += v.x;
        s.y += v.y;
    }
    a.grad_h[e] = s;
}

int grad_segments(int64_t E, int P)
{
    const int64_t blocks = (E + 255) / 256;
    const int64_t want = (2048 + blocks - 1) / blocks;  // about 2048 workgroups in the partial sums
    return (int)std::max<int64_t>(1, std::min<int64_t>({want, 64, (int64_t)std::max(P, 1)}));
}

size_t grad_smem_bytes(int Lmax)
{
    const size_t w = 2 * (size_t)Lmax + 1;
    return sizeof(float) * w * w + sizeof(float2) * 2 * (Lmax + 1) + sizeof(float2) * 2 * kAdjShellChunk * w;
}

hipError_t launch_grad(const GradArgs &a, hipStream_t s)
{
    if (a.ws) {
        hipLaunchKernelGGL(k_term_offsets, dim3(1), dim3(kScanThreads), 0, s, a.Lp, a.Rp, a.P, a.ws_off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_grad_particle, dim3(a.P), dim3(kAdjThreads), grad_smem_bytes(a.L_max), s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.grad_h) return e;
    GradArgs b = a;
    const int64_t n = (int64_t)(a.Lh + 1) * (a.Lh + 1) * a.Rh;
    b.n_seg = grad_segments(n, a.P);
    b.seg_len = (a.P + b.n_seg - 1) / b.n_seg;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_grad_reduce, dim3(nb, (unsigned)b.n_seg), dim3(256), 0, s, b);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad_segments, dim3(nb), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace matcha
