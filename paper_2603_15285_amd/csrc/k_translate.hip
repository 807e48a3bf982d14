// k_translate.hip -- the translation half of the rotation-translation alternation (App. C).
//
// Volumes are [N][N][N] (x fastest, then y, then z) with voxel centres -1 + (2/N)(i + 1/2); shifts are
// in voxels along (x, y, z); spectra are the half-complex transforms [N][N][N/2 + 1] (x halved) of an
// unnormalised forward DFT, F(k) = sum_x f(x) e^{-2 pi i k.x / N}.  With the pose written as
// f = S_s (g o h), (S_s u)(x) = u(x - s) and (g o h)(x) = h(R_g^T x):
//   - the rotation step aligns f(x + s) (its spectrum times e^{+2 pi i k.s / N}) to h,
//   - the translation step maximises c(s) = sum_x f(x) u(x - s) over s for u = g o h; its transform
//     is F conj(U), so the inverse DFT gives c on the integer shifts (cyclic), and
//       c(s) = (1/N^3) Re sum over the half spectrum of w_kx F conj(U)(k) e^{2 pi i k.s / N}
//     (w = 1 for kx = 0 and N/2, 2 otherwise) evaluates it at any real s: the upsampled refinement
//     around the best integer shift, as three separable DFT contractions (x, then y, then z), on a
//     second copy of F conj(U) (the inverse transform consumes its own).
// The Nyquist planes of a shifted spectrum are zeroed (a real volume's Nyquist term has no
// consistent phase at a non-integer shift).
#include "matcha_launch.hpp"

namespace matcha {

__device__ __forceinline__ int signed_freq(int k, int N) { return k <= N / 2 ? k : k - N; }

// u_p(x) = h(R_p^T x): trilinear interpolation of the template at the rotated voxel centre, zero
// outside the grid.  R_p = Rz(a) Ry(b) Rz(c) from euler[p] = (a, b, c, .) (float4).  Grid: voxel
// bricks x particles.
__global__ void __launch_bounds__(256) k_rotate_volume(TransArgs a)
{
    __shared__ float Rs[9];
    const int N = a.N, p = blockIdx.y;
    if (threadIdx.x == 0) {
        const float4 eu = a.euler[p];
        float sa, ca, sb, cb, sc, cc;
        sincosf(eu.x, &sa, &ca);
        sincosf(eu.y, &sb, &cb);
        sincosf(eu.z, &sc, &cc);
        // R = Rz(a) Ry(b) Rz(c), row-major
        Rs[0] = ca * cb * cc - sa * sc;
        Rs[1] = -ca * cb * sc - sa * cc;
        Rs[2] = ca * sb;
        Rs[3] = sa * cb * cc + ca * sc;
        Rs[4] = -sa * cb * sc + ca * cc;
        Rs[5] = sa * sb;
        Rs[6] = -sb * cc;
        Rs[7] = sb * sc;
        Rs[8] = cb;
    }
    __syncthreads();
    // a workgroup takes an 8 x 8 x 4 brick (x, y, z) and each wave a 4 x 4 x 4 brick of it, so that
    // the rotated footprint of a wave's gathers stays compact
    const int n3 = N * N * N, bx = (N + 7) / 8, by = (N + 7) / 8;
    const int b = blockIdx.x, bxi = b % bx, byi = (b / bx) % by, bzi = b / (bx * by);
    const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
    const int ix = 8 * bxi + 4 * (wv & 1) + (ln & 3), iy = 8 * byi + 4 * (wv >> 1) + ((ln >> 2) & 3),
              iz = 4 * bzi + (ln >> 4);
    if (ix >= N || iy >= N || iz >= N) return;
    const int v = (iz * N + iy) * N + ix;
    const float h2 = 2.f / N;
    const float x = -1.f + h2 * (ix + 0.5f), y = -1.f + h2 * (iy + 0.5f), z = -1.f + h2 * (iz + 0.5f);
    // q = R^T x, as fractional indices
    const float qx = Rs[0] * x + Rs[3] * y + Rs[6] * z, qy = Rs[1] * x + Rs[4] * y + Rs[7] * z,
                qz = Rs[2] * x + Rs[5] * y + Rs[8] * z;
    const float fx = (qx + 1.f) * (0.5f * N) - 0.5f, fy = (qy + 1.f) * (0.5f * N) - 0.5f, fz = (qz + 1.f) * (0.5f * N) - 0.5f;
    const int x0 = (int)floorf(fx), y0 = (int)floorf(fy), z0 = (int)floorf(fz);
    const float tx = fx - x0, ty = fy - y0, tz = fz - z0;
    float acc = 0.f;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int xx = x0 + dx, yy = y0 + dy, zz = z0 + dz;
                if (xx < 0 || yy < 0 || zz < 0 || xx >= N || yy >= N || zz >= N) continue;
                const float wgt = (dx ? tx : 1.f - tx) * (dy ? ty : 1.f - ty) * (dz ? tz : 1.f - tz);
                acc = fmaf(wgt, a.h[(zz * N + yy) * N + xx], acc);
            }
    a.vol[(int64_t)p * n3 + v] = acc;
}

// out_p(k) = in_p(k) e^{2 pi i k.s_p / N} / N^3 (so that the inverse transform gives f_p(x + s_p)),
// Nyquist planes zeroed.
__global__ void __launch_bounds__(256) k_phase_shift(TransArgs a)
{
    const int N = a.N, NH = N / 2 + 1;
    const int64_t per = (int64_t)N * N * NH, total = per * a.P;
    const double inv = 1.0 / ((double)N * N * N);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int p = (int)(e / per);
        const int64_t q = e - (int64_t)p * per;
        const int kz = (int)(q / ((int64_t)N * NH)), ky = (int)((q / NH) % N), kx = (int)(q % NH);
        const float4 s = a.shift[p];
        float2 r = make_float2(0.f, 0.f);
        if (kx != N / 2 && ky != N / 2 && kz != N / 2) {
            // phase in turns, reduced before the sine and cosine
            double t = ((double)kx * s.x + (double)signed_freq(ky, N) * s.y + (double)signed_freq(kz, N) * s.z) / N;
            t -= rint(t);
            double sn, cs;
            sincospi(2.0 * t, &sn, &cs);
            const float2 x = a.spec_in[e];
            r = make_float2((float)((x.x * cs - x.y * sn) * inv), (float)((x.x * sn + x.y * cs) * inv));
        }
        a.spec_out[e] = r;
    }
}

// X = F conj(U) in place of U, and a copy for the inverse transform (which consumes its input).
__global__ void __launch_bounds__(256) k_cross_spectrum(TransArgs a)
{
    const int N = a.N, NH = N / 2 + 1;
    const int64_t total = (int64_t)N * N * NH * a.P;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const float2 f = a.spec_in[e], u = a.spec_out[e];
        const float2 x = make_float2(f.x * u.x + f.y * u.y, f.y * u.x - f.x * u.y);
        a.spec_out[e] = x;
        a.spec_aux[e] = x;
    }
}

// Best integer shift of each particle's correlation volume within |s_i| <= window (signed shifts,
// the volume index of s is s mod N); ties go to the smaller volume index.  One workgroup per
// particle, over the (2 window + 1)^3 shifts only.
__global__ void __launch_bounds__(256) k_corr_peak(TransArgs a)
{
    __shared__ float bv[256];
    __shared__ int bi[256];
    const int N = a.N, p = blockIdx.x, W = a.window, span = 2 * W + 1;
    const float *c = a.vol + (int64_t)p * N * N * N;
    float best = -INFINITY;
    int besti = 0x7fffffff;
    for (int t = threadIdx.x; t < span * span * span; t += 256) {
        const int sx = t % span - W, sy = (t / span) % span - W, sz = t / (span * span) - W;
        const int v = (((sz + N) % N) * N + (sy + N) % N) * N + (sx + N) % N;
        const float x = c[v];
        if (x > best || (x == best && v < besti)) {
            best = x;
            besti = v;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = besti;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const float ov = bv[threadIdx.x + o];
            const int oi = bi[threadIdx.x + o];
            if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = ov;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int v = bi[0];
        const int iz = v / (N * N), iy = (v / N) % N, ix = v % N;
        a.peak[p] = make_int4(signed_freq(ix, N), signed_freq(iy, N), signed_freq(iz, N), 0);
    }
}

// Phase tables of the refinement, once per particle (workgroup per particle), for the m offsets
// delta_j = (j - (m - 1) / 2) / kappa around the integer peak s0:
//   Ex[kx][j] = w_kx e^{2 pi i kx (s0x + delta_j) / N},  Ey[ky][j] = e^{2 pi i ky' (s0y + delta_j) / N}.
__global__ void __launch_bounds__(256) k_upsample_tables(TransArgs a)
{
    const int N = a.N, NH = N / 2 + 1, m = a.m, p = blockIdx.x;
    float2 *Ex = a.ups_tab + (int64_t)p * (NH + N) * m, *Ey = Ex + NH * m;
    const int4 s0 = a.peak[p];
    for (int i = threadIdx.x; i < (NH + N) * m; i += 256) {
        const bool isx = i < NH * m;
        const int r = isx ? i : i - NH * m, k = r / m, j = r - (r / m) * m;
        const double d = (isx ? s0.x : s0.y) + (j - 0.5 * (m - 1)) / a.kappa;
        double t = (double)(isx ? k : signed_freq(k, N)) * d / N;
        t -= rint(t);
        double sn, cs;
        sincospi(2.0 * t, &sn, &cs);
        const double w = isx ? ((k == 0 || 2 * k == N) ? 1.0 : 2.0) : 1.0;
        (isx ? Ex : Ey)[isx ? i : r] = make_float2((float)(w * cs), (float)(w * sn));
    }
}

// Stage 1 (workgroup per particle and kz), X = F conj(U) from the cross spectrum:
//   A[ky][a] = sum_kx X[kz][ky][kx] Ex[kx][a]        (in LDS)
//   B[kz][a][b] = sum_ky A[ky][a] Ey[ky][b]          (to the workspace)
__global__ void __launch_bounds__(256) k_upsample_xy(TransArgs a)
{
    extern __shared__ __align__(16) unsigned char ups_smem[];
    const int N = a.N, NH = N / 2 + 1, m = a.m;
    const int p = blockIdx.x / N, kz = blockIdx.x % N;
    float2 *Ex = reinterpret_cast<float2 *>(ups_smem);  // [NH][m]
    float2 *Ey = Ex + NH * m;                             // [N][m]
    float2 *A = Ey + N * m;                               // [N][m]
    const float2 *tab = a.ups_tab + (int64_t)p * (NH + N) * m;
    for (int i = threadIdx.x; i < (NH + N) * m; i += 256) Ex[i] = tab[i];
    __syncthreads();
    const float2 *X = a.spec_out + ((int64_t)p * N + kz) * N * NH;
    for (int i = threadIdx.x; i < N * m; i += 256) {
        const int ky = i / m, j = i - (i / m) * m;
        float re = 0.f, im = 0.f;
        for (int kx = 0; kx < NH; ++kx) {
            const float2 x = X[ky * NH + kx], e = Ex[kx * m + j];
            re = fmaf(x.x, e.x, fmaf(-x.y, e.y, re));
            im = fmaf(x.x, e.y, fmaf(x.y, e.x, im));
        }
        A[i] = make_float2(re, im);
    }
    __syncthreads();
    float2 *Bo = a.ups + ((int64_t)p * N + kz) * m * m;
    for (int i = threadIdx.x; i < m * m; i += 256) {
        const int ja = i / m, jb = i - (i / m) * m;
        float re = 0.f, im = 0.f;
        for (int ky = 0; ky < N; ++ky) {
            const float2 x = A[ky * m + ja], e = Ey[ky * m + jb];
            re = fmaf(x.x, e.x, fmaf(-x.y, e.y, re));
            im = fmaf(x.x, e.y, fmaf(x.y, e.x, im));
        }
        Bo[i] = make_float2(re, im);
    }
}

// Stage 2 (workgroup per particle): c[a][b][cz] = Re sum_kz B[kz][a][b] e^{2 pi i kz' (s0z + delta_cz) / N}
// over the m^3 offsets, then the refined shift at its maximum (ties: the smaller offset index) and
// that value / N^3.
__global__ void __launch_bounds__(256) k_upsample_z(TransArgs a)
{
    extern __shared__ __align__(16) unsigned char ups_smem[];
    __shared__ float bv[256];
    __shared__ int bi[256];
    const int N = a.N, m = a.m, p = blockIdx.x;
    float2 *Ez = reinterpret_cast<float2 *>(ups_smem);  // [N][m]
    const int4 s0 = a.peak[p];
    for (int i = threadIdx.x; i < N * m; i += 256) {
        const int kz = i / m, j = i - (i / m) * m;
        const double d = s0.z + (j - 0.5 * (m - 1)) / a.kappa;
        double t = (double)signed_freq(kz, N) * d / N;
        t -= rint(t);
        double sn, cs;
        sincospi(2.0 * t, &sn, &cs);
        Ez[i] = make_float2((float)cs, (float)sn);
    }
    __syncthreads();
    const float2 *B = a.ups + (int64_t)p * N * m * m;
    float best = -INFINITY;
    int besti = 0x7fffffff;
    const int m3 = m * m * m;
    for (int i = threadIdx.x; i < m3; i += 256) {
        const int ja = i % m, jb = (i / m) % m, jc = i / (m * m);  // x fastest
        float re = 0.f;
        for (int kz = 0; kz < N; ++kz) {
            const float2 x = B[(int64_t)kz * m * m + ja * m + jb], e = Ez[kz * m + jc];
            re = fmaf(x.x, e.x, fmaf(-x.y, e.y, re));
        }
        if (re > best || (re == best && i < besti)) {
            best = re;
            besti = i;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = besti;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const float ov = bv[threadIdx.x + o];
            const int oi = bi[threadIdx.x + o];
            if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = ov;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int i = bi[0], ja = i % m, jb = (i / m) % m, jc = i / (m * m);
        const float h = 0.5f * (m - 1);
        a.shift_out[p] = make_float4(s0.x + (ja - h) / a.kappa, s0.y + (jb - h) / a.kappa, s0.z + (jc - h) / a.kappa,
                                     bv[0] / ((float)N * N * N));
    }
}

static unsigned grid_1d(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16)); }

hipError_t launch_rotate_volume(const TransArgs &a, hipStream_t s)
{
    const int nb = ((a.N + 7) / 8) * ((a.N + 7) / 8) * ((a.N + 3) / 4);
    hipLaunchKernelGGL(k_rotate_volume, dim3(nb, a.P), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_phase_shift(const TransArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_phase_shift, dim3(grid_1d((int64_t)a.N * a.N * (a.N / 2 + 1) * a.P)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cross_spectrum(const TransArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_cross_spectrum, dim3(grid_1d((int64_t)a.N * a.N * (a.N / 2 + 1) * a.P)), dim3(256), 0, s,
                       a);
    return hipGetLastError();
}

size_t upsample_xy_smem(int N, int m) { return sizeof(float2) * (size_t)m * ((N / 2 + 1) + 2 * N); }

hipError_t launch_peak_refine(const TransArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_corr_peak, dim3(a.P), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_upsample_tables, dim3(a.P), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_upsample_xy, dim3(a.P * a.N), dim3(256), upsample_xy_smem(a.N, a.m), s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_upsample_z, dim3(a.P), dim3(256), sizeof(float2) * (size_t)a.N * a.m, s, a);
    return hipGetLastError();
}

}  // namespace matcha
