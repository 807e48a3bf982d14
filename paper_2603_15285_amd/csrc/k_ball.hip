// k_ball.hip -- ball-harmonic (Fourier-Bessel) coefficients of volumes on a Cartesian grid, the step
// before the alignment path (App. A.1):
//   u_klm = (2/N)^3 sum over voxel centres x_v inside the unit ball of u(x_v) conj(psi_klm(x_v)),
//   psi_klm(x) = c_lk j_l(lam_lk |x|) Y_lm(x / |x|),  c_lk = sqrt(2) / |j_{l+1}(lam_lk)|,
// lam_lk the k-th positive zero of the spherical Bessel function j_l, kept while lam_lk <= Lambda
// (the index set I_Lambda; |K_l| radial indices at degree l).  Voxel centres sit at
// -1 + (2/N)(i + 1/2) per axis; a volume is [N][N][N] with x fastest, then y, then z.
//
// The sum is computed exactly (no fast transform): for each degree l it is a product over the
// voxels inside the ball,
//   out_l[(p, k)][(m, re/im)] = sum_v (u_p(v) R_lk(v)) A_lm(v),
//   R_lk(v) = (2/N)^3 c_lk j_l(lam_lk r_v),  A_lm(v) = conj Y_lm(v) = Ybar_l^m(cos t_v) e^{-i m p_v},
// with rows (volume, radial index) and columns (m >= 0, real and imaginary part), on the matrix
// cores.  Real volumes give u_{k,l,-m} = (-1)^m conj(u_klm), written from the m >= 0 columns.  The
// tables R and A are built once per (N, Lambda) on the host in FP64 (spherical Bessel values by
// recurrence, zeros by bracketing and bisection, normalised associated Legendre functions by the
// standard three-term recurrence) and kept on the device in FP32.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "matcha_ball.hpp"

namespace matcha {

// ---------------------------------------------------------------- host: tables
namespace {

// j_0 .. j_n at x >= 0 (FP64): upward recurrence where it is stable (n < x), else Miller's
// downward recurrence normalised by j_0 or j_1, whichever is farther from zero.
void sph_jn_all(int n, double x, double *j)
{
    if (x == 0.0) {
        j[0] = 1.0;
        for (int l = 1; l <= n; ++l) j[l] = 0.0;
        return;
    }
    const double s = std::sin(x), c = std::cos(x);
    const double j0 = s / x, j1 = s / (x * x) - c / x;
    if (n < x) {
        j[0] = j0;
        if (n >= 1) j[1] = j1;
        for (int l = 1; l < n; ++l) j[l + 1] = (2.0 * l + 1.0) / x * j[l] - j[l - 1];
        return;
    }
    // f_{top+1} = 0, f_top tiny, f_{l-1} = (2l+1)/x f_l - f_{l+1}: proportional to j_l for l well
    // below top; rescaled whenever it grows large
    const int top = n + 20 + (int)std::sqrt(40.0 * (n + 1));
    std::vector<double> f((size_t)top + 2, 0.0);
    f[(size_t)top] = 1e-250;
    for (int l = top; l >= 1; --l) {
        f[(size_t)(l - 1)] = (2.0 * l + 1.0) / x * f[(size_t)l] - f[(size_t)(l + 1)];
        if (std::fabs(f[(size_t)(l - 1)]) > 1e200)
            for (int q = l - 1; q <= top + 1; ++q) f[(size_t)q] *= 1e-200;
    }
    const double scale = std::fabs(j0) >= std::fabs(j1) ? j0 / f[0] : j1 / f[1];
    for (int l = 0; l <= n; ++l) j[l] = f[(size_t)l] * scale;
}

double sph_jn(int l, double x)
{
    std::vector<double> j((size_t)l + 2);
    sph_jn_all(l, x, j.data());
    return j[(size_t)l];
}

// Positive zeros of j_l up to lam: sign changes on a 0.05 grid from l (the first zero lies above
// l), each refined by bisection to the last bit.
std::vector<double> sph_jn_zeros(int l, double lam)
{
    std::vector<double> z;
    if (lam <= l) return z;
    double x0 = std::max((double)l, 1e-3), v0 = sph_jn(l, x0);
    for (double x1 = x0 + 0.05; x0 < lam + 0.5; x1 += 0.05) {
        const double v1 = sph_jn(l, x1);
        if (v0 == 0.0) {
            z.push_back(x0);
        } else if (v0 * v1 < 0.0) {
            double a = x0, b = x1, fa = v0;
            for (int it = 0; it < 200 && b - a > 0.0; ++it) {
                const double mid = 0.5 * (a + b);
                if (mid <= a || mid >= b) break;
                const double fm = sph_jn(l, mid);
                if ((fm < 0.0) == (fa < 0.0)) {
                    a = mid;
                    fa = fm;
                } else {
                    b = mid;
                }
            }
            z.push_back(0.5 * (a + b));
        }
        x0 = x1;
        v0 = v1;
    }
    std::vector<double> out;
    for (double x : z)
        if (x <= lam) out.push_back(x);
    return out;
}

// Ybar_l^m(t) for 0 <= m <= l <= L at t = cos(theta), s = sin(theta) >= 0, with the Condon-Shortley
// phase and Y_lm = Ybar_l^m e^{i m phi} orthonormal on the sphere; out[l (l+1)/2 + m].
void legendre_all(int L, double t, double s, double *out)
{
    double pmm = 1.0 / std::sqrt(4.0 * M_PI);
    for (int m = 0; m <= L; ++m) {
        if (m > 0) pmm = -std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * pmm;
        out[m * (m + 1) / 2 + m] = pmm;
        if (m == L) break;
        double p2 = pmm, p1 = std::sqrt(2.0 * m + 3.0) * t * pmm;
        out[(m + 1) * (m + 2) / 2 + m] = p1;
        for (int l = m + 2; l <= L; ++l) {
            const double a = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            const double b = std::sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
            const double p = a * (t * p1 - b * p2);
            out[l * (l + 1) / 2 + m] = p;
            p2 = p1;
            p1 = p;
        }
    }
}

template <typename F>
void parallel_for(int64_t n, F &&f)
{
    const int nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int64_t i = t; i < n; i += nt) f(i);
        });
    for (auto &x : th) x.join();
}

}  // namespace

bool ball_index(double lam, BallIndex &ix)
{
    ix.zeros.clear();
    if (!(lam > 0.0) || lam > 1000.0) return false;
    for (int l = 0;; ++l) {
        std::vector<double> z = sph_jn_zeros(l, lam);
        if (z.empty()) break;
        ix.zeros.push_back(z);
    }
    if (ix.zeros.empty()) return false;
    ix.L = (int)ix.zeros.size() - 1;
    ix.Kmax = (int)ix.zeros[0].size();
    ix.nk = 0;
    for (const auto &z : ix.zeros) ix.nk += (int)z.size();
    return true;
}

void ball_build_tables(int N, const BallIndex &ix, std::vector<int32_t> &vidx, std::vector<float> &R,
                       std::vector<float> &A)
{
    vidx.clear();
    std::vector<double> xs, ys, zs;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int k = 0; k < N; ++k) {
                const double z = -1.0 + (2.0 / N) * (i + 0.5), y = -1.0 + (2.0 / N) * (j + 0.5),
                             x = -1.0 + (2.0 / N) * (k + 0.5);
                if (std::sqrt(x * x + y * y + z * z) < 1.0) {
                    vidx.push_back((int32_t)((i * N + j) * N + k));
                    xs.push_back(x);
                    ys.push_back(y);
                    zs.push_back(z);
                }
            }
    const int64_t V = (int64_t)vidx.size();
    const int L = ix.L;
    const double dv = std::pow(2.0 / N, 3);
    // radial table, rows (l, k) in degree-major order: dv c_lk j_l(lam_lk r_v)
    std::vector<double> clk;
    std::vector<std::pair<int, double>> lk;
    for (int l = 0; l <= L; ++l)
        for (double lam : ix.zeros[(size_t)l]) {
            lk.push_back({l, lam});
            clk.push_back(std::sqrt(2.0) / std::fabs(sph_jn(l + 1, lam)));
        }
    R.assign((size_t)ix.nk * (size_t)V, 0.f);
    parallel_for((int64_t)lk.size(), [&](int64_t q) {
        const int l = lk[(size_t)q].first;
        const double lam = lk[(size_t)q].second, c = dv * clk[(size_t)q];
        std::vector<double> j((size_t)l + 2);
        for (int64_t v = 0; v < V; ++v) {
            const double r = std::sqrt(xs[(size_t)v] * xs[(size_t)v] + ys[(size_t)v] * ys[(size_t)v] +
                                       zs[(size_t)v] * zs[(size_t)v]);
            sph_jn_all(l, lam * r, j.data());
            R[(size_t)q * (size_t)V + (size_t)v] = (float)(c * j[(size_t)l]);
        }
    });
    // angular table, rows (l, m >= 0, re / im): conj Y_lm = Ybar_l^m(cos t) (cos m p - i sin m p)
    const int ncol = (L + 1) * (L + 2);  // 2 per (l, m >= 0)
    A.assign((size_t)ncol * (size_t)V, 0.f);
    parallel_for(V, [&](int64_t v) {
        const double x = xs[(size_t)v], y = ys[(size_t)v], z = zs[(size_t)v];
        const double r = std::sqrt(x * x + y * y + z * z);
        const double t = r > 0.0 ? std::max(-1.0, std::min(1.0, z / r)) : 1.0;
        const double s = std::sqrt(std::max(0.0, 1.0 - t * t));
        const double ph = std::atan2(y, x);
        std::vector<double> P((size_t)(L + 1) * (L + 2) / 2);
        legendre_all(L, t, s, P.data());
        for (int l = 0; l <= L; ++l)
            for (int m = 0; m <= l; ++m) {
                const int col = 2 * (l * (l + 1) / 2 + m);
                const double p = P[(size_t)(l * (l + 1) / 2 + m)];
                A[(size_t)col * (size_t)V + (size_t)v] = (float)(p * std::cos(m * ph));
                A[(size_t)(col + 1) * (size_t)V + (size_t)v] = (float)(-p * std::sin(m * ph));
            }
    });
}

// ---------------------------------------------------------------- device
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBallThreads = 256;  // 4 waves; the workgroup's tile is 64 rows x all columns of its degree
constexpr int kBallRows = 64;
constexpr int kBallChunk = 32;     // voxels per staged chunk (8 matrix-core K steps of 4)
constexpr int kBallMaxCT = 8;      // 16-column tiles per degree: 2 (l + 1) <= 128, l <= 63

// Entries of radial indices k >= |K_l| are zero.
__global__ void __launch_bounds__(256) k_ball_zero(BallArgs a)
{
    const int64_t nlm = (int64_t)(a.L + 1) * (a.L + 1);
    const int64_t n = (int64_t)a.P * a.Kmax * nlm;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t lm = e % nlm;
        const int k = (int)((e / nlm) % a.Kmax);
        const int l = (int)sqrtf((float)lm + 0.5f);
        if (k >= a.nk_l[l]) reinterpret_cast<float2 *>(a.out)[e] = make_float2(0.f, 0.f);
    }
}

// One workgroup per (degree l, tile of 64 rows (volume, radial index)), highest degrees first; wave w
// owns rows 16 w .. 16 w + 15 and every 16-column tile of the degree.  Voxels are staged in chunks
// of 32: the A tile (u_p(v) R_lk(v), rows x voxels) and the B tile (A_lm(v), voxels x columns) in
// LDS, zero outside the degree's rows, columns and the voxel count.
__global__ void __launch_bounds__(kBallThreads) k_ball_gemm(BallArgs a)
{
    __shared__ float As[kBallRows][kBallChunk + 1];
    __shared__ float Bs[kBallChunk][16 * kBallMaxCT + 4];
    int d = 0;
    while ((int)blockIdx.x >= a.blk_lo[d + 1]) ++d;
    const int l = a.L - d, rt = blockIdx.x - a.blk_lo[d];
    const int K = a.nk_l[l], M = a.P * K, NC = 2 * (l + 1), CT = (NC + 15) / 16;
    const int rbase = a.rk_off[l];  // first row of degree l in the radial table
    const int cbase = l * (l + 1);  // first column of degree l in the angular table
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int col = lane % 16, kq = lane / 16;
    const int64_t V = a.V, N3 = (int64_t)a.N * a.N * a.N;
    // the staging assignment of this thread: rows / columns t / 32 + 8 i, voxel t % 32
    const int tv = threadIdx.x % kBallChunk, tr = threadIdx.x / kBallChunk;
    int prow[kBallRows / 8], krow[kBallRows / 8];
    bool rok[kBallRows / 8];
#pragma unroll
    for (int i = 0; i < kBallRows / 8; ++i) {
        const int rg = rt * kBallRows + tr + 8 * i;
        rok[i] = rg < M;
        const int rc = min(rg, M - 1);
        prow[i] = rc / K;
        krow[i] = rc - prow[i] * K;
    }
    f32x4 acc[kBallMaxCT];
#pragma unroll
    for (int c = 0; c < kBallMaxCT; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t v0 = 0; v0 < V; v0 += kBallChunk) {
        const int64_t v = v0 + tv;
        const bool vok = v < V;
        const int64_t vc = vok ? v : V - 1;
        const int gi = a.vidx[vc];
#pragma unroll
        for (int i = 0; i < kBallRows / 8; ++i) {
            const float u = a.u[(int64_t)prow[i] * N3 + gi];
            const float r = a.R[(int64_t)(rbase + krow[i]) * V + vc];
            As[tr + 8 * i][tv] = (rok[i] && vok) ? u * r : 0.f;
        }
        for (int c = tr; c < 16 * CT; c += kBallThreads / kBallChunk) {
            const float b = a.A[(int64_t)(cbase + min(c, NC - 1)) * V + vc];
            Bs[tv][c] = (c < NC && vok) ? b : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kBallChunk / 4; ++ks) {
            const float av = As[16 * wave + col][4 * ks + kq];
#pragma unroll
            for (int c = 0; c < kBallMaxCT; ++c)
                if (c < CT) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Bs[4 * ks + kq][16 * c + col], acc[c], 0, 0, 0);
        }
        __syncthreads();
    }
    // lane (kq, col) holds rows 4 kq .. 4 kq + 3 of column col of each tile: write u_klm and, for
    // m > 0, u_{k,l,-m} = (-1)^m conj(u_klm)
    const int64_t nlm = (int64_t)(a.L + 1) * (a.L + 1);
#pragma unroll
    for (int c = 0; c < kBallMaxCT; ++c) {
        if (c >= CT) continue;
        const int cc = 16 * c + col;
        if (cc >= NC) continue;
        const int m = cc / 2, part = cc % 2;
        const float sgn = (m & 1) ? -1.f : 1.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rg = rt * kBallRows + 16 * wave + 4 * kq + q;
            if (rg >= M) continue;
            const int p = rg / K, k = rg - (rg / K) * K;
            float *o = a.out + 2 * (((int64_t)p * a.Kmax + k) * nlm + (int64_t)l * l + l);
            o[2 * m + part] = acc[c][q];
            if (m > 0) o[-2 * m + part] = part ? -sgn * acc[c][q] : sgn * acc[c][q];
        }
    }
}

hipError_t launch_ball(const BallArgs &a0, hipStream_t s)
{
    BallArgs a = a0;
    int nb = 0;
    for (int d = 0; d <= a.L; ++d) {
        const int l = a.L - d;
        a.blk_lo[d] = nb;
        nb += (int)(((int64_t)a.P * a.nk_l[l] + kBallRows - 1) / kBallRows);
    }
    a.blk_lo[a.L + 1] = nb;
    const int64_t n = (int64_t)a.P * a.Kmax * (a.L + 1) * (a.L + 1);
    const unsigned zb = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_ball_zero, dim3(std::max(zb, 1u)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 0) return e;
    hipLaunchKernelGGL(k_ball_gemm, dim3(nb), dim3(kBallThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace matcha
