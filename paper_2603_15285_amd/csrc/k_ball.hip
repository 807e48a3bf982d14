// k_ball.hip -- ball-harmonic (Fourier-Bessel) coefficients of volumes on a Cartesian grid, the step
// before the alignment path (App. A.1):
//   u_klm = (2/N)^3 sum over voxel centres x_v inside the unit ball of u(x_v) conj(psi_klm(x_v)),
//   psi_klm(x) = c_lk j_l(lam_lk |x|) Y_lm(x / |x|),  c_lk = sqrt(2) / |j_{l+1}(lam_lk)|,
// lam_lk the k-th positive zero of the spherical Bessel function j_l, kept while lam_lk <= Lambda
// (the index set I_Lambda; |K_l| radial indices at degree l).  Voxel centres sit at
// -1 + (2/N)(i + 1/2) per axis; a volume is [N][N][N] with x fastest, then y, then z.
//
// The sum is computed exactly (no fast transform), folded onto one octant.  The grid is mapped onto
// itself by the three mirrors x -> -x, y -> -y, z -> -z, and each real column function of the
// transform has a definite sign under each of them:
//   Re conj psi_klm = c_lk j_l Ybar_l^m(cos t) cos(m p),  Im conj psi_klm = -c_lk j_l Ybar_l^m(cos t) sin(m p),
//   z -> -z: (-1)^(l+m) (Ybar_l^m(-t) = (-1)^(l+m) Ybar_l^m(t));  y -> -y: +1 (Re), -1 (Im);
//   x -> -x: (-1)^m (Re), -(-1)^m (Im)   (p -> pi - p).
// So with sigma = (s_x, s_y, s_z) the column's signs and, for an octant voxel v0 (x, y, z >= 0),
//   usym_sigma(v0) = sum over the 8 mirror images g v0 of sign_sigma(g) u(g v0),
// the coefficient is  sum over octant voxels of usym_sigma(v0) psi*(v0) / |Stab v0|  (a voxel on a
// mirror plane, odd N only, is its own image: the orbit sum counts it |Stab| times).  Per class sigma
// that is one plain product over the octant voxels:
//   out_sigma[p][c] = sum_v0 usym_sigma[p][v0] T[c][v0],  T[c][v0] = (2/N)^3 / |Stab v0| psi*_c(v0),
// rows = volumes, columns = the (l, k, m, Re/Im) of class sigma (8 classes, 8 times fewer terms than the
// full-grid sum).  Three kernels: the sign-symmetrised volumes (k_ball_sym), the products on the
// matrix cores in K-split partial sums (k_ball_gemm), and the sum of the partials scattered into the
// [Kmax][(L+1)^2] layout with u_{k,l,-m} = (-1)^m conj(u_klm) and zeros where k >= |K_l|
// (k_ball_scatter).  The table T is built once per (N, Lambda) on the host in FP64 (spherical Bessel
// values by recurrence, zeros by bracketing and bisection, normalised associated Legendre functions
// by the standard three-term recurrence) and kept on the device in FP32.
#include <algorithm>
#include <cmath>
#include <thread>
#include <type_traits>
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

void ball_build_tables(int N, const BallIndex &ix, BallHostTables &t)
{
    // octant voxels (z, y, x >= 0: indices >= N / 2 rounded down), raster order, and |Stab|
    const int i0 = N / 2;
    std::vector<double> xs, ys, zs, wt;
    t.oct.clear();
    for (int i = i0; i < N; ++i)
        for (int j = i0; j < N; ++j)
            for (int k = i0; k < N; ++k) {
                const double z = -1.0 + (2.0 / N) * (i + 0.5), y = -1.0 + (2.0 / N) * (j + 0.5),
                             x = -1.0 + (2.0 / N) * (k + 0.5);
                if (std::sqrt(x * x + y * y + z * z) >= 1.0) continue;
                t.oct.push_back((int32_t)((i * N + j) * N + k));
                xs.push_back(x);
                ys.push_back(y);
                zs.push_back(z);
                const int on_planes = (2 * i + 1 == N) + (2 * j + 1 == N) + (2 * k + 1 == N);
                wt.push_back(std::pow(2.0 / N, 3) / (double)(1 << on_planes));
            }
    const int64_t Vo = (int64_t)t.oct.size();
    t.Vo = Vo;
    t.Vo_pad = (Vo + kBallChunk - 1) / kBallChunk * kBallChunk;
    const int L = ix.L;
    // columns by class, in (l, k, m, part) order within a class
    struct Col {
        int l, k, m, part;
    };
    std::vector<Col> cols[8];
    for (int l = 0; l <= L; ++l)
        for (int k = 0; k < (int)ix.zeros[(size_t)l].size(); ++k)
            for (int m = 0; m <= l; ++m)
                for (int part = 0; part < 2; ++part) {
                    if (part == 1 && m == 0) continue;  // Im conj psi_kl0 = 0
                    const int sz = (l + m) & 1, sy = part, sx = (m & 1) ^ part;
                    cols[sx | (sy << 1) | (sz << 2)].push_back({l, k, m, part});
                }
    std::vector<Col> all;
    for (int c = 0; c < 8; ++c) {
        t.col_off[c] = (int)all.size();
        all.insert(all.end(), cols[c].begin(), cols[c].end());
    }
    t.col_off[8] = (int)all.size();
    const int64_t nc = (int64_t)all.size();
    // scatter map: per output entry (k, lm) the columns of Re and Im (-1: none) and the signs
    const int nlm = (L + 1) * (L + 1);
    t.map.assign((size_t)ix.Kmax * nlm, BallMapEntry{-1, -1, 1.f, 1.f});
    for (int64_t c = 0; c < nc; ++c) {
        const Col &q = all[(size_t)c];
        for (int sgn : {1, -1}) {
            if (sgn < 0 && q.m == 0) continue;
            const int m = sgn * q.m;
            BallMapEntry &e = t.map[(size_t)q.k * nlm + q.l * q.l + q.l + m];
            const float par = (q.m & 1) ? -1.f : 1.f;  // u_{k,l,-m} = (-1)^m conj(u_klm)
            if (q.part == 0) {
                e.col_re = (int32_t)c;
                e.s_re = sgn > 0 ? 1.f : par;
            } else {
                e.col_im = (int32_t)c;
                e.s_im = sgn > 0 ? 1.f : -par;
            }
        }
    }
    // normalisation c_lk and the table T [nc][Vo_pad], zero in the padding
    std::vector<double> clk;
    std::vector<int> clk_off((size_t)L + 2, 0);
    for (int l = 0; l <= L; ++l) {
        clk_off[(size_t)l + 1] = clk_off[(size_t)l] + (int)ix.zeros[(size_t)l].size();
        for (double lam : ix.zeros[(size_t)l]) clk.push_back(std::sqrt(2.0) / std::fabs(sph_jn(l + 1, lam)));
    }
    t.T.assign((size_t)nc * (size_t)t.Vo_pad, 0.f);
    parallel_for(Vo, [&](int64_t v) {
        const double x = xs[(size_t)v], y = ys[(size_t)v], z = zs[(size_t)v];
        const double r = std::sqrt(x * x + y * y + z * z);
        const double ct = r > 0.0 ? std::max(-1.0, std::min(1.0, z / r)) : 1.0;
        const double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
        const double ph = std::atan2(y, x);
        std::vector<double> P((size_t)(L + 1) * (L + 2) / 2), jr((size_t)clk.size()), j((size_t)L + 2);
        legendre_all(L, ct, st, P.data());
        for (int l = 0; l <= L; ++l)
            for (int k = 0; k < (int)ix.zeros[(size_t)l].size(); ++k) {
                sph_jn_all(l, ix.zeros[(size_t)l][(size_t)k] * r, j.data());
                jr[(size_t)(clk_off[(size_t)l] + k)] = clk[(size_t)(clk_off[(size_t)l] + k)] * j[(size_t)l];
            }
        for (int64_t c = 0; c < nc; ++c) {
            const Col &q = all[(size_t)c];
            const double ang = q.part == 0 ? std::cos(q.m * ph) : -std::sin(q.m * ph);
            const double val = wt[(size_t)v] * jr[(size_t)(clk_off[(size_t)q.l] + q.k)] *
                               P[(size_t)(q.l * (q.l + 1) / 2 + q.m)] * ang;
            t.T[(size_t)c * (size_t)t.Vo_pad + (size_t)v] = (float)val;
        }
    });
}

// ---------------------------------------------------------------- device
typedef float f32x4 __attribute__((ext_vector_type(4)));

// usym[sigma][p][v] for v < Vo_pad (zero in the padding), sigma = s_x | s_y << 1 | s_z << 2 (bit set:
// odd under that mirror).  One thread per (p, v): the 8 mirror images, then three sum/difference steps.
__global__ void __launch_bounds__(256) k_ball_sym(BallSymArgs a)
{
    const int64_t n = (int64_t)a.P * a.Vo_pad;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int p = (int)(e / a.Vo_pad);
        const int64_t v = e - (int64_t)p * a.Vo_pad;
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (v < a.Vo) {
            const int N = a.N, f = a.oct[v];
            const int i = f / (N * N), j = (f / N) % N, k = f % N;
            const float *up = a.u + (int64_t)p * N * N * N;
            // s[g], g = gx | gy << 1 | gz << 2: the image with the flagged coordinates negated
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const int ii = (g & 4) ? N - 1 - i : i, jj = (g & 2) ? N - 1 - j : j, kk = (g & 1) ? N - 1 - k : k;
                s[g] = up[((int64_t)ii * N + jj) * N + kk];
            }
            // butterflies: along x (bit 0), y (bit 1), z (bit 2): even part in the low slot, odd in the high
#pragma unroll
            for (int b = 1; b < 8; b <<= 1)
#pragma unroll
                for (int g = 0; g < 8; ++g)
                    if (!(g & b)) {
                        const float lo = s[g], hi = s[g | b];
                        s[g] = lo + hi;
                        s[g | b] = lo - hi;
                    }
        }
#pragma unroll
        for (int sg = 0; sg < 8; ++sg) a.usym[((int64_t)sg * a.P + p) * a.Vo_pad + v] = s[sg];
    }
}

constexpr int kBallThreads = 256;   // 4 waves as 2 x 2
constexpr int kBallTileN = 128;     // columns per workgroup
constexpr int kBallLds = kBallChunk + 4;  // floats per staged row (K contiguous, padded)

// One workgroup: class sigma and a 128-column tile of it (blockIdx.x), TM volumes (blockIdx.y), one
// K split (blockIdx.z), over the octant voxels [z kper, min((z + 1) kper, Vo_pad)); wave (wr, wc)
// owns TM / 2 rows x 64 columns.  Both operands are K-contiguous rows staged through LDS in chunks
// of 32 voxels, double-buffered (the next chunk's global loads are in flight during the current
// chunk's products).  In each 16-voxel group lane (kq, i) takes voxels 4 kq .. 4 kq + 3 of rows /
// columns i as one float4 and feeds them to four 16x16x4 steps: the voxel order within the group is
// permuted identically on both operands.  Partial sums go to part[z][p][col].
template <int TM>
__global__ void __launch_bounds__(kBallThreads) k_ball_gemm(BallGemmArgs a)
{
    constexpr int RT = TM / 32;  // 16-row tiles per wave
    __shared__ __align__(16) float As[2][TM][kBallLds];
    __shared__ __align__(16) float Bs[2][kBallTileN][kBallLds];
    int sg = 0;
    while ((int)blockIdx.x >= a.tile_lo[sg + 1]) ++sg;
    const int c0 = (blockIdx.x - a.tile_lo[sg]) * kBallTileN;     // first column of the tile in its class
    const int ncls = a.col_off[sg + 1] - a.col_off[sg];
    const int p0 = blockIdx.y * TM;
    const int64_t v_lo = (int64_t)blockIdx.z * a.kper;
    const int64_t v_hi = min(v_lo + a.kper, a.Vo_pad);
    const int nch = (int)((v_hi - v_lo) / kBallChunk);
    const float *Ag = a.usym + ((int64_t)sg * a.P) * a.Vo_pad;
    const float *Bg = a.T + (int64_t)a.col_off[sg] * a.Vo_pad;
    // staging: A TM rows x 8 float4 (TM / 32 per thread), B 128 rows x 8 float4 (4 per thread).  Rows
    // past the last volume and columns past the class's last are loaded from the last one instead:
    // an output entry depends on its own row and column only, and those entries are not written.
    const int t = threadIdx.x, sq = t % 8, sr = t / 8;  // float4 sq of rows sr, sr + 32, ...
    f32x4 ra[TM / 32], rb[4];
    auto load = [&](int ch) {
        const int64_t v = v_lo + (int64_t)ch * kBallChunk + 4 * sq;
#pragma unroll
        for (int i = 0; i < TM / 32; ++i)
            ra[i] = *reinterpret_cast<const f32x4 *>(Ag + (int64_t)min(p0 + sr + 32 * i, a.P - 1) * a.Vo_pad + v);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            rb[i] = *reinterpret_cast<const f32x4 *>(Bg + (int64_t)min(c0 + sr + 32 * i, ncls - 1) * a.Vo_pad + v);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < TM / 32; ++i) *reinterpret_cast<f32x4 *>(&As[buf][sr + 32 * i][4 * sq]) = ra[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) *reinterpret_cast<f32x4 *>(&Bs[buf][sr + 32 * i][4 * sq]) = rb[i];
    };
    const int wave = t / kWave, lane = t % kWave, li = lane % 16, kq = lane / 16;
    const int wr = (TM / 2) * (wave / 2), wc = 64 * (wave % 2);
    // this wave's 16-column tiles that hold columns of the class (wave-uniform)
    const int ntj = min(4, max(0, (ncls - c0 - wc + 15) / 16));
    f32x4 acc[RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (nch > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) load(ch + 1);
        // a wave whose 16-column tiles all hold columns of the class runs them unchecked; the last
        // tile of a class skips the products of its tiles past the class's last column
        auto products = [&](auto full) {
#pragma unroll
            for (int g = 0; g < kBallChunk / 16; ++g) {
                f32x4 av[RT], bv[4];
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    av[i] = *reinterpret_cast<const f32x4 *>(&As[buf][wr + 16 * i + li][16 * g + 4 * kq]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bv[j] = *reinterpret_cast<const f32x4 *>(&Bs[buf][wc + 16 * j + li][16 * g + 4 * kq]);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int i = 0; i < RT; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (decltype(full)::value || j < ntj)
                                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][s], bv[j][s], acc[i][j], 0, 0, 0);
            }
        };
        if (ntj == 4)
            products(std::true_type{});
        else
            products(std::false_type{});
        if (ch + 1 < nch) store(buf ^ 1);
        __syncthreads();
    }
    // lane (kq, li) holds rows 4 kq .. 4 kq + 3 of column li of each 16 x 16 tile
    float *out = a.part + (int64_t)blockIdx.z * a.P * a.ncol + a.col_off[sg];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = c0 + wc + 16 * j + li;
        if (col >= ncls) continue;
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = p0 + wr + 16 * i + 4 * kq + q;
                if (row < a.P) out[(int64_t)row * a.ncol + col] = acc[i][j][q];
            }
    }
}

// out[p][e] = (s_re sum_z part[z][p][col_re], s_im sum_z part[z][p][col_im]), zero where a column is -1.
__global__ void __launch_bounds__(256) k_ball_scatter(BallScatterArgs a)
{
    const int64_t n = (int64_t)a.P * a.n_entries;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int p = (int)(e / a.n_entries);
        const BallMapEntry m = a.map[e - (int64_t)p * a.n_entries];
        // unconditional loads (column 0 stands in for a missing column, masked afterwards), so that
        // the partials' loads are all in flight together rather than one behind each branch
        const int cre = max(m.col_re, 0), cim = max(m.col_im, 0);
        const float *pz = a.part + (int64_t)p * a.ncol;
        const int64_t zs = (int64_t)a.P * a.ncol;
        float vr[kBallMaxSplits], vi[kBallMaxSplits];
#pragma unroll
        for (int z = 0; z < kBallMaxSplits; ++z) {
            const int64_t o = (int64_t)min(z, a.S - 1) * zs;  // splits past S re-read the last one
            vr[z] = pz[o + cre];
            vi[z] = pz[o + cim];
        }
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int z = 0; z < kBallMaxSplits; ++z)
            if (z < a.S) {
                re += vr[z];
                im += vi[z];
            }
        re = m.col_re >= 0 ? m.s_re * re : 0.f;
        im = m.col_im >= 0 ? m.s_im * im : 0.f;
        reinterpret_cast<float2 *>(a.out)[e] = make_float2(re, im);
    }
}

// The same sums, one workgroup per volume when the volume's column sums fit in LDS: the partials
// are read in coalesced runs (16 columns per thread, every split's loads of a run in flight
// together) and summed per column in split order, as above, then the entries read their columns
// from LDS and are written in order.
constexpr int kBallScatterCols = 16 * 256;  // columns per pass
constexpr int kBallScatterLdsCols = 16384;
__global__ void __launch_bounds__(256) k_ball_scatter_vol(BallScatterArgs a)
{
    extern __shared__ float colsum[];  // [ncol]
    const int p = blockIdx.x, t = threadIdx.x;
    const int64_t zs = (int64_t)a.P * a.ncol;
    const float *pp = a.part + (int64_t)p * a.ncol;
    for (int c0 = 0; c0 < a.ncol; c0 += kBallScatterCols) {
        float acc[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = 0.f;
        for (int z = 0; z < a.S; ++z) {
            const float *pz = pp + z * zs;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] += pz[min(c0 + u * 256 + t, a.ncol - 1)];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = c0 + u * 256 + t;
            if (c < a.ncol) colsum[c] = acc[u];
        }
    }
    __syncthreads();
    // eight map entries per thread loaded before any output is stored (the stores could otherwise
    // alias the map for the compiler, which would then wait for each load in turn)
    float2 *out = reinterpret_cast<float2 *>(a.out) + (int64_t)p * a.n_entries;
    for (int e0 = 0; e0 < a.n_entries; e0 += 8 * 256) {
        BallMapEntry mv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) mv[u] = a.map[min(e0 + u * 256 + t, a.n_entries - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * 256 + t;
            if (e < a.n_entries) {
                const float re = mv[u].col_re >= 0 ? mv[u].s_re * colsum[max(mv[u].col_re, 0)] : 0.f;
                const float im = mv[u].col_im >= 0 ? mv[u].s_im * colsum[max(mv[u].col_im, 0)] : 0.f;
                out[e] = make_float2(re, im);
            }
        }
    }
}

int ball_tile_m(int P) { return P >= kBallTileMBig ? 128 : 64; }

int ball_splits(int P, int ncol_tiles, int64_t Vo_pad, int n_cu)
{
    const int tm = ball_tile_m(P);
    const int64_t tiles = (int64_t)((P + tm - 1) / tm) * ncol_tiles;
    const int64_t want = std::max<int64_t>(1, (8LL * n_cu + tiles - 1) / tiles);  // about 8 workgroups per CU
    const int64_t max_s = std::max<int64_t>(1, Vo_pad / (8 * kBallChunk));           // at least 8 chunks each
    return (int)std::min<int64_t>(std::min<int64_t>(want, max_s), kBallMaxSplits);
}

int ball_col_tiles(const int *col_off, int *tile_lo)
{
    int nt = 0;
    for (int c = 0; c < 8; ++c) {
        if (tile_lo) tile_lo[c] = nt;
        nt += (col_off[c + 1] - col_off[c] + kBallTileN - 1) / kBallTileN;
    }
    if (tile_lo) tile_lo[8] = nt;
    return nt;
}

hipError_t launch_ball(const BallSymArgs &sa, const BallGemmArgs &ga0, const BallScatterArgs &ca, hipStream_t s)
{
    {
        const int64_t n = (int64_t)sa.P * sa.Vo_pad;
        const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16);
        hipLaunchKernelGGL(k_ball_sym, dim3(std::max(nb, 1u)), dim3(256), 0, s, sa);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    BallGemmArgs ga = ga0;
    const int nt = ball_col_tiles(ga.col_off, ga.tile_lo);
    if (nt > 0) {
        const int tm = ball_tile_m(ga.P);
        if (tm == 128)
            hipLaunchKernelGGL(k_ball_gemm<128>, dim3(nt, (ga.P + 127) / 128, ga.S), dim3(kBallThreads), 0, s, ga);
        else
            hipLaunchKernelGGL(k_ball_gemm<64>, dim3(nt, (ga.P + 63) / 64, ga.S), dim3(kBallThreads), 0, s, ga);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // per volume when the column sums fit in LDS and the volumes give at least two workgroups per
    // CU (1024 volumes: 1.62 against 1.71 ms for the transform; 256 volumes: 0.44 against 0.42 ms)
    if (ca.ncol <= kBallScatterLdsCols && ca.P >= 512) {
        hipLaunchKernelGGL(k_ball_scatter_vol, dim3(ca.P), dim3(256), sizeof(float) * (size_t)ca.ncol, s, ca);
        return hipGetLastError();
    }
    const int64_t n = (int64_t)ca.P * ca.n_entries;
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(k_ball_scatter, dim3(std::max(nb, 1u)), dim3(256), 0, s, ca);
    return hipGetLastError();
}

}  // namespace matcha
