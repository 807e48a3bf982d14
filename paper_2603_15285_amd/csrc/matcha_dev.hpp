// matcha_dev.hpp -- device-side types and helpers shared by the libmatcha kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace matcha {

constexpr int kWave = 64;
constexpr int kMaxL = 64;
constexpr int kMaxLevels = 16;
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

// Wedge pair (m, n), 0 <= |n| <= m, at q = m*m + m + n.  lbh2 = log2 sqrt(binom(2m, m+n)),
// the magnitude of d^m_mn's single explicit-sum term without the trigonometric powers.
struct PairInfo {
    int m, n;
    double lbh2;
};

// Rows of the wedge layout: row l holds the (l+1)^2 pairs with m <= l, starting at
// l(l+1)(2l+1)/6 pairs (each pair = one float4 of C or of the coefficient table).
__host__ __device__ inline int64_t wedge_row(int l) { return (int64_t)l * (l + 1) * (2 * l + 1) / 6; }

__device__ inline int isqrt_dev(int q)
{
    int m = (int)sqrtf((float)q);
    while (m * m > q) --m;
    while ((m + 1) * (m + 1) <= q) ++m;
    return m;
}

// Per-rotation constants of the Wigner-d evaluation at polar angle b, formed in FP64
// from the FP64 angle and rounded once.  The half-angle sine and cosine are clamped
// at 1e-15 so that the edge seeds never meet 0 * inf at the chart poles.
struct BetaConst {
    float cb, sb;     // cos b, sin b
    double cbd, sbd;  // cos b, sin b in FP64 (for the FP64 recurrence)
    float ct, tn;     // cot(b/2), tan(b/2)
    float ct2, tn2;   // cot^2(b/2), tan^2(b/2)
    double lc2, ls2;  // log2 cos(b/2), log2 sin(b/2)
    double ctd, tnd;  // cot(b/2), tan(b/2) in FP64
};

__device__ __forceinline__ BetaConst beta_const(double b)
{
    BetaConst k;
    double s, c;
    sincos(0.5 * b, &s, &c);
    k.cbd = (c - s) * (c + s);  // cos b and sin b by the double-angle identities
    k.sbd = 2.0 * s * c;
    c = fmax(fabs(c), 1e-15);
    s = fmax(fabs(s), 1e-15);
    k.cb = (float)k.cbd;
    k.sb = (float)k.sbd;
    k.ct = (float)(c / s);
    k.tn = (float)(s / c);
    k.ct2 = (float)((c * c) / (s * s));
    k.tn2 = (float)((s * s) / (c * c));
    k.lc2 = log2(c);
    k.ls2 = log2(s);
    k.ctd = c / s;
    k.tnd = s / c;
    return k;
}

// d^m_mn(b) and its first two b-derivatives on the edge l = m of the wedge pair:
//   d = (-1)^k sqrt(binom(2m, p)) cos^p(b/2) sin^k(b/2),  p = m + n, k = m - n,
//   d'/d = (k cot(b/2) - p tan(b/2)) / 2,  d''/d = (d'/d)^2 - (k csc^2(b/2) + p sec^2(b/2)) / 4.
// With csc^2 = 1 + cot^2 and sec^2 = 1 + tan^2 the second ratio is
//   d''/d = (k (k - 1) cot^2(b/2) + p (p - 1) tan^2(b/2) - 2 k p - k - p) / 4,
// a sum of terms of one sign that does not cancel near the poles the way the first form does
// (for k = 1 its two terms are each about csc^2(b/2) / 4).
// The magnitude is formed as 2^x with x in FP64 and split into an exact power of two
// and a fraction, so the seed keeps FP32 relative accuracy however small it is.
__device__ inline void edge_seed(int m, int n, double lbh2, const BetaConst &k, float &d0, float &d1, float &d2)
{
    const int p = m + n, kk = m - n;
    const double x = lbh2 + (double)p * k.lc2 + (double)kk * k.ls2;
    const double fl = floor(x);
    float e = exp2f((float)(x - fl));
    e = ldexpf(e, (int)fmax(fl, -1000.0));
    if (kk & 1) e = -e;
    const float h1 = 0.5f * ((float)kk * k.ct - (float)p * k.tn);
    const float h2 = 0.25f * ((float)(kk * (kk - 1)) * k.ct2 + (float)(p * (p - 1)) * k.tn2 - (float)(2 * kk * p + kk + p));
    d0 = e;
    d1 = e * h1;
    d2 = e * h2;
}

// The same edge values in FP64 (for the FP64 recurrence above the threshold degree).
__device__ inline void edge_seed_d(int m, int n, double lbh2, const BetaConst &k, double &d0, double &d1, double &d2)
{
    const int p = m + n, kk = m - n;
    const double x = lbh2 + (double)p * k.lc2 + (double)kk * k.ls2;
    double e = exp2(x);
    if (kk & 1) e = -e;
    const double ct = k.ctd, tn = k.tnd;
    const double h1 = 0.5 * ((double)kk * ct - (double)p * tn);
    const double h2 = 0.25 * ((double)(kk * (kk - 1)) * (ct * ct) + (double)(p * (p - 1)) * (tn * tn) - (double)(2 * kk * p + kk + p));
    d0 = e;
    d1 = e * h1;
    d2 = e * h2;
}

// Orders the LDS accesses of one wave's lanes.  A wave's LDS operations complete in issue
// order, so only the compiler must be kept from moving accesses across this point; waves of
// the same workgroup do not wait for each other.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline float bcast(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }

__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Order-preserving map of a float onto uint32 (larger float -> larger integer).
__device__ inline uint32_t ordered_bits(float v)
{
    uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float unordered_bits(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

}  // namespace matcha
