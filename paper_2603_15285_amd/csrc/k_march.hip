// k_march.hip -- objective, gradient and Hessian of the band-limited correlation and the
// frequency-marched Newton refinement (Sec. 2.2, 2.4, Alg. 1).
//
// Work decomposition.  A wave owns NC candidates of one particle.  Its 64 lanes walk the
// "wedge" pairs (m, n), 0 <= |n| <= m <= L, in tiles of 64; each lane runs the Wigner-d
// three-term recurrence in l for its pair, with its first and second b-derivatives,
// for all NC candidates at once (the recurrence coefficients and the C loads are shared
// by the candidates).  For real inputs C^l_{-m,-n} = (-1)^{m-n} conj(C^l_mn), and
// d_mn = (-1)^{m-n} d_nm = d_{-n,-m}, so one recurrence step serves four terms of the
// full sum: the pair, its partner (n, m) or (-n, -m), and their Hermitian mirrors.
//
// Per lane and candidate the l-sums U_s = sum_l C^l P_l D^l_s (s = value, d/db, d2/db2)
// are accumulated for the pair and its partner; the e^{i(ma+nc)} phase, constant in l,
// is applied once per pair afterwards, together with the m and n weights of the
// a / c derivatives.  D^l = d^l / P_l is the recurrence normalised so that its
// three-term relation has unit coefficient on D^{l-2} (P_l is tabulated per pair).
#include <algorithm>

#include "matcha_launch.hpp"

#include <type_traits>

namespace matcha {


// Phase tables of the wave's candidates.
template <int NC>
struct __align__(16) WaveScratch {
    struct {
        float2 ea[NC][kMaxL + 1];      // e^{i k a_c}, k = 0 .. L
        float2 eg[NC][2 * kMaxL + 1];  // e^{i k c_c} at kMaxL + k, k = -L .. L
    } ph;
};

template <int NC>
struct WaveState {
    BetaConst bc[NC];
    double th[NC][3];
    float tot[NC][10];
    uint32_t st[NC];
    int frozen[NC];
    int moved[NC];  // a Newton step moved the candidate since the last prepare_step
    float fprev[NC];
};

// e^{i k a_c} and e^{i k c_c} of the wave's NC candidates, k = 0 .. L, one (candidate, k) per
// lane.  Inlined into its callers so that the tables are addressed as LDS, never through generic
// pointers.
template <int NC>
__device__ __forceinline__ void fill_phases(const WaveState<NC> &st, WaveScratch<NC> &ws, int L, int lane)
{
    for (int i = lane; i < NC * (L + 1); i += kWave) {
        const int c = i / (L + 1), k = i - c * (L + 1);
        // k a reduced to [-pi, pi] in FP64 (exact enough for |k a| < 1e6), then sin / cos in FP32
        const double xa = (double)k * st.th[c][0], xc = (double)k * st.th[c][2];
        const double ta = fma(-kTwoPi, rint(xa * (1.0 / kTwoPi)), xa), tc = fma(-kTwoPi, rint(xc * (1.0 / kTwoPi)), xc);
        float sa, ca, sc, cc;
        sincosf((float)ta, &sa, &ca);
        sincosf((float)tc, &sc, &cc);
        ws.ph.ea[c][k] = make_float2(ca, sa);
        ws.ph.eg[c][kMaxL + k] = make_float2(cc, sc);
        ws.ph.eg[c][kMaxL - k] = make_float2(cc, -sc);
    }
}

// One recurrence row for NC candidates in arithmetic T (float, or double above the FP64
// threshold).  On entry X = D^{l-1}, Y = D^{l-2} (X1, Y1: first b-derivative; X2, Y2: half the
// second b-derivative); on exit Y holds row l.  (A, AC) are the row's recurrence coefficients,
// (PW, PWT) = (tb.z, tb.w) its weights, cc = (C^l_pair, C^l_partner).  U[c] accumulates
// sum_l C^l PW_l D^l for the pair (0, 1) and C^l PWT_l D^l for the partner (2, 3), then the same
// for D' (4..7) and D''/2 (8..11).  With u = A cos b - AC, v = A sin b, h = A cos b / 2:
//   D'^l = u D'^{l-1} - v D^{l-1} - D'^{l-2},  (D''/2)^l = u (D''/2)^{l-1} - v D'^{l-1} - h D^{l-1} - (D''/2)^{l-2}.
// SEED: rows where pairs of the tile start; lanes with seed set take the edge values (S0, S1, S2)
// instead.  Lanes whose pair starts later hold a zero state, which the step keeps at zero.
// FIRST = 1: the tile's first row, where X and Y are zero (neither is read) and U is set rather
// than accumulated; FIRST = 2: its second row, where Y is zero (not read).
template <int NC, bool DERIV, bool SEED, typename T, int FIRST = 0>
__device__ __forceinline__ void row_step(const T A, const T AC, const float4 tb, const float4 cc, const bool seed,
                                         const T (&S0)[NC], const T (&S1)[NC], const T (&S2)[NC], const T *cbv,
                                         const T *sbv, const T *chv, T (&X)[NC], T (&Y)[NC], T (&X1)[NC],
                                         T (&Y1)[NC], T (&X2)[NC], T (&Y2)[NC], float (&U)[NC][DERIV ? 12 : 4])
{
    // the l-sums are FP32 in both arithmetics (an FP64 row's values are rounded once before them)
    const float s0r = cc.x * tb.z, s0i = cc.y * tb.z, s1r = cc.z * tb.w, s1i = cc.w * tb.w;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const T u = fma(A, cbv[c], -AC);
        T dn = FIRST == 1 ? (T)0 : FIRST == 2 ? u * X[c] : fma(u, X[c], -Y[c]);
        if (SEED) dn = seed ? S0[c] : dn;
        const float df = (float)dn;
        if (FIRST == 1) {
            U[c][0] = s0r * df;
            U[c][1] = s0i * df;
            U[c][2] = s1r * df;
            U[c][3] = s1i * df;
        } else {
            U[c][0] = fmaf(s0r, df, U[c][0]);
            U[c][1] = fmaf(s0i, df, U[c][1]);
            U[c][2] = fmaf(s1r, df, U[c][2]);
            U[c][3] = fmaf(s1i, df, U[c][3]);
        }
        if (DERIV) {
            T d1n, d2n;
            if (FIRST == 1) {
                d1n = d2n = (T)0;
            } else {
                const T v = A * sbv[c];
                const T h = A * chv[c];
                d1n = FIRST == 2 ? fma(u, X1[c], -v * X[c]) : fma(u, X1[c], fma(-v, X[c], -Y1[c]));
                d2n = FIRST == 2 ? fma(u, X2[c], fma(-v, X1[c], -h * X[c])) : fma(u, X2[c], fma(-v, X1[c], fma(-h, X[c], -Y2[c])));
            }
            if (SEED) {
                d1n = seed ? S1[c] : d1n;
                d2n = seed ? S2[c] : d2n;
            }
            Y1[c] = d1n;
            Y2[c] = d2n;
            const float d1f = (float)d1n, d2f = (float)d2n;
            if (FIRST == 1) {
                U[c][4] = s0r * d1f;
                U[c][5] = s0i * d1f;
                U[c][6] = s1r * d1f;
                U[c][7] = s1i * d1f;
                U[c][8] = s0r * d2f;
                U[c][9] = s0i * d2f;
                U[c][10] = s1r * d2f;
                U[c][11] = s1i * d2f;
            } else {
                U[c][4] = fmaf(s0r, d1f, U[c][4]);
                U[c][5] = fmaf(s0i, d1f, U[c][5]);
                U[c][6] = fmaf(s1r, d1f, U[c][6]);
                U[c][7] = fmaf(s1i, d1f, U[c][7]);
                U[c][8] = fmaf(s0r, d2f, U[c][8]);
                U[c][9] = fmaf(s0i, d2f, U[c][9]);
                U[c][10] = fmaf(s1r, d2f, U[c][10]);
                U[c][11] = fmaf(s1i, d2f, U[c][11]);
            }
        }
        Y[c] = dn;
    }
}

__device__ __forceinline__ float4 ld_row(const float4 *base, int row, uint32_t lane_bytes)
{
    const char *p = reinterpret_cast<const char *>(base + row);
    return *reinterpret_cast<const float4 *>(p + lane_bytes);
}

__device__ __forceinline__ double2 ld_row(const double2 *base, int row, uint32_t lane_bytes)
{
    const char *p = reinterpret_cast<const char *>(base + row);
    return *reinterpret_cast<const double2 *>(p + lane_bytes);
}

// Recurrence coefficients of a row in arithmetic T: the FP32 table, or the FP64 table for the
// double recurrence.
template <typename T>
struct Coef;
template <>
struct Coef<float> {
    __device__ static void get(const float4 tb, const double2 *, int, uint32_t, float &A, float &AC)
    {
        A = tb.x;
        AC = tb.y;
    }
};
template <>
struct Coef<double> {
    __device__ static void get(const float4, const double2 *t64, int row, uint32_t lb, double &A, double &AC)
    {
        const double2 c = ld_row(t64, row, lb);  // one 16-byte (A, AC) per pair, like tab
        A = c.x;
        AC = c.y;
    }
};

// f(integral_constant<int, B>), ..., f(integral_constant<int, E - 1>), unrolled at compile time.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Rows in flight in the value-only evaluation.  Its row costs a quarter of a derivative row's
// arithmetic, so two rows in flight (the derivative evaluation's depth) leave it waiting on the
// loads; the registers that the derivative state would hold carry the deeper prefetch.
constexpr int kValueDepth = 8;

template <typename T>
__device__ inline void seed_T(int m, int n, double lbh2, const BetaConst &k, T &d0, T &d1, T &d2);
template <>
__device__ inline void seed_T<float>(int m, int n, double lbh2, const BetaConst &k, float &d0, float &d1, float &d2)
{
    edge_seed(m, n, lbh2, k, d0, d1, d2);
}
template <>
__device__ inline void seed_T<double>(int m, int n, double lbh2, const BetaConst &k, double &d0, double &d1, double &d2)
{
    edge_seed_d(m, n, lbh2, k, d0, d1, d2);
}

template <typename T>
__device__ inline T bcastT(T x);
template <>
__device__ inline float bcastT<float>(float x) { return bcast(x); }
template <>
__device__ inline double bcastT<double>(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll)), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over all wedge pairs of one level for the NC candidates c0 .. c0+NC-1 of a wave that owns
// NCW.  acc[c0+c][0..9] receive the (positive-sign, undoubled) sums described at the top of the
// file, the b-b sum (7) from D''/2, i.e. halved; with DERIV == false only acc[.][0] (the value)
// is formed.  T is the arithmetic of the recurrence; the l-sums are FP32.
template <int NC, int NCW, bool DERIV, typename T>
__device__ void eval_level(const float4 *__restrict__ Cp, const float4 *__restrict__ tab,
                           const double2 *__restrict__ tab64, const PairInfo *__restrict__ pinfo, int L,
                           const BetaConst *bc, const WaveScratch<NCW> &ws, float (&acc)[NCW][10], int c0, int lane)
{
    constexpr int NU = DERIV ? 12 : 4;
    T cbv[NC], sbv[NC], chv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        cbv[c] = bcastT<T>((T)bc[c0 + c].cbd);
        sbv[c] = bcastT<T>((T)bc[c0 + c].sbd);
        chv[c] = (T)0.5 * cbv[c];
#pragma unroll
        for (int v = 0; v < 10; ++v) acc[c0 + c][v] = 0.f;
    }
    const int npairs = (L + 1) * (L + 1);
    const int ntiles = (npairs + kWave - 1) / kWave;
    const int rowL = (int)wedge_row(L);
    // each tile loads the next tile's pairs while it runs
    PairInfo pn = pinfo[min(lane, npairs - 1)];
    // Derivative evaluation: a tile's first two rows are loaded before the previous tile's phase
    // and weighting work, so that work covers their latency (the recurrence state is dead by then,
    // so the loads take no extra registers).  ml: the tile's smallest m; lbx: the lane's offset.
    float4 tb0, cc0, tb1, cc1;
    T A0, AC0, A1, AC1;
    int row_next = 0;
    auto first_rows = [&](int ml, uint32_t lbx) {
        int rw = (int)wedge_row(ml);
        tb0 = ld_row(tab, rw, lbx);
        cc0 = ld_row(Cp, rw, lbx);
        Coef<T>::get(tb0, tab64, rw, lbx, A0, AC0);
        rw += (ml + 1) * (ml + 1);
        const int rr = min(rw, rowL);
        tb1 = ld_row(tab, rr, lbx);
        cc1 = ld_row(Cp, rr, lbx);
        Coef<T>::get(tb1, tab64, rr, lbx, A1, AC1);
        row_next = rw + (ml + 2) * (ml + 2);
    };
    // Value-only evaluation: likewise, a tile's first kValueDepth rows are loaded before the previous
    // tile's phase work.
    float4 tbk[kValueDepth], cck[kValueDepth];
    T Ak[kValueDepth], ACk[kValueDepth];
    auto first_rows_v = [&](int ml, uint32_t lbx) {
        int rw = (int)wedge_row(ml);
        static_for<0, kValueDepth>([&](auto jc) {
            constexpr int J = decltype(jc)::value;
            const int r = min(rw, rowL);
            tbk[J] = ld_row(tab, r, lbx);
            cck[J] = ld_row(Cp, r, lbx);
            Coef<T>::get(tbk[J], tab64, r, lbx, Ak[J], ACk[J]);
            rw += (ml + J + 1) * (ml + J + 1);
        });
        row_next = rw;
    };
    if constexpr (DERIV)
        first_rows(__builtin_amdgcn_readfirstlane(pn.m), (uint32_t)min(lane, npairs - 1) * 16u);
    else
        first_rows_v(__builtin_amdgcn_readfirstlane(pn.m), (uint32_t)min(lane, npairs - 1) * 16u);
    for (int t = 0; t < ntiles; ++t) {
        const int q0 = t * kWave;
        const int q = q0 + lane;
        const bool valid = q < npairs;
        const uint32_t lb = (uint32_t)(valid ? q : npairs - 1) * 16u;
        const PairInfo pi = pn;
        pn = pinfo[min(q + kWave, npairs - 1)];
        const int m = pi.m, n = pi.n;
        // lane 0 holds the tile's smallest m, the last valid lane its largest
        const int mlo = __builtin_amdgcn_readfirstlane(m);
        const int mhi = __builtin_amdgcn_readlane(m, min(npairs - 1 - q0, kWave - 1));

        // Rows mlo .. L, two per trip: the state ping-pongs between (D, Dm), and the loads of the
        // next two rows are in flight meanwhile.  Every lane loads at its own pair's offset in
        // every row, also before its pair starts (the offset then falls in a later row of the
        // same array) and past row L (row L is re-read, never used), so no load needs a branch.
        int l = mlo;
        int row = (int)wedge_row(mlo);
        int r1;
        // the tile's first rows (two, or kValueDepth for the value only) are in flight since the
        // previous tile
        row = row_next;

        // edge values of every lane's pair, computed once per tile without divergence
        T sd0[NC], sd1[NC], sd2[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            seed_T<T>(m, n, pi.lbh2, bc[c0 + c], sd0[c], sd1[c], sd2[c]);
            sd2[c] *= (T)0.5;
        }
        // the state before row mlo is zero: the first two rows take it as such (row_step FIRST)
        T D[NC], Dm[NC], D1[NC], D1m[NC], D2[NC], D2m[NC];
        float U[NC][NU];
#define MARCH_ROW0(SEEDROW, FST)                                                                         \
    row_step<NC, DERIV, SEEDROW, T, FST>(A0, AC0, tb0, cc0, m == l, sd0, sd1, sd2, cbv, sbv, chv, D, Dm, D1, D1m, D2, \
                                         D2m, U)
#define MARCH_ROW1(SEEDROW, FST)                                                                             \
    row_step<NC, DERIV, SEEDROW, T, FST>(A1, AC1, tb1, cc1, m == l + 1, sd0, sd1, sd2, cbv, sbv, chv, Dm, D, D1m, D1, \
                                         D2m, D2, U)
#define MARCH_LOAD0()                                                                                    \
    do {                                                                                                 \
        __builtin_amdgcn_sched_barrier(0);                                                               \
        const int r0 = min(row, rowL);                                                                   \
        tb0 = ld_row(tab, r0, lb);                                                                       \
        cc0 = ld_row(Cp, r0, lb);                                                                        \
        Coef<T>::get(tb0, tab64, r0, lb, A0, AC0);                                                       \
        row += (l + 3) * (l + 3);                                                                        \
        __builtin_amdgcn_sched_barrier(0);                                                               \
    } while (0)
#define MARCH_LOAD1()                                                                                    \
    do {                                                                                                 \
        __builtin_amdgcn_sched_barrier(0);                                                               \
        r1 = min(row, rowL);                                                                             \
        tb1 = ld_row(tab, r1, lb);                                                                       \
        cc1 = ld_row(Cp, r1, lb);                                                                        \
        Coef<T>::get(tb1, tab64, r1, lb, A1, AC1);                                                       \
        row += (l + 4) * (l + 4);                                                                        \
        __builtin_amdgcn_sched_barrier(0);                                                               \
    } while (0)
        if constexpr (DERIV) {
            // rows where pairs of the tile start (mlo .. mhi, rounded up to an even count, at most L)
            const int lseed = min(mhi + ((mhi - mlo) & 1 ? 0 : 1), L);
            MARCH_ROW0(true, 1);
            MARCH_LOAD0();
            if (l < L) MARCH_ROW1(true, 2);
            MARCH_LOAD1();
            for (l += 2; l <= lseed; l += 2) {
                MARCH_ROW0(true, 0);
                MARCH_LOAD0();
                if (l < L) MARCH_ROW1(true, 0);
                MARCH_LOAD1();
            }
            // rows where every pair of the tile has started
            for (; l + 1 <= L; l += 2) {
                MARCH_ROW0(false, 0);
                MARCH_LOAD0();
                MARCH_ROW1(false, 0);
                MARCH_LOAD1();
            }
            if (l <= L) MARCH_ROW0(false, 0);
        } else {
            // Trips of kValueDepth rows l .. l + depth - 1: row l + J comes from set J, which then
            // takes row l + J + depth (clamped to row L, never used past it).  The state alternates
            // between D and Dm with the row's parity (the depth is even).  GUARD: rows past L are
            // skipped (the loads are not, so none sits behind a branch).
            auto trip = [&](auto seed_c, auto first_c, auto guard_c) {
                constexpr bool SEEDR = decltype(seed_c)::value;
                constexpr bool FIRSTT = decltype(first_c)::value;
                constexpr bool GUARD = decltype(guard_c)::value;
                static_for<0, kValueDepth>([&](auto jc) {
                    constexpr int J = decltype(jc)::value;
                    constexpr int FST = FIRSTT ? (J == 0 ? 1 : J == 1 ? 2 : 0) : 0;
                    const int lr = l + J;
                    if (!GUARD || lr <= L) {
                        if constexpr (J % 2 == 0)
                            row_step<NC, false, SEEDR, T, FST>(Ak[J], ACk[J], tbk[J], cck[J], m == lr, sd0, sd1, sd2,
                                                               cbv, sbv, chv, D, Dm, D1, D1m, D2, D2m, U);
                        else
                            row_step<NC, false, SEEDR, T, FST>(Ak[J], ACk[J], tbk[J], cck[J], m == lr, sd0, sd1, sd2,
                                                               cbv, sbv, chv, Dm, D, D1m, D1, D2m, D2, U);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    const int r = min(row, rowL);
                    tbk[J] = ld_row(tab, r, lb);
                    cck[J] = ld_row(Cp, r, lb);
                    Coef<T>::get(tbk[J], tab64, r, lb, Ak[J], ACk[J]);
                    row += (lr + kValueDepth + 1) * (lr + kValueDepth + 1);
                    __builtin_amdgcn_sched_barrier(0);
                });
                l += kValueDepth;
            };
            using yes = std::true_type;
            using no = std::false_type;
            // the first trip holds row mlo (FIRST) and the rows where pairs start up to mhi
            trip(yes{}, yes{}, yes{});
            while (l <= mhi) trip(yes{}, no{}, yes{});
            // rows where every pair of the tile has started
            while (l + kValueDepth - 1 <= L) trip(no{}, no{}, no{});
            if (l <= L) trip(no{}, no{}, yes{});
        }
#undef MARCH_ROW0
#undef MARCH_ROW1
#undef MARCH_LOAD0
#undef MARCH_LOAD1
        if (t + 1 < ntiles) {  // the next tile's first rows, before this tile's phase work
            if constexpr (DERIV)
                first_rows(__builtin_amdgcn_readfirstlane(pn.m), (uint32_t)min(q + kWave, npairs - 1) * 16u);
            else
                first_rows_v(__builtin_amdgcn_readfirstlane(pn.m), (uint32_t)min(q + kWave, npairs - 1) * 16u);
        }
        if (!valid) continue;
        // phases and the m, n weights of the a / c derivatives
        const int an = n >= 0 ? n : -n, b2i = n >= 0 ? m : -m;
        const float a1 = (float)m, b1 = (float)n;
        const float a2 = (float)an, b2 = (float)b2i;
        const float a11 = a1 * a1, a22 = a2 * a2, b11 = b1 * b1, b22 = b2 * b2, ab1 = a1 * b1, ab2 = a2 * b2;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int cw = c0 + c;
            const float2 am = ws.ph.ea[cw][m], aN = ws.ph.ea[cw][an];
            const float2 gN = ws.ph.eg[cw][kMaxL + n], gm = ws.ph.eg[cw][kMaxL + b2i];
            const float2 p1 = cmul(am, gN);  // e^{i(m a + n c)}
            const float2 p2 = cmul(aN, gm);  // e^{i(a2 a + b2 c)}
            float u[NU];
#pragma unroll
            for (int v = 0; v < NU; ++v) u[v] = (float)U[c][v];
            const float R0 = p1.x * u[0] - p1.y * u[1];
            const float T0 = p2.x * u[2] - p2.y * u[3];
            acc[cw][0] += R0 + T0;
            if (DERIV) {
                const float I0 = p1.x * u[1] + p1.y * u[0];
                const float J0 = p2.x * u[3] + p2.y * u[2];
                const float R1 = p1.x * u[4] - p1.y * u[5];
                const float I1 = p1.x * u[5] + p1.y * u[4];
                const float T1 = p2.x * u[6] - p2.y * u[7];
                const float J1 = p2.x * u[7] + p2.y * u[6];
                const float R2 = p1.x * u[8] - p1.y * u[9];  // half of the D'' terms (D''/2 is carried)
                const float T2 = p2.x * u[10] - p2.y * u[11];
                acc[cw][1] = fmaf(a1, I0, fmaf(a2, J0, acc[cw][1]));
                acc[cw][2] += R1 + T1;
                acc[cw][3] = fmaf(b1, I0, fmaf(b2, J0, acc[cw][3]));
                acc[cw][4] = fmaf(a11, R0, fmaf(a22, T0, acc[cw][4]));
                acc[cw][5] = fmaf(a1, I1, fmaf(a2, J1, acc[cw][5]));
                acc[cw][6] = fmaf(ab1, R0, fmaf(ab2, T0, acc[cw][6]));
                acc[cw][7] += R2 + T2;
                acc[cw][8] = fmaf(b1, I1, fmaf(b2, J1, acc[cw][8]));
                acc[cw][9] = fmaf(b11, R0, fmaf(b22, T0, acc[cw][9]));
            }
        }
    }
}

// A whole level for the wave's NC candidates: FP32 recurrence at or below the FP64 threshold,
// FP64 recurrence (up to four candidates per pass, to bound registers) above it.  F64 = false
// builds the FP32 recurrence only, for launches with no level above the threshold (the FP64
// path's registers would otherwise bound the whole kernel).
template <int NC, bool DERIV, bool F64>
__device__ void eval_level_any(const float4 *Cp, const float4 *tab, const double2 *tab64, const PairInfo *pinfo,
                               int L, int fp64_above, const BetaConst *bc, const WaveScratch<NC> &ws,
                               float (&acc)[NC][10], int lane)
{
    if (!F64 || L <= fp64_above || tab64 == nullptr) {
        eval_level<NC, NC, DERIV, float>(Cp, tab, tab64, pinfo, L, bc, ws, acc, 0, lane);
    } else {
        constexpr int H = NC < 4 ? NC : 4;
#pragma unroll
        for (int c0 = 0; c0 < NC; c0 += H) eval_level<H, NC, DERIV, double>(Cp, tab, tab64, pinfo, L, bc, ws, acc, c0, lane);
    }
}

// Sum of v over the 16 lanes of each lane row (DPP row mirror, half mirror and two quad
// permutations); every lane of a row ends with its row's sum.
__device__ __forceinline__ float row_sum16(float v)
{
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xf, 0xf, false));  // lane i <-> 15 - i
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xf, 0xf, false));  // i <-> 7 - i in halves
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4e, 0xf, 0xf, false));   // i <-> i ^ 2
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xb1, 0xf, 0xf, false));   // i <-> i ^ 1
    return v;
}

// Lane-sums of the wave's NC x NV accumulators, on the VALU: v_permlane32_swap folds lanes
// i and i + 32 of two values at once (the first value's sums land in lanes 0..31, the second's
// in 32..63), v_permlane16_swap folds lanes i and i + 16 of two such registers, so that each
// register then holds four values' partial sums, one per 16-lane row (rows 0..3: values 0, 2,
// 1, 3 of its group of four), and the rows are summed with DPP.  Total v ends in st.tot.
template <int NC, int NV>
__device__ __forceinline__ void wave_reduce(float (&acc)[NC][10], WaveState<NC> &st, int lane)
{
    constexpr int NT = NC * NV, NG = (NT + 3) / 4;
    float z[NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        float y[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i0 = 4 * k + 2 * j, i1 = i0 + 1;
            const float x0 = i0 < NT ? acc[i0 / NV][i0 % NV] : 0.f;
            const float x1 = i1 < NT ? acc[i1 / NV][i1 % NV] : 0.f;
            const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(x0), __float_as_uint(x1), false, false);
            y[j] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
        }
        const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(y[0]), __float_as_uint(y[1]), false, false);
        z[k] = row_sum16(__uint_as_float(s[0]) + __uint_as_float(s[1]));
    }
    if ((lane & 15) == 0) {
        const int r = lane >> 4, e = ((r & 1) << 1) | (r >> 1);
        float *tot = &st.tot[0][0];
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int i = 4 * k + e;
            if (i < NT) tot[(i / NV) * 10 + i % NV] = z[k];
        }
    }
    wave_sync();
}

// x mod 2 pi in [0, 2 pi).  For |x| < 4 pi the remainder is x -+ 2 pi, which FP64 forms exactly
// (Sterbenz), so fmod is called only beyond that.
__device__ inline double wrap2pi(double x)
{
    if (!(fabs(x) < 2.0 * kTwoPi))
        x = fmod(x, kTwoPi);
    else if (x >= kTwoPi)
        x -= kTwoPi;
    else if (x <= -kTwoPi)
        x += kTwoPi;
    return x < 0.0 ? x + kTwoPi : x;
}

// Newton step theta <- theta - H^{-1} grad in FP64 with the explicit 3x3 inverse; the
// readings for indefinite / singular H, clipping and chart wrapping are those of the
// interface documentation.  e = F, Fa, Fb, Fc, Faa, Fab, Fac, Fbb, Fbc, Fcc.
// theta += d (largest component clipped to max_step when positive), b reflected into [0, pi] with
// (a + pi, c + pi), a and c wrapped into [0, 2 pi).
__device__ void apply_step(double d0, double d1, double d2, double max_step, double *th, double *step_inf)
{
    double mx = fmax(fabs(d0), fmax(fabs(d1), fabs(d2)));
    if (max_step > 0.0 && mx > max_step) {
        const double s = max_step / mx;
        d0 *= s;
        d1 *= s;
        d2 *= s;
        mx = max_step;
    }
    *step_inf = mx;
    double a = th[0] + d0, b = th[1] + d1, c = th[2] + d2;
    b = wrap2pi(b);
    if (b > kPi) {
        b = kTwoPi - b;
        a += kPi;
        c += kPi;
    }
    th[0] = wrap2pi(a);
    th[1] = b;
    th[2] = wrap2pi(c);
}

// Gradient ascent step, the first-order comparator: theta += t grad with
// t = rate / ((1 + L)^2 |F|) (the Hessian's Bernstein bound as smoothness constant).
__device__ uint32_t gradient_step(const double *e, double rate, int L, double max_step, double *th,
                                  double *step_inf)
{
    for (int i = 0; i < 4; ++i)
        if (!isfinite(e[i])) {
            *step_inf = 0.0;
            return 1u;
        }
    const double t = rate / ((1.0 + L) * (1.0 + L) * fmax(fabs(e[0]), 1e-300));
    apply_step(t * e[1], t * e[2], t * e[3], max_step, th, step_inf);
    return 0u;
}

__device__ uint32_t newton_step(const double *e, double max_step, double *th, double *step_inf)
{
    for (int i = 0; i < 10; ++i)
        if (!isfinite(e[i])) {
            *step_inf = 0.0;
            return 1u;
        }
    const double h00 = e[4], h01 = e[5], h02 = e[6], h11 = e[7], h12 = e[8], h22 = e[9];
    const double c00 = h11 * h22 - h12 * h12, c01 = h02 * h12 - h01 * h22, c02 = h01 * h12 - h02 * h11;
    const double c11 = h00 * h22 - h02 * h02, c12 = h02 * h01 - h00 * h12, c22 = h00 * h11 - h01 * h01;
    const double det = h00 * c00 + h01 * c01 + h02 * c02;
    double hmax = fmax(fmax(fabs(h00), fabs(h01)), fmax(fmax(fabs(h02), fabs(h11)), fmax(fabs(h12), fabs(h22))));
    uint32_t st = 0;
    if (!(-h00 > 0.0 && c22 > 0.0 && -det > 0.0)) st |= 2u;
    if (!(fabs(det) > 1e-30 * hmax * hmax * hmax)) {
        *step_inf = 0.0;
        return st | 4u;
    }
    const double g0 = e[1], g1 = e[2], g2 = e[3];
    const double d0 = -(c00 * g0 + c01 * g1 + c02 * g2) / det;
    const double d1 = -(c01 * g0 + c11 * g1 + c12 * g2) / det;
    const double d2 = -(c02 * g0 + c12 * g1 + c22 * g2) / det;
    apply_step(d0, d1, d2, max_step, th, step_inf);
    return st;
}

// Per-rotation constants and phase tables of the wave's candidates.  With POLE, a candidate that
// a Newton step has moved is flagged (status bit 8) when its new b has sin b < 1e-3.  Inlined into
// the kernels: the wave state and scratch are then addressed as LDS (a generic pointer formed as
// base - offset can leave the shared aperture when the base sits at LDS 0).
template <int NC, bool POLE>
__device__ __forceinline__ void prepare_step(WaveState<NC> &st, WaveScratch<NC> &ws, int L, int lane)
{
    if (lane < NC) {
        const BetaConst k = beta_const(st.th[lane][1]);
        st.bc[lane] = k;
        if (POLE && st.moved[lane]) {
            if (k.sbd < 1e-3) st.st[lane] |= 8u;
            st.moved[lane] = 0;
        }
    }
    fill_phases<NC>(st, ws, L, lane);
    wave_sync();
}

// One workgroup per particle (the hardware starts workgroups in index order as slots free up), or,
// with a.queue, a persistent grid that fills the chip once: each workgroup takes the next particle
// index from the counter until the batch is done (every workgroup then sees an index >= P and
// leaves).  Either way particle b of the order is processed the same way.
template <int NC, bool F64>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) k_march(MarchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int next_b;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int G = blockDim.x / kWave;
    WaveScratch<NC> &ws = reinterpret_cast<WaveScratch<NC> *>(smem)[wave];
    WaveState<NC> &st = reinterpret_cast<WaveState<NC> *>(smem + G * sizeof(WaveScratch<NC>))[wave];
    float *fin = reinterpret_cast<float *>(smem + G * (sizeof(WaveScratch<NC>) + sizeof(WaveState<NC>)));
    uint32_t *fst = reinterpret_cast<uint32_t *>(fin + G * NC);

    int b = (int)blockIdx.x;
    if (a.queue) {
        if (threadIdx.x == 0) next_b = atomicAdd(a.queue, 1);
        __syncthreads();
        b = next_b;
    }
    while (b < a.P) {
    const int p = a.order ? a.order[b] : b;
    const int Lp = a.Lp[p];
    const float4 *Cp = a.C + a.C_off[p] / 2;
    const float4 *Cf = (a.C_fin ? a.C_fin : a.C) + a.C_off[p] / 2;  // the final level's coefficients
    if (lane < NC) {
        const int k = wave * NC + lane;
        float4 c0 = k < a.Kc ? a.cand[(int64_t)p * a.Kc + k] : make_float4(0.f, 1.5707964f, 0.f, 0.f);
        st.th[lane][0] = c0.x;
        st.th[lane][1] = c0.y;
        st.th[lane][2] = c0.z;
        st.st[lane] = 0;
        st.frozen[lane] = 0;
        st.moved[lane] = 0;
        st.fprev[lane] = 0.f;
    }
    __syncthreads();

    float acc[NC][10];
    // schedule: every global level below Lp, then Lp
    int ns = 1;
    for (int j = 0; j < a.n_levels; ++j) ns += a.levels[j] < Lp;
    for (int j = 0; j < ns; ++j) {
        const int L = j + 1 < ns ? a.levels[j] : Lp;
        const float4 *Cl = j + 1 < ns ? Cp : Cf;
        if (lane < NC) st.frozen[lane] = 0;
        for (int s = 0; s < a.steps; ++s) {
            if (a.early_stop) {
                // every candidate of the wave has stopped at this level: its later steps change nothing
                int all = 1;
#pragma unroll
                for (int c = 0; c < NC; ++c) all &= st.frozen[c];
                if (__builtin_amdgcn_readfirstlane(all)) break;
            }
            prepare_step<NC, true>(st, ws, L, lane);
            eval_level_any<NC, true, F64>(Cl, a.tab, a.tab64, a.pinfo, L, a.fp64_above, st.bc, ws, acc, lane);
            wave_reduce<NC, 10>(acc, st, lane);
            if (lane < NC && !st.frozen[lane]) {
                double e[10];
                const float *tv = st.tot[lane];
                e[0] = 2.0 * tv[0];
                e[1] = -2.0 * tv[1];
                e[2] = 2.0 * tv[2];
                e[3] = -2.0 * tv[3];
                e[4] = -2.0 * tv[4];
                e[5] = -2.0 * tv[5];
                e[6] = -2.0 * tv[6];
                e[7] = 4.0 * tv[7];  // the b-b sum is accumulated from D''/2
                e[8] = -2.0 * tv[8];
                e[9] = -2.0 * tv[9];
                bool stop = false;
                if (a.early_stop) {
                    const double gn = sqrt(e[1] * e[1] + e[2] * e[2] + e[3] * e[3]);
                    if (gn <= a.tol_grad * fabs(e[0]) || (s > 0 && fabs(e[0] - st.fprev[lane]) <= a.tol_rel * fabs(e[0])))
                        stop = true;
                }
                st.fprev[lane] = (float)e[0];
                if (stop) {
                    st.st[lane] |= 32u;
                    st.frozen[lane] = 1;
                } else {
                    double sinf_ = 0.0;
                    st.st[lane] |= a.gd_rate > 0.0 ? gradient_step(e, a.gd_rate, L, a.max_step, st.th[lane], &sinf_)
                                                   : newton_step(e, a.max_step, st.th[lane], &sinf_);
                    st.moved[lane] = 1;  // near-pole test at the next prepare_step, from its sin b
                    if (a.early_stop && sinf_ <= a.tol_step) {
                        st.st[lane] |= 32u;
                        st.frozen[lane] = 1;
                    }
                }
            }
            wave_sync();
        }
    }
    // value at the final points on the last level, then selection
    prepare_step<NC, true>(st, ws, Lp, lane);
    eval_level_any<NC, false, F64>(Cf, a.tab, a.tab64, a.pinfo, Lp, a.fp64_above, st.bc, ws, acc, lane);
    wave_reduce<NC, 1>(acc, st, lane);
    if (lane < NC) {
        const int k = wave * NC + lane;
        const float F = 2.f * st.tot[lane][0];
        uint32_t s = st.st[lane];
        if (!isfinite(F)) s |= 1u;
        fin[wave * NC + lane] = F;
        fst[wave * NC + lane] = s;
        if (k < a.Kc)
            a.cand[(int64_t)p * a.Kc + k] = make_float4((float)st.th[lane][0], (float)st.th[lane][1],
                                                        (float)st.th[lane][2], F);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int bi = 0;
        for (int k = 1; k < a.Kc; ++k) {
            const float F = fin[k], Fb = fin[bi];
            if (isfinite(F) && (!isfinite(Fb) || F > Fb)) bi = k;
        }
        a.best[p] = a.cand[(int64_t)p * a.Kc + bi];
        a.best_idx[p] = bi;
        a.status[p] |= fst[bi];
    }
    if (!a.queue) break;
    __syncthreads();  // the selection has read fin / fst and every wave is done with its LDS state
    if (threadIdx.x == 0) next_b = atomicAdd(a.queue, 1);
    __syncthreads();
    b = next_b;
    }
}

__global__ void k_zero_counter(int *q) { *q = 0; }

// Objective, gradient and Hessian at one rotation per particle (one wave per particle).
__global__ void __launch_bounds__(64) k_evaluate(EvalArgs a)
{
    __shared__ WaveScratch<1> ws;
    __shared__ WaveState<1> st;
    const int p = blockIdx.x, lane = threadIdx.x;
    const float4 *Cp = a.C + a.C_off[p] / 2;
    const int L = a.L > 0 ? a.L : a.Lp[p];
    if (lane == 0) {
        const float4 t = a.theta[p];
        st.th[0][0] = t.x;
        st.th[0][1] = t.y;
        st.th[0][2] = t.z;
    }
    __syncthreads();
    prepare_step<1, false>(st, ws, L, lane);
    float acc[1][10];
    eval_level_any<1, true, true>(Cp, a.tab, a.tab64, a.pinfo, L, a.fp64_above, st.bc, ws, acc, lane);
    wave_reduce<1, 10>(acc, st, lane);
    if (lane < 10) {
        // signs and factors of the 10 sums; the b-b sum is accumulated from D''/2
        const float sgn = lane == 7 ? 4.f : ((lane == 0 || lane == 2) ? 2.f : -2.f);
        a.out[(int64_t)p * 10 + lane] = sgn * st.tot[0][lane];
    }
}

template <int NC>
size_t march_smem_bytes(int G)
{
    return (size_t)G * (sizeof(WaveScratch<NC>) + sizeof(WaveState<NC>)) + (size_t)G * NC * 8;
}

// Workgroups of a persistent launch: as many as are resident at once (at most one per particle).
template <typename K>
int persistent_grid(K kernel, int threads, size_t smem, int P)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, smem) != hipSuccess)
        return -1;
    return std::max(1, std::min(P, std::max(1, per_cu) * cus));
}

template <int NC>
hipError_t launch_march(const MarchArgs &a0, int P, bool f64, hipStream_t s)
{
    MarchArgs a = a0;
    a.P = P;
    const int G = (a.Kc + NC - 1) / NC;
    const size_t sm = march_smem_bytes<NC>(G);
    auto kern = f64 ? k_march<NC, true> : k_march<NC, false>;
    int grid = P;
    if (a.queue) {
        grid = persistent_grid(kern, G * kWave, sm, P);
        if (grid < 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, a.queue);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(G * kWave), sm, s, a);
    return hipGetLastError();
}

hipError_t launch_march_any(const MarchArgs &a, int P, int nc, bool f64, hipStream_t s)
{
    switch (nc) {
    case 1: return launch_march<1>(a, P, f64, s);
    case 2: return launch_march<2>(a, P, f64, s);
    case 4: return launch_march<4>(a, P, f64, s);
    case 8: return launch_march<8>(a, P, f64, s);
    default: return hipErrorInvalidValue;
    }
}

size_t march_smem_any(int Kc, int nc)
{
    switch (nc) {
    case 1: return march_smem_bytes<1>((Kc + 0) / 1);
    case 2: return march_smem_bytes<2>((Kc + 1) / 2);
    case 4: return march_smem_bytes<4>((Kc + 3) / 4);
    case 8: return march_smem_bytes<8>((Kc + 7) / 8);
    default: return 0;
    }
}

hipError_t launch_evaluate(const EvalArgs &a, int P, hipStream_t s)
{
    hipLaunchKernelGGL(k_evaluate, dim3(P), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

}  // namespace matcha
