// k_lowrank.hip -- singular values of the correlation blocks and their effective rank (App. A.6, B.1).
//
// Per particle and degree l the block C^l = sum_r w_r f_l(r) h_l(r)^H is F H^H with the
// (2l+1) x K matrices F = [sqrt(w_r) f_lm(r)], H = [sqrt(w_r) h_lm(r)], K = R_p shells, so its rank is
// at most K (eq. rank_bound with shells for the radial index).  Its singular values are reached
// without forming anything of size 2l+1 beyond the input:
//   G_F = F^H F, G_H = H^H H (K x K Gram matrices, Hermitian positive semi-definite),
//   G_F = X_F X_F^H, G_H = X_H X_H^H by outer-product Cholesky with diagonal pivoting, stopped at the
//   numerical rank (X: K x r),
//   C^H C = H G_F H^H has the nonzero eigenvalues of G_F G_H = X_F X_F^H X_H X_H^H, i.e. of Z Z^H with
//   Z = X_F^H X_H (r_F x r_H), so the singular values of C^l are those of Z.
// Z's singular values come from one-sided (Hestenes) Jacobi: column pairs are rotated until every
// pair is orthogonal to working precision; the singular values are then the column norms.  All of it
// in FP64 in one wave per (particle, degree), the matrices in LDS.  The effective rank (App. B.1) is
//   r_eff = min { k >= 1 : s_{k+1} / s_k < rho },  s_1 >= s_2 >= ...  (the number of values when no
//   ratio falls below rho; 0 for a zero block).
#include "matcha_launch.hpp"

namespace matcha {

typedef double2 cplx;

__device__ __forceinline__ cplx cmul_conj(cplx a, cplx b)  // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Outer-product Cholesky with diagonal pivoting of the K x K Hermitian PSD matrix G (row-major in
// LDS, destroyed): X[:, j] = G[:, q] / sqrt(G[q][q]) for the largest remaining diagonal q, then
// G -= X[:, j] X[:, j]^H; stops when the largest remaining diagonal is <= tol times the largest
// initial one.  X is stored column-major (X[j * K + i]).  Returns the rank r.  Wave-uniform.
__device__ __forceinline__ int pivoted_cholesky(cplx *G, cplx *X, int K, int lane)
{
    double d0 = 0.0;
    for (int i = lane; i < K; i += kWave) d0 = fmax(d0, G[i * K + i].x);
    d0 = wave_max(d0);
    if (!(d0 > 0.0)) return 0;
    const double tol = 1e-13 * d0;
    int r = 0;
    for (; r < K; ++r) {
        double best = -1.0;
        int q = 0;
        for (int i = lane; i < K; i += kWave) {
            const double d = G[i * K + i].x;
            if (d > best) {
                best = d;
                q = i;
            }
        }
        // wave argmax (ties: the smaller index)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ob = __shfl_xor(best, o, kWave);
            const int oq = __shfl_xor(q, o, kWave);
            if (ob > best || (ob == best && oq < q)) {
                best = ob;
                q = oq;
            }
        }
        if (!(best > tol)) break;
        const double inv = 1.0 / sqrt(best);
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < K; i += kWave) {
            const cplx g = G[i * K + q];
            X[r * K + i] = make_double2(g.x * inv, g.y * inv);
        }
        __builtin_amdgcn_wave_barrier();
        __syncthreads();
        for (int e = lane; e < K * K; e += kWave) {
            const int i = e / K, k = e - (e / K) * K;
            const cplx xi = X[r * K + i], xk = X[r * K + k];
            // G[i][k] -= xi * conj(xk)
            G[e].x -= xi.x * xk.x + xi.y * xk.y;
            G[e].y -= xi.y * xk.x - xi.x * xk.y;
        }
        __syncthreads();
    }
    return r;
}

__global__ void __launch_bounds__(kWave) k_lowrank_sv(LowRankArgs a)
{
    extern __shared__ __align__(16) unsigned char lr_smem[];
    const int p = blockIdx.x / (a.L_max + 1), l = blockIdx.x % (a.L_max + 1);
    const int lane = threadIdx.x;
    double *sv = a.sv + ((int64_t)p * (a.L_max + 1) + l) * a.n_sv;
    const int Lp = a.Lp[p], K = a.Rp[p], n = 2 * l + 1;
    if (l > Lp || K <= 0) {
        for (int j = lane; j < a.n_sv; j += kWave) sv[j] = 0.0;
        if (lane == 0) a.r_eff[(int64_t)p * (a.L_max + 1) + l] = 0;
        return;
    }
    cplx *G = reinterpret_cast<cplx *>(lr_smem);  // K x K
    cplx *XF = G + K * K;                          // K x K (column-major, r_F columns used)
    cplx *XH = XF + K * K;
    const float2 *fp = a.f + a.f_off[p] + l * l;            // f_lm(r) at fp[r (Lp+1)^2 + m + l]
    const float2 *hp = a.h + l * l;                          // h_lm(r) at hp[r (Lh+1)^2 + m + l]
    const int sf = (Lp + 1) * (Lp + 1), sh = (a.Lh + 1) * (a.Lh + 1);
    int rk[2];
    for (int side = 0; side < 2; ++side) {
        const float2 *src = side == 0 ? fp : hp;
        const int st = side == 0 ? sf : sh;
        // G[i][k] = sqrt(w_i w_k) sum_m conj(v_m(i)) v_m(k)
        for (int e = lane; e < K * K; e += kWave) {
            const int i = e / K, k = e - (e / K) * K;
            double sr = 0.0, si = 0.0;
            for (int m = 0; m < n; ++m) {
                const float2 x = src[(int64_t)i * st + m], y = src[(int64_t)k * st + m];
                sr += (double)x.x * y.x + (double)x.y * y.y;
                si += (double)x.x * y.y - (double)x.y * y.x;
            }
            const double wik = sqrt((double)a.w[i] * (double)a.w[k]);
            G[e] = make_double2(wik * sr, wik * si);
        }
        __syncthreads();
        rk[side] = pivoted_cholesky(G, side == 0 ? XF : XH, K, lane);
        __syncthreads();
    }
    const int rF = rk[0], rH = rk[1];
    // Z = XF^H XH (rF x rH), column-major in G: Z[j * rF + i] = sum_k conj(XF[i][k]) XH[j][k]
    cplx *Z = G;
    for (int e = lane; e < rF * rH; e += kWave) {
        const int j = e / rF, i = e - (e / rF) * rF;
        double zr = 0.0, zi = 0.0;
        for (int k = 0; k < K; ++k) {
            const cplx t = cmul_conj(XF[i * K + k], XH[j * K + k]);
            zr += t.x;
            zi += t.y;
        }
        Z[j * rF + i] = make_double2(zr, zi);
    }
    __syncthreads();
    // one-sided Jacobi on the columns of Z; lane i holds row i (rF <= K <= 64)
    const bool row = lane < rF;
    for (int sweep = 0; sweep < 40 && rF > 0 && rH > 1; ++sweep) {
        int rotated = 0;
        for (int c0 = 0; c0 < rH - 1; ++c0)
            for (int c1 = c0 + 1; c1 < rH; ++c1) {
                const cplx za = row ? Z[c0 * rF + lane] : make_double2(0.0, 0.0);
                const cplx zb = row ? Z[c1 * rF + lane] : make_double2(0.0, 0.0);
                const double al = wave_sum(za.x * za.x + za.y * za.y);
                const double be = wave_sum(zb.x * zb.x + zb.y * zb.y);
                const cplx gp = cmul_conj(za, zb);
                const double gr = wave_sum(gp.x), gi = wave_sum(gp.y);
                const double g = sqrt(gr * gr + gi * gi);
                if (!(g > 1e-15 * sqrt(al * be)) || !(g > 1e-300)) continue;
                ++rotated;
                const double zeta = (be - al) / (2.0 * g);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                // b~ = e^{-i phi} zb with e^{i phi} = gamma / |gamma|: conj(za) . b~ = |gamma|
                const double er = gr / g, ei = -gi / g;
                const cplx bt = make_double2(er * zb.x - ei * zb.y, er * zb.y + ei * zb.x);
                if (row) {
                    Z[c0 * rF + lane] = make_double2(c * za.x - s * bt.x, c * za.y - s * bt.y);
                    Z[c1 * rF + lane] = make_double2(s * za.x + c * bt.x, s * za.y + c * bt.y);
                }
                __builtin_amdgcn_wave_barrier();
            }
        if (rotated == 0) break;
    }
    // column norms, sorted descending across the lanes (bitonic on 64 values, padding -1)
    double v = -1.0;
    if (lane < rH) {
        double s2 = 0.0;
        for (int i = 0; i < rF; ++i) {
            const cplx z = Z[lane * rF + i];
            s2 += z.x * z.x + z.y * z.y;
        }
        v = sqrt(s2);
    }
    if (rF == 0) v = lane < 1 ? 0.0 : -1.0;
    for (int k = 2; k <= kWave; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            const double o = __shfl_xor(v, j, kWave);
            const bool up = ((lane & k) == 0);  // descending blocks
            const bool lower = (lane & j) == 0;
            const bool take_max = (lower == up);
            v = take_max ? fmax(v, o) : fmin(v, o);
        }
    const int nv = min(n, K);  // singular values reported per block (the rest are zero)
    for (int j = lane; j < a.n_sv; j += kWave) sv[j] = 0.0;
    __builtin_amdgcn_wave_barrier();
    if (lane < nv && lane < a.n_sv) sv[lane] = fmax(v, 0.0);
    // r_eff: the first k (1-based) with s_{k+1} / s_k < rho, among the nv values
    const double s_k = fmax(v, 0.0), s_k1 = fmax(__shfl_down(v, 1, kWave), 0.0);
    const double s1 = __shfl(v, 0, kWave);
    const bool cut = lane + 1 < nv && s_k > 0.0 && s_k1 < a.rho * s_k;
    const unsigned long long bal = __ballot(cut);
    if (lane == 0) {
        int r = 0;
        if (s1 > 0.0) r = bal ? (int)__builtin_ctzll(bal) + 1 : nv;
        a.r_eff[(int64_t)p * (a.L_max + 1) + l] = r;
    }
}

size_t lowrank_smem_bytes(int Rmax) { return 3 * sizeof(cplx) * (size_t)Rmax * Rmax; }

hipError_t launch_lowrank(const LowRankArgs &a, hipStream_t s)
{
    const int64_t nb = (int64_t)a.P * (a.L_max + 1);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lowrank_sv, dim3((unsigned)nb), dim3(kWave), lowrank_smem_bytes(a.R_max), s, a);
    return hipGetLastError();
}

}  // namespace matcha
