// matcha_launch.hpp -- kernel argument blocks and launchers (host side of the kernels).
#pragma once
#include "matcha_dev.hpp"

namespace matcha {

struct AsmArgs {
    const float2 *f;
    const int64_t *f_off;
    const float2 *h;
    const float *w;
    const int32_t *Lp;
    const int32_t *Rp;
    int Lh;
    float4 *C;
    const int64_t *C_off;
    const int32_t *by_L;      // nullable: particle indices by decreasing L_p (k_order_by_L); null: all L_p equal
    int P, Lmax, Rmax;        // set by the launcher
    int tiles_per_wave;       // 16-row tiles per wave and workgroup (0: default)
    int blk_lo[kMaxL + 2];    // first workgroup of degree Lmax - d, d = 0 .. Lmax; [Lmax+1]: total
    int np_l[kMaxL + 1];      // particles with L_p >= l: the first np_l[l] entries of by_L (or all P)
};

struct AsmBArgs {
    const __bf16 *f;          // complex BF16 pairs (re, im)
    const int64_t *f_off;     // complex offsets
    const __bf16 *h;
    const float *w;
    const int32_t *Lp;
    const int32_t *Rp;
    int Lh;
    float4 *C;
    const int64_t *C_off;
    const int32_t *by_L;      // nullable: particle indices by decreasing L_p (k_order_by_L); null: all L_p equal
    int P, Lmax, Rmax;        // set by the launcher
    int tiles_per_wave;       // 16-row tiles per wave and workgroup (0: default)
    int blk_lo[kMaxL + 2];    // first workgroup of degree Lmax - d, d = 0 .. Lmax; [Lmax+1]: total
    int np_l[kMaxL + 1];      // particles with L_p >= l: the first np_l[l] entries of by_L (or all P)
};

struct SoftArgs {
    const float4 *C;
    const int64_t *C_off;
    const float2 *dgrid;      // [n][wedge_row(B+1)]: weighted d^l(b_i) of each wedge pair and its partner
    const float *dft;         // DFT tables of the grid kernel (build_soft_dft)
    const PairInfo *pinfo;
    int B, n, Kc;
    int gslices;              // waves per workgroup of the grid kernel (set by its launcher)
    int grid_nodes;           // polar nodes per wave of the register-resident grid kernel (even; 0: default)
    int p0;                   // first particle of this launch
    int np;                   // particles in this launch (set by the grid launcher)
    float *grid;              // [launch particles][n][n][n] workspace: C_B on the grid
    float2 *S;                // [launch particles][n][(B+1)(2B+1)] workspace: Wigner transforms
    unsigned long long *mlist;  // [launch particles][mcap] keys of the local maxima (workspace)
    uint32_t *mcount;         // [launch particles] maxima found (may exceed mcap)
    int mcap;                 // keys kept per particle (set by the select launcher)
    float4 *cand;
    uint32_t *status;
};

struct MarchArgs {
    const float4 *C;          // wedge layout, float4 = (C^l_mn, C^l_partner)
    const float4 *C_fin;      // nullable: coefficients of each particle's final level (same offsets as C)
    const int64_t *C_off;     // complex offsets (even)
    const int32_t *Lp;
    const float4 *tab;        // per (l, q): A = abar_{l-1}, AC = abar_{l-1} c_{l-1}, PW = w P_l, PWT = w~ s P_l
    const double2 *tab64;     // per (l, q): (A, AC) in FP64 for the FP64 recurrence
    int fp64_above;           // levels above this degree run the recurrence in FP64
    const PairInfo *pinfo;
    int n_levels;
    int levels[kMaxLevels];
    int steps;
    double max_step;
    int early_stop;
    double tol_grad, tol_step, tol_rel;
    double gd_rate;           // > 0: gradient ascent steps instead of Newton steps
    int Kc;
    float4 *cand;
    float4 *best;
    int32_t *best_idx;
    uint32_t *status;
    const int32_t *order;     // nullable processing order (the b-th particle taken is order[b])
    int P;                    // particles
    int *queue;               // nullable: work counter of the persistent kernel (zeroed by its launcher)
};

struct EvalArgs {
    const float4 *C;
    const int64_t *C_off;
    const float4 *tab;
    const double2 *tab64;
    int fp64_above;
    const PairInfo *pinfo;
    const int32_t *Lp;
    int L;                    // > 0: this band for every particle; 0: each particle's L_p
    const float4 *theta;
    float *out;
};

struct GradArgs {
    const float2 *f;
    const int64_t *f_off;
    const float2 *h;
    const float *w;
    const int32_t *Lp;
    const int32_t *Rp;
    int Lh, Rh, L_max, P;
    const float4 *best;
    const float *g;
    float2 *grad_f;           // may be null
    float2 *ws;               // per-particle grad_h terms at ws_off[p] (null if grad_h is null)
    int64_t *ws_off;          // [P] packed offsets of the terms, written by the first kernel
    float2 *part;             // [n_seg][R_h][(L_h+1)^2] partial sums over segments of particles
    int n_seg, seg_len;       // set by the launcher (grad_segments)
    float2 *grad_h;           // may be null
    const PairInfo *pinfo;
    const float4 *tab;
};

struct LowRankArgs {
    const float2 *f;
    const int64_t *f_off;
    const float2 *h;
    const float *w;
    const int32_t *Lp;
    const int32_t *Rp;
    int Lh, L_max, R_max, P;
    double rho;
    double *sv;               // [P][L_max + 1][n_sv], descending, zero-padded
    int32_t *r_eff;           // [P][L_max + 1]
    int n_sv;
};

struct TransArgs {
    int N, P;
    const float *h;           // [N^3] template volume
    const float4 *euler;      // [P] rotations (a, b, c, .)
    float *vol;               // [P][N^3] real volumes (rotated templates, correlations)
    const float2 *spec_in;    // [P][N][N][N/2+1]
    float2 *spec_out;         // [P][N][N][N/2+1]
    float2 *spec_aux;         // [P][N][N][N/2+1] copy of the cross spectrum for the inverse transform
    const float4 *shift;      // [P] shifts (x, y, z, .) in voxels
    int window;               // integer search window, |s_i| <= window
    int4 *peak;               // [P] best integer shift
    float2 *ups;              // [P][N][m][m] refinement partials
    float2 *ups_tab;          // [P][(N/2+1) + N][m] refinement phase tables
    int m;                    // refinement offsets per axis
    double kappa;             // refinement steps per voxel
    float4 *shift_out;        // [P] refined shift (x, y, z, correlation)
};

size_t assemble_smem_bytes(int Lmax, int Rmax);
hipError_t launch_assemble_f32(const AsmArgs &a, int P, int Lmax, int Rmax, hipStream_t s);
// by_L[0 .. P-1] = the particle indices ordered by decreasing L_p (equal L_p in any order).
hipError_t launch_order_by_L(const int32_t *Lp, int P, int Lmax, int32_t *by_L, hipStream_t s);

size_t assemble_bf16_smem_bytes(int Lmax, int Rmax);
hipError_t launch_assemble_bf16(const AsmBArgs &a, int P, int Lmax, int Rmax, hipStream_t s);

size_t soft_grid_smem_bytes(int n, int B);
size_t soft_dft_floats(int n, int B);
void build_soft_dft(int B, int n, float *t);
size_t soft_select_smem_bytes(int n, int threads);
hipError_t launch_soft_wigner(const SoftArgs &a, int P, hipStream_t s);
hipError_t launch_soft_grid(const SoftArgs &a, int P, hipStream_t s);
hipError_t launch_soft_select(const SoftArgs &a, int P, int threads, hipStream_t s);

size_t march_smem_any(int Kc, int nc);
// f64: some level of the batch lies above the FP64 threshold (otherwise the FP32-only kernel runs).
hipError_t launch_march_any(const MarchArgs &a, int P, int nc, bool f64, hipStream_t s);
hipError_t launch_evaluate(const EvalArgs &a, int P, hipStream_t s);

size_t grad_smem_bytes(int Lmax);
// Segments of particles whose template terms the adjoint sums separately before adding the
// segments in order (E = R_h (L_h+1)^2 template entries).
int grad_segments(int64_t E, int P);
hipError_t launch_grad(const GradArgs &a, hipStream_t s);
size_t lowrank_smem_bytes(int Rmax);
hipError_t launch_rotate_volume(const TransArgs &a, hipStream_t s);
hipError_t launch_phase_shift(const TransArgs &a, hipStream_t s);
hipError_t launch_cross_spectrum(const TransArgs &a, hipStream_t s);
size_t upsample_xy_smem(int N, int m);
hipError_t launch_peak_refine(const TransArgs &a, hipStream_t s);
hipError_t launch_lowrank(const LowRankArgs &a, hipStream_t s);

}  // namespace matcha
