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
};

struct SoftArgs {
    const float4 *C;
    const int64_t *C_off;
    const float4 *tab;
    const PairInfo *pinfo;
    int B, n, Kc;
    float4 *cand;
    uint32_t *status;
};

struct MarchArgs {
    const float4 *C;          // wedge layout, float4 = (C^l_mn, C^l_partner)
    const int64_t *C_off;     // complex offsets (even)
    const int32_t *Lp;
    const float4 *tab;        // per (l, q): A = abar_{l-1}, AC = abar_{l-1} c_{l-1}, PW = w P_l, PWT = w~ s P_l
    const PairInfo *pinfo;
    int n_levels;
    int levels[kMaxLevels];
    int steps;
    double max_step;
    int early_stop;
    double tol_grad, tol_step, tol_rel;
    int Kc;
    float4 *cand;
    float4 *best;
    int32_t *best_idx;
    uint32_t *status;
};

struct EvalArgs {
    const float4 *C;
    const int64_t *C_off;
    const float4 *tab;
    const PairInfo *pinfo;
    int L;
    const float4 *theta;
    float *out;
};

size_t assemble_smem_bytes(int Lmax, int Rmax);
hipError_t launch_assemble_f32(const AsmArgs &a, int P, int Lmax, int Rmax, hipStream_t s);

size_t soft_smem_bytes(int n, int B);
hipError_t launch_soft(const SoftArgs &a, int P, hipStream_t s);

size_t march_smem_any(int Kc, int nc);
hipError_t launch_march_any(const MarchArgs &a, int P, int nc, hipStream_t s);
hipError_t launch_evaluate(const EvalArgs &a, int P, hipStream_t s);

}  // namespace matcha
