// matcha_ball.hpp -- the ball-harmonic transform's index set, device tables and launch.
#pragma once
#include <vector>

#include "matcha_dev.hpp"

namespace matcha {

constexpr int kBallMaxL = 64;

// I_Lambda: zeros[l] = the kept lam_lk of degree l (|K_l| of them), l <= L.
struct BallIndex {
    std::vector<std::vector<double>> zeros;
    int L = -1, Kmax = 0, nk = 0;  // nk = sum_l |K_l|
};

// Zeros of the spherical Bessel functions up to lam; false if lam is out of range.
bool ball_index(double lam, BallIndex &ix);
// Host tables for an N^3 grid: vidx [V] (flat indices of the voxels inside the ball, raster order),
// R [nk][V] (rows (l, k) degree-major: (2/N)^3 c_lk j_l(lam_lk r_v)), A [(L+1)(L+2)][V] (rows
// (l, m >= 0, re / im) of conj Y_lm at the voxel), all rounded to FP32 from FP64.
void ball_build_tables(int N, const BallIndex &ix, std::vector<int32_t> &vidx, std::vector<float> &R,
                       std::vector<float> &A);

struct BallArgs {
    const float *u;        // [P][N][N][N] real volumes
    float *out;            // [P][Kmax][(L+1)^2] complex
    const int32_t *vidx;   // [V]
    const float *R;        // [nk][V]
    const float *A;        // [(L+1)(L+2)][V]
    int64_t V;
    int N, P, L, Kmax;
    int nk_l[kBallMaxL + 1];    // |K_l|
    int rk_off[kBallMaxL + 1];  // first row of degree l in R
    int blk_lo[kBallMaxL + 2];  // first workgroup of degree L - d (set by the launcher)
};

hipError_t launch_ball(const BallArgs &a, hipStream_t s);

}  // namespace matcha
