// matcha_ball.hpp -- the ball-harmonic transform's index set, tables and launch.
#pragma once
#include <vector>

#include "matcha_dev.hpp"

namespace matcha {

constexpr int kBallChunk = 32;       // octant voxels per staged chunk; rows are padded to a multiple
constexpr int kBallMaxSplits = 16;   // K splits of the product
constexpr int kBallTileMBig = 256;   // from this many volumes on, 128-volume row tiles (else 64)

// I_Lambda: zeros[l] = the kept lam_lk of degree l (|K_l| of them), l <= L.
struct BallIndex {
    std::vector<std::vector<double>> zeros;
    int L = -1, Kmax = 0, nk = 0;  // nk = sum_l |K_l|
};

// Output entry (k, lm) of a volume: (s_re x column col_re, s_im x column col_im), a column -1 gives 0.
struct BallMapEntry {
    int32_t col_re, col_im;
    float s_re, s_im;
};

// Host tables of one (N, Lambda).
struct BallHostTables {
    std::vector<int32_t> oct;      // [Vo] flat grid index of each octant voxel
    std::vector<float> T;          // [ncol][Vo_pad], columns grouped by class (col_off)
    std::vector<BallMapEntry> map;  // [Kmax][(L+1)^2]
    int col_off[9] = {0};
    int64_t Vo = 0, Vo_pad = 0;
};

// Zeros of the spherical Bessel functions up to lam; false if the set is empty or lam out of range.
bool ball_index(double lam, BallIndex &ix);
void ball_build_tables(int N, const BallIndex &ix, BallHostTables &t);

struct BallSymArgs {
    const float *u;       // [P][N][N][N]
    const int32_t *oct;   // [Vo]
    float *usym;          // [8][P][Vo_pad]
    int64_t Vo, Vo_pad;
    int N, P;
};

struct BallGemmArgs {
    const float *usym;    // [8][P][Vo_pad]
    const float *T;       // [ncol][Vo_pad]
    float *part;          // [S][P][ncol]
    int64_t Vo_pad, kper;  // kper: voxels per split, a multiple of kBallChunk
    int P, ncol, S;
    int col_off[9];
    int tile_lo[9];       // set by the launcher
};

struct BallScatterArgs {
    const float *part;
    const BallMapEntry *map;
    float *out;           // [P][n_entries] complex
    int P, ncol, S, n_entries;
};

// Volumes per row tile of the product for P volumes (64 or 128).
int ball_tile_m(int P);
// K splits for P volumes: about eight workgroups per compute unit, at least 8 chunks per split.
int ball_splits(int P, int ncol_tiles, int64_t Vo_pad, int n_cu);
// 128-column tiles over the classes; tile_lo (optional, 9 entries) = first tile of each class.
int ball_col_tiles(const int *col_off, int *tile_lo);
hipError_t launch_ball(const BallSymArgs &sa, const BallGemmArgs &ga, const BallScatterArgs &ca, hipStream_t s);

}  // namespace matcha
