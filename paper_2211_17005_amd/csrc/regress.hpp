// Internal interface of the regression kernels (NN^+ networks trained by BaseAlg).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsim {

constexpr int kMlpThreads = 512;     // 8 waves per workgroup; a team of workgroups per date
constexpr int kMlpWaves = kMlpThreads / 64;
constexpr int kMlpRows = 64;         // rows of a chunk staged in LDS
constexpr int kMlpDin = 32;          // input width, padded to one MFMA K step
constexpr int kMlpTiles = 3;         // wave tiling variants of the kernels
constexpr int kMaxRegDates = 512;
constexpr int kTeamSpinLimit = 1 << 22;  // default polls before a bounded wait gives up (several seconds)
constexpr double kRefitGuard = 1e-12; // refit: a Cholesky pivot at or below this times its diagonal drops the column

// Layout of one date's model record (floats; doubles on the FP64 path), D = the padded input
// width (32, or 64 on the FP32 / FP64 path for 33..64 inputs):
//   [ W_1 (U x D) | b_1 (U) | W_2 (U x U) | b_2 | ... | W_H | b_H | w_out (U) | b_out | mu |
//     x_mean (D) | x_inv_std (D) | y_scale | trained ]
// W_1 columns >= d_in stay zero.  Prediction: ((f)^+ + mu) * y_scale, 0 when untrained.
constexpr int kMlpDinWide = 64;
__host__ __device__ inline int din_pad(int d_in) { return d_in <= kMlpDin ? kMlpDin : kMlpDinWide; }

struct MlpLayout {
  int U, H, D = kMlpDin;
  __host__ __device__ int w_off(int l) const {   // l = 1..H
    return l == 1 ? 0 : U * D + U + (l - 2) * (U * U + U);
  }
  __host__ __device__ int b_off(int l) const { return w_off(l) + U * (l == 1 ? D : U); }
  __host__ __device__ int wout_off() const { return b_off(H) + U; }
  __host__ __device__ int bout_off() const { return wout_off() + U; }
  __host__ __device__ int mu_off() const { return bout_off() + 1; }
  __host__ __device__ int n_params() const { return mu_off() + 1; }
  __host__ __device__ int xmean_off() const { return n_params(); }
  __host__ __device__ int xinv_off() const { return xmean_off() + D; }
  __host__ __device__ int yscale_off() const { return xinv_off() + D; }
  __host__ __device__ int trained_off() const { return yscale_off() + 1; }
  __host__ __device__ int record() const { return trained_off() + 1; }
};

struct MlpArgs {
  int32_t U, H, d_in;
  int32_t epochs, batch;
  float lr, beta1, beta2, eps;
  int32_t n_reg;
  int64_t M;
  int32_t n_feat;                 // feature stride of X: X[date][f][k] at (date*n_feat + f)*M + k
  int32_t init_tag;               // Philox date word of the initial weights
  uint32_t key0, key1;
  const float* X;                 // [n+1][n_feat][M]
  const float* Y;                 // [n+1][M]
  const float* Wt;                // [n+1][M] row weights, or null (all 1)
  float* model;                   // [n_reg][record]   (best parameters + scaling)
  float* cur;                     // [n_reg][n_params] current parameters (one copy per team)
  float* adam_m;                  // [n_reg][n_params]
  float* adam_v;                  // [n_reg][n_params]
  float* partial;                 // [n_teams][G][n_params] per-workgroup gradients (G > 1)
  double* gram;                   // [n_teams][G][(U+1)*(U+2)] refit normal equations
  double* loss_part;              // [n_teams][G] per-workgroup loss sums
  int32_t* team_ctr;              // [n_teams] barrier arrivals (zeroed before the launch)
  int32_t* status;                // one word: nonzero when a bounded wait gave up (zeroed per fit)
  int32_t spin_limit;             // polls before a bounded wait gives up
  float* loss_hist;               // [n_reg][epochs] or null
  int32_t G;                      // workgroups per team (one team trains one date at a time)
  int32_t n_teams;
  int32_t use_init;               // 1: start from `model` (warm start), 0: from the Philox draw
  int32_t tile;                   // wave tiling variant, 0 .. kMlpTiles - 1 (predictions: any)
  // Loss helpers (all dates trained at once): the full-sample loss of every epoch is computed by
  // workgroups without a team (and by teams once they are done) from per-epoch parameter
  // snapshots; the best epoch is chosen when a date's last loss is in.  snaps null: the teams
  // compute the loss themselves.
  float* snaps;                   // [n_reg][epochs][n_params]
  int32_t* ready;                 // [n_reg][epochs] members' snapshot arrivals, or a marker < 0
  int32_t* done;                  // [n_reg] losses computed
  int32_t* lqueue;                // helper work counter
  float* losses;                  // [n_reg][epochs]
  int32_t n_blocks;               // workgroups of the launch (trainers first)
  int32_t dates[kMaxRegDates];
};

// The kernels of each wave tiling variant (regress.hip compiled once per variant).
#define HSIM_MLP_TILE_DECL(ns)                                                                  \
  namespace ns {                                                                                \
  hipError_t launch_mlp_stats(const MlpArgs& a, hipStream_t s);                                 \
  int mlp_max_teams(int U, int H, int G);                                                       \
  hipError_t launch_mlp_train(const MlpArgs& a, hipStream_t s);                                 \
  hipError_t launch_mlp_predict(const MlpArgs& a, float* out, hipStream_t s);                   \
  bool mlp_supported(int U, int H);                                                             \
  }
HSIM_MLP_TILE_DECL(tile0)
HSIM_MLP_TILE_DECL(tile1)
HSIM_MLP_TILE_DECL(tile2)
#undef HSIM_MLP_TILE_DECL

inline hipError_t launch_mlp_stats(const MlpArgs& a, hipStream_t s) { return tile0::launch_mlp_stats(a, s); }
// Teams that fit on the device at once for team size G (all workgroups of a launch are resident;
// every variant has the same LDS and registers per workgroup).
inline int mlp_max_teams(int U, int H, int G) { return tile0::mlp_max_teams(U, H, G); }
// Launch with a.G, a.n_teams set (a.n_teams <= mlp_max_teams); zeroes the team counters first.
inline hipError_t launch_mlp_train(const MlpArgs& a, hipStream_t s) {
  return a.tile == 1 ? tile1::launch_mlp_train(a, s) : a.tile == 2 ? tile2::launch_mlp_train(a, s)
                                                                  : tile0::launch_mlp_train(a, s);
}
inline hipError_t launch_mlp_predict(const MlpArgs& a, float* out, hipStream_t s) {
  return a.tile == 1 ? tile1::launch_mlp_predict(a, out, s) : a.tile == 2 ? tile2::launch_mlp_predict(a, out, s)
                                                                          : tile0::launch_mlp_predict(a, out, s);
}
inline bool mlp_supported(int U, int H) { return tile0::mlp_supported(U, H); }

}  // namespace hsim
