// Internal interface between the C-ABI layer and the simulation kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsim {

constexpr int kMaxCcy = 16;
constexpr int kMaxCpty = 16;

// Per-call simulation arguments, passed by value.  Small per-factor Euler coefficients
// live here; the Cholesky factor, the zero-coupon coefficient tables and the bucketed
// swap weights live in a device table pointed to by `table`.
template <typename Real>
struct SimArgs {
  int64_t M;              // paths in this call
  uint32_t path_begin;    // global index of the first path
  uint32_t key0, key1;    // Philox key
  int32_t n_ccy, n_cpty;
  int32_t n_dates, n_sub;
  int32_t q;              // pricing steps per reset period
  int32_t n_periods;      // largest maturity in reset periods
  int32_t feature_mode;   // 0: factors, 1: factors + I + sum Lambda
  int32_t n_feat;
  Real dt;
  double half_dt;
  Real r0[kMaxCcy], x0[kMaxCcy], g0[kMaxCpty];
  Real lgd[kMaxCpty];
  // Euler coefficients, read from device memory inside the sub-step loop:
  //   r^e      <- r^e + r_adt[e] (r_lvl[e] - r^e) + r_vol[e] * W_e
  //   log chi^e <- x + (r^0 - r^e) dt + x_add[e-1] + x_vol[e-1] * W_{n_e+e-1}
  //   gamma^c  <- g + g_add[c] - g_kd[c] g^+ + g_vol[c] sqrt(g^+) z_c
  // laid out as [r_adt | r_lvl | r_vol]  (n_ccy each), [x_add | x_vol] (n_ccy-1 each),
  // [g_add | g_kd | g_vol] (n_cpty each); see coef_* offsets below.
  const Real* coef;
  // device tables (see TableLayout)
  const Real* chol;       // packed lower triangle of the market correlation, row by row
  const Real* lnA;        // [n_ccy][n_dates+1]  Vasicek ln A(tau_j), tau_j = j * horizon / n_dates
  const Real* Bv;         // [n_ccy][n_dates+1]  Vasicek B(tau_j)
  const Real* W1;         // [n_cpty][n_ccy][n_periods+2] sum of payer*notional by maturity period
  const Real* CW1;        // suffix sums of W1 over periods >= p
  const Real* CW2;        // suffix sums of payer*notional*delta*Sigma over periods >= p
  const Real* G;          // W1[p] + CW2[p]
  // outputs
  Real* features;         // [n+1][n_feat][M] or null
  double* I;              // [n+1][M]
  double* Lam;            // [n+1][C][M]
  Real* D;                // [n+1][C][M]
  Real* MtM;              // [n+1][C][M] or null
};

struct InnerArgs {
  int64_t M;
  uint32_t path_begin;
  uint32_t key0, key1;
  int32_t n_dates, n_cpty;
  int32_t n_b;                       // uniform n_b when nb_block is null
  const int32_t* nb_block;           // device [ceil(M/block_paths)] or null
  int32_t block_paths;
  const double* Lam;                 // [n+1][C][M]
  int32_t* counts;                   // [n+1][C][M]
  int32_t* order;                    // uneven n_b: [tiles] tiles by decreasing n_b, then the
                                     // work counter (workspace); null: one workgroup per tile
};

template <typename Real>
struct TargetArgs {
  int64_t M;
  int32_t n_dates, n_cpty;
  int32_t n_b;
  const int32_t* nb_block;
  int32_t block_paths;
  const double* I;
  const Real* D;
  const int32_t* counts;             // default counts of the inner draws, or
  const double* Lam;                 // (intensity form, counts null) the intensity integrals [n+1][C][M]
  Real* T;                           // [n+1][M]
  float* weight;                     // alive-group form (one counterparty): [n+1][M] A_i / n_b, else null
  double* partial;                   // [ceil(M / kTargetBlock)]
  double* cva0;                      // one double
};

// Per-inner-sample regression rows (market state + default indicators) of M x n_b samples.
template <typename Real>
struct SampleArgs {
  int64_t M;
  uint32_t path_begin;
  uint32_t key0, key1;
  int32_t n_dates, n_cpty, d, n_b;
  const Real* features;              // [n+1][d][M]
  const double* I;                   // [n+1][M]
  const double* Lam;                 // [n+1][C][M]
  const Real* D;                     // [n+1][C][M]
  float* X;                          // [n+1][d + C][n_b M]
  float* Y;                          // [n+1][n_b M]
};

// Branched re-simulation: continuations b < n_branch of every path after pricing date `date`.
struct BranchArgs {
  int32_t date;
  int32_t n_branch;
  double* xi;                        // [n_branch][M] intensity-form samples at t_date
};
constexpr int kBranchStats = 6;      // nu, nu^2, U, (phi - nu)^2, phi^2 - 2 phi nu + U, phi

// Fused simulation (hsim_fused): the per-path tables of the inner stage, path-major in the
// workspace, and the outputs.
struct FusedArgs {
  int32_t n_b;                       // uniform n_b when nb_block is null
  const int32_t* nb_block;           // device [ceil(M/block_paths)] or null
  int32_t block_paths;               // a multiple of 64
  uint32_t* K;                       // [M][n+1][C] default thresholds
  void* Dv;                          // [M][n+1][C] exposures (Real)
  double* Iv;                        // [M][n+1] discount integrals
  void* T;                           // [n+1][M] targets (Real)
  double* T0;                        // [M] T_0 in FP64 (the CVA_0 reduction's input)
  // forward states of the paths kl < n_keep, date-major with leading dimension M (as
  // hsim_outer_paths writes them), for a later adjoint; n_keep = 0: none
  int64_t n_keep;
  double* I_keep;                    // [n+1][M]
  double* Lam_keep;                  // [n+1][C][M]
  void* D_keep;                      // [n+1][C][M] (Real)
};

// LDS of one fused workgroup: thresholds and histogram [n+1][C] uint32 each, then (8-byte
// aligned) I and the date terms [n+1] double each, then the exposures [n+1][C].
__host__ __device__ inline size_t fused_lds_offset_f64(int n, int C) {
  return ((size_t)2 * (n + 1) * C * 4 + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t fused_lds_bytes(int n, int C, size_t real_bytes) {
  return fused_lds_offset_f64(n, C) + (size_t)2 * (n + 1) * 8 + (size_t)(n + 1) * C * real_bytes;
}
constexpr size_t kFusedMaxLds = 64 * 1024;   // beyond: the separate stages (occupancy of the outer phase)

// offsets into SimArgs::coef
template <int NE, int NC>
struct CoefLayout {
  static constexpr int r_adt = 0, r_lvl = NE, r_vol = 2 * NE;
  static constexpr int x_add = 3 * NE, x_vol = 3 * NE + (NE - 1);
  static constexpr int g_add = 3 * NE + 2 * (NE - 1), g_kd = g_add + NC, g_vol = g_add + 2 * NC;
  static constexpr int size = g_add + 3 * NC;
};
inline int coef_size(int ne, int nc) { return 3 * ne + 2 * (ne - 1) + 3 * nc; }

constexpr int kOuterBlock = 64;
constexpr int kInnerBlock = 64;
constexpr int kTargetBlock = 256;

// Launchers; return hipSuccess or the launch error.  `supported` reports whether a
// (n_ccy, n_cpty) pair has a compiled instantiation.
bool outer_supported(int n_ccy, int n_cpty);
// fp32_integrals (Real = float only): the discount and intensity integrals accumulate in FP32
// (the plain form) instead of FP64.
template <typename Real>
hipError_t launch_outer(const SimArgs<Real>& a, hipStream_t stream, bool fp32_integrals = false);
hipError_t launch_inner(const InnerArgs& a, hipStream_t stream);
// Workspace of the longest-first schedule of an uneven-n_b inner launch over M paths.
size_t inner_order_bytes(int64_t M);
template <typename Real>
hipError_t launch_targets(const TargetArgs<Real>& a, hipStream_t stream);
// Fused simulation, then the CVA_0 reduction of f.T0 (partial: ceil(M / kTargetBlock) doubles).
template <typename Real>
hipError_t launch_fused(const SimArgs<Real>& a, const FusedArgs& f, double* partial, double* cva0, hipStream_t stream);
template <typename Real>
hipError_t launch_branch(const SimArgs<Real>& a, const BranchArgs& b, hipStream_t stream);
template <typename Real>
hipError_t launch_sample_rows(const SampleArgs<Real>& a, hipStream_t stream);
// Workspace of launch_branch_stats (FP64 block partials of the kBranchStats statistics).
size_t branch_stats_bytes(int64_t M);
// out[kBranchStats] = path means of the statistics; phi may be null (phi = 0).
hipError_t launch_branch_stats(int64_t M, int32_t B, bool phi_fp32, const void* phi, const double* xi,
                               double* partial, double* out, hipStream_t stream);
hipError_t launch_philox_fill(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3,
                              int64_t k_begin, int64_t count, uint32_t* out, hipStream_t s);
template <typename Real>
hipError_t launch_normals_fill(uint64_t seed, int64_t path_begin, int64_t count, int32_t step,
                               int32_t n_z, Real* out, hipStream_t s);

}  // namespace hsim
