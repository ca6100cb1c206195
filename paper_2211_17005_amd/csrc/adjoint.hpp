// Internal interface of the sensitivity kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sim.hpp"

namespace hsim {

// Offsets of the parameter vector: r0[n_e] fx0[n_e-1] lambda0[C] a[n_e] b[n_e] sigma_r[n_e]
// sigma_fx[n_e-1] kappa[C] theta[C] nu[C].
struct AdjParams {
  int off_r0, off_fx0, off_l0, off_a, off_b, off_sr, off_sx, off_kappa, off_theta, off_nu, n_params;
  __host__ __device__ static AdjParams make(int ne, int nc) {
    AdjParams p;
    p.off_r0 = 0;
    p.off_fx0 = ne;
    p.off_l0 = p.off_fx0 + ne - 1;
    p.off_a = p.off_l0 + nc;
    p.off_b = p.off_a + ne;
    p.off_sr = p.off_b + ne;
    p.off_sx = p.off_sr + ne;
    p.off_kappa = p.off_sx + ne - 1;
    p.off_theta = p.off_kappa + nc;
    p.off_nu = p.off_theta + nc;
    p.n_params = p.off_nu + nc;
    return p;
  }
};

struct AdjArgs {
  SimArgs<float> sim;            // tables and the forward outputs (features, I, Lam, D)
  int64_t ld;                    // row stride of the forward outputs (>= sim.M)
  const float* dlnA_da;          // [n_ccy][n+1] derivatives of the Vasicek coefficient tables
  const float* dlnA_db;
  const float* dlnA_ds;
  const float* dB_da;
  float dlvl_da[kMaxCcy], dlvl_ds[kMaxCcy], dlvl_dsx[kMaxCcy];   // Q^0 level b - rho s sx / a
  float sigma_fx[kMaxCcy], fx0[kMaxCcy], theta[kMaxCpty];
  float dt_f, sqrt_dt;
  AdjParams par;
  double* grad_path;             // [n_params + 1][M]: per-path gradient rows, then J
  double* grad_out;              // [n_params] or null
  double* cva0_out;              // one double
};

// with_grad = false: CVA_0 only (the credit sweep computes J; no market sweep, no gradient)
hipError_t launch_adjoint(const AdjArgs& a, bool with_grad, hipStream_t stream);

}  // namespace hsim
