// C-ABI of the sensitivities: cva_adjoint.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/hsim.h"
#include "abi_internal.hpp"
#include "adjoint.hpp"

using namespace hsim;

namespace {

struct AdjLayout {
  size_t feat, I, Lam, D, grad;
  size_t total;
};

AdjLayout adj_layout(const hsim_market* m, const hsim_grid* g, int64_t M) {
  const size_t n1 = (size_t)g->n_dates + 1, C = (size_t)m->n_cpty;
  const size_t d = (size_t)(2 * m->n_ccy - 1 + m->n_cpty);
  const size_t P = (size_t)AdjParams::make(m->n_ccy, m->n_cpty).n_params;
  AdjLayout L;
  L.feat = 0;
  L.I = L.feat + align256(n1 * d * M * sizeof(float));
  L.Lam = L.I + align256(n1 * M * sizeof(double));
  L.D = L.Lam + align256(n1 * C * M * sizeof(double));
  L.grad = L.D + align256(n1 * C * M * sizeof(float));
  L.total = L.grad + align256((P + 1) * M * sizeof(double));
  return L;
}

// Vasicek coefficient tables and their derivatives in (a, b, sigma) on the lattice tau_j = j h.
void vasicek_derivs(double a, double b, double s, double tau, double* dlA_da, double* dlA_db, double* dlA_ds,
                    double* dB_da) {
  const double e = std::exp(-a * tau);
  const double B = -std::expm1(-a * tau) / a;
  const double Ba = (tau * e - B) / a;
  const double k = b - s * s / (2.0 * a * a);
  *dlA_db = B - tau;
  *dlA_ds = -s / (a * a) * (B - tau) - s * B * B / (2.0 * a);
  *dlA_da = s * s / (a * a * a) * (B - tau) + k * Ba - s * s * B * Ba / (2.0 * a) + s * s * B * B / (4.0 * a * a);
  *dB_da = Ba;
}

}  // namespace

size_t hsim_adjoint_workspace(int op, const hsim_market* m, const hsim_grid* g, int64_t M, int precision) {
  (void)precision;
  if (op != HSIM_OP_ADJOINT || !m || !g || M < 1) return 0;
  return adj_layout(m, g, M).total;
}

extern "C" {

int hsim_n_params(const hsim_market* m) {
  if (!m) return fail(HSIM_EINVAL, "market is NULL");
  return AdjParams::make(m->n_ccy, m->n_cpty).n_params;
}

}  // extern "C"

namespace {

// Forward outputs handed in by the caller (features with the market factors first, row stride ld).
struct Forward {
  const float* features;
  int32_t n_feat;
  const double* I;
  const double* Lam;
  const float* D;
  int64_t ld;
};

int run_adjoint(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed, int64_t path_begin,
                int64_t M, const Forward* fw, double* cva0_dev, double* grad_dev, void* workspace_dev,
                size_t ws_bytes, void* stream) {
  AdjArgs a;
  memset(&a, 0, sizeof(a));
  int rc = build_sim_args<float>(m, p, g, seed, path_begin, M, HSIM_FEAT_FACTORS, a.sim);
  if (rc) return rc;
  if (!cva0_dev) return fail(HSIM_EINVAL, "cva0 must not be NULL");
  const AdjLayout L = adj_layout(m, g, M);
  const size_t need = fw ? L.total - L.grad : L.total;
  if (!workspace_dev || ws_bytes < need) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, need);
  char* w = (char*)workspace_dev;
  if (fw) {
    a.sim.features = const_cast<float*>(fw->features);
    a.sim.n_feat = fw->n_feat;
    a.sim.I = const_cast<double*>(fw->I);
    a.sim.Lam = const_cast<double*>(fw->Lam);
    a.sim.D = const_cast<float*>(fw->D);
    a.ld = fw->ld;
    a.grad_path = (double*)w;
  } else {
    a.sim.features = (float*)(w + L.feat);
    a.sim.I = (double*)(w + L.I);
    a.sim.Lam = (double*)(w + L.Lam);
    a.sim.D = (float*)(w + L.D);
    a.ld = M;
    a.grad_path = (double*)(w + L.grad);
  }
  a.sim.MtM = nullptr;
  a.grad_out = grad_dev;
  a.cva0_out = cva0_dev;
  const int NE = m->n_ccy, NC = m->n_cpty, n = g->n_dates;
  const int d = 2 * NE - 1;
  a.par = AdjParams::make(NE, NC);
  const double dt = g->horizon / ((double)n * g->n_sub);
  a.dt_f = (float)dt;
  a.sqrt_dt = (float)std::sqrt(dt);
  for (int e = 0; e < NE; ++e) {
    const double rho = e > 0 ? m->corr[e * d + (NE + e - 1)] : 0.0;
    const double sx = e > 0 ? m->sigma_fx[e - 1] : 0.0;
    a.dlvl_da[e] = (float)(rho * m->sigma_r[e] * sx / (m->a[e] * m->a[e]));
    a.dlvl_ds[e] = (float)(-rho * sx / m->a[e]);
    a.dlvl_dsx[e] = (float)(-rho * m->sigma_r[e] / m->a[e]);
  }
  for (int e = 1; e < NE; ++e) {
    a.sigma_fx[e - 1] = (float)m->sigma_fx[e - 1];
    a.fx0[e - 1] = (float)m->fx0[e - 1];
  }
  for (int c = 0; c < NC; ++c) a.theta[c] = (float)m->theta[c];
  // derivative tables of the zero-coupon coefficients
  const size_t nz = (size_t)NE * (n + 1);
  std::vector<float> T(4 * nz);
  const double h = g->horizon / n;
  for (int e = 0; e < NE; ++e)
    for (int j = 0; j <= n; ++j) {
      double da, db, ds, dB;
      vasicek_derivs(m->a[e], m->b[e], m->sigma_r[e], j * h, &da, &db, &ds, &dB);
      const size_t o = (size_t)e * (n + 1) + j;
      T[o] = (float)da;
      T[nz + o] = (float)db;
      T[2 * nz + o] = (float)ds;
      T[3 * nz + o] = (float)dB;
    }
  std::vector<unsigned char> blob(T.size() * sizeof(float));
  memcpy(blob.data(), T.data(), blob.size());
  void* dev = nullptr;
  if ((rc = device_table(blob, &dev))) return rc;
  a.dlnA_da = (const float*)dev;
  a.dlnA_db = a.dlnA_da + nz;
  a.dlnA_ds = a.dlnA_db + nz;
  a.dB_da = a.dlnA_ds + nz;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (!fw) {
    e = launch_outer<float>(a.sim, s);
    if (e != hipSuccess) return device_error(e, "forward simulation launch");
  }
  e = launch_adjoint(a, grad_dev != nullptr, s);
  if (e != hipSuccess) return device_error(e, "adjoint launch");
  return HSIM_OK;
}

}  // namespace

extern "C" {

int cva_adjoint(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed, int64_t path_begin,
                int64_t M, double* cva0_dev, double* grad_dev, void* workspace_dev, size_t ws_bytes, void* stream) {
  return run_adjoint(m, p, g, seed, path_begin, M, nullptr, cva0_dev, grad_dev, workspace_dev, ws_bytes, stream);
}

int cva_adjoint_forward(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed,
                        int64_t path_begin, int64_t M, int64_t ld, int32_t n_feat, const float* features_dev,
                        const double* I_dev, const double* Lambda_dev, const float* D_dev, double* cva0_dev,
                        double* grad_dev, void* workspace_dev, size_t ws_bytes, void* stream) {
  if (!m || !g) return fail(HSIM_EINVAL, "market and grid must not be NULL");
  if (ld < M) return fail(HSIM_EINVAL, "ld=%lld < M=%lld", (long long)ld, (long long)M);
  if (n_feat < 2 * m->n_ccy - 1 + m->n_cpty)
    return fail(HSIM_EINVAL, "n_feat=%d: the market factors (%d) must come first", n_feat, 2 * m->n_ccy - 1 + m->n_cpty);
  if (!features_dev || !I_dev || !Lambda_dev || !D_dev) return fail(HSIM_EINVAL, "forward outputs must not be NULL");
  const Forward fw{features_dev, n_feat, I_dev, Lambda_dev, D_dev, ld};
  return run_adjoint(m, p, g, seed, path_begin, M, &fw, cva0_dev, grad_dev, workspace_dev, ws_bytes, stream);
}

}  // extern "C"
