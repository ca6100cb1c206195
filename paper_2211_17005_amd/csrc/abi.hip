// C-ABI layer of libhsim: argument validation, parameter tables, launches.
//
// Validation is pure host code and runs before any launch, so every error path can be
// exercised without a device.  Parameter tables (Cholesky factor of the market
// correlation, Vasicek zero-coupon coefficients on the pricing-date lattice, bucketed
// swap weights) are built on the host in FP64, converted to the simulation precision and
// kept in a per-device cache keyed by their bytes; a table is uploaded once and reused
// by every later call with the same parameters.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hsim.h"
#include "sim.hpp"
#include "abi_internal.hpp"

namespace hsim {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int device_error(hipError_t e, const char* what) {
  return fail(HSIM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------- validation
int check_market(const hsim_market* m) {
  if (!m) return fail(HSIM_EINVAL, "market is NULL");
  if (m->n_ccy < 1 || m->n_ccy > HSIM_MAX_CCY) return fail(HSIM_ERANGE, "n_ccy=%d out of [1,%d]", m->n_ccy, HSIM_MAX_CCY);
  if (m->n_cpty < 1 || m->n_cpty > HSIM_MAX_CPTY) return fail(HSIM_ERANGE, "n_cpty=%d out of [1,%d]", m->n_cpty, HSIM_MAX_CPTY);
  if (!m->a || !m->b || !m->sigma_r || !m->r0 || !m->corr || !m->kappa || !m->theta || !m->nu ||
      !m->lambda0 || !m->lgd)
    return fail(HSIM_EINVAL, "market has a NULL array");
  if (m->n_ccy > 1 && (!m->sigma_fx || !m->fx0)) return fail(HSIM_EINVAL, "market FX arrays are NULL");
  for (int e = 0; e < m->n_ccy; ++e) {
    if (!(m->a[e] > 0.0) || !std::isfinite(m->a[e])) return fail(HSIM_EINVAL, "a[%d] must be > 0", e);
    if (!(m->sigma_r[e] >= 0.0) || !std::isfinite(m->sigma_r[e])) return fail(HSIM_EINVAL, "sigma_r[%d] must be >= 0", e);
    if (!std::isfinite(m->b[e]) || !std::isfinite(m->r0[e])) return fail(HSIM_EINVAL, "b/r0[%d] not finite", e);
  }
  for (int e = 1; e < m->n_ccy; ++e) {
    if (!(m->sigma_fx[e - 1] >= 0.0) || !std::isfinite(m->sigma_fx[e - 1])) return fail(HSIM_EINVAL, "sigma_fx[%d] must be >= 0", e - 1);
    if (!(m->fx0[e - 1] > 0.0) || !std::isfinite(m->fx0[e - 1])) return fail(HSIM_EINVAL, "fx0[%d] must be > 0", e - 1);
  }
  for (int c = 0; c < m->n_cpty; ++c) {
    if (!(m->kappa[c] >= 0.0) || !(m->theta[c] >= 0.0) || !(m->nu[c] >= 0.0) || !(m->lambda0[c] >= 0.0) ||
        !std::isfinite(m->kappa[c]) || !std::isfinite(m->theta[c]) || !std::isfinite(m->nu[c]) ||
        !std::isfinite(m->lambda0[c]))
      return fail(HSIM_EINVAL, "CIR parameters of counterparty %d must be finite and >= 0", c);
    if (!std::isfinite(m->lgd[c])) return fail(HSIM_EINVAL, "lgd[%d] not finite", c);
  }
  const int d = 2 * m->n_ccy - 1;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const double v = m->corr[i * d + j];
      if (!std::isfinite(v) || std::fabs(v - m->corr[j * d + i]) > 1e-12)
        return fail(HSIM_EINVAL, "correlation is not symmetric/finite at (%d,%d)", i, j);
      if (i == j && std::fabs(v - 1.0) > 1e-12) return fail(HSIM_EINVAL, "correlation diagonal (%d) != 1", i);
    }
  return HSIM_OK;
}

int check_grid(const hsim_grid* g) {
  if (!g) return fail(HSIM_EINVAL, "grid is NULL");
  if (g->n_dates < 1 || g->n_dates > HSIM_MAX_DATES) return fail(HSIM_ERANGE, "n_dates=%d out of [1,%d]", g->n_dates, HSIM_MAX_DATES);
  if (g->n_sub < 1) return fail(HSIM_EINVAL, "n_sub must be >= 1");
  if ((int64_t)g->n_dates * g->n_sub >= (int64_t)1 << 31) return fail(HSIM_ERANGE, "too many sub-steps");
  if (!(g->horizon > 0.0) || !std::isfinite(g->horizon)) return fail(HSIM_EINVAL, "horizon must be > 0");
  return HSIM_OK;
}

int check_book(const hsim_portfolio* p, const hsim_market* m, const hsim_grid* g, int* q_out, int* P_out) {
  if (!p) return fail(HSIM_EINVAL, "portfolio is NULL");
  if (p->n_swaps < 1) return fail(HSIM_EINVAL, "n_swaps must be >= 1");
  if (!p->ccy || !p->cpty || !p->periods || !p->notional || !p->fixed_rate || !p->payer)
    return fail(HSIM_EINVAL, "portfolio has a NULL array");
  if (!(p->delta > 0.0)) return fail(HSIM_EINVAL, "delta must be > 0");
  const double qd = g->n_dates * p->delta / g->horizon;
  const int q = (int)std::lround(qd);
  if (q < 1 || std::fabs(qd - q) > 1e-9) return fail(HSIM_EINVAL, "delta*n_dates/horizon=%g is not a whole number", qd);
  int P = 0;
  for (int s = 0; s < p->n_swaps; ++s) {
    if (p->ccy[s] < 0 || p->ccy[s] >= m->n_ccy) return fail(HSIM_EINVAL, "swap %d: currency %d out of range", s, p->ccy[s]);
    if (p->cpty[s] < 0 || p->cpty[s] >= m->n_cpty) return fail(HSIM_EINVAL, "swap %d: counterparty %d out of range", s, p->cpty[s]);
    if (p->periods[s] < 1 || p->periods[s] > HSIM_MAX_PERIODS) return fail(HSIM_ERANGE, "swap %d: periods %d out of [1,%d]", s, p->periods[s], HSIM_MAX_PERIODS);
    if ((int64_t)p->periods[s] * q > g->n_dates) return fail(HSIM_EINVAL, "swap %d matures after the horizon", s);
    if (!(p->notional[s] >= 0.0) || !std::isfinite(p->notional[s])) return fail(HSIM_EINVAL, "swap %d: notional must be >= 0", s);
    if (!std::isfinite(p->fixed_rate[s])) return fail(HSIM_EINVAL, "swap %d: fixed rate not finite", s);
    if (p->payer[s] != 1 && p->payer[s] != -1) return fail(HSIM_EINVAL, "swap %d: payer must be +1 or -1", s);
    if (p->periods[s] > P) P = p->periods[s];
  }
  *q_out = q;
  *P_out = P;
  return HSIM_OK;
}

int check_precision(int precision) {
  if (precision != HSIM_FP32 && precision != HSIM_FP64) return fail(HSIM_EINVAL, "unknown precision %d", precision);
  return HSIM_OK;
}

int check_paths(int64_t path_begin, int64_t M) {
  if (M < 1) return fail(HSIM_EINVAL, "M must be >= 1");
  if (path_begin < 0 || path_begin + M > ((int64_t)1 << 32)) return fail(HSIM_ERANGE, "path range exceeds 2^32");
  return HSIM_OK;
}

int check_nb(int32_t n_b, const int32_t* nb_block, int32_t block_paths) {
  if (nb_block) {
    if (block_paths < 64 || block_paths % 64 != 0) return fail(HSIM_EINVAL, "block_paths must be a positive multiple of 64");
  } else if (n_b < 1 || n_b > (1 << 24)) {
    return fail(HSIM_ERANGE, "n_b=%d out of [1, 2^24]", n_b);
  }
  return HSIM_OK;
}

// Cholesky-Banachiewicz; returns false if the matrix is not positive definite.
bool cholesky(const double* A, int d, std::vector<double>& L) {
  L.assign((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = A[i * d + j];
      for (int k = 0; k < j; ++k) s -= L[i * d + k] * L[j * d + k];
      if (i == j) {
        if (!(s > 1e-14)) return false;
        L[i * d + i] = std::sqrt(s);
      } else {
        L[i * d + j] = s / L[j * d + j];
      }
    }
  return true;
}

double vasicek_B(double a, double tau) { return -std::expm1(-a * tau) / a; }
double vasicek_lnA(double a, double b, double s, double tau) {
  const double B = vasicek_B(a, tau);
  return (b - s * s / (2.0 * a * a)) * (B - tau) - s * s * B * B / (4.0 * a);
}

// ---------------------------------------------------------------------------- table cache
struct TableCache {
  std::mutex mu;
  std::map<std::pair<int, std::string>, void*> entries;
};
TableCache& table_cache() {
  static TableCache c;
  return c;
}

int device_table(const std::vector<unsigned char>& blob, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e, "hipGetDevice");
  TableCache& c = table_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  auto key = std::make_pair(dev, std::string(blob.begin(), blob.end()));
  auto it = c.entries.find(key);
  if (it != c.entries.end()) {
    *out = it->second;
    return HSIM_OK;
  }
  void* p = nullptr;
  e = hipMalloc(&p, blob.size());
  if (e != hipSuccess) return device_error(e, "hipMalloc(table)");
  e = hipMemcpy(p, blob.data(), blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(p);
    return device_error(e, "hipMemcpy(table)");
  }
  c.entries.emplace(std::move(key), p);
  *out = p;
  return HSIM_OK;
}

template <typename Real>
int build_sim_args(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed,
                   int64_t path_begin, int64_t M, int feature_mode, SimArgs<Real>& a) {
  int rc = check_market(m);
  if (rc) return rc;
  if ((rc = check_grid(g))) return rc;
  int q = 0, P = 0;
  if ((rc = check_book(p, m, g, &q, &P))) return rc;
  if ((rc = check_paths(path_begin, M))) return rc;
  if (feature_mode != HSIM_FEAT_FACTORS && feature_mode != HSIM_FEAT_FACTORS_PLUS)
    return fail(HSIM_EINVAL, "unknown feature mode %d", feature_mode);
  if (!outer_supported(m->n_ccy, m->n_cpty))
    return fail(HSIM_EUNSUPPORTED, "no kernel built for n_ccy=%d, n_cpty=%d", m->n_ccy, m->n_cpty);
  const int NE = m->n_ccy, NC = m->n_cpty, n = g->n_dates;
  const int d = 2 * NE - 1;
  std::vector<double> L;
  if (!cholesky(m->corr, d, L)) return fail(HSIM_EINVAL, "correlation matrix is not positive definite");

  memset(&a, 0, sizeof(a));
  a.M = M;
  a.path_begin = (uint32_t)path_begin;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.n_ccy = NE;
  a.n_cpty = NC;
  a.n_dates = n;
  a.n_sub = g->n_sub;
  a.q = q;
  a.n_periods = P;
  a.feature_mode = feature_mode;
  a.n_feat = hsim_n_features(m, feature_mode);
  const double dt = g->horizon / ((double)n * g->n_sub);
  const double sq = std::sqrt(dt);
  a.dt = (Real)dt;
  a.half_dt = 0.5 * dt;
  const int ncoef = coef_size(NE, NC);
  std::vector<double> cf(ncoef, 0.0);
  const int o_rmul = 0, o_radd = NE, o_rvol = 2 * NE, o_xadd = 3 * NE, o_xvol = 3 * NE + (NE - 1);
  const int o_gadd = 3 * NE + 2 * (NE - 1), o_gkd = o_gadd + NC, o_gvol = o_gadd + 2 * NC;
  for (int e = 0; e < NE; ++e) {
    const double quanto = e > 0 ? m->corr[e * d + (NE + e - 1)] * m->sigma_r[e] * m->sigma_fx[e - 1] : 0.0;
    // a (b - r) - quanto = a (b - quanto / a - r): the Q^0 level of r^e
    cf[o_rmul + e] = m->a[e] * dt;
    cf[o_radd + e] = m->b[e] - quanto / m->a[e];
    cf[o_rvol + e] = m->sigma_r[e] * sq;
    a.r0[e] = (Real)m->r0[e];
  }
  for (int e = 1; e < NE; ++e) {
    cf[o_xadd + e - 1] = -0.5 * m->sigma_fx[e - 1] * m->sigma_fx[e - 1] * dt;
    cf[o_xvol + e - 1] = m->sigma_fx[e - 1] * sq;
    a.x0[e - 1] = (Real)std::log(m->fx0[e - 1]);
  }
  for (int c = 0; c < NC; ++c) {
    cf[o_gadd + c] = m->kappa[c] * m->theta[c] * dt;
    cf[o_gkd + c] = m->kappa[c] * dt;
    cf[o_gvol + c] = m->nu[c] * sq;
    a.g0[c] = (Real)m->lambda0[c];
    a.lgd[c] = (Real)m->lgd[c];
  }

  // device table: coef | chol | lnA | B | W1 | CW1 | CW2 | G
  const size_t n_coef = (size_t)ncoef;
  const size_t n_chol = (size_t)d * (d + 1) / 2;
  const size_t n_zc = (size_t)NE * (n + 1);
  const size_t n_w = (size_t)NC * NE * (P + 2);
  std::vector<Real> T(n_coef + n_chol + 2 * n_zc + 4 * n_w, (Real)0);
  for (int i = 0; i < ncoef; ++i) T[i] = (Real)cf[i];
  Real* chol = T.data() + n_coef;
  Real* lnA = chol + n_chol;
  Real* Bv = lnA + n_zc;
  Real* W1 = Bv + n_zc;
  Real* CW1 = W1 + n_w;
  Real* CW2 = CW1 + n_w;
  Real* G = CW2 + n_w;
  size_t o = 0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j <= i; ++j) chol[o++] = (Real)L[i * d + j];
  const double h = g->horizon / n;
  for (int e = 0; e < NE; ++e)
    for (int j = 0; j <= n; ++j) {
      lnA[e * (n + 1) + j] = (Real)vasicek_lnA(m->a[e], m->b[e], m->sigma_r[e], j * h);
      Bv[e * (n + 1) + j] = (Real)vasicek_B(m->a[e], j * h);
    }
  std::vector<double> w1(n_w, 0.0), w2(n_w, 0.0);
  for (int s = 0; s < p->n_swaps; ++s) {
    const size_t base = ((size_t)p->cpty[s] * NE + p->ccy[s]) * (P + 2);
    const double wn = p->payer[s] * p->notional[s];
    w1[base + p->periods[s]] += wn;
    w2[base + p->periods[s]] += wn * p->delta * p->fixed_rate[s];
  }
  for (int c = 0; c < NC; ++c)
    for (int e = 0; e < NE; ++e) {
      const size_t base = ((size_t)c * NE + e) * (P + 2);
      double s1 = 0.0, s2 = 0.0;
      for (int pp = P + 1; pp >= 0; --pp) {
        s1 += w1[base + pp];
        s2 += w2[base + pp];
        W1[base + pp] = (Real)w1[base + pp];
        CW1[base + pp] = (Real)s1;
        CW2[base + pp] = (Real)s2;
        G[base + pp] = (Real)(w1[base + pp] + s2);
      }
    }
  std::vector<unsigned char> blob(T.size() * sizeof(Real));
  memcpy(blob.data(), T.data(), blob.size());
  void* dev = nullptr;
  if ((rc = device_table(blob, &dev))) return rc;
  Real* base = (Real*)dev;
  a.coef = base;
  a.chol = base + n_coef;
  a.lnA = a.chol + n_chol;
  a.Bv = a.lnA + n_zc;
  a.W1 = a.Bv + n_zc;
  a.CW1 = a.W1 + n_w;
  a.CW2 = a.CW1 + n_w;
  a.G = a.CW2 + n_w;
  return HSIM_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename Real>
int run_outer(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed,
              int64_t path_begin, int64_t M, int feature_mode, void* features, double* I, double* Lam,
              void* D, void* MtM, hipStream_t stream, bool fp32_integrals = false) {
  SimArgs<Real> a;
  int rc = build_sim_args<Real>(m, p, g, seed, path_begin, M, feature_mode, a);
  if (rc) return rc;
  a.features = (Real*)features;
  a.I = I;
  a.Lam = Lam;
  a.D = (Real*)D;
  a.MtM = (Real*)MtM;
  hipError_t e = launch_outer<Real>(a, stream, fp32_integrals);
  if (e != hipSuccess) return device_error(e, "outer kernel launch");
  return HSIM_OK;
}

template <typename Real>
int run_targets(const hsim_grid* g, int32_t n_cpty, int64_t M, int32_t n_b, const int32_t* nb_block,
                int32_t block_paths, const double* I, const void* D, const int32_t* counts, void* T,
                double* cva0, void* ws, size_t ws_bytes, hipStream_t stream, float* weight = nullptr) {
  const size_t need = hsim_workspace_bytes(HSIM_OP_TARGETS, nullptr, g, M, 0);
  if (ws_bytes < need || !ws) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, need);
  TargetArgs<Real> a;
  a.M = M;
  a.n_dates = g->n_dates;
  a.n_cpty = n_cpty;
  a.n_b = n_b;
  a.nb_block = nb_block;
  a.block_paths = block_paths;
  a.I = I;
  a.D = (const Real*)D;
  a.counts = counts;
  a.Lam = nullptr;
  a.T = (Real*)T;
  a.weight = weight;
  a.partial = (double*)ws;
  a.cva0 = cva0;
  hipError_t e = launch_targets<Real>(a, stream);
  if (e != hipSuccess) return device_error(e, "targets kernel launch");
  return HSIM_OK;
}

// ---------------------------------------------------------------------------- static scratch
// Device memory of hsim_targets_cva_noalloc: the FP64 block partials of CVA_0 for up to
// kNoAllocMaxPaths paths.  Every GPU the library runs on holds its own copy of the array until the
// process ends; host code reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is a host-side stand-in, not a device address).
constexpr int64_t kNoAllocMaxPaths = (int64_t)1 << 24;
constexpr size_t kScratchDoubles = (size_t)((kNoAllocMaxPaths + kTargetBlock - 1) / kTargetBlock);
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];

// Address of `scratch` on the current device, looked up once per device with that device current.
int scratch_address(double** out) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(HSIM_ERANGE, "device ordinal %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(HSIM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    addr[dev] = (double*)p;
  }
  *out = addr[dev];
  return HSIM_OK;
}

}  // namespace hsim

using namespace hsim;

extern "C" {

int hsim_abi_version(void) { return HSIM_ABI_VERSION; }

const char* hsim_last_error(void) { return g_last_error.c_str(); }

int hsim_n_features(const hsim_market* m, int feature_mode) {
  if (!m) return fail(HSIM_EINVAL, "market is NULL");
  const int d = m->n_ccy + (m->n_ccy - 1) + m->n_cpty;
  return feature_mode == HSIM_FEAT_FACTORS_PLUS ? d + 2 : d;
}

int hsim_par_rates(const hsim_market* m, const hsim_portfolio* p, double* par_out) {
  int rc = check_market(m);
  if (rc) return rc;
  if (!p || !par_out || !p->ccy || !p->periods || p->n_swaps < 1 || !(p->delta > 0.0))
    return fail(HSIM_EINVAL, "bad portfolio or output");
  for (int s = 0; s < p->n_swaps; ++s) {
    const int e = p->ccy[s];
    if (e < 0 || e >= m->n_ccy || p->periods[s] < 1) return fail(HSIM_EINVAL, "swap %d out of range", s);
    double ann = 0.0;
    for (int k = 1; k <= p->periods[s]; ++k) {
      const double tau = k * p->delta;
      ann += std::exp(vasicek_lnA(m->a[e], m->b[e], m->sigma_r[e], tau) - vasicek_B(m->a[e], tau) * m->r0[e]);
    }
    const double T = p->periods[s] * p->delta;
    const double zT = std::exp(vasicek_lnA(m->a[e], m->b[e], m->sigma_r[e], T) - vasicek_B(m->a[e], T) * m->r0[e]);
    par_out[s] = (1.0 - zT) / (p->delta * ann);
  }
  return HSIM_OK;
}

int hsim_philox_fill(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t k_begin,
                     int64_t count, uint32_t* out_dev, void* stream) {
  if (!out_dev) return fail(HSIM_EINVAL, "out_dev is NULL");
  if (count < 1 || k_begin < 0 || k_begin + count > ((int64_t)1 << 32)) return fail(HSIM_ERANGE, "bad counter range");
  hipError_t e = launch_philox_fill(seed, c1, c2, c3, k_begin, count, out_dev, (hipStream_t)stream);
  return e == hipSuccess ? HSIM_OK : device_error(e, "philox fill");
}

int hsim_normals_fill(uint64_t seed, int64_t path_begin, int64_t count, int32_t s, int32_t n_z,
                      int precision, void* out_dev, void* stream) {
  if (!out_dev) return fail(HSIM_EINVAL, "out_dev is NULL");
  int rc = check_precision(precision);
  if (rc) return rc;
  if ((rc = check_paths(path_begin, count))) return rc;
  if (n_z < 1 || n_z > 4 * 64 || s < 0) return fail(HSIM_EINVAL, "bad n_z or sub-step");
  hipError_t e = precision == HSIM_FP32
                     ? launch_normals_fill<float>(seed, path_begin, count, s, n_z, (float*)out_dev, (hipStream_t)stream)
                     : launch_normals_fill<double>(seed, path_begin, count, s, n_z, (double*)out_dev, (hipStream_t)stream);
  return e == hipSuccess ? HSIM_OK : device_error(e, "normals fill");
}

int hsim_outer_paths(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed,
                     int64_t path_begin, int64_t M, int precision, int feature_mode, void* features_dev,
                     double* I_dev, double* Lambda_dev, void* D_dev, void* MtM_dev, void* stream) {
  const bool plain = precision == HSIM_FP32_PLAIN;
  int rc = plain ? HSIM_OK : check_precision(precision);
  if (rc) return rc;
  if (!I_dev || !Lambda_dev || !D_dev) return fail(HSIM_EINVAL, "I, Lambda and D outputs must not be NULL");
  return precision != HSIM_FP64
             ? run_outer<float>(m, p, g, seed, path_begin, M, feature_mode, features_dev, I_dev, Lambda_dev,
                                D_dev, MtM_dev, (hipStream_t)stream, plain)
             : run_outer<double>(m, p, g, seed, path_begin, M, feature_mode, features_dev, I_dev, Lambda_dev,
                                 D_dev, MtM_dev, (hipStream_t)stream);
}

int hsim_inner_defaults(const hsim_grid* g, int32_t n_cpty, uint64_t seed, int64_t path_begin, int64_t M,
                        int32_t n_b, const int32_t* n_b_per_block, int32_t block_paths,
                        const double* Lambda_dev, int32_t* counts_dev, void* workspace_dev, size_t ws_bytes,
                        void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_paths(path_begin, M))) return rc;
  if ((rc = check_nb(n_b, n_b_per_block, block_paths))) return rc;
  if (n_cpty < 1 || n_cpty > HSIM_MAX_CPTY) return fail(HSIM_ERANGE, "n_cpty out of range");
  if (!Lambda_dev || !counts_dev) return fail(HSIM_EINVAL, "Lambda and counts must not be NULL");
  if ((size_t)2 * (g->n_dates + 1) * kInnerBlock * 4 > 64 * 1024)
    return fail(HSIM_ERANGE, "n_dates too large for the inner kernel's LDS tile");
  InnerArgs a;
  a.M = M;
  a.path_begin = (uint32_t)path_begin;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.n_dates = g->n_dates;
  a.n_cpty = n_cpty;
  a.n_b = n_b;
  a.nb_block = n_b_per_block;
  a.block_paths = block_paths;
  a.Lam = Lambda_dev;
  a.counts = counts_dev;
  a.order = nullptr;
  if (n_b_per_block) {                   // uneven n_b: longest-first persistent schedule
    const size_t need = align256(inner_order_bytes(M));
    if (!workspace_dev || ws_bytes < need)
      return fail(HSIM_ENOWS, "uneven n_b needs a workspace of %zu bytes (got %zu)", need, ws_bytes);
    a.order = (int32_t*)workspace_dev;
  }
  hipError_t e = launch_inner(a, (hipStream_t)stream);
  return e == hipSuccess ? HSIM_OK : device_error(e, "inner kernel launch");
}

int hsim_targets_cva(const hsim_grid* g, int32_t n_cpty, int64_t M, int32_t n_b, const int32_t* n_b_per_block,
                     int32_t block_paths, int precision, const double* I_dev, const void* D_dev,
                     const int32_t* counts_dev, void* target_dev, double* cva0_dev, void* workspace_dev,
                     size_t ws_bytes, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if ((rc = check_paths(0, M))) return rc;
  if ((rc = check_nb(n_b, n_b_per_block, block_paths))) return rc;
  if (n_cpty < 1 || n_cpty > HSIM_MAX_CPTY) return fail(HSIM_ERANGE, "n_cpty out of range");
  if (!I_dev || !D_dev || !counts_dev || !target_dev || !cva0_dev) return fail(HSIM_EINVAL, "NULL array");
  return precision == HSIM_FP32
             ? run_targets<float>(g, n_cpty, M, n_b, n_b_per_block, block_paths, I_dev, D_dev, counts_dev,
                                  target_dev, cva0_dev, workspace_dev, ws_bytes, (hipStream_t)stream)
             : run_targets<double>(g, n_cpty, M, n_b, n_b_per_block, block_paths, I_dev, D_dev, counts_dev,
                                   target_dev, cva0_dev, workspace_dev, ws_bytes, (hipStream_t)stream);
}

int hsim_targets_cva_noalloc(const hsim_grid* g, int32_t n_cpty, int64_t M, int32_t n_b,
                             const int32_t* n_b_per_block, int32_t block_paths, int precision, const double* I_dev,
                             const void* D_dev, const int32_t* counts_dev, void* target_dev, double* cva0_dev,
                             void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if ((rc = check_paths(0, M))) return rc;
  if (M > kNoAllocMaxPaths)
    return fail(HSIM_ERANGE, "M = %lld exceeds the %lld paths of the static scratch (use hsim_targets_cva)",
                (long long)M, (long long)kNoAllocMaxPaths);
  if ((rc = check_nb(n_b, n_b_per_block, block_paths))) return rc;
  if (n_cpty < 1 || n_cpty > HSIM_MAX_CPTY) return fail(HSIM_ERANGE, "n_cpty out of range");
  if (!I_dev || !D_dev || !counts_dev || !target_dev || !cva0_dev) return fail(HSIM_EINVAL, "NULL array");
  double* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  const size_t ws_bytes = kScratchDoubles * sizeof(double);
  return precision == HSIM_FP32
             ? run_targets<float>(g, n_cpty, M, n_b, n_b_per_block, block_paths, I_dev, D_dev, counts_dev,
                                  target_dev, cva0_dev, ws, ws_bytes, (hipStream_t)stream)
             : run_targets<double>(g, n_cpty, M, n_b, n_b_per_block, block_paths, I_dev, D_dev, counts_dev,
                                   target_dev, cva0_dev, ws, ws_bytes, (hipStream_t)stream);
}

int hsim_sample_rows(const hsim_grid* g, int32_t n_cpty, int32_t d, uint64_t seed, int64_t path_begin, int64_t M,
                     int32_t n_b, int precision, const void* features_dev, const double* I_dev,
                     const double* Lambda_dev, const void* D_dev, float* X_dev, float* Y_dev, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if ((rc = check_paths(path_begin, M))) return rc;
  if (n_cpty < 1 || n_cpty > HSIM_MAX_CPTY) return fail(HSIM_ERANGE, "n_cpty out of range");
  if (d < 0 || d > 4096) return fail(HSIM_EINVAL, "bad feature count %d", d);
  if (n_b < 1 || n_b > (1 << 24)) return fail(HSIM_ERANGE, "n_b %d outside [1, 2^24]", n_b);
  if (M * (int64_t)n_b > ((int64_t)1 << 31)) return fail(HSIM_ERANGE, "M * n_b exceeds 2^31 samples");
  if ((d > 0 && !features_dev) || !I_dev || !Lambda_dev || !D_dev || !X_dev || !Y_dev)
    return fail(HSIM_EINVAL, "NULL array");
  auto run = [&](auto tag) -> int {
    using Real = decltype(tag);
    SampleArgs<Real> a;
    a.M = M;
    a.path_begin = (uint32_t)path_begin;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.n_dates = g->n_dates;
    a.n_cpty = n_cpty;
    a.d = d;
    a.n_b = n_b;
    a.features = (const Real*)features_dev;
    a.I = I_dev;
    a.Lam = Lambda_dev;
    a.D = (const Real*)D_dev;
    a.X = X_dev;
    a.Y = Y_dev;
    const hipError_t e = launch_sample_rows<Real>(a, (hipStream_t)stream);
    return e == hipSuccess ? HSIM_OK : device_error(e, "sample rows launch");
  };
  return precision == HSIM_FP32 ? run(0.0f) : run(0.0);
}

int hsim_targets_alive(const hsim_grid* g, int64_t M, int32_t n_b, const int32_t* n_b_per_block, int32_t block_paths,
                       int precision, const double* I_dev, const void* D_dev, const int32_t* counts_dev,
                       void* target_dev, float* weight_dev, double* cva0_dev, void* workspace_dev, size_t ws_bytes,
                       void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if ((rc = check_paths(0, M))) return rc;
  if ((rc = check_nb(n_b, n_b_per_block, block_paths))) return rc;
  if (!I_dev || !D_dev || !counts_dev || !target_dev || !weight_dev || !cva0_dev)
    return fail(HSIM_EINVAL, "NULL array");
  return precision == HSIM_FP32
             ? run_targets<float>(g, 1, M, n_b, n_b_per_block, block_paths, I_dev, D_dev, counts_dev, target_dev,
                                  cva0_dev, workspace_dev, ws_bytes, (hipStream_t)stream, weight_dev)
             : run_targets<double>(g, 1, M, n_b, n_b_per_block, block_paths, I_dev, D_dev, counts_dev, target_dev,
                                   cva0_dev, workspace_dev, ws_bytes, (hipStream_t)stream, weight_dev);
}

int hsim_targets_intensity(const hsim_grid* g, int32_t n_cpty, int64_t M, int precision, const double* I_dev,
                           const double* Lambda_dev, const void* D_dev, void* target_dev, double* cva0_dev,
                           void* workspace_dev, size_t ws_bytes, void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if ((rc = check_paths(0, M))) return rc;
  if (n_cpty < 1 || n_cpty > HSIM_MAX_CPTY) return fail(HSIM_ERANGE, "n_cpty out of range");
  if (!I_dev || !Lambda_dev || !D_dev || !target_dev || !cva0_dev) return fail(HSIM_EINVAL, "NULL array");
  const size_t need = hsim_workspace_bytes(HSIM_OP_TARGETS, nullptr, g, M, 0);
  if (ws_bytes < need || !workspace_dev) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, need);
  auto run = [&](auto tag) -> int {
    using Real = decltype(tag);
    TargetArgs<Real> a;
    memset(&a, 0, sizeof(a));
    a.M = M;
    a.n_dates = g->n_dates;
    a.n_cpty = n_cpty;
    a.n_b = 1;
    a.I = I_dev;
    a.D = (const Real*)D_dev;
    a.Lam = Lambda_dev;
    a.T = (Real*)target_dev;
    a.partial = (double*)workspace_dev;
    a.cva0 = cva0_dev;
    const hipError_t e = launch_targets<Real>(a, (hipStream_t)stream);
    return e == hipSuccess ? HSIM_OK : device_error(e, "targets kernel launch");
  };
  return precision == HSIM_FP32 ? run(0.0f) : run(0.0);
}

int hsim_branch_cva(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed,
                    int64_t path_begin, int64_t M, int32_t date, int32_t n_branch, int precision, double* xi_dev,
                    void* stream) {
  int rc = check_precision(precision);
  if (rc) return rc;
  if (!xi_dev) return fail(HSIM_EINVAL, "xi_dev is NULL");
  if ((rc = check_grid(g))) return rc;
  if (date < 0 || date > g->n_dates) return fail(HSIM_EINVAL, "branching date %d outside [0, %d]", date, g->n_dates);
  if (n_branch < 1 || n_branch > HSIM_MAX_BRANCH) return fail(HSIM_ERANGE, "n_branch %d outside [1, %d]", n_branch, HSIM_MAX_BRANCH);
  if (M > 0 && M * (int64_t)n_branch > ((int64_t)1 << 31))
    return fail(HSIM_ERANGE, "M * n_branch = %lld exceeds 2^31", (long long)(M * (int64_t)n_branch));
  auto run = [&](auto tag) -> int {
    using Real = decltype(tag);
    SimArgs<Real> a;
    const int r = build_sim_args<Real>(m, p, g, seed, path_begin, M, HSIM_FEAT_FACTORS, a);
    if (r) return r;
    BranchArgs b;
    b.date = date;
    b.n_branch = n_branch;
    b.xi = xi_dev;
    const hipError_t e = launch_branch<Real>(a, b, (hipStream_t)stream);
    return e == hipSuccess ? HSIM_OK : device_error(e, "branch kernel launch");
  };
  return precision == HSIM_FP32 ? run(0.0f) : run(0.0);
}

int hsim_branch_errors(int64_t M, int32_t n_branch, int precision, const void* phi_dev, const double* xi_dev,
                       double* out_dev, void* workspace_dev, size_t ws_bytes, void* stream) {
  int rc = check_precision(precision);
  if (rc) return rc;
  if ((rc = check_paths(0, M))) return rc;
  if (n_branch < 2 || n_branch > HSIM_MAX_BRANCH)
    return fail(HSIM_ERANGE, "n_branch %d outside [2, %d] (the twin estimator needs two continuations)", n_branch,
                HSIM_MAX_BRANCH);
  if (!xi_dev || !out_dev) return fail(HSIM_EINVAL, "NULL array");
  const size_t need = align256(branch_stats_bytes(M));
  if (ws_bytes < need || !workspace_dev) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, need);
  const hipError_t e = launch_branch_stats(M, n_branch, precision == HSIM_FP32, phi_dev, xi_dev,
                                           (double*)workspace_dev, out_dev, (hipStream_t)stream);
  return e == hipSuccess ? HSIM_OK : device_error(e, "branch statistics launch");
}

static size_t partial_bytes_of(int64_t M) {
  return align256(sizeof(double) * (size_t)((M + kTargetBlock - 1) / kTargetBlock));
}

size_t hsim_workspace_bytes(int op, const hsim_market* m, const hsim_grid* g, int64_t M, int precision) {
  if (M < 1) return 0;
  if (op == HSIM_OP_BRANCH) return align256(branch_stats_bytes(M));
  if (!g) return 0;
  const size_t n1 = (size_t)g->n_dates + 1;
  const size_t partial = partial_bytes_of(M);
  switch (op) {
    case HSIM_OP_INNER:
      return align256(inner_order_bytes(M));
    case HSIM_OP_TARGETS:
      return partial;
    case HSIM_OP_FUSED: {
      if (!m) return 0;
      const size_t C = (size_t)m->n_cpty;
      const size_t rs = precision == HSIM_FP64 ? sizeof(double) : sizeof(float);
      return align256(n1 * M * sizeof(double)) + align256(n1 * C * M * sizeof(double)) +
             align256(n1 * C * M * rs) + align256(n1 * C * M * sizeof(int32_t)) + partial +
             align256(inner_order_bytes(M));
    }
    case HSIM_OP_FUSED_LAUNCH: {
      if (!m) return 0;
      const size_t nc = n1 * (size_t)m->n_cpty, Mz = (size_t)M;
      const size_t rs = precision == HSIM_FP64 ? sizeof(double) : sizeof(float);
      return align256(Mz * nc * sizeof(uint32_t)) + align256(Mz * nc * rs) + align256(Mz * n1 * sizeof(double)) +
             align256(Mz * sizeof(double)) + partial;
    }
    default:
      return hsim_adjoint_workspace(op, m, g, M, precision);
  }
}

int hsim_fused(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed, int64_t path_begin,
               int64_t M, int32_t n_b, const int32_t* n_b_per_block, int32_t block_paths, int precision,
               int feature_mode, void* features_dev, void* target_dev, double* cva0_dev, void* workspace_dev,
               size_t ws_bytes, void* stream) {
  return hsim_fused_keep(m, p, g, seed, path_begin, M, n_b, n_b_per_block, block_paths, precision, feature_mode,
                         features_dev, target_dev, cva0_dev, 0, nullptr, nullptr, nullptr, workspace_dev, ws_bytes,
                         stream);
}

int hsim_fused_keep(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed,
                    int64_t path_begin, int64_t M, int32_t n_b, const int32_t* n_b_per_block, int32_t block_paths,
                    int precision, int feature_mode, void* features_dev, void* target_dev, double* cva0_dev,
                    int64_t n_keep, double* I_dev, double* Lambda_dev, void* D_dev, void* workspace_dev,
                    size_t ws_bytes, void* stream) {
  int rc = check_precision(precision);
  if (rc) return rc;
  if ((rc = check_market(m))) return rc;
  if ((rc = check_grid(g))) return rc;
  if ((rc = check_paths(path_begin, M))) return rc;
  if ((rc = check_nb(n_b, n_b_per_block, block_paths))) return rc;
  if (!target_dev || !cva0_dev) return fail(HSIM_EINVAL, "target and cva0 must not be NULL");
  if (n_keep < 0 || n_keep > M) return fail(HSIM_EINVAL, "n_keep=%lld out of [0, M=%lld]", (long long)n_keep, (long long)M);
  if (n_keep > 0 && (!I_dev || !Lambda_dev || !D_dev))
    return fail(HSIM_EINVAL, "I, Lambda and D must not be NULL when n_keep > 0");
  const size_t rs = precision == HSIM_FP64 ? sizeof(double) : sizeof(float);
  if (fused_lds_bytes(g->n_dates, m->n_cpty, rs) > kFusedMaxLds)
    return fail(HSIM_ERANGE, "n_dates x n_cpty too large for the fused kernel's LDS (%zu > %zu bytes): use "
                "hsim_inner_defaults_cva", fused_lds_bytes(g->n_dates, m->n_cpty, rs), kFusedMaxLds);
  const size_t need = hsim_workspace_bytes(HSIM_OP_FUSED_LAUNCH, m, g, M, precision);
  if (!workspace_dev || ws_bytes < need) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, need);
  const size_t n1 = (size_t)g->n_dates + 1, nc = n1 * (size_t)m->n_cpty, Mz = (size_t)M;
  char* w = (char*)workspace_dev;
  FusedArgs f;
  f.n_b = n_b;
  f.nb_block = n_b_per_block;
  f.block_paths = block_paths;
  f.K = (uint32_t*)w;
  w += align256(Mz * nc * sizeof(uint32_t));
  f.Dv = w;
  w += align256(Mz * nc * rs);
  f.Iv = (double*)w;
  w += align256(Mz * n1 * sizeof(double));
  f.T0 = (double*)w;
  w += align256(Mz * sizeof(double));
  double* partial = (double*)w;
  f.T = target_dev;
  f.n_keep = n_keep;
  f.I_keep = I_dev;
  f.Lam_keep = Lambda_dev;
  f.D_keep = D_dev;
  auto run = [&](auto tag) -> int {
    using Real = decltype(tag);
    SimArgs<Real> a;
    const int r = build_sim_args<Real>(m, p, g, seed, path_begin, M, feature_mode, a);
    if (r) return r;
    a.features = (Real*)features_dev;
    const hipError_t e = launch_fused<Real>(a, f, partial, cva0_dev, (hipStream_t)stream);
    return e == hipSuccess ? HSIM_OK : device_error(e, "fused simulation launch");
  };
  return precision == HSIM_FP32 ? run(0.0f) : run(0.0);
}

int hsim_inner_defaults_cva(const hsim_market* m, const hsim_portfolio* p, const hsim_grid* g, uint64_t seed,
                            int64_t path_begin, int64_t M, int32_t n_b, const int32_t* n_b_per_block,
                            int32_t block_paths, int precision, int feature_mode, void* features_dev,
                            void* target_dev, double* cva0_dev, void* workspace_dev, size_t ws_bytes,
                            void* stream) {
  // the plain FP32 form differs in the simulation's integrals only; the later stages read them
  // as FP32 runs do
  const int stage_precision = precision == HSIM_FP32_PLAIN ? HSIM_FP32 : precision;
  int rc = check_precision(stage_precision);
  if (rc) return rc;
  if ((rc = check_market(m))) return rc;
  if ((rc = check_grid(g))) return rc;
  if ((rc = check_paths(path_begin, M))) return rc;
  if ((rc = check_nb(n_b, n_b_per_block, block_paths))) return rc;
  if (!target_dev || !cva0_dev) return fail(HSIM_EINVAL, "target and cva0 must not be NULL");
  const size_t need = hsim_workspace_bytes(HSIM_OP_FUSED, m, g, M, precision);
  if (!workspace_dev || ws_bytes < need) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, need);
  const size_t n1 = (size_t)g->n_dates + 1, C = (size_t)m->n_cpty;
  const size_t rs = precision == HSIM_FP64 ? sizeof(double) : sizeof(float);
  char* w = (char*)workspace_dev;
  double* I = (double*)w;
  w += align256(n1 * M * sizeof(double));
  double* Lam = (double*)w;
  w += align256(n1 * C * M * sizeof(double));
  void* D = w;
  w += align256(n1 * C * M * rs);
  int32_t* cnt = (int32_t*)w;
  w += align256(n1 * C * M * sizeof(int32_t));
  void* partial = w;
  w += partial_bytes_of(M);
  void* order = w;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = hsim_outer_paths(m, p, g, seed, path_begin, M, precision, feature_mode, features_dev, I, Lam, D,
                             nullptr, s)))
    return rc;
  if ((rc = hsim_inner_defaults(g, m->n_cpty, seed, path_begin, M, n_b, n_b_per_block, block_paths, Lam, cnt,
                                order, align256(inner_order_bytes(M)), s)))
    return rc;
  return hsim_targets_cva(g, m->n_cpty, M, n_b, n_b_per_block, block_paths, stage_precision, I, D, cnt,
                          target_dev, cva0_dev, partial, hsim_workspace_bytes(HSIM_OP_TARGETS, m, g, M, precision), s);
}

}  // extern "C"
