// Pilot moments of the oversimulation chooser (Section 3.3, Proposition p:heurisN).
//
// For every date i (one workgroup) and outer path k, the two pilot continuations of the
// pathwise loss are xi1 = T1 and xi2 = 2 T2 - T1 (T1, T2 the n_b = 1 and n_b = 2 targets of
// one seed: with common random numbers the first continuation of T2 is T1), the pointwise
// losses g = (xi - phi)^2 against the prediction phi (0 without one), and the workgroup
// reduces, in FP64 and a fixed order, E[g] and E[g^2] (both continuations pooled) and
// E[g g'].  R = E[g g'] - E[g]^2 and Q = E[g^2] - E[g g'] follow on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>

#include "../../include/hsim.h"
#include "abi_internal.hpp"

namespace hsim {
namespace {

constexpr int kMomBlock = 256;

template <typename Real>
__global__ __launch_bounds__(kMomBlock) void pilot_moments_kernel(int64_t M, const Real* T1, const Real* T2,
                                                                  const Real* pred, double* out) {
  __shared__ double red[3][kMomBlock];
  const int i = blockIdx.x;
  const Real* t1 = T1 + (int64_t)i * M;
  const Real* t2 = T2 + (int64_t)i * M;
  const Real* ph = pred ? pred + (int64_t)i * M : nullptr;
  double s1 = 0.0, s2 = 0.0, s12 = 0.0;
  for (int64_t k = threadIdx.x; k < M; k += kMomBlock) {
    const double x1 = (double)t1[k], x2 = 2.0 * (double)t2[k] - x1;
    const double phi = ph ? (double)ph[k] : 0.0;
    const double g1 = (x1 - phi) * (x1 - phi), g2 = (x2 - phi) * (x2 - phi);
    s1 += g1 + g2;
    s2 += g1 * g1 + g2 * g2;
    s12 += g1 * g2;
  }
  red[0][threadIdx.x] = s1;
  red[1][threadIdx.x] = s2;
  red[2][threadIdx.x] = s12;
  __syncthreads();
  for (int w = kMomBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double inv = 1.0 / (double)M;
    out[3 * i + 0] = 0.5 * red[0][0] * inv;
    out[3 * i + 1] = 0.5 * red[1][0] * inv;
    out[3 * i + 2] = red[2][0] * inv;
  }
}

}  // namespace
}  // namespace hsim

using namespace hsim;

extern "C" int hsim_oversim_moments(const hsim_grid* g, int64_t M, int precision, const void* T1_dev,
                                    const void* T2_dev, const void* pred_dev, double* moments_dev,
                                    void* stream) {
  int rc = check_grid(g);
  if (rc) return rc;
  if ((rc = check_precision(precision))) return rc;
  if (M < 1) return fail(HSIM_EINVAL, "M must be >= 1");
  if (!T1_dev || !T2_dev || !moments_dev) return fail(HSIM_EINVAL, "T1, T2 and moments must not be NULL");
  const dim3 grid((unsigned)(g->n_dates + 1));
  hipStream_t s = (hipStream_t)stream;
  if (precision == HSIM_FP32)
    hipLaunchKernelGGL(pilot_moments_kernel<float>, grid, dim3(kMomBlock), 0, s, M, (const float*)T1_dev,
                       (const float*)T2_dev, (const float*)pred_dev, moments_dev);
  else
    hipLaunchKernelGGL(pilot_moments_kernel<double>, grid, dim3(kMomBlock), 0, s, M, (const double*)T1_dev,
                       (const double*)T2_dev, (const double*)pred_dev, moments_dev);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HSIM_OK : device_error(e, "pilot moments launch");
}

extern "C" int hsim_oversim_cost_ratio(double t, double t_prime, double N, double N_prime, double* P_out) {
  if (!P_out) return fail(HSIM_EINVAL, "P_out is NULL");
  if (!(t > 0.0) || !(t_prime > 0.0)) return fail(HSIM_EINVAL, "times must be positive");
  if (N == N_prime || t == t_prime) return fail(HSIM_EINVAL, "the two runs must differ in n_b and in time");
  const double P = (t_prime * N - t * N_prime) / (t - t_prime);
  if (!(P > 0.0) || !std::isfinite(P))
    return fail(HSIM_EINVAL, "timings %.6g s (N=%g) and %.6g s (N'=%g) do not resolve a positive cost ratio", t,
                N, t_prime, N_prime);
  *P_out = P;
  return HSIM_OK;
}

extern "C" int hsim_oversim_choose(int32_t n_dates1, const double* mom, double P, double Psi, double* R_out,
                                   double* Q_out, double* Nstar_out, double* N_out, double* M_out) {
  if (n_dates1 < 1 || !mom || !N_out || !M_out) return fail(HSIM_EINVAL, "bad dates, moments or outputs");
  if (!(P > 0.0) || !(Psi > 0.0)) return fail(HSIM_EINVAL, "P and Psi must be positive");
  const double nan = std::numeric_limits<double>::quiet_NaN();
  double sum = 0.0;
  int defined = 0;
  for (int i = 0; i < n_dates1; ++i) {
    const double R = mom[3 * i + 2] - mom[3 * i + 0] * mom[3 * i + 0];
    const double Q = mom[3 * i + 1] - mom[3 * i + 2];
    double ns = nan;
    if (R > 0.0 && Q >= 0.0) {
      ns = std::sqrt(Q * P / R);
      sum += ns;
      ++defined;
    }
    if (R_out) R_out[i] = R;
    if (Q_out) Q_out[i] = Q;
    if (Nstar_out) Nstar_out[i] = ns;
  }
  const double N = defined ? std::fmax(1.0, sum / defined) : 1.0;
  *N_out = N;
  *M_out = Psi / (N + P);
  return defined;
}
