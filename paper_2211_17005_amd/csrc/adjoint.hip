// Sensitivities of CVA_0 (smoothed estimator) by hand-written tangent and adjoint sweeps.
//
// The differentiated quantity is, per outer path k,
//     J_k = sum_c sum_{j=1}^{n} D^c_j p^c_j,   p^c_j = exp(-Lambda^c_{j-1}) - exp(-Lambda^c_j),
// the exact inner conditional expectation of the pathwise loss (the indicator estimator is
// piecewise constant in Lambda, so its pathwise derivative in the credit parameters is 0);
// CVA_0 = mean_k J_k.  Market and credit are driven by independent Brownians, so
//   * the credit parameters (lambda0, kappa, theta, nu of every counterparty) reach J only
//     through p: a forward-mode sweep carries d(gamma, Lambda)/d(4 parameters) per
//     counterparty along the CIR Euler scheme (credit_kernel);
//   * the market parameters (r0, FX0, a, b, sigma_r, sigma_fx) reach J only through D: a
//     reverse sweep (market_adjoint_kernel) runs the Vasicek / log-FX Euler recursion
//     backwards.  That recursion is affine in the state, so each sub-step is inverted exactly
//     (up to rounding) from the state after it, re-drawing its normals from the counter-based
//     generator: every pricing-date interval starts from the state stored at its end by the
//     forward pass (the per-date feature rows are the checkpoints), and nothing per sub-step
//     is stored.  The pricing at each date is differentiated through the zero-coupon
//     coefficient tables, whose derivatives in (a, b, sigma_r) are tabulated on the host.
// Per-path gradients go to a [P+1][M] buffer that a fixed-order reduction averages.
#include <hip/hip_runtime.h>

#include <mutex>

#include "philox.hpp"
#include "sim.hpp"
#include "adjoint.hpp"

namespace hsim {

// ------------------------------------------------------------------------------------------
// credit: CIR tangents (forward mode) and J
// ------------------------------------------------------------------------------------------
template <int NE, int NC>
__global__ __launch_bounds__(kOuterBlock) __attribute__((amdgpu_waves_per_eu(2)))
void credit_kernel(const AdjArgs a) {
  constexpr int DW = 2 * NE - 1;
  using CL = CoefLayout<NE, NC>;
  const SimArgs<float>& s = a.sim;
  const int64_t kl = (int64_t)blockIdx.x * kOuterBlock + threadIdx.x;
  if (kl >= s.M) return;
  const uint32_t k = s.path_begin + (uint32_t)kl;
  const int64_t M = s.M;
  const int n = s.n_dates;

  float g[NC], gc[NC];
  double Lam[NC], Sprev[NC];
  float dg[NC][4], dL[NC][4], dSprev[NC][4], gr[NC][4];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    g[c] = s.g0[c];
    gc[c] = 0.0f;
    Lam[c] = 0.0;
    Sprev[c] = 1.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dg[c][q] = q == 0 ? 1.0f : 0.0f;     // d gamma_0 / d lambda0 = 1
      dL[c][q] = 0.0f;
      dSprev[c][q] = 0.0f;
      gr[c][q] = 0.0f;
    }
  }
  double J = 0.0;
  const float sqdt = a.sqrt_dt;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < s.n_sub; ++j) {
      asm volatile("" ::: "memory");
      const float* cf = s.coef;
      const double hdt = s.half_dt;
      const uint32_t st = (uint32_t)(i * s.n_sub + j);
#pragma unroll
      for (int gcall = DW / 4; gcall <= (DW + NC - 1) / 4; ++gcall) {
        float z[4];
        normals4<float>(k, st, (uint32_t)gcall, s.key0, s.key1, z);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int f = 4 * gcall + t;
          if (f < DW || f >= DW + NC) continue;
          const int c = f - DW;
          const float kdt = cf[CL::g_kd + c], gadd = cf[CL::g_add + c], gvol = cf[CL::g_vol + c];
          const bool act = g[c] > 0.0f;
          const float gp = act ? g[c] : 0.0f;
          const float sq = sqrtf(gp);
          const float inc = gadd - kdt * gp + gvol * sq * z[t] + gc[c];
          const float gs = g[c] + inc;
          gc[c] = inc - (gs - g[c]);
          g[c] = gs;
          const bool actn = g[c] > 0.0f;
          const float gn = actn ? g[c] : 0.0f;
          Lam[c] += hdt * ((double)gp + (double)gn);
          // tangents: explicit parameter derivatives of the increment
          const float dsq_fac = (act && gp > 0.0f) ? gvol * z[t] * 0.5f / sq : 0.0f;
          const float ex[4] = {0.0f, a.dt_f * (a.theta[c] - gp), kdt, sqdt * sq * z[t]};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float dgp = act ? dg[c][q] : 0.0f;
            const float dnew = dg[c][q] - kdt * dgp + dsq_fac * dgp + ex[q];
            dg[c][q] = dnew;
            const float dgn = actn ? dnew : 0.0f;
            dL[c][q] += (float)hdt * (dgp + dgn);
          }
        }
      }
    }
    // pricing date i + 1
    const int jd = i + 1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double S = exp(-Lam[c]);
      const double D = (double)s.D[((int64_t)jd * NC + c) * a.ld + kl];
      J += D * (Sprev[c] - S);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float dS = -(float)S * dL[c][q];
        gr[c][q] += (float)D * (dSprev[c][q] - dS);
        dSprev[c][q] = dS;
      }
      Sprev[c] = S;
    }
  }
  const AdjParams& P = a.par;
  a.grad_path[(int64_t)P.n_params * M + kl] = J;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    a.grad_path[(int64_t)(P.off_l0 + c) * M + kl] = gr[c][0];
    a.grad_path[(int64_t)(P.off_kappa + c) * M + kl] = gr[c][1];
    a.grad_path[(int64_t)(P.off_theta + c) * M + kl] = gr[c][2];
    a.grad_path[(int64_t)(P.off_nu + c) * M + kl] = gr[c][3];
  }
}

// ------------------------------------------------------------------------------------------
// market: reverse sweep
// ------------------------------------------------------------------------------------------
template <int NE, int NC>
struct MarketAdj {
  float rb[NE];        // adjoint of r^e at the current time point
  float xb[NE > 1 ? NE - 1 : 1];
  float Ib;            // adjoint of I
  float pend[NE];      // adjoint of r^e at the last reset date, from later dates
  float ga[NE], gb[NE], gs[NE], gx[NE > 1 ? NE - 1 : 1];
};

// Adjoint of the pricing and of the exposure weights at date i, state (r, x, I) at date i and
// r at the reset date preceding it.  Adds to the state adjoints, the pending reset adjoints and
// the parameter adjoints.
// Tables read through the scalar cache (read-only for the launch; every lane of a wave reads the
// same entry).
typedef const __attribute__((address_space(4))) float* ConstF;

template <int NE, int NC>
__device__ void pricing_adjoint(const AdjArgs& a, int i, int64_t kl, const float* r, const float* x,
                                double I, const float* rlr, MarketAdj<NE, NC>& ad) {
  const SimArgs<float>& s = a.sim;
  const ConstF G = (ConstF)s.G, CW1 = (ConstF)s.CW1, CW2 = (ConstF)s.CW2, W1 = (ConstF)s.W1;
  const int n = s.n_dates, q = s.q, P2 = s.n_periods + 2;
  const int64_t M = s.M;
  const bool reset = (i % q) == 0;
  const bool coupon = reset && i > 0;
  const int kfirst = i / q + 1;
  const int pmin = min((i + q - 1) / q, s.n_periods + 1);
  const int pnow = min(i / q, s.n_periods + 1);
  const double beta = exp(-I);
  // weights of MtM^c in J: p^c_i LGD_c beta_i 1{MtM^c > 0}; need MtM^c first
  float mtm[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) mtm[c] = 0.0f;
  float Fv[NE], fxv[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const ConstF lnA = (ConstF)s.lnA + e * (n + 1);
    const ConstF Bv = (ConstF)s.Bv + e * (n + 1);
    const float invzc = i == 0 ? 1.0f : expf(-lnA[q] + Bv[q] * rlr[e]);
    float F;
    if (i == 0) F = 1.0f;
    else if (reset) F = invzc;
    else {
      const int tau = kfirst * q - i;
      F = expf(lnA[tau] - Bv[tau] * r[e]) * invzc;
    }
    Fv[e] = F;
    float acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0f;
    for (int kk = kfirst; kk <= s.n_periods; ++kk) {
      const int tau = kk * q - i;
      const float zc = expf(lnA[tau] - Bv[tau] * r[e]);
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += zc * G[(c * NE + e) * P2 + kk];
    }
    const float fx = e == 0 ? 1.0f : expf(x[e > 0 ? e - 1 : 0]);
    fxv[e] = fx;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int base = (c * NE + e) * P2;
      float v = F * CW1[base + pmin] - acc[c];
      if (coupon) v -= CW2[base + pmin] + W1[base + pnow];
      mtm[c] += fx * v;
    }
  }
  float wc[NC];
  double Jd = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double S1 = exp(-a.sim.Lam[((int64_t)(i - 1) * NC + c) * a.ld + kl]);
    const double S2 = exp(-a.sim.Lam[((int64_t)i * NC + c) * a.ld + kl]);
    const double p = S1 - S2;
    const double pos = mtm[c] > 0.0f ? (double)mtm[c] : 0.0;
    Jd += p * (double)s.lgd[c] * beta * pos;
    wc[c] = mtm[c] > 0.0f ? (float)(p * (double)s.lgd[c] * beta) : 0.0f;
  }
  ad.Ib += (float)(-Jd);
  // back through each currency
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const ConstF lnA = (ConstF)s.lnA + e * (n + 1);
    const ConstF Bv = (ConstF)s.Bv + e * (n + 1);
    const ConstF dAa = (ConstF)a.dlnA_da + e * (n + 1);
    const ConstF dAb = (ConstF)a.dlnA_db + e * (n + 1);
    const ConstF dAs = (ConstF)a.dlnA_ds + e * (n + 1);
    const ConstF dBa = (ConstF)a.dB_da + e * (n + 1);
    const float fx = fxv[e];
    float Fb = 0.0f, Ae_sum = 0.0f;
    // x adjoint needs sum_c w^c A^{c,e}; A^{c,e} = F CW1 - acc - coupon terms
    float acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0f;
    for (int kk = kfirst; kk <= s.n_periods; ++kk) {
      const int tau = kk * q - i;
      const float zc = expf(lnA[tau] - Bv[tau] * r[e]);
      float zb = 0.0f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const float g = G[(c * NE + e) * P2 + kk];
        acc[c] += zc * g;
        zb -= wc[c] * fx * g;                  // dJ/dZ_k
      }
      // Z = exp(lnA - B r)
      ad.rb[e] += zb * (-Bv[tau] * zc);
      const float lAb = zb * zc, Bb = -zb * zc * r[e];
      ad.ga[e] += lAb * dAa[tau] + Bb * dBa[tau];
      ad.gb[e] += lAb * dAb[tau];
      ad.gs[e] += lAb * dAs[tau];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int base = (c * NE + e) * P2;
      float v = Fv[e] * CW1[base + pmin] - acc[c];
      if (coupon) v -= CW2[base + pmin] + W1[base + pnow];
      Ae_sum += wc[c] * v;
      Fb += wc[c] * fx * CW1[base + pmin];
    }
    if (e > 0) ad.xb[e - 1] += fx * Ae_sum;   // d chi / d x = chi
    if (i > 0) {
      const float F = Fv[e];
      // invzc = exp(-lnA(q) + B(q) r_lr): F depends on it linearly
      ad.pend[e] += Fb * Bv[q] * F;
      const float lAb = -Fb * F, Bb = Fb * F * rlr[e];
      ad.ga[e] += lAb * dAa[q] + Bb * dBa[q];
      ad.gb[e] += lAb * dAb[q];
      ad.gs[e] += lAb * dAs[q];
      if (!reset) {                        // times Z(tau+) = exp(lnA(tau+) - B(tau+) r)
        const int tau = kfirst * q - i;
        ad.rb[e] += Fb * (-Bv[tau] * F);
        const float lAb2 = Fb * F, Bb2 = -Fb * F * r[e];
        ad.ga[e] += lAb2 * dAa[tau] + Bb2 * dBa[tau];
        ad.gb[e] += lAb2 * dAb[tau];
        ad.gs[e] += lAb2 * dAs[tau];
      }
    }
  }
}

template <int NE, int NC>
__global__ __launch_bounds__(kOuterBlock) __attribute__((amdgpu_waves_per_eu(2)))
void market_adjoint_kernel(const AdjArgs a) {
  constexpr int DW = 2 * NE - 1;
  constexpr int NCALLM = (DW + 3) / 4;
  using CL = CoefLayout<NE, NC>;
  const SimArgs<float>& s = a.sim;
  const int64_t kl = (int64_t)blockIdx.x * kOuterBlock + threadIdx.x;
  if (kl >= s.M) return;
  const uint32_t k = s.path_begin + (uint32_t)kl;
  const int64_t M = s.M;
  const int n = s.n_dates, q = s.q, nf = s.n_feat;

  MarketAdj<NE, NC> ad;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    ad.rb[e] = 0.0f;
    ad.pend[e] = 0.0f;
    ad.ga[e] = ad.gb[e] = ad.gs[e] = 0.0f;
  }
#pragma unroll
  for (int e = 1; e < NE; ++e) ad.xb[e - 1] = ad.gx[e - 1] = 0.0f;
  ad.Ib = 0.0f;

  const float* Fe = s.features;
  auto load_state = [&](int i, float* r, float* x) {
#pragma unroll
    for (int e = 0; e < NE; ++e) r[e] = Fe[((int64_t)i * nf + e) * a.ld + kl];
#pragma unroll
    for (int e = 1; e < NE; ++e) x[e - 1] = Fe[((int64_t)i * nf + NE + e - 1) * a.ld + kl];
  };

  for (int i = n; i >= 1; --i) {
    float r[NE], x[NE > 1 ? NE - 1 : 1], rlr[NE], xd[NE > 1 ? NE - 1 : 1];
    load_state(i, r, x);
    const double Ii = s.I[(int64_t)i * a.ld + kl];
    const int lr = (i % q == 0) ? i - q : (i / q) * q;
    load_state(lr, rlr, xd);
    if (i % q == 0) {                      // later dates priced off r at this reset date
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        ad.rb[e] += ad.pend[e];
        ad.pend[e] = 0.0f;
      }
    }
    pricing_adjoint<NE, NC>(a, i, kl, r, x, Ii, rlr, ad);
    // reverse the sub-steps of (t_{i-1}, t_i]
    for (int j = s.n_sub - 1; j >= 0; --j) {
      asm volatile("" ::: "memory");
      const float* cf = s.coef;
      const float dt = s.dt;
      const float hdt = (float)s.half_dt;
      const uint32_t st = (uint32_t)((i - 1) * s.n_sub + j);
      float W[DW];
#pragma unroll
      for (int p = 0; p < DW; ++p) W[p] = 0.0f;
#pragma unroll
      for (int gcall = 0; gcall < NCALLM; ++gcall) {
        float z[4];
        normals4<float>(k, st, (uint32_t)gcall, s.key0, s.key1, z);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int f = 4 * gcall + t;
          if (f < DW) {
#pragma unroll
            // rows p >= f of column f; the loop runs over every row so that its trip count is a
          // constant and it unrolls to constant indices (W stays in registers, the factor is
          // read at fixed offsets)
          for (int p = 0; p < DW; ++p)
            if (p >= f) W[p] += s.chol[p * (p + 1) / 2 + f] * z[t];
          }
        }
      }
      // state before the sub-step: invert r_{k+1} = r_k + adt (lvl - r_k) + vol W
      float rk[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const float adt = cf[CL::r_adt + e], lvl = cf[CL::r_lvl + e], vol = cf[CL::r_vol + e];
        rk[e] = (r[e] - adt * lvl - vol * W[e]) / (1.0f - adt);
      }
      // adjoint of I_{k+1} = I_k + hdt (r0_k + r0_{k+1})
      ad.rb[0] += hdt * ad.Ib;             // r0 at k+1
      float rbk[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const float adt = cf[CL::r_adt + e], lvl = cf[CL::r_lvl + e];
        const float rbn = ad.rb[e];
        rbk[e] = (1.0f - adt) * rbn;
        ad.ga[e] += rbn * (dt * (lvl - rk[e]) + adt * a.dlvl_da[e]);
        ad.gb[e] += rbn * adt;
        ad.gs[e] += rbn * (a.sqrt_dt * W[e] + adt * a.dlvl_ds[e]);
        if (e > 0) ad.gx[e - 1] += rbn * adt * a.dlvl_dsx[e];
      }
      rbk[0] += hdt * ad.Ib;               // r0 at k
#pragma unroll
      for (int e = 1; e < NE; ++e) {
        const float xbn = ad.xb[e - 1];
        rbk[0] += dt * xbn;
        rbk[e] -= dt * xbn;
        ad.gx[e - 1] += xbn * (-a.sigma_fx[e - 1] * dt + a.sqrt_dt * W[NE + e - 1]);
      }
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        ad.rb[e] = rbk[e];
        r[e] = rk[e];
      }
    }
  }
  // date 0: the reset at t = 0 prices the first period off r_0
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    ad.rb[e] += ad.pend[e];
    ad.pend[e] = 0.0f;
  }
  const AdjParams& P = a.par;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    a.grad_path[(int64_t)(P.off_r0 + e) * M + kl] = ad.rb[e];
    a.grad_path[(int64_t)(P.off_a + e) * M + kl] = ad.ga[e];
    a.grad_path[(int64_t)(P.off_b + e) * M + kl] = ad.gb[e];
    a.grad_path[(int64_t)(P.off_sr + e) * M + kl] = ad.gs[e];
  }
#pragma unroll
  for (int e = 1; e < NE; ++e) {
    a.grad_path[(int64_t)(P.off_fx0 + e - 1) * M + kl] = ad.xb[e - 1] / a.fx0[e - 1];
    a.grad_path[(int64_t)(P.off_sx + e - 1) * M + kl] = ad.gx[e - 1];
  }
}

// Fixed-order mean over paths of every row of grad_path (row n_params is J, i.e. CVA_0).
__global__ __launch_bounds__(256) void adj_reduce(const double* gp, int64_t M, int n_params, double* grad,
                                                  double* cva0) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < M; k += 256) s += gp[(int64_t)p * M + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = red[0] / (double)M;
    if (p < n_params) grad[p] = v;
    else cva0[0] = v;
  }
}

__global__ __launch_bounds__(256) void adj_reduce_one(const double* row, int64_t M, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < M; k += 256) s += row[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / (double)M;
}

#define HSIM_ADJ_SHAPES(X) X(1, 1) X(1, 2) X(2, 1) X(2, 2) X(3, 3) X(10, 8)

// A second stream per device (default priority, non-blocking), created once: the credit sweep
// runs on it beside the market sweep on the caller's stream (the two write disjoint rows of the
// per-path buffer), forked and joined by events, so the two one-wave-per-SIMD launches share the
// SIMDs.  Calls on one device share it: concurrent callers serialise their credit sweeps there.
static hipError_t side_stream(hipStream_t* out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static hipStream_t streams[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev] && (e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking)) != hipSuccess) return e;
  *out = streams[dev];
  return hipSuccess;
}

hipError_t launch_adjoint(const AdjArgs& a, bool with_grad, hipStream_t stream) {
  const dim3 grid((unsigned)((a.sim.M + kOuterBlock - 1) / kOuterBlock));
  hipStream_t credit_stream = stream;
  hipEvent_t fork = nullptr, join = nullptr;
  hipError_t e = hipSuccess;
  if (with_grad) {
    if ((e = side_stream(&credit_stream)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&join, hipEventDisableTiming)) != hipSuccess) {
      hipEventDestroy(fork);
      return e;
    }
    if ((e = hipEventRecord(fork, stream)) == hipSuccess) e = hipStreamWaitEvent(credit_stream, fork, 0);
  }
  bool done = false;
#define X(ne, nc)                                                                                  \
  if (e == hipSuccess && !done && a.sim.n_ccy == ne && a.sim.n_cpty == nc) {                      \
    hipLaunchKernelGGL((credit_kernel<ne, nc>), grid, dim3(kOuterBlock), 0, credit_stream, a);     \
    if (with_grad)                                                                                 \
      hipLaunchKernelGGL((market_adjoint_kernel<ne, nc>), grid, dim3(kOuterBlock), 0, stream, a);  \
    done = true;                                                                                   \
  }
  HSIM_ADJ_SHAPES(X)
#undef X
  if (e == hipSuccess && !done) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = hipGetLastError();
  if (with_grad) {
    // join even after a failed launch, so the caller's stream never runs ahead of the side one
    const hipError_t j = hipEventRecord(join, credit_stream);
    const hipError_t w = j == hipSuccess ? hipStreamWaitEvent(stream, join, 0) : j;
    hipEventDestroy(fork);
    hipEventDestroy(join);
    if (e == hipSuccess) e = w;
  }
  if (e != hipSuccess) return e;
  if (with_grad)
    hipLaunchKernelGGL(adj_reduce, dim3(a.par.n_params + 1), dim3(256), 0, stream, a.grad_path, a.sim.M,
                       a.par.n_params, a.grad_out, a.cva0_out);
  else                                    // the J row only
    hipLaunchKernelGGL(adj_reduce_one, dim3(1), dim3(256), 0, stream, a.grad_path + (int64_t)a.par.n_params * a.sim.M,
                       a.sim.M, a.cva0_out);
  return hipGetLastError();
}

}  // namespace hsim
