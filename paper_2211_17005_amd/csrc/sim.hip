// Simulation kernels of the hierarchical CVA path (gfx950).
//
//   outer_kernel    one lane per outer path: Euler sub-steps of the market factors
//                   (Appendix B, e:sde1/e:sde2, Q^0 drift of foreign rates), FP64
//                   trapezoid integrals of r^0 and gamma^{c,+} (rem:finecoarse), and at
//                   every pricing date the swap book priced by the three-case formula of
//                   Appendix B, exposures D^c_j = LGD_c beta_j (MtM^c_j)^+, features.
//   inner_kernel    one lane per outer path, the path's default thresholds staged in LDS:
//                   the n_b inner draws per counterparty are resolved to a default date by
//                   the rule of e:tau (Lambda_j >= -log u), counted per date.
//   targets_kernel  one lane per path: the suffix sums of eq:CVA_portfolio over the date
//                   histogram give T_i (or, in the intensity form of eq:CVAint, over the
//                   survival increments); FP64 block partials give CVA_0 in a fixed order.
//   branch_kernel   one lane per (continuation, path): the outer path up to a branching
//                   date, then an independent continuation whose eq:CVAint sample is
//                   accumulated in registers (nested / twin Monte Carlo).
//
// The outer state is kept in registers for the whole horizon; the only HBM traffic is
// the per-date outputs.  All parameters that are the same for every lane (Cholesky
// factor, zero-coupon coefficients, bucketed swap weights) are read with uniform
// indices, so they come through the scalar cache.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "philox.hpp"
#include "sim.hpp"

namespace hsim {

__device__ __forceinline__ float exp_r(float x) { return expf(x); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
__device__ __forceinline__ float sqrt_r(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

// Acc: type of the discount and intensity integrals (double; float in the plain FP32 form).
template <typename Real, int NE, int NC, typename Acc = double>
struct OuterState {
  Real r[NE];
  Real x[NE > 1 ? NE - 1 : 1];
  Real g[NC];
  Real gcomp[NC];          // rounding error carried by the compensated intensity update
  Real invzc[NE];          // 1 / ZC^e_{t-}(t-+delta), from r^e at the last reset date
  Acc I;
  Acc Lam[NC];
};

// 1 / ZC^e_t(t + delta) from r^e at a reset date: the next floating coupon's discount.
template <typename Real, int NE, int NC>
__device__ __forceinline__ Real reset_inv_zc(const SimArgs<Real>& a, int e, Real re) {
  const Real* lnA = a.lnA + e * (a.n_dates + 1);
  const Real* Bv = a.Bv + e * (a.n_dates + 1);
  return exp_r(-lnA[a.q] + Bv[a.q] * re);
}

// The reset bookkeeping of pricing date i without the pricing itself.
template <typename Real, int NE, int NC, typename Acc = double>
__device__ __forceinline__ void reset_only(const SimArgs<Real>& a, OuterState<Real, NE, NC, Acc>& st, int i) {
  if ((i % a.q) != 0) return;
#pragma unroll
  for (int e = 0; e < NE; ++e) st.invzc[e] = reset_inv_zc<Real, NE, NC>(a, e, st.r[e]);
}

// The pricing tables through the scalar cache: read-only for the launch, and every lane of a
// wave reads the same entry (the indices depend on the date and the currency only).
template <typename Real>
using ConstTable = const __attribute__((address_space(4))) Real*;

// Value of the book per counterparty at pricing date i (updates the reset state).
template <typename Real, int NE, int NC, typename Acc = double>
__device__ __forceinline__ void price(const SimArgs<Real>& a, OuterState<Real, NE, NC, Acc>& st, int i,
                                      Real mtm[NC]) {
  const ConstTable<Real> G = (ConstTable<Real>)a.G, CW1 = (ConstTable<Real>)a.CW1,
                         CW2 = (ConstTable<Real>)a.CW2, W1 = (ConstTable<Real>)a.W1;
  const int n = a.n_dates;
  const int q = a.q;
  const int P2 = a.n_periods + 2;
  const bool reset = (i % q) == 0;
  const bool coupon = reset && i > 0;
  const int kfirst = i / q + 1;             // first reset date strictly after t_i
  // shortest maturity still alive at t_i, and the maturity ending at t_i (if a reset); past
  // the longest maturity both point at the zero entry n_periods + 1 of the weight tables
  const int pmin = min((i + q - 1) / q, a.n_periods + 1);
  const int pnow = min(i / q, a.n_periods + 1);

#pragma unroll
  for (int c = 0; c < NC; ++c) mtm[c] = (Real)0;

#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const Real re = st.r[e];
    const ConstTable<Real> lnA = (ConstTable<Real>)a.lnA + e * (n + 1);
    const ConstTable<Real> Bv = (ConstTable<Real>)a.Bv + e * (n + 1);
    Real F;
    if (i == 0) {
      F = (Real)1;
    } else if (reset) {
      F = st.invzc[e];                      // 1 / ZC_{t - delta}(t): the floating coupon
    } else {
      const int tau = kfirst * q - i;       // ZC_t(t_+) / ZC_{t_-}(t_+)
      F = exp_r(lnA[tau] - Bv[tau] * re) * st.invzc[e];
    }
    Real acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = (Real)0;
    for (int kk = kfirst; kk <= a.n_periods; ++kk) {
      const int tau = kk * q - i;
      const Real zc = exp_r(lnA[tau] - Bv[tau] * re);
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += zc * G[(c * NE + e) * P2 + kk];
    }
    const Real fx = (e == 0) ? (Real)1 : exp_r(st.x[e > 0 ? e - 1 : 0]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int base = (c * NE + e) * P2;
      Real v = F * CW1[base + pmin] - acc[c];
      if (coupon) v -= CW2[base + pmin] + W1[base + pnow];
      mtm[c] += fx * v;
    }
    if (reset) st.invzc[e] = reset_inv_zc<Real, NE, NC>(a, e, re);
  }
}

// Price the book and emit every per-date output at date i.
// Exposure D^c = LGD_c beta (MtM^c)^+ of one counterparty.
template <typename Real, typename Acc>
__device__ __forceinline__ Real exposure(const SimArgs<Real>& a, Acc beta, Real mtm, int c) {
  const Real pos = mtm > (Real)0 ? mtm : (Real)0;
  return (Real)((Acc)a.lgd[c] * beta * (Acc)pos);
}

// Regression features of date i (date-major rows, one column per lane).
template <typename Real, int NE, int NC, typename Acc>
__device__ __forceinline__ void emit_features(const SimArgs<Real>& a, const OuterState<Real, NE, NC, Acc>& st,
                                              int i, int64_t kl) {
  if (!a.features) return;
  const int64_t M = a.M;
  Real* f = a.features + (int64_t)i * a.n_feat * M + kl;
  int col = 0;
#pragma unroll
  for (int e = 0; e < NE; ++e) f[(int64_t)(col++) * M] = st.r[e];
#pragma unroll
  for (int e = 1; e < NE; ++e) f[(int64_t)(col++) * M] = st.x[e - 1];
#pragma unroll
  for (int c = 0; c < NC; ++c) f[(int64_t)(col++) * M] = st.g[c];
  if (a.feature_mode == 1) {
    Acc sl = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) sl += st.Lam[c];
    f[(int64_t)(col++) * M] = (Real)st.I;
    f[(int64_t)(col++) * M] = (Real)sl;
  }
}

// Price the book and emit every per-date output at date i.
template <typename Real, int NE, int NC, typename Acc = double>
__device__ __forceinline__ void price_and_emit(const SimArgs<Real>& a, OuterState<Real, NE, NC, Acc>& st,
                                               int i, int64_t kl) {
  const int64_t M = a.M;
  Real mtm[NC];
  price<Real, NE, NC, Acc>(a, st, i, mtm);
  const Acc beta = exp_r(-st.I);
  a.I[(int64_t)i * M + kl] = (double)st.I;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t o = ((int64_t)i * NC + c) * M + kl;
    a.Lam[o] = (double)st.Lam[c];
    a.D[o] = exposure<Real, Acc>(a, beta, mtm[c], c);
    if (a.MtM) a.MtM[o] = mtm[c];
  }
  emit_features<Real, NE, NC, Acc>(a, st, i, kl);
}

template <typename Real, int NE, int NC, typename Acc = double>
__device__ __forceinline__ void init_state(const SimArgs<Real>& a, OuterState<Real, NE, NC, Acc>& st) {
#pragma unroll
  for (int e = 0; e < NE; ++e) st.r[e] = a.r0[e];
#pragma unroll
  for (int e = 1; e < NE; ++e) st.x[e - 1] = a.x0[e - 1];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    st.g[c] = a.g0[c];
    st.gcomp[c] = (Real)0;
    st.Lam[c] = 0;
  }
  st.I = 0;
}

// The n_sub Euler sub-steps from t_i to t_{i+1}, normals from the Philox counters
// (k, s, c2 + (f >> 2), tag).
template <typename Real, int NE, int NC, typename Acc = double>
__device__ __forceinline__ void advance(const SimArgs<Real>& a, OuterState<Real, NE, NC, Acc>& st, int i,
                                        uint32_t k, uint32_t c2, uint32_t tag) {
  constexpr int DW = 2 * NE - 1;
  constexpr int NZ = DW + NC;
  constexpr int NCALL = (NZ + 3) / 4;
  for (int j = 0; j < a.n_sub; ++j) {
    // Keep the uniform parameters (kernel arguments, Cholesky factor) in memory: they are
    // re-read through the scalar cache every sub-step instead of being hoisted into
    // registers, which would cost more registers than the whole path state.
    asm volatile("" ::: "memory");
    using CL = CoefLayout<NE, NC>;
    const Real* cf = a.coef;
    const Real dt = a.dt;
    const Acc hdt = (Acc)a.half_dt;
    const uint32_t s = (uint32_t)(i * a.n_sub + j);
    // Normals arrive four at a time; each market normal z_f is folded at once into the
    // correlated increments W_p += L_{pf} z_f (p >= f), each CIR normal drives its
    // intensity step, so only W and the current four normals are live.
    Real W[DW];
#pragma unroll
    for (int p = 0; p < DW; ++p) W[p] = (Real)0;
#pragma unroll
    for (int g = 0; g < NCALL; ++g) {
      Real z[4];
      normals4<Real>(k, s, c2 + (uint32_t)g, a.key0, a.key1, z, tag);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int f = 4 * g + t;
        if (f < DW) {
#pragma unroll
          // rows p >= f of column f; the loop runs over every row so that its trip count is a
          // constant and it unrolls to constant indices (W stays in registers, the factor is
          // read at fixed offsets)
          for (int p = 0; p < DW; ++p)
            if (p >= f) W[p] += a.chol[p * (p + 1) / 2 + f] * z[t];
        } else if (f < NZ) {
          const int c = f - DW;
          const Real gp = st.g[c] > (Real)0 ? st.g[c] : (Real)0;
          // compensated (Fast2Sum) state update: the CIR diffusion amplifies rounding
          // errors of the state near zero, so the increment's rounding error is carried
          const Real inc = cf[CL::g_add + c] - cf[CL::g_kd + c] * gp + cf[CL::g_vol + c] * sqrt_r(gp) * z[t]
                           + st.gcomp[c];
          const Real gs = st.g[c] + inc;
          st.gcomp[c] = inc - (gs - st.g[c]);
          st.g[c] = gs;
          const Real gn = st.g[c] > (Real)0 ? st.g[c] : (Real)0;
          st.Lam[c] += hdt * ((Acc)gp + (Acc)gn);
        }
      }
    }
    const Real r0old = st.r[0];
#pragma unroll
    for (int e = 1; e < NE; ++e)
      st.x[e - 1] += (r0old - st.r[e]) * dt + cf[CL::x_add + e - 1] + cf[CL::x_vol + e - 1] * W[NE + e - 1];
#pragma unroll
    for (int e = 0; e < NE; ++e)
      st.r[e] = st.r[e] + cf[CL::r_adt + e] * (cf[CL::r_lvl + e] - st.r[e]) + cf[CL::r_vol + e] * W[e];
    st.I += hdt * ((Acc)r0old + (Acc)st.r[0]);
  }
}

template <typename Real, int NE, int NC, typename Acc>
__global__ __launch_bounds__(kOuterBlock) __attribute__((amdgpu_waves_per_eu(NE > 4 ? 2 : 4)))
void outer_kernel(const SimArgs<Real> a) {
  const int64_t kl = (int64_t)blockIdx.x * kOuterBlock + threadIdx.x;
  if (kl >= a.M) return;
  const uint32_t k = a.path_begin + (uint32_t)kl;
  OuterState<Real, NE, NC, Acc> st;
  init_state<Real, NE, NC, Acc>(a, st);
  price_and_emit<Real, NE, NC, Acc>(a, st, 0, kl);
  for (int i = 0; i < a.n_dates; ++i) {
    advance<Real, NE, NC, Acc>(a, st, i, k, 0u, kTagOuter);
    price_and_emit<Real, NE, NC, Acc>(a, st, i + 1, kl);
  }
}

// ------------------------------------------------------------------------------------
// branched re-simulation (nested and twin Monte Carlo)
// ------------------------------------------------------------------------------------
// Lane (b, k): outer path k exactly as outer_kernel simulates it up to t_date (pricing
// replaced by the reset bookkeeping it would do), then continuation b with the branch
// counters; the intensity-form sample of eq. CVAint at t_date is accumulated on the way:
//   xi = sum_{j > date} sum_c LGD_c exp(I_date - I_j) (MtM^c_j)^+
//        (exp(-Lambda^c_{j-1}) - exp(-Lambda^c_j)).
template <typename Real, int NE, int NC>
__global__ __launch_bounds__(kOuterBlock) __attribute__((amdgpu_waves_per_eu(NE > 4 ? 2 : 4)))
void branch_kernel(const SimArgs<Real> a, const BranchArgs b) {
  const int64_t lane = (int64_t)blockIdx.x * kOuterBlock + threadIdx.x;
  if (lane >= a.M * b.n_branch) return;
  const int64_t kl = lane % a.M;
  const uint32_t br = (uint32_t)(lane / a.M);
  const uint32_t k = a.path_begin + (uint32_t)kl;
  OuterState<Real, NE, NC> st;
  init_state<Real, NE, NC>(a, st);
  reset_only<Real, NE, NC>(a, st, 0);
  for (int i = 0; i < b.date; ++i) {
    advance<Real, NE, NC>(a, st, i, k, 0u, kTagOuter);
    reset_only<Real, NE, NC>(a, st, i + 1);
  }
  const double I0 = st.I;
  double surv[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) surv[c] = exp(-st.Lam[c]);
  double xi = 0.0;
  for (int i = b.date; i < a.n_dates; ++i) {
    advance<Real, NE, NC>(a, st, i, k, 16u * br, kTagBranch);
    Real mtm[NC];
    price<Real, NE, NC>(a, st, i + 1, mtm);
    const double disc = exp(I0 - st.I);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double sn = exp(-st.Lam[c]);
      const double pos = mtm[c] > (Real)0 ? (double)mtm[c] : 0.0;
      xi += (double)a.lgd[c] * disc * pos * (surv[c] - sn);
      surv[c] = sn;
    }
  }
  b.xi[lane] = xi;
}

// Per-path nested / twin statistics over the continuations, FP64 block partials
// (row r of `partial` holds statistic r of every block):
//   nu, nu^2, U = ((sum xi)^2 - sum xi^2) / (B (B-1)), (phi - nu)^2, phi^2 - 2 phi nu + U, phi.
template <typename PhiT>
__global__ __launch_bounds__(kTargetBlock) void branch_stats_kernel(int64_t M, int32_t B, const PhiT* phi,
                                                                   const double* xi, double* partial,
                                                                   int64_t nblk) {
  __shared__ double red[kBranchStats][kTargetBlock];
  const int64_t k = (int64_t)blockIdx.x * kTargetBlock + threadIdx.x;
  double v[kBranchStats] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (k < M) {
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < B; ++b) {
      const double x = xi[(int64_t)b * M + k];
      s1 += x;
      s2 += x * x;
    }
    const double nu = s1 / B;
    const double U = (s1 * s1 - s2) / ((double)B * (double)(B - 1));
    const double f = phi ? (double)phi[k] : 0.0;
    v[0] = nu;
    v[1] = nu * nu;
    v[2] = U;
    v[3] = (f - nu) * (f - nu);
    v[4] = f * f - 2.0 * f * nu + U;
    v[5] = f;
  }
#pragma unroll
  for (int r = 0; r < kBranchStats; ++r) red[r][threadIdx.x] = v[r];
  __syncthreads();
  for (int w = kTargetBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int r = 0; r < kBranchStats; ++r) red[r][threadIdx.x] += red[r][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < kBranchStats) partial[threadIdx.x * nblk + blockIdx.x] = red[threadIdx.x][0];
}

// ------------------------------------------------------------------------------------
// inner default draws
// ------------------------------------------------------------------------------------
// Threshold form of the default rule on the 23-bit uniform u = (2m+1) 2^-24:
//   Lambda >= -log u  <=>  u >= exp(-Lambda)  <=>  m >= ceil((exp(-Lambda) 2^24 - 1) / 2).
__device__ __forceinline__ uint32_t default_threshold(double lam) {
  const double S = exp(-lam);
  const double t = ceil((S * 16777216.0 - 1.0) * 0.5);
  return t <= 0.0 ? 0u : (uint32_t)t;
}

// The draws of one tile of 64 paths (one lane per path).
__device__ void inner_tile(const InnerArgs& a, uint32_t* lds, int64_t tile) {
  const int lane = threadIdx.x;
  const int n = a.n_dates;
  const int C = a.n_cpty;
  const int64_t M = a.M;
  const int64_t kl = tile * kInnerBlock + lane;
  const bool valid = kl < M;
  const uint32_t k = a.path_begin + (uint32_t)kl;
  const int nb = a.nb_block ? a.nb_block[(tile * kInnerBlock) / a.block_paths] : a.n_b;
  uint32_t* K = lds;                       // [(n+1)][64], column `lane` is private to it
  uint32_t* cnt = lds + (n + 1) * kInnerBlock;

  for (int c = 0; c < C; ++c) {
    // Threshold form of the default rule: with u = (2m+1) 2^-24,
    //   Lambda_j >= -log u  <=>  u >= exp(-Lambda_j)  <=>  m >= ceil((exp(-Lambda_j) 2^24 - 1)/2).
    for (int j = 0; j <= n; ++j) {
      const uint32_t th = valid ? default_threshold(a.Lam[((int64_t)j * C + c) * M + kl]) : 0xFFFFFFFFu;
      K[j * kInnerBlock + lane] = th;
      cnt[j * kInnerBlock + lane] = 0u;
    }
    if (valid) {
      const uint32_t Kn = K[n * kInnerBlock + lane];
      for (int l4 = 0; l4 < nb; l4 += 4) {
        const u32x4 w = philox4x32_10(k, (uint32_t)(l4 >> 2), (uint32_t)c, kTagInner, a.key0, a.key1);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (l4 + t >= nb) break;
          const uint32_t m = grid23(ws[t]);
          if (m >= Kn) {                   // defaults by the horizon: smallest j with K_j <= m
            int lo = 1, hi = n;
            while (lo < hi) {
              const int mid = (lo + hi) >> 1;
              if (m >= K[mid * kInnerBlock + lane]) hi = mid; else lo = mid + 1;
            }
            cnt[lo * kInnerBlock + lane] += 1u;
          }
        }
      }
      for (int j = 0; j <= n; ++j)
        a.counts[((int64_t)j * C + c) * M + kl] = (int32_t)cnt[j * kInnerBlock + lane];
    }
  }
}

// One workgroup (one wave) per tile of 64 paths, or, with uneven n_b, a persistent grid that
// takes the tiles longest-first from a work counter.  Every tile is computed the same way in
// either schedule, so the counts do not depend on it.
__global__ __launch_bounds__(kInnerBlock) void inner_kernel(const InnerArgs a) {
  extern __shared__ uint32_t lds[];
  if (a.order == nullptr) {
    inner_tile(a, lds, blockIdx.x);
    return;
  }
  const int64_t tiles = (a.M + kInnerBlock - 1) / kInnerBlock;
  int32_t* queue = a.order + tiles;
  for (;;) {
    int t = 0;
    if (threadIdx.x == 0) t = atomicAdd(queue, 1);
    t = __shfl(t, 0);
    if (t >= tiles) break;
    inner_tile(a, lds, a.order[t]);
  }
}

// Per-inner-sample regression rows: one lane per sample (draw l, path k), row r = l M + k (the
// order whose contiguous slices are the paper's minibatches).  The draw is the inner kernel's
// (same Philox word, same threshold rule); its default date per counterparty comes from a
// binary search on the thresholds of Lambda^c, and at every date i the row holds the path's
// market features, the indicators 1{j*_c <= i} and the label
//   xi_i = exp(I_i) sum_{c : j*_c > i} D^c_{j*_c}.
template <typename Real>
__global__ __launch_bounds__(kTargetBlock) void sample_rows_kernel(const SampleArgs<Real> a) {
  const int64_t r = (int64_t)blockIdx.x * kTargetBlock + threadIdx.x;
  const int64_t M = a.M;
  if (r >= M * a.n_b) return;
  const int64_t kl = r % M;
  const uint32_t l = (uint32_t)(r / M);
  const uint32_t k = a.path_begin + (uint32_t)kl;
  const int n = a.n_dates, C = a.n_cpty, d = a.d;
  const int64_t R = M * a.n_b;
  int js[kMaxCpty];
  double dv[kMaxCpty];                      // D^c at the default date (0 without default)
#pragma unroll
  for (int c = 0; c < kMaxCpty; ++c) {
    js[c] = n + 1;
    dv[c] = 0.0;
    if (c >= C) continue;
    const u32x4 w = philox4x32_10(k, l >> 2, (uint32_t)c, kTagInner, a.key0, a.key1);
    const uint32_t word = (l & 3) == 0 ? w.x : (l & 3) == 1 ? w.y : (l & 3) == 2 ? w.z : w.w;
    const uint32_t m = grid23(word);
    if (m >= default_threshold(a.Lam[((int64_t)n * C + c) * M + kl])) {   // defaults by the horizon
      int lo = 1, hi = n;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (m >= default_threshold(a.Lam[((int64_t)mid * C + c) * M + kl])) hi = mid; else lo = mid + 1;
      }
      js[c] = lo;
      dv[c] = (double)a.D[((int64_t)lo * C + c) * M + kl];
    }
  }
  for (int i = 0; i <= n; ++i) {
    float* X = a.X + (int64_t)i * (d + C) * R + r;
    for (int f = 0; f < d; ++f) X[(int64_t)f * R] = (float)a.features[((int64_t)i * d + f) * M + kl];
    double S = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxCpty; ++c) {
      if (c >= C) continue;
      X[(int64_t)(d + c) * R] = js[c] <= i ? 1.0f : 0.0f;
      if (js[c] > i) S += dv[c];
    }
    a.Y[(int64_t)i * R + r] = (float)(S * exp(a.I[(int64_t)i * M + kl]));
  }
}

// Longest-first order of the tiles of an uneven-n_b launch: tiles bucketed by floor(log2 n_b)
// (largest first, tile order inside a bucket arbitrary); also clears the work counter.
__global__ __launch_bounds__(1024) void inner_order_kernel(const int32_t* nb_block, int32_t block_paths,
                                                           int64_t M, int32_t* order) {
  __shared__ int cnt[32], off[32];
  const int64_t tiles = (M + kInnerBlock - 1) / kInnerBlock;
  if (threadIdx.x < 32) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < tiles; i += blockDim.x) {
    const int nb = nb_block[(i * kInnerBlock) / block_paths];
    atomicAdd(&cnt[__clz(nb > 0 ? nb : 1)], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int b = 0; b < 32; ++b) {
      off[b] = s;
      s += cnt[b];
    }
    order[tiles] = 0;
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < tiles; i += blockDim.x) {
    const int nb = nb_block[(i * kInnerBlock) / block_paths];
    order[atomicAdd(&off[__clz(nb > 0 ? nb : 1)], 1)] = (int32_t)i;
  }
}

// ------------------------------------------------------------------------------------
// targets and CVA_0
// ------------------------------------------------------------------------------------
// T_i = exp(I_i) sum_{j > i} sum_c D^c_j w^c_j with w^c_j = counts^c_j / n_b (the inner average of
// the pathwise loss) or, in the intensity form, w^c_j = exp(-Lambda^c_{j-1}) - exp(-Lambda^c_j)
// (its conditional expectation given the outer path: one default per counterparty falls in
// (t_{j-1}, t_j] with that probability).  In the alive-group form (one counterparty) the sum is
// divided by the A_i draws still alive at t_i instead of n_b, and A_i / n_b is the row weight:
// A_i = n_b - (defaults up to t_i) = n_b - total + (defaults after t_i).
enum TargetMode { kNested = 0, kIntensity = 1, kAlive = 2 };

// One term of a date's part of the suffix sum: H + D^c_j w^c_j in FP64 (shared by the fused
// kernel so that both forms round identically).
template <typename Real>
__device__ __forceinline__ double date_term(double H, Real D, double w) {
  return __builtin_fma((double)D, w, H);
}

template <typename Real, int kMode>
__global__ __launch_bounds__(kTargetBlock) void targets_kernel(const TargetArgs<Real> a) {
  __shared__ double red[kTargetBlock];
  const int64_t M = a.M;
  const int n = a.n_dates;
  const int C = a.n_cpty;
  const int64_t kl = (int64_t)blockIdx.x * kTargetBlock + threadIdx.x;
  double t0 = 0.0;
  if (kl < M) {
    const int nb = a.nb_block ? a.nb_block[kl / a.block_paths] : a.n_b;
    const double inv_nb = kMode == kIntensity ? 1.0 : 1.0 / (double)nb;
    double S = 0.0;                        // sum_{j > i} sum_c D^c_j w^c_j
    int alive0 = 0, later = 0;             // alive form: draws alive at the horizon, defaults after t_i
    if constexpr (kMode == kAlive) {
      int total = 0;
      for (int j = 1; j <= n; ++j) total += a.counts[(int64_t)j * M + kl];
      alive0 = nb - total;
      a.weight[(int64_t)n * M + kl] = (float)((double)alive0 * inv_nb);
    }
    a.T[(int64_t)n * M + kl] = (Real)0;
    for (int i = n - 1; i >= 0; --i) {
      double Hj = 0.0;                     // this date's terms, summed over c in order
      for (int c = 0; c < C; ++c) {
        const int64_t o = ((int64_t)(i + 1) * C + c) * M + kl;
        double wgt;
        if constexpr (kMode == kIntensity) {
          wgt = exp(-a.Lam[((int64_t)i * C + c) * M + kl]) - exp(-a.Lam[o]);
        } else {
          wgt = (double)a.counts[o];
        }
        Hj = date_term(Hj, a.D[o], wgt);
      }
      S += Hj;
      double Ti;
      if constexpr (kMode == kAlive) {
        later += a.counts[(int64_t)(i + 1) * M + kl];
        const int A = alive0 + later;
        Ti = A > 0 ? S * exp(a.I[(int64_t)i * M + kl]) / (double)A : 0.0;
        a.weight[(int64_t)i * M + kl] = (float)((double)A * inv_nb);
      } else {
        Ti = S * exp(a.I[(int64_t)i * M + kl]) * inv_nb;
      }
      a.T[(int64_t)i * M + kl] = (Real)Ti;
      if (i == 0) t0 = Ti;
    }
  }
  red[threadIdx.x] = t0;
  __syncthreads();
  for (int w = kTargetBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kTargetBlock) void reduce_partials(const double* partial, int64_t nblk,
                                                                double inv_M, double* out) {
  __shared__ double red[kTargetBlock];
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nblk; b += kTargetBlock) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kTargetBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * inv_M;
}

// ------------------------------------------------------------------------------------
// fused simulation: outer paths, inner draws and targets in one launch
// ------------------------------------------------------------------------------------
// One workgroup (one wave) per tile of 64 outer paths.  Phase 1 is outer_kernel's simulation,
// one lane per path; at every pricing date a lane writes its features (as outer_kernel) and, into
// a path-major table in the workspace, what the inner draws and the targets need: the integer
// default threshold of every counterparty (the rule Lambda_j >= -log u on the 23-bit uniforms),
// the exposures D^c_j and the discount integral I_j.  Phase 2 takes the tile's paths one at a
// time: the wave stages the path's table (contiguous, just written by this workgroup) in LDS and
// draws its n_b x C inner defaults cooperatively (lanes = Philox calls of four draws), locating
// each default date by the same binary search as inner_kernel and counting it in an LDS
// histogram; lanes then form the per-date terms sum_c D^c_j counts^c_j, one lane the suffix sums
// over dates, and lanes the targets T_i.  The order of every floating-point operation is that of
// targets_kernel, so targets and CVA_0 equal the separate stages' bit for bit.
template <typename Real, int NE, int NC>
__device__ __forceinline__ void fused_emit(const SimArgs<Real>& a, const FusedArgs& f,
                                           OuterState<Real, NE, NC, double>& st, int i, int64_t kl) {
  const int n1 = a.n_dates + 1;
  Real mtm[NC];
  price<Real, NE, NC, double>(a, st, i, mtm);
  const double beta = exp(-st.I);
  const int64_t row = (kl * n1 + i) * NC;
  Real* Dv = (Real*)f.Dv;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    f.K[row + c] = default_threshold(st.Lam[c]);
    Dv[row + c] = exposure<Real, double>(a, beta, mtm[c], c);
  }
  f.Iv[kl * n1 + i] = st.I;
  if (kl < f.n_keep) {                       // the date-major states of hsim_outer_paths
    const int64_t M = a.M;
    f.I_keep[(int64_t)i * M + kl] = st.I;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t o = ((int64_t)i * NC + c) * M + kl;
      f.Lam_keep[o] = st.Lam[c];
      ((Real*)f.D_keep)[o] = Dv[row + c];
    }
  }
  emit_features<Real, NE, NC, double>(a, st, i, kl);
}

template <typename Real>
__device__ void fused_inner_targets(const SimArgs<Real>& a, const FusedArgs& f, int64_t tile, char* lds) {
  const int lane = threadIdx.x, n = a.n_dates, C = a.n_cpty, n1 = n + 1;
  const int64_t M = a.M;
  const int nc = n1 * C;
  uint32_t* Kl = (uint32_t*)lds;                          // [n1][C] thresholds
  uint32_t* hist = Kl + nc;                               // [n1][C] defaults per date
  double* Il = (double*)(lds + fused_lds_offset_f64(n, C)); // [n1] I_j
  double* Hs = Il + n1;                                   // [n1] date terms, then suffix sums
  Real* Dl = (Real*)(Hs + n1);                            // [n1][C] exposures
  const Real* Dv = (const Real*)f.Dv;
  Real* T = (Real*)f.T;
  const int nb = f.nb_block ? f.nb_block[(tile * kOuterBlock) / f.block_paths] : f.n_b;
  const double inv_nb = 1.0 / (double)nb;
  const int calls = (nb + 3) / 4;
  const int64_t first = tile * kOuterBlock;
  const int count = (int)min((int64_t)kOuterBlock, M - first);
  for (int p = 0; p < count; ++p) {
    const int64_t kl = first + p;
    const uint32_t k = a.path_begin + (uint32_t)kl;
    for (int e = lane; e < nc; e += kOuterBlock) {
      Kl[e] = f.K[kl * nc + e];
      Dl[e] = Dv[kl * nc + e];
      hist[e] = 0u;
    }
    for (int e = lane; e < n1; e += kOuterBlock) Il[e] = f.Iv[kl * n1 + e];
    __syncthreads();
    for (int q = lane; q < C * calls; q += kOuterBlock) {
      const int c = q / calls, l4 = 4 * (q - c * calls);
      const uint32_t Kn = Kl[n * C + c];
      const u32x4 w = philox4x32_10(k, (uint32_t)(l4 >> 2), (uint32_t)c, kTagInner, a.key0, a.key1);
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (l4 + t >= nb) break;
        const uint32_t m = grid23(ws[t]);
        if (m >= Kn) {                       // defaults by the horizon: smallest j with K_j <= m
          int lo = 1, hi = n;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (m >= Kl[mid * C + c]) hi = mid; else lo = mid + 1;
          }
          atomicAdd(&hist[lo * C + c], 1u);
        }
      }
    }
    __syncthreads();
    for (int j = 1 + lane; j <= n; j += kOuterBlock) {
      double H = 0.0;
      for (int c = 0; c < C; ++c) H = date_term(H, Dl[j * C + c], (double)hist[j * C + c]);
      Hs[j] = H;
    }
    __syncthreads();
    if (lane == 0) {                         // S_i = sum_{j > i} H_j, added from the last date down
      double S = 0.0;
      for (int i = n - 1; i >= 0; --i) {
        S += Hs[i + 1];
        Hs[i + 1] = S;
      }
    }
    __syncthreads();
    for (int i = lane; i <= n; i += kOuterBlock) {
      const double Ti = i == n ? 0.0 : Hs[i + 1] * exp(Il[i]) * inv_nb;
      T[(int64_t)i * M + kl] = (Real)Ti;
      if (i == 0) f.T0[kl] = Ti;
    }
    __syncthreads();
  }
}

template <typename Real, int NE, int NC>
__global__ __launch_bounds__(kOuterBlock) __attribute__((amdgpu_waves_per_eu(NE > 4 ? 2 : 4)))
void fused_kernel(const SimArgs<Real> a, const FusedArgs f) {
  extern __shared__ __attribute__((aligned(16))) char fused_lds[];
  const int64_t tile = blockIdx.x;
  const int64_t kl = tile * kOuterBlock + threadIdx.x;
  if (kl < a.M) {
    const uint32_t k = a.path_begin + (uint32_t)kl;
    OuterState<Real, NE, NC, double> st;
    init_state<Real, NE, NC, double>(a, st);
    fused_emit<Real, NE, NC>(a, f, st, 0, kl);
    for (int i = 0; i < a.n_dates; ++i) {
      advance<Real, NE, NC, double>(a, st, i, k, 0u, kTagOuter);
      fused_emit<Real, NE, NC>(a, f, st, i + 1, kl);
    }
  }
  __threadfence_block();
  __syncthreads();                           // the tile's table is complete and visible
  fused_inner_targets<Real>(a, f, tile, fused_lds);
}

// FP64 block partials of CVA_0 from the T_0 values of the fused kernel, in targets_kernel's order.
__global__ __launch_bounds__(kTargetBlock) void cva0_partials_kernel(int64_t M, const double* T0, double* partial) {
  __shared__ double red[kTargetBlock];
  const int64_t kl = (int64_t)blockIdx.x * kTargetBlock + threadIdx.x;
  red[threadIdx.x] = kl < M ? T0[kl] : 0.0;
  __syncthreads();
  for (int w = kTargetBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------------------------
// test hooks
// ------------------------------------------------------------------------------------
__global__ void philox_fill_kernel(uint32_t key0, uint32_t key1, uint32_t c1, uint32_t c2, uint32_t c3,
                                   int64_t k_begin, int64_t count, uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const u32x4 w = philox4x32_10((uint32_t)(k_begin + i), c1, c2, c3, key0, key1);
  out[4 * i + 0] = w.x;
  out[4 * i + 1] = w.y;
  out[4 * i + 2] = w.z;
  out[4 * i + 3] = w.w;
}

template <typename Real>
__global__ void normals_fill_kernel(uint32_t key0, uint32_t key1, int64_t path_begin, int64_t count,
                                    uint32_t step, int32_t n_z, Real* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t k = (uint32_t)(path_begin + i);
  for (int g = 0; 4 * g < n_z; ++g) {
    Real z[4];
    normals4<Real>(k, step, (uint32_t)g, key0, key1, z);
    for (int t = 0; t < 4 && 4 * g + t < n_z; ++t) out[i * n_z + 4 * g + t] = z[t];
  }
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------
#define HSIM_SHAPES(X) X(1, 1) X(1, 2) X(2, 1) X(2, 2) X(3, 3) X(10, 8)

bool outer_supported(int n_ccy, int n_cpty) {
#define X(ne, nc) if (n_ccy == ne && n_cpty == nc) return true;
  HSIM_SHAPES(X)
#undef X
  return false;
}

template <typename Real>
hipError_t launch_outer(const SimArgs<Real>& a, hipStream_t stream, bool fp32_integrals) {
  const dim3 grid((unsigned)((a.M + kOuterBlock - 1) / kOuterBlock));
  if constexpr (std::is_same<Real, float>::value) {
    if (fp32_integrals) {
#define X(ne, nc)                                                                                  \
      if (a.n_ccy == ne && a.n_cpty == nc) {                                                       \
        hipLaunchKernelGGL((outer_kernel<float, ne, nc, float>), grid, dim3(kOuterBlock), 0, stream, a); \
        return hipGetLastError();                                                                  \
      }
      HSIM_SHAPES(X)
#undef X
      return hipErrorInvalidValue;
    }
  }
#define X(ne, nc)                                                                   \
  if (a.n_ccy == ne && a.n_cpty == nc) {                                            \
    hipLaunchKernelGGL((outer_kernel<Real, ne, nc, double>), grid, dim3(kOuterBlock), 0, stream, a); \
    return hipGetLastError();                                                       \
  }
  HSIM_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename Real>
hipError_t launch_fused(const SimArgs<Real>& a, const FusedArgs& f, double* partial, double* cva0, hipStream_t stream) {
  const int64_t tiles = (a.M + kOuterBlock - 1) / kOuterBlock;
  const size_t lds = fused_lds_bytes(a.n_dates, a.n_cpty, sizeof(Real));
  hipError_t e = hipErrorInvalidValue;
#define X(ne, nc)                                                                                   \
  if (a.n_ccy == ne && a.n_cpty == nc) {                                                            \
    hipLaunchKernelGGL((fused_kernel<Real, ne, nc>), dim3((unsigned)tiles), dim3(kOuterBlock), lds, stream, a, f); \
    e = hipGetLastError();                                                                          \
  }
  HSIM_SHAPES(X)
#undef X
  if (e != hipSuccess) return e;
  const int64_t nblk = (a.M + kTargetBlock - 1) / kTargetBlock;
  hipLaunchKernelGGL(cva0_partials_kernel, dim3((unsigned)nblk), dim3(kTargetBlock), 0, stream, a.M, f.T0, partial);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kTargetBlock), 0, stream, partial, nblk, 1.0 / (double)a.M, cva0);
  return hipGetLastError();
}
template hipError_t launch_fused<float>(const SimArgs<float>&, const FusedArgs&, double*, double*, hipStream_t);
template hipError_t launch_fused<double>(const SimArgs<double>&, const FusedArgs&, double*, double*, hipStream_t);

size_t inner_order_bytes(int64_t M) { return (size_t)((M + kInnerBlock - 1) / kInnerBlock + 1) * sizeof(int32_t); }

hipError_t launch_inner(const InnerArgs& a, hipStream_t stream) {
  const int64_t tiles = (a.M + kInnerBlock - 1) / kInnerBlock;
  const size_t lds = (size_t)2 * (a.n_dates + 1) * kInnerBlock * sizeof(uint32_t);
  unsigned grid = (unsigned)tiles;
  if (a.order != nullptr) {
    hipLaunchKernelGGL(inner_order_kernel, dim3(1), dim3(1024), 0, stream, a.nb_block, a.block_paths, a.M, a.order);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int dev = 0, ncu = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, inner_kernel, kInnerBlock, lds)) != hipSuccess)
      return e;
    const int64_t resident = (int64_t)ncu * (per_cu > 0 ? per_cu : 1);
    grid = (unsigned)(tiles < resident ? tiles : resident);
  }
  hipLaunchKernelGGL(inner_kernel, dim3(grid), dim3(kInnerBlock), lds, stream, a);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_sample_rows(const SampleArgs<Real>& a, hipStream_t stream) {
  const int64_t nblk = (a.M * a.n_b + kTargetBlock - 1) / kTargetBlock;
  hipLaunchKernelGGL((sample_rows_kernel<Real>), dim3((unsigned)nblk), dim3(kTargetBlock), 0, stream, a);
  return hipGetLastError();
}
template hipError_t launch_sample_rows<float>(const SampleArgs<float>&, hipStream_t);
template hipError_t launch_sample_rows<double>(const SampleArgs<double>&, hipStream_t);

template <typename Real>
hipError_t launch_branch(const SimArgs<Real>& a, const BranchArgs& b, hipStream_t stream) {
  const dim3 grid((unsigned)((a.M * b.n_branch + kOuterBlock - 1) / kOuterBlock));
#define X(ne, nc)                                                                                  \
  if (a.n_ccy == ne && a.n_cpty == nc) {                                                           \
    hipLaunchKernelGGL((branch_kernel<Real, ne, nc>), grid, dim3(kOuterBlock), 0, stream, a, b);    \
    return hipGetLastError();                                                                      \
  }
  HSIM_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

size_t branch_stats_bytes(int64_t M) {
  return (size_t)kBranchStats * (size_t)((M + kTargetBlock - 1) / kTargetBlock) * sizeof(double);
}

hipError_t launch_branch_stats(int64_t M, int32_t B, bool phi_fp32, const void* phi, const double* xi,
                               double* partial, double* out, hipStream_t stream) {
  const int64_t nblk = (M + kTargetBlock - 1) / kTargetBlock;
  if (phi_fp32)
    hipLaunchKernelGGL((branch_stats_kernel<float>), dim3((unsigned)nblk), dim3(kTargetBlock), 0, stream, M, B,
                       (const float*)phi, xi, partial, nblk);
  else
    hipLaunchKernelGGL((branch_stats_kernel<double>), dim3((unsigned)nblk), dim3(kTargetBlock), 0, stream, M, B,
                       (const double*)phi, xi, partial, nblk);
  hipError_t e = hipGetLastError();
  for (int r = 0; r < kBranchStats && e == hipSuccess; ++r) {
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kTargetBlock), 0, stream, partial + r * nblk, nblk,
                       1.0 / (double)M, out + r);
    e = hipGetLastError();
  }
  return e;
}

template <typename Real>
hipError_t launch_targets(const TargetArgs<Real>& a, hipStream_t stream) {
  const int64_t nblk = (a.M + kTargetBlock - 1) / kTargetBlock;
  if (a.Lam)
    hipLaunchKernelGGL((targets_kernel<Real, kIntensity>), dim3((unsigned)nblk), dim3(kTargetBlock), 0, stream, a);
  else if (a.weight)
    hipLaunchKernelGGL((targets_kernel<Real, kAlive>), dim3((unsigned)nblk), dim3(kTargetBlock), 0, stream, a);
  else
    hipLaunchKernelGGL((targets_kernel<Real, kNested>), dim3((unsigned)nblk), dim3(kTargetBlock), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(kTargetBlock), 0, stream, a.partial, nblk,
                     1.0 / (double)a.M, a.cva0);
  return hipGetLastError();
}

hipError_t launch_philox_fill(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t k_begin,
                              int64_t count, uint32_t* out, hipStream_t s) {
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(philox_fill_kernel, dim3(blocks), dim3(256), 0, s, (uint32_t)seed,
                     (uint32_t)(seed >> 32), c1, c2, c3, k_begin, count, out);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_normals_fill(uint64_t seed, int64_t path_begin, int64_t count, int32_t step,
                               int32_t n_z, Real* out, hipStream_t s) {
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL((normals_fill_kernel<Real>), dim3(blocks), dim3(256), 0, s, (uint32_t)seed,
                     (uint32_t)(seed >> 32), path_begin, count, (uint32_t)step, n_z, out);
  return hipGetLastError();
}

template hipError_t launch_outer<float>(const SimArgs<float>&, hipStream_t, bool);
template hipError_t launch_outer<double>(const SimArgs<double>&, hipStream_t, bool);
template hipError_t launch_branch<float>(const SimArgs<float>&, const BranchArgs&, hipStream_t);
template hipError_t launch_branch<double>(const SimArgs<double>&, const BranchArgs&, hipStream_t);
template hipError_t launch_targets<float>(const TargetArgs<float>&, hipStream_t);
template hipError_t launch_targets<double>(const TargetArgs<double>&, hipStream_t);
template hipError_t launch_normals_fill<float>(uint64_t, int64_t, int64_t, int32_t, int32_t, float*,
                                               hipStream_t);
template hipError_t launch_normals_fill<double>(uint64_t, int64_t, int64_t, int32_t, int32_t,
                                                double*, hipStream_t);

}  // namespace hsim
