// Regression of the CVA targets by NN^+ networks (Section 2.1, e:nnp), trained by BaseAlg
// (Algorithm 1) with Adam, on gfx950 matrix cores.
//
// One workgroup (8 waves) trains the network of one pricing date; a persistent grid pulls
// dates from an atomic work counter, so every date of a regression set trains in one launch.
// Inside a workgroup a batch is processed in chunks of 64 rows staged in LDS:
//   forward   Z_l^T = W_l A_{l-1}^T         (MFMA 16x16x32 BF16, FP32 accumulation)
//   backward  dW_l += dZ_l^T A_{l-1}        (accumulated in registers over the whole batch)
//             dH_{l-1}^T = W_l^T dZ_l^T     (masked by the ReLU of layer l-1, in place)
// Weights and activations are BF16; accumulators, master weights, Adam moments, the output
// layer, the loss and the refit are FP32 (FP64 for the refit solve).  All reductions run in a
// fixed order, so results are bitwise reproducible.
//
// BaseAlg details (the readings of the listing): pos = 0 until epoch floor(E/2); at the end of
// that epoch the output layer is refitted by least squares on the full sample with the hidden
// layers frozen and mu fixed, then pos = 1; after every epoch the full-sample pos = 1 loss is
// evaluated and the best parameters are kept.  Inputs are standardised per date and targets
// divided by their root mean square.
#include <hip/hip_runtime.h>

#include "philox.hpp"
#include "regress.hpp"

namespace hsim {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Thread index hidden from loop-invariant code motion: address arithmetic derived from it is
// recomputed where it is used instead of being hoisted (and kept live) across the training loops.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------------------------------
// per-date input scaling (population mean / std of each feature, RMS of the target)
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_stats_kernel(const MlpArgs a) {
  __shared__ double s1[256], s2[256];
  const int job = blockIdx.x;
  const int f = blockIdx.y;                    // f < d_in: feature, f == d_in: target
  const int date = a.dates[job];
  const MlpLayout L{a.U, a.H};
  const float* src = f < a.d_in ? a.X + ((int64_t)date * a.n_feat + f) * a.M : a.Y + (int64_t)date * a.M;
  double x1 = 0.0, x2 = 0.0;
  for (int64_t k = threadIdx.x; k < a.M; k += 256) {
    const double v = src[k];
    x1 += v;
    x2 += v * v;
  }
  s1[threadIdx.x] = x1;
  s2[threadIdx.x] = x2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float* rec = a.model + (int64_t)job * L.record();
    const double inv_m = 1.0 / (double)a.M;
    if (f < a.d_in) {
      const double mean = s1[0] * inv_m;
      const double var = fmax(s2[0] * inv_m - mean * mean, 0.0);
      const double sd = sqrt(var);
      rec[L.xmean_off() + f] = (float)mean;
      rec[L.xinv_off() + f] = sd > 0.0 ? (float)(1.0 / sd) : 1.0f;
    } else {
      const double ys = sqrt(s2[0] * inv_m);
      rec[L.yscale_off()] = (float)ys;
      rec[L.trained_off()] = ys > 0.0 ? 1.0f : 0.0f;
      for (int p = a.d_in; p < kMlpDin; ++p) {
        rec[L.xmean_off() + p] = 0.0f;
        rec[L.xinv_off() + p] = 1.0f;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// shared-memory layout of the training / prediction workgroup
// ------------------------------------------------------------------------------------------
template <int U, int H>
struct Smem {
  static constexpr int D = kMlpDin, R = kMlpRows;
  static constexpr int SW0 = D + 8;            // padded row strides (bf16 elements)
  static constexpr int SW = U + 8;
  static constexpr int NT = U / 16;
  static constexpr int w_bytes = (U * SW0 + (H - 1) * U * SW) * (int)sizeof(__bf16);
  static constexpr int a_bytes = (R * SW0 + H * R * SW) * (int)sizeof(__bf16);
  static constexpr int f_count = 2 * H * U + 2 * U + 4 * R + 2 * D + 8;
  static constexpr int red_bytes = kMlpThreads * 8;
  static constexpr int bytes = w_bytes + a_bytes + f_count * 4 + red_bytes;

  __bf16* base;
  __device__ __bf16* W(int l) const {          // l = 1..H : [U][K_l + 8]
    return l == 1 ? base : base + U * SW0 + (l - 2) * U * SW;
  }
  __device__ __bf16* A(int l) const {          // l = 0..H : [R][K + 8]
    __bf16* a0 = base + w_bytes / (int)sizeof(__bf16);
    return l == 0 ? a0 : a0 + R * SW0 + (l - 1) * R * SW;
  }
  __device__ float* F() const { return (float*)((char*)base + w_bytes + a_bytes); }
  __device__ float* bias(int l) const { return F() + (l - 1) * U; }
  __device__ float* gbias(int l) const { return F() + H * U + (l - 1) * U; }
  __device__ float* wout() const { return F() + 2 * H * U; }
  __device__ float* gwout() const { return wout() + U; }
  __device__ float* fbuf() const { return gwout() + U; }
  __device__ float* ybuf() const { return fbuf() + R; }
  __device__ float* dpred() const { return ybuf() + R; }
  __device__ float* dff() const { return dpred() + R; }
  __device__ float* xmean() const { return dff() + R; }
  __device__ float* xinv() const { return xmean() + D; }
  __device__ float* scal() const { return xinv() + D; }   // [0] bout [1] mu [2] gbout [3] gmu [4] yscale
  __device__ double* red() const { return (double*)((char*)base + w_bytes + a_bytes + f_count * 4); }
  static constexpr int ldk(int l) { return l == 1 ? D : U; }
  static constexpr int lds(int l) { return l == 1 ? SW0 : SW; }
};

// Copy the FP32 parameters of one network into the workgroup's BF16 / FP32 LDS copies.
template <int U, int H>
__device__ void load_weights(const Smem<U, H>& S, const float* P, const MlpLayout& L) {
  for (int l = 1; l <= H; ++l) {
    const int K = S.ldk(l), SWl = S.lds(l);
    __bf16* W = S.W(l);
    const float* src = P + L.w_off(l);
    for (int e = opaque_tid(); e < U * K; e += kMlpThreads) W[(e / K) * SWl + e % K] = (__bf16)src[e];
    for (int e = opaque_tid(); e < U; e += kMlpThreads) S.bias(l)[e] = P[L.b_off(l) + e];
  }
  for (int e = opaque_tid(); e < U; e += kMlpThreads) S.wout()[e] = P[L.wout_off() + e];
  if (opaque_tid() == 0) {
    S.scal()[0] = P[L.bout_off()];
    S.scal()[1] = P[L.mu_off()];
  }
}

// Stage rows [r0, r0 + n) of one date: standardised inputs (BF16) and scaled targets.
template <int U, int H>
__device__ void load_chunk(const Smem<U, H>& S, const MlpArgs& a, int date, int64_t r0, int n) {
  constexpr int R = kMlpRows, D = kMlpDin;
  __bf16* A0 = S.A(0);
  for (int e = opaque_tid(); e < R * D; e += kMlpThreads) {
    const int r = e % R, f = e / R;
    float v = 0.0f;
    if (f < a.d_in && r < n)
      v = (a.X[((int64_t)date * a.n_feat + f) * a.M + r0 + r] - S.xmean()[f]) * S.xinv()[f];
    A0[r * S.SW0 + f] = (__bf16)v;
  }
  if (a.Y != nullptr && opaque_tid() < R) {     // prediction has no targets
    const int r = opaque_tid();
    S.ybuf()[r] = r < n ? a.Y[(int64_t)date * a.M + r0 + r] / S.scal()[4] : 0.0f;
  }
}

// Forward through the hidden layers (BF16 activations left in A(1..H)) and the output layer
// (FP32, into fbuf).
template <int U, int H>
__device__ void forward(const Smem<U, H>& S) {
  constexpr int R = kMlpRows, NT = U / 16, RT = R / 16;
  const int tid = opaque_tid(), wave = tid / 64, lane = tid % 64;
  const int li = lane % 16, lk = 8 * (lane / 16);
  for (int l = 1; l <= H; ++l) {
    const int K = S.ldk(l), SWl = S.lds(l);
    const __bf16* W = S.W(l);
    const __bf16* Ain = S.A(l - 1);
    __bf16* Aout = S.A(l);
    const float* b = S.bias(l);
#pragma unroll 1
    for (int j = wave; j < NT * RT; j += kMlpWaves) {
      const int ot = j / RT, rt = j % RT;
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int k0 = 0; k0 < K; k0 += 32) {
        const bf16x8 av = *(const bf16x8*)&W[(16 * ot + li) * SWl + k0 + lk];
        const bf16x8 bv = *(const bf16x8*)&Ain[(16 * rt + li) * SWl + k0 + lk];
        acc = mfma16(av, bv, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int out = 16 * ot + 4 * (lane / 16) + v, r = 16 * rt + li;
        const float h = acc[v] + b[out];
        Aout[r * S.SW + out] = (__bf16)(h > 0.0f ? h : 0.0f);
      }
    }
    __syncthreads();
  }
  // output layer: 8 threads per row, fixed-order butterfly of the partial sums
  {
    const int r = opaque_tid() / 8, qd = opaque_tid() % 8;
    const __bf16* Hh = S.A(H) + r * S.SW;
    float s = 0.0f;
    for (int u = qd * (U / 8); u < (qd + 1) * (U / 8); ++u) s += (float)Hh[u] * S.wout()[u];
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 4);
    if (qd == 0) S.fbuf()[r] = s + S.scal()[0];
  }
  __syncthreads();
}

template <int U, int H>
struct Tiles {
  static constexpr int NT = U / 16;
  static constexpr int T1 = NT * (kMlpDin / 16);
  static constexpr int TL = NT * NT;
  static constexpr int total = T1 + (H - 1) * TL;
  static constexpr int slots = (total + kMlpWaves - 1) / kMlpWaves;
  __device__ static int base(int l) { return l == 1 ? 0 : T1 + (l - 2) * TL; }
  __device__ static int count(int l) { return l == 1 ? T1 : TL; }
};

// dW_l += dZ_l^T A_{l-1} for the tiles this wave owns (tile g: wave g % waves, slot g / waves).
template <int U, int H>
__device__ void accumulate_dw(const Smem<U, H>& S, int l, f32x4* accW) {
  using TT = Tiles<U, H>;
  const int tid = opaque_tid(), wave = tid / 64, lane = tid % 64;
  const int li = lane % 16, lk = 8 * (lane / 16);
  const int K = S.ldk(l), SWin = S.lds(l), KT = K / 16;
  const __bf16* dZ = S.A(l);
  const __bf16* Ain = S.A(l - 1);
  const int b = TT::base(l), c = TT::count(l);
#pragma unroll
  for (int s = 0; s < TT::slots; ++s) {
    const int g = kMlpWaves * s + wave;
    if (g < b || g >= b + c) continue;
    const int ot = (g - b) / KT, it = (g - b) % KT;
    f32x4 acc = accW[s];
#pragma unroll
    for (int k0 = 0; k0 < kMlpRows; k0 += 32) {
      bf16x8 av, bv;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        av[t] = dZ[(k0 + lk + t) * S.SW + 16 * ot + li];
        bv[t] = Ain[(k0 + lk + t) * SWin + 16 * it + li];
      }
      acc = mfma16(av, bv, acc);
    }
    accW[s] = acc;
    asm volatile("" ::: "memory");      // keep the gathers of one tile together
  }
}

// dH_{l-1} = dZ_l W_l masked by the ReLU of layer l-1, written over A(l-1) (l >= 2).
template <int U, int H>
__device__ void backprop_layer(const Smem<U, H>& S, int l) {
  constexpr int R = kMlpRows, NT = U / 16, RT = R / 16, NJ = (NT * RT + kMlpWaves - 1) / kMlpWaves;
  const int tid = opaque_tid(), wave = tid / 64, lane = tid % 64;
  const int li = lane % 16, lk = 8 * (lane / 16);
  const __bf16* W = S.W(l);
  const __bf16* dZ = S.A(l);
  __bf16* Aprev = S.A(l - 1);
  f32x4 dh[NJ];
#pragma unroll
  for (int m = 0; m < NJ; ++m) {
    const int j = wave + kMlpWaves * m, it = j / RT, rt = j % RT;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if (j >= NT * RT) {
      dh[m] = acc;
      continue;
    }
    for (int k0 = 0; k0 < U; k0 += 32) {
      bf16x8 av;
#pragma unroll
      for (int t = 0; t < 8; ++t) av[t] = W[(k0 + lk + t) * S.SW + 16 * it + li];
      const bf16x8 bv = *(const bf16x8*)&dZ[(16 * rt + li) * S.SW + k0 + lk];
      acc = mfma16(av, bv, acc);
    }
    dh[m] = acc;
  }
  __syncthreads();                      // every read of A(l-1) and dZ_l is done
#pragma unroll
  for (int m = 0; m < NJ; ++m) {
    const int j = wave + kMlpWaves * m, it = j / RT, rt = j % RT;
    if (j >= NT * RT) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int in = 16 * it + 4 * (lane / 16) + v, r = 16 * rt + li;
      __bf16* p = &Aprev[r * S.SW + in];
      *p = (float)*p > 0.0f ? (__bf16)dh[m][v] : (__bf16)0.0f;
    }
  }
}

// out[u] += sum_r w[r] X[r][u] (w = 1 if null) over the R rows of a chunk: every thread sums a
// slice of rows of one column, the slices are combined in a fixed order.  Ends with a barrier
// only through the caller's next synchronisation; uses the reduction scratch.
template <int U, int H>
__device__ void column_sums(const Smem<U, H>& S, const __bf16* X, const float* w, float* out) {
  constexpr int R = kMlpRows, P = kMlpThreads / U, RP = R / P;
  float* part = (float*)S.red();
  const int tid = opaque_tid(), u = tid % U, p = tid / U;
  float acc = 0.0f;
#pragma unroll
  for (int r = p * RP; r < (p + 1) * RP; ++r) acc += (w ? w[r] : 1.0f) * (float)X[r * S.SW + u];
  part[p * U + u] = acc;
  __syncthreads();
  if (tid < U) {
    float sum = out[tid];
#pragma unroll
    for (int q = 0; q < P; ++q) sum += part[q * U + tid];
    out[tid] = sum;
  }
  __syncthreads();
}

// Gradients of one chunk, accumulated over the batch.
template <int U, int H>
__device__ void backward(const Smem<U, H>& S, int n, int pos, float inv_batch, f32x4* accW) {
  constexpr int R = kMlpRows;
  if (opaque_tid() < R) {
    const int r = opaque_tid();
    const float f = S.fbuf()[r];
    const float pred = (pos ? (f > 0.0f ? f : 0.0f) : f) + S.scal()[1];
    const float dp = r < n ? 2.0f * (pred - S.ybuf()[r]) * inv_batch : 0.0f;
    S.dpred()[r] = dp;
    S.dff()[r] = pos ? (f > 0.0f ? dp : 0.0f) : dp;
  }
  __syncthreads();
  if (opaque_tid() < 64) {                       // wave 0: fixed-order butterfly over the rows
    float gm = S.dpred()[opaque_tid()], gb = S.dff()[opaque_tid()];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      gm += __shfl_xor(gm, m);
      gb += __shfl_xor(gb, m);
    }
    if (opaque_tid() == 0) {
      S.scal()[3] += gm;
      S.scal()[2] += gb;
    }
  }
  column_sums<U, H>(S, S.A(H), S.dff(), S.gwout());
  {
    __bf16* Hh = S.A(H);
    for (int e = opaque_tid(); e < R * U; e += kMlpThreads) {
      const int r = e / U, u = e % U;
      __bf16* p = &Hh[r * S.SW + u];
      *p = (float)*p > 0.0f ? (__bf16)(S.dff()[r] * S.wout()[u]) : (__bf16)0.0f;
    }
  }
  __syncthreads();
  for (int l = H; l >= 1; --l) {
    accumulate_dw<U, H>(S, l, accW);
    column_sums<U, H>(S, S.A(l), nullptr, S.gbias(l));
    if (l > 1) backprop_layer<U, H>(S, l);
    __syncthreads();
  }
}

struct AdamStep {
  float lr, b1, b2, eps, ic1, ic2;      // ic1 = 1 / (1 - b1^t), ic2 = 1 / (1 - b2^t)
  __device__ float operator()(float p, float g, float* m, float* v) const {
    const float mm = b1 * *m + (1.0f - b1) * g;
    const float vv = b2 * *v + (1.0f - b2) * g * g;
    *m = mm;
    *v = vv;
    // hardware square root and reciprocal (about 1 ulp): the step size needs no more
    const float den = __builtin_amdgcn_sqrtf(vv * ic2) + eps;
    return p - lr * (mm * ic1) * __builtin_amdgcn_rcpf(den);
  }
};

template <int U, int H>
__device__ void adam_update(const Smem<U, H>& S, const MlpLayout& L, float* P, float* Mm, float* Vv,
                            const AdamStep& st, f32x4* accW) {
  using TT = Tiles<U, H>;
  const int tid = opaque_tid(), wave = tid / 64, lane = tid % 64;
  const int li = lane % 16;
#pragma unroll
  for (int s = 0; s < TT::slots; ++s) {
    const int g = kMlpWaves * s + wave;
    if (g >= TT::total) continue;
    const int l = g < TT::T1 ? 1 : 2 + (g - TT::T1) / TT::TL;
    const int b = TT::base(l), K = S.ldk(l), KT = K / 16;
    const int ot = (g - b) / KT, it = (g - b) % KT;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int out = 16 * ot + 4 * (lane / 16) + v, in = 16 * it + li;
      const int idx = L.w_off(l) + out * K + in;
      const float p = st(P[idx], accW[s][v], &Mm[idx], &Vv[idx]);
      P[idx] = p;
      S.W(l)[out * S.lds(l) + in] = (__bf16)p;
    }
    accW[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    asm volatile("" ::: "memory");      // one tile's moments in flight at a time
  }
  for (int l = 1; l <= H; ++l)
    for (int u = opaque_tid(); u < U; u += kMlpThreads) {
      const int idx = L.b_off(l) + u;
      const float p = st(P[idx], S.gbias(l)[u], &Mm[idx], &Vv[idx]);
      P[idx] = p;
      S.bias(l)[u] = p;
      S.gbias(l)[u] = 0.0f;
    }
  for (int u = opaque_tid(); u < U; u += kMlpThreads) {
    const int idx = L.wout_off() + u;
    const float p = st(P[idx], S.gwout()[u], &Mm[idx], &Vv[idx]);
    P[idx] = p;
    S.wout()[u] = p;
    S.gwout()[u] = 0.0f;
  }
  if (opaque_tid() == 0) {
    int idx = L.bout_off();
    float p = st(P[idx], S.scal()[2], &Mm[idx], &Vv[idx]);
    P[idx] = p;
    S.scal()[0] = p;
    idx = L.mu_off();
    p = st(P[idx], S.scal()[3], &Mm[idx], &Vv[idx]);
    P[idx] = p;
    S.scal()[1] = p;
    S.scal()[2] = 0.0f;
    S.scal()[3] = 0.0f;
  }
  __syncthreads();
}

// Full-sample loss with the output ReLU (pos = 1).
template <int U, int H>
__device__ float full_loss(const Smem<U, H>& S, const MlpArgs& a, int date) {
  double e = 0.0;
  for (int64_t r0 = 0; r0 < a.M; r0 += kMlpRows) {
    const int n = (int)min((int64_t)kMlpRows, a.M - r0);
    load_chunk<U, H>(S, a, date, r0, n);
    __syncthreads();
    forward<U, H>(S);
    if (opaque_tid() < n) {
      const float f = S.fbuf()[opaque_tid()];
      const float d = (f > 0.0f ? f : 0.0f) + S.scal()[1] - S.ybuf()[opaque_tid()];
      e += (double)d * (double)d;
    }
    __syncthreads();
  }
  double* red = S.red();
  red[opaque_tid()] = e;
  __syncthreads();
  for (int w = kMlpThreads / 2; w > 0; w >>= 1) {
    if (opaque_tid() < w) red[opaque_tid()] += red[opaque_tid() + w];
    __syncthreads();
  }
  const float L = (float)(red[0] / (double)a.M);
  __syncthreads();
  return L;
}

// Least-squares refit of (w_out, b_out) on the frozen hidden features, mu fixed.
template <int U, int H>
__device__ void refit(const Smem<U, H>& S, const MlpArgs& a, int date, const MlpLayout& L, float* P,
                      double* G) {
  constexpr int NT = U / 16, NG = NT * NT, GS = (NG + kMlpWaves - 1) / kMlpWaves, N = U + 1;
  const int tid = opaque_tid(), wave = tid / 64, lane = tid % 64;
  const int li = lane % 16, lk = 8 * (lane / 16);
  // per-chunk Gram tiles come from the matrix cores in FP32 (exact products of BF16 values,
  // 64-term sums); the sum over chunks is carried in FP64
  double accG[GS][4];
#pragma unroll
  for (int s = 0; s < GS; ++s)
#pragma unroll
    for (int v = 0; v < 4; ++v) accG[s][v] = 0.0;
  double hs = 0.0, hy = 0.0, ys = 0.0;        // thread u: sum h_u, sum h_u (y - mu); thread U: sum (y - mu)
  const float mu = S.scal()[1];
  for (int64_t r0 = 0; r0 < a.M; r0 += kMlpRows) {
    const int n = (int)min((int64_t)kMlpRows, a.M - r0);
    load_chunk<U, H>(S, a, date, r0, n);
    __syncthreads();
    forward<U, H>(S);
    const __bf16* Hh = S.A(H);
#pragma unroll
    for (int s = 0; s < GS; ++s) {
      const int g = kMlpWaves * s + wave;
      if (g >= NG) continue;
      const int ot = g / NT, it = g % NT;
      f32x4 part = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k0 = 0; k0 < kMlpRows; k0 += 32) {
        bf16x8 av, bv;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const bool ok = k0 + lk + t < n;
          av[t] = ok ? Hh[(k0 + lk + t) * S.SW + 16 * ot + li] : (__bf16)0.0f;
          bv[t] = ok ? Hh[(k0 + lk + t) * S.SW + 16 * it + li] : (__bf16)0.0f;
        }
        part = mfma16(av, bv, part);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) accG[s][v] += (double)part[v];
    }
    if (opaque_tid() < U) {
      const int u = opaque_tid();
#pragma unroll 1
      for (int r = 0; r < n; ++r) {
        const double h = (float)Hh[r * S.SW + u];
        hs += h;
        hy += h * (double)(S.ybuf()[r] - mu);
      }
    } else if (opaque_tid() == U) {
      for (int r = 0; r < n; ++r) ys += (double)(S.ybuf()[r] - mu);
    }
    __syncthreads();
  }
  // normal equations [H 1]^T [H 1] x = [H 1]^T (y - mu), stored row-major N x N, rhs after it
#pragma unroll
  for (int s = 0; s < GS; ++s) {
    const int g = kMlpWaves * s + wave;
    if (g >= NG) continue;
    const int ot = g / NT, it = g % NT;
#pragma unroll
    for (int v = 0; v < 4; ++v) G[(16 * ot + 4 * (lane / 16) + v) * N + 16 * it + li] = accG[s][v];
  }
  double* rhs = G + N * N;
  if (opaque_tid() < U) {
    G[opaque_tid() * N + U] = hs;
    G[U * N + opaque_tid()] = hs;
    rhs[opaque_tid()] = hy;
  } else if (opaque_tid() == U) {
    G[U * N + U] = (double)a.M;
    rhs[U] = ys;
  }
  __threadfence_block();
  __syncthreads();
  // ridge of kRefitRidge times the mean diagonal: keeps dead units (zero columns) at weight 0 and
  // bounds the conditioning of the normal equations
  if (opaque_tid() == 0) {
    double tr = 0.0;
#pragma unroll 1
    for (int i = 0; i < N; ++i) tr += G[i * N + i];
    const double lam = kRefitRidge * tr / N + 1e-300;
#pragma unroll 1
    for (int i = 0; i < N; ++i) G[i * N + i] += lam;
  }
  __threadfence_block();
  __syncthreads();
  // Cholesky (lower, in place), all threads on the trailing update
  for (int k = 0; k < N; ++k) {
    if (opaque_tid() == 0) G[k * N + k] = sqrt(G[k * N + k]);
    __threadfence_block();
    __syncthreads();
    const double dkk = G[k * N + k];
    for (int i = k + 1 + opaque_tid(); i < N; i += kMlpThreads) G[i * N + k] /= dkk;
    __threadfence_block();
    __syncthreads();
    const int m = N - k - 1;
    for (int e = opaque_tid(); e < m * m; e += kMlpThreads) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) G[i * N + j] -= G[i * N + k] * G[j * N + k];
    }
    __threadfence_block();
    __syncthreads();
  }
  if (opaque_tid() == 0) {
#pragma unroll 1
    for (int i = 0; i < N; ++i) {          // L y = rhs
      double s = rhs[i];
#pragma unroll 1
      for (int j = 0; j < i; ++j) s -= G[i * N + j] * rhs[j];
      rhs[i] = s / G[i * N + i];
    }
#pragma unroll 1
    for (int i = N - 1; i >= 0; --i) {     // L^T x = y
      double s = rhs[i];
#pragma unroll 1
      for (int j = i + 1; j < N; ++j) s -= G[j * N + i] * rhs[j];
      rhs[i] = s / G[i * N + i];
    }
  }
  __threadfence_block();
  __syncthreads();
  for (int u = opaque_tid(); u < U; u += kMlpThreads) {
    const float w = (float)rhs[u];
    P[L.wout_off() + u] = w;
    S.wout()[u] = w;
  }
  if (opaque_tid() == 0) {
    const float b = (float)rhs[U];
    P[L.bout_off()] = b;
    S.scal()[0] = b;
  }
  __threadfence_block();
  __syncthreads();
}

template <int U, int H>
__device__ void train_one(const Smem<U, H>& S, const MlpArgs& a, int job) {
  using TT = Tiles<U, H>;
  const MlpLayout L{U, H};
  const int date = a.dates[job];
  const int NP = L.n_params();
  float* rec = a.model + (int64_t)job * L.record();
  float* P = a.cur + (int64_t)job * NP;
  float* Mm = a.adam_m + (int64_t)job * NP;
  float* Vv = a.adam_v + (int64_t)job * NP;
  for (int e = opaque_tid(); e < kMlpDin; e += kMlpThreads) {
    S.xmean()[e] = rec[L.xmean_off() + e];
    S.xinv()[e] = rec[L.xinv_off() + e];
  }
  if (opaque_tid() == 0) S.scal()[4] = rec[L.yscale_off()];
  const bool trained = rec[L.trained_off()] != 0.0f;
  // initial parameters
  for (int l = 1; l <= H + 1; ++l) {
    const int fan_in = l == 1 ? a.d_in : U;
    const int rows = l <= H ? U : 1;
    const int stride = l == 1 ? kMlpDin : U;
    const int off = l <= H ? L.w_off(l) : L.wout_off();
    const float bound = rsqrtf((float)fan_in);
    for (int e = opaque_tid(); e < rows * stride; e += kMlpThreads) {
      const int o = e / stride, i = e % stride;
      float w = 0.0f;
      if (a.use_init) {
        w = rec[off + e];
      } else if (i < fan_in) {
        const uint32_t idx = (uint32_t)(o * fan_in + i);
        const u32x4 ph = philox4x32_10((uint32_t)(l - 1), idx >> 2, (uint32_t)a.init_tag, kTagInit, a.key0, a.key1);
        const uint32_t wd = (idx & 3) == 0 ? ph.x : (idx & 3) == 1 ? ph.y : (idx & 3) == 2 ? ph.z : ph.w;
        const double u = (2.0 * (double)grid23(wd) + 1.0) * 5.9604644775390625e-8;
        w = (float)((2.0 * u - 1.0) / sqrt((double)fan_in));
      }
      (void)bound;
      P[off + e] = w;
    }
    if (l <= H)
      for (int e = opaque_tid(); e < U; e += kMlpThreads) P[L.b_off(l) + e] = a.use_init ? rec[L.b_off(l) + e] : 0.0f;
  }
  if (opaque_tid() == 0) {
    P[L.bout_off()] = a.use_init ? rec[L.bout_off()] : 0.0f;
    P[L.mu_off()] = a.use_init ? rec[L.mu_off()] : 0.0f;
  }
  for (int e = opaque_tid(); e < NP; e += kMlpThreads) {
    Mm[e] = 0.0f;
    Vv[e] = 0.0f;
  }
  __threadfence_block();
  __syncthreads();
  if (!trained) {
    for (int e = opaque_tid(); e < NP; e += kMlpThreads) rec[e] = P[e];
    if (a.loss_hist)
      for (int e = opaque_tid(); e < a.epochs; e += kMlpThreads) a.loss_hist[(int64_t)job * a.epochs + e] = 0.0f;
    __syncthreads();
    return;
  }
  load_weights<U, H>(S, P, L);
  for (int l = 1; l <= H; ++l)
    for (int u = opaque_tid(); u < U; u += kMlpThreads) S.gbias(l)[u] = 0.0f;
  for (int u = opaque_tid(); u < U; u += kMlpThreads) S.gwout()[u] = 0.0f;
  if (opaque_tid() == 0) {
    S.scal()[2] = 0.0f;
    S.scal()[3] = 0.0f;
  }
  __syncthreads();

  float best = INFINITY;
  int pos = 0;
  int t = 0;
  float p1 = 1.0f, p2 = 1.0f;
  for (int epoch = 1; epoch <= a.epochs; ++epoch) {
    for (int64_t b0 = 0; b0 < a.M; b0 += a.batch) {
      const int64_t b1 = min(b0 + (int64_t)a.batch, a.M);
      const float inv_batch = 1.0f / (float)(b1 - b0);
      f32x4 accW[TT::slots];
#pragma unroll
      for (int s = 0; s < TT::slots; ++s) accW[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      for (int64_t r0 = b0; r0 < b1; r0 += kMlpRows) {
        const int n = (int)min((int64_t)kMlpRows, b1 - r0);
        load_chunk<U, H>(S, a, date, r0, n);
        __syncthreads();
        forward<U, H>(S);
        backward<U, H>(S, n, pos, inv_batch, accW);
      }
      ++t;
      p1 *= a.beta1;
      p2 *= a.beta2;
      const AdamStep st{a.lr, a.beta1, a.beta2, a.eps, 1.0f / (1.0f - p1), 1.0f / (1.0f - p2)};
      adam_update<U, H>(S, L, P, Mm, Vv, st, accW);
    }
    if (epoch == a.epochs / 2) {
      refit<U, H>(S, a, date, L, P, a.gram + (int64_t)job * (U + 1) * (U + 2));
      pos = 1;
    }
    const float loss = full_loss<U, H>(S, a, date);
    if (a.loss_hist && opaque_tid() == 0) a.loss_hist[(int64_t)job * a.epochs + epoch - 1] = loss;
    if (loss < best) {
      best = loss;
      __threadfence_block();
      __syncthreads();
      for (int e = opaque_tid(); e < NP; e += kMlpThreads) rec[e] = P[e];
    }
    __syncthreads();
  }
}

template <int U, int H>
__global__ __launch_bounds__(kMlpThreads) void mlp_train_kernel(const MlpArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  Smem<U, H> S{(__bf16*)smem_raw};
  __shared__ int s_job;
  for (;;) {
    if (opaque_tid() == 0) s_job = atomicAdd(a.queue, 1);
    __syncthreads();
    const int job = s_job;
    __syncthreads();
    if (job >= a.n_reg) break;
    train_one<U, H>(S, a, job);
    __syncthreads();
  }
}

// Prediction with the best parameters: out[job][k] = ((f)^+ + mu) * y_scale (0 if untrained).
template <int U, int H>
__global__ __launch_bounds__(kMlpThreads) void mlp_predict_kernel(const MlpArgs a, float* out) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  Smem<U, H> S{(__bf16*)smem_raw};
  const MlpLayout L{U, H};
  const int job = blockIdx.y;
  const int date = a.dates[job];
  const float* rec = a.model + (int64_t)job * L.record();
  const int64_t rows_per_block = 64 * kMlpRows;
  const int64_t k0 = (int64_t)blockIdx.x * rows_per_block;
  if (k0 >= a.M) return;
  const bool trained = rec[L.trained_off()] != 0.0f;
  if (!trained) {
    for (int64_t k = k0 + opaque_tid(); k < min(k0 + rows_per_block, a.M); k += kMlpThreads)
      out[(int64_t)job * a.M + k] = 0.0f;
    return;
  }
  for (int e = opaque_tid(); e < kMlpDin; e += kMlpThreads) {
    S.xmean()[e] = rec[L.xmean_off() + e];
    S.xinv()[e] = rec[L.xinv_off() + e];
  }
  if (opaque_tid() == 0) S.scal()[4] = rec[L.yscale_off()];
  load_weights<U, H>(S, rec, L);
  __syncthreads();
  const float ysc = rec[L.yscale_off()];
  for (int64_t r0 = k0; r0 < min(k0 + rows_per_block, a.M); r0 += kMlpRows) {
    const int n = (int)min((int64_t)kMlpRows, a.M - r0);
    load_chunk<U, H>(S, a, date, r0, n);
    __syncthreads();
    forward<U, H>(S);
    if (opaque_tid() < n) {
      const float f = S.fbuf()[opaque_tid()];
      out[(int64_t)job * a.M + r0 + opaque_tid()] = ((f > 0.0f ? f : 0.0f) + S.scal()[1]) * ysc;
    }
    __syncthreads();
  }
}

__global__ void fill_i32(int32_t* p, int32_t v) { p[opaque_tid()] = v; }

#define HSIM_MLP_SHAPES(X) X(32, 1) X(32, 2) X(64, 2) X(128, 2) X(128, 3)

bool mlp_supported(int U, int H) {
#define X(u, h) if (U == u && H == h) return true;
  HSIM_MLP_SHAPES(X)
#undef X
  return false;
}

hipError_t launch_mlp_stats(const MlpArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mlp_stats_kernel, dim3(a.n_reg, a.d_in + 1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_train(const MlpArgs& a, int n_workgroups, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(1), 0, s, a.queue, 0);
#define X(u, h)                                                                                  \
  if (a.U == u && a.H == h) {                                                                    \
    const int bytes = Smem<u, h>::bytes;                                                         \
    hipFuncSetAttribute((const void*)mlp_train_kernel<u, h>,                                     \
                        hipFuncAttributeMaxDynamicSharedMemorySize, bytes);                      \
    hipLaunchKernelGGL((mlp_train_kernel<u, h>), dim3(n_workgroups), dim3(kMlpThreads), bytes, s, a); \
    return hipGetLastError();                                                                    \
  }
  HSIM_MLP_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_predict(const MlpArgs& a, float* out, hipStream_t s) {
  const unsigned gx = (unsigned)((a.M + 64 * kMlpRows - 1) / (64 * kMlpRows));
#define X(u, h)                                                                                  \
  if (a.U == u && a.H == h) {                                                                    \
    const int bytes = Smem<u, h>::bytes;                                                         \
    hipFuncSetAttribute((const void*)mlp_predict_kernel<u, h>,                                   \
                        hipFuncAttributeMaxDynamicSharedMemorySize, bytes);                      \
    hipLaunchKernelGGL((mlp_predict_kernel<u, h>), dim3(gx, a.n_reg), dim3(kMlpThreads), bytes, s, a, out); \
    return hipGetLastError();                                                                    \
  }
  HSIM_MLP_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace hsim
