// The regression of the CVA targets in FP32 or FP64 (Section 2.1 e:nnp; Algorithms 1 and 2),
// date after date, every product a rocBLAS GEMM / GEMV in the working precision and every
// elementwise step a small kernel.  This is the library's precision path for the FP64 method and
// the plain FP32 baseline that the BF16 matrix-core kernel is measured against; it trains the
// same networks from the same initial draw with the same readings of the listing:
//   * inputs standardised per date (population mean / std in FP64), targets divided by their
//     root mean square; a date whose targets are all zero is not trained and predicts 0;
//   * contiguous batches of the stored row order; one simultaneous backpropagation step and one
//     Adam step per batch (fresh moments per date);
//   * pos = 0 until epoch floor(E/2); at its end the output layer is refitted by least squares on
//     the full sample (normal equations in FP64, guarded Cholesky: a column whose diagonal is
//     zero or whose pivot falls to 1e-12 of its diagonal gets weight 0), mu fixed; then pos = 1;
//   * after every epoch the full-sample pos = 1 loss (FP64 sums in a fixed order) and the best
//     parameters are kept, on the device.
// Buffers are column-major "unit-major per row": activation (u, r) at r * U + u.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "../../include/hsim.h"
#include "abi_internal.hpp"
#include "philox.hpp"
#include "regress.hpp"
#include "regress_plain.hpp"

namespace hsim {
namespace {

constexpr int kPB = 256;             // threads of the elementwise kernels
constexpr int64_t kPlainChunk = 4096;  // rows of a full-sample pass (at least)

// ---------------------------------------------------------------------------------- rocBLAS
template <typename T>
struct Blas;
template <>
struct Blas<float> {
  static rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                             const float* A, int lda, const float* B, int ldb, float beta, float* C, int ldc) {
    const float one = 1.0f;
    return rocblas_sgemm(h, ta, tb, m, n, k, &one, A, lda, B, ldb, &beta, C, ldc);
  }
  static rocblas_status gemv(rocblas_handle h, rocblas_operation t, int m, int n, const float* A, int lda,
                             const float* x, float beta, float* y) {
    const float one = 1.0f;
    return rocblas_sgemv(h, t, m, n, &one, A, lda, x, 1, &beta, y, 1);
  }
};
template <>
struct Blas<double> {
  static rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
                             const double* A, int lda, const double* B, int ldb, double beta, double* C, int ldc) {
    const double one = 1.0;
    return rocblas_dgemm(h, ta, tb, m, n, k, &one, A, lda, B, ldb, &beta, C, ldc);
  }
  static rocblas_status gemv(rocblas_handle h, rocblas_operation t, int m, int n, const double* A, int lda,
                             const double* x, double beta, double* y) {
    const double one = 1.0;
    return rocblas_dgemv(h, t, m, n, &one, A, lda, x, 1, &beta, y, 1);
  }
};

// One rocBLAS handle per device, created on first use with that device current.
int blas_handle(rocblas_handle* out) {
  static std::mutex mu;
  static rocblas_handle handles[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_error(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(HSIM_ERANGE, "device ordinal %d", dev);
  std::lock_guard<std::mutex> lock(mu);
  if (!handles[dev] && rocblas_create_handle(&handles[dev]) != rocblas_status_success)
    return fail(HSIM_EDEVICE, "rocblas_create_handle failed");
  *out = handles[dev];
  return HSIM_OK;
}

// ---------------------------------------------------------------------------------- kernels
// Fixed-order sum over a block of kPB threads (tree on LDS); the result in every thread.
template <typename A>
__device__ A block_sum(A v, A* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const A s = red[0];
  __syncthreads();
  return s;
}

// Scaling of one date into its record: block f < d_in a feature's mean and inverse std, block
// d_in the target's root mean square and the trained flag (FP64 sums over the M rows).
template <typename T>
__global__ __launch_bounds__(kPB) void plain_stats(const T* X, const T* Y, int64_t M, int n_feat, int d_in,
                                                   int date, T* rec, MlpLayout L) {
  __shared__ double r1[kPB], r2[kPB];
  const int f = blockIdx.x;
  const T* src = f < d_in ? X + ((int64_t)date * n_feat + f) * M : Y + (int64_t)date * M;
  double x1 = 0.0, x2 = 0.0;
  for (int64_t k = threadIdx.x; k < M; k += kPB) {
    const double v = (double)src[k];
    x1 += v;
    x2 += v * v;
  }
  x1 = block_sum(x1, r1);
  x2 = block_sum(x2, r2);
  if (threadIdx.x != 0) return;
  const double inv_m = 1.0 / (double)M;
  if (f < d_in) {
    const double mean = x1 * inv_m;
    const double sd = sqrt(fmax(x2 * inv_m - mean * mean, 0.0));
    rec[L.xmean_off() + f] = (T)mean;
    rec[L.xinv_off() + f] = sd > 0.0 ? (T)(1.0 / sd) : (T)1;
  } else {
    const double ys = sqrt(x2 * inv_m);
    rec[L.yscale_off()] = (T)ys;
    rec[L.trained_off()] = ys > 0.0 ? (T)1 : (T)0;
    for (int p = d_in; p < L.D; ++p) {
      rec[L.xmean_off() + p] = (T)0;
      rec[L.xinv_off() + p] = (T)1;
    }
  }
}

// Initial parameters of one date (the Philox draw U(-1/sqrt(fan_in), 1/sqrt(fan_in)) of the
// matrix-core kernel, biases and mu 0; or, warm-started, the parameters of `prev`), zero moments.
template <typename T>
__global__ __launch_bounds__(kPB) void plain_init(T* P, T* Mm, T* Vv, const T* prev, MlpLayout L, int d_in,
                                                  int init_tag, uint32_t key0, uint32_t key1) {
  const int np = L.n_params();
  for (int e = threadIdx.x; e < np; e += kPB) {
    Mm[e] = (T)0;
    Vv[e] = (T)0;
    if (prev) {
      P[e] = prev[e];
      continue;
    }
    T w = (T)0;
    int l = 0, o = 0, i = 0, fan = 0;
    if (e < L.wout_off()) {
      for (l = L.H; l >= 1 && e < L.w_off(l); --l) {
      }
      const int stride = l == 1 ? L.D : L.U;
      if (e < L.b_off(l)) {
        o = (e - L.w_off(l)) / stride;
        i = (e - L.w_off(l)) % stride;
        fan = l == 1 ? d_in : L.U;
        if (i < fan) {
          const uint32_t idx = (uint32_t)(o * fan + i);
          const u32x4 ph = philox4x32_10((uint32_t)(l - 1), idx >> 2, (uint32_t)init_tag, kTagInit, key0, key1);
          const uint32_t wd = (idx & 3) == 0 ? ph.x : (idx & 3) == 1 ? ph.y : (idx & 3) == 2 ? ph.z : ph.w;
          const double u = (2.0 * (double)grid23(wd) + 1.0) * 5.9604644775390625e-8;
          w = (T)((2.0 * u - 1.0) / sqrt((double)fan));
        }
      }
    } else if (e < L.bout_off()) {
      const int idx = e - L.wout_off();
      const u32x4 ph = philox4x32_10((uint32_t)L.H, (uint32_t)idx >> 2, (uint32_t)init_tag, kTagInit, key0, key1);
      const uint32_t wd = (idx & 3) == 0 ? ph.x : (idx & 3) == 1 ? ph.y : (idx & 3) == 2 ? ph.z : ph.w;
      const double u = (2.0 * (double)grid23(wd) + 1.0) * 5.9604644775390625e-8;
      w = (T)((2.0 * u - 1.0) / sqrt((double)L.U));
    }
    P[e] = w;
  }
}

// Rows [r0, r0 + n) of a date: standardised inputs A0 [n][d_in], scaled targets and weights.
template <typename T>
__global__ __launch_bounds__(kPB) void plain_stage(const T* X, const T* Y, const T* W, int64_t M, int n_feat,
                                                   int d_in, int date, int64_t r0, int n, const T* rec, MlpLayout L,
                                                   T* A0, T* y, T* w) {
  const int64_t t = (int64_t)blockIdx.x * kPB + threadIdx.x;
  if (t < (int64_t)n * d_in) {
    const int r = (int)(t / d_in), f = (int)(t % d_in);
    const T x = X[((int64_t)date * n_feat + f) * M + r0 + r];
    A0[t] = (x - rec[L.xmean_off() + f]) * rec[L.xinv_off() + f];
  }
  if (t < n && y) {
    y[t] = Y[(int64_t)date * M + r0 + t] / rec[L.yscale_off()];
    w[t] = W ? W[(int64_t)date * M + r0 + t] : (T)1;
  }
}

// A = relu(Z + b) in place on [n][U].
template <typename T>
__global__ __launch_bounds__(kPB) void plain_bias_relu(T* A, const T* b, int U, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * kPB + threadIdx.x;
  if (t >= total) return;
  const T z = A[t] + b[t % U];
  A[t] = z > (T)0 ? z : (T)0;
}

// Output rows: f = A_H w_out + b_out (f holds A_H w_out on entry).  Training: dpred and df of the
// batch loss (1/n) sum w (pred - y)^2, their sums for mu and b_out in the last two entries of
// `sums`.  Loss: the FP64 block sums of w (pred - y)^2 (pos = 1) into partial[blockIdx.x].
template <typename T>
__global__ __launch_bounds__(kPB) void plain_head(T* f, const T* y, const T* w, int n, const T* P, MlpLayout L,
                                                  int pos, int train, T* df, double* partial) {
  __shared__ double red[kPB];
  const int r = blockIdx.x * kPB + threadIdx.x;
  const T bout = P[L.bout_off()], mu = P[L.mu_off()];
  double v = 0.0;
  if (r < n) {
    const T fr = f[r] + bout;
    const T pred = (pos ? (fr > (T)0 ? fr : (T)0) : fr) + mu;
    if (train) {
      const T dp = (T)2 * w[r] * (pred - y[r]) / (T)n;
      f[r] = dp;                                  // dpred
      df[r] = pos ? (fr > (T)0 ? dp : (T)0) : dp;
    } else {
      const double e = (double)pred - (double)y[r];
      v = (double)w[r] * e * e;
    }
  }
  if (!train) {
    v = block_sum(v, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = v;
  }
}

// dZ_H = relu'(A_H) (w_out df^T), [n][U].
template <typename T>
__global__ __launch_bounds__(kPB) void plain_head_back(const T* A, const T* wout, const T* df, T* dZ, int U,
                                                       int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * kPB + threadIdx.x;
  if (t >= total) return;
  dZ[t] = A[t] > (T)0 ? wout[t % U] * df[t / U] : (T)0;
}

// dZ = dA masked by the ReLU of A (in place).
template <typename T>
__global__ __launch_bounds__(kPB) void plain_mask(T* dA, const T* A, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * kPB + threadIdx.x;
  if (t >= total) return;
  if (!(A[t] > (T)0)) dA[t] = (T)0;
}

// Gradients of mu and b_out: sums of dpred and df in a fixed order (one block).
template <typename T>
__global__ __launch_bounds__(kPB) void plain_head_sums(const T* dpred, const T* df, int n, T* G, MlpLayout L) {
  __shared__ T red[kPB];
  T a = (T)0, b = (T)0;
  for (int r = threadIdx.x; r < n; r += kPB) {
    a += dpred[r];
    b += df[r];
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) {
    G[L.mu_off()] = a;
    G[L.bout_off()] = b;
  }
}

// Adam on every parameter (ic1 = 1 / (1 - b1^t), ic2 = 1 / (1 - b2^t)).
template <typename T>
__global__ __launch_bounds__(kPB) void plain_adam(T* P, const T* G, T* Mm, T* Vv, int np, T lr, T b1, T b2, T eps,
                                                  T ic1, T ic2) {
  const int e = blockIdx.x * kPB + threadIdx.x;
  if (e >= np) return;
  const T g = G[e];
  const T m = b1 * Mm[e] + ((T)1 - b1) * g;
  const T v = b2 * Vv[e] + ((T)1 - b2) * g * g;
  Mm[e] = m;
  Vv[e] = v;
  P[e] = P[e] - lr * (m * ic1) / (sqrt(v * ic2) + eps);
}

// Weighted rows of the refit's normal equations in FP64: Hw[r] = sqrt(w_r) [A_H[r], 1],
// t[r] = sqrt(w_r) (y_r - mu).
template <typename T>
__global__ __launch_bounds__(kPB) void plain_gram_rows(const T* A, const T* y, const T* w, const T* P, MlpLayout L,
                                                       int n, double* Hw, double* t) {
  const int N = L.U + 1;
  const int64_t e = (int64_t)blockIdx.x * kPB + threadIdx.x;
  if (e >= (int64_t)n * N) return;
  const int r = (int)(e / N), u = (int)(e % N);
  const double s = sqrt((double)w[r]);
  Hw[e] = u < L.U ? s * (double)A[(int64_t)r * L.U + u] : s;
  if (u == 0) t[r] = s * ((double)y[r] - (double)P[L.mu_off()]);
}

// Least squares of the output layer from the normal equations G x = rhs (N = U + 1, column-major,
// the constant column last), guarded Cholesky in FP64 (one block): a column whose diagonal is zero
// or whose pivot falls to kRefitGuard times its diagonal is dependent on the columns before it
// and gets weight 0, which leaves the fitted values those of the full problem.
template <typename T>
__global__ __launch_bounds__(kPB) void plain_refit(double* G, double* rhs, T* P, MlpLayout L) {
  __shared__ double diag[kPlainMaxWidth + 1];
  const int N = L.U + 1;
  for (int k = threadIdx.x; k < N; k += kPB) diag[k] = G[(int64_t)k * N + k];
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    if (threadIdx.x == 0) {
      const double d = diag[k], p = G[(int64_t)k * N + k];
      G[(int64_t)k * N + k] = (d > 0.0 && p > kRefitGuard * d) ? sqrt(p) : 0.0;
    }
    __syncthreads();
    const double dkk = G[(int64_t)k * N + k];
    for (int i = k + 1 + threadIdx.x; i < N; i += kPB) G[(int64_t)k * N + i] = dkk > 0.0 ? G[(int64_t)k * N + i] / dkk : 0.0;
    __syncthreads();
    if (dkk > 0.0) {
      const int m = N - k - 1;
      for (int e = threadIdx.x; e < m * m; e += kPB) {
        const int i = k + 1 + e / m, j = k + 1 + e % m;   // L(i, j) -= L(i, k) L(j, k), j <= i
        if (j <= i) G[(int64_t)j * N + i] -= G[(int64_t)k * N + i] * G[(int64_t)k * N + j];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < N; ++i) {          // L y = rhs
      double s = rhs[i];
      for (int j = 0; j < i; ++j) s -= G[(int64_t)j * N + i] * rhs[j];
      rhs[i] = G[(int64_t)i * N + i] > 0.0 ? s / G[(int64_t)i * N + i] : 0.0;
    }
    for (int i = N - 1; i >= 0; --i) {     // L^T x = y
      double s = rhs[i];
      for (int j = i + 1; j < N; ++j) s -= G[(int64_t)i * N + j] * rhs[j];
      rhs[i] = G[(int64_t)i * N + i] > 0.0 ? s / G[(int64_t)i * N + i] : 0.0;
    }
  }
  __syncthreads();
  for (int u = threadIdx.x; u < L.U; u += kPB) P[L.wout_off() + u] = (T)rhs[u];
  if (threadIdx.x == 0) P[L.bout_off()] = (T)rhs[L.U];
}

// End of an epoch: loss = (1/M) sum of the partials (fixed order); loss history; the parameters
// are copied to the record when the loss is below the best so far (best[0], +inf at the start).
template <typename T>
__global__ __launch_bounds__(kPB) void plain_epoch_end(const double* partial, int nparts, double inv_m, double* best,
                                                       const T* P, T* rec, int np, T* hist) {
  __shared__ double red[kPB];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kPB) s += partial[i];
  s = block_sum(s, red) * inv_m;
  __shared__ int better;
  if (threadIdx.x == 0) {
    if (hist) *hist = (T)s;
    better = s < best[0];
    if (better) best[0] = s;
  }
  __syncthreads();
  if (better)
    for (int e = threadIdx.x; e < np; e += kPB) rec[e] = P[e];
}

template <typename T>
__global__ void plain_fill(T* p, T v, int64_t n, double* best) {
  const int64_t t = (int64_t)blockIdx.x * kPB + threadIdx.x;
  if (t < n) p[t] = v;
  if (best && t == 0) best[0] = INFINITY;
}

// Predictions of rows [r0, r0 + n): ((f)^+ + mu) y_scale, 0 for an untrained date.
template <typename T>
__global__ __launch_bounds__(kPB) void plain_out(const T* f, const T* rec, MlpLayout L, int n, T* out) {
  const int r = blockIdx.x * kPB + threadIdx.x;
  if (r >= n) return;
  const T fr = f[r] + rec[L.bout_off()];
  out[r] = rec[L.trained_off()] > (T)0 ? ((fr > (T)0 ? fr : (T)0) + rec[L.mu_off()]) * rec[L.yscale_off()] : (T)0;
}

unsigned blocks(int64_t n) { return (unsigned)((n + kPB - 1) / kPB); }

// ---------------------------------------------------------------------------------- buffers
struct PlainBufs {
  int64_t C;          // rows of the largest chunk
  size_t bytes;
  size_t o_state, o_grad, o_act, o_d0, o_d1, o_vec, o_ones, o_hw, o_t, o_gram, o_rhs, o_part, o_best;
};

template <typename T>
PlainBufs plain_layout(const cva_mlp_cfg* c, int n_reg, int64_t M) {
  const MlpLayout L{c->width, c->hidden, din_pad(c->d_in)};
  const int64_t batch = std::min<int64_t>(c->batch, M);
  PlainBufs b;
  b.C = std::max<int64_t>(batch, std::min<int64_t>(M, kPlainChunk));
  const size_t np = (size_t)L.n_params(), C = (size_t)b.C, U = (size_t)c->width, N = U + 1;
  const size_t D = (size_t)din_pad(c->d_in);
  const size_t dmax = std::max<size_t>(U, D);
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t r = o; o += align256(bytes); return r; };
  b.o_state = take(3 * np * n_reg * sizeof(T));            // parameters, m, v of every date
  b.o_grad = take(np * sizeof(T));
  b.o_act = take((D + c->hidden * U) * C * sizeof(T));  // A_0, A_1 .. A_H
  b.o_d0 = take(dmax * C * sizeof(T));
  b.o_d1 = take(dmax * C * sizeof(T));
  b.o_vec = take(4 * C * sizeof(T));                       // f, df, y, w
  b.o_ones = take(C * sizeof(T));
  b.o_hw = take(N * C * sizeof(double));
  b.o_t = take(C * sizeof(double));
  b.o_gram = take(N * N * sizeof(double));
  b.o_rhs = take(N * sizeof(double));
  b.o_part = take(((M + C - 1) / C) * ((C + kPB - 1) / kPB) * sizeof(double));
  b.o_best = take(sizeof(double));
  b.bytes = o;
  return b;
}

template <typename T>
struct PlainRun {
  const cva_mlp_cfg* c;
  MlpLayout L;
  rocblas_handle h;
  hipStream_t s;
  int64_t M;
  int n_feat, d_in;
  const T *X, *Y, *W;
  PlainBufs b;
  char* ws;
  T *A0, *Al[3], *d0, *d1, *f, *df, *y, *w, *ones;
  double *hw, *t, *gram, *rhs, *part, *best;

  int err = HSIM_OK;
  void blas(rocblas_status st, const char* what) {
    if (st != rocblas_status_success && err == HSIM_OK) err = fail(HSIM_EDEVICE, "rocBLAS %s failed (%d)", what, (int)st);
  }
  void launched(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess && err == HSIM_OK) err = device_error(e, what);
  }

  void bind() {
    A0 = (T*)(ws + b.o_act);
    for (int l = 0; l < 3; ++l) Al[l] = A0 + (size_t)L.D * b.C + (size_t)l * L.U * b.C;
    d0 = (T*)(ws + b.o_d0);
    d1 = (T*)(ws + b.o_d1);
    f = (T*)(ws + b.o_vec);
    df = f + b.C;
    y = df + b.C;
    w = y + b.C;
    ones = (T*)(ws + b.o_ones);
    hw = (double*)(ws + b.o_hw);
    t = (double*)(ws + b.o_t);
    gram = (double*)(ws + b.o_gram);
    rhs = (double*)(ws + b.o_rhs);
    part = (double*)(ws + b.o_part);
    best = (double*)(ws + b.o_best);
  }

  // Inputs of rows [r0, r0 + n) and the forward pass to f = A_H w_out (without b_out).
  void forward(const T* rec, const T* P, int date, int64_t r0, int n, bool with_targets) {
    hipLaunchKernelGGL(plain_stage<T>, dim3(blocks((int64_t)n * std::max(d_in, 1))), dim3(kPB), 0, s, X, Y, W, M,
                       n_feat, d_in, date, r0, n, rec, L, A0, with_targets ? y : (T*)nullptr, w);
    launched("input staging");
    const T* in = A0;
    int K = d_in, ldw = L.D;
    for (int l = 1; l <= L.H; ++l) {
      blas(Blas<T>::gemm(h, rocblas_operation_transpose, rocblas_operation_none, L.U, n, K, P + L.w_off(l), ldw, in,
                         K, (T)0, Al[l - 1], L.U),
           "forward GEMM");
      hipLaunchKernelGGL(plain_bias_relu<T>, dim3(blocks((int64_t)n * L.U)), dim3(kPB), 0, s, Al[l - 1],
                         P + L.b_off(l), L.U, (int64_t)n * L.U);
      launched("bias and ReLU");
      in = Al[l - 1];
      K = L.U;
      ldw = L.U;
    }
    blas(Blas<T>::gemv(h, rocblas_operation_transpose, L.U, n, Al[L.H - 1], L.U, P + L.wout_off(), (T)0, f),
         "output GEMV");
  }

  // Gradient of the batch loss into G (record order).
  void backward(const T* P, T* G, int n, int pos) {
    hipLaunchKernelGGL(plain_head<T>, dim3(blocks(n)), dim3(kPB), 0, s, f, y, w, n, P, L, pos, 1, df,
                       (double*)nullptr);
    launched("output rows");
    hipLaunchKernelGGL(plain_head_sums<T>, dim3(1), dim3(kPB), 0, s, f, df, n, G, L);
    launched("output sums");
    blas(Blas<T>::gemv(h, rocblas_operation_none, L.U, n, Al[L.H - 1], L.U, df, (T)0, G + L.wout_off()),
         "output-weight GEMV");
    hipLaunchKernelGGL(plain_head_back<T>, dim3(blocks((int64_t)n * L.U)), dim3(kPB), 0, s, Al[L.H - 1],
                       P + L.wout_off(), df, d0, L.U, (int64_t)n * L.U);
    launched("output backprop");
    T* dz = d0;
    T* da = d1;
    for (int l = L.H; l >= 1; --l) {
      const T* in = l == 1 ? A0 : Al[l - 2];
      const int K = l == 1 ? d_in : L.U, ldw = l == 1 ? L.D : L.U;
      blas(Blas<T>::gemm(h, rocblas_operation_none, rocblas_operation_transpose, K, L.U, n, in, K, dz, L.U, (T)0,
                         G + L.w_off(l), ldw),
           "weight-gradient GEMM");
      blas(Blas<T>::gemv(h, rocblas_operation_none, L.U, n, dz, L.U, ones, (T)0, G + L.b_off(l)), "bias GEMV");
      if (l > 1) {
        blas(Blas<T>::gemm(h, rocblas_operation_none, rocblas_operation_none, K, n, L.U, P + L.w_off(l), ldw, dz,
                           L.U, (T)0, da, K),
             "backprop GEMM");
        hipLaunchKernelGGL(plain_mask<T>, dim3(blocks((int64_t)n * K)), dim3(kPB), 0, s, da, Al[l - 2],
                           (int64_t)n * K);
        launched("ReLU mask");
        T* tmp = dz;
        dz = da;
        da = tmp;
      }
    }
  }

  // Full-sample pos = 1 loss after an epoch (best tracking on the device).
  void epoch_loss(const T* rec_scale, const T* P, T* rec, int date, T* hist) {
    int nparts = 0;
    for (int64_t r0 = 0; r0 < M; r0 += b.C) {
      const int n = (int)std::min<int64_t>(b.C, M - r0);
      forward(rec_scale, P, date, r0, n, true);
      hipLaunchKernelGGL(plain_head<T>, dim3(blocks(n)), dim3(kPB), 0, s, f, y, w, n, P, L, 1, 0, df,
                         part + nparts);
      launched("loss rows");
      nparts += (int)blocks(n);
    }
    hipLaunchKernelGGL(plain_epoch_end<T>, dim3(1), dim3(kPB), 0, s, part, nparts, 1.0 / (double)M, best, P, rec,
                       L.n_params(), hist);
    launched("epoch end");
  }

  // Algorithm 1's least-squares refit of the output layer on the full sample.
  void refit(const T* rec_scale, T* P, int date) {
    const int N = L.U + 1;
    bool first = true;
    for (int64_t r0 = 0; r0 < M; r0 += b.C) {
      const int n = (int)std::min<int64_t>(b.C, M - r0);
      forward(rec_scale, P, date, r0, n, true);
      hipLaunchKernelGGL(plain_gram_rows<T>, dim3(blocks((int64_t)n * N)), dim3(kPB), 0, s, Al[L.H - 1], y, w, P, L,
                         n, hw, t);
      launched("normal-equation rows");
      blas(Blas<double>::gemm(h, rocblas_operation_none, rocblas_operation_transpose, N, N, n, hw, N, hw, N,
                              first ? 0.0 : 1.0, gram, N),
           "Gram GEMM");
      blas(Blas<double>::gemv(h, rocblas_operation_none, N, n, hw, N, t, first ? 0.0 : 1.0, rhs), "rhs GEMV");
      first = false;
    }
    hipLaunchKernelGGL(plain_refit<T>, dim3(1), dim3(kPB), 0, s, gram, rhs, P, L);
    launched("refit solve");
  }
};

template <typename T>
int plain_fit(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int64_t M, int32_t n_feat, const void* X,
              const void* Y, const void* Wt, uint64_t seed, void* model, void* loss_hist, void* ws, size_t ws_bytes,
              hipStream_t s) {
  PlainRun<T> R;
  R.c = c;
  R.L = MlpLayout{c->width, c->hidden, din_pad(c->d_in)};
  R.s = s;
  R.M = M;
  R.n_feat = n_feat;
  R.d_in = c->d_in;
  R.X = (const T*)X;
  R.Y = (const T*)Y;
  R.W = (const T*)Wt;
  R.b = plain_layout<T>(c, n_reg, M);
  if (!ws || ws_bytes < R.b.bytes) return fail(HSIM_ENOWS, "workspace %zu < %zu bytes", ws_bytes, R.b.bytes);
  int rc = blas_handle(&R.h);
  if (rc) return rc;
  if (rocblas_set_stream(R.h, s) != rocblas_status_success) return fail(HSIM_EDEVICE, "rocblas_set_stream failed");
  R.ws = (char*)ws;
  R.bind();
  const MlpLayout& L = R.L;
  const int np = L.n_params(), rec_n = L.record();
  T* recs = (T*)model;
  T* state = (T*)(R.ws + R.b.o_state);
  T* G = (T*)(R.ws + R.b.o_grad);
  hipLaunchKernelGGL(plain_fill<T>, dim3(blocks(R.b.C)), dim3(kPB), 0, s, R.ones, (T)1, R.b.C, (double*)nullptr);
  hipLaunchKernelGGL(plain_fill<T>, dim3(blocks(np)), dim3(kPB), 0, s, G, (T)0, (int64_t)np, (double*)nullptr);
  R.launched("fill");
  const int64_t batch = std::min<int64_t>(c->batch, M);
  for (int j = 0; j < n_reg && R.err == HSIM_OK; ++j) {
    const int date = dates[j];
    T* rec = recs + (size_t)j * rec_n;
    T* P = state + (size_t)j * np;
    T* Mm = state + (size_t)(n_reg + j) * np;
    T* Vv = state + (size_t)(2 * n_reg + j) * np;
    T* hist = loss_hist ? (T*)loss_hist + (size_t)j * c->epochs : nullptr;
    hipLaunchKernelGGL(plain_stats<T>, dim3(c->d_in + 1), dim3(kPB), 0, s, R.X, R.Y, M, n_feat, c->d_in, date, rec, L);
    const T* prev = (c->warm_start && j > 0) ? recs + (size_t)(j - 1) * rec_n : nullptr;
    hipLaunchKernelGGL(plain_init<T>, dim3(1), dim3(kPB), 0, s, P, Mm, Vv, prev, L, c->d_in, c->init_tag,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    R.launched("stats and init");
    T trained = (T)0;
    if (hipMemcpyAsync(&trained, rec + L.trained_off(), sizeof(T), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return device_error(hipGetLastError(), "trained flag read");
    if (!(trained > (T)0)) {                     // all-zero targets: the initial network, predicts 0
      if (hipMemcpyAsync(rec, P, np * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return device_error(hipGetLastError(), "untrained record");
      if (hist && hipMemsetAsync(hist, 0, c->epochs * sizeof(T), s) != hipSuccess)
        return device_error(hipGetLastError(), "untrained loss history");
      continue;
    }
    hipLaunchKernelGGL(plain_fill<T>, dim3(1), dim3(kPB), 0, s, (T*)nullptr, (T)0, (int64_t)0, R.best);
    int pos = 0;
    double p1 = 1.0, p2 = 1.0;
    for (int epoch = 1; epoch <= c->epochs && R.err == HSIM_OK; ++epoch) {
      for (int64_t r0 = 0; r0 < M; r0 += batch) {
        const int n = (int)std::min<int64_t>(batch, M - r0);
        R.forward(rec, P, date, r0, n, true);
        R.backward(P, G, n, pos);
        p1 *= (double)c->beta1;
        p2 *= (double)c->beta2;
        hipLaunchKernelGGL(plain_adam<T>, dim3(blocks(np)), dim3(kPB), 0, s, P, G, Mm, Vv, np, (T)c->lr,
                           (T)c->beta1, (T)c->beta2, (T)c->eps, (T)(1.0 / (1.0 - p1)), (T)(1.0 / (1.0 - p2)));
        R.launched("Adam");
      }
      if (epoch == c->epochs / 2) {
        R.refit(rec, P, date);
        pos = 1;
      }
      R.epoch_loss(rec, P, rec, date, hist ? hist + (epoch - 1) : nullptr);
    }
  }
  if (R.err) return R.err;
  const hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? HSIM_OK : device_error(e, "plain regression");
}

template <typename T>
int plain_predict(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int64_t M, int32_t n_feat,
                  const void* X, const void* model, void* out, hipStream_t s) {
  // predictions need only the input buffers: a one-date layout without training state
  PlainRun<T> R;
  R.c = c;
  R.L = MlpLayout{c->width, c->hidden, din_pad(c->d_in)};
  R.s = s;
  R.M = M;
  R.n_feat = n_feat;
  R.d_in = c->d_in;
  R.X = (const T*)X;
  R.Y = nullptr;
  R.W = nullptr;
  cva_mlp_cfg cc = *c;
  cc.batch = (int32_t)std::min<int64_t>(M, kPlainChunk);
  R.b = plain_layout<T>(&cc, 1, M);
  int rc = blas_handle(&R.h);
  if (rc) return rc;
  if (rocblas_set_stream(R.h, s) != rocblas_status_success) return fail(HSIM_EDEVICE, "rocblas_set_stream failed");
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, R.b.bytes, s);
  if (e != hipSuccess) return device_error(e, "prediction buffers");
  R.ws = (char*)ws;
  R.bind();
  const int rec_n = R.L.record();
  for (int j = 0; j < n_reg && R.err == HSIM_OK; ++j) {
    const T* rec = (const T*)model + (size_t)j * rec_n;
    for (int64_t r0 = 0; r0 < M; r0 += R.b.C) {
      const int n = (int)std::min<int64_t>(R.b.C, M - r0);
      R.forward(rec, rec, dates[j], r0, n, false);
      hipLaunchKernelGGL(plain_out<T>, dim3(blocks(n)), dim3(kPB), 0, s, R.f, rec, R.L, n,
                         (T*)out + (size_t)j * M + r0);
      R.launched("prediction rows");
    }
  }
  e = hipFreeAsync(ws, s);
  if (R.err) return R.err;
  return e == hipSuccess ? HSIM_OK : device_error(e, "prediction buffers");
}

}  // namespace

size_t plain_workspace_bytes(const cva_mlp_cfg* c, int32_t n_reg, int64_t M) {
  return c->dtype == HSIM_REG_FP64 ? plain_layout<double>(c, n_reg, M).bytes : plain_layout<float>(c, n_reg, M).bytes;
}

int plain_fit(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int64_t M, int32_t n_feat, const void* X,
              const void* Y, const void* W, uint64_t seed, void* model, void* loss_hist, void* ws, size_t ws_bytes,
              hipStream_t s) {
  return c->dtype == HSIM_REG_FP64
             ? plain_fit<double>(c, n_reg, dates, M, n_feat, X, Y, W, seed, model, loss_hist, ws, ws_bytes, s)
             : plain_fit<float>(c, n_reg, dates, M, n_feat, X, Y, W, seed, model, loss_hist, ws, ws_bytes, s);
}

int plain_predict(const cva_mlp_cfg* c, int32_t n_reg, const int32_t* dates, int64_t M, int32_t n_feat,
                  const void* X, const void* model, void* out, hipStream_t s) {
  return c->dtype == HSIM_REG_FP64 ? plain_predict<double>(c, n_reg, dates, M, n_feat, X, model, out, s)
                                   : plain_predict<float>(c, n_reg, dates, M, n_feat, X, model, out, s);
}

}  // namespace hsim
