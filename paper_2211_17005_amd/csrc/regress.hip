// Regression of the CVA targets by NN^+ networks (Section 2.1, e:nnp), trained by BaseAlg
// (Algorithm 1) with Adam, on gfx950 matrix cores.
//
// One workgroup (8 waves) trains the network of one pricing date; a persistent grid pulls
// dates from an atomic work counter, so every date of a regression set trains in one launch.
// Inside a workgroup a batch is processed in chunks of 64 rows staged in LDS, every matrix kept
// row-major ([row][feature], weights [out][in]):
//   forward   Z_l^T = W_l A_{l-1}^T         (MFMA 16x16x32 BF16, FP32 accumulation)
//   backward  dW_l += dZ_l^T A_{l-1}        (accumulated in registers over the whole batch)
//             dH_{l-1}^T = W_l^T dZ_l^T     (masked by the ReLU of layer l-1, in place)
// Operands whose contraction runs down a column (dZ_l^T, A_{l-1} and W_l^T above) are read
// with the LDS transpose load of gfx950, so no matrix is stored twice and no operand is
// gathered element by element.  Each wave computes a block of output tiles so that every
// fragment it reads feeds several MFMAs.
// Weights and activations are BF16; accumulators, master weights, Adam moments, the output
// layer, the loss and the refit are FP32 (FP64 for the refit solve).  All reductions run in a
// fixed order, so results are bitwise reproducible.
//
// BaseAlg details (the readings of the listing): pos = 0 until epoch floor(E/2); at the end of
// that epoch the output layer is refitted by least squares on the full sample with the hidden
// layers frozen and mu fixed, then pos = 1; after every epoch the full-sample pos = 1 loss is
// evaluated and the best parameters are kept.  Inputs are standardised per date and targets
// divided by their root mean square.
//
// Wave tiling variants (the autotuner's tile shapes): this file is compiled once per variant
// HSIM_MLP_TILE (0: the default; regress_tile1.hip, regress_tile2.hip), each into a namespace
// of its own, and the C ABI dispatches on cva_mlp_cfg.tile.  A variant changes the block of
// output tiles a wave owns in the forward and back-propagation products (out x row tiles) and in
// the weight-gradient products (out x in tiles); the arithmetic of each tile is the same.
#include <hip/hip_runtime.h>

#include "philox.hpp"
#include "regress.hpp"

#ifndef HSIM_MLP_TILE
#define HSIM_MLP_TILE 0
#endif
#define HSIM_MLP_NS_CAT(t) tile##t
#define HSIM_MLP_NS(t) HSIM_MLP_NS_CAT(t)

namespace hsim {
namespace HSIM_MLP_NS(HSIM_MLP_TILE) {

constexpr int kTile = HSIM_MLP_TILE;
static_assert(kTile >= 0 && kTile < kMlpTiles, "tile variant");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
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

// LDS transpose load: inside each group of 16 lanes, lane 4t + q supplies the address of four
// consecutive 16-bit elements, and lane i of the group receives element i % 4 of lane
// 4t + i / 4 as its element t (t, q = 0..3).
__device__ __forceinline__ bf16x4 lds_read_tr(const __bf16* p) {
  typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
  return __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)p);
}

// Element (row, col) of a row-major LDS matrix.  The 16-byte granules of a row are swizzled (granule
// index XOR bit 2 of the row) and rows are padded to 32 bytes modulo 128, so that the 16-byte row
// reads of eight consecutive rows and the transpose loads of four consecutive rows both spread
// over distinct banks.
__device__ __forceinline__ int lidx(int row, int col, int stride) {
  return row * stride + (col ^ (((row >> 2) & 1) << 3));
}

// Per-lane element offsets of the operand reads and tile writes of one swizzled LDS matrix of
// stride S.  Fragments start at row0 % 16 == 0 (row reads) or row0 % 8 == 0 (column reads) and at
// col0 % 16 == 0, so the swizzle of every address a lane touches is fixed by the lane: each read
// is one instruction at a constant offset from these.
struct LaneOffsets {
  int rows, cols_lo, cols_hi, tile;
  __device__ __forceinline__ explicit LaneOffsets(int S) {
    const int lane = (int)((unsigned)opaque_tid() & 63u), i = lane & 15, g = lane >> 4, s = ((i >> 2) & 1) << 3;
    rows = i * S + ((8 * g) ^ s);
    cols_lo = (8 * g + i / 4) * S + 4 * (i % 4);
    cols_hi = (8 * g + i / 4 + 4) * S + ((4 * (i % 4)) ^ 8);
    tile = i * S + ((4 * g) ^ s);
  }
};

// The offsets of a thread for the two row strides of the workgroup (inputs / first layer and
// hidden layers), built once and kept in registers through the training loops.
struct Lanes {
  LaneOffsets o0, o;
  // The same with the wave's own output block (forward and back-propagation products) folded in,
  // so that those reads and stores are one instruction at an immediate offset: row reads of its
  // out block of W (strides S0, S), of its row block of the layer input or dZ (S0, S), its tile
  // strips (S), and the transpose loads of its out block of W in the back-propagation (S).
  int rows_ob0, rows_ob, rows_rb0, rows_rb, tile_w, bp_lo, bp_hi;
  __device__ __forceinline__ Lanes(int S0, int S) : o0(S0), o(S) {}
  __device__ __forceinline__ const LaneOffsets& of(int S, int S0) const { return S == S0 ? o0 : o; }
};

// Wave index of the thread, wave-uniform (scalar register).
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Lane permutations of the data-parallel primitives (row = 16 lanes): swap neighbours, swap pairs,
// mirror inside each half row, mirror inside each row.
#define HSIM_DPP(v, ctrl) __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, false))

// Sum of v over the 64 lanes of the wave in a fixed order, returned in every lane.
__device__ __forceinline__ float wave_sum(float v) {
  v += HSIM_DPP(v, 0xB1);               // quad_perm (1, 0, 3, 2)
  v += HSIM_DPP(v, 0x4E);               // quad_perm (2, 3, 0, 1)
  v += HSIM_DPP(v, 0x141);              // half-row mirror
  v += HSIM_DPP(v, 0x140);              // row mirror
  return (__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)) +
          __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16))) +
         (__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32)) +
          __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48)));
}

// v + (v of lane l ^ m) for m = 16 or 32, with the gfx950 lane swaps (across 16-lane rows, across
// the wave's halves): a swap of v with itself leaves the partner lane's v in one of the results.
template <int m>
__device__ __forceinline__ float xor_sum(float v) {
  static_assert(m == 16 || m == 32, "row or half-wave exchange");
  const unsigned x = __float_as_uint(v);
  const auto sw = m == 32 ? __builtin_amdgcn_permlane32_swap(x, x, false, false)
                          : __builtin_amdgcn_permlane16_swap(x, x, false, false);
  return __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
}

// MFMA operand whose eight k values run down a column: lane l receives
// M[row0 + 8 (l / 16) + t][col0 + l % 16], t = 0..7 (two transpose loads of four rows each).
__device__ __forceinline__ bf16x8 frag_cols(const __bf16* M, const LaneOffsets& o, int S, int row0, int col0) {
  const bf16x4 lo = lds_read_tr(M + o.cols_lo + row0 * S + col0);
  const bf16x4 hi = lds_read_tr(M + o.cols_hi + row0 * S + col0);
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
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
  static constexpr int SW0 = D + 16;           // padded row strides (bf16 elements)
  static constexpr int SW = U + 16;
  static constexpr int w_bytes = (U * SW0 + (H - 1) * U * SW) * (int)sizeof(__bf16);
  static constexpr int a_bytes = (2 * R * SW0 + H * R * SW) * (int)sizeof(__bf16);
  static constexpr int f_count = 2 * H * U + 2 * U + 5 * R + 2 * D + 8;
  static constexpr int red_bytes = kMlpThreads * 8;
  static constexpr int bytes = w_bytes + a_bytes + f_count * 4 + red_bytes;
  static_assert(bytes <= 160 * 1024, "LDS of one workgroup");
  static_assert(w_bytes % 16 == 0 && a_bytes % 16 == 0 && (f_count * 4) % 16 == 0, "16-byte sections");

  __bf16* base;
  __device__ __bf16* W(int l) const {          // l = 1..H : [U][K_l + 8]
    return l == 1 ? base : base + U * SW0 + (l - 2) * U * SW;
  }
  __device__ __bf16* A(int l) const {          // l = 0..H : [R][K + 8]
    __bf16* a0 = base + w_bytes / (int)sizeof(__bf16);
    return l == 0 ? a0 : a0 + 2 * R * SW0 + (l - 1) * R * SW;
  }
  // the second input buffer: a training chunk's successor is staged while it is back-propagated
  __device__ __bf16* A0b() const { return base + w_bytes / (int)sizeof(__bf16) + R * SW0; }
  __device__ __bf16* in_buf(int parity) const { return parity ? A0b() : A(0); }
  __device__ float* F() const { return (float*)((char*)base + w_bytes + a_bytes); }
  __device__ float* bias(int l) const { return F() + (l - 1) * U; }
  __device__ float* gbias(int l) const { return F() + H * U + (l - 1) * U; }
  __device__ float* wout() const { return F() + 2 * H * U; }
  __device__ float* gwout() const { return wout() + U; }
  __device__ float* fbuf() const { return gwout() + U; }
  __device__ float* ybuf() const { return fbuf() + R; }
  __device__ float* dpred() const { return ybuf() + R; }
  __device__ float* dff() const { return dpred() + R; }
  __device__ float* wbuf() const { return dff() + R; }     // row weights of the chunk (refit)
  __device__ float* xmean() const { return wbuf() + R; }
  __device__ float* xinv() const { return xmean() + D; }
  __device__ float* scal() const { return xinv() + D; }   // [0] bout [1] mu [2] gbout [3] gmu [4] yscale
  // [6..7] base of the row weights (null: none), kept in LDS so that no register holds it
  __device__ const float** wbase() const { return (const float**)(scal() + 6); }
  __device__ char* red() const { return (char*)base + w_bytes + a_bytes + f_count * 4; }
  __device__ float* fpart() const { return (float*)red(); }   // [U/16/BO][R] output partials
  static constexpr int ldk(int l) { return l == 1 ? D : U; }
  static constexpr int lds(int l) { return l == 1 ? SW0 : SW; }
};

// Output tiles (16 x 16) of a forward or backprop layer, U/16 by 4 per chunk: each wave owns a
// block of BO x BR of them, waves laid out out-block fastest.
template <int U>
struct Blk {
  static constexpr int NT = U / 16, RT = kMlpRows / 16;
  // variant 0: 2 x 2 tiles at 128 units; 1: 4 x 1; 2: 1 x 4
  static constexpr int BO = kTile == 0 ? (U >= 64 ? 2 : 1) : kTile == 1 ? (U >= 128 ? 4 : U >= 64 ? 2 : 1) : 1;
  static constexpr int BR = kTile == 0 ? (U >= 128 ? 2 : 1) : kTile == 1 ? 1 : (U >= 128 ? 4 : U >= 64 ? 2 : 1);
  static constexpr int NOB = NT / BO;
  static_assert(NOB * (RT / BR) == kMlpWaves, "one block per wave");
  static_assert(BO * BR <= 8, "a lane's ReLU mask bits of a layer fit in one word");
};

// A thread's lane offsets with its wave's output block of the forward and back-propagation
// products (built once per fit).
template <int U, int H>
__device__ __forceinline__ Lanes make_lanes() {
  using B = Blk<U>;
  constexpr int S0 = Smem<U, H>::SW0, S = Smem<U, H>::SW;
  Lanes ln(S0, S);
  const int wave = wave_id(), ob = wave % B::NOB, rb = wave / B::NOB;
  ln.rows_ob0 = ln.o0.rows + 16 * ob * B::BO * S0;
  ln.rows_ob = ln.o.rows + 16 * ob * B::BO * S;
  ln.rows_rb0 = ln.o0.rows + 16 * rb * B::BR * S0;
  ln.rows_rb = ln.o.rows + 16 * rb * B::BR * S;
  ln.tile_w = ln.o.tile + 16 * rb * B::BR * S + 16 * ob * B::BO;
  ln.bp_lo = ln.o.cols_lo + 16 * ob * B::BO;
  ln.bp_hi = ln.o.cols_hi + 16 * ob * B::BO;
  return ln;
}

// Weight-gradient tiles of layer L (U/16 out tiles by K_L/16 in tiles), held in registers over a
// batch: each wave owns a block of BO x BI of them (in block fastest); with fewer tiles than
// waves the remaining waves own none.
constexpr int dw_kt(int U, int L) { return (L == 1 ? kMlpDin : U) / 16; }
constexpr int dw_tw(int U, int L) {
  return (U / 16) * dw_kt(U, L) >= kMlpWaves ? (U / 16) * dw_kt(U, L) / kMlpWaves : 1;
}
constexpr int dw_base(int U, int L) { return L == 1 ? 0 : dw_tw(U, 1) + (L - 2) * dw_tw(U, 2); }
constexpr int dw_slots(int U, int H) { return dw_tw(U, 1) + (H - 1) * dw_tw(U, 2); }
constexpr int cmin(int a, int b) { return a < b ? a : b; }

template <int U, int L>
struct DwMap {
  static constexpr int NT = U / 16, KT = dw_kt(U, L), TW = dw_tw(U, L);
  static constexpr int BI = cmin(cmin(KT, TW), kTile == 0 ? 4 : kTile == 1 ? 2 : KT);
  static constexpr int BO = TW / BI;
  static constexpr int NIB = KT / BI, NOB = NT / BO;
  static_assert(BO * BI == TW && NIB * NOB * TW == NT * KT && NIB * NOB <= kMlpWaves, "tiling");
  // Block (in block fastest) of a wave.  The waves of a workgroup are placed on the four SIMDs in
  // turn (wave w on SIMD w % 4), so waves w and w + 4 share a SIMD; they take neighbouring blocks,
  // which puts the blocks of in block 0 (the bias tiles' extra products) on different SIMDs.
  static __device__ __forceinline__ int block(int wave) { return (wave % 4) * 2 + wave / 4; }
  static __device__ __forceinline__ int ib_of(int wave) { return block(wave) % NIB; }
  static __device__ __forceinline__ int ob_of(int wave) { return block(wave) / NIB; }
  static_assert(kMlpWaves == 8, "block(): two waves per SIMD");
};

// Weights of layer l from FP32 global memory into the BF16 LDS copy, two consecutive inputs of
// one output per thread and vector: an 8-byte global load (a network's parameters start 8-byte
// aligned: their count is even) and one 4-byte LDS store; each thread issues the loads of a batch
// of pairs before it stores any of them (the copy is latency-bound otherwise).
template <int U, int H, int l>
__device__ __forceinline__ void load_layer_weights(const Smem<U, H>& S, const float* __restrict__ src, int t) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  constexpr int K = Smem<U, H>::ldk(l), SWl = Smem<U, H>::lds(l);
  constexpr int PER = U * K / (2 * kMlpThreads), kBatch = PER < 8 ? PER : 8;   // pairs per thread
  static_assert(PER * 2 * kMlpThreads == U * K && PER % kBatch == 0, "whole batches of pairs per thread");
  __bf16* W = S.W(l);
  for (int i0 = 0; i0 < PER; i0 += kBatch) {
    f32x2 v[kBatch];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) v[i] = *(const f32x2*)&src[2 * (t + (i0 + i) * kMlpThreads)];
#pragma unroll
    for (int i = 0; i < kBatch; ++i) {
      const int e = 2 * (t + (i0 + i) * kMlpThreads);
      bf16x2 h;
      h[0] = (__bf16)v[i][0];
      h[1] = (__bf16)v[i][1];
      *(bf16x2*)&W[lidx(e / K, e % K, SWl)] = h;
    }
  }
}

// Copy the FP32 parameters of one network into the workgroup's BF16 / FP32 LDS copies.
template <int U, int H>
__device__ void load_weights(const Smem<U, H>& S, const float* P, const MlpLayout& L) {
  const int t = opaque_tid();
  load_layer_weights<U, H, 1>(S, P + L.w_off(1), t);
  if constexpr (H >= 2) load_layer_weights<U, H, 2>(S, P + L.w_off(2), t);
  if constexpr (H >= 3) load_layer_weights<U, H, 3>(S, P + L.w_off(3), t);
  for (int l = 1; l <= H; ++l)
    for (int e = opaque_tid(); e < U; e += kMlpThreads) S.bias(l)[e] = P[L.b_off(l) + e];
  for (int e = opaque_tid(); e < U; e += kMlpThreads) S.wout()[e] = P[L.wout_off() + e];
  if (opaque_tid() == 0) {
    S.scal()[0] = P[L.bout_off()];
    S.scal()[1] = P[L.mu_off()];
  }
}

// ------------------------------------------------------------------------------------------
// chunk staging: global -> registers (issued one chunk ahead) -> LDS
// ------------------------------------------------------------------------------------------
static_assert(kMlpThreads == kMlpRows * (kMlpDin / 4), "one feature quad of one row per thread");

struct ChunkRegs {
  float x[4];                   // features 4 (t / 64) .. + 3 of row t % 64
  float y;                      // target of row t (threads t < 64)
};

// Target and weight of the row a thread t < 64 holds after staging a chunk.
struct RowTarget {
  float y, w;
};

// Per-thread source of the chunk staging for one date, set up once: thread t loads features
// f0 .. f0 + 3 (f0 = 4 (t / 64)) of row t % 64 and, for t < 64, the target of row t.
struct Feeder {
  const float* x;
  const float* Y;               // uniform base of the targets
  int64_t yo;                   // this thread's row offset in Y and in the weights (t < 64), else -1
  int64_t M;
  int nf, r;
  __device__ __forceinline__ Feeder(const MlpArgs& a, int date) {
    const int t = opaque_tid(), f0 = 4 * (t / kMlpRows);
    r = t % kMlpRows;
    x = a.X + ((int64_t)date * a.n_feat + f0) * a.M + r;
    Y = a.Y;
    yo = (a.Y != nullptr && t < kMlpRows) ? (int64_t)date * a.M + t : -1;
    M = a.M;
    nf = max(0, min(4, a.d_in - f0));
  }
  // rows [r0, r0 + n) (zero beyond the sample and beyond d_in)
  __device__ __forceinline__ ChunkRegs load(int64_t r0, int n) const {
    ChunkRegs c;
    const bool row_ok = r < n;
#pragma unroll
    for (int q = 0; q < 4; ++q) c.x[q] = (row_ok && q < nf) ? x[q * M + r0] : 0.0f;
    c.y = (yo >= 0 && row_ok) ? Y[yo + r0] : 0.0f;
    return c;
  }
  // weight of row r0 + t (1 without weights), from the base in LDS; read when the chunk is
  // staged, not one chunk ahead, so the weights cost no register over the chunk
  __device__ __forceinline__ float weight(const float* const* wbase, int64_t r0, int n) const {
    const float* W = *wbase;
    return (W != nullptr && yo >= 0 && r < n) ? W[yo + r0] : 1.0f;
  }
};

// Standardised inputs (BF16) into A(0); returns the scaled target and the weight of row t held by
// thread t < 64 (and stores them in ybuf / wbuf, which hold them until the next chunk is staged).
template <int U, int H>
__device__ __forceinline__ RowTarget store_chunk(const Smem<U, H>& S, const ChunkRegs& c, float cw, int n,
                                                 __bf16* dst = nullptr) {
  const int t = opaque_tid(), r = t % kMlpRows, f0 = 4 * (t / kMlpRows);
  const f32x4 mean = *(const f32x4*)&S.xmean()[f0];
  const f32x4 inv = *(const f32x4*)&S.xinv()[f0];
  bf16x4 v;
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = (__bf16)(r < n ? (c.x[q] - mean[q]) * inv[q] : 0.0f);
  *(bf16x4*)&(dst ? dst : S.A(0))[lidx(r, f0, S.SW0)] = v;
  float y = 0.0f, w = 0.0f;
  if (t < kMlpRows) {
    y = t < n ? c.y / S.scal()[4] : 0.0f;
    w = t < n ? cw : 0.0f;
    S.ybuf()[t] = y;
    S.wbuf()[t] = w;
  }
  return RowTarget{y, w};
}

// ------------------------------------------------------------------------------------------
// forward
// ------------------------------------------------------------------------------------------
// Packed BF16 pairs: element 0 in the low half of a 32-bit word, element 1 in the high half.
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// (lo, hi) rounded to BF16 (nearest even) in one word: one v_cvt_pk_bf16_f32.  The empty asm
// hands the word on as it is: followed by 16-bit integer arithmetic, the pair would otherwise be
// converted element by element and repacked.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  uint32_t w = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
  asm("" : "+v"(w));
  return w;
}

// ReLU of a rounded pair: a BF16 value is below zero exactly when its sign bit is set, i.e. when
// it is negative as a 16-bit integer, so max(half, 0) over integers is the ReLU (rounding to
// nearest commutes with it; -0 becomes +0).
__device__ __forceinline__ uint32_t relu_pair(uint32_t w) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, w), (s16x2)0));
}

// 1 in each half of w that is not zero (for a ReLU output: that is positive), else 0: one
// v_pk_min_u16 with (1, 1).  Written as an instruction: the compiler rewrites min(h, 1) as a
// comparison per half, which costs a compare, a select and a repack per half.
__device__ __forceinline__ uint32_t nonzero_halves(uint32_t w) {
  uint32_t r;
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(w), "s"(0x00010001u));
  return r;
}

// 0xFFFF in each half of the word where bit k of that half of m is set, else 0 (k < 16; a
// constant once the caller's loops are unrolled).
__device__ __forceinline__ uint32_t expand_bit(uint32_t m, int k) {
  const u16x2 up = __builtin_bit_cast(u16x2, m) << (u16x2)(unsigned short)(15 - k);
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(s16x2, up) >> (s16x2)15);
}

// Hidden layer L: A_L = relu(W_L A_{L-1} + b_L), BF16 into A(L).  Returns the lane's ReLU mask:
// for tile strip s = x BR + y (elements v = 0..3, packed in the words (v0, v1) and (v2, v3)),
// bits 2 s and 2 s + 1 hold "v0 > 0" and "v2 > 0", bits 16 + 2 s and 17 + 2 s "v1 > 0" and
// "v3 > 0" (each word's halves in the matching halves of the mask); the backward pass produces
// dH_L in the same lanes and tile order, so the mask never goes through LDS.
//
// a0 is the input buffer of layer 1; with kKeep false the last layer does not store A_H (only the
// output partials) and leaves its closing barrier to the caller (the scans stage the next
// chunk's inputs in that phase).
template <int U, int H, int L, bool kKeep = true>
__device__ uint32_t forward_layer(const Smem<U, H>& S, const Lanes& ln, const __bf16* a0) {
  using B = Blk<U>;
  constexpr int K = Smem<U, H>::ldk(L), SWl = Smem<U, H>::lds(L);
  constexpr int SW = Smem<U, H>::SW;
  const int wave = wave_id(), lane = lane_id();
  const int ob = wave % B::NOB, rb = wave / B::NOB;
  const int w_rows = L == 1 ? ln.rows_ob0 : ln.rows_ob, in_rows = L == 1 ? ln.rows_rb0 : ln.rows_rb;
  const __bf16* W = S.W(L);
  const __bf16* Ain = L == 1 ? a0 : S.A(L - 1);
  __bf16* Aout = S.A(L);
  // the accumulators start from the bias of their output units (the 16 x 16 tile layout puts
  // units 4 (lane / 16) .. + 3 of the tile in a lane), so the epilogue adds nothing
  const float* b = S.bias(L);
  f32x4 acc[B::BO][B::BR];
#pragma unroll
  for (int x = 0; x < B::BO; ++x) {
    const f32x4 bb = *(const f32x4*)&b[16 * (ob * B::BO + x) + 4 * (lane / 16)];
#pragma unroll
    for (int y = 0; y < B::BR; ++y) acc[x][y] = bb;
  }
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 av[B::BO], bv[B::BR];
#pragma unroll
    for (int x = 0; x < B::BO; ++x) av[x] = *(const bf16x8*)&W[w_rows + 16 * x * SWl + k0];
#pragma unroll
    for (int y = 0; y < B::BR; ++y) bv[y] = *(const bf16x8*)&Ain[in_rows + 16 * y * SWl + k0];
#pragma unroll
    for (int x = 0; x < B::BO; ++x)
#pragma unroll
      for (int y = 0; y < B::BR; ++y) acc[x][y] = mfma16(av[x], bv[y], acc[x][y]);
  }
  uint32_t mask = 0u;
  float pf[B::BR];                      // last layer: this lane's part of f = A_H w_out
#pragma unroll
  for (int y = 0; y < B::BR; ++y) pf[y] = 0.0f;
#pragma unroll
  for (int x = 0; x < B::BO; ++x) {
    const int out0 = 16 * (ob * B::BO + x) + 4 * (lane / 16);
    f32x4 wo = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (L == H) wo = *(const f32x4*)&S.wout()[out0];
#pragma unroll
    for (int y = 0; y < B::BR; ++y) {
      typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
      const uint32_t w0 = relu_pair(pack_bf16(acc[x][y][0], acc[x][y][1]));
      const uint32_t w1 = relu_pair(pack_bf16(acc[x][y][2], acc[x][y][3]));
      const bf16x4 h = __builtin_bit_cast(bf16x4, (u32x2){w0, w1});
      if constexpr (L == H)
#pragma unroll
        for (int v = 0; v < 4; ++v) pf[y] += (float)h[v] * wo[v];
      if constexpr (L < H) mask |= (nonzero_halves(w0) | (nonzero_halves(w1) << 1)) << (2 * (x * B::BR + y));
      if (kKeep || L < H) *(bf16x4*)&Aout[ln.tile_w + 16 * y * SW + 16 * x] = h;
    }
  }
  if constexpr (L == H) {
    // the four lane groups hold the same rows: fold them, then one partial per out block and row
#pragma unroll
    for (int y = 0; y < B::BR; ++y) {
      pf[y] = xor_sum<16>(pf[y]);
      pf[y] = xor_sum<32>(pf[y]);
      if (lane < 16) S.fpart()[ob * kMlpRows + 16 * (rb * B::BR + y) + lane] = pf[y];
    }
  }
  if (kKeep || L < H) __syncthreads();
  return mask;
}

// f of row r (after the forward): the out-block partials in a fixed order, plus b_out.
template <int U, int H>
__device__ __forceinline__ float output_of_row(const Smem<U, H>& S, int r) {
  float f = 0.0f;
#pragma unroll
  for (int q = 0; q < Blk<U>::NOB; ++q) f += S.fpart()[q * kMlpRows + r];
  return f + S.scal()[0];
}

// ReLU masks of the hidden layers below the last (layer l in m[l - 1]).
struct Masks {
  uint32_t m[2];
};

template <int U, int H>
__device__ Masks forward(const Smem<U, H>& S, const Lanes& ln, const __bf16* a0) {
  Masks k{{0u, 0u}};
  k.m[0] = forward_layer<U, H, 1>(S, ln, a0);
  if constexpr (H >= 2) k.m[1] = forward_layer<U, H, 2>(S, ln, a0);
  if constexpr (H >= 3) forward_layer<U, H, 3>(S, ln, a0);
  return k;
}

// Forward of a scan over the sample (loss, prediction): inputs from a0, A_H not kept, the last
// layer's barrier left to the caller.
template <int U, int H>
__device__ void forward_scan(const Smem<U, H>& S, const Lanes& ln, const __bf16* a0) {
  forward_layer<U, H, 1, false>(S, ln, a0);
  if constexpr (H >= 2) forward_layer<U, H, 2, false>(S, ln, a0);
  if constexpr (H >= 3) forward_layer<U, H, 3, false>(S, ln, a0);
}

// Input buffers of a scan: A(0) and the buffer of A_H (unused by a scan), alternating by chunk,
// so the next chunk is staged while the current one is in its last layer.
template <int U, int H>
__device__ __forceinline__ __bf16* scan_buf(const Smem<U, H>& S, int parity) {
  static_assert(Smem<U, H>::SW >= Smem<U, H>::SW0, "input rows fit in a hidden-layer buffer");
  return parity ? S.A(H) : S.A(0);
}

// LDS buffer holding dZ_l in the backward pass.  dZ_H overwrites A_H and dZ_{H-1} overwrites
// A_{H-1} (after a barrier); every lower dZ_l goes to the buffer of A_{l+2}, whose gradient was
// consumed two layers up, so it is written in the same phase as the products that read A_l.
constexpr int dz_buf(int l, int H) { return l >= H - 1 ? l : l + 2; }

// ------------------------------------------------------------------------------------------
// backward
// ------------------------------------------------------------------------------------------
// dW_L += dZ_L^T A_{L-1} over the chunk for the tiles this wave owns, and the bias gradient of
// its out tiles (dZ_L^T times a ones column, in the waves owning in block 0).
template <int U, int H, int L>
__device__ void accumulate_dw(const Smem<U, H>& S, const Lanes& ln, f32x4* accW, const __bf16* a0) {
  using M = DwMap<U, L>;
  const int wave = wave_id(), lane = lane_id();
  const int ib = M::ib_of(wave), ob = M::ob_of(wave);
  if (ob >= M::NOB) return;
  const __bf16* dZ = S.A(dz_buf(L, H));
  const __bf16* Ain = L == 1 ? a0 : S.A(L - 1);
  constexpr int SW = Smem<U, H>::SW, SWin = Smem<U, H>::lds(L);
  const LaneOffsets& oz = ln.o;
  const LaneOffsets& oi = L == 1 ? ln.o0 : ln.o;
  f32x4* acc = accW + dw_base(U, L);
  f32x4 gb[M::BO];
#pragma unroll
  for (int x = 0; x < M::BO; ++x) gb[x] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  bf16x8 ones;
#pragma unroll
  for (int t = 0; t < 8; ++t) ones[t] = (__bf16)1.0f;
#pragma unroll
  for (int k0 = 0; k0 < kMlpRows; k0 += 32) {
    bf16x8 av[M::BO], bv[M::BI];
#pragma unroll
    for (int x = 0; x < M::BO; ++x) av[x] = frag_cols(dZ, oz, SW, k0, 16 * (ob * M::BO + x));
#pragma unroll
    for (int y = 0; y < M::BI; ++y) bv[y] = frag_cols(Ain, oi, SWin, k0, 16 * (ib * M::BI + y));
#pragma unroll
    for (int x = 0; x < M::BO; ++x)
#pragma unroll
      for (int y = 0; y < M::BI; ++y) acc[x * M::BI + y] = mfma16(av[x], bv[y], acc[x * M::BI + y]);
    if (ib == 0) {
#pragma unroll
      for (int x = 0; x < M::BO; ++x) gb[x] = mfma16(av[x], ones, gb[x]);
    }
  }
  if (ib == 0 && lane % 16 == 0) {
#pragma unroll
    for (int x = 0; x < M::BO; ++x)
#pragma unroll
      for (int v = 0; v < 4; ++v) S.gbias(L)[16 * (ob * M::BO + x) + 4 * (lane / 16) + v] += gb[x][v];
  }
}

// dH_{L-1}^T = W_L^T dZ_L^T for the tiles this wave owns (L >= 2).
template <int U, int H, int L>
__device__ void backprop_compute(const Smem<U, H>& S, const Lanes& ln, f32x4 (&dh)[Blk<U>::BO][Blk<U>::BR]) {
  using B = Blk<U>;
  constexpr int SW = Smem<U, H>::SW;
  const __bf16* W = S.W(L);
  const __bf16* dZ = S.A(dz_buf(L, H));
#pragma unroll
  for (int x = 0; x < B::BO; ++x)
#pragma unroll
    for (int y = 0; y < B::BR; ++y) dh[x][y] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k0 = 0; k0 < U; k0 += 32) {
    bf16x8 av[B::BO], bv[B::BR];
#pragma unroll
    for (int x = 0; x < B::BO; ++x) {
      const bf16x4 lo = lds_read_tr(W + ln.bp_lo + k0 * SW + 16 * x);
      const bf16x4 hi = lds_read_tr(W + ln.bp_hi + k0 * SW + 16 * x);
      av[x] = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    }
#pragma unroll
    for (int y = 0; y < B::BR; ++y) bv[y] = *(const bf16x8*)&dZ[ln.rows_rb + 16 * y * SW + k0];
#pragma unroll
    for (int x = 0; x < B::BO; ++x)
#pragma unroll
      for (int y = 0; y < B::BR; ++y) dh[x][y] = mfma16(av[x], bv[y], dh[x][y]);
  }
}

// dZ_{L-1} = dH_{L-1} masked by the ReLU of layer L-1 (the forward pass's mask bits of these
// lanes), into its backward buffer.
template <int U, int H, int L>
__device__ void backprop_store(const Smem<U, H>& S, const Lanes& ln, const f32x4 (&dh)[Blk<U>::BO][Blk<U>::BR],
                               uint32_t mask) {
  using B = Blk<U>;
  constexpr int SW = Smem<U, H>::SW;
  __bf16* dst = S.A(dz_buf(L - 1, H));
#pragma unroll
  for (int x = 0; x < B::BO; ++x)
#pragma unroll
    for (int y = 0; y < B::BR; ++y) {
      typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
      const int k = 2 * (x * B::BR + y);
      const uint32_t z0 = pack_bf16(dh[x][y][0], dh[x][y][1]) & expand_bit(mask, k);
      const uint32_t z1 = pack_bf16(dh[x][y][2], dh[x][y][3]) & expand_bit(mask, k + 1);
      *(bf16x4*)&dst[ln.tile_w + 16 * y * SW + 16 * x] = __builtin_bit_cast(bf16x4, (u32x2){z0, z1});
    }
}

template <int U, int H, int L>
__device__ void layer_backward(const Smem<U, H>& S, const Lanes& ln, const Masks& mk, f32x4* accW,
                               const __bf16* a0) {
  accumulate_dw<U, H, L>(S, ln, accW, a0);
  if constexpr (L > 1) {
    f32x4 dh[Blk<U>::BO][Blk<U>::BR];
    backprop_compute<U, H, L>(S, ln, dh);
    if constexpr (dz_buf(L - 1, H) == L - 1) __syncthreads();   // in place: A(L-1) is read above
    backprop_store<U, H, L>(S, ln, dh, mk.m[L - 2]);
    __syncthreads();
    layer_backward<U, H, L - 1>(S, ln, mk, accW, a0);
  } else {
    __syncthreads();
  }
}

// Output unit of one chunk after its forward pass, and dZ_H = [A_H > 0] dff w_out^T in place.
// The waves derive dff of their own rows from the out-block partials (the same sum in the same
// order as a single wave would, so no phase of one wave precedes the others), keep the
// partial sums of dff^T A_H (output weights) per wave in the reduction area, and leave each row's
// loss and output gradients in dpred / dff for their fixed-order sums after the barrier.  ybuf / wbuf still hold this chunk's rows: the next chunk is staged
// after the barrier.
template <int U, int H>
__device__ void backward_output(const Smem<U, H>& S, int n, float inv_batch, int pos) {
  const int tid = opaque_tid();
  constexpr int UQ = U / 4, RS = kMlpThreads / UQ, RPS = kMlpRows / RS, NG = 64 / UQ;
  const int uq = (int)((unsigned)tid % UQ), rs = (int)((unsigned)tid / UQ);
  const f32x4 wo = *(const f32x4*)&S.wout()[4 * uq];
  const float mu = S.scal()[1];
  // lane uq of a row group (UQ lanes, NG groups per wave) derives row rs RPS + uq % RPS (each row
  // once per RPS lanes), its inputs read without a branch; the group's lanes then take the
  // values of their rows from the group's first RPS lanes
  float dp, dmine;
  {
    const int r = rs * RPS + (int)((unsigned)uq % RPS);
    const float w = S.wbuf()[r], y = S.ybuf()[r];
    const float f = output_of_row<U, H>(S, r);
    const float pred = (pos ? fmaxf(f, 0.0f) : f) + mu;
    dp = r < n ? 2.0f * w * (pred - y) * inv_batch : 0.0f;
    dmine = pos ? (f > 0.0f ? dp : 0.0f) : dp;
    if (uq < RPS) {
      S.dpred()[r] = dp;
      S.dff()[r] = dmine;
    }
  }
  f32x4 g = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < RPS; ++k) {
    const int r = rs * RPS + k;
    // d of row r: lane k of this lane's row group (v_readlane of each group, then a select)
    float d = dmine;
    if constexpr (RPS > 1) {
      d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dmine), k));
#pragma unroll
      for (int gi = 1; gi < NG; ++gi) {
        const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dmine), gi * UQ + k));
        d = lane_id() >= gi * UQ ? v : d;
      }
    }
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    u32x2* p = (u32x2*)&S.A(H)[lidx(r, 4 * uq, Smem<U, H>::SW)];
    const u32x2 aw = *p;
    const bf16x4 a = __builtin_bit_cast(bf16x4, aw);
#pragma unroll
    for (int q = 0; q < 4; ++q) g[q] += d * (float)a[q];
    // z = d w_out where A_H > 0 (A_H holds no negative word), else +0: the halves' nonzero flags
    // (0 or 1) negated are the word masks
    const u16x2 zero = {0, 0};
    const uint32_t m0 = __builtin_bit_cast(uint32_t, zero - __builtin_bit_cast(u16x2, nonzero_halves(aw.x)));
    const uint32_t m1 = __builtin_bit_cast(uint32_t, zero - __builtin_bit_cast(u16x2, nonzero_halves(aw.y)));
    *p = (u32x2){pack_bf16(d * wo[0], d * wo[1]) & m0, pack_bf16(d * wo[2], d * wo[3]) & m1};
  }
  // lanes of a wave that share uq first (the reduction area holds one partial per wave)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if constexpr (UQ <= 8) g[q] += __shfl_xor(g[q], 8);
    if constexpr (UQ <= 16) g[q] = xor_sum<16>(g[q]);
    g[q] = xor_sum<32>(g[q]);
  }
  if (lane_id() < UQ) ((f32x4*)S.red())[wave_id() * UQ + uq] = g;
  __syncthreads();
}

// Gradients of one chunk, accumulated over the batch (after backward_output): the output
// weights' and the output bias / shift's chunk sums, then the hidden layers.
template <int U, int H>
__device__ void backward_layers(const Smem<U, H>& S, const Lanes& ln, const Masks& mk, f32x4* accW,
                                const __bf16* a0) {
  // These sums go to the second wave of each SIMD (waves 4 .. 7), whose weight-gradient blocks
  // carry no bias tiles when a layer has two or more in blocks: the output weights' chunk sums
  // (one unit per thread), and the chunk's sums of the loss gradient (output shift) and of dff
  // (output bias), one row per lane, in waves 6 and 7.
  static_assert(U <= 2 * 64 && kMlpRows == 64, "waves 4 and 5 hold the output units");
  const int u = opaque_tid() - 4 * 64;
  if (u >= 0 && u < U) {
    const float* part = (const float*)S.red();
    float s = S.gwout()[u];
#pragma unroll
    for (int w = 0; w < kMlpWaves; ++w) s += part[w * U + u];
    S.gwout()[u] = s;
  }
  const int wave = wave_id();
  if (wave >= 6) {
    const int r = lane_id();
    const float t = wave_sum(wave == 6 ? S.dpred()[r] : S.dff()[r]);
    if (r == 0) S.scal()[wave == 6 ? 3 : 2] += t;
  }
  layer_backward<U, H, H>(S, ln, mk, accW, a0);
}

// ------------------------------------------------------------------------------------------
// teams: G workgroups training one date together
// ------------------------------------------------------------------------------------------
// Barrier of the G workgroups of a team: a monotonic arrival counter in global memory.  Every
// wave waits for its global stores to complete, the workgroup's arrival (an agent-scope release)
// publishes them; the arriving thread polls the counter without ordering, acquires once when it
// is reached, and after the barrier every wave invalidates its stale cached lines.  All workgroups of a launch are resident
// (cooperative launch), so the wait ends; should it not within the poll limit, the workgroup
// marks itself failed, records the give-up in the launch's status word, stops waiting at later
// barriers (it still arrives) and leaves the fit at the end of the epoch with a NaN loss, so a
// launch always terminates and the host learns of it.
struct Team {
  int32_t* ctr;
  int G, member, arrivals;
  bool failed;
  int32_t* status;
  int spin_limit;
  __device__ void sync() {
    if (G == 1) {
      __syncthreads();
      return;
    }
    // every wave's global stores have completed before the barrier; the one agent-scope release
    // of the arrival then publishes them all (a per-wave device fence would write the L2 back
    // once per wave)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    ++arrivals;
    __shared__ int s_failed;
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const int target = arrivals * G;
      int polls = failed ? spin_limit : 0;
      // relaxed polls (an acquiring poll would invalidate the cache on every iteration), one
      // acquire fence once the count is reached
      while (polls < spin_limit &&
             __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        ++polls;
      }
      s_failed = polls >= spin_limit &&
                 __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target;
      if (s_failed && status) __hip_atomic_fetch_or(status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    failed = failed || s_failed;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
};

// ------------------------------------------------------------------------------------------
// Adam
// ------------------------------------------------------------------------------------------
struct AdamStep {
  float lr, b1, b2, eps, ic1, ic2;      // ic1 = 1 / (1 - b1^t), ic2 = 1 / (1 - b2^t)
  // The fused multiply-adds are written out: left to contraction, which products fuse would
  // depend on the code around each call site, and so would the rounding of the step.
  __device__ float operator()(float p, float g, float* m, float* v) const {
    const float mm = __builtin_fmaf(1.0f - b1, g, b1 * *m);
    const float vv = __builtin_fmaf((1.0f - b2) * g, g, b2 * *v);
    *m = mm;
    *v = vv;
    // hardware square root and reciprocal (about 1 ulp): the step size needs no more
    const float den = __builtin_amdgcn_sqrtf(vv * ic2) + eps;
    return __builtin_fmaf(-(lr * (mm * ic1)), __builtin_amdgcn_rcpf(den), p);
  }
};

template <int U, int H, int L>
__device__ void adam_layer(const Smem<U, H>& S, const MlpLayout& Lay, float* P, float* Mm, float* Vv,
                           const AdamStep& st, f32x4* accW) {
  using M = DwMap<U, L>;
  constexpr int K = L == 1 ? kMlpDin : U, SWl = Smem<U, H>::lds(L);
  const int wave = wave_id(), lane = lane_id();
  const int ib = M::ib_of(wave), ob = M::ob_of(wave);
  if (ob >= M::NOB) return;
  f32x4* acc = accW + dw_base(U, L);
#pragma unroll
  for (int x = 0; x < M::BO; ++x)
#pragma unroll
    for (int y = 0; y < M::BI; ++y) {
      const int s = x * M::BI + y, ot = ob * M::BO + x, it = ib * M::BI + y;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int out = 16 * ot + 4 * (lane / 16) + v, in = 16 * it + lane % 16;
        const int idx = Lay.w_off(L) + out * K + in;
        const float p = st(P[idx], acc[s][v], &Mm[idx], &Vv[idx]);
        P[idx] = p;
        S.W(L)[lidx(out, in, SWl)] = (__bf16)p;
      }
      acc[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      asm volatile("" ::: "memory");    // one tile's moments in flight at a time
    }
}

template <int U, int H>
__device__ void adam_update(const Smem<U, H>& S, const MlpLayout& L, float* P, float* Mm, float* Vv,
                            const AdamStep& st, f32x4* accW) {
  adam_layer<U, H, 1>(S, L, P, Mm, Vv, st, accW);
  if constexpr (H >= 2) adam_layer<U, H, 2>(S, L, P, Mm, Vv, st, accW);
  if constexpr (H >= 3) adam_layer<U, H, 3>(S, L, P, Mm, Vv, st, accW);
  static_assert(H <= 3, "up to three hidden layers");
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

// One Adam step of a team: every workgroup publishes its batch gradient in parameter order,
// each member sums the G gradients of its slice of the parameters (fixed order) and updates that
// slice, and every workgroup reloads the new parameters.
template <int U, int H, int L>
__device__ void publish_dw(const MlpLayout& Lay, float* part, f32x4* accW) {
  using M = DwMap<U, L>;
  constexpr int K = L == 1 ? kMlpDin : U;
  const int wave = wave_id(), lane = lane_id();
  const int ib = M::ib_of(wave), ob = M::ob_of(wave);
  if (ob >= M::NOB) return;
  f32x4* acc = accW + dw_base(U, L);
#pragma unroll
  for (int x = 0; x < M::BO; ++x)
#pragma unroll
    for (int y = 0; y < M::BI; ++y) {
      const int s = x * M::BI + y, ot = ob * M::BO + x, it = ib * M::BI + y;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        part[Lay.w_off(L) + (16 * ot + 4 * (lane / 16) + v) * K + 16 * it + lane % 16] = acc[s][v];
      acc[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
}

template <int U, int H>
__device__ void team_step(const Smem<U, H>& S, const MlpArgs& a, Team& tm, int team, const MlpLayout& L,
                          float* P, float* Mm, float* Vv, const AdamStep& st, f32x4* accW) {
  const int NP = L.n_params();
  float* part = a.partial + ((int64_t)team * tm.G + tm.member) * NP;
  publish_dw<U, H, 1>(L, part, accW);
  if constexpr (H >= 2) publish_dw<U, H, 2>(L, part, accW);
  if constexpr (H >= 3) publish_dw<U, H, 3>(L, part, accW);
  for (int l = 1; l <= H; ++l)
    for (int u = opaque_tid(); u < U; u += kMlpThreads) {
      part[L.b_off(l) + u] = S.gbias(l)[u];
      S.gbias(l)[u] = 0.0f;
    }
  for (int u = opaque_tid(); u < U; u += kMlpThreads) {
    part[L.wout_off() + u] = S.gwout()[u];
    S.gwout()[u] = 0.0f;
  }
  if (opaque_tid() == 0) {
    part[L.bout_off()] = S.scal()[2];
    part[L.mu_off()] = S.scal()[3];
    S.scal()[2] = 0.0f;
    S.scal()[3] = 0.0f;
  }
  tm.sync();
  // this member's slice of the parameters, kAdamBatch elements per thread at a time (restrict
  // views: the stores of a batch do not alias the next batch's loads)
  const float* __restrict__ part0 = a.partial + (int64_t)team * tm.G * NP;
  float* __restrict__ Pr = P;
  float* __restrict__ Mr = Mm;
  float* __restrict__ Vr = Vv;
  const int lo = (int)((int64_t)NP * tm.member / tm.G), hi = (int)((int64_t)NP * (tm.member + 1) / tm.G);
  constexpr int kAdamBatch = 8;
  for (int p0 = lo + opaque_tid(); p0 < hi; p0 += kMlpThreads * kAdamBatch) {
    // a batch element past the slice reads the slice's last parameter (in bounds, never stored),
    // so no load is predicated; the members' gradients are summed first (in member order), then
    // the batch's Adam state is loaded
    float g[kAdamBatch], pv[kAdamBatch], mv[kAdamBatch], vv[kAdamBatch];
    int qc[kAdamBatch];
#pragma unroll
    for (int u = 0; u < kAdamBatch; ++u) {
      qc[u] = min(p0 + u * kMlpThreads, hi - 1);
      g[u] = 0.0f;
    }
    for (int j = 0; j < tm.G; ++j) {
      const float* __restrict__ pj = part0 + (int64_t)j * NP;
      float t[kAdamBatch];
#pragma unroll
      for (int u = 0; u < kAdamBatch; ++u) t[u] = pj[qc[u]];
      // all of a member's loads are issued before the first add (left alone, the register
      // allocator gives them one register and waits for each load in turn)
      static_assert(kAdamBatch == 8, "one operand per batch element");
      asm volatile("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]),
                   "+v"(t[7]));
#pragma unroll
      for (int u = 0; u < kAdamBatch; ++u) g[u] += t[u];
    }
#pragma unroll
    for (int u = 0; u < kAdamBatch; ++u) {
      pv[u] = Pr[qc[u]];
      mv[u] = Mr[qc[u]];
      vv[u] = Vr[qc[u]];
    }
#pragma unroll
    for (int u = 0; u < kAdamBatch; ++u) {
      const int q = p0 + u * kMlpThreads;
      if (q < hi) {
        const float np = st(pv[u], g[u], &mv[u], &vv[u]);
        Pr[q] = np;
        Mr[q] = mv[u];
        Vr[q] = vv[u];
      }
    }
  }
  tm.sync();
  load_weights<U, H>(S, P, L);
  __syncthreads();
}

// ------------------------------------------------------------------------------------------
// full-sample passes: loss and refit
// ------------------------------------------------------------------------------------------
// Full-sample loss with the output ReLU (pos = 1).
template <int U, int H>
__device__ float full_loss(const Smem<U, H>& S, const Lanes& ln, const Feeder& feed, const MlpArgs& a, Team& tm,
                           int team) {
  constexpr int R = kMlpRows;
  const int64_t stride = (int64_t)R * tm.G;
  double e = 0.0;
  const int64_t first = (int64_t)R * tm.member;
  auto rows = [&](int64_t r0) { return (int)max((int64_t)0, min((int64_t)R, a.M - r0)); };
  ChunkRegs c = feed.load(first, rows(first));
  RowTarget y = store_chunk<U, H>(S, c, feed.weight(S.wbase(), first, rows(first)), rows(first), scan_buf(S, 0));
  c = feed.load(first + stride, rows(first + stride));
  __syncthreads();
  int parity = 0;
  for (int64_t r0 = first; r0 < a.M; r0 += stride) {
    const int n = rows(r0);
    RowTarget y_next{0.0f, 0.0f};
    forward_scan<U, H>(S, ln, scan_buf(S, parity));
    // the next chunk goes into the other buffer in this chunk's last-layer phase
    if (r0 + stride < a.M) {
      y_next = store_chunk<U, H>(S, c, feed.weight(S.wbase(), r0 + stride, rows(r0 + stride)), rows(r0 + stride),
                                 scan_buf(S, parity ^ 1));
      c = feed.load(r0 + 2 * stride, rows(r0 + 2 * stride));
    }
    __syncthreads();
    const int t = opaque_tid();
    if (t < n) {
      const float d = fmaxf(output_of_row<U, H>(S, t), 0.0f) + S.scal()[1] - y.y;
      e += (double)y.w * (double)d * (double)d;
    }
    // with one hidden layer the next chunk's only layer writes the output partials at once: wait
    // until they have been read (deeper networks wait at their first layer's barrier)
    if constexpr (H == 1) __syncthreads();
    y = y_next;
    parity ^= 1;
  }
  __syncthreads();
  double* red = (double*)S.red();
  red[opaque_tid()] = e;
  __syncthreads();
  for (int w = kMlpThreads / 2; w > 0; w >>= 1) {
    if (opaque_tid() < w) red[opaque_tid()] += red[opaque_tid() + w];
    __syncthreads();
  }
  double sum = red[0];
  __syncthreads();
  if (tm.G > 1) {
    double* lp = a.loss_part + (int64_t)team * tm.G;
    if (opaque_tid() == 0) lp[tm.member] = sum;
    tm.sync();
    sum = 0.0;
    for (int j = 0; j < tm.G; ++j) sum += lp[j];
  }
  return (float)(sum / (double)a.M);
}

// Least-squares refit of (w_out, b_out) on the frozen hidden features, mu fixed.
template <int U, int H>
__device__ void refit(const Smem<U, H>& S, const Lanes& ln, const Feeder& feed, const MlpArgs& a,
                      const MlpLayout& L, float* P, Team& tm, int team) {
  double* G = a.gram + ((int64_t)team * tm.G + tm.member) * (U + 1) * (U + 2);
  constexpr int NT = U / 16, NG = NT * NT, GS = (NG + kMlpWaves - 1) / kMlpWaves, N = U + 1;
  constexpr int R = kMlpRows;
  const int tid = opaque_tid(), wave = wave_id(), lane = lane_id();
  // per-chunk Gram tiles come from the matrix cores in FP32 (exact products of BF16 values,
  // 64-term sums); the sum over chunks is carried in FP64
  double accG[GS][4];
#pragma unroll
  for (int s = 0; s < GS; ++s)
#pragma unroll
    for (int v = 0; v < 4; ++v) accG[s][v] = 0.0;
  // thread t, column u = t % U, row group t / U of the chunk: sum w h_u, sum w h_u (y - mu); the
  // threads of column 0 also sum w (y - mu) and w.  Groups are combined in a fixed order below.
  constexpr int NGRP = kMlpThreads / U;
  static_assert(NGRP * U == kMlpThreads && kMlpThreads * 8 <= Smem<U, H>::red_bytes, "column groups");
  double hs = 0.0, hy = 0.0, ys = 0.0, sw = 0.0;
  const float mu = S.scal()[1];
  const int64_t stride = (int64_t)R * tm.G, first = (int64_t)R * tm.member;
  ChunkRegs c = feed.load(first, (int)max((int64_t)0, min((int64_t)R, a.M - first)));
  for (int64_t r0 = first; r0 < a.M; r0 += stride) {
    const int n = (int)min((int64_t)R, a.M - r0);
    store_chunk<U, H>(S, c, feed.weight(S.wbase(), r0, n), n);
    if (r0 + stride < a.M) c = feed.load(r0 + stride, (int)min((int64_t)R, a.M - r0 - stride));
    __syncthreads();
    forward<U, H>(S, ln, S.A(0));
    __bf16* Hh = S.A(H);
    const LaneOffsets& oh = ln.o;
    if (n < R) {                              // rows beyond the sample take no part
      for (int e = tid; e < (R - n) * U; e += kMlpThreads) Hh[lidx(n + e / U, e % U, Smem<U, H>::SW)] = (__bf16)0.0f;
      __syncthreads();
    }
    const bool weighted = *S.wbase() != nullptr;
    if (weighted) {                           // weighted rows: H <- diag(sqrt w) H for the Gram tiles
      for (int e = tid; e < n * U; e += kMlpThreads) {
        const int r = e / U, u = e % U;
        __bf16& h = Hh[lidx(r, u, Smem<U, H>::SW)];
        h = (__bf16)((float)h * sqrtf(S.wbuf()[r]));
      }
      __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < GS; ++s) {
      const int g = kMlpWaves * s + wave;
      if (g >= NG) continue;
      const int ot = g / NT, it = g % NT;
      f32x4 part = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int k0 = 0; k0 < R; k0 += 32)
        part = mfma16(frag_cols(Hh, oh, Smem<U, H>::SW, k0, 16 * ot), frag_cols(Hh, oh, Smem<U, H>::SW, k0, 16 * it), part);
#pragma unroll
      for (int v = 0; v < 4; ++v) accG[s][v] += (double)part[v];
    }
    {
      const int u = tid % U, grp = tid / U;
      // with weights the stored row is sqrt(w) h: one more sqrt(w) gives w h
      auto column_row = [&](int r) {
        const double h = (double)(float)Hh[lidx(r, u, Smem<U, H>::SW)] * (weighted ? sqrt((double)S.wbuf()[r]) : 1.0);
        hs += h;
        hy += h * (double)(S.ybuf()[r] - mu);
      };
      if (n == R && !weighted) {
        // a full chunk: the thread's rows unrolled, so that their LDS reads are issued together
        // (the sums keep the row order)
#pragma unroll
        for (int r = grp; r < R; r += NGRP) column_row(r);
      } else {
#pragma unroll 1
        for (int r = grp; r < n; r += NGRP) column_row(r);
      }
      if (u == 0)
        for (int r = grp; r < n; r += NGRP) {
          const double w = S.wbuf()[r];
          ys += w * (double)(S.ybuf()[r] - mu);
          sw += w;
        }
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
    for (int v = 0; v < 4; ++v) G[(16 * ot + 4 * (lane / 16) + v) * N + 16 * it + lane % 16] = accG[s][v];
  }
  double* rhs = G + N * N;
  {
    double* red = (double*)S.red();         // one double per thread: the two sums in turn
    const int u = tid % U, grp = tid / U;
    double a = 0.0, b = 0.0;
    red[tid] = hs;
    __syncthreads();
    if (tid < U)
      for (int g = 0; g < NGRP; ++g) a += red[g * U + tid];
    __syncthreads();
    red[tid] = hy;
    __syncthreads();
    if (tid < U) {
      for (int g = 0; g < NGRP; ++g) b += red[g * U + tid];
      G[tid * N + U] = a;
      G[U * N + tid] = a;
      rhs[tid] = b;
    }
    __syncthreads();
    if (u == 0) {
      red[2 * grp] = ys;
      red[2 * grp + 1] = sw;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int g = 0; g < NGRP; ++g) {
        a += red[2 * g];
        b += red[2 * g + 1];
      }
      G[U * N + U] = b;
      rhs[U] = a;
    }
  }
  tm.sync();
  if (tm.member != 0) {                 // the first workgroup solves; the others wait for w_out
    tm.sync();
    for (int u = opaque_tid(); u < U; u += kMlpThreads) S.wout()[u] = P[L.wout_off() + u];
    if (opaque_tid() == 0) S.scal()[0] = P[L.bout_off()];
    __syncthreads();
    return;
  }
  for (int j = 1; j < tm.G; ++j) {      // sum of the partial normal equations, fixed order
    const double* Gj = G + (int64_t)j * (U + 1) * (U + 2);
    for (int e = opaque_tid(); e < N * N + N; e += kMlpThreads) G[e] += Gj[e];
  }
  __threadfence_block();
  __syncthreads();
  // Algorithm 1's refit is the plain least-squares argmin.  Its fitted values are unique; where
  // [H 1] is rank deficient (a dead ReLU unit is an all-zero column, two units may coincide) the
  // weights are not, and a column whose diagonal is zero, or whose Cholesky pivot falls to
  // kRefitGuard times its diagonal (dependent on the columns before it to working precision),
  // is dropped with weight 0: the fitted values are those of the full problem.  A dropped
  // column is marked by a zero on the factor's diagonal; its entries below are zeroed so it
  // takes no part in the trailing updates or the triangular solves.  The original diagonal of
  // column k >= 1 is kept in the unused upper triangle at (k - 1, k).
  for (int k = 1 + opaque_tid(); k < N; k += kMlpThreads) G[(k - 1) * N + k] = G[k * N + k];
  __threadfence_block();
  __syncthreads();
  // Cholesky (lower, in place), all threads on the trailing update
  for (int k = 0; k < N; ++k) {
    if (opaque_tid() == 0) {
      const double d = k == 0 ? G[0] : G[(k - 1) * N + k];
      const double p = G[k * N + k];
      G[k * N + k] = (d > 0.0 && p > kRefitGuard * d) ? sqrt(p) : 0.0;
    }
    __threadfence_block();
    __syncthreads();
    const double dkk = G[k * N + k];
    for (int i = k + 1 + opaque_tid(); i < N; i += kMlpThreads) G[i * N + k] = dkk > 0.0 ? G[i * N + k] / dkk : 0.0;
    __threadfence_block();
    __syncthreads();
    if (dkk > 0.0) {
      const int m = N - k - 1;
      for (int e = opaque_tid(); e < m * m; e += kMlpThreads) {
        const int i = k + 1 + e / m, j = k + 1 + e % m;
        if (j <= i) G[i * N + j] -= G[i * N + k] * G[j * N + k];
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  if (opaque_tid() == 0) {
#pragma unroll 1
    for (int i = 0; i < N; ++i) {          // L y = rhs (dropped columns: 0)
      double s = rhs[i];
#pragma unroll 1
      for (int j = 0; j < i; ++j) s -= G[i * N + j] * rhs[j];
      rhs[i] = G[i * N + i] > 0.0 ? s / G[i * N + i] : 0.0;
    }
#pragma unroll 1
    for (int i = N - 1; i >= 0; --i) {     // L^T x = y
      double s = rhs[i];
#pragma unroll 1
      for (int j = i + 1; j < N; ++j) s -= G[j * N + i] * rhs[j];
      rhs[i] = G[i * N + i] > 0.0 ? s / G[i * N + i] : 0.0;
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
  if (tm.G > 1) tm.sync();
}

// ------------------------------------------------------------------------------------------
// BaseAlg for one date
// ------------------------------------------------------------------------------------------
// ------------------------------------------------------------------------------------------
// loss helpers: the full-sample loss of each epoch off the teams' critical path
// ------------------------------------------------------------------------------------------
// The loss only decides which epoch's parameters are kept (Algorithm 1's best tracking), never
// the training itself, so a team publishes a snapshot of its parameters after every epoch and
// goes on; workgroups without a team (and teams that are done) compute the losses, and the
// helper that computes a date's last loss keeps the first epoch of least loss.
constexpr int kReadySkip = -2;    // untrained date: loss 0, no selection
constexpr int kReadyFail = -1;    // failed team: loss NaN

__device__ __forceinline__ void mark_epochs(const MlpArgs& a, int job, int e0, int value) {
  for (int e = e0; e < a.epochs; ++e)
    __hip_atomic_exchange(a.ready + (int64_t)job * a.epochs + e, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// This member's slice of the parameters into the snapshot of `epoch` (1-based), then its arrival.
__device__ void publish_snapshot(const MlpArgs& a, int job, int epoch, const float* P, int NP, const Team& tm) {
  float* __restrict__ dst = a.snaps + ((int64_t)job * a.epochs + epoch - 1) * NP;
  const float* __restrict__ src = P;
  const int lo = (int)((int64_t)NP * tm.member / tm.G), hi = (int)((int64_t)NP * (tm.member + 1) / tm.G);
  constexpr int kBatch = 8;
  for (int p0 = lo + opaque_tid(); p0 < hi; p0 += kMlpThreads * kBatch) {
    float v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) v[u] = p0 + u * kMlpThreads < hi ? src[p0 + u * kMlpThreads] : 0.0f;
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (p0 + u * kMlpThreads < hi) dst[p0 + u * kMlpThreads] = v[u];
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_fetch_add(a.ready + (int64_t)job * a.epochs + epoch - 1, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int U, int H>
__device__ void loss_helper(const Smem<U, H>& S, const MlpArgs& a) {
  const MlpLayout L{U, H};
  const int NP = L.n_params();
  const int total = a.n_reg * a.epochs;
  // the helper's shared words live in the dpred area (unused by the loss pass)
  int& s_q = ((int*)S.dpred())[0];
  int& s_state = ((int*)S.dpred())[1];
  int& s_best = ((int*)S.dpred())[2];
  const Lanes ln = make_lanes<U, H>();
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_q = __hip_atomic_fetch_add(a.lqueue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int q = s_q;
    if (q >= total) break;
    const int e = q / a.n_reg, job = q % a.n_reg;           // earlier epochs first
    if (threadIdx.x == 0) {
      const int32_t* rdy = a.ready + (int64_t)job * a.epochs + e;
      int polls = 0, v = __hip_atomic_load(rdy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (v >= 0 && v < a.G && polls < a.spin_limit) {
        __builtin_amdgcn_s_sleep(2);
        ++polls;
        v = __hip_atomic_load(rdy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_state = v >= a.G ? 1 : v == kReadySkip ? 2 : 0;
      // a snapshot that never came: the wait gave up (a failed team has recorded its own)
      if (v >= 0 && v < a.G && a.status)
        __hip_atomic_fetch_or(a.status, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int state = s_state;
    float loss = state == 2 ? 0.0f : NAN;
    if (state == 1) {
      const float* rec = a.model + (int64_t)job * L.record();
      for (int f = opaque_tid(); f < kMlpDin; f += kMlpThreads) {
        S.xmean()[f] = rec[L.xmean_off() + f];
        S.xinv()[f] = rec[L.xinv_off() + f];
      }
      if (opaque_tid() == 0) {
        S.scal()[4] = rec[L.yscale_off()];
        *S.wbase() = a.Wt;
      }
      load_weights<U, H>(S, a.snaps + ((int64_t)job * a.epochs + e) * NP, L);
      __syncthreads();
      const Feeder feed(a, a.dates[job]);
      Team solo{nullptr, 1, 0, 0, false, nullptr, 0};
      loss = full_loss<U, H>(S, ln, feed, a, solo, 0);
    }
    if (threadIdx.x == 0) {
      a.losses[(int64_t)job * a.epochs + e] = loss;
      if (a.loss_hist) a.loss_hist[(int64_t)job * a.epochs + e] = loss;
      const int old = __hip_atomic_fetch_add(a.done + job, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      int best = -1;
      if (old == a.epochs - 1) {                             // the date's last loss: keep the best epoch
        float bl = INFINITY;
        for (int k = 0; k < a.epochs; ++k) {
          const float lk = a.losses[(int64_t)job * a.epochs + k];
          if (lk < bl) {
            bl = lk;
            best = k;
          }
        }
        if (a.model[(int64_t)job * L.record() + L.trained_off()] == 0.0f) best = -1;
      }
      s_best = best;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int best = s_best;
    if (best >= 0) {
      const float* src = a.snaps + ((int64_t)job * a.epochs + best) * NP;
      float* rec = a.model + (int64_t)job * L.record();
      for (int p = opaque_tid(); p < NP; p += kMlpThreads) rec[p] = src[p];
    }
  }
}

template <int U, int H>
__device__ void train_one(const Smem<U, H>& S, const MlpArgs& a, int job, Team& tm, int team) {
  constexpr int R = kMlpRows;
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
  if (opaque_tid() == 0) {
    S.scal()[4] = rec[L.yscale_off()];
    *S.wbase() = a.Wt;
  }
  const bool trained = rec[L.trained_off()] != 0.0f;
  // initial parameters (written by the first workgroup of the team)
  for (int l = 1; l <= H + 1 && tm.member == 0; ++l) {
    const int fan_in = l == 1 ? a.d_in : U;
    const int rows = l <= H ? U : 1;
    const int stride = l == 1 ? kMlpDin : U;
    const int off = l <= H ? L.w_off(l) : L.wout_off();
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
      P[off + e] = w;
    }
    if (l <= H)
      for (int e = opaque_tid(); e < U; e += kMlpThreads) P[L.b_off(l) + e] = a.use_init ? rec[L.b_off(l) + e] : 0.0f;
  }
  if (tm.member == 0) {
    if (opaque_tid() == 0) {
      P[L.bout_off()] = a.use_init ? rec[L.bout_off()] : 0.0f;
      P[L.mu_off()] = a.use_init ? rec[L.mu_off()] : 0.0f;
    }
    for (int e = opaque_tid(); e < NP; e += kMlpThreads) {
      Mm[e] = 0.0f;
      Vv[e] = 0.0f;
    }
  }
  __threadfence_block();
  tm.sync();
  if (!trained) {
    if (tm.member == 0) {
      for (int e = opaque_tid(); e < NP; e += kMlpThreads) rec[e] = P[e];
      if (a.loss_hist)
        for (int e = opaque_tid(); e < a.epochs; e += kMlpThreads) a.loss_hist[(int64_t)job * a.epochs + e] = 0.0f;
    }
    tm.sync();
    if (a.snaps && tm.member == 0 && threadIdx.x == 0) mark_epochs(a, job, 0, kReadySkip);
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

  const Lanes ln = make_lanes<U, H>();
  const Feeder feed(a, date);
  float best = INFINITY;
  int pos = 0;
  float p1 = 1.0f, p2 = 1.0f;
  const int64_t cstride = (int64_t)R * tm.G;   // this workgroup's chunks of a batch
  for (int epoch = 1; epoch <= a.epochs; ++epoch) {
    for (int64_t b0 = 0; b0 < a.M; b0 += a.batch) {
      const int64_t b1 = min(b0 + (int64_t)a.batch, a.M);
      const float inv_batch = 1.0f / (float)(b1 - b0);
      f32x4 accW[dw_slots(U, H)];
#pragma unroll
      for (int s = 0; s < dw_slots(U, H); ++s) accW[s] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      const int64_t first = b0 + (int64_t)R * tm.member;
      auto rows = [&](int64_t r) { return (int)max((int64_t)0, min((int64_t)R, b1 - r)); };
      // the batch's first chunk is staged here, every later one into the other input buffer while
      // its predecessor is back-propagated (the last barrier of that pass publishes it)
      ChunkRegs c = feed.load(first, rows(first));
      if (first < b1) store_chunk<U, H>(S, c, feed.weight(S.wbase(), first, rows(first)), rows(first), S.in_buf(0));
      if (first + cstride < b1) c = feed.load(first + cstride, rows(first + cstride));
      __syncthreads();
      int parity = 0;
      for (int64_t r0 = first; r0 < b1; r0 += cstride) {
        const int n = rows(r0);
        const __bf16* a0 = S.in_buf(parity);
        const Masks mk = forward<U, H>(S, ln, a0);
        backward_output<U, H>(S, n, inv_batch, pos);
        if (r0 + cstride < b1) {
          const int nn = rows(r0 + cstride);
          store_chunk<U, H>(S, c, feed.weight(S.wbase(), r0 + cstride, nn), nn, S.in_buf(parity ^ 1));
          if (r0 + 2 * cstride < b1) c = feed.load(r0 + 2 * cstride, rows(r0 + 2 * cstride));
        }
        backward_layers<U, H>(S, ln, mk, accW, a0);
        parity ^= 1;
      }
      p1 *= a.beta1;
      p2 *= a.beta2;
      const AdamStep st{a.lr, a.beta1, a.beta2, a.eps, 1.0f / (1.0f - p1), 1.0f / (1.0f - p2)};
      if (tm.G == 1)
        adam_update<U, H>(S, L, P, Mm, Vv, st, accW);
      else
        team_step<U, H>(S, a, tm, team, L, P, Mm, Vv, st, accW);
    }
    if (epoch == a.epochs / 2) {
      refit<U, H>(S, ln, feed, a, L, P, tm, team);
      pos = 1;
    }
    if (a.snaps) {                       // the loss helpers take the loss and the best tracking
      if (tm.failed) {
        if (threadIdx.x == 0) mark_epochs(a, job, epoch - 1, kReadyFail);
        return;
      }
      publish_snapshot(a, job, epoch, P, NP, tm);
      continue;
    }
    float loss = full_loss<U, H>(S, ln, feed, a, tm, team);
    if (tm.failed) loss = NAN;
    if (a.loss_hist && (tm.member == 0 || tm.failed) && opaque_tid() == 0)
      a.loss_hist[(int64_t)job * a.epochs + epoch - 1] = loss;
    if (tm.failed) return;
    if (loss < best) {
      best = loss;
      __threadfence_block();
      __syncthreads();
      if (tm.member == 0)
        for (int e = opaque_tid(); e < NP; e += kMlpThreads) rec[e] = P[e];
    }
    __syncthreads();
  }
}

// Workgroup b belongs to team (b % 8) + 8 ((b / 8) / G) as member (b / 8) % G: consecutive
// workgroups go to different XCDs, so the members of a team share one XCD (and its L2).  Teams
// take the dates team, team + n_teams, ...
template <int U, int H>
__global__ __launch_bounds__(kMlpThreads) void mlp_train_kernel(const MlpArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  Smem<U, H> S{(__bf16*)smem_raw};
  const int b = blockIdx.x;
  const int tgrid = 8 * a.G * ((a.n_teams + 7) / 8);
  const int team = b % 8 + 8 * ((b / 8) / a.G), member = (b / 8) % a.G;
  if (b < tgrid && team < a.n_teams) {
    Team tm{a.team_ctr + team, a.G, member, 0, false, a.status, a.spin_limit};
    for (int job = team; job < a.n_reg && !tm.failed; job += a.n_teams) train_one<U, H>(S, a, job, tm, team);
  }
  if (a.snaps) loss_helper<U, H>(S, a);
}

// Prediction with the best parameters: out[job][k] = ((f)^+ + mu) * y_scale (0 if untrained).
template <int U, int H>
__global__ __launch_bounds__(kMlpThreads) void mlp_predict_kernel(const MlpArgs a, float* out) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  Smem<U, H> S{(__bf16*)smem_raw};
  constexpr int R = kMlpRows;
  const MlpLayout L{U, H};
  const int job = blockIdx.y;
  const int date = a.dates[job];
  const float* rec = a.model + (int64_t)job * L.record();
  const int64_t rows_per_block = 64 * R;
  const int64_t k0 = (int64_t)blockIdx.x * rows_per_block;
  if (k0 >= a.M) return;
  const int64_t k1 = min(k0 + rows_per_block, a.M);
  const bool trained = rec[L.trained_off()] != 0.0f;
  if (!trained) {
    for (int64_t k = k0 + opaque_tid(); k < k1; k += kMlpThreads) out[(int64_t)job * a.M + k] = 0.0f;
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
  const Lanes ln = make_lanes<U, H>();
  const Feeder feed(a, date);
  auto rows = [&](int64_t r0) { return (int)max((int64_t)0, min((int64_t)R, k1 - r0)); };
  ChunkRegs c = feed.load(k0, rows(k0));
  store_chunk<U, H>(S, c, 1.0f, rows(k0), scan_buf(S, 0));
  c = feed.load(k0 + R, rows(k0 + R));
  __syncthreads();
  int parity = 0;
  for (int64_t r0 = k0; r0 < k1; r0 += R) {
    const int n = rows(r0);
    forward_scan<U, H>(S, ln, scan_buf(S, parity));
    if (r0 + R < k1) {
      store_chunk<U, H>(S, c, 1.0f, rows(r0 + R), scan_buf(S, parity ^ 1));
      c = feed.load(r0 + 2 * R, rows(r0 + 2 * R));
    }
    __syncthreads();
    const int t = opaque_tid();
    if (t < n) out[(int64_t)job * a.M + r0 + t] = (fmaxf(output_of_row<U, H>(S, t), 0.0f) + S.scal()[1]) * ysc;
    if constexpr (H == 1) __syncthreads();   // the output partials are read before the next chunk writes them
    parity ^= 1;
  }
}

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

__global__ void zero_i32(int32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

int mlp_max_teams(int U, int H, int G) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
#define X(u, h)                                                                                  \
  if (U == u && H == h) {                                                                        \
    hipFuncSetAttribute((const void*)mlp_train_kernel<u, h>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                        Smem<u, h>::bytes);                                                      \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mlp_train_kernel<u, h>, kMlpThreads, \
                                                     Smem<u, h>::bytes) != hipSuccess)           \
      return 0;                                                                                  \
  }
  HSIM_MLP_SHAPES(X)
#undef X
  if (G < 1) return 0;
  return 8 * ((ncu * per_cu) / (8 * G));   // whole groups of 8 teams (one per XCD)
}

hipError_t launch_mlp_train(const MlpArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(zero_i32, dim3(1), dim3(256), 0, s, a.team_ctr, a.n_teams);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.snaps) {
    hipLaunchKernelGGL(zero_i32, dim3(1), dim3(256), 0, s, a.ready, a.n_reg * a.epochs);
    hipLaunchKernelGGL(zero_i32, dim3(1), dim3(256), 0, s, a.done, a.n_reg);
    hipLaunchKernelGGL(zero_i32, dim3(1), dim3(256), 0, s, a.lqueue, 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const unsigned tgrid = 8u * (unsigned)a.G * (unsigned)((a.n_teams + 7) / 8);
  const unsigned grid = a.snaps ? (unsigned)a.n_blocks : tgrid;
  void* args[] = {(void*)&a};
#define X(u, h)                                                                                  \
  if (a.U == u && a.H == h) {                                                                    \
    const int bytes = Smem<u, h>::bytes;                                                         \
    hipFuncSetAttribute((const void*)mlp_train_kernel<u, h>,                                     \
                        hipFuncAttributeMaxDynamicSharedMemorySize, bytes);                      \
    return hipLaunchCooperativeKernel((const void*)mlp_train_kernel<u, h>, dim3(grid), dim3(kMlpThreads), \
                                      args, bytes, s);                                           \
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

}  // namespace tile<HSIM_MLP_TILE>
}  // namespace hsim
