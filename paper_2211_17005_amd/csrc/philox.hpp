// Counter-based random numbers for the hierarchical simulation (device side).
//
// Philox4x32-10 as defined by Salmon, Moraes, Dror & Shaw (SC'11, Section 3): two
// 32x32->64 products per round, XOR mixing and a Weyl key schedule, ten rounds.
// Counters are built from global indices only:
//   outer normals  (k, s, f >> 2, 0)   path k, global Euler sub-step s, normal index f
//   inner defaults (k, l >> 2, c, 1)   draw l of counterparty c
//   network init   (layer, idx >> 2, date, 2)
// Uniforms use 23 bits on a half-offset grid, u = (2 floor(x / 2^9) + 1) 2^-24, which
// is exact in FP32 and FP64 so both precisions see identical uniforms.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hsim {

struct u32x4 {
  uint32_t x, y, z, w;
};

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

enum : uint32_t { kTagOuter = 0, kTagInner = 1, kTagInit = 2, kTagBranch = 3 };

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return {c0, c1, c2, c3};
}

// 23-bit grid index of a word; the uniform is (2m + 1) 2^-24.
__device__ __forceinline__ uint32_t grid23(uint32_t x) { return x >> 9; }

template <typename Real>
__device__ __forceinline__ Real uniform_of(uint32_t x) {
  return (Real)(2u * grid23(x) + 1u) * (Real)5.9604644775390625e-8;  // 2^-24
}

// Box & Muller (1958): (R cos 2 pi u_b, R sin 2 pi u_b), R = sqrt(-2 log u_a).
// FP32: the gfx950 transcendental instructions, which need no range reduction here (u_a in
// [2^-24, 1), u_b in (0, 1)): v_log_f32 is log2, so -2 log u = -2 ln 2 log2 u, and v_sin_f32 /
// v_cos_f32 take their argument in revolutions, so sin 2 pi u_b is one instruction.  The normals
// stay within 3e-7 of the FP64 ones (the library functions spend most of their instructions on
// arguments that cannot occur here).
__device__ __forceinline__ void box_muller(float ua, float ub, float& z0, float& z1) {
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
  z0 = rad * __builtin_amdgcn_cosf(ub);
  z1 = rad * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ void box_muller(double ua, double ub, double& z0, double& z1) {
  const double rad = sqrt(-2.0 * log(ua));
  double s, c;
  sincospi(2.0 * ub, &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

// Four normals from one Philox call: (w0, w1) -> z0, z1 and (w2, w3) -> z2, z3.
// Counter (k, s, c2, tag): c2 = g for the outer path, 16 b + g for its continuation b
// (tag kTagBranch) after a branching date.
template <typename Real>
__device__ __forceinline__ void normals4(uint32_t k, uint32_t s, uint32_t c2, uint32_t key0,
                                         uint32_t key1, Real z[4], uint32_t tag = kTagOuter) {
  const u32x4 w = philox4x32_10(k, s, c2, tag, key0, key1);
  box_muller(uniform_of<Real>(w.x), uniform_of<Real>(w.y), z[0], z[1]);
  box_muller(uniform_of<Real>(w.z), uniform_of<Real>(w.w), z[2], z[3]);
}

}  // namespace hsim
