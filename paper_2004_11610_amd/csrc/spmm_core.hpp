// Matrix-core engines of the banded product (shared by the product kernels
// and the persistent executor).  One wave accumulates a 16 x 16 output tile
// (16 rows x 16 right-hand sides); a step covers 16 complex columns: lane l
// (m = l % 16, g = l / 16) holds the columns 4g .. 4g+3 of row m of the tile
// box and of right-hand side m.  The complex band is made real by doubling K:
//   sum_k Re(a_k z_k) = sum_k (Re a_k Re z_k - Im a_k Im z_k).
#pragma once

#include "common.hpp"

namespace spt {
namespace spmmcore {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

typedef float f32x8 __attribute__((ext_vector_type(8)));

// f = p0 + p1 + p2 with bfloat16 pieces: each piece is the round-to-nearest-
// even bfloat16 of what the previous ones leave (the residuals are exact in
// float32); eight values at a time with the packed conversion instructions.
struct Split8 {
  bf16x8 p[3];
  __device__ __forceinline__ explicit Split8(f32x8 f) {
    p[0] = __builtin_convertvector(f, bf16x8);
    const f32x8 r1 = f - __builtin_convertvector(p[0], f32x8);
    p[1] = __builtin_convertvector(r1, bf16x8);
    const f32x8 r2 = r1 - __builtin_convertvector(p[1], f32x8);
    p[2] = __builtin_convertvector(r2, bf16x8);
  }
  __device__ __forceinline__ bf16x8 get(int i) const { return p[i]; }
};

// Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b % 8).
// Row tile of workgroup b: consecutive tiles on the same XCD, so that the
// half-spectrum columns shared by neighbouring tiles are fetched into that
// XCD's L2 once.  A bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int n8 = n >> 3;
  return b < 8 * n8 ? (b & 7) * n8 + (b >> 3) : b;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// the same three pieces for a pair of values, each pair packed in 32 bits
__device__ __forceinline__ void split2(f32x2 f, uint32_t out[3]) {
  const bf16x2 p0 = __builtin_convertvector(f, bf16x2);
  const f32x2 r1 = f - __builtin_convertvector(p0, f32x2);
  const bf16x2 p1 = __builtin_convertvector(r1, bf16x2);
  const f32x2 r2 = r1 - __builtin_convertvector(p1, f32x2);
  const bf16x2 p2 = __builtin_convertvector(r2, bf16x2);
  out[0] = __builtin_bit_cast(uint32_t, p0);
  out[1] = __builtin_bit_cast(uint32_t, p1);
  out[2] = __builtin_bit_cast(uint32_t, p2);
}

// Engines: the accumulation of one step (4 complex columns per lane, i.e. 32
// real K per 16 x 16 tile) and of one real step (8 reals per lane).
//
// v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; element i of its accumulator is D[l/16 + 4i][l%16] for
// f64 and D[4(l/16) + i][l%16] for f32.
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l%16][8(l/16)+j] and
// B[8(l/16)+j][l%16], j < 8; D as for f32.
struct EngF64 {
  using T = double;
  using Acc = f64x4;
  static constexpr int SB = 1;
  __device__ static int row(int g, int i) { return g + 4 * i; }
  __device__ static Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ static Acc step(const double2* a, const double2* z, Acc acc) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j].x, z[j].x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[j].y, z[j].y, acc, 0, 0, 0);
    }
    return acc;
  }
  __device__ static Acc step_real(const double* a, const double* x, Acc acc) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], x[j], acc, 0, 0, 0);
    return acc;
  }
};

struct EngF32 {
  using T = float;
  using Acc = f32x4;
  static constexpr int SB = 2;
  __device__ static int row(int g, int i) { return 4 * g + i; }
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  // a step's eight products are summed from zero, then added to the running
  // sum (one rounding of the running sum per step)
  __device__ static Acc step(const float2* a, const float2* z, Acc acc) {
    Acc t = zero();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      t = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j].x, z[j].x, t, 0, 0, 0);
      t = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[j].y, z[j].y, t, 0, 0, 0);
    }
    return acc + t;
  }
  __device__ static Acc step_real(const float* a, const float* x, Acc acc) {
    Acc t = zero();
#pragma unroll
    for (int j = 0; j < 8; ++j) t = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], x[j], t, 0, 0, 0);
    return acc + t;
  }
};

// three bfloat16 pieces per operand, the six products of order <= 2 (small
// ones first), float32 accumulation: a step's products are summed from zero,
// then added to the running sum
struct EngSplitBf16 {
  using T = float;
  using Acc = f32x4;
  static constexpr int SB = 2;
  __device__ static int row(int g, int i) { return 4 * g + i; }
  __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static Acc mma6(const Split8& A, const Split8& B, Acc acc) {
    Acc t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(2), B.get(0), zero(), 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(1), B.get(1), t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(0), B.get(2), t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(1), B.get(0), t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(0), B.get(1), t, 0, 0, 0);
    t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(0), B.get(0), t, 0, 0, 0);
    return acc + t;
  }
  __device__ static Acc step(const float2* a, const float2* z, Acc acc) {
    f32x8 fa, fz;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      fa[2 * j] = a[j].x;
      fa[2 * j + 1] = -a[j].y;
      fz[2 * j] = z[j].x;
      fz[2 * j + 1] = z[j].y;
    }
    return mma6(Split8(fa), Split8(fz), acc);
  }
  __device__ static Acc step_real(const float* a, const float* x, Acc acc) {
    f32x8 fa, fx;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      fa[j] = a[j];
      fx[j] = x[j];
    }
    return mma6(Split8(fa), Split8(fx), acc);
  }
};

template <typename T>
struct StepRegs {
  cplx_t<T> a[4];
  cplx_t<T> z[4];
};

// value of lane b (b wave-uniform) as a wave-uniform scalar
__device__ __forceinline__ int lane_i32(int v, int b) { return __builtin_amdgcn_readlane(v, b); }
__device__ __forceinline__ int64_t lane_i64(int64_t v, int b) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), b);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

}  // namespace spmmcore
}  // namespace spt
