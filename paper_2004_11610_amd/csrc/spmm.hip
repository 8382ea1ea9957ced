// Banded products with the compressed blocks (E3 + E5 of the computation
// stage, eq. comp1) and with their transposes (Alg. 2 step 2.1).
//
// Storage of a compressed block (built by the precomputation): the N rows are
// cut into tiles of TILE_ROWS consecutive rows; tile t keeps the columns
// k0[t] .. k0[t]+kw[t]-1 of the half spectrum as a dense box, stored k-major
// (val[off[t] + kk*TILE_ROWS + q] is row 16t+q, column k0[t]+kk), entries
// below the threshold stored as zero, and already multiplied by c_k (1 at
// k = 0 and k = P, 2 otherwise) so that y = Re(sum_k c_k Add_k z_k) is the
// full-spectrum sum Add z for real A and real x (sec. 5.1).
//
// All blocks of a plan share the same row tiles, so one wave owns 16 output
// rows for a chunk of right-hand sides and sums every block and the direct
// tail in registers before writing y once (E5: blocks are independent).

#include "common.hpp"

namespace spt {
namespace {

constexpr int WAVES_PER_WG = 4;

// ---------------------------------------------------------------- VALU, T = double/float
// lane = right-hand side, wave = one row tile; the box values are uniform
// across the wave (scalar loads), z is per lane.
template <typename T>
__global__ __launch_bounds__(64 * WAVES_PER_WG) void spmm_valu_kernel(SpmmArgs<T> a) {
  using C = cplx_t<T>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = blockIdx.x * WAVES_PER_WG + wave;
  if (tile >= a.n_tiles) return;
  const int r = blockIdx.y * 64 + lane;
  const bool active = r < a.R;
  const int rr = active ? r : 0;
  T acc[TILE_ROWS];
#pragma unroll
  for (int q = 0; q < TILE_ROWS; ++q) acc[q] = T(0);

  for (int b = 0; b < a.nblk; ++b) {
    const int k0 = a.k0[b][tile];
    const int kw = a.kw[b][tile];
    const C* __restrict__ val = a.val[b] + a.off[b][tile];
    const C* __restrict__ z = a.z[b] + (int64_t)rr * a.ldz[b] + k0;
    for (int kk = 0; kk < kw; ++kk) {
      const C zv = z[kk];
#pragma unroll
      for (int q = 0; q < TILE_ROWS; ++q) {
        const C av = val[kk * TILE_ROWS + q];
        acc[q] += av.x * zv.x - av.y * zv.y;
      }
    }
  }
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  const int64_t ldt = (int64_t)a.n_tiles * TILE_ROWS;  // tail rows padded to tiles
  const T* __restrict__ x = a.X + (int64_t)rr * a.N;
  for (int m = 0; m < a.tail; ++m) {
    const T xv = x[m];
    const T* __restrict__ col = a.tailmat + (int64_t)m * ldt + n0;
#pragma unroll
    for (int q = 0; q < TILE_ROWS; ++q) acc[q] += col[q] * xv;
  }
  if (active) {
    T* __restrict__ y = a.Y + (int64_t)r * a.N + n0;
#pragma unroll
    for (int q = 0; q < TILE_ROWS; ++q)
      if (n0 + q < a.N) y[q] = acc[q];
  }
}

// ---------------------------------------------------------------- split-bf16 MFMA
// v_mfma_f32_16x16x32_bf16: D(16x16) += A(16x32) B(32x16) with, for lane l,
// A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16] (j < 8) and
// D[4 (l / 16) + i][l % 16] (i < 4).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even bfloat16, returned as the float it represents
__device__ __forceinline__ float bf16_round(float f) {
  uint32_t u = __float_as_uint(f);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

// f = p0 + p1 + p2 with bfloat16 pieces (each residual is exact in float32)
__device__ __forceinline__ void split3(float f, unsigned short& p0, unsigned short& p1,
                                       unsigned short& p2) {
  const float f0 = bf16_round(f);
  const float e1 = f - f0;
  const float f1 = bf16_round(e1);
  const float f2 = bf16_round(e1 - f1);
  p0 = (unsigned short)(__float_as_uint(f0) >> 16);
  p1 = (unsigned short)(__float_as_uint(f1) >> 16);
  p2 = (unsigned short)(__float_as_uint(f2) >> 16);
}

struct Split8 {
  u16x8 p[3];
  __device__ __forceinline__ void set(int j, float f) {
    unsigned short a, b, c;
    split3(f, a, b, c);
    p[0][j] = a;
    p[1][j] = b;
    p[2][j] = c;
  }
  __device__ __forceinline__ bf16x8 get(int i) const { return __builtin_bit_cast(bf16x8, p[i]); }
};

// acc += sum over the six products A_i B_j with i + j <= 2
__device__ __forceinline__ f32x4 mfma6(const Split8& A, const Split8& B, f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(2), B.get(0), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(1), B.get(1), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(0), B.get(2), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(1), B.get(0), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(0), B.get(1), acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.get(0), B.get(0), acc, 0, 0, 0);
  return acc;
}

// One wave: 16 rows x 64 right-hand sides (four 16x16 output tiles).  The
// complex band is made real by K' = 2K: A'[q][2kk] = Re a, A'[q][2kk+1] = -Im a,
// B'[2kk][r] = Re z, B'[2kk+1][r] = Im z, so sum_k' A' B' = Re(a z).
__global__ __launch_bounds__(64 * WAVES_PER_WG) void spmm_split_bf16_kernel(SpmmArgs<float> a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = blockIdx.x * WAVES_PER_WG + wave;
  if (tile >= a.n_tiles) return;
  const int m = lane & 15, g = lane >> 4;
  const int r_base = blockIdx.y * 64;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int b = 0; b < a.nblk; ++b) {
    const int k0 = a.k0[b][tile];
    const int kw = a.kw[b][tile];
    const float2* __restrict__ val = a.val[b] + a.off[b][tile];
    const float2* __restrict__ zb = a.z[b] + k0;
    const int ldz = a.ldz[b];
    for (int ks = 0; ks < kw; ks += 16) {
      Split8 A;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int kk = ks + 4 * g + j;
        const float2 av = kk < kw ? val[kk * TILE_ROWS + m] : float2{0.f, 0.f};
        A.set(2 * j, av.x);
        A.set(2 * j + 1, -av.y);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = r_base + 16 * t + m;
        Split8 B;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int kk = ks + 4 * g + j;
          const float2 zv = (kk < kw && r < a.R) ? zb[(int64_t)r * ldz + kk] : float2{0.f, 0.f};
          B.set(2 * j, zv.x);
          B.set(2 * j + 1, zv.y);
        }
        acc[t] = mfma6(A, B, acc[t]);
      }
    }
  }
  // direct tail: A'[q][m'] = tail[m'][row q], B'[m'][r] = x[r][m'], K = tail
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  const int64_t ldt = (int64_t)a.n_tiles * TILE_ROWS;
  for (int ks = 0; ks < a.tail; ks += 32) {
    Split8 A;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int mm = ks + 8 * g + j;
      A.set(j, mm < a.tail ? a.tailmat[(int64_t)mm * ldt + n0 + m] : 0.f);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = r_base + 16 * t + m;
      Split8 B;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int mm = ks + 8 * g + j;
        B.set(j, (mm < a.tail && r < a.R) ? a.X[(int64_t)r * a.N + mm] : 0.f);
      }
      acc[t] = mfma6(A, B, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = r_base + 16 * t + m;
    if (r < a.R) {
      float* __restrict__ y = a.Y + (int64_t)r * a.N + n0 + 4 * g;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (n0 + 4 * g + i < a.N) y[i] = acc[t][i];
    }
  }
}

// ---------------------------------------------------------------- transposed
// u[r][k] = sum_n Add[n][k] f[r][n] over the half spectrum (c_k removed), one
// wave per row tile, lane = right-hand side, accumulated with atomics since
// neighbouring tiles share columns.
template <typename T>
__global__ __launch_bounds__(64 * WAVES_PER_WG) void spmm_transposed_kernel(SpmmTArgs<T> a) {
  using C = cplx_t<T>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = blockIdx.x * WAVES_PER_WG + wave;
  if (tile >= a.n_tiles) return;
  const int r = blockIdx.y * 64 + lane;
  if (r >= a.R) return;
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  T f[TILE_ROWS];
  const T* __restrict__ fr = a.F + (int64_t)r * a.N;
#pragma unroll
  for (int q = 0; q < TILE_ROWS; ++q) f[q] = (n0 + q < a.N) ? fr[n0 + q] : T(0);
  const int k0 = a.k0[tile], kw = a.kw[tile];
  const C* __restrict__ val = a.val + a.off[tile];
  C* __restrict__ u = a.u + (int64_t)r * a.ldu;
  for (int kk = 0; kk < kw; ++kk) {
    T sr = T(0), si = T(0);
#pragma unroll
    for (int q = 0; q < TILE_ROWS; ++q) {
      const C av = val[kk * TILE_ROWS + q];
      sr += av.x * f[q];
      si += av.y * f[q];
    }
    const int k = k0 + kk;
    const T ck = (k == 0 || k == a.P) ? T(1) : T(0.5);
    atomicAdd(&u[k].x, sr * ck);
    atomicAdd(&u[k].y, si * ck);
  }
}

// fhat[r][m] = sum_j tail[m][j] f[r][j] for m < tail: one workgroup per (m, r)
template <typename T>
__global__ __launch_bounds__(256) void tail_transposed_kernel(const T* __restrict__ tailmat,
                                                              int64_t ldt, const T* __restrict__ F,
                                                              T* __restrict__ Y, int64_t N) {
  const int m = blockIdx.x, r = blockIdx.y;
  const T* __restrict__ col = tailmat + (int64_t)m * ldt;
  const T* __restrict__ f = F + (int64_t)r * N;
  T s = T(0);
  for (int64_t j = threadIdx.x; j < N; j += blockDim.x) s += col[j] * f[j];
  __shared__ T part[256];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) Y[(int64_t)r * N + m] = part[0];
}

dim3 spmm_grid(int n_tiles, int R) {
  return dim3((n_tiles + WAVES_PER_WG - 1) / WAVES_PER_WG, (R + 63) / 64);
}

}  // namespace

template <typename T>
void launch_spmm(const SpmmArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL(spmm_valu_kernel<T>, spmm_grid(a.n_tiles, a.R), dim3(64 * WAVES_PER_WG), 0,
                     s, a);
  SPT_HIP(hipGetLastError());
}

void launch_spmm_split_bf16(const SpmmArgs<float>& a, hipStream_t s) {
  hipLaunchKernelGGL(spmm_split_bf16_kernel, spmm_grid(a.n_tiles, a.R),
                     dim3(64 * WAVES_PER_WG), 0, s, a);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_spmm_transposed(const SpmmTArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL(spmm_transposed_kernel<T>, spmm_grid(a.n_tiles, a.R),
                     dim3(64 * WAVES_PER_WG), 0, s, a);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_tail_transposed(const T* tailmat, int tail, const T* F, T* Y, int R, int64_t N,
                            hipStream_t s) {
  if (tail <= 0) return;
  const int64_t ldt = ((N + TILE_ROWS - 1) / TILE_ROWS) * TILE_ROWS;
  hipLaunchKernelGGL(tail_transposed_kernel<T>, dim3(tail, R), dim3(256), 0, s, tailmat, ldt, F,
                     Y, N);
  SPT_HIP(hipGetLastError());
}

template void launch_spmm<double>(const SpmmArgs<double>&, hipStream_t);
template void launch_spmm<float>(const SpmmArgs<float>&, hipStream_t);
template void launch_spmm_transposed<double>(const SpmmTArgs<double>&, hipStream_t);
template void launch_spmm_transposed<float>(const SpmmTArgs<float>&, hipStream_t);
template void launch_tail_transposed<double>(const double*, int, const double*, double*, int,
                                             int64_t, hipStream_t);
template void launch_tail_transposed<float>(const float*, int, const float*, float*, int,
                                            int64_t, hipStream_t);

}  // namespace spt
