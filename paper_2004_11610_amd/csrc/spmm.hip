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
//
// The product is a chain of small dense contractions (each tile box is a
// dense 16 x kw complex matrix), run on the matrix cores in all precisions.

#include <type_traits>

#include "spmm_core.hpp"

namespace spt {
namespace {

using namespace spmmcore;

constexpr int WAVES_PER_WG = 4;

// ---------------------------------------------------------------- matrix-core product
// One workgroup = one row tile (16 rows) x 64 right-hand sides; wave w owns the
// right-hand sides 16w .. 16w+15, i.e. one 16 x 16 output tile, accumulated by
// matrix-core instructions over the columns of every block's tile box and of
// the direct tail.  Steps are taken in batches of E::SB (across block
// boundaries): all loads of a batch are issued before its first matrix
// instruction, so a wave waits for memory about once per batch.
// one workgroup: row tile `tile` x right-hand sides r0 .. r0 + 63
template <typename E>
__device__ __forceinline__ void mfma_tile(const SpmmArgs<typename E::T>& args, int tile, int r0) {
  using T = typename E::T;
  using C = cplx_t<T>;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int r_wave = r0 + wave * 16;
  if (r_wave >= args.R) return;  // wave-uniform: no right-hand side left
  const int m = lane & 15, g = lane >> 4;
  const int r = r_wave + m;
  const bool rok = r < args.R;
  const int64_t rr = rok ? r : r_wave;

  // lane b holds the tile box and block descriptor of block b (one load each)
  int k0_l = 0, kw_l = 0;
  int64_t off_l = 0, val_l = 0, zoff_l = 0;
  int ldz_l = 0;
  if (lane < args.nblk) {
    const TileMeta tm = args.meta[(int64_t)tile * args.nblk + lane];
    const SpmmBlock<T> bd = args.blocks[lane];
    k0_l = tm.k0;
    kw_l = tm.kw;
    off_l = tm.off;
    val_l = (int64_t)(uintptr_t)bd.val;
    zoff_l = bd.zoff;
    ldz_l = bd.ldz;
  }
  auto next_item = [&](int b, int kk, int& ob, int& okk) {
    while (b < args.nblk && kk >= lane_i32(kw_l, b)) {
      ++b;
      kk = 0;
    }
    ob = b;
    okk = kk;
  };
  auto load = [&](int b, int kk, StepRegs<T>& s) {
    const int kw = lane_i32(kw_l, b);
    const int k0 = lane_i32(k0_l, b);
    const C* __restrict__ val = (const C*)(uintptr_t)lane_i64(val_l, b) + lane_i64(off_l, b);
    const C* __restrict__ zb =
        args.Z + (int64_t)args.R * lane_i64(zoff_l, b) + rr * lane_i32(ldz_l, b) + k0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = kk + 4 * g + j;
      const bool ok = c < kw;
      s.a[j] = ok ? val[c * TILE_ROWS + m] : C{T(0), T(0)};
      s.z[j] = (ok && rok) ? zb[c] : C{T(0), T(0)};
    }
  };

  typename E::Acc acc = E::zero();
  int b, kk;
  next_item(0, 0, b, kk);
  while (b < args.nblk) {
    StepRegs<T> batch[E::SB];
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < E::SB; ++i) {
      if (b < args.nblk) {
        load(b, kk, batch[i]);
        cnt = i + 1;
        next_item(b, kk + 16, b, kk);
      }
    }
#pragma unroll
    for (int i = 0; i < E::SB; ++i)
      if (i < cnt) acc = E::step(batch[i].a, batch[i].z, acc);
  }

  // direct tail: A'[q][m'] = tail[m'][row q], B'[m'][r] = x[r][m']
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  const int64_t ldt = (int64_t)args.n_tiles * TILE_ROWS;
  const T* __restrict__ xr = args.X + rr * args.N;
  for (int ks = 0; ks < args.tail; ks += 32) {
    T av[8], xv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int mm = ks + 8 * g + j;
      const bool ok = mm < args.tail;
      av[j] = ok ? args.tailmat[(int64_t)mm * ldt + n0 + m] : T(0);
      xv[j] = (ok && rok) ? xr[mm] : T(0);
    }
    acc = E::step_real(av, xv, acc);
  }
  if (rok) {
    T* __restrict__ y = args.Y + (int64_t)r * args.N + n0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = E::row(g, i);
      if (n0 + q < args.N) y[q] = acc[i];
    }
  }
}

// ---------------------------------------------------------------- pre-split product
// Same tiling as spmm_mfma_kernel (workgroup = tile x 64 right-hand sides,
// wave = 16 of them); both operands arrive as bfloat16 pieces (layout in
// common.hpp), so a step is three 16-byte loads of each operand and the six
// matrix-core products, with no conversion in the loop.
constexpr int PRESPLIT_SB = 4;

struct PieceRegs {
  bf16x8 a[3];
  bf16x8 z[3];
};

__device__ __forceinline__ f32x4 mma6_pieces(const bf16x8* A, const bf16x8* B, f32x4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], B[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[0], acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ void presplit_tile(const SpmmSplitArgs& args, int tile, int r0) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int r_wave = r0 + wave * 16;
  if (r_wave >= args.R) return;  // wave-uniform
  const int m = lane & 15, g = lane >> 4;
  const int r = r_wave + m;
  const bool rok = r < args.R;
  const int64_t rr = rok ? r : r_wave;
  const bf16x8 zero8 = bf16x8{};

  int k0_l = 0, kw_l = 0, ldz_l = 0;
  int64_t off_l = 0, val_l = 0, zoff_l = 0;
  if (lane < args.nblk) {
    const TileMeta tm = args.meta[(int64_t)tile * args.nblk + lane];
    const SpmmSplitBlock bd = args.blocks[lane];
    k0_l = tm.k0;
    kw_l = tm.kw;
    off_l = tm.off;
    val_l = (int64_t)(uintptr_t)bd.val;
    zoff_l = bd.zoff;
    ldz_l = bd.ldz;
  }
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int b = 0; b < args.nblk; ++b) {
    const int kw = lane_i32(kw_l, b);
    const int steps = (kw + 15) >> 4;
    const bf16x8* __restrict__ va =
        reinterpret_cast<const bf16x8*>((const uint16_t*)(uintptr_t)lane_i64(val_l, b) +
                                        lane_i64(off_l, b)) + lane;
    // pieces of z: rhs rr, complex columns k0 + 16 s + 4 g .. + 3 (16 bytes)
    const uint32_t* __restrict__ zb = args.Zs + (int64_t)args.R * lane_i64(zoff_l, b) +
                                      rr * lane_i32(ldz_l, b) + lane_i32(k0_l, b) + 4 * g;
    for (int s0 = 0; s0 < steps; s0 += PRESPLIT_SB) {
      PieceRegs st[PRESPLIT_SB];
#pragma unroll
      for (int i = 0; i < PRESPLIT_SB; ++i) {
        const int s = s0 + i;
        const bool in = s < steps;
        const bool zin = in && rok && 16 * s + 4 * g < kw;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          st[i].a[p] = in ? va[(3 * s + p) * 64] : zero8;
          st[i].z[p] = zin ? *reinterpret_cast<const bf16x8*>(zb + p * args.zplane + 16 * s)
                           : zero8;
        }
      }
#pragma unroll
      for (int i = 0; i < PRESPLIT_SB; ++i)
        if (s0 + i < steps) acc = mma6_pieces(st[i].a, st[i].z, acc);
    }
  }
  // direct tail: pre-split rows, x split here
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  const float* __restrict__ xr = args.X + rr * args.N;
  const int tsteps = (args.tail + 31) / 32;
  const bf16x8* __restrict__ ta = reinterpret_cast<const bf16x8*>(args.tailmat);
  for (int s = 0; s < tsteps; ++s) {
    f32x8 xv;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int mm = 32 * s + 8 * g + j;
      xv[j] = (mm < args.tail && rok) ? xr[mm] : 0.f;
    }
    const Split8 xs(xv);
    bf16x8 A[3], B[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      A[p] = ta[(((int64_t)tile * tsteps + s) * 3 + p) * 64 + lane];
      B[p] = xs.get(p);
    }
    acc = mma6_pieces(A, B, acc);
  }
  if (rok) {
    float* __restrict__ y = args.Y + (int64_t)r * args.N + n0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = 4 * g + i;
      if (n0 + q < args.N) y[q] = acc[i];
    }
  }
}

template <typename E>
__global__ __launch_bounds__(256) void spmm_mfma_kernel(SpmmArgs<typename E::T> args) {
  mfma_tile<E>(args, xcd_tile(blockIdx.x, args.n_tiles), blockIdx.y * 64);
}

__global__ __launch_bounds__(256) void spmm_presplit_kernel(SpmmSplitArgs args) {
  presplit_tile(args, xcd_tile(blockIdx.x, args.n_tiles), blockIdx.y * 64);
}

// Several plans in one launch: workgroup b takes item b = (plan, tile, r0);
// tile < 0 pads a plan's items to a multiple of 8 (XCD order as above).
template <typename E>
__global__ __launch_bounds__(256) void spmm_mfma_items_kernel(SpmmBatch<typename E::T> b) {
  const int4 it = b.items[blockIdx.x];
  if (it.y < 0) return;
  SpmmArgs<typename E::T> a = b.plans[it.x];
  a.X = b.X[it.x];
  a.Y = b.Y[it.x];
  mfma_tile<E>(a, it.y, it.z);
}

__global__ __launch_bounds__(256) void spmm_presplit_items_kernel(SpmmSplitBatch b) {
  const int4 it = b.items[blockIdx.x];
  if (it.y < 0) return;
  SpmmSplitArgs a = b.plans[it.x];
  a.X = b.X[it.x];
  a.Y = b.Y[it.x];
  presplit_tile(a, it.y, it.z);
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
  using E = typename std::conditional<std::is_same<T, double>::value, EngF64, EngF32>::type;
  hipLaunchKernelGGL(spmm_mfma_kernel<E>, dim3(a.n_tiles, (a.R + 63) / 64), dim3(256), 0, s, a);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_spmm_items(const SpmmBatch<T>& b, int n_items, hipStream_t s) {
  if (n_items <= 0) return;
  using E = typename std::conditional<std::is_same<T, double>::value, EngF64, EngF32>::type;
  hipLaunchKernelGGL(spmm_mfma_items_kernel<E>, dim3(n_items), dim3(256), 0, s, b);
  SPT_HIP(hipGetLastError());
}
template void launch_spmm_items<double>(const SpmmBatch<double>&, int, hipStream_t);
template void launch_spmm_items<float>(const SpmmBatch<float>&, int, hipStream_t);

void launch_spmm_presplit_items(const SpmmSplitBatch& b, int n_items, hipStream_t s) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(spmm_presplit_items_kernel, dim3(n_items), dim3(256), 0, s, b);
  SPT_HIP(hipGetLastError());
}

void launch_spmm_presplit(const SpmmSplitArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(spmm_presplit_kernel, dim3(a.n_tiles, (a.R + 63) / 64), dim3(256), 0, s, a);
  SPT_HIP(hipGetLastError());
}

void launch_spmm_split_bf16(const SpmmArgs<float>& a, hipStream_t s) {
  hipLaunchKernelGGL(spmm_mfma_kernel<EngSplitBf16>, dim3(a.n_tiles, (a.R + 63) / 64),
                     dim3(256), 0, s, a);
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
