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
#include <vector>

#include "spmm_core.hpp"

namespace spt {
namespace {

using namespace spmmcore;

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

// The six piece products of a step are summed from zero (their rounding is
// relative to the step's own sum) and the step's sum is then added to the
// running sum: one rounding of the running sum per step instead of six.
__device__ __forceinline__ f32x4 mma6_pieces(const bf16x8* A, const bf16x8* B, f32x4 acc) {
  f32x4 t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], B[0], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[1], t, 0, 0, 0);
  t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[2], t, 0, 0, 0);
  t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[0], t, 0, 0, 0);
  t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[1], t, 0, 0, 0);
  t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[0], t, 0, 0, 0);
  return acc + t;
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

// ---------------------------------------------------------------- windowed pre-split product
// One workgroup = WIN_TILES consecutive row tiles x 16 RG right-hand sides
// (RG = 4 or 2); wave w owns row tile w for all of them (RG 16 x 16
// accumulators).
// Neighbouring tiles need overlapping columns of each block's half spectra, so
// the workgroup first copies, for every block, the union of its tiles' boxes
// (all three pieces, all the workgroup's right-hand sides) into LDS with direct
// global-to-LDS loads, which hold no registers while in flight; every wave then
// reads its steps' spectra from LDS and only its matrix pieces from memory.
// Each spectrum column crosses from L2 once per workgroup, not once per tile
// and group of 16 right-hand sides.
constexpr int WIN_SLOTS = 8;  // steps whose matrix pieces are loaded together

// acc[q] += A * B[q] over the six piece products (small ones first, summed
// from zero as in mma6_pieces), the RG accumulators interleaved
template <int RG>
__device__ __forceinline__ void mma6xg(const bf16x8* A, const bf16x8 (*B)[3], f32x4* acc) {
  constexpr int ia[6] = {2, 1, 0, 1, 0, 0};
  constexpr int ib[6] = {0, 1, 2, 0, 1, 0};
  f32x4 t[RG];
#pragma unroll
  for (int q = 0; q < RG; ++q) t[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 6; ++k)
#pragma unroll
    for (int q = 0; q < RG; ++q)
      t[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ia[k]], B[q][ib[k]], t[q], 0, 0, 0);
#pragma unroll
  for (int q = 0; q < RG; ++q) acc[q] += t[q];
}

// RG: groups of 16 right-hand sides per wave (4 or 2); WS: waves per row tile
// (1, or 2 sharing the tile's matrix pieces, each with its own RG groups of
// right-hand sides: 8 waves); the windows hold 3 * 16 RG WS rows.
template <int RG, int WS>
__global__ __launch_bounds__(256 * WS) void spmm_window_kernel(SpmmSplitArgs args,
                                                               const WinMeta* __restrict__ win,
                                                               int n_groups, int xlds, int tpad) {
  extern __shared__ __align__(16) uint4 zl[];
  const int grp = xcd_tile(blockIdx.x, n_groups);
  // the metadata, window and matrix loads at raised wave priority, so that
  // beside other streams' FFT workgroups (long runs of vector work) they are
  // issued first; back to normal for the matrix-core steps
  __builtin_amdgcn_s_setprio(3);
  constexpr int NR = 16 * RG * WS;  // right-hand sides of the workgroup
  constexpr int NW = WIN_TILES * WS;  // waves
  const int r0 = blockIdx.y * NR;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, g = lane >> 4;
  const int nblk = args.nblk;
  // wave: row tile wave % WIN_TILES, right-hand sides rw .. rw + 16 RG - 1 of
  // the workgroup's
  const int rw = (wave / WIN_TILES) * 16 * RG;
  const int tile = grp * WIN_TILES + wave % WIN_TILES;
  const bool has_tile = tile < args.n_tiles;  // wave-uniform
  const bf16x8 zero8 = bf16x8{};

  // lane b < nblk: the window of block b, its descriptor and the box of (tile, b)
  int wk0_l = 0, ww4_l = 0, wpitch_l = 3, wlds_l = 0, wunits_l = 0, wmagic_l = 0;
  int k0_l = 0, kw_l = 0, ldz_l = 0;
  int64_t off_l = 0, val_l = 0, zoff_l = 0;
  if (lane < nblk) {
    const WinMeta wm = win[(int64_t)grp * nblk + lane];
    wk0_l = wm.k0;
    ww4_l = wm.w4;
    wpitch_l = wm.pitch;
    wlds_l = wm.lds;
    wunits_l = wm.units;
    wmagic_l = (int)wm.magic;
    const SpmmSplitBlock bd = args.blocks[lane];
    val_l = (int64_t)(uintptr_t)bd.val;
    zoff_l = bd.zoff;
    ldz_l = bd.ldz;
    if (has_tile) {
      const TileMeta tm = args.meta[(int64_t)tile * nblk + lane];
      k0_l = tm.k0;
      kw_l = tm.kw;
      off_l = tm.off;
    }
  }
  // every address below derives from these: waiting here, on every path, keeps
  // the loads issued below free of waits for one another
  __builtin_amdgcn_s_waitcnt(0);
  // steps of the tile are numbered through the blocks in order; lane b holds
  // the number of the first step of block b
  int start_l = 0, total = 0;
  for (int bb = 0; bb < nblk; ++bb) {
    if (lane == bb) start_l = total;
    total += (lane_i32(kw_l, bb) + 15) >> 4;
  }
  const int end_l = start_l + (lane < nblk ? (kw_l + 15) >> 4 : 0);

  // 1. windows -> LDS: unit u of a window is row u / pitch, column group
  // u % pitch; units past the window's width or rows (padding) and right-hand
  // sides past R load a valid neighbour and are never read
  for (int bw = 0; bw < nblk; ++bw) {
    const int units = lane_i32(wunits_l, bw);
    if (units == 0) continue;
    const int w4 = lane_i32(ww4_l, bw), pitch = lane_i32(wpitch_l, bw);
    const uint32_t magic = (uint32_t)lane_i32(wmagic_l, bw);
    const int ldz = lane_i32(ldz_l, bw);
    uint4* __restrict__ dst = zl + lane_i32(wlds_l, bw);
    // byte offsets from the window's first column fit 32 bits (checked on the host)
    const char* __restrict__ zw = reinterpret_cast<const char*>(
        args.Zs + (int64_t)args.R * lane_i64(zoff_l, bw) + lane_i32(wk0_l, bw));
    for (int c = wave; c * 64 < units; c += NW) {
      const uint32_t u = (uint32_t)(c * 64 + lane);
      const uint32_t q = __umulhi(u, magic);
      const uint32_t cg = min(u - q * (uint32_t)pitch, (uint32_t)w4 - 1u);
      const uint32_t p = min(q / NR, 2u);
      const uint32_t rhs = (uint32_t)min(r0 + (int)(q % NR), args.R - 1);
      const uint32_t off = (p * (uint32_t)args.zplane + rhs * (uint32_t)ldz + 4u * cg) * 4u;
      __builtin_amdgcn_global_load_lds(zw + off, dst + c * 64, 16, 0, 0);
    }
  }
  // x of the direct tail -> LDS after the windows: right-hand side r0 + i at
  // xl + i * tpad (tpad = 32 * tail steps + 4 floats, NR * tpad a multiple of
  // 64); columns past the tail repeat its last one and are never used
  float* __restrict__ xl = reinterpret_cast<float*>(zl + xlds);
  for (int c = wave; c * 64 < NR * tpad; c += NW) {
    const int u = c * 64 + lane;
    const int i = u / tpad, mm = u - i * tpad;
    const float* src = args.X + (int64_t)min(r0 + i, args.R - 1) * args.N + min(mm, args.tail - 1);
    __builtin_amdgcn_global_load_lds(src, xl + c * 64, 4, 0, 0);
  }

  // 2. while those are in flight: the matrix pieces of the tile's first
  // WIN_SLOTS steps and of its first tail step (branch-free: past the last
  // step the loads repeat it, so that they are all in flight together)
  bf16x8 A[WIN_SLOTS][3];
  int sb[WIN_SLOTS], ss[WIN_SLOTS];
  int next = 0, cnt = 0;
  auto load_steps = [&]() {
#pragma unroll
    for (int i = 0; i < WIN_SLOTS; ++i) {
      const int j = min(next + i, total - 1);
      const int bk = (int)__popcll(__ballot(lane < nblk && end_l <= j));
      const int st = j - lane_i32(start_l, bk);
      const bf16x8* __restrict__ va =
          reinterpret_cast<const bf16x8*>((const uint16_t*)(uintptr_t)lane_i64(val_l, bk) +
                                          lane_i64(off_l, bk)) + lane;
#pragma unroll
      for (int p = 0; p < 3; ++p) A[i][p] = gload(va + (3 * st + p) * 64);
      sb[i] = bk;
      ss[i] = st;
    }
    cnt = min(WIN_SLOTS, total - next);
    next += WIN_SLOTS;
  };
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  const int tsteps = has_tile ? (args.tail + 31) / 32 : 0;
  const bf16x8* __restrict__ ta = reinterpret_cast<const bf16x8*>(args.tailmat);
  bf16x8 TA[3];
  auto load_tail = [&](int st) {
#pragma unroll
    for (int p = 0; p < 3; ++p)
      TA[p] = gload(ta + (((int64_t)tile * tsteps + st) * 3 + p) * 64 + lane);
  };
  if (total > 0) load_steps();
  if (tsteps > 0) load_tail(0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);
  if (!has_tile) return;

  // 3. every block's steps: matrix pieces from memory, spectra from LDS
  f32x4 acc[RG];
#pragma unroll
  for (int q = 0; q < RG; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  while (cnt > 0) {
#pragma unroll
    for (int i = 0; i < WIN_SLOTS; ++i) {
      if (i < cnt) {
        const int bk = sb[i], st = ss[i];
        const int pitch = lane_i32(wpitch_l, bk);
        // columns k0 + 16 st + 4 g .. + 3 of the tile's box, in the window;
        // groups past the box (whose matrix pieces are zero) read the window's
        // last group instead, a finite value
        const int cg = min(((lane_i32(k0_l, bk) - lane_i32(wk0_l, bk)) >> 2) + 4 * st + g,
                           lane_i32(ww4_l, bk) - 1);
        const uint4* __restrict__ zr = zl + lane_i32(wlds_l, bk) + cg + m * pitch;
        bf16x8 Z[RG][3];
#pragma unroll
        for (int q = 0; q < RG; ++q)
#pragma unroll
          for (int p = 0; p < 3; ++p)
            Z[q][p] = __builtin_bit_cast(bf16x8, zr[(p * NR + rw + 16 * q) * pitch]);
        mma6xg<RG>(A[i], Z, acc);
      }
    }
    if (next >= total) break;
    load_steps();
  }

  // 4. direct tail: x from LDS, split here
  for (int st = 0; st < tsteps; ++st) {
    if (st > 0) load_tail(st);
    bf16x8 B[RG][3];
#pragma unroll
    for (int q = 0; q < RG; ++q) {
      const float4* xq =
          reinterpret_cast<const float4*>(xl + (rw + 16 * q + m) * tpad + 32 * st + 8 * g);
      const float4 lo = xq[0], hi = xq[1];
      const float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      f32x8 xv;
#pragma unroll
      for (int j = 0; j < 8; ++j) xv[j] = 32 * st + 8 * g + j < args.tail ? v[j] : 0.f;
      const Split8 xs(xv);
#pragma unroll
      for (int p = 0; p < 3; ++p) B[q][p] = xs.get(p);
    }
    mma6xg<RG>(TA, B, acc);
  }

  // 5. y: lane (m, g) holds rows 4g .. 4g+3 of right-hand side r0 + rw + 16 q + m
#pragma unroll
  for (int q = 0; q < RG; ++q) {
    const int rhs = r0 + rw + 16 * q + m;
    if (rhs < args.R) {
      float* __restrict__ y = args.Y + (int64_t)rhs * args.N + n0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (n0 + 4 * g + i < args.N) y[4 * g + i] = acc[q][i];
    }
  }
}

// ---------------------------------------------------------------- chunked windowed product
// For plans whose windows do not fit a workgroup's LDS (wide boxes, e.g. the
// Laguerre and Hermite functions, where the product is a nearly dense
// contraction): the workgroup of the windowed product (WIN_TILES row tiles x
// CK_NR right-hand sides, wave = one tile), but each block's union window
// passes through LDS in chunks of CK_G column groups of 4, plus CK_HALO groups
// so that every step starting in the chunk lies in it.  Two buffers: the next
// chunk (direct global-to-LDS loads) and the tile's matrix pieces for it are
// requested before the current chunk is used.  The spectra of a chunk cross
// from L2 once for the four tiles instead of once per tile.  A tile's steps
// are taken in the per-tile product's order (blocks in order, steps in order
// within a block), so the sums are the same bits.
constexpr int CK_G = 8;
constexpr int CK_HALO = 3;
constexpr int CK_PITCH = 11;  // LDS row pitch in 16-byte units: odd, >= CK_G + CK_HALO
constexpr int CK_NR = 64;
constexpr int CK_UNITS = 3 * CK_NR * CK_PITCH;  // 16-byte units of one buffer
static_assert(CK_UNITS % 64 == 0 && CK_PITCH >= CK_G + CK_HALO, "chunk buffer layout");

__device__ __forceinline__ void chunk_group(const SpmmSplitArgs& args,
                                            const WinMeta* __restrict__ win, int grp, int r0,
                                            int tpad) {
  constexpr int RG = CK_NR / 16, NR = CK_NR;
  extern __shared__ __align__(16) uint4 zl[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, g = lane >> 4;
  const int nblk = args.nblk;
  const int tile = grp * WIN_TILES + wave;
  const bool has_tile = tile < args.n_tiles;  // wave-uniform
  const bf16x8 zero8 = bf16x8{};

  // lane b < nblk: the union window of block b (k0, w4), its descriptor and
  // the box of (tile, b)
  int wk0_l = 0, ww4_l = 0, k0_l = 0, kw_l = 0, ldz_l = 0;
  int64_t off_l = 0, val_l = 0, zoff_l = 0;
  if (lane < nblk) {
    const WinMeta wm = win[(int64_t)grp * nblk + lane];
    wk0_l = wm.k0;
    ww4_l = wm.w4;
    const SpmmSplitBlock bd = args.blocks[lane];
    val_l = (int64_t)(uintptr_t)bd.val;
    zoff_l = bd.zoff;
    ldz_l = bd.ldz;
    if (has_tile) {
      const TileMeta tm = args.meta[(int64_t)tile * nblk + lane];
      k0_l = tm.k0;
      kw_l = tm.kw;
      off_l = tm.off;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  // chunks are numbered through the blocks in order; lane b holds the number
  // of the first chunk of block b
  int cstart_l = 0, nch = 0;
  for (int bb = 0; bb < nblk; ++bb) {
    if (lane == bb) cstart_l = nch;
    nch += (lane_i32(ww4_l, bb) + CK_G - 1) / CK_G;
  }
  const int cend_l = cstart_l + (lane < nblk ? (ww4_l + CK_G - 1) / CK_G : 0);
  auto block_of = [&](int c) { return (int)__popcll(__ballot(lane < nblk && cend_l <= c)); };

  // chunk c (block b, chunk j: window groups CK_G j .. CK_G j + nst - 1) into
  // buffer c & 1: row q = p NR + i (piece p, right-hand side r0 + i), groups
  // past the window repeat its last one, right-hand sides past R the last one
  auto stage = [&](int c) {
    const int b = block_of(c);
    const int j = c - lane_i32(cstart_l, b);
    const int gbeg = j * CK_G;
    const int nst = min(CK_G + CK_HALO, lane_i32(ww4_l, b) - gbeg);
    const int64_t ldz = lane_i32(ldz_l, b);
    const char* __restrict__ zw = reinterpret_cast<const char*>(
        args.Zs + (int64_t)args.R * lane_i64(zoff_l, b) + lane_i32(wk0_l, b) + 4 * gbeg);
    uint4* __restrict__ dst = zl + (c & 1) * CK_UNITS;
    for (int cc = wave; cc * 64 < CK_UNITS; cc += 4) {
      const int u = cc * 64 + lane;
      const int row = u / CK_PITCH, col = min(u - row * CK_PITCH, nst - 1);
      const int p = row / NR, rhs = min(r0 + row - p * NR, args.R - 1);
      const int64_t off = ((int64_t)p * args.zplane + rhs * ldz + 4 * col) * 4;
      __builtin_amdgcn_global_load_lds(zw + off, dst + cc * 64, 16, 0, 0);
    }
  };
  // the tile's steps in chunk c: s_lo .. s_lo + ns - 1 (at most 2: the steps
  // whose first group base + 4 s lies in [CK_G j, CK_G j + CK_G)), their
  // matrix pieces
  auto load_a = [&](int c, bf16x8 (*Ar)[3], int& s_lo, int& ns) {
    const int b = block_of(c);
    const int j = c - lane_i32(cstart_l, b);
    const int base = (lane_i32(k0_l, b) - lane_i32(wk0_l, b)) >> 2;
    const int S = (lane_i32(kw_l, b) + 15) >> 4;
    const int lo = max(0, (CK_G * j - base + 3) >> 2);
    const int hi = min(S, (CK_G * j + CK_G - base + 3) >> 2);
    s_lo = lo;
    ns = has_tile ? max(0, hi - lo) : 0;
    const bf16x8* __restrict__ va =
        reinterpret_cast<const bf16x8*>((const uint16_t*)(uintptr_t)lane_i64(val_l, b) +
                                        lane_i64(off_l, b)) + lane;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int p = 0; p < 3; ++p) Ar[i][p] = i < ns ? gload(va + (3 * (lo + i) + p) * 64) : zero8;
  };

  // x of the direct tail -> LDS after the two buffers (as the windowed product)
  float* __restrict__ xl = reinterpret_cast<float*>(zl + 2 * CK_UNITS);
  for (int c = wave; c * 64 < NR * tpad; c += 4) {
    const int u = c * 64 + lane;
    const int i = u / tpad, mm = u - i * tpad;
    const float* src = args.X + (int64_t)min(r0 + i, args.R - 1) * args.N + min(mm, args.tail - 1);
    __builtin_amdgcn_global_load_lds(src, xl + c * 64, 4, 0, 0);
  }
  bf16x8 Acur[2][3], Anext[2][3];
  int slo_c = 0, ns_c = 0, slo_n = 0, ns_n = 0;
  if (nch > 0) {
    stage(0);
    load_a(0, Acur, slo_c, ns_c);
  }
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  const int tsteps = has_tile ? (args.tail + 31) / 32 : 0;
  const bf16x8* __restrict__ ta = reinterpret_cast<const bf16x8*>(args.tailmat);
  bf16x8 TA[3];
  auto load_tail = [&](int st) {
#pragma unroll
    for (int p = 0; p < 3; ++p)
      TA[p] = gload(ta + (((int64_t)tile * tsteps + st) * 3 + p) * 64 + lane);
  };
  if (tsteps > 0) load_tail(0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  f32x4 acc[RG];
#pragma unroll
  for (int q = 0; q < RG; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < nch; ++c) {
    // buffer (c + 1) & 1 was last read for chunk c - 1, before the barrier
    if (c + 1 < nch) {
      stage(c + 1);
      load_a(c + 1, Anext, slo_n, ns_n);
    }
    if (ns_c > 0) {
      const int b = block_of(c);
      const int j = c - lane_i32(cstart_l, b);
      const int base = (lane_i32(k0_l, b) - lane_i32(wk0_l, b)) >> 2;
      const int nst = min(CK_G + CK_HALO, lane_i32(ww4_l, b) - CK_G * j);
      const uint4* __restrict__ zb = zl + (c & 1) * CK_UNITS + m * CK_PITCH;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (i < ns_c) {
          // groups past the tile's box (zero matrix pieces) read the chunk's
          // last staged group, a finite value
          const int lg = min(base + 4 * (slo_c + i) + g - CK_G * j, nst - 1);
          bf16x8 Z[RG][3];
#pragma unroll
          for (int q = 0; q < RG; ++q)
#pragma unroll
            for (int p = 0; p < 3; ++p)
              Z[q][p] = __builtin_bit_cast(bf16x8, zb[(p * NR + 16 * q) * CK_PITCH + lg]);
          mma6xg<RG>(Acur[i], Z, acc);
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int p = 0; p < 3; ++p) Acur[i][p] = Anext[i][p];
    slo_c = slo_n;
    ns_c = ns_n;
  }
  if (!has_tile) return;

  // direct tail: x from LDS, split here
  for (int st = 0; st < tsteps; ++st) {
    if (st > 0) load_tail(st);
    bf16x8 B[RG][3];
#pragma unroll
    for (int q = 0; q < RG; ++q) {
      const float4* xq = reinterpret_cast<const float4*>(xl + (16 * q + m) * tpad + 32 * st + 8 * g);
      const float4 lo = xq[0], hi = xq[1];
      const float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      f32x8 xv;
#pragma unroll
      for (int j = 0; j < 8; ++j) xv[j] = 32 * st + 8 * g + j < args.tail ? v[j] : 0.f;
      const Split8 xs(xv);
#pragma unroll
      for (int p = 0; p < 3; ++p) B[q][p] = xs.get(p);
    }
    mma6xg<RG>(TA, B, acc);
  }

  // y: lane (m, g) holds rows 4g .. 4g+3 of right-hand side r0 + 16 q + m
#pragma unroll
  for (int q = 0; q < RG; ++q) {
    const int rhs = r0 + 16 * q + m;
    if (rhs < args.R) {
      float* __restrict__ y = args.Y + (int64_t)rhs * args.N + n0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (n0 + 4 * g + i < args.N) y[4 * g + i] = acc[q][i];
    }
  }
}

// The chunked windows for the float64 matrix-core product (spmm_mfma_kernel's
// steps): workgroup = WIN_TILES row tiles x 64 right-hand sides, wave = one
// tile (four groups of 16 right-hand sides); each chunk of a block's union
// window lands in LDS as complex float64 values, row i for right-hand side
// r0 + i (one 16-byte unit per column).  A tile's steps are taken in the
// per-tile product's order, so the sums are the same bits.
constexpr int CKF_COLS = 4 * (CK_G + CK_HALO);  // columns of a staged chunk
constexpr int CKF_PITCH = CKF_COLS + 1;         // odd row pitch (16-byte units)
constexpr int CKF_UNITS = CK_NR * CKF_PITCH;    // units of one buffer
static_assert(CKF_UNITS % 64 == 0, "chunk buffer layout");

// tile group grp, right-hand sides r0 .. r0 + CK_NR - 1 of one plan
__device__ __forceinline__ void chunk_group_f64(const SpmmArgs<double>& args,
                                                const WinMeta* __restrict__ win, int grp,
                                                int r0) {
  using E = EngF64;
  using C = double2;
  constexpr int NR = CK_NR, RG = NR / 16;
  extern __shared__ __align__(16) C zc[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, g = lane >> 4;
  const int nblk = args.nblk;
  const int tile = grp * WIN_TILES + wave;
  const bool has_tile = tile < args.n_tiles;  // wave-uniform

  int wk0_l = 0, ww4_l = 0, k0_l = 0, kw_l = 0, ldz_l = 0;
  int64_t off_l = 0, val_l = 0, zoff_l = 0;
  if (lane < nblk) {
    const WinMeta wm = win[(int64_t)grp * nblk + lane];
    wk0_l = wm.k0;
    ww4_l = wm.w4;
    const SpmmBlock<double> bd = args.blocks[lane];
    val_l = (int64_t)(uintptr_t)bd.val;
    zoff_l = bd.zoff;
    ldz_l = bd.ldz;
    if (has_tile) {
      const TileMeta tm = args.meta[(int64_t)tile * nblk + lane];
      k0_l = tm.k0;
      kw_l = tm.kw;
      off_l = tm.off;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  int cstart_l = 0, nch = 0;
  for (int bb = 0; bb < nblk; ++bb) {
    if (lane == bb) cstart_l = nch;
    nch += (lane_i32(ww4_l, bb) + CK_G - 1) / CK_G;
  }
  const int cend_l = cstart_l + (lane < nblk ? (ww4_l + CK_G - 1) / CK_G : 0);
  auto block_of = [&](int c) { return (int)__popcll(__ballot(lane < nblk && cend_l <= c)); };

  // chunk c (block b, columns 4 CK_G j .. + ncol - 1 of the window) into
  // buffer c & 1; columns past the window, or past a spectrum row (P + 1
  // values: a window ends on a multiple of 4 columns), repeat the last one,
  // right-hand sides past R the last one
  auto stage = [&](int c) {
    const int b = block_of(c);
    const int j = c - lane_i32(cstart_l, b);
    const int ncol = 4 * min(CK_G + CK_HALO, lane_i32(ww4_l, b) - CK_G * j);
    const int64_t ldz = lane_i32(ldz_l, b);
    const int c0 = lane_i32(wk0_l, b) + 4 * CK_G * j;  // <= P: a chunk starts inside its window
    const int cmax = min(ncol, (int)ldz - c0) - 1;
    const C* __restrict__ zw = args.Z + (int64_t)args.R * lane_i64(zoff_l, b) + c0;
    C* __restrict__ dst = zc + (c & 1) * CKF_UNITS;
    for (int cc = wave; cc * 64 < CKF_UNITS; cc += 4) {
      const int u = cc * 64 + lane;
      const int row = u / CKF_PITCH, col = min(u - row * CKF_PITCH, cmax);
      const int64_t rhs = min(r0 + row, args.R - 1);
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const char*>(zw + rhs * ldz + col),
                                       dst + cc * 64, 16, 0, 0);
    }
  };
  // the tile's steps in chunk c (at most 2) and their matrix values: step s
  // covers box columns 16 s .. 16 s + 15, lane (m, g) column 16 s + 4 g + j of row m
  auto load_a = [&](int c, C (*Ar)[4], int& s_lo, int& ns) {
    const int b = block_of(c);
    const int j = c - lane_i32(cstart_l, b);
    const int base = (lane_i32(k0_l, b) - lane_i32(wk0_l, b)) >> 2;
    const int kw = lane_i32(kw_l, b);
    const int S = (kw + 15) >> 4;
    const int lo = max(0, (CK_G * j - base + 3) >> 2);
    const int hi = min(S, (CK_G * j + CK_G - base + 3) >> 2);
    s_lo = lo;
    ns = has_tile ? max(0, hi - lo) : 0;
    const C* __restrict__ val = (const C*)(uintptr_t)lane_i64(val_l, b) + lane_i64(off_l, b);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int col = 16 * (lo + i) + 4 * g + jj;
        Ar[i][jj] = (i < ns && col < kw) ? gload(val + (int64_t)col * TILE_ROWS + m) : C{0.0, 0.0};
      }
  };

  C Acur[2][4], Anext[2][4];
  int slo_c = 0, ns_c = 0, slo_n = 0, ns_n = 0;
  if (nch > 0) {
    stage(0);
    load_a(0, Acur, slo_c, ns_c);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  typename E::Acc acc[RG];
#pragma unroll
  for (int q = 0; q < RG; ++q) acc[q] = E::zero();
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) {
      stage(c + 1);
      load_a(c + 1, Anext, slo_n, ns_n);
    }
    if (ns_c > 0) {
      const int b = block_of(c);
      const int j = c - lane_i32(cstart_l, b);
      const int base = (lane_i32(k0_l, b) - lane_i32(wk0_l, b)) >> 2;
      const int ncol = 4 * min(CK_G + CK_HALO, lane_i32(ww4_l, b) - CK_G * j);
      const C* __restrict__ zb = zc + (c & 1) * CKF_UNITS + m * CKF_PITCH;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (i < ns_c) {
#pragma unroll
          for (int q = 0; q < RG; ++q) {
            C z[4];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              // columns past the tile's box (zero matrix values) may read
              // the chunk's last staged column, a finite value
              const int lc = min(4 * (base + 4 * (slo_c + i) - CK_G * j) + 4 * g + jj, ncol - 1);
              z[jj] = zb[16 * q * CKF_PITCH + lc];
            }
            acc[q] = E::step(Acur[i], z, acc[q]);
          }
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) Acur[i][jj] = Anext[i][jj];
    slo_c = slo_n;
    ns_c = ns_n;
  }
  if (!has_tile) return;

  // direct tail (as spmm_mfma_kernel, per group of 16 right-hand sides)
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  const int64_t ldt = (int64_t)args.n_tiles * TILE_ROWS;
#pragma unroll
  for (int q = 0; q < RG; ++q) {
    const int r = r0 + 16 * q + m;
    const bool rok = r < args.R;
    const int64_t rr = rok ? r : r0 + 16 * q;
    const bool qok = r0 + 16 * q < args.R;  // wave-uniform
    if (!qok) continue;
    const double* __restrict__ xr = args.X + rr * args.N;  // rr < R (qok)
    for (int ks = 0; ks < args.tail; ks += 32) {
      double av[8], xv[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int mm = ks + 8 * g + jj;
        const bool ok = mm < args.tail;
        av[jj] = ok ? args.tailmat[(int64_t)mm * ldt + n0 + m] : 0.0;
        xv[jj] = (ok && rok) ? xr[mm] : 0.0;
      }
      acc[q] = E::step_real(av, xv, acc[q]);
    }
    if (rok) {
      double* __restrict__ y = args.Y + (int64_t)r * args.N + n0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = E::row(g, i);
        if (n0 + row < args.N) y[row] = acc[q][i];
      }
    }
  }
}

__global__ __launch_bounds__(256) void spmm_chunk_f64_kernel(SpmmArgs<double> args,
                                                             const WinMeta* __restrict__ win,
                                                             int n_groups) {
  chunk_group_f64(args, win, xcd_tile(blockIdx.x, n_groups), blockIdx.y * CK_NR);
}

// Several plans in one launch: workgroup b takes item b = (plan, group, r0)
__global__ __launch_bounds__(256) void spmm_chunk_f64_items_kernel(SpmmBatch<double> b) {
  const int4 it = b.items[blockIdx.x];
  if (it.y < 0) return;
  SpmmArgs<double> a = b.plans[it.x];
  a.X = b.X[it.x];
  a.Y = b.Y[it.x];
  chunk_group_f64(a, a.win, it.y, it.z);
}

__global__ __launch_bounds__(256) void spmm_chunk_kernel(SpmmSplitArgs args,
                                                         const WinMeta* __restrict__ win,
                                                         int n_groups, int tpad) {
  chunk_group(args, win, xcd_tile(blockIdx.x, n_groups), blockIdx.y * CK_NR, tpad);
}

// Several plans in one launch: workgroup b takes item b = (plan, group, r0)
__global__ __launch_bounds__(256) void spmm_chunk_items_kernel(SpmmSplitBatch b) {
  const int4 it = b.items[blockIdx.x];
  if (it.y < 0) return;
  SpmmSplitArgs a = b.plans[it.x];
  a.X = b.X[it.x];
  a.Y = b.Y[it.x];
  chunk_group(a, a.win, it.y, it.z, a.tpad);
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
// u[r][k] = c'_k sum_n Add[n][k] f[r][n] over the half spectrum (c'_k = 1 at
// k = 0 and P, else 1/2: the c_k folded into the stored values taken out).
// By columns: the row tiles whose boxes meet the columns [TCHUNK c, TCHUNK c +
// TCHUNK) of a block are listed at precompute and split into segments (TSEG
// tiles, longer on nearly dense plans, whose partial sums would otherwise
// outgrow the workspace); one launch takes the segments of every block.  The
// list entries are staged 256 at a time.  Workgroup
// (s, g) takes segment s for the right-hand sides 64 g .. 64 g + 63, staging
// the tiles' f values (64 x 16) and box columns (16 x TCHUNK) in LDS two tiles
// at a time (the next two are requested before the current ones are used).
// The only segment of a chunk stores its sums in u; when there are several (a
// short block's few columns gather thousands of tiles, spread over many
// workgroups) each stores into a slot of partial sums, and
// spmm_t_reduce_kernel adds a chunk's slots in order (deterministic, no
// atomics).  Thread: columns 2 cg, 2 cg + 1 and right-hand sides 4 rq ..
// 4 rq + 3 of the chunk.  The tiles' sums are added in float64 for either
// precision (rounded to the working precision once, where they are stored);
// a tile's 16 rows are summed in the working precision, or in float64 (PD:
// float32 plans whose spectra-side arithmetic runs in float64,
// spt_params.reduced_fft).
template <typename T, bool PD>
__global__ __launch_bounds__(256) void spmm_transposed_kernel(SpmmTArgs<T> a) {
  using C = cplx_t<T>;
  using D = double2;
  using PT = typename std::conditional<PD, double, T>::type;  // a tile's sums
  using PC = cplx_t<PT>;
  static_assert(TCHUNK == 32, "thread layout: 16 column pairs x 16 groups of 4 right-hand sides");
  constexpr int FPT = 64 * TILE_ROWS / 256;      // f values per thread and tile
  constexpr int APT = TILE_ROWS * TCHUNK / 256;  // box values per thread and tile
  constexpr int EB = 256;                        // list entries staged at a time
  constexpr int TPR = 2;                         // tiles staged per round
  __shared__ T fs[TPR][64][TILE_ROWS + 1];
  __shared__ C as[TPR][TILE_ROWS][TCHUNK];
  __shared__ TChunkEnt ents[EB];
  const int tid = threadIdx.x;
  const int4 seg = a.segs[blockIdx.x];
  const TBlkInfo bi = a.blk[(seg.w >> 1) & ((1 << TSEG_BLOCK_BITS) - 1)];
  const C* __restrict__ vals = static_cast<const C*>(sizeof(T) == 8 ? bi.val64 : bi.val32);
  const int P = bi.P;
  const int64_t ldu = P + 1;
  C* __restrict__ u = a.u + bi.uoff * a.R;
  const int r0 = blockIdx.y * 64;
  const int kc = seg.x * TCHUNK;
  const int cg = tid & 15, rq = tid >> 4;
  D acc[4][2];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j][0] = acc[j][1] = D{0.0, 0.0};
  T fr[TPR][FPT];
  C ar[TPR][APT];
  auto fetch = [&](int t, const TChunkEnt& e) {
    const int64_t n0 = (int64_t)e.tile * TILE_ROWS;
#pragma unroll
    for (int i = 0; i < FPT; ++i) {
      const int idx = tid + i * 256, r = r0 + (idx >> 4);
      const int64_t n = n0 + (idx & 15);
      fr[t][i] = (r < a.R && n < a.N) ? gload(a.F + (int64_t)r * a.N + n) : T(0);
    }
    const C* __restrict__ val = vals + e.off;
#pragma unroll
    for (int i = 0; i < APT; ++i) {
      const int idx = tid + i * 256;
      const int kk = kc + (idx >> 4) - e.k0;
      ar[t][i] = (kk >= 0 && kk < e.kw) ? gload(val + (int64_t)kk * TILE_ROWS + (idx & 15))
                                        : C{T(0), T(0)};
    }
  };
  auto fetch_round = [&](int i0, int nb) {
#pragma unroll
    for (int t = 0; t < TPR; ++t)
      if (i0 + t < nb) fetch(t, ents[i0 + t]);
  };
  const int e_begin = seg.y, e_end = seg.z;
  for (int b0 = e_begin; b0 < e_end; b0 += EB) {
    const int nb = min(EB, e_end - b0);
    __syncthreads();
    if (tid < nb) ents[tid] = a.ents[b0 + tid];
    __syncthreads();
    fetch_round(0, nb);
    for (int i0 = 0; i0 < nb; i0 += TPR) {
      const int cnt = min(TPR, nb - i0);
      __syncthreads();
#pragma unroll
      for (int t = 0; t < TPR; ++t) {
        if (t >= cnt) break;
#pragma unroll
        for (int j = 0; j < FPT; ++j) {
          const int idx = tid + j * 256;
          fs[t][idx >> 4][idx & 15] = fr[t][j];
        }
#pragma unroll
        for (int j = 0; j < APT; ++j) {
          const int idx = tid + j * 256;
          as[t][idx & 15][idx >> 4] = ar[t][j];
        }
      }
      __syncthreads();
      if (i0 + TPR < nb) fetch_round(i0 + TPR, nb);
#pragma unroll
      for (int t = 0; t < TPR; ++t) {
        if (t >= cnt) break;
        // the tile's 16 rows summed first, then added (running sums stay short)
        PC part[4][2];
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j][0] = part[j][1] = PC{PT(0), PT(0)};
#pragma unroll
        for (int q = 0; q < TILE_ROWS; ++q) {
          const C a0 = as[t][q][2 * cg], a1 = as[t][q][2 * cg + 1];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const PT fv = fs[t][4 * rq + j][q];
            part[j][0].x += PT(a0.x) * fv;
            part[j][0].y += PT(a0.y) * fv;
            part[j][1].x += PT(a1.x) * fv;
            part[j][1].y += PT(a1.y) * fv;
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int c2 = 0; c2 < 2; ++c2) {
            acc[j][c2].x += part[j][c2].x;
            acc[j][c2].y += part[j][c2].y;
          }
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = r0 + 4 * rq + j;
    if (r >= a.R) continue;
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
      const int k = kc + 2 * cg + c2;
      if (k > P) continue;
      const double ck = (k == 0 || k == P) ? 1.0 : 0.5;
      const C v = C{T(acc[j][c2].x * ck), T(acc[j][c2].y * ck)};
      if (seg.w & 1)
        u[(int64_t)r * ldu + k] = v;
      else
        a.part[((int64_t)(seg.w >> (TSEG_BLOCK_BITS + 1)) * a.R + r) * TCHUNK + 2 * cg + c2] = v;
    }
  }
}

// u of the chunks with several segments (and zeros for chunks no tile meets):
// workgroup (i, g) adds the slots of chunk red[i] in order for the right-hand
// sides 8 g .. 8 g + 7, one value per thread, eight slots requested at a time
template <typename T>
__global__ __launch_bounds__(256) void spmm_t_reduce_kernel(SpmmTArgs<T> a) {
  using C = cplx_t<T>;
  static_assert(TCHUNK == 32, "256 threads: 8 right-hand sides x 32 columns");
  const int4 rd = a.red[blockIdx.x];
  const TBlkInfo bi = a.blk[rd.x];
  const int P = bi.P;
  const int r = blockIdx.y * 8 + (threadIdx.x >> 5), c = threadIdx.x & 31, k = rd.y * TCHUNK + c;
  if (r >= a.R || k > P) return;
  const int64_t stride = (int64_t)a.R * TCHUNK;
  const C* __restrict__ p = a.part + ((int64_t)rd.z * a.R + r) * TCHUNK + c;
  double2 s = double2{0.0, 0.0};  // float64 sums, as in spmm_transposed_kernel
  int i = 0;
  for (; i + 8 <= rd.w; i += 8) {
    C v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = p[(int64_t)(i + j) * stride];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      s.x += v[j].x;
      s.y += v[j].y;
    }
  }
  for (; i < rd.w; ++i) {
    const C v = p[(int64_t)i * stride];
    s.x += v.x;
    s.y += v.y;
  }
  a.u[bi.uoff * a.R + (int64_t)r * (P + 1) + k] = C{T(s.x), T(s.y)};
}

// fhat[r][m] = sum_j tail[m][j] f[r][j] for m < tail: one workgroup per (m, r)
template <typename T>
__global__ __launch_bounds__(256) void tail_transposed_kernel(const T* __restrict__ tailmat,
                                                              int64_t ldt, const T* __restrict__ F,
                                                              T* __restrict__ Y, int64_t N) {
  const int m = blockIdx.x, r = blockIdx.y;
  const T* __restrict__ col = tailmat + (int64_t)m * ldt;
  const T* __restrict__ f = F + (int64_t)r * N;
  // eight loads of each in flight per thread (blockDim.x is 256); sums in
  // float64 for either precision, rounded once when stored
  double s = 0.0;
  int64_t j = threadIdx.x;
  for (; j + 7 * 256 < N; j += 8 * 256) {
    T cv[8], fv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      cv[u] = col[j + u * 256];
      fv[u] = f[j + u * 256];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (double)cv[u] * fv[u];
  }
  for (; j < N; j += 256) s += (double)col[j] * f[j];
  __shared__ double part[256];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) Y[(int64_t)r * N + m] = T(part[0]);
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

void launch_spmm_chunk_items(const SpmmSplitBatch& b, int n_items, size_t lds, hipStream_t s) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(spmm_chunk_items_kernel, dim3(n_items), dim3(256), lds, s, b);
  SPT_HIP(hipGetLastError());
}

void launch_spmm_chunk_f64_items(const SpmmBatch<double>& b, int n_items, hipStream_t s) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(spmm_chunk_f64_items_kernel, dim3(n_items), dim3(256),
                     (size_t)2 * CKF_UNITS * sizeof(double2), s, b);
  SPT_HIP(hipGetLastError());
}

void launch_spmm_chunk_f64(const SpmmArgs<double>& a, const WinMeta* win, int n_groups,
                           hipStream_t s) {
  hipLaunchKernelGGL(spmm_chunk_f64_kernel, dim3(n_groups, (a.R + CK_NR - 1) / CK_NR), dim3(256),
                     (size_t)2 * CKF_UNITS * sizeof(double2), s, a, win, n_groups);
  SPT_HIP(hipGetLastError());
}

size_t spmm_chunk_lds_bytes(int tpad) {
  return (size_t)2 * CK_UNITS * 16 + (size_t)CK_NR * tpad * sizeof(float);
}

void launch_spmm_chunk(const SpmmSplitArgs& a, const WinMeta* win, int n_groups, int tpad,
                       hipStream_t s) {
  hipLaunchKernelGGL(spmm_chunk_kernel, dim3(n_groups, (a.R + CK_NR - 1) / CK_NR), dim3(256),
                     spmm_chunk_lds_bytes(tpad), s, a, win, n_groups, tpad);
  SPT_HIP(hipGetLastError());
}

void launch_spmm_window(const SpmmSplitArgs& a, const WinMeta* win, int n_groups, int rg,
                        int waves, int xlds, int tpad, size_t lds_bytes, hipStream_t s) {
  if (rg == 4 && waves == 2)
    hipLaunchKernelGGL((spmm_window_kernel<2, 2>), dim3(n_groups, (a.R + 63) / 64), dim3(512),
                       lds_bytes, s, a, win, n_groups, xlds, tpad);
  else if (rg == 4)
    hipLaunchKernelGGL((spmm_window_kernel<4, 1>), dim3(n_groups, (a.R + 63) / 64), dim3(256),
                       lds_bytes, s, a, win, n_groups, xlds, tpad);
  else
    hipLaunchKernelGGL((spmm_window_kernel<2, 1>), dim3(n_groups, (a.R + 31) / 32), dim3(256),
                       lds_bytes, s, a, win, n_groups, xlds, tpad);
  SPT_HIP(hipGetLastError());
}

// Allow the windowed product the whole LDS of a workgroup (once per device).
void init_spmm_kernels(size_t max_lds) {
  static std::vector<int> done;
  int dev = 0;
  SPT_HIP(hipGetDevice(&dev));
  for (int d : done)
    if (d == dev) return;
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(spmm_window_kernel<4, 1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds));
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(spmm_window_kernel<2, 1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds));
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(spmm_window_kernel<2, 2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds));
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(spmm_chunk_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds));
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(spmm_chunk_items_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds));
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(spmm_chunk_f64_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds));
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(spmm_chunk_f64_items_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds));
  done.push_back(dev);
}

void launch_spmm_split_bf16(const SpmmArgs<float>& a, hipStream_t s) {
  hipLaunchKernelGGL(spmm_mfma_kernel<EngSplitBf16>, dim3(a.n_tiles, (a.R + 63) / 64),
                     dim3(256), 0, s, a);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_spmm_transposed(const SpmmTArgs<T>& a, bool products64, hipStream_t s) {
  if (a.R > 65535 * 8) throw Error(SPT_E_INVALID_ARG, "too many right-hand sides");
  if (a.n_segs <= 0) return;
  if (products64 && !std::is_same<T, double>::value)
    hipLaunchKernelGGL((spmm_transposed_kernel<T, true>), dim3(a.n_segs, (a.R + 63) / 64),
                       dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((spmm_transposed_kernel<T, false>), dim3(a.n_segs, (a.R + 63) / 64),
                       dim3(256), 0, s, a);
  SPT_HIP(hipGetLastError());
  if (a.n_red <= 0) return;
  hipLaunchKernelGGL(spmm_t_reduce_kernel<T>, dim3(a.n_red, (a.R + 7) / 8), dim3(256), 0, s, a);
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
template void launch_spmm_transposed<double>(const SpmmTArgs<double>&, bool, hipStream_t);
template void launch_spmm_transposed<float>(const SpmmTArgs<float>&, bool, hipStream_t);
template void launch_tail_transposed<double>(const double*, int, const double*, double*, int,
                                             int64_t, hipStream_t);
template void launch_tail_transposed<float>(const float*, int, const float*, float*, int,
                                            int64_t, hipStream_t);

}  // namespace spt
