// Persistent executor kernel: the work items described in exec.hpp.

#include <type_traits>

#include "exec.hpp"
#include "fft_core.hpp"
#include "spmm_core.hpp"

namespace spt {
namespace {

using namespace fftcore;
using namespace spmmcore;

// a wait gives up after sync[EXEC_SYNC_WAIT] ticks of the 100 MHz wall clock
// (1 s unless the host set another bound) or once another wait of the launch
// has given up; what the waiting item writes is then NaN

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// wait until *p >= target (wave-uniform result); false when the wait gave up
__device__ bool wait_count(uint32_t* sync, const uint32_t* p, uint32_t target) {
  if (__builtin_amdgcn_readfirstlane(ld_relaxed(p)) >= target) return true;
  const uint64_t t0 = wall_clock64();
  const uint64_t limit = __builtin_amdgcn_readfirstlane(ld_relaxed(sync + EXEC_SYNC_WAIT));
  for (int it = 1;; ++it) {
    __builtin_amdgcn_s_sleep(2);
    if (__builtin_amdgcn_readfirstlane(ld_relaxed(p)) >= target) return true;
    if ((it & 7) == 0) {
      if (__builtin_amdgcn_readfirstlane(ld_relaxed(sync + EXEC_SYNC_ERR)) != 0) return false;
      if (wall_clock64() - t0 > limit) {
        __hip_atomic_store(sync + EXEC_SYNC_ERR, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
}

__device__ __forceinline__ void acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Publication by a workgroup: every wave waits for its own memory operations
// (its global stores have then reached the L2 of its XCD), a barrier, and one
// agent-scope release by thread 0 (which writes the L2 back for the other
// XCDs) before the counter update.  The cache-wide write-back then happens
// once per item instead of once per wave.
__device__ __forceinline__ void publish_prologue() {
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
}

// Workgroup-wide wait: thread 0 polls, acquires for the workgroup (the
// invalidation covers the CU's vector cache and the XCD's L2), and a barrier
// releases the other waves.  Returns false (for every thread) when the wait
// gave up.
__device__ __forceinline__ bool wg_wait(uint32_t* sync, const uint32_t* p, uint32_t target,
                                        int* s_flag) {
  if (threadIdx.x < 64) {
    const bool ok = wait_count(sync, p, target);
    if (threadIdx.x == 0) {
      acquire();
      *s_flag = ok;
    }
  }
  __syncthreads();
  const bool ok = *s_flag != 0;
  __syncthreads();  // s_flag is reused by the next wait
  return ok;
}

__device__ __forceinline__ uint32_t udiv(uint32_t u, uint32_t magic) {
  return __umulhi(u, magic);
}

// all threads: publish this workgroup's global writes, then thread 0 adds n
__device__ __forceinline__ void signal(uint32_t* p, uint32_t n) {
  publish_prologue();
  if (threadIdx.x == 0 && n) __hip_atomic_fetch_add(p, n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int SIGN = +1, typename C, typename T>
__device__ __forceinline__ C unpack_pair(C ck, C cm, C t, T scale) {
  // Z_k = E_k + exp(SIGN i pi k/P) O_k, E = (C_k + conj C_{P-k})/2,
  // O = (C_k - conj C_{P-k})/(2i); t = exp(+i pi k/P)
  if (SIGN < 0) t.y = -t.y;
  cm.y = -cm.y;
  const C e = C{T(0.5) * (ck.x + cm.x), T(0.5) * (ck.y + cm.y)};
  const C d = C{T(0.5) * (ck.x - cm.x), T(0.5) * (ck.y - cm.y)};
  const C o = C{d.y, -d.x};
  const C z = cadd(e, cmul(t, o));
  return C{z.x * scale, z.y * scale};
}

template <typename T>
__device__ __forceinline__ T nan_of() {
  return __builtin_nan("");
}

// copy the block's twiddle tables into LDS (read back after the next barrier)
template <typename T>
__device__ __forceinline__ void load_tables(const ExecBlock<T>& B, double2* ltw, bool post) {
  for (int i = threadIdx.x; i < B.ntw; i += EXEC_THREADS) {
    ltw[i] = B.tw[i];
    if (post) ltw[B.ntw + i] = B.tw2[i];
  }
}

// ------------------------------------------------------------------ ITEM_FFT
// 2^lb right-hand sides r0 .. of one block; point j of rhs r0 + t at
// lds[(j << lb) + t]
// the half-spectrum value k of rhs r: complex, or its three bfloat16 pieces
template <bool SPLIT, typename T, typename C>
__device__ __forceinline__ void store_z(const ExecPlan<T>& pl, const ExecBlock<T>& B, int r, int k,
                                        C z) {
  if constexpr (SPLIT) {
    uint32_t pc[3];
    split2(f32x2{(float)z.x, (float)z.y}, pc);
    uint32_t* zs = pl.Zs + (int64_t)pl.R * B.zoff4 + (int64_t)r * B.ldz4 + k;
#pragma unroll
    for (int p = 0; p < 3; ++p) zs[p * pl.zplane] = pc[p];
  } else {
    const int64_t i = (int64_t)pl.R * B.zoff + (int64_t)r * (B.P + 1) + k;
    if (pl.Zf)
      pl.Zf[i] = float2{(float)z.x, (float)z.y};
    else
      pl.Z[i] = z;
  }
}

// pre-split spectra are zero past P up to the row length ldz4
template <bool SPLIT, typename T>
__device__ __forceinline__ void store_z_pad(const ExecPlan<T>& pl, const ExecBlock<T>& B, int r) {
  if constexpr (SPLIT)
    for (int k = B.P + 1; k < B.ldz4; ++k) store_z<true>(pl, B, r, k, cplx_t<T>{T(0), T(0)});
}

template <typename T, bool SYNC, bool SPLIT, typename TI = T>
__device__ __forceinline__ void item_fft(const ExecPlan<T>& pl, const ExecBlock<T>& B, const TI* __restrict__ X,
                         int r0, int lb, cplx_t<T>* lds, double2* ltw, uint32_t* sync) {
  using C = cplx_t<T>;
  const int tid = threadIdx.x;
  load_tables(B, ltw, true);
  const int P = B.P, nt = 1 << lb;
  const uint32_t total = (uint32_t)P << lb;
  const int R = pl.R;
  const int64_t N = pl.N;
  const int c_lo = B.c_lo, c_hi = B.c_hi, m_off = B.m_off;
  const T* __restrict__ winv = B.winv;
  {
    T v0[EXEC_EPT], v1[EXEC_EPT];
#pragma unroll
    for (int e = 0; e < EXEC_EPT; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;
      const int t = (int)udiv(u, B.magic), j = (int)u - t * P;
      const int r = r0 + t;
      const bool ok = u < total && r < R;
      const int c0 = 2 * j, c1 = 2 * j + 1;
      const TI* __restrict__ x = X + (int64_t)r * N + m_off;
      v0[e] = (ok && c0 >= c_lo && c0 < c_hi) ? T(x[c0]) * winv[c0] : T(0);
      v1[e] = (ok && c1 >= c_lo && c1 < c_hi) ? T(x[c1]) * winv[c1] : T(0);
    }
#pragma unroll
    for (int e = 0; e < EXEC_EPT; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;
      const int t = (int)udiv(u, B.magic), j = (int)u - t * P;
      if (u < total) lds[(j << lb) + t] = C{v0[e], v1[e]};
    }
  }
  __syncthreads();
  run_fft<+1, true, EXEC_EPT>(lds, P, lb, B.f1.npass, B.f1.radix, ltw, 1, tid, EXEC_THREADS,
                              true);
  // half spectra, k = 0 .. P of every rhs (u = t * (P + 1) + k)
  const uint32_t total1 = (uint32_t)(P + 1) << lb;
  {
    constexpr int NE = EXEC_EPT + 1;  // (P + 1) 2^lb <= EXEC_POINTS + 64
    C tw[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;
      const int t = (int)udiv(u, B.magic1), k = (int)u - t * (P + 1);
      tw[e] = u < total1 ? to_c<C>(twiddle(ltw + B.ntw, k)) : C{T(0), T(0)};
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;
      const int t = (int)udiv(u, B.magic1), k = (int)u - t * (P + 1);
      const int r = r0 + t;
      if (u < total1 && r < R) {
        const C ck = lds[((k == P ? 0 : k) << lb) + t];
        const C cm = lds[((k == 0 ? 0 : P - k) << lb) + t];
        store_z<SPLIT>(pl, B, r, k, unpack_pair(ck, cm, tw[e], B.scale));
      }
    }
  }
  if (SPLIT && tid < nt && r0 + tid < R) store_z_pad<SPLIT>(pl, B, r0 + tid);
  if (!SYNC) return;
  // one count per complete rhs, per group of 16
  publish_prologue();
  if (tid == 0) {
    const int r1 = min(r0 + nt, R);
    for (int g = r0 >> 4; g <= (r1 - 1) >> 4; ++g) {
      const int n = min(r1, 16 * g + 16) - max(r0, 16 * g);
      __hip_atomic_fetch_add(sync + B.ctr + g, (uint32_t)n, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ------------------------------------------------------------------ ITEM_COL
// u[n] = v[2n] + i v[2n+1], n = P2 n1 + n2.  Columns n2 = grp * 2^lcw + t:
// point n1 of column t at lds[(n1 << lcw) + t] (that is lds[u] for the
// load order u = (n1 << lcw) + t), length-P1 transforms, then
// W[k1 * P2 + n2] = (sum_n1 u[P2 n1 + n2] w_P1^(n1 k1)) w_P^(n2 k1).
// SIGN -1 (the precomputation's F): rows of X are taken as they are
// (B.winv == nullptr, no window division, no extras)
template <typename T, bool SYNC, int SIGN = +1, typename TI = T>
__device__ __forceinline__ void item_col(const ExecPlan<T>& pl, const ExecBlock<T>& B, const TI* __restrict__ X,
                         int r, int grp, cplx_t<T>* lds, double2* ltw, uint32_t* sync) {
  using C = cplx_t<T>;
  const int tid = threadIdx.x;
  load_tables(B, ltw, false);
  const int lcw = B.lcw, cw = 1 << lcw;
  const int P1 = B.P1, P2 = B.P2;
  const uint32_t total = (uint32_t)P1 << lcw;
  const int c_lo = B.c_lo, c_hi = B.c_hi;
  const TI* __restrict__ x = X + (int64_t)r * pl.N + B.m_off;
  const T* __restrict__ winv = B.winv;
  const int n2base = grp << lcw;
  {
    T v0[EXEC_EPT], v1[EXEC_EPT];
#pragma unroll
    for (int e = 0; e < EXEC_EPT; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;
      const int t = (int)u & (cw - 1), n1 = (int)(u >> lcw);
      const int n = n1 * P2 + n2base + t;
      const int c0 = 2 * n, c1 = 2 * n + 1;
      const bool ok = u < total;
      if (SIGN > 0) {
        v0[e] = (ok && c0 >= c_lo && c0 < c_hi) ? T(x[c0]) * winv[c0] : T(0);
        v1[e] = (ok && c1 >= c_lo && c1 < c_hi) ? T(x[c1]) * winv[c1] : T(0);
      } else {
        v0[e] = ok ? T(x[c0]) : T(0);
        v1[e] = ok ? T(x[c1]) : T(0);
      }
    }
#pragma unroll
    for (int e = 0; e < EXEC_EPT; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;
      if (u < total) lds[u] = C{v0[e], v1[e]};
    }
  }
  __syncthreads();
  run_fft<SIGN, true, EXEC_EPT>(lds, P1, lcw, B.f1.npass, B.f1.radix, ltw, P2, tid, EXEC_THREADS,
                                true);
  C* __restrict__ W = pl.W + (int64_t)pl.R * B.woff + (int64_t)r * B.P;
#pragma unroll
  for (int e = 0; e < EXEC_EPT; ++e) {
    const uint32_t u = tid + e * EXEC_THREADS;
    if (u < total) {
      const int t = (int)u & (cw - 1), k1 = (int)(u >> lcw);
      const int n2 = n2base + t;
      double2 w64 = twiddle(ltw, n2 * k1);
      if (SIGN < 0) w64.y = -w64.y;
      const C w = to_c<C>(w64);
      W[(int64_t)k1 * P2 + n2] = cmul(lds[u], w);
    }
  }
  if (SYNC) signal(sync + B.cctr + r, 1);
}

// ------------------------------------------------------------------ ITEM_ROW
// Row pairs j = grp * 2^lgp + i, i < 2^lgp: slot 2i holds row k1 = j, slot
// 2i + 1 row (P1 - j) mod P1 (the same row for j = 0 and j = P1 / 2); point k2
// of slot s at lds[(k2 << ls) + s], ls = lgp + 1.  After the length-P2
// transforms slot s, point k2 is U_k, k = k1 + P1 k2, and its partner
// U_{P-k} sits in the other slot of the pair at P2 - 1 - k2 (k1 > 0) or in the
// same slot at (P2 - k2) mod P2 (k1 = 0).
template <typename T, bool SYNC, bool SPLIT, int SIGN = +1>
__device__ __forceinline__ void item_row(const ExecPlan<T>& pl, const ExecBlock<T>& B, int r, int grp,
                         cplx_t<T>* lds, double2* ltw, uint32_t* sync, int* s_flag) {
  using C = cplx_t<T>;
  const int tid = threadIdx.x;
  load_tables(B, ltw, true);
  const int P = B.P, P1 = B.P1, P2 = B.P2;
  const int ls = B.lgp + 1, ns = 1 << ls;
  const int npairs = P1 / 2 + 1;
  const int j0 = grp << B.lgp;
  const bool ok = SYNC ? wg_wait(sync, sync + B.cctr + r, (uint32_t)B.n_col, s_flag) : true;
  const uint32_t total = (uint32_t)P2 << ls;
  const C* __restrict__ W = pl.W + (int64_t)pl.R * B.woff + (int64_t)r * P;
  auto row_of = [&](int s, bool& valid) {
    const int j = j0 + (s >> 1);
    valid = j < npairs;
    return (s & 1) ? (P1 - j) % P1 : j;
  };
  {
    C v[EXEC_EPT];
#pragma unroll
    for (int e = 0; e < EXEC_EPT; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;  // u = s * P2 + k2: rows read in order
      const int s = (int)udiv(u, B.magic2), k2 = (int)u - s * P2;
      bool valid;
      const int k1 = row_of(s, valid);
      v[e] = (u < total && valid) ? W[(int64_t)k1 * P2 + k2] : C{T(0), T(0)};
    }
#pragma unroll
    for (int e = 0; e < EXEC_EPT; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;
      const int s = (int)udiv(u, B.magic2), k2 = (int)u - s * P2;
      if (u < total) lds[(k2 << ls) + s] = v[e];
    }
  }
  __syncthreads();
  run_fft<SIGN, true, EXEC_EPT>(lds, P2, ls, B.f2.npass, B.f2.radix, ltw, P1, tid, EXEC_THREADS,
                                true);
  const T nanv = nan_of<T>();
  {
    C tw[EXEC_EPT];
    int kk[EXEC_EPT];
#pragma unroll
    for (int e = 0; e < EXEC_EPT; ++e) {
      const uint32_t u = tid + e * EXEC_THREADS;  // u = (k2 << ls) + s
      const int s = (int)u & (ns - 1), k2 = (int)(u >> ls);
      bool valid;
      const int k1 = row_of(s, valid);
      bool own = u < total && valid;
      if (s & 1) {
        bool v2;
        own = own && k1 != row_of(s - 1, v2);  // a self-paired row is written by its even slot
      }
      kk[e] = own ? k1 + P1 * k2 : -1;
      tw[e] = own ? to_c<C>(twiddle(ltw + B.ntw, kk[e])) : C{T(0), T(0)};
    }
#pragma unroll
    for (int e = 0; e < EXEC_EPT; ++e) {
      if (kk[e] >= 0) {
        const uint32_t u = tid + e * EXEC_THREADS;
        const int s = (int)u & (ns - 1), k2 = (int)(u >> ls);
        const int k1 = kk[e] - P1 * k2;
        const C ck = lds[u];
        const C cm = k1 == 0 ? lds[(((P2 - k2) % P2) << ls) + s]
                             : lds[((P2 - 1 - k2) << ls) + (s ^ 1)];
        C z = unpack_pair<SIGN>(ck, cm, tw[e], B.scale);
        if (!ok) z = C{nanv, nanv};
        store_z<SPLIT>(pl, B, r, kk[e], z);
      }
    }
  }
  if (grp == 0 && tid == 0) {  // k = P: C_P = C_0
    const C c0 = lds[0];
    C z = unpack_pair<SIGN>(c0, c0, to_c<C>(twiddle(ltw + B.ntw, P)), B.scale);
    if (!ok) z = C{nanv, nanv};
    store_z<SPLIT>(pl, B, r, P, z);
    store_z_pad<SPLIT>(pl, B, r);
  }
  if (SYNC) signal(sync + B.ctr + (r >> 4), 1);
}

// ------------------------------------------------------------------ ITEM_SPMM
// Tiles tile0, tile0 + 1 x 64 right-hand sides; wave w: tile tile0 + w / 4,
// right-hand sides r0 + 16 (w % 4) ..
template <typename E>
__device__ __forceinline__ void item_spmm(const ExecPlan<typename E::T>& pl, const typename E::T* __restrict__ X,
                          typename E::T* __restrict__ Y, int tile0, int r0, uint32_t* sync,
                          int* s_flag) {
  using T = typename E::T;
  using C = cplx_t<T>;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int R = pl.R;
  const int tile = tile0 + (wave >> 2);
  const int r_wave = r0 + (wave & 3) * 16;
  // waves without work still take part in the workgroup's waits
  const bool active = r_wave < R && tile < pl.n_tiles;
  const int g0 = r0 >> 4, g1 = (min(r0 + 64, R) - 1) >> 4;  // rhs groups of the item
  const int m = lane & 15, g = lane >> 4;
  const int r = r_wave + m;
  const bool rok = r < R;
  const int64_t rr = rok ? r : r_wave;
  const int nblk = pl.nblk;

  // lane b < nblk holds the tile box and descriptor fields of block b
  int k0_l = 0, kw_l = 0, ldz_l = 0, ctr_l = 0, parts_l = 0;
  int64_t off_l = 0, val_l = 0, zoff_l = 0;
  if (lane < nblk) {
    const TileMeta tm = active ? pl.meta[(int64_t)tile * nblk + lane] : TileMeta{0, 0, 0};
    const ExecBlock<T>& bd = pl.blocks[lane];
    k0_l = tm.k0;
    kw_l = tm.kw;
    off_l = tm.off;
    val_l = (int64_t)(uintptr_t)bd.val;
    zoff_l = bd.zoff;
    ldz_l = bd.P + 1;
    ctr_l = bd.ctr;
    parts_l = bd.parts;
  }

  typename E::Acc acc = E::zero();
  // direct tail: A'[q][m'] = tail[m'][row q], B'[m'][r] = x[r][m']
  const int64_t n0 = (int64_t)tile * TILE_ROWS;
  const int64_t ldt = (int64_t)pl.n_tiles * TILE_ROWS;
  const T* __restrict__ xr = X + rr * pl.N;
  for (int ks = 0; active && ks < pl.tail; ks += 32) {
    T av[8], xv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int mm = ks + 8 * g + j;
      const bool ok = mm < pl.tail;
      av[j] = ok ? pl.tailmat[(int64_t)mm * ldt + n0 + m] : T(0);
      xv[j] = (ok && rok) ? xr[mm] : T(0);
    }
    acc = E::step_real(av, xv, acc);
  }

  bool ok = true;
  for (int b = nblk - 1; b >= 0; --b) {
    // every group of the item complete for block b (thread 0 waits for all)
    {
      const ExecBlock<T>& bd = pl.blocks[b];
      bool okb = true;
      if (threadIdx.x < 64) {
        for (int g2 = g0; g2 <= g1; ++g2) {
          const uint32_t need = (uint32_t)(bd.parts * min(16, R - 16 * g2));
          if (!wait_count(sync, sync + bd.ctr + g2, need)) okb = false;
        }
        if (threadIdx.x == 0) {
          acquire();
          *s_flag = okb;
        }
      }
      __syncthreads();
      if (!*s_flag) ok = false;
      __syncthreads();
    }
    const int kw = active ? lane_i32(kw_l, b) : 0;
    if (kw == 0) continue;
    const int k0 = lane_i32(k0_l, b);
    const C* __restrict__ val = (const C*)(uintptr_t)lane_i64(val_l, b) + lane_i64(off_l, b);
    const C* __restrict__ zb =
        pl.Z + (int64_t)R * lane_i64(zoff_l, b) + rr * lane_i32(ldz_l, b) + k0;
    for (int kk = 0; kk < kw; kk += 16 * E::SB) {
      StepRegs<T> batch[E::SB];
#pragma unroll
      for (int i = 0; i < E::SB; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = kk + 16 * i + 4 * g + j;
          const bool in = c < kw;
          batch[i].a[j] = in ? val[c * TILE_ROWS + m] : C{T(0), T(0)};
          batch[i].z[j] = (in && rok) ? zb[c] : C{T(0), T(0)};
        }
      }
#pragma unroll
      for (int i = 0; i < E::SB; ++i)
        if (kk + 16 * i < kw) acc = E::step(batch[i].a, batch[i].z, acc);
    }
  }
  if (active && rok) {
    T* __restrict__ y = Y + (int64_t)r * pl.N + n0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = E::row(g, i);
      if (n0 + q < pl.N) y[q] = ok ? acc[i] : nan_of<T>();
    }
  }
}

// ------------------------------------------------------------------ kernel
template <typename E>
__global__ __launch_bounds__(EXEC_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void exec_kernel(ExecArgs<typename E::T> a) {
  using T = typename E::T;
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  double2* ltw = reinterpret_cast<double2*>(smem_raw + EXEC_POINTS * sizeof(C));
  __shared__ int4 s_item[2];
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  uint32_t* sync = a.sync;
  if (tid == 0) {
    const uint32_t i = __hip_atomic_fetch_add(sync + EXEC_SYNC_HEAD, 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    s_item[0] = i < (uint32_t)a.n_items ? a.items[i] : make_int4(-1, 0, 0, 0);
  }
  __syncthreads();
  int cur = 0;
  for (;;) {
    const int4 it = s_item[cur];
    if (it.x < 0) break;
    // take the next item now; it is stored for the next round after this one
    uint32_t nxt = 0;
    if (tid == 0)
      nxt = __hip_atomic_fetch_add(sync + EXEC_SYNC_HEAD, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    const int kind = it.x & 15, p = it.x >> 4;
    const ExecPlan<T>& pl = a.plans[p];
    switch (kind) {
      case ITEM_FFT:
        item_fft<T, true, false>(pl, pl.blocks[it.y], static_cast<const T*>(a.X[p]), it.z, it.w,
                                 lds, ltw, sync);
        break;
      case ITEM_COL:
        item_col<T, true>(pl, pl.blocks[it.y], static_cast<const T*>(a.X[p]), it.z, it.w, lds,
                          ltw, sync);
        break;
      case ITEM_ROW:
        item_row<T, true, false>(pl, pl.blocks[it.y], it.z, it.w, lds, ltw, sync, &s_flag);
        break;
      default:
        item_spmm<E>(pl, static_cast<const T*>(a.X[p]), a.Y[p], it.y, it.z, sync, &s_flag);
        break;
    }
    if (tid == 0)
      s_item[cur ^ 1] = nxt < (uint32_t)a.n_items ? a.items[nxt] : make_int4(-1, 0, 0, 0);
    __syncthreads();
    cur ^= 1;
  }
  // the last workgroup to finish reports whether a wait gave up (to the
  // host-visible word) and clears the queue, the counters and that flag; the
  // host-set wait bound stays
  if (tid == 0) {
    release();
    const uint32_t d = __hip_atomic_fetch_add(sync + EXEC_SYNC_DONE, 1u, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
    s_flag = d == gridDim.x - 1;
  }
  __syncthreads();
  if (s_flag) {
    acquire();
    if (tid == 0 && a.err_out)
      __hip_atomic_store(a.err_out, ld_relaxed(sync + EXEC_SYNC_ERR), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    __syncthreads();
    for (int i = tid; i < a.n_sync; i += EXEC_THREADS)
      if (i != EXEC_SYNC_WAIT) sync[i] = 0u;
  }
}

// FFT items without queue or counters: workgroup b runs item b; TI is the
// type of the right-hand sides
template <typename T, typename TI, bool SPLIT>
__global__ __launch_bounds__(EXEC_THREADS) void fft_items_kernel(ExecArgs<T> a) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  double2* ltw = reinterpret_cast<double2*>(smem_raw + EXEC_POINTS * sizeof(C));
  __shared__ int s_flag;
  const int4 it = a.items[blockIdx.x];
  const int kind = it.x & 15, p = it.x >> 4;
  const ExecPlan<T>& pl = a.plans[p];
  switch (kind) {
    case ITEM_FFT:
      item_fft<T, false, SPLIT, TI>(pl, pl.blocks[it.y], static_cast<const TI*>(a.X[p]), it.z,
                                    it.w, lds, ltw, nullptr);
      break;
    case ITEM_COL:
      item_col<T, false, +1, TI>(pl, pl.blocks[it.y], static_cast<const TI*>(a.X[p]), it.z, it.w,
                                 lds, ltw, nullptr);
      break;
    default:
      item_row<T, false, SPLIT>(pl, pl.blocks[it.y], it.z, it.w, lds, ltw, nullptr, &s_flag);
      break;
  }
}

// Precomputation (float64, F): the column or the row halves of four-step
// transforms of the rows of a panel; items as in fft_items_kernel.
__global__ __launch_bounds__(EXEC_THREADS) void row_fft4_kernel(ExecArgs<double> a) {
  using C = double2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  double2* ltw = reinterpret_cast<double2*>(smem_raw + EXEC_POINTS * sizeof(C));
  __shared__ int s_flag;
  const int4 it = a.items[blockIdx.x];
  const ExecPlan<double>& pl = a.plans[0];
  if ((it.x & 15) == ITEM_COL)
    item_col<double, false, -1>(pl, pl.blocks[it.y], static_cast<const double*>(a.X[0]), it.z,
                                it.w, lds, ltw, nullptr);
  else
    item_row<double, false, false, -1>(pl, pl.blocks[it.y], it.z, it.w, lds, ltw, nullptr,
                                       &s_flag);
}

template <typename K>
void set_lds(K kernel, size_t bytes) {
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

template <typename E>
int occupancy_of(size_t lds) {
  int n = 0;
  SPT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &n, reinterpret_cast<const void*>(exec_kernel<E>), EXEC_THREADS, lds));
  return n;
}

size_t device_lds() {
  int dev = 0, v = 0;
  SPT_HIP(hipGetDevice(&dev));
  SPT_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  return (size_t)v;
}

}  // namespace

void init_exec_kernels() {
  static std::vector<int> done;
  int dev = 0;
  SPT_HIP(hipGetDevice(&dev));
  for (int d : done)
    if (d == dev) return;
  // the kernels' static LDS (item slots, flags) stays below 256 bytes
  const size_t lds = device_lds() - 256;
  set_lds(exec_kernel<EngF64>, lds);
  set_lds(exec_kernel<EngF32>, lds);
  set_lds(exec_kernel<EngSplitBf16>, lds);
  set_lds(fft_items_kernel<double, double, false>, lds);
  set_lds(fft_items_kernel<double, float, true>, lds);
  set_lds(fft_items_kernel<double, float, false>, lds);
  set_lds(fft_items_kernel<float, float, false>, lds);
  set_lds(fft_items_kernel<float, float, true>, lds);
  set_lds(row_fft4_kernel, lds);
  done.push_back(dev);
}

int exec_occupancy(int engine, int ntw) {
  switch (engine) {
    case 0: return occupancy_of<EngF64>(exec_lds_bytes<double>(ntw));
    case 1: return occupancy_of<EngF32>(exec_lds_bytes<float>(ntw));
    default: return occupancy_of<EngSplitBf16>(exec_lds_bytes<float>(ntw));
  }
}

template <>
void launch_exec<double>(const ExecArgs<double>& a, int engine, int grid, hipStream_t s) {
  (void)engine;
  hipLaunchKernelGGL(exec_kernel<EngF64>, dim3(grid), dim3(EXEC_THREADS),
                     exec_lds_bytes<double>(a.ntw), s, a);
  SPT_HIP(hipGetLastError());
}

template <>
void launch_exec<float>(const ExecArgs<float>& a, int engine, int grid, hipStream_t s) {
  if (engine == 2)
    hipLaunchKernelGGL(exec_kernel<EngSplitBf16>, dim3(grid), dim3(EXEC_THREADS),
                       exec_lds_bytes<float>(a.ntw), s, a);
  else
    hipLaunchKernelGGL(exec_kernel<EngF32>, dim3(grid), dim3(EXEC_THREADS),
                       exec_lds_bytes<float>(a.ntw), s, a);
  SPT_HIP(hipGetLastError());
}

void launch_row_fft4(const ExecArgs<double>& a, hipStream_t s) {
  if (a.n_items <= 0) return;
  hipLaunchKernelGGL(row_fft4_kernel, dim3(a.n_items), dim3(EXEC_THREADS),
                     exec_lds_bytes<double>(a.ntw), s, a);
  SPT_HIP(hipGetLastError());
}

template <>
void launch_fft_items<double>(const ExecArgs<double>& a, bool split, bool xf, hipStream_t s) {
  if (a.n_items <= 0) return;
  if (split)
    hipLaunchKernelGGL((fft_items_kernel<double, float, true>), dim3(a.n_items),
                       dim3(EXEC_THREADS), exec_lds_bytes<double>(a.ntw), s, a);
  else if (xf)
    hipLaunchKernelGGL((fft_items_kernel<double, float, false>), dim3(a.n_items),
                       dim3(EXEC_THREADS), exec_lds_bytes<double>(a.ntw), s, a);
  else
    hipLaunchKernelGGL((fft_items_kernel<double, double, false>), dim3(a.n_items),
                       dim3(EXEC_THREADS), exec_lds_bytes<double>(a.ntw), s, a);
  SPT_HIP(hipGetLastError());
}

template <>
void launch_fft_items<float>(const ExecArgs<float>& a, bool split, bool xf, hipStream_t s) {
  (void)xf;
  if (a.n_items <= 0) return;
  if (split)
    hipLaunchKernelGGL((fft_items_kernel<float, float, true>), dim3(a.n_items),
                       dim3(EXEC_THREADS), exec_lds_bytes<float>(a.ntw), s, a);
  else
    hipLaunchKernelGGL((fft_items_kernel<float, float, false>), dim3(a.n_items),
                       dim3(EXEC_THREADS), exec_lds_bytes<float>(a.ntw), s, a);
  SPT_HIP(hipGetLastError());
}

}  // namespace spt
