// Batched real <-> half-complex FFTs in LDS for gfx950.
//
// A real vector of even length L = 2P is packed as P complex points
// c_j = v_{2j} + i v_{2j+1}, transformed by a mixed-radix (2, 3, 4, 5, 8)
// Stockham autosort FFT held entirely in LDS (one workgroup per vector, each
// pass reads its radix-R butterfly inputs into registers, synchronises, and
// writes the outputs in place), and unpacked into the half spectrum
// Z_k, k = 0 .. P, of the length-L DFT (sec. 5.1: real rows and real inputs
// only need half of the spectrum).
//
// Conventions: F of eq. (1) has the kernel exp(-2 pi i jk/L)/sqrt(L) (SIGN -1,
// used by the precomputation A_e W F); the computation stage applies F*
// (SIGN +1).  The fused computation-stage kernel in float32 reads its pass
// twiddles exp(+2 pi i jm r/(Ns R)) from one table per block (each entry
// rounded once from extended precision); the other kernels form them from two
// float64 tables of 128 + P/128 entries (w^q = lo[q % 128]
// hi[q / 128]), a butterfly taking w^jm once and its powers in float64.  The
// unpack twiddles exp(+i pi k/P) (k <= P) are a table in the working
// precision.  SIGN -1 uses the conjugates.

#include <algorithm>
#include <type_traits>

#include "fft_core.hpp"
#include "spmm_core.hpp"

namespace spt {
namespace {

using namespace fftcore;

// Workgroups of the FFT kernels have at most FFT_MAX_THREADS threads (16
// waves: 4 per SIMD, which hide each other's LDS and memory waits), which
// leaves each thread up to 128 registers for its butterflies.
constexpr int FFT_MAX_THREADS = 1024;

template <typename T>
__global__ __launch_bounds__(FFT_MAX_THREADS) void exec_fft_kernel(ExecFftArgs<T> a, FftPlan fp) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int r = blockIdx.x;
  const T* __restrict__ x = a.X + (int64_t)r * a.N;
  for (int j = tid; j < a.P; j += nt) {
    const int c0 = 2 * j, c1 = 2 * j + 1;
    T v0 = (c0 >= a.c_lo && c0 < a.c_hi) ? x[c0 + a.m_off] * a.winv[c0] : T(0);
    T v1 = (c1 >= a.c_lo && c1 < a.c_hi) ? x[c1 + a.m_off] * a.winv[c1] : T(0);
    lds[j] = C{v0, v1};
  }
  __syncthreads();
  run_fft<+1>(lds, fp, a.tw, tid, nt);
  C* __restrict__ z = a.Z + (int64_t)r * a.ldz;
  for (int k = tid; k <= a.P; k += nt) z[k] = unpack<+1>(lds, a.P, k, a.post, a.scale);
}

// The twiddles of a block staged into LDS after its points, so that the
// passes and the unpacking wait for no global memory: the two-level float64
// tables of exp(2 pi i q / P) (tw) and of exp(i pi k / P) (tw2), ntw entries
// each (a few KB, which leaves LDS for other workgroups on the CU).  load()
// requests them; store() writes them once they arrive, after the caller has
// requested its points, so both share one wait.
template <typename T, int EI>
struct TabStage {
  static constexpr int SLOTS = 2;
  double2 v[2][SLOTS];
  const double2* src[2];
  int n;
  __device__ __forceinline__ void load(const FftDesc<T>* d, int tid, int nt) {
    src[0] = d->tw;
    src[1] = d->tw2;
    n = d->ntw;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int e = 0; e < SLOTS; ++e) v[t][e] = gload(src[t] + min(tid + e * nt, n - 1));
  }
  __device__ __forceinline__ void store(double2* dst, int tid, int nt) const {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int e = 0; e < SLOTS; ++e)
        if (tid + e * nt < n) dst[t * n + tid + e * nt] = v[t][e];
      for (int i = tid + SLOTS * nt; i < n; i += nt) dst[t * n + i] = gload(src[t] + i);
    }
  }
};

// LDS byte offset of the staged twiddles behind pts points
template <typename T>
__host__ __device__ inline size_t tab_offset(int pts) {
  return ((size_t)pts * sizeof(cplx_t<T>) + 15) & ~(size_t)15;
}

// (v_c, v_(c+1)) = x_(c + m_off) / w_c on the retained columns [c_lo, c_hi),
// 0 elsewhere, for an even c.  VEC (m_off, N, c_lo and c_hi even, so that a
// pair lies wholly inside or outside the retained columns): x and 1/w are read
// as aligned pairs, from column c_lo when the pair is outside (a valid
// address; the value is discarded).
// x is of type TI (float32 input of the split-bf16 path whose transform runs
// in float64 arithmetic: T = double, TI = float), the window reciprocals of T.
template <bool VEC, typename T, typename TI>
__device__ __forceinline__ cplx_t<T> point_pair(const TI* __restrict__ x, const T* __restrict__ winv,
                                                int c, int c_lo, int c_hi, int m_off) {
  using C = cplx_t<T>;
  if constexpr (VEC) {
    const bool in = c >= c_lo && c < c_hi;
    const int cc = in ? c : c_lo;
    const cplx_t<TI> xv = gload(reinterpret_cast<const cplx_t<TI>*>(x + m_off + cc));
    const C wv = gload(reinterpret_cast<const C*>(winv + cc));
    return in ? C{T(xv.x) * wv.x, T(xv.y) * wv.y} : C{T(0), T(0)};
  } else {
    auto val = [&](int cv) {
      return cv >= c_lo && cv < c_hi ? T(gload(x + cv + m_off)) * gload(winv + cv) : T(0);
    };
    return C{val(c), val(c + 1)};
  }
}

// The retained columns [c_lo, c_hi) of one row of X and of the window
// reciprocals as raw buffers: a load outside them returns zeros, so that
// v_c = x_(c + m_off) / w_c needs neither an index clamp nor a select, and
// every address is one 32-bit offset.
template <typename T, typename TI>
struct RowSrc {
  buf_t xr, wr;
  int c_lo;
  __device__ __forceinline__ RowSrc(const TI* x, const T* winv, int c_lo_, int c_hi, int m_off)
      : c_lo(c_lo_) {
    const uint32_t n = c_hi > c_lo_ ? (uint32_t)(c_hi - c_lo_) : 0u;
    xr = buf_rsrc(x + m_off + c_lo_, n * (uint32_t)sizeof(TI));
    wr = buf_rsrc(winv + c_lo_, n * (uint32_t)sizeof(T));
  }
  // v_c
  __device__ __forceinline__ T one(int c) const {
    const int o = c - c_lo;
    return T(buf_ld<TI>(xr, o * (int)sizeof(TI))) * buf_ld<T>(wr, o * (int)sizeof(T));
  }
  // (v_c, v_(c+1)) for an even c, when m_off, c_lo and c_hi are even (a pair
  // lies wholly inside or outside the retained columns)
  __device__ __forceinline__ cplx_t<T> pair(int c) const {
    const int o = c - c_lo;
    const cplx_t<TI> xv = buf_ld<cplx_t<TI>>(xr, o * (int)sizeof(TI));
    const cplx_t<T> wv = buf_ld<cplx_t<T>>(wr, o * (int)sizeof(T));
    return cplx_t<T>{T(xv.x) * wv.x, T(xv.y) * wv.y};
  }
  // float32: (v_c, v_(c+1)) and (v_(c+2), v_(c+3)) for c a multiple of 4,
  // when m_off, c_lo and c_hi are too (16-byte loads)
  __device__ __forceinline__ void quad(int c, float2& lo, float2& hi) const {
    const int o = (c - c_lo) * 4;
    const float4 xv = buf_f32x4(xr, o), wv = buf_f32x4(wr, o);
    lo = float2{xv.x * wv.x, xv.y * wv.y};
    hi = float2{xv.z * wv.z, xv.w * wv.w};
  }
};

// Every block of a plan and every right-hand side in one grid (FftGrid: block
// b, sorted by decreasing length, owns workgroups wg0[b] .. wg0[b+1] - 1);
// workgroup x of a block takes either a part of a split transform of one
// right-hand side (FftDesc::half: one parity half, or one residue mod 8), or
// the right-hand sides r0 = x 2^lb .. r0 + 2^lb - 1 (lb = FftDesc::lb), their
// transforms interleaved in LDS (point j of transform t at lds[(j << lb) + t])
// so that a short block fills the workgroup as a long one does.

// SPLIT: the half spectra are written as three bfloat16 planes (the pieces of
// the split-bf16 product, layout in common.hpp) instead of complex values.
// BATCH == false: one transform (lb == 0), indexed without the interleaving.
// EI: points per thread, FFT_EPT or fewer (2^lb P <= EI nt): loops over the
// thread's points stop there instead of clamping indexes past the end
template <typename T, typename TI, bool SPLIT, bool BATCH, int EI>
__device__ __forceinline__ void fft_multi_body(const FftDesc<T>* __restrict__ d,
                                               const TI* __restrict__ X, cplx_t<TI>* __restrict__ Z,
                                               uint32_t* __restrict__ Zs, int64_t zplane, int R,
                                               int64_t N, int lb_, int r0) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int lb = BATCH ? lb_ : 0;
  const int cnt = BATCH ? min(1 << lb, R - r0) : 1;  // transforms of the workgroup
  const int tmask = (1 << lb) - 1;
  const int P = d->fp.P, nt = blockDim.x;
  const int tid = threadIdx.x;
  const int c_lo = d->c_lo, c_hi = d->c_hi, m_off = d->m_off;
  const T* __restrict__ winv = d->winv;
  const T scale = d->scale;
  // The twiddle tables are requested first, then the points, so that all of
  // them arrive within one wait.
  constexpr int GS = EI / 4 + 2;  // output groups per thread (SPLIT)
  TabStage<T, EI> ts;
  ts.load(d, tid, nt);
  // E1: the thread's points (float32: all at once; float64: in two rounds, for
  // registers), written to LDS; transforms past the last right-hand side are
  // zero.  Loads are branch-free: indexes past the end are clamped.
  constexpr int ROUND = (sizeof(T) == 4 || EI <= FFT_EPT / 2) ? EI : FFT_EPT / 2;
  const int pts = P << lb;
  double2* ltab = reinterpret_cast<double2*>(smem_raw + tab_offset<T>(pts));
  const double2* ltab2 = ltab + d->ntw;  // exp(i pi k / P)
  auto input = [&](auto vtag) {
    constexpr bool VEC = decltype(vtag)::value;
#pragma unroll
    for (int h = 0; h < EI; h += ROUND) {
      C v[ROUND];
#pragma unroll
      for (int e = 0; e < ROUND; ++e) {
        const int u = tid + (h + e) * nt;
        if constexpr (VEC && !BATCH) {
          // one row: points past the transform read past c_hi (zeros)
          const RowSrc<T, TI> src(X + (int64_t)r0 * N, winv, c_lo, c_hi, m_off);
          v[e] = src.pair(2 * u);
          continue;
        }
        const int uu = min(u, pts - 1);
        const int j = uu >> lb, t = uu & tmask;
        const TI* __restrict__ x = X + (int64_t)(r0 + (BATCH ? min(t, cnt - 1) : 0)) * N;
        const C pr = point_pair<VEC>(x, winv, 2 * j, c_lo, c_hi, m_off);
        v[e] = u < pts && t < cnt ? pr : C{T(0), T(0)};
      }
      if (h == 0) ts.store(ltab, tid, nt);
#pragma unroll
      for (int e = 0; e < ROUND; ++e) {
        const int u = tid + (h + e) * nt;
        if (u < pts) lds[u] = v[e];
      }
    }
  };
  // pairs: columns and the base of X aligned to two elements
  const int xa = (int)((uintptr_t)X / sizeof(TI));
  if (((m_off | (int)N | c_lo | c_hi | xa) & 1) == 0)
    input(std::true_type{});
  else
    input(std::false_type{});
  __syncthreads();
  // E2: F*, the pass twiddles formed from the two-level table
  run_fft<+1, BATCH, EI, true>(lds, P, lb, d->fp.npass, d->fp.radix, ltab, 1, tid, nt, true);
  // unpack point k of transform t (see unpack_with)
  auto unpack_at = [&](int k, int t, C tw) {
    C ck = lds[((k == P ? 0 : k) << lb) + t];
    C cm = lds[((k == 0 ? 0 : P - k) << lb) + t];
    cm.y = -cm.y;
    const C e = C{T(0.5) * (ck.x + cm.x), T(0.5) * (ck.y + cm.y)};
    const C dd = C{T(0.5) * (ck.x - cm.x), T(0.5) * (ck.y - cm.y)};
    const C o = C{dd.y, -dd.x};  // dd / i
    const C z = cadd(e, cmul(tw, o));
    return C{z.x * scale, z.y * scale};
  };
  // the thread's outputs u = tid + e nt (u < (P + 1) << lb <= EI nt + 2^lb)
  if constexpr (!SPLIT) {
    const int n = (P + 1) << lb;
#pragma unroll
    for (int e = 0; e <= EI; ++e) {
      const int u = tid + e * nt;
      const int k = u >> lb, t = u & tmask;
      if (u < n && t < cnt) {
        const C z = unpack_at(k, t, to_c<C>(twiddle(ltab2, k)));
        Z[(int64_t)R * d->zoff + (int64_t)(r0 + t) * d->ldz + k] = cplx_t<TI>{TI(z.x), TI(z.y)};
      }
    }
  } else {
    // four consecutive k per thread (ldz4 is a multiple of 4): each plane gets
    // one 16-byte store per group; zeros past P.  Groups u = tid + e nt, e <
    // GS (n <= EI nt / 4 + 2^lb + 1 <= GS nt)
    const int n = (d->ldz4 / 4) << lb;
#pragma unroll
    for (int e = 0; e < GS; ++e) {
      const int u = tid + e * nt;
      if (u >= n) break;
      const int q = u >> lb, t = u & tmask;
      if (t >= cnt) continue;
      uint32_t pc[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * q + j;
        const C z = k <= P ? unpack_at(k, t, to_c<C>(twiddle(ltab2, k))) : C{T(0), T(0)};
        spmmcore::split2(spmmcore::f32x2{(float)z.x, (float)z.y}, pc[j]);
      }
      uint32_t* __restrict__ zs = Zs + (int64_t)R * d->zoff4 + (int64_t)(r0 + t) * d->ldz4;
#pragma unroll
      for (int p = 0; p < 3; ++p)
        *reinterpret_cast<uint4*>(zs + p * zplane + 4 * q) =
            uint4{pc[0][p], pc[1][p], pc[2][p], pc[3][p]};
    }
  }
}

// One half of a transform split by output parity (FftDesc::half): with
// w = exp(2 pi i / P) and H = P / 2, the outputs of parity p are
//   C[2m + p] = sum_n w^(2nm) y_n,  y_n = w^(np) (c_n + (-1)^p c_(n+H)),
// a transform of H points (one decimation-in-frequency step).  The unpack
// pairs C_k with C_(P-k), of the same parity, so the half is complete: it
// writes the half spectrum at every k of parity p (zeros past P).
template <typename T, typename TI, bool SPLIT, int EI>
__device__ __forceinline__ void fft_half_body(const FftDesc<T>* __restrict__ d,
                                              const TI* __restrict__ X, cplx_t<TI>* __restrict__ Z,
                                              uint32_t* __restrict__ Zs, int64_t zplane, int R,
                                              int64_t N, int r, int par) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int H = d->fp.P, P = 2 * H, nt = blockDim.x;
  const int tid = threadIdx.x;
  const int c_lo = d->c_lo, c_hi = d->c_hi, m_off = d->m_off;
  const T* __restrict__ winv = d->winv;
  const TI* __restrict__ x = X + (int64_t)r * N;
  const C* __restrict__ post = d->post;  // post[2n] = w^n
  // the twiddle tables first, then the points: one wait for all of them
  TabStage<T, EI> ts;
  ts.load(d, tid, nt);
  double2* ltab = reinterpret_cast<double2*>(smem_raw + tab_offset<T>(H));
  const double2* ltab2 = ltab + d->ntw;  // exp(i pi k / P)
  constexpr int ROUND = (sizeof(T) == 4 || EI <= FFT_EPT / 2) ? EI : FFT_EPT / 2;
  auto input = [&](auto vtag) {
    constexpr bool VEC = decltype(vtag)::value;
    // VEC: buffer loads, zeros outside the retained columns and past the end
    // of post (points n >= H are not stored)
    const RowSrc<T, TI> src(x, winv, c_lo, c_hi, m_off);
    const buf_t postr = buf_rsrc(post, (uint32_t)(P + 1) * (uint32_t)sizeof(C));
#pragma unroll
    for (int h = 0; h < EI; h += ROUND) {
      C y[ROUND];
#pragma unroll
      for (int e = 0; e < ROUND; ++e) {
        if constexpr (VEC) {
          const int n = tid + (h + e) * nt;
          const C a = src.pair(2 * n);
          const C b = src.pair(2 * n + P);
          y[e] = par ? cmul(csub(a, b), buf_ld<C>(postr, 2 * n * (int)sizeof(C))) : cadd(a, b);
          continue;
        }
        const int n = min(tid + (h + e) * nt, H - 1);
        const C a = point_pair<VEC>(x, winv, 2 * n, c_lo, c_hi, m_off);
        const C b = point_pair<VEC>(x, winv, 2 * n + P, c_lo, c_hi, m_off);
        y[e] = par ? cmul(csub(a, b), gload(post + 2 * n)) : cadd(a, b);
      }
      if (h == 0) ts.store(ltab, tid, nt);
#pragma unroll
      for (int e = 0; e < ROUND; ++e) {
        const int n = tid + (h + e) * nt;
        if (n < H) lds[n] = y[e];
      }
    }
  };
  // float32 with columns aligned to 4: two points per thread and load (16
  // bytes of x and of 1/w from each half of the row), in two rounds
  auto input_quads = [&]() {
    if constexpr (sizeof(T) == 4 && sizeof(TI) == 4) {
      constexpr int EH = (EI + 1) / 2;  // pairs of points per thread
      constexpr int RQ = (EH + 1) / 2;
      const RowSrc<T, TI> src(x, winv, c_lo, c_hi, m_off);
      const buf_t postr = buf_rsrc(post, (uint32_t)(P + 1) * (uint32_t)sizeof(C));
#pragma unroll
      for (int h = 0; h < EH; h += RQ) {
        C y[RQ][2];
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
          const int j = tid + (h + e) * nt;  // points 2j and 2j + 1
          C a0, a1, b0, b1;
          src.quad(4 * j, a0, a1);
          src.quad(4 * j + P, b0, b1);
          if (par) {
            const C w0 = buf_ld<C>(postr, 4 * j * (int)sizeof(C));
            const C w1 = buf_ld<C>(postr, (4 * j + 2) * (int)sizeof(C));
            y[e][0] = cmul(csub(a0, b0), w0);
            y[e][1] = cmul(csub(a1, b1), w1);
          } else {
            y[e][0] = cadd(a0, b0);
            y[e][1] = cadd(a1, b1);
          }
        }
        if (h == 0) ts.store(ltab, tid, nt);
#pragma unroll
        for (int e = 0; e < RQ; ++e) {
          const int j = tid + (h + e) * nt;
          if (h + e < EH && 2 * j < H)
            *reinterpret_cast<float4*>(lds + 2 * j) =
                float4{y[e][0].x, y[e][0].y, y[e][1].x, y[e][1].y};
        }
      }
    }
  };
  // quads and pairs: columns and the base of X aligned to four and two elements
  const int xa = (int)((uintptr_t)X / sizeof(TI));
  if (sizeof(T) == 4 && sizeof(TI) == 4 && ((m_off | (int)N | c_lo | c_hi | xa) & 3) == 0)
    input_quads();
  else if (((m_off | (int)N | c_lo | c_hi | xa) & 1) == 0)
    input(std::true_type{});
  else
    input(std::false_type{});
  __syncthreads();
  // the two-level table is of length P = 2H: index scale 2
  run_fft<+1, false, EI, true>(lds, H, 0, d->fp.npass, d->fp.radix, ltab, 2, tid, nt, true);
  // k = 2m + par: C_k at lds[m mod H], C_(P-k) at lds[(H - m) mod H] (par 0)
  // or lds[H - 1 - m] (par 1)
  const T scale = d->scale;
  auto zval = [&](int m) {
    const C tw = to_c<C>(twiddle(ltab2, min(2 * m + par, P)));
    const int k = 2 * m + par;
    if (k > P) return C{T(0), T(0)};
    C ck = lds[m == H ? 0 : m];
    C cm = lds[par ? H - 1 - m : (m == 0 || m == H ? 0 : H - m)];
    cm.y = -cm.y;
    const C e = C{T(0.5) * (ck.x + cm.x), T(0.5) * (ck.y + cm.y)};
    const C dd = C{T(0.5) * (ck.x - cm.x), T(0.5) * (ck.y - cm.y)};
    const C o = C{dd.y, -dd.x};  // dd / i
    const C z = cadd(e, cmul(tw, o));
    return C{z.x * scale, z.y * scale};
  };
  // outputs k = 2m + par < kend; the thread's m are tid + e nt, e <= EI
  // (H <= EI nt)
  const int kend = SPLIT ? d->ldz4 : P + 1;
#pragma unroll
  for (int e = 0; e <= EI; ++e) {
    const int m = tid + e * nt, k = 2 * m + par;
    if (k >= kend) break;
    const C z = zval(m);
    if constexpr (!SPLIT) {
      Z[(int64_t)R * d->zoff + (int64_t)r * d->ldz + k] = cplx_t<TI>{TI(z.x), TI(z.y)};
    } else {
      uint32_t pc[3];
      spmmcore::split2(spmmcore::f32x2{(float)z.x, (float)z.y}, pc);
      uint32_t* __restrict__ zs = Zs + (int64_t)R * d->zoff4 + (int64_t)r * d->ldz4 + k;
#pragma unroll
      for (int p = 0; p < 3; ++p) zs[p * zplane] = pc[p];
    }
  }
}

// Eight-way split of the real transform of L = 2P points by output residue
// (FftDesc::half == FFT_SPLIT_EIGHT), one workgroup per residue p = 0..4: with
// W = exp(2 pi i / L), omega = exp(2 pi i / 8) and M = L / 8,
//   X[8m + p] = sum_{n<M} exp(2 pi i nm / M) y_n,
//   y_n = W^(np) sum_{q<8} v_(n + qM) omega^(pq),
// one decimation-in-frequency step of radix 8, then a transform of M points.
// v is real, so X[L - k] = conj(X[k]) and the transform Y of residue p also
// gives residue 8 - p: X[8m + 8 - p] = conj(Y[M - 1 - m]).  The five
// workgroups of a right-hand side write the half spectrum k = 0..P between
// them (zeros past P in the split planes), and each reads the whole row, so
// that the transform of a long block is spread over five CUs.
template <typename T, typename TI, bool SPLIT, int EI>
__device__ __forceinline__ void fft_rdif_body(const FftDesc<T>* __restrict__ d,
                                              const TI* __restrict__ X, cplx_t<TI>* __restrict__ Z,
                                              uint32_t* __restrict__ Zs, int64_t zplane, int R,
                                              int64_t N, int r, int p) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int M = d->fp.P, P = 4 * M, nt = blockDim.x;
  const int tid = threadIdx.x;
  const int c_lo = d->c_lo, c_hi = d->c_hi, m_off = d->m_off;
  const T* __restrict__ winv = d->winv;
  const TI* __restrict__ x = X + (int64_t)r * N;
  TabStage<T, EI> ts;
  ts.load(d, tid, nt);
  double2* ltab = reinterpret_cast<double2*>(smem_raw + tab_offset<T>(M));
  const double2* ltab2 = ltab + d->ntw;  // W^k = exp(i pi k / P)
  // omega^t = (cos, sin)(2 pi t / 8) for t = (p q) mod 8
  constexpr T h = T(0.70710678118654752440);
  T co[8], si[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int t = (p * q) & 7;
    co[q] = t == 0 ? T(1) : t == 4 ? T(-1) : (t == 2 || t == 6) ? T(0) : (t == 1 || t == 7) ? h : -h;
    si[q] = t == 2 ? T(1) : t == 6 ? T(-1) : (t == 0 || t == 4) ? T(0) : (t == 1 || t == 3) ? h : -h;
  }
  // E1 and the radix-8 step: y_n without the factor W^(np), in rounds of RD
  // points (16 loads each)
  constexpr int RD = 2;
  const RowSrc<T, TI> src(x, winv, c_lo, c_hi, m_off);  // zeros outside [c_lo, c_hi)
#pragma unroll
  for (int e0 = 0; e0 < EI; e0 += RD) {
    T v[RD][8];
#pragma unroll
    for (int e = 0; e < RD; ++e) {
      const int n = tid + (e0 + e) * nt;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[e][q] = src.one(n + q * M);
    }
    if (e0 == 0) ts.store(ltab, tid, nt);
#pragma unroll
    for (int e = 0; e < RD; ++e) {
      const int n = tid + (e0 + e) * nt;
      T re = T(0), im = T(0);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        re += v[e][q] * co[q];
        im += v[e][q] * si[q];
      }
      if (e0 + e < EI && n < M) lds[n] = C{re, im};
    }
  }
  __syncthreads();
  // the factor W^(np) on the thread's own points (the tables are in LDS now)
  if (p != 0) {
#pragma unroll
    for (int e = 0; e < EI; ++e) {
      const int n = tid + e * nt;
      if (n < M) lds[n] = cmul(lds[n], to_c<C>(twiddle(ltab2, n * p)));
    }
    __syncthreads();
  }
  // the table is of length P = 4M: index scale 4
  run_fft<+1, false, EI, true>(lds, M, 0, d->fp.npass, d->fp.radix, ltab, 4, tid, nt, true);
  // outputs: residue p at k = 8m + p (Y[m]) and, for p = 1..3, residue 8 - p
  // at k = 8m + 8 - p (conj Y[M - 1 - m]); output u of the workgroup is
  // residue p at m = u (p = 0, 4) or, alternately, the two residues at m = u / 2
  const T scale = d->scale;
  const int kend = SPLIT ? d->ldz4 : P + 1;
  const bool two = p != 0 && p != 4;
  const int n_p = (kend - p + 7) / 8;
  const int n_out = two ? n_p + (kend - (8 - p) + 7) / 8 : n_p;
  for (int u = tid; u < n_out; u += nt) {
    const bool mirror = two && (u & 1);
    const int m = two ? u >> 1 : u;
    const int k = mirror ? 8 * m + 8 - p : 8 * m + p;
    if (mirror && k >= kend) continue;
    C z = C{T(0), T(0)};
    if (k <= P) {
      const C y = lds[mirror ? M - 1 - m : m];
      z = C{y.x * scale, (mirror ? -y.y : y.y) * scale};
    }
    if constexpr (!SPLIT) {
      Z[(int64_t)R * d->zoff + (int64_t)r * d->ldz + k] = cplx_t<TI>{TI(z.x), TI(z.y)};
    } else {
      uint32_t pc[3];
      spmmcore::split2(spmmcore::f32x2{(float)z.x, (float)z.y}, pc);
      uint32_t* __restrict__ zs = Zs + (int64_t)R * d->zoff4 + (int64_t)r * d->ldz4 + k;
#pragma unroll
      for (int q = 0; q < 3; ++q) zs[q * zplane] = pc[q];
    }
  }
}

// MAXT: the launch's threads are at most MAXT (512 leaves each thread 256
// registers, 768 leaves 168, 1024 leaves 128; float64 arithmetic takes 768
// where it fits, as it spills under 128).  TI: type of X and of the complex spectra Z
// (float with T = double: the float32 paths' transforms in float64
// arithmetic, each spectrum value rounded once to float32).
// Float32 arithmetic at 512 threads is held to 128 registers, so that two
// workgroups share a CU (their memory waits and passes overlap).
template <typename T, typename TI, bool SPLIT, int MAXT>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 4 && MAXT <= 512 ? 4 : 1))) void exec_fft_multi_kernel(
    const FftDesc<T>* __restrict__ descs, FftGrid g, const TI* __restrict__ X,
    cplx_t<TI>* __restrict__ Z, uint32_t* __restrict__ Zs, int64_t zplane, int R, int64_t N) {
  // transforms of at most EI_SHORT points per thread take the variant whose
  // loops stop there
  constexpr int EI_SHORT = FFT_EPT / 2;
  // the workgroup's block: the last b with wg0[b] <= blockIdx.x
  int b = 0;
#pragma unroll
  for (int i = 1; i < FFT_GRID_MAX; ++i)
    if (i < g.nblk && (int)blockIdx.x >= g.wg0[i]) b = i;
  const int wx = (int)blockIdx.x - g.wg0[b];
  const FftDesc<T>* __restrict__ d = descs + b;
  if (d->half == FFT_SPLIT_EIGHT) {
    // workgroup wx = p R + r: the five workgroups of a right-hand side are R
    // apart, on one XCD when R is a multiple of 8 (their reads of the row and
    // their interleaved writes meet in one L2)
    const int p = wx / R, r = wx - p * R;
    if (d->fp.P <= EI_SHORT * (int)blockDim.x)
      fft_rdif_body<T, TI, SPLIT, EI_SHORT>(d, X, Z, Zs, zplane, R, N, r, p);
    else
      fft_rdif_body<T, TI, SPLIT, FFT_EPT>(d, X, Z, Zs, zplane, R, N, r, p);
    return;
  }
  if (d->half == FFT_SPLIT_PARITY) {
    // workgroup wx = parity R + r: the two halves of a right-hand side are R
    // workgroups apart, on the same XCD when R is a multiple of 8, so that
    // their reads of the row and their interleaved writes meet in one L2
    const int par = wx >= R ? 1 : 0;
    const int r = wx - par * R;
    if (d->fp.P <= EI_SHORT * (int)blockDim.x)
      fft_half_body<T, TI, SPLIT, EI_SHORT>(d, X, Z, Zs, zplane, R, N, r, par);
    else
      fft_half_body<T, TI, SPLIT, FFT_EPT>(d, X, Z, Zs, zplane, R, N, r, par);
    return;
  }
  const int lb = d->lb;
  const int r0 = wx << lb;
  if (r0 >= R) return;
  const bool short_pts = (d->fp.P << lb) <= EI_SHORT * (int)blockDim.x;
  if (lb == 0) {
    if (short_pts)
      fft_multi_body<T, TI, SPLIT, false, EI_SHORT>(d, X, Z, Zs, zplane, R, N, 0, r0);
    else
      fft_multi_body<T, TI, SPLIT, false, FFT_EPT>(d, X, Z, Zs, zplane, R, N, 0, r0);
  } else {
    if (short_pts)
      fft_multi_body<T, TI, SPLIT, true, EI_SHORT>(d, X, Z, Zs, zplane, R, N, lb, r0);
    else
      fft_multi_body<T, TI, SPLIT, true, FFT_EPT>(d, X, Z, Zs, zplane, R, N, lb, r0);
  }
}

// ---------------------------------------------------------------- transposed: E4
// One workgroup per right-hand side: half spectrum U (k = 0..P) -> real g of
// length 2P by F*, then y_{c + m_off} = g_c / w_c on the retained columns only
// (the extras are discarded, eq. Fe2).
template <typename T>
__global__ __launch_bounds__(FFT_MAX_THREADS) void inv_fft_kernel(InvFftArgs<T> a, FftPlan fp) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int r = blockIdx.x;
  const C* __restrict__ u = a.U + (int64_t)r * a.ldu;
  for (int k = tid; k < a.P; k += nt) {
    C uk = u[k];
    C um = u[a.P - k];
    um.y = -um.y;  // conj U_{P-k}
    C ge = cadd(uk, um);
    C go = cmul(csub(uk, um), a.post[k]);
    lds[k] = C{ge.x - go.y, ge.y + go.x};  // ge + i go
  }
  __syncthreads();
  run_fft<+1>(lds, fp, a.tw, tid, nt);
  T* __restrict__ y = a.Y + (int64_t)r * a.N;
  for (int j = tid; j < a.P; j += nt) {
    const C c = lds[j];
    const int c0 = 2 * j, c1 = 2 * j + 1;
    if (c0 >= a.c_lo && c0 < a.c_hi) y[c0 + a.m_off] = c.x * a.scale * a.winv[c0];
    if (c1 >= a.c_lo && c1 < a.c_hi) y[c1 + a.m_off] = c.y * a.scale * a.winv[c1];
  }
}

// The same for every block of a plan in one launch (descriptors in device
// memory; the workgroup has the threads of the longest transform).
// TI: type of U and Y (float with T = double: the float32 path's transform in
// float64 arithmetic)
template <typename T, typename TI = T>
__global__ __launch_bounds__(FFT_MAX_THREADS) void inv_fft_multi_kernel(
    const InvFftDesc<T>* __restrict__ descs, const cplx_t<TI>* __restrict__ U, TI* __restrict__ Y,
    int R, int64_t N) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const InvFftDesc<T>* __restrict__ d = descs + blockIdx.y;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int r = blockIdx.x;
  const int P = d->P;
  const cplx_t<TI>* __restrict__ u = U + d->uoff * R + (int64_t)r * (P + 1);
  const C* __restrict__ post = d->post;
  for (int k = tid; k < P; k += nt) {
    const C uk = C{T(u[k].x), T(u[k].y)};
    C um = C{T(u[P - k].x), T(u[P - k].y)};
    um.y = -um.y;  // conj U_(P-k)
    const C ge = cadd(uk, um);
    const C go = cmul(csub(uk, um), post[k]);
    lds[k] = C{ge.x - go.y, ge.y + go.x};  // ge + i go
  }
  __syncthreads();
  run_fft<+1, false>(lds, P, 0, d->fp.npass, d->fp.radix, d->tw, 1, tid, nt, true);
  const T scale = d->scale;
  const T* __restrict__ winv = d->winv;
  const int c_lo = d->c_lo, c_hi = d->c_hi, m_off = d->m_off;
  TI* __restrict__ y = Y + (int64_t)r * N;
  for (int j = tid; j < P; j += nt) {
    const C c = lds[j];
    const int c0 = 2 * j, c1 = 2 * j + 1;
    if (c0 >= c_lo && c0 < c_hi) y[c0 + m_off] = TI(c.x * scale * winv[c0]);
    if (c1 >= c_lo && c1 < c_hi) y[c1 + m_off] = TI(c.y * scale * winv[c1]);
  }
}

// ---------------------------------------------------------------- transposed: E4 in four steps
// Blocks whose transform does not fit one workgroup, P = P1 P2.  With a_k the
// packed half spectrum of inv_fft_kernel, k = k1 + P1 k2 and j = j2 + P2 j1,
//   c_j = sum_k1 w_P1^(j1 k1) [ w_P^(j2 k1) sum_k2 w_P2^(j2 k2) a_(k1 + P1 k2) ]
// (w_n = exp(2 pi i / n)).  inv_fft4_col_kernel: per right-hand side and group
// of 2^lb1 consecutive k1, the P2-point transforms over k2 (interleaved in LDS,
// point k2 of transform t at lds[(k2 << lb) + t]), times w_P^(j2 k1), written to
// W[j2 P1 + k1].  inv_fft4_row_kernel: per group of 2^lb2 consecutive j2, the
// P1-point transforms over k1, then g_2j + i g_(2j+1) = c_j is divided by the
// window on the retained columns (eq. Fe2).  Workgroup b takes right-hand side
// b / groups and group b % groups.
template <typename T, typename TI>
__global__ __launch_bounds__(FFT_MAX_THREADS) void inv_fft4_col_kernel(InvFft4Args<T, TI> a) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lb = a.lb1, tmask = (1 << lb) - 1;
  const int groups = (a.P1 + tmask) >> lb;
  const int r = (int)blockIdx.x / groups;
  const int k1_0 = ((int)blockIdx.x - r * groups) << lb;
  const cplx_t<TI>* __restrict__ u = a.U + (int64_t)r * a.ldu;
  const int pts = a.P2 << lb;
  for (int i = tid; i < pts; i += nt) {
    const int k2 = i >> lb, k1 = k1_0 + (i & tmask);
    C v = C{T(0), T(0)};
    if (k1 < a.P1) {
      const int k = k1 + a.P1 * k2;
      const C uk = C{T(u[k].x), T(u[k].y)};
      C um = C{T(u[a.P - k].x), T(u[a.P - k].y)};
      um.y = -um.y;  // conj U_(P-k)
      const C ge = cadd(uk, um);
      const C go = cmul(csub(uk, um), a.post[k]);
      v = C{ge.x - go.y, ge.y + go.x};  // ge + i go
    }
    lds[i] = v;
  }
  __syncthreads();
  // w_P2 = w_P^P1: the length-P table at index scale P1
  run_fft<+1, true>(lds, a.P2, lb, a.f2.npass, a.f2.radix, a.tw, a.P1, tid, nt, true);
  C* __restrict__ w = a.W + (int64_t)r * a.P;
  for (int i = tid; i < pts; i += nt) {
    const int j2 = i >> lb, k1 = k1_0 + (i & tmask);
    if (k1 < a.P1) w[(int64_t)j2 * a.P1 + k1] = cmul(lds[i], to_c<C>(twiddle(a.tw, j2 * k1)));
  }
}

template <typename T, typename TI>
__global__ __launch_bounds__(FFT_MAX_THREADS) void inv_fft4_row_kernel(InvFft4Args<T, TI> a) {
  using C = cplx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lb = a.lb2, tmask = (1 << lb) - 1;
  const int groups = (a.P2 + tmask) >> lb;
  const int r = (int)blockIdx.x / groups;
  const int j2_0 = ((int)blockIdx.x - r * groups) << lb;
  const int ncol = min(1 << lb, a.P2 - j2_0);
  // the group's rows W[j2_0 .. j2_0 + ncol - 1][*] are contiguous
  const C* __restrict__ w = a.W + (int64_t)r * a.P + (int64_t)j2_0 * a.P1;
  const int pts = a.P1 << lb;
  for (int i = tid; i < pts; i += nt) {
    const int t = i / a.P1, k1 = i - t * a.P1;
    lds[(k1 << lb) + t] = t < ncol ? w[i] : C{T(0), T(0)};
  }
  __syncthreads();
  // w_P1 = w_P^P2
  run_fft<+1, true>(lds, a.P1, lb, a.f1.npass, a.f1.radix, a.tw, a.P2, tid, nt, true);
  TI* __restrict__ y = a.Y + (int64_t)r * a.N;
  for (int i = tid; i < pts; i += nt) {
    const int j1 = i >> lb, t = i & tmask;
    if (t >= ncol) continue;
    const int j = j2_0 + t + a.P2 * j1;
    const C c = lds[i];
    const int c0 = 2 * j, c1 = 2 * j + 1;
    if (c0 >= a.c_lo && c0 < a.c_hi) y[c0 + a.m_off] = TI(c.x * a.scale * a.winv[c0]);
    if (c1 >= a.c_lo && c1 < a.c_hi) y[c1 + a.m_off] = TI(c.y * a.scale * a.winv[c1]);
  }
}

// ---------------------------------------------------------------- precompute: P5
// One workgroup per row: F of a windowed row (float64), half spectrum out.
__global__ __launch_bounds__(FFT_MAX_THREADS) void row_fft_kernel(RowFftArgs a, FftPlan fp) {
  using C = double2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t row = blockIdx.x;
  const double* __restrict__ v = a.rows + row * a.L;
  for (int j = tid; j < a.P; j += nt) lds[j] = C{v[2 * j], v[2 * j + 1]};
  __syncthreads();
  run_fft<-1>(lds, fp, a.tw, tid, nt);
  C* __restrict__ s = a.spec + row * (a.P + 1);
  for (int k = tid; k <= a.P; k += nt) s[k] = unpack<-1>(lds, a.P, k, a.post, a.scale);
}

// points, then (float32) the two twiddle tables of 128 + P / 128 + 1 entries


template <typename K>
void set_lds(K kernel, size_t bytes) {
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

// Allow every FFT kernel the whole LDS of a workgroup (once per device; kept
// out of the launch path so that launches can be captured in graphs).
void init_fft_kernels(size_t max_lds) {
  static std::vector<int> done;
  int dev = 0;
  SPT_HIP(hipGetDevice(&dev));
  for (int d : done)
    if (d == dev) return;
  set_lds(exec_fft_kernel<double>, max_lds);
  set_lds(exec_fft_kernel<float>, max_lds);
  set_lds(inv_fft_kernel<double>, max_lds);
  set_lds(inv_fft_kernel<float>, max_lds);
  set_lds(inv_fft_multi_kernel<double>, max_lds);
  set_lds(inv_fft_multi_kernel<double, float>, max_lds);
  set_lds(inv_fft_multi_kernel<float>, max_lds);
  set_lds(inv_fft4_col_kernel<double, double>, max_lds);
  set_lds(inv_fft4_col_kernel<float, float>, max_lds);
  set_lds(inv_fft4_col_kernel<double, float>, max_lds);
  set_lds(inv_fft4_row_kernel<double, double>, max_lds);
  set_lds(inv_fft4_row_kernel<float, float>, max_lds);
  set_lds(inv_fft4_row_kernel<double, float>, max_lds);
  set_lds(row_fft_kernel, max_lds);
  set_lds(exec_fft_multi_kernel<double, double, false, 512>, max_lds);
  set_lds(exec_fft_multi_kernel<float, float, false, 512>, max_lds);
  set_lds(exec_fft_multi_kernel<float, float, true, 512>, max_lds);
  set_lds(exec_fft_multi_kernel<double, float, true, 512>, max_lds);
  set_lds(exec_fft_multi_kernel<double, float, false, 512>, max_lds);
  set_lds(exec_fft_multi_kernel<double, double, false, 768>, max_lds);
  set_lds(exec_fft_multi_kernel<double, float, true, 768>, max_lds);
  set_lds(exec_fft_multi_kernel<double, float, false, 768>, max_lds);
  set_lds(exec_fft_multi_kernel<double, double, false, 1024>, max_lds);
  set_lds(exec_fft_multi_kernel<float, float, false, 1024>, max_lds);
  set_lds(exec_fft_multi_kernel<float, float, true, 1024>, max_lds);
  set_lds(exec_fft_multi_kernel<double, float, true, 1024>, max_lds);
  set_lds(exec_fft_multi_kernel<double, float, false, 1024>, max_lds);
  done.push_back(dev);
}

FftPlan make_fft_plan(int P, bool radix10) {
  FftPlan fp;
  fp.P = P;
  int n = P;
  // radix 8 first (fewest passes), then 4 / 2, then 3 and 5
  std::vector<int> rad;
  while (n % 8 == 0) { rad.push_back(8); n /= 8; }
  while (n % 4 == 0) { rad.push_back(4); n /= 4; }
  while (n % 2 == 0) { rad.push_back(2); n /= 2; }
  while (n % 3 == 0) { rad.push_back(3); n /= 3; }
  while (n % 5 == 0) { rad.push_back(5); n /= 5; }
  if (n != 1) throw Error(SPT_E_UNSUPPORTED, "FFT length half " + std::to_string(P) +
                                                 " is not 2^a 3^b 5^c");
  // a lone radix 2 and a radix 5 become one radix-10 pass (one LDS round trip
  // fewer) for the kernels that take radix 10 (the fused FFT)
  const auto two = std::find(rad.begin(), rad.end(), 2);
  const auto five = std::find(rad.begin(), rad.end(), 5);
  if (radix10 && two != rad.end() && five != rad.end()) {
    *five = 10;
    rad.erase(two);
  }
  if ((int)rad.size() > MAX_PASSES) throw Error(SPT_E_UNSUPPORTED, "too many FFT passes");
  fp.npass = (int)rad.size();
  for (int i = 0; i < fp.npass; ++i) fp.radix[i] = rad[i];
  int t = (P + FFT_EPT - 1) / FFT_EPT;
  t = ((t + 63) / 64) * 64;
  if (t < 64) t = 64;
  if (t > FFT_MAX_THREADS)
    throw Error(SPT_E_UNSUPPORTED, "FFT length half " + std::to_string(P) +
                                       " exceeds the single-workgroup FFT");
  fp.threads = t;
  return fp;
}

template <typename T>
void launch_exec_fft(const ExecFftArgs<T>& a, const FftPlan& fp, hipStream_t s) {
  const size_t lds = sizeof(cplx_t<T>) * (size_t)a.P;
  hipLaunchKernelGGL(exec_fft_kernel<T>, dim3(a.R), dim3(fp.threads), lds, s, a, fp);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_inv_fft(const InvFftArgs<T>& a, const FftPlan& fp, hipStream_t s) {
  const size_t lds = sizeof(cplx_t<T>) * (size_t)a.P;
  hipLaunchKernelGGL(inv_fft_kernel<T>, dim3(a.R), dim3(fp.threads), lds, s, a, fp);
  SPT_HIP(hipGetLastError());
}

void launch_row_fft(const RowFftArgs& a, const FftPlan& fp, hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)a.P;
  hipLaunchKernelGGL(row_fft_kernel, dim3(a.nrows), dim3(fp.threads), lds, s, a, fp);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_exec_fft_multi(const FftDesc<T>* descs, const FftGrid& g, int threads, size_t lds,
                           const T* X, cplx_t<T>* Z, int R, int64_t N, hipStream_t s) {
  const dim3 grid(g.wg0[g.nblk]);
  // float64 between 512 and 768 threads: the 768-thread build (no spills)
  constexpr int MID = std::is_same<T, double>::value ? 768 : 1024;
  if (threads <= 512)
    hipLaunchKernelGGL((exec_fft_multi_kernel<T, T, false, 512>), grid, dim3(threads), lds, s,
                       descs, g, X, Z, (uint32_t*)nullptr, (int64_t)0, R, N);
  else if (threads <= MID)
    hipLaunchKernelGGL((exec_fft_multi_kernel<T, T, false, MID>), grid, dim3(threads), lds, s,
                       descs, g, X, Z, (uint32_t*)nullptr, (int64_t)0, R, N);
  else
    hipLaunchKernelGGL((exec_fft_multi_kernel<T, T, false, 1024>), grid, dim3(threads), lds, s,
                       descs, g, X, Z, (uint32_t*)nullptr, (int64_t)0, R, N);
  SPT_HIP(hipGetLastError());
}

void launch_exec_fft_multi_split(const FftDesc<float>* descs, const FftGrid& g, int threads,
                                 size_t lds, const float* X, uint32_t* Zs, int64_t zplane, int R,
                                 int64_t N, hipStream_t s) {
  const dim3 grid(g.wg0[g.nblk]);
  if (threads <= 512)
    hipLaunchKernelGGL((exec_fft_multi_kernel<float, float, true, 512>), grid, dim3(threads), lds,
                       s, descs, g, X, (float2*)nullptr, Zs, zplane, R, N);
  else
    hipLaunchKernelGGL((exec_fft_multi_kernel<float, float, true, 1024>), grid, dim3(threads),
                       lds, s, descs, g, X, (float2*)nullptr, Zs, zplane, R, N);
  SPT_HIP(hipGetLastError());
}

void launch_exec_fft_multi_x32(const FftDesc<double>* descs, const FftGrid& g, int threads,
                               size_t lds, const float* X, float2* Z, uint32_t* Zs,
                               int64_t zplane, int R, int64_t N, hipStream_t s) {
  const dim3 grid(g.wg0[g.nblk]);
  if (Zs) {
    if (threads <= 512)
      hipLaunchKernelGGL((exec_fft_multi_kernel<double, float, true, 512>), grid, dim3(threads),
                         lds, s, descs, g, X, (float2*)nullptr, Zs, zplane, R, N);
    else if (threads <= 768)
      hipLaunchKernelGGL((exec_fft_multi_kernel<double, float, true, 768>), grid, dim3(threads),
                         lds, s, descs, g, X, (float2*)nullptr, Zs, zplane, R, N);
    else
      hipLaunchKernelGGL((exec_fft_multi_kernel<double, float, true, 1024>), grid, dim3(threads),
                         lds, s, descs, g, X, (float2*)nullptr, Zs, zplane, R, N);
  } else {
    if (threads <= 512)
      hipLaunchKernelGGL((exec_fft_multi_kernel<double, float, false, 512>), grid, dim3(threads),
                         lds, s, descs, g, X, Z, (uint32_t*)nullptr, (int64_t)0, R, N);
    else if (threads <= 768)
      hipLaunchKernelGGL((exec_fft_multi_kernel<double, float, false, 768>), grid, dim3(threads),
                         lds, s, descs, g, X, Z, (uint32_t*)nullptr, (int64_t)0, R, N);
    else
      hipLaunchKernelGGL((exec_fft_multi_kernel<double, float, false, 1024>), grid,
                         dim3(threads), lds, s, descs, g, X, Z, (uint32_t*)nullptr, (int64_t)0, R,
                         N);
  }
  SPT_HIP(hipGetLastError());
}

template void launch_exec_fft_multi<double>(const FftDesc<double>*, const FftGrid&, int, size_t,
                                            const double*, double2*, int, int64_t, hipStream_t);
template void launch_exec_fft_multi<float>(const FftDesc<float>*, const FftGrid&, int, size_t,
                                           const float*, float2*, int, int64_t, hipStream_t);
template void launch_exec_fft<double>(const ExecFftArgs<double>&, const FftPlan&, hipStream_t);
template void launch_exec_fft<float>(const ExecFftArgs<float>&, const FftPlan&, hipStream_t);
template void launch_inv_fft<double>(const InvFftArgs<double>&, const FftPlan&, hipStream_t);
template void launch_inv_fft<float>(const InvFftArgs<float>&, const FftPlan&, hipStream_t);

// threads for pts points of batched transforms (FFT_EPT per thread)
static int batch_threads(int pts) {
  int t = (pts + FFT_EPT - 1) / FFT_EPT;
  t = ((t + 63) / 64) * 64;
  return t < 64 ? 64 : t;
}

template <typename T, typename TI>
void launch_inv_fft4(const InvFft4Args<T, TI>& a, hipStream_t s) {
  const int p1 = a.P2 << a.lb1, p2 = a.P1 << a.lb2;
  if (p1 > FFT_EPT * FFT_MAX_THREADS || p2 > FFT_EPT * FFT_MAX_THREADS)
    throw Error(SPT_E_INVALID_ARG, "four-step inverse transform groups exceed one workgroup");
  const int64_t g1 = (int64_t)a.R * ((a.P1 + (1 << a.lb1) - 1) >> a.lb1);
  const int64_t g2 = (int64_t)a.R * ((a.P2 + (1 << a.lb2) - 1) >> a.lb2);
  if (g1 > INT32_MAX || g2 > INT32_MAX) throw Error(SPT_E_INVALID_ARG, "too many right-hand sides");
  hipLaunchKernelGGL((inv_fft4_col_kernel<T, TI>), dim3((unsigned)g1), dim3(batch_threads(p1)),
                     sizeof(cplx_t<T>) * (size_t)p1, s, a);
  SPT_HIP(hipGetLastError());
  hipLaunchKernelGGL((inv_fft4_row_kernel<T, TI>), dim3((unsigned)g2), dim3(batch_threads(p2)),
                     sizeof(cplx_t<T>) * (size_t)p2, s, a);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_inv_fft_multi(const InvFftDesc<T>* descs, int nblk, int threads, size_t lds,
                          const cplx_t<T>* U, T* Y, int R, int64_t N, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL(inv_fft_multi_kernel<T>, dim3(R, nblk), dim3(threads), lds, s, descs, U, Y,
                     R, N);
  SPT_HIP(hipGetLastError());
}

void launch_inv_fft_multi_x32(const InvFftDesc<double>* descs, int nblk, int threads, size_t lds,
                              const float2* U, float* Y, int R, int64_t N, hipStream_t s) {
  if (nblk <= 0) return;
  hipLaunchKernelGGL((inv_fft_multi_kernel<double, float>), dim3(R, nblk), dim3(threads), lds, s,
                     descs, U, Y, R, N);
  SPT_HIP(hipGetLastError());
}

template void launch_inv_fft_multi<double>(const InvFftDesc<double>*, int, int, size_t,
                                           const double2*, double*, int, int64_t, hipStream_t);
template void launch_inv_fft_multi<float>(const InvFftDesc<float>*, int, int, size_t,
                                          const float2*, float*, int, int64_t, hipStream_t);
template void launch_inv_fft4<double, double>(const InvFft4Args<double, double>&, hipStream_t);
template void launch_inv_fft4<float, float>(const InvFft4Args<float, float>&, hipStream_t);
template void launch_inv_fft4<double, float>(const InvFft4Args<double, float>&, hipStream_t);

}  // namespace spt
