// Device building blocks of the FFTs (shared by the FFT kernels and the
// persistent executor): complex helpers, in-register DFTs of radix 2, 3, 4, 5,
// 8 and 10, a batched LDS Stockham radix pass, two leading radix-8 passes
// joined by an exchange of lane shuffles, and the unpacking of a packed real
// transform into its half spectrum.
//
// Conventions: F of eq. (1) has the kernel exp(-2 pi i jk/L)/sqrt(L) (SIGN -1,
// used by the precomputation A_e W F); the computation stage applies F*
// (SIGN +1).  stockham_pass takes its twiddles exp(+2 pi i q/Pt) from two
// float64 tables of 128 + Pt/128 entries for the block's length Pt (w^q =
// lo[q % 128] hi[q / 128]; a sub-transform of length P < Pt uses index
// q * (Pt / P)); a butterfly forms w^jm once and its powers in float64, for
// every precision.  SIGN -1 uses the conjugates.
#pragma once

#include "common.hpp"

namespace spt {
namespace fftcore {

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by SIGN * i
template <int SIGN, typename C>
__device__ __forceinline__ C mul_si(C a) {
  return SIGN > 0 ? C{-a.y, a.x} : C{a.y, -a.x};
}

// In-register DFTs X_k = sum_n x_n exp(SIGN 2 pi i n k / R).
template <int SIGN, int R, typename C>
struct Dft;

template <int SIGN, typename C>
struct Dft<SIGN, 2, C> {
  __device__ __forceinline__ static void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int SIGN, typename C>
struct Dft<SIGN, 4, C> {
  __device__ __forceinline__ static void run(C* v) {
    C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    C s13 = cadd(v[1], v[3]), d13 = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  }
};

template <int SIGN, typename C>
struct Dft<SIGN, 8, C> {
  __device__ __forceinline__ static void run(C* v) {
    using T = decltype(v[0].x);
    const T h = T(0.70710678118654752440);  // 1/sqrt(2)
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Dft<SIGN, 4, C>::run(e);
    Dft<SIGN, 4, C>::run(o);
    // o_k *= exp(SIGN i pi k / 4)
    C o1 = C{h * (o[1].x - SIGN * o[1].y), h * (o[1].y + SIGN * o[1].x)};
    C o2 = mul_si<SIGN>(o[2]);
    C o3 = C{h * (-o[3].x - SIGN * o[3].y), h * (-o[3].y + SIGN * o[3].x)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <int SIGN, typename C>
struct Dft<SIGN, 3, C> {
  __device__ __forceinline__ static void run(C* v) {
    using T = decltype(v[0].x);
    const T s3 = T(0.86602540378443864676);  // sqrt(3)/2
    C t = cadd(v[1], v[2]);
    C d = csub(v[1], v[2]);
    C m = C{v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
    C r = mul_si<SIGN>(C{s3 * d.x, s3 * d.y});
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
};

template <int SIGN, typename C>
struct Dft<SIGN, 5, C> {
  __device__ __forceinline__ static void run(C* v) {
    using T = decltype(v[0].x);
    const T c1 = T(0.30901699437494742410);   // cos(2 pi/5)
    const T c2 = T(-0.80901699437494742410);  // cos(4 pi/5)
    const T s1 = T(0.95105651629515357212);   // sin(2 pi/5)
    const T s2 = T(0.58778525229247312917);   // sin(4 pi/5)
    C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    C d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    C a1 = C{v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    C a2 = C{v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    C b1 = mul_si<SIGN>(C{s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y});
    C b2 = mul_si<SIGN>(C{s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y});
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// radix 10 as two radix-5 DFTs of the even and odd points and one radix-2
// step: X_k = E_k + w^k O_k, X_(k+5) = E_k - w^k O_k, w = exp(SIGN 2 pi i / 10)
template <int SIGN, typename C>
struct Dft<SIGN, 10, C> {
  __device__ __forceinline__ static void run(C* v) {
    using T = decltype(v[0].x);
    const T c[5] = {T(1), T(0.80901699437494742410), T(0.30901699437494742410),
                    T(-0.30901699437494742410), T(-0.80901699437494742410)};
    const T sn[5] = {T(0), T(0.58778525229247312917), T(0.95105651629515357212),
                     T(0.95105651629515357212), T(0.58778525229247312917)};
    C e[5] = {v[0], v[2], v[4], v[6], v[8]};
    C o[5] = {v[1], v[3], v[5], v[7], v[9]};
    Dft<SIGN, 5, C>::run(e);
    Dft<SIGN, 5, C>::run(o);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const C t = k == 0 ? o[0]
                         : C{o[k].x * c[k] - SIGN * o[k].y * sn[k],
                             o[k].y * c[k] + SIGN * o[k].x * sn[k]};
      v[k] = cadd(e[k], t);
      v[k + 5] = csub(e[k], t);
    }
  }
};

// two-level twiddle table of a length P: tw[i] = exp(2 pi i i / P) for
// i < TW_LO, tw[TW_LO + i] = exp(2 pi i TW_LO i / P) for i <= P / TW_LO
constexpr int TW_LO_BITS = 7;
constexpr int TW_LO = 1 << TW_LO_BITS;
// elements of the transforms per thread (workgroups are sized so that
// threads >= elements / FFT_EPT)
constexpr int FFT_EPT = 10;

template <typename C>
__device__ __forceinline__ C to_c(double2 t) {
  using T = decltype(C{}.x);
  return C{(T)t.x, (T)t.y};
}

// w^q of the length-Pt table (two-level, float64)
__device__ __forceinline__ double2 twiddle(const double2* __restrict__ tw, int q) {
  return cmul(tw[q & (TW_LO - 1)], tw[TW_LO + (q >> TW_LO_BITS)]);
}

// One Stockham pass of radix R over 2^lb transforms of length P in LDS (in
// place through registers).  BATCH == false: one transform, point j at lds[j].
// BATCH == true: the transforms are interleaved, point j of transform t at
// lds[(j << lb) + t], so neighbouring lanes touch neighbouring words.
// Butterflies are spread over the nt threads; requires 2^lb * P <= EPT * nt,
// so a thread owns at most ceil(EPT / R) butterflies.  tmul scales the
// twiddle index when P divides the length of the table.
template <int SIGN, int R, bool BATCH, int EPT, typename C>
__device__ __forceinline__ void stockham_pass(C* lds, int P, int lb, int Ns,
                                              const double2* __restrict__ tw, int tmul, int tid,
                                              int nt, bool active) {
  constexpr int MAXB = (EPT + R - 1) / R;
  const int nb = P / R;
  const int nbt = BATCH ? nb << lb : nb;
  const int tmask = BATCH ? (1 << lb) - 1 : 0;
  auto at = [&](int j, int t) { return BATCH ? (j << lb) + t : j; };
  C v[MAXB][R];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int u = tid + b * nt;
    if (active && u < nbt) {
      const int j = BATCH ? u >> lb : u, t = u & tmask;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = lds[at(j + r * nb, t)];
    }
  }
  __syncthreads();
  const int stride = P / (Ns * R) * tmul;
  // j mod Ns by a multiply-high: with m = ceil(2^32 / Ns), umulhi(j, m) =
  // floor(j / Ns) exactly while j Ns < 2^32 (j and Ns are below P, and a
  // workgroup's transform has P < 2^16 points); Ns = 1 (m would be 2^32) is
  // the first pass, whose jm is 0
  const uint32_t mag = Ns > 1 ? 0xFFFFFFFFu / (uint32_t)Ns + 1u : 0u;
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int u = tid + b * nt;
    if (active && u < nbt) {
      const int j = BATCH ? u >> lb : u, t = u & tmask;
      const int jm = Ns > 1 ? j - (int)__umulhi((uint32_t)j, mag) * Ns : 0;
      if (Ns > 1) {
        // w^(jm r) = (w^jm)^r, powers in float64
        double2 t1 = twiddle(tw, jm * stride);
        if (SIGN < 0) t1.y = -t1.y;
        double2 w = t1;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[b][r] = cmul(v[b][r], to_c<C>(w));
          if (r + 1 < R) w = cmul(w, t1);
        }
      }
      Dft<SIGN, R, C>::run(v[b]);
      const int base = (j - jm) * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[at(base + r * Ns, t)] = v[b][r];
    }
  }
  __syncthreads();
}

// v from lane (lane ^ S) of the same group of 8 lanes: S = 1 and 2 by DPP
// quad permutations, S = 4 by a bit-mode LDS swizzle (xor 4 within 32 lanes;
// no LDS memory).  Every lane of a group must be active.
template <int S>
__device__ __forceinline__ int xor_lane_i(int v) {
  static_assert(S == 1 || S == 2 || S == 4, "lane partner");
  if constexpr (S == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  if constexpr (S == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  return __builtin_amdgcn_ds_swizzle(v, (S << 10) | 0x1F);  // and 0x1f, or 0, xor S
}
template <int S>
__device__ __forceinline__ float xor_lane(float v) {
  return __builtin_bit_cast(float, xor_lane_i<S>(__builtin_bit_cast(int, v)));
}
template <int S>
__device__ __forceinline__ double xor_lane(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)xor_lane_i<S>((int)(unsigned)u);
  const unsigned hi = (unsigned)xor_lane_i<S>((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// 8 x 8 transpose over a group of 8 lanes: lane c ends with element c of every
// lane's eight.  Stage S exchanges, between lanes c and c ^ S, the elements
// whose index differs from the lane in bit S; after the three stages element
// i of lane c has moved to element c of lane i.
template <int S, typename C>
__device__ __forceinline__ void transpose8_stage(C* v, int c) {
  using T = decltype(v[0].x);
  const bool hi = (c & S) != 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (i & S) continue;
    const T sx = hi ? v[i].x : v[i | S].x, sy = hi ? v[i].y : v[i | S].y;
    const T rx = xor_lane<S>(sx), ry = xor_lane<S>(sy);
    if (hi) {
      v[i].x = rx;
      v[i].y = ry;
    } else {
      v[i | S].x = rx;
      v[i | S].y = ry;
    }
  }
}

// The first two passes (radix 8, then radix 8 with Ns = 8) of one transform
// of length P in LDS, with one LDS round trip instead of two.  The second
// pass's butterfly 8g + c takes element c of the first pass's butterflies
// g + r M (r < 8, M = P / 64); lane c of an 8-lane group g holds butterfly
// g + c M, so after the first DFT the group exchanges its 64 values in
// registers (transpose8) and runs the second pass's twiddles and DFT.
// Requires P % 64 == 0 and P / 8 <= ceil(EPT / 8) nt, and nt a multiple of 8
// (groups are then all active or all idle).
template <int SIGN, int EPT, typename C>
__device__ __forceinline__ void stockham_pass88(C* lds, int P, const double2* __restrict__ tw,
                                                int tmul, int tid, int nt, bool active) {
  constexpr int MAXB = (EPT + 7) / 8;
  const int nb = P / 8, M = P / 64;
  C v[MAXB][8];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int u = tid + b * nt;
    if (active && u < nb) {
      const int j = (u >> 3) + (u & 7) * M;
#pragma unroll
      for (int r = 0; r < 8; ++r) v[b][r] = lds[j + r * nb];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int u = tid + b * nt;
    if (active && u < nb) {
      const int g = u >> 3, c = u & 7;
      Dft<SIGN, 8, C>::run(v[b]);
      transpose8_stage<1>(v[b], c);
      transpose8_stage<2>(v[b], c);
      transpose8_stage<4>(v[b], c);
      if (c > 0) {
        // w^(c r) with w = exp(SIGN 2 pi i M / P), powers in float64
        double2 t1 = twiddle(tw, c * M * tmul);
        if (SIGN < 0) t1.y = -t1.y;
        double2 w = t1;
#pragma unroll
        for (int r = 1; r < 8; ++r) {
          v[b][r] = cmul(v[b][r], to_c<C>(w));
          if (r + 1 < 8) w = cmul(w, t1);
        }
      }
      Dft<SIGN, 8, C>::run(v[b]);
#pragma unroll
      for (int r = 0; r < 8; ++r) lds[64 * g + c + 8 * r] = v[b][r];
    }
  }
  __syncthreads();
}

// all passes; threads with active == false only take part in the barriers.
// R10: the plan may hold radix-10 passes (make_fft_plan(P, true)); the other
// kernels leave them out, which keeps their registers down.  Those kernels
// (single transforms) also take two leading radix-8 passes together
// (stockham_pass88).
template <int SIGN, bool BATCH, int EPT = FFT_EPT, bool R10 = false, typename C>
__device__ __forceinline__ void run_fft(C* lds, int P, int lb, int npass, const int* radix,
                        const double2* __restrict__ tw, int tmul, int tid, int nt, bool active) {
  int Ns = 1;
  int p0 = 0;
  if (R10 && !BATCH && npass >= 2 && radix[0] == 8 && radix[1] == 8) {
    stockham_pass88<SIGN, EPT>(lds, P, tw, tmul, tid, nt, active);
    Ns = 64;
    p0 = 2;
  }
  for (int p = p0; p < npass; ++p) {
    const int R = radix[p];
    if (R10 && R == 10) {
      stockham_pass<SIGN, R10 ? 10 : 2, BATCH, EPT>(lds, P, lb, Ns, tw, tmul, tid, nt, active);
      Ns *= R;
      continue;
    }
    switch (R) {
      case 8: stockham_pass<SIGN, 8, BATCH, EPT>(lds, P, lb, Ns, tw, tmul, tid, nt, active); break;
      case 4: stockham_pass<SIGN, 4, BATCH, EPT>(lds, P, lb, Ns, tw, tmul, tid, nt, active); break;
      case 2: stockham_pass<SIGN, 2, BATCH, EPT>(lds, P, lb, Ns, tw, tmul, tid, nt, active); break;
      case 5: stockham_pass<SIGN, 5, BATCH, EPT>(lds, P, lb, Ns, tw, tmul, tid, nt, active); break;
      default: stockham_pass<SIGN, 3, BATCH, EPT>(lds, P, lb, Ns, tw, tmul, tid, nt, active); break;
    }
    Ns *= R;
  }
}

template <int SIGN, typename C>
__device__ __forceinline__ void run_fft(C* lds, const FftPlan& fp, const double2* __restrict__ tw,
                                        int tid, int nt) {
  run_fft<SIGN, false, FFT_EPT>(lds, fp.P, 0, fp.npass, fp.radix, tw, 1, tid, nt, true);
}

// Unpack the packed length-P transform C into the half spectrum of the real
// length-2P vector: Z_k = E_k + exp(SIGN i pi k/P) O_k, with
// E_k = (C_k + conj C_{P-k})/2 and O_k = (C_k - conj C_{P-k})/(2i);
// t = exp(+i pi k/P).
template <int SIGN, typename C, typename T>
__device__ __forceinline__ C unpack_with(const C* lds, int P, int k, C t, T scale) {
  C ck = lds[k == P ? 0 : k];
  C cm = lds[k == 0 ? 0 : P - k];
  cm.y = -cm.y;
  C e = C{T(0.5) * (ck.x + cm.x), T(0.5) * (ck.y + cm.y)};
  C d = C{T(0.5) * (ck.x - cm.x), T(0.5) * (ck.y - cm.y)};
  C o = C{d.y, -d.x};  // d / i
  if (SIGN < 0) t.y = -t.y;
  C z = cadd(e, cmul(t, o));
  return C{z.x * scale, z.y * scale};
}

template <int SIGN, typename C, typename T>
__device__ __forceinline__ C unpack(const C* lds, int P, int k, const C* __restrict__ post,
                                    T scale) {
  return unpack_with<SIGN>(lds, P, k, post[k], scale);
}

}  // namespace fftcore
}  // namespace spt
