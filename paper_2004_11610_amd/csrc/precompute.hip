// Precomputation kernels (float64): quadrature nodes and weights, rows of the
// extended matrix A_e times the window (Alg. 1 step 1.2, sec. 3), the maximum
// of |A_e W F| and the threshold eps1 * max (Alg. 1 step 1.3), band extents and
// packing of the kept entries into row tiles.

#include "common.hpp"
#include "spmm_core.hpp"

namespace spt {
namespace {

constexpr double LN2 = 0.69314718055994530942;
// ln 2 = LN2_HI + LN2_LO: LN2_HI = round(2^32 ln 2) / 2^32 has 32 significant
// bits, so n * LN2_HI is exact for |n| < 2^21; LN2_LO is the rounded remainder.
constexpr double LN2_HI = 0x1.62e42ff000000p-1;
constexpr double LN2_LO = -0x1.718432a1b0e26p-35;
constexpr double BIG = 0x1p500;
constexpr double RESCALE = 0x1p-500;

// exp(-a) = mant * 2^E, a >= 0, with the Cody-Waite reduction a = E' ln 2 + r
__device__ __forceinline__ void exp_neg_scaled(double a, double& mant, int& E) {
  const double n = rint(a * (1.0 / LN2));
  double r = fma(-n, LN2_HI, a);
  r = fma(-n, LN2_LO, r);
  mant = exp(-r);
  E = -(int)n;
}

// Recurrence state of one row, advanced one degree at a time.
struct RowRec {
  int family, power;
  double x, p_prev, p, scale;  // value = p * 2^E * scale
  int E;
  int m;                       // degree of p
  int64_t j, N;                // node index (Chebyshev)

  __device__ void init(const FamilyArgs& f, int64_t jj) {
    family = f.family;
    power = f.power;
    j = jj;
    N = f.N;
    x = f.x[jj];
    m = 0;
    E = 0;
    p_prev = 0.0;
    scale = 1.0;
    if (family == SPT_LEGENDRE || family == SPT_JACOBI) {
      p = f.p0;
      if (f.rowscale) scale = f.rowscale[jj];
    } else if (family == SPT_LAGUERRE_FN) {
      exp_neg_scaled(0.5 * x, p, E);
    } else if (family == SPT_HERMITE_FN) {
      const double hi = x * x;
      const double lo = fma(x, x, -hi);
      exp_neg_scaled(0.5 * hi, p, E);
      p *= (1.0 - 0.5 * lo) * 0.75112554446494248286;  // pi^{-1/4}
    } else {
      p = 1.0;
    }
  }
  // value at degree mm of a trigonometric generator: closed form with an exact
  // angle, m theta_j = pi q / (2N) with q = m (2j+1) mod 4N
  __device__ double trig(int64_t mm) const {
    const int64_t fourN = 4 * N;
    int64_t q = ((mm % fourN) * ((2 * j + 1) % fourN)) % fourN;
    if (q < 0) q += fourN;
    const double a = (double)q / (double)(2 * N);
    if (family == SPT_SINE) return sinpi(a);
    const double c = cospi(a);
    if (family == SPT_COS_POWER) {
      double v = c;
      for (int i = 1; i < power; ++i) v *= c;
      return v;
    }
    return c;
  }
  __device__ double value() const { return ldexp(p, E) * scale; }
  __device__ void advance(const FamilyArgs& f) {
    double nxt;
    if (family == SPT_LEGENDRE || family == SPT_JACOBI) {
      nxt = ((x - f.cb[m]) * p - f.ca[m] * p_prev) / f.ca[m + 1];
    } else if (family == SPT_LAGUERRE_FN) {
      nxt = ((2.0 * m + 1.0 - x) * p - (double)m * p_prev) / (double)(m + 1);
    } else {  // Hermite functions
      nxt = f.ca[m] * x * p - f.cb[m] * p_prev;
    }
    p_prev = p;
    p = nxt;
    ++m;
    if (fabs(p) > BIG) {
      p *= RESCALE;
      p_prev *= RESCALE;
      E += 500;
    }
  }
};

// ---------------------------------------------------------------- nodes
// Gauss nodes: bisection with Sturm counts on the symmetric tridiagonal Jacobi
// matrix (diag d_i, squared off-diagonal e_i^2), then Newton on the degree-N
// polynomial by its recurrence.  Chebyshev-Gauss nodes in closed form.
__device__ int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int64_t n,
                           double lam, double pivmin) {
  int cnt = 0;
  double q = d[0] - lam;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int64_t i = 1; i < n; ++i) {
    q = (d[i] - lam) - e2[i] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// (p_N, p_N') up to a common positive factor
__device__ void poly_and_derivative(const FamilyArgs& f, double x, double& pn, double& dpn) {
  double p_prev = 0.0, p = 1.0, d_prev = 0.0, d = 0.0;
  const int64_t N = f.N;
  if (f.family == SPT_LEGENDRE || f.family == SPT_JACOBI) p = f.p0;
  for (int64_t m = 0; m < N; ++m) {
    double pn1, dn1;
    if (f.family == SPT_LEGENDRE || f.family == SPT_JACOBI) {
      pn1 = ((x - f.cb[m]) * p - f.ca[m] * p_prev) / f.ca[m + 1];
      dn1 = ((x - f.cb[m]) * d + p - f.ca[m] * d_prev) / f.ca[m + 1];
    } else if (f.family == SPT_LAGUERRE_FN) {
      pn1 = ((2.0 * m + 1.0 - x) * p - (double)m * p_prev) / (double)(m + 1);
      dn1 = ((2.0 * m + 1.0 - x) * d - p - (double)m * d_prev) / (double)(m + 1);
    } else {
      pn1 = f.ca[m] * x * p - f.cb[m] * p_prev;
      dn1 = f.ca[m] * (p + x * d) - f.cb[m] * d_prev;
    }
    p_prev = p;
    p = pn1;
    d_prev = d;
    d = dn1;
    if (fmax(fabs(p), fabs(d)) > BIG) {
      p *= RESCALE;
      p_prev *= RESCALE;
      d *= RESCALE;
      d_prev *= RESCALE;
    }
  }
  pn = p;
  dpn = d;
}

// double-double helpers (error-free transformations with fma).  Contraction
// of a*b+c into fma is switched off in them: it would fuse the rounded product
// with a later sum and break the exact error terms.
struct DD {
  double hi, lo;
};
__device__ __forceinline__ DD dd_norm(double hi, double lo) {
#pragma clang fp contract(off)
  const double s = hi + lo;
  return DD{s, lo - (s - hi)};
}
__device__ __forceinline__ DD two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  return DD{s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ DD dd_mul(DD a, DD b) {
#pragma clang fp contract(off)
  const double p = a.hi * b.hi;
  const double e = fma(a.hi, b.hi, -p);
  return dd_norm(p, e + (a.hi * b.lo + a.lo * b.hi));
}
__device__ __forceinline__ DD dd_sub(DD a, DD b) {
#pragma clang fp contract(off)
  const DD s = two_sum(a.hi, -b.hi);
  return dd_norm(s.hi, s.lo + (a.lo - b.lo));
}
__device__ __forceinline__ DD dd_div(DD a, double d) {
#pragma clang fp contract(off)
  const double q = a.hi / d;
  const double p = q * d;
  const double e = fma(q, d, -p);
  return dd_norm(q, ((a.hi - p) - e + a.lo) / d);
}

// One Newton correction for a Laguerre root with L_N, L_N' in double-double:
// near x = 0 the float64 recurrence loses ~k^2 eps (double characteristic root).
__device__ double laguerre_dd_newton(int64_t N, double x) {
#pragma clang fp contract(off)
  DD Lp{0.0, 0.0}, L{1.0, 0.0}, dp{0.0, 0.0}, d{0.0, 0.0};
  for (int64_t m = 0; m < N; ++m) {
    const DD c = two_sum(2.0 * (double)m + 1.0, -x);
    const DD mm{(double)m, 0.0};
    const DD Ln = dd_div(dd_sub(dd_mul(c, L), dd_mul(mm, Lp)), (double)(m + 1));
    const DD dn = dd_div(dd_sub(dd_sub(dd_mul(c, d), L), dd_mul(mm, dp)), (double)(m + 1));
    Lp = L;
    L = Ln;
    dp = d;
    d = dn;
    if (fmax(fabs(L.hi), fabs(d.hi)) > BIG) {
      Lp = DD{Lp.hi * RESCALE, Lp.lo * RESCALE};
      L = DD{L.hi * RESCALE, L.lo * RESCALE};
      dp = DD{dp.hi * RESCALE, dp.lo * RESCALE};
      d = DD{d.hi * RESCALE, d.lo * RESCALE};
    }
  }
  return x - (L.hi + L.lo) / (d.hi + d.lo);
}

__global__ void nodes_kernel(FamilyArgs f, const double* __restrict__ diag,
                             const double* __restrict__ off2, double lo0, double hi0,
                             double* __restrict__ x_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = f.N;
  if (j >= N) return;
  if (is_trig(f.family)) {  // Chebyshev-Gauss nodes x_j = cos(theta_j)
    x_out[j] = cospi((double)(2 * j + 1) / (double)(2 * N));
    return;
  }
  // the Jacobi family is stored with x descending, the others ascending
  const int64_t k = (f.family == SPT_LEGENDRE || f.family == SPT_JACOBI) ? N - 1 - j : j;
  const double eps = 2.220446049250313e-16;
  const double pivmin = 1e-290;
  double lo = lo0, hi = hi0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi))) break;
    if (sturm_count(diag, off2, N, mid, pivmin) > k) hi = mid;
    else lo = mid;
  }
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 8; ++it) {
    double pn, dpn;
    poly_and_derivative(f, x, pn, dpn);
    const double dx = pn / dpn;
    x -= dx;
    if (fabs(dx) <= 4.0 * eps * fabs(x)) break;
  }
  if (f.family == SPT_LAGUERRE_FN) x = laguerre_dd_newton(N, x);
  x_out[j] = x;
}

// Christoffel weights of the orthonormal Jacobi system: scale_j = lambda_j^{1/2}
// = (sum_{m<N} p_m(x_j)^2)^{-1/2}
__global__ void weights_kernel(FamilyArgs f, double* __restrict__ rowscale) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= f.N) return;
  FamilyArgs g = f;
  g.rowscale = nullptr;
  RowRec rec;
  rec.init(g, j);
  double s = 0.0;
  for (int64_t m = 0; m < f.N; ++m) {
    const double v = rec.value();
    s += v * v;
    if (m + 1 < f.N) rec.advance(g);
  }
  rowscale[j] = 1.0 / sqrt(s);
}

// ---------------------------------------------------------------- panels of A_e W
// One wave per 64 rows, lane = row; 64-column chunks go through an LDS tile so
// that each row's columns are written contiguously.
__global__ __launch_bounds__(64) void rec_rows_kernel(FamilyArgs f, int64_t row0, int nrows,
                                                      int m0, int L, const double* __restrict__ w,
                                                      double* __restrict__ out) {
  __shared__ double tile[64][65];
  const int lane = threadIdx.x;
  const int lr = blockIdx.x * 64 + lane;  // local row
  const int64_t j = row0 + lr;
  const bool active = lr < nrows && j < f.N;
  RowRec rec;
  rec.init(f, active ? j : 0);
  const bool trig = is_trig(f.family);
  // m0 < 0 only for the trigonometric generators (extras on both sides)
  for (int c0 = 0; c0 < L; c0 += 64) {
    for (int cc = 0; cc < 64; ++cc) {
      const int c = c0 + cc;
      double v = 0.0;
      if (c < L) {
        if (trig) {
          v = rec.trig((int64_t)m0 + c);
        } else {
          v = rec.value();
          if (c + 1 < L) rec.advance(f);
        }
        if (w) v *= w[c];
      }
      tile[lane][cc] = active ? v : 0.0;
    }
    __syncthreads();
    const int ncols = min(64, L - c0);
    for (int rr = 0; rr < 64; ++rr) {
      const int lr2 = blockIdx.x * 64 + rr;
      if (lr2 < nrows && lane < ncols) out[(int64_t)lr2 * L + c0 + lane] = tile[rr][lane];
    }
    __syncthreads();
  }
}

// tail[m * ldt + j] = A[j, m] for m < t; rows j >= N are zero
__global__ void rec_tail_kernel(FamilyArgs f, int t, int64_t ldt, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ldt) return;
  if (j >= f.N) {
    for (int m = 0; m < t; ++m) out[(int64_t)m * ldt + j] = 0.0;
    return;
  }
  RowRec rec;
  rec.init(f, j);
  for (int m = 0; m < t; ++m) {
    out[(int64_t)m * ldt + j] = is_trig(f.family) ? rec.trig(m) : rec.value();
    if (!is_trig(f.family) && m + 1 < t) rec.advance(f);
  }
}

// ---------------------------------------------------------------- threshold
// ---------------------------------------------------------------- Appendix A
// G_k(phi) = L^{-1/2} sum_{c<L} exp(i c phi) exp(-2 pi i c k/L) for phi = t theta_j
// (t may be negative), by the geometric series with the angle kept exact: with
// x = phi - 2 pi k/L = pi n / (2 N L), n = t (2j+1) L - 4 N k an integer,
//   G = L^{-1/2} exp(i (L-1) x/2) sin(L x/2) / sin(x/2),  or L^{1/2} when x = 0 mod 2 pi.
__device__ double2 trig_geometric(int64_t t, int64_t j, int64_t k, int64_t N, int64_t L) {
  const int64_t M4 = 4 * N * L;             // x / 2 = pi n / M4
  const int64_t M8 = 2 * M4;
  int64_t n = (t * (2 * j + 1) * L - 4 * N * k) % M8;
  if (n < 0) n += M8;
  const double rl = 1.0 / sqrt((double)L);
  if (n % M4 == 0) return double2{sqrt((double)L), 0.0};
  const int64_t n8 = n % (8 * N);           // L x / 2 = pi n / (4N)
  const double s1 = sinpi((double)n8 / (double)(4 * N));
  const double s2 = sinpi((double)n / (double)M4);
  const int64_t ph = (int64_t)(((unsigned __int128)(L - 1) * (unsigned __int128)n) %
                               (unsigned __int128)M8);
  double sp, cp;
  sincospi((double)ph / (double)M4, &sp, &cp);
  const double a = rl * s1 / s2;
  return double2{a * cp, a * sp};
}

// One thread per (row, tone, bin offset d in [-B, B]): entry k of the half
// spectrum near the tone's bin t (2j+1) L / (4N) (mirrored into 0 .. P)
__global__ void trig_spec_kernel(TrigSpecArgs a) {
  const int64_t per_row = (int64_t)a.ntones * (2 * a.B + 1);
  const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= per_row * a.nrows) return;
  const int r = (int)(item / per_row);
  const int rem = (int)(item % per_row);
  const int ti = rem / (2 * a.B + 1), d = rem % (2 * a.B + 1) - a.B;
  const int64_t N = a.N, L = a.L, j = a.row0 + r;
  const int64_t t0 = a.tone[ti];
  int64_t kc = ((t0 * (2 * j + 1) * L + 2 * N) / (4 * N)) % L;  // nearest bin of the tone
  int64_t k = ((kc + d) % L + L) % L;
  if (k > a.P) k = L - k;
  // U_k' = sum_tones coef (ph G(t) +- conj(ph) G(-t)) / 2 (cos) or / 2i (sin),
  // ph = exp(i t m_off theta_j)
  double2 ph[TRIG_MAX_TONES];
  for (int u = 0; u < a.ntones; ++u) {
    int64_t qv = ((int64_t)a.tone[u] * a.m_off % (4 * N)) * ((2 * j + 1) % (4 * N)) % (4 * N);
    if (qv < 0) qv += 4 * N;
    double sp, cp;
    sincospi((double)qv / (double)(2 * N), &sp, &cp);
    ph[u] = double2{cp, sp};
  }
  double vr = 0.0, vi = 0.0;
  for (int m = -a.q; m <= a.q; ++m) {
    const int64_t kp = ((k - m) % L + L) % L;
    double ur = 0.0, ui = 0.0;
    for (int u = 0; u < a.ntones; ++u) {
      const double2 gp = trig_geometric(a.tone[u], j, kp, N, L);
      const double2 gm = trig_geometric(-(int64_t)a.tone[u], j, kp, N, L);
      const double2 p = ph[u];
      // ph gp and conj(ph) gm
      const double ar = p.x * gp.x - p.y * gp.y, ai = p.x * gp.y + p.y * gp.x;
      const double br = p.x * gm.x + p.y * gm.y, bi = p.x * gm.y - p.y * gm.x;
      const double c = 0.5 * a.coef[u];
      if (a.sine) {  // (A - B) / (2i) = -i (A - B) / 2
        ur += c * (ai - bi);
        ui -= c * (ar - br);
      } else {
        ur += c * (ar + br);
        ui += c * (ai + bi);
      }
    }
    const double2 w = a.vt[m + a.q];
    vr += w.x * ur - w.y * ui;
    vi += w.x * ui + w.y * ur;
  }
  const double rl = 1.0 / sqrt((double)L);
  a.spec[(int64_t)r * (a.P + 1) + k] = double2{vr * rl, vi * rl};
}

__global__ void maxabs_kernel(const double2* __restrict__ s, int64_t n,
                              unsigned long long* __restrict__ max_bits) {
  double mx = 0.0;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2 v = s[i];
    const double a = v.x * v.x + v.y * v.y;
    bad |= !isfinite(a);
    mx = fmax(mx, a);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  const unsigned long long anybad = __any(bad);
  if ((threadIdx.x & 63) == 0) {
    // non-negative doubles order like their bit patterns; a non-finite value
    // is reported as +inf
    const unsigned long long bits =
        anybad ? 0x7FF0000000000000ull : (unsigned long long)__double_as_longlong(mx);
    atomicMax(max_bits, bits);
  }
}

// per row: first and last half-spectrum index with |a| > thr, and the count
__global__ __launch_bounds__(256) void extents_kernel(const double2* __restrict__ s, int nrows,
                                                      int P, double thr, int32_t* __restrict__ klo,
                                                      int32_t* __restrict__ khi,
                                                      int32_t* __restrict__ cnt) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + wave;
  if (row >= nrows) return;
  const double2* __restrict__ r = s + (int64_t)row * (P + 1);
  int lo = 0x7FFFFFFF, hi = -1, n = 0;
  for (int k = lane; k <= P; k += 64) {
    const double2 v = r[k];
    if (sqrt(v.x * v.x + v.y * v.y) > thr) {
      lo = min(lo, k);
      hi = max(hi, k);
      ++n;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o));
    hi = max(hi, __shfl_xor(hi, o));
    n += __shfl_xor(n, o);
  }
  if (lane == 0) {
    klo[row] = hi < 0 ? -1 : lo;
    khi[row] = hi;
    cnt[row] = n;
  }
}

// kept entries times c_k into the tile boxes; thread = (tile, kk, q)
__global__ __launch_bounds__(256) void pack_kernel(const double2* __restrict__ s, int64_t row0,
                                                   int nrows, int64_t N, int P, double thr,
                                                   const int32_t* __restrict__ tk0,
                                                   const int32_t* __restrict__ tkw,
                                                   const int64_t* __restrict__ toff, int tile0,
                                                   double2* __restrict__ v64,
                                                   float2* __restrict__ v32) {
  const int t = tile0 + blockIdx.x;  // global tile index
  const int k0 = tk0[t], kw = tkw[t];
  const int64_t off = toff[t];
  for (int e = threadIdx.x; e < kw * TILE_ROWS; e += blockDim.x) {
    const int kk = e / TILE_ROWS, q = e % TILE_ROWS;
    const int64_t n = (int64_t)t * TILE_ROWS + q;
    const int64_t lr = n - row0;
    double2 v = double2{0.0, 0.0};
    if (n < N && lr >= 0 && lr < nrows) {
      const int k = k0 + kk;
      const double2 a = s[lr * (P + 1) + k];
      if (sqrt(a.x * a.x + a.y * a.y) > thr) {
        const double ck = (k == 0 || k == P) ? 1.0 : 2.0;
        v = double2{a.x * ck, a.y * ck};
      }
    }
    if (v64) v64[off + e] = v;
    if (v32) v32[off + e] = float2{(float)v.x, (float)v.y};
  }
}

__global__ void to_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// Pre-split tile boxes (layout in common.hpp): one workgroup per tile, one
// thread per (step, lane) of the box.
__global__ __launch_bounds__(256) void split_pack_kernel(const float2* __restrict__ val32,
                                                         const int32_t* __restrict__ tkw,
                                                         const int64_t* __restrict__ toff,
                                                         const int64_t* __restrict__ tsoff,
                                                         uint16_t* __restrict__ valbf) {
  using namespace spmmcore;
  const int t = blockIdx.x;
  const int kw = tkw[t];
  const int steps = (kw + 15) / 16;
  const float2* __restrict__ v = val32 + toff[t];
  bf16x8* __restrict__ out = reinterpret_cast<bf16x8*>(valbf + tsoff[t]);
  for (int idx = threadIdx.x; idx < steps * 64; idx += blockDim.x) {
    const int st = idx / 64, lane = idx % 64;
    const int m = lane & 15, g = lane >> 4;
    f32x8 f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = 16 * st + 4 * g + (j >> 1);
      const float2 a = c < kw ? v[c * TILE_ROWS + m] : float2{0.f, 0.f};
      f[j] = (j & 1) ? -a.y : a.x;
    }
    const Split8 sp(f);
#pragma unroll
    for (int p = 0; p < 3; ++p) out[(3 * st + p) * 64 + lane] = sp.get(p);
  }
}

__global__ __launch_bounds__(256) void split_tail_kernel(const float* __restrict__ tail32,
                                                         int64_t ldt, int tail,
                                                         uint16_t* __restrict__ tailbf) {
  using namespace spmmcore;
  const int t = blockIdx.x;
  const int tsteps = (tail + 31) / 32;
  bf16x8* __restrict__ out = reinterpret_cast<bf16x8*>(tailbf);
  for (int idx = threadIdx.x; idx < tsteps * 64; idx += blockDim.x) {
    const int st = idx / 64, lane = idx % 64;
    const int m = lane & 15, g = lane >> 4;
    f32x8 f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int mm = 32 * st + 8 * g + j;
      f[j] = mm < tail ? tail32[(int64_t)mm * ldt + (int64_t)t * TILE_ROWS + m] : 0.f;
    }
    const Split8 sp(f);
#pragma unroll
    for (int p = 0; p < 3; ++p) out[(((int64_t)t * tsteps + st) * 3 + p) * 64 + lane] = sp.get(p);
  }
}

int blocks_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 65535 * 16);
}

}  // namespace

void launch_nodes(const FamilyArgs& f, const double* diag, const double* off2, double lo,
                  double hi, double* x_out, hipStream_t s) {
  hipLaunchKernelGGL(nodes_kernel, dim3(blocks_for(f.N, 64)), dim3(64), 0, s, f, diag, off2, lo,
                     hi, x_out);
  SPT_HIP(hipGetLastError());
}

void launch_weights(const FamilyArgs& f, double* rowscale, hipStream_t s) {
  hipLaunchKernelGGL(weights_kernel, dim3(blocks_for(f.N, 64)), dim3(64), 0, s, f, rowscale);
  SPT_HIP(hipGetLastError());
}

void launch_rec_rows(const FamilyArgs& f, int64_t row0, int nrows, int m0, int L,
                     const double* w, double* out, hipStream_t s) {
  hipLaunchKernelGGL(rec_rows_kernel, dim3((nrows + 63) / 64), dim3(64), 0, s, f, row0, nrows,
                     m0, L, w, out);
  SPT_HIP(hipGetLastError());
}

void launch_trig_spec(const TrigSpecArgs& a, hipStream_t s) {
  const int64_t items = (int64_t)a.nrows * a.ntones * (2 * a.B + 1);
  if (items <= 0) return;
  hipLaunchKernelGGL(trig_spec_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, a);
  SPT_HIP(hipGetLastError());
}

void launch_rec_tail(const FamilyArgs& f, int t, double* out, hipStream_t s) {
  const int64_t ldt = ((f.N + TILE_ROWS - 1) / TILE_ROWS) * TILE_ROWS;
  hipLaunchKernelGGL(rec_tail_kernel, dim3(blocks_for(ldt, 64)), dim3(64), 0, s, f, t, ldt,
                     out);
  SPT_HIP(hipGetLastError());
}

void launch_maxabs(const double2* spec, int64_t count, unsigned long long* max_bits,
                   hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(maxabs_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, s, spec, count,
                     max_bits);
  SPT_HIP(hipGetLastError());
}

void launch_extents(const double2* spec, int nrows, int P, double thr, int32_t* klo,
                    int32_t* khi, int32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(extents_kernel, dim3((nrows + 3) / 4), dim3(256), 0, s, spec, nrows, P,
                     thr, klo, khi, cnt);
  SPT_HIP(hipGetLastError());
}

void launch_pack(const double2* spec, int64_t row0, int nrows, int64_t N, int P, double thr,
                 const int32_t* tile_k0, const int32_t* tile_kw, const int64_t* tile_off,
                 int tile0, double2* val64, float2* val32, hipStream_t s) {
  const int ntile = (nrows + TILE_ROWS - 1) / TILE_ROWS;
  hipLaunchKernelGGL(pack_kernel, dim3(ntile), dim3(256), 0, s, spec, row0, nrows, N, P, thr,
                     tile_k0, tile_kw, tile_off, tile0, val64, val32);
  SPT_HIP(hipGetLastError());
}

void launch_split_pack(const float2* val32, const int32_t* tile_kw, const int64_t* tile_off,
                       const int64_t* tile_soff, int ntiles, uint16_t* valbf, hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(split_pack_kernel, dim3(ntiles), dim3(256), 0, s, val32, tile_kw, tile_off,
                     tile_soff, valbf);
  SPT_HIP(hipGetLastError());
}

void launch_split_tail(const float* tail32, int64_t ldt, int tail, int ntiles, uint16_t* tailbf,
                       hipStream_t s) {
  if (ntiles <= 0 || tail <= 0) return;
  hipLaunchKernelGGL(split_tail_kernel, dim3(ntiles), dim3(256), 0, s, tail32, ldt, tail, tailbf);
  SPT_HIP(hipGetLastError());
}

void launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
  SPT_HIP(hipGetLastError());
}

}  // namespace spt
