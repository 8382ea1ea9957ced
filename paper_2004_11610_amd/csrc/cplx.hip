// Complex generators (sec. 2, after Algorithm 2: exp(i m theta); sec. 4.1,
// eq. lag_matrix: the spectral-domain Laguerre matrix C) through Algorithm 1
// (extras on both sides, one block) and Algorithm 2: complex data, the full
// spectrum of length L (no half-spectrum symmetry), tile boxes that may run
// past column L - 1 (the spectra carry a copy of their first `pad` columns
// behind column L - 1).
//
// Kernels: the rows of A_e W by their closed forms, their transforms F (one
// workgroup per row), and the computation stage: extend, divide by the window
// and F* (one workgroup per right-hand side), the banded product; and for the
// transposed product the gathered banded product A^T, F*, division by the
// window and truncation.  Transforms run in float64 arithmetic for either
// precision of the data (float32 data: each spectrum value and each output is
// rounded once).

#include "common.hpp"
#include "fft_core.hpp"

namespace spt {
namespace {

using namespace fftcore;

// exp(i pi q / (2N)) for an integer q reduced mod 4N: the exact angle m theta_j
// of theta_j = pi (2j + 1) / (2N)
__device__ __forceinline__ double2 cexp_exact(int64_t m, int64_t j, int64_t N) {
  const int64_t N4 = 4 * N;
  int64_t q = (m % N4) * ((2 * j + 1) % N4) % N4;
  if (q < 0) q += N4;
  double s, c;
  sincospi((double)q / (double)(2 * N), &s, &c);
  return double2{c, s};
}

__global__ __launch_bounds__(256) void cplx_rows_kernel(CplxRowsArgs a) {
  const int64_t row = a.row0 + blockIdx.y;
  if (row >= a.N) return;
  double2* __restrict__ out = a.out + (int64_t)blockIdx.y * a.L;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.L; c += gridDim.x * 256) {
    const int64_t m = (int64_t)c + a.m_off;
    double2 v;
    if (a.family == SPT_CEXP) {
      v = cexp_exact(m, row, a.N);
    } else {
      // exp(i m phi_j) / (eta/2 - i k_j): the phase a float64 product
      double s, cs;
      sincos(a.phi[row] * (double)m, &s, &cs);
      v = cmul(double2{cs, s}, a.rowf[row]);
    }
    const double w = a.w[c];
    out[c] = double2{v.x * w, v.y * w};
  }
}

// F of a row of L points (SIGN -1, unitary), in place
__global__ __launch_bounds__(1024) void cplx_row_fft_kernel(double2* rows, int L, FftPlan fp,
                                                             const double2* __restrict__ tw,
                                                             double scale) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* lds = reinterpret_cast<double2*>(smem_raw);
  double2* __restrict__ v = rows + (int64_t)blockIdx.x * L;
  for (int j = threadIdx.x; j < L; j += blockDim.x) lds[j] = v[j];
  __syncthreads();
  run_fft<-1>(lds, fp, tw, threadIdx.x, blockDim.x);
  for (int j = threadIdx.x; j < L; j += blockDim.x)
    v[j] = double2{lds[j].x * scale, lds[j].y * scale};
}

// z = F* W^{-1} v per right-hand side: z[r][k], k < L, and its first pad
// columns again at L .. L + pad - 1
template <typename TI>
__global__ __launch_bounds__(1024) void cplx_exec_fft_kernel(CplxExecArgs<TI> a, FftPlan fp) {
  using CI = cplx_t<TI>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* lds = reinterpret_cast<double2*>(smem_raw);
  const int r = blockIdx.x;
  const CI* __restrict__ x = a.X + (int64_t)r * a.N;
  for (int c = threadIdx.x; c < a.L; c += blockDim.x) {
    double2 v = double2{0.0, 0.0};
    if (c >= a.c_lo && c < a.c_hi) {
      const CI xv = x[c + a.m_off];
      const double wi = a.winv[c];
      v = double2{(double)xv.x * wi, (double)xv.y * wi};
    }
    lds[c] = v;
  }
  __syncthreads();
  run_fft<+1>(lds, fp, a.tw, threadIdx.x, blockDim.x);
  CI* __restrict__ z = a.Z + (int64_t)r * a.ldz;
  for (int k = threadIdx.x; k < a.ldz; k += blockDim.x) {
    const double2 v = lds[k < a.L ? k : k - a.L];
    z[k] = CI{(TI)(v.x * a.scale), (TI)(v.y * a.scale)};
  }
}

// y[r][n] = sum over the tile box of A[n][k] z[r][k]: workgroup = tile x 16
// right-hand sides x KQ parts of the box's columns, thread = (row q,
// right-hand side, part).  The parts' sums meet in LDS and are added in a
// fixed order.  The widest boxes (the low frequencies of the Laguerre
// spectral matrix, near a thousand columns) set the launch's length: a
// thread's columns are a chain of memory round trips, so plans with wide
// boxes take KQ = 4, the others 1.
template <typename T, int KQ>
__global__ __launch_bounds__(256 * KQ) void cplx_spmm_kernel(CplxSpmmArgs<T> a) {
  using C = cplx_t<T>;
  __shared__ double2 part[KQ > 1 ? KQ - 1 : 1][256];
  const int tile = blockIdx.x;
  const int t = threadIdx.x & 255, ks = threadIdx.x >> 8;
  const int q = t & 15, rl = t >> 4;
  const int r = blockIdx.y * 16 + rl;
  const int64_t n = (int64_t)tile * TILE_ROWS + q;
  const bool live = r < a.R && n < a.N;
  const TileMeta tm = a.meta[tile];
  const int kq = (tm.kw + KQ - 1) / KQ;
  const int k1 = min(tm.kw, (ks + 1) * kq);
  // eight columns per step, their loads issued together, into four partial
  // sums added in a fixed order
  constexpr int U = 8;
  double2 acc[4] = {};
  if (live) {
    const C* __restrict__ val = a.val + tm.off + q;
    const C* __restrict__ z = a.Z + (int64_t)r * a.ldz + tm.k0;
    int kk = ks * kq;
    for (; kk + U <= k1; kk += U) {
      C av[U], zv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        av[u] = val[(int64_t)(kk + u) * TILE_ROWS];
        zv[u] = z[kk + u];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc[u & 3].x += (double)av[u].x * zv[u].x - (double)av[u].y * zv[u].y;
        acc[u & 3].y += (double)av[u].x * zv[u].y + (double)av[u].y * zv[u].x;
      }
    }
    for (; kk < k1; ++kk) {
      const C av = val[(int64_t)kk * TILE_ROWS];
      const C zv = z[kk];
      acc[0].x += (double)av.x * zv.x - (double)av.y * zv.y;
      acc[0].y += (double)av.x * zv.y + (double)av.y * zv.x;
    }
  }
  double2 sum = double2{(acc[0].x + acc[1].x) + (acc[2].x + acc[3].x),
                        (acc[0].y + acc[1].y) + (acc[2].y + acc[3].y)};
  if (KQ > 1) {
    if (ks > 0) part[ks - 1][t] = sum;
    __syncthreads();
  }
  if (ks == 0 && live) {
#pragma unroll
    for (int i = 0; i < KQ - 1; ++i) {
      sum.x += part[i][t].x;
      sum.y += part[i][t].y;
    }
    a.Y[(int64_t)r * a.N + n] = C{(T)sum.x, (T)sum.y};
  }
}

// u[r][k'] = sum_n A[n][k'] f[r][n] for the columns k' < L + pad of the tile
// boxes: workgroup = 32 columns x 8 right-hand sides x KQ parts of the tile
// list, over the tiles whose boxes meet the 32 columns (list ents[tptr[c] ..
// tptr[c + 1])).  Where many rows' tones share a few columns (the high
// frequencies of the Laguerre spectral matrix) the lists run to hundreds of
// tiles, a chain per thread: plans with such lists take KQ = 4 parts, whose
// sums meet in LDS and are added in a fixed order.
template <typename T, int KQ>
__global__ __launch_bounds__(256 * KQ) void cplx_spmm_t_kernel(CplxSpmmTArgs<T> a) {
  using C = cplx_t<T>;
  __shared__ double2 part[KQ > 1 ? KQ - 1 : 1][256];
  const int c = blockIdx.x;
  const int t = threadIdx.x & 255, ks = threadIdx.x >> 8;
  const int col = t & 31, rl = t >> 5;
  const int r = blockIdx.y * 8 + rl;
  const int k = c * 32 + col;
  const bool live = r < a.R && k < a.ldu;
  // a tile's 16 rows in two groups of eight, each group's loads issued
  // together, into four partial sums added in a fixed order at the end
  double2 acc[4] = {};
  if (live) {
    const C* __restrict__ f = a.F + (int64_t)r * a.N;
    const int e0 = a.tptr[c], n_e = a.tptr[c + 1] - e0;
    const int per = (n_e + KQ - 1) / KQ;
    const int e1 = e0 + min(n_e, (ks + 1) * per);
    int e = e0 + ks * per;
    // the list is read ahead (the tile two entries on, the box of the next),
    // so that an entry waits for one memory round trip instead of three
    int tile_a = e < e1 ? a.tents[e] : 0;          // entry e
    int tile_b = e + 1 < e1 ? a.tents[e + 1] : 0;  // entry e + 1
    TileMeta meta_a = e < e1 ? a.meta[tile_a] : TileMeta{};
    for (; e < e1; ++e) {
      const int tile = tile_a;
      const TileMeta tm = meta_a;
      if (e + 1 < e1) meta_a = a.meta[tile_b];
      tile_a = tile_b;
      if (e + 2 < e1) tile_b = a.tents[e + 2];
      const int kk = k - tm.k0;
      if (kk < 0 || kk >= tm.kw) continue;
      const C* __restrict__ val = a.val + tm.off + (int64_t)kk * TILE_ROWS;
      const int64_t n0 = (int64_t)tile * TILE_ROWS;
      if (n0 + TILE_ROWS <= a.N) {
#pragma unroll
        for (int h = 0; h < TILE_ROWS; h += 8) {
          C av[8], fv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            av[u] = val[h + u];
            fv[u] = f[n0 + h + u];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            acc[u & 3].x += (double)av[u].x * fv[u].x - (double)av[u].y * fv[u].y;
            acc[u & 3].y += (double)av[u].x * fv[u].y + (double)av[u].y * fv[u].x;
          }
        }
      } else {
        for (int q = 0; q < TILE_ROWS && n0 + q < a.N; ++q) {
          const C av = val[q];
          const C fv = f[n0 + q];
          acc[0].x += (double)av.x * fv.x - (double)av.y * fv.y;
          acc[0].y += (double)av.x * fv.y + (double)av.y * fv.x;
        }
      }
    }
  }
  double2 sum = double2{(acc[0].x + acc[1].x) + (acc[2].x + acc[3].x),
                        (acc[0].y + acc[1].y) + (acc[2].y + acc[3].y)};
  if (KQ > 1) {
    if (ks > 0) part[ks - 1][t] = sum;
    __syncthreads();
  }
  if (ks == 0 && live) {
#pragma unroll
    for (int i = 0; i < KQ - 1; ++i) {
      sum.x += part[i][t].x;
      sum.y += part[i][t].y;
    }
    a.U[(int64_t)r * a.ldu + k] = C{(T)sum.x, (T)sum.y};
  }
}

// y_m = (F* u)_c / w_c on the retained columns, m = c + m_off; u[k] takes the
// box columns past L - 1 back (u[k] + u[L + k], k < pad)
template <typename TI>
__global__ __launch_bounds__(1024) void cplx_inv_fft_kernel(CplxInvArgs<TI> a, FftPlan fp) {
  using CI = cplx_t<TI>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2* lds = reinterpret_cast<double2*>(smem_raw);
  const int r = blockIdx.x;
  const CI* __restrict__ u = a.U + (int64_t)r * a.ldu;
  for (int k = threadIdx.x; k < a.L; k += blockDim.x) {
    const CI v = u[k];
    double2 s = double2{(double)v.x, (double)v.y};
    if (k + a.L < a.ldu) {
      const CI w = u[k + a.L];
      s.x += (double)w.x;
      s.y += (double)w.y;
    }
    lds[k] = s;
  }
  __syncthreads();
  run_fft<+1>(lds, fp, a.tw, threadIdx.x, blockDim.x);
  CI* __restrict__ y = a.Y + (int64_t)r * a.N;
  for (int c = threadIdx.x; c < a.L; c += blockDim.x) {
    if (c < a.c_lo || c >= a.c_hi) continue;
    const double2 v = lds[c];
    const double g = a.scale * a.winv[c];
    y[c + a.m_off] = CI{(TI)(v.x * g), (TI)(v.y * g)};
  }
}

template <typename K>
void allow_lds(K kernel) {
  SPT_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
}

}  // namespace

void launch_cplx_rows(const CplxRowsArgs& a, int nrows, hipStream_t s) {
  if (nrows <= 0) return;
  const int gx = std::max(1, std::min((a.L + 255) / 256, 64));
  hipLaunchKernelGGL(cplx_rows_kernel, dim3(gx, nrows), dim3(256), 0, s, a);
  SPT_HIP(hipGetLastError());
}

void launch_cplx_row_fft(double2* rows, int nrows, int L, const FftPlan& fp, const double2* tw,
                         hipStream_t s) {
  if (nrows <= 0) return;
  allow_lds(cplx_row_fft_kernel);
  hipLaunchKernelGGL(cplx_row_fft_kernel, dim3(nrows), dim3(fp.threads),
                     (size_t)L * sizeof(double2), s, rows, L, fp, tw, 1.0 / std::sqrt((double)L));
  SPT_HIP(hipGetLastError());
}

template <typename TI>
void launch_cplx_exec_fft(const CplxExecArgs<TI>& a, const FftPlan& fp, int R, hipStream_t s) {
  allow_lds(cplx_exec_fft_kernel<TI>);
  hipLaunchKernelGGL(cplx_exec_fft_kernel<TI>, dim3(R), dim3(fp.threads),
                     (size_t)a.L * sizeof(double2), s, a, fp);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_cplx_spmm(const CplxSpmmArgs<T>& a, int n_tiles, int max_kw, hipStream_t s) {
  const dim3 grid(n_tiles, (a.R + 15) / 16);
  if (max_kw > 128)
    hipLaunchKernelGGL((cplx_spmm_kernel<T, 4>), grid, dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL((cplx_spmm_kernel<T, 1>), grid, dim3(256), 0, s, a);
  SPT_HIP(hipGetLastError());
}

template <typename T>
void launch_cplx_spmm_t(const CplxSpmmTArgs<T>& a, int n_chunks, int max_list, hipStream_t s) {
  const dim3 grid(n_chunks, (a.R + 7) / 8);
  if (max_list > 32)
    hipLaunchKernelGGL((cplx_spmm_t_kernel<T, 4>), grid, dim3(1024), 0, s, a);
  else
    hipLaunchKernelGGL((cplx_spmm_t_kernel<T, 1>), grid, dim3(256), 0, s, a);
  SPT_HIP(hipGetLastError());
}

template <typename TI>
void launch_cplx_inv_fft(const CplxInvArgs<TI>& a, const FftPlan& fp, int R, hipStream_t s) {
  allow_lds(cplx_inv_fft_kernel<TI>);
  hipLaunchKernelGGL(cplx_inv_fft_kernel<TI>, dim3(R), dim3(fp.threads),
                     (size_t)a.L * sizeof(double2), s, a, fp);
  SPT_HIP(hipGetLastError());
}

template void launch_cplx_exec_fft<double>(const CplxExecArgs<double>&, const FftPlan&, int,
                                           hipStream_t);
template void launch_cplx_exec_fft<float>(const CplxExecArgs<float>&, const FftPlan&, int,
                                          hipStream_t);
template void launch_cplx_spmm<double>(const CplxSpmmArgs<double>&, int, int, hipStream_t);
template void launch_cplx_spmm<float>(const CplxSpmmArgs<float>&, int, int, hipStream_t);
template void launch_cplx_spmm_t<double>(const CplxSpmmTArgs<double>&, int, int, hipStream_t);
template void launch_cplx_spmm_t<float>(const CplxSpmmTArgs<float>&, int, int, hipStream_t);
template void launch_cplx_inv_fft<double>(const CplxInvArgs<double>&, const FftPlan&, int,
                                          hipStream_t);
template void launch_cplx_inv_fft<float>(const CplxInvArgs<float>&, const FftPlan&, int,
                                         hipStream_t);

}  // namespace spt
