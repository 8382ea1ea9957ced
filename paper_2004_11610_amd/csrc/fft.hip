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

// Every block of a plan and every right-hand side in one grid: workgroup
// (x, y) takes block y (blocks sorted by decreasing length) and its
// right-hand sides r0 = x 2^lb .. r0 + 2^lb - 1 (lb = FftDesc::lb), their
// transforms interleaved in LDS (point j of transform t at lds[(j << lb) + t])
// so that a short block fills the workgroup as a long one does; workgroups
// past a block's right-hand sides return at once.

// SPLIT: the half spectra are written as three bfloat16 planes (the pieces of
// the split-bf16 product, layout in common.hpp) instead of complex values.
// BATCH == false: one transform (lb == 0), indexed without the interleaving.
template <typename T, bool SPLIT, bool BATCH>
__device__ __forceinline__ void fft_multi_body(const FftDesc<T>* __restrict__ d,
                                               const T* __restrict__ X, cplx_t<T>* __restrict__ Z,
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
  // E1: the thread's points requested together (float32: all at once;
  // float64: in two rounds, for registers), then written to LDS; transforms
  // past the last right-hand side are zero
  constexpr int ROUND = sizeof(T) == 4 ? FFT_EPT : FFT_EPT / 2;
  const int pts = P << lb;
#pragma unroll
  for (int h = 0; h < FFT_EPT; h += ROUND) {
    T v0[ROUND], v1[ROUND];
#pragma unroll
    for (int e = 0; e < ROUND; ++e) {
      const int u = tid + (h + e) * nt;
      const int j = u >> lb, t = u & tmask;
      const int c0 = 2 * j, c1 = 2 * j + 1;
      const bool in = u < pts && t < cnt;
      const T* __restrict__ x = X + (int64_t)(r0 + (BATCH && in ? t : 0)) * N;
      v0[e] = in && c0 >= c_lo && c0 < c_hi ? gload(x + c0 + m_off) * gload(winv + c0) : T(0);
      v1[e] = in && c1 >= c_lo && c1 < c_hi ? gload(x + c1 + m_off) * gload(winv + c1) : T(0);
    }
#pragma unroll
    for (int e = 0; e < ROUND; ++e) {
      const int u = tid + (h + e) * nt;
      if (u < pts) lds[u] = C{v0[e], v1[e]};
    }
  }
  __syncthreads();
  // E2: F*; float32 reads its pass twiddles from the block's table, float64
  // forms them from the two-level table (its registers hold no prefetch)
  if constexpr (sizeof(T) == 4)
    run_fft_tab<+1, BATCH>(lds, P, lb, d->fp.npass, d->fp.radix, d->ptw, tid, nt, true);
  else
    run_fft<+1, BATCH>(lds, P, lb, d->fp.npass, d->fp.radix, d->tw, 1, tid, nt, true);
  // unpack point k of transform t (see unpack_with)
  const T scale = d->scale;
  const C* __restrict__ post = d->post;
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
  if constexpr (!SPLIT) {
    const int n = (P + 1) << lb;
    for (int u = tid; u < n; u += nt) {
      const int k = u >> lb, t = u & tmask;
      if (t < cnt)
        Z[(int64_t)R * d->zoff + (int64_t)(r0 + t) * d->ldz + k] = unpack_at(k, t, gload(post + k));
    }
  } else {
    // four consecutive k per thread (ldz4 is a multiple of 4): each plane gets
    // one 16-byte store per group; zeros past P
    const int n = (d->ldz4 / 4) << lb;
    for (int u = tid; u < n; u += nt) {
      const int q = u >> lb, t = u & tmask;
      if (t >= cnt) continue;
      C tw[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) tw[j] = gload(post + min(4 * q + j, P));
      uint32_t pc[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * q + j;
        const C z = k <= P ? unpack_at(k, t, tw[j]) : C{T(0), T(0)};
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

template <typename T, bool SPLIT>
__global__ __launch_bounds__(FFT_MAX_THREADS) void exec_fft_multi_kernel(
    const FftDesc<T>* __restrict__ descs, const T* __restrict__ X, cplx_t<T>* __restrict__ Z,
    uint32_t* __restrict__ Zs, int64_t zplane, int R, int64_t N) {
  const FftDesc<T>* __restrict__ d = descs + blockIdx.y;
  const int lb = d->lb;
  const int r0 = (int)blockIdx.x << lb;
  if (r0 >= R) return;
  if (lb == 0)
    fft_multi_body<T, SPLIT, false>(d, X, Z, Zs, zplane, R, N, 0, r0);
  else
    fft_multi_body<T, SPLIT, true>(d, X, Z, Zs, zplane, R, N, lb, r0);
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
template <typename T>
size_t fused_lds_bytes(int max_P) {
  return (size_t)max_P * sizeof(cplx_t<T>);
}

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
  set_lds(row_fft_kernel, max_lds);
  set_lds(exec_fft_multi_kernel<double, false>, max_lds);
  set_lds(exec_fft_multi_kernel<float, false>, max_lds);
  set_lds(exec_fft_multi_kernel<float, true>, max_lds);
  done.push_back(dev);
}

FftPlan make_fft_plan(int P) {
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
void launch_exec_fft_multi(const FftDesc<T>* descs, int nblk, int threads, int max_P,
                           const T* X, cplx_t<T>* Z, int R, int64_t N, hipStream_t s) {
  const size_t lds = fused_lds_bytes<T>(max_P);
  hipLaunchKernelGGL((exec_fft_multi_kernel<T, false>), dim3(R, nblk), dim3(threads), lds, s,
                     descs, X, Z, (uint32_t*)nullptr, (int64_t)0, R, N);
  SPT_HIP(hipGetLastError());
}

void launch_exec_fft_multi_split(const FftDesc<float>* descs, int nblk, int threads, int max_P,
                                 const float* X, uint32_t* Zs, int64_t zplane, int R, int64_t N,
                                 hipStream_t s) {
  const size_t lds = fused_lds_bytes<float>(max_P);
  hipLaunchKernelGGL((exec_fft_multi_kernel<float, true>), dim3(R, nblk), dim3(threads), lds, s,
                     descs, X, (float2*)nullptr, Zs, zplane, R, N);
  SPT_HIP(hipGetLastError());
}

template void launch_exec_fft_multi<double>(const FftDesc<double>*, int, int, int, const double*,
                                            double2*, int, int64_t, hipStream_t);
template void launch_exec_fft_multi<float>(const FftDesc<float>*, int, int, int, const float*,
                                           float2*, int, int64_t, hipStream_t);
template void launch_exec_fft<double>(const ExecFftArgs<double>&, const FftPlan&, hipStream_t);
template void launch_exec_fft<float>(const ExecFftArgs<float>&, const FftPlan&, hipStream_t);
template void launch_inv_fft<double>(const InvFftArgs<double>&, const FftPlan&, hipStream_t);
template void launch_inv_fft<float>(const InvFftArgs<float>&, const FftPlan&, hipStream_t);

}  // namespace spt
