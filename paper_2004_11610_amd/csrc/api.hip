// C ABI of the spt library: plans, the precomputation (Alg. 1 steps 1.1-1.3 and
// the block version of sec. 3), the computation stage (Alg. 1 steps 2.1-2.2),
// the transposed computation (Alg. 2) and batched execution.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "common.hpp"
#include "exec.hpp"
#include "planner.hpp"
#include "worklist.hpp"

namespace spt {
namespace {

thread_local std::string g_last_error;

int64_t next_serial() {
  static std::atomic<int64_t> n{0};
  return ++n;
}

// ---------------------------------------------------------------- device buffers
// The allocator of device memory (spt_set_allocator): a caller's hook pair, or
// hipMalloc / hipFree when none is set.  A buffer remembers the hook that
// allocated it and is freed through the same one.
struct Allocator {
  spt_alloc_fn alloc = nullptr;
  spt_free_fn free = nullptr;
  void* ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

Allocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Allocator a;             // who allocated p
  hipStream_t st = nullptr;  // the stream passed to the hook
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    if (p) {
      if (a.free)
        a.free(p, st, a.ctx);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n, hipStream_t s = nullptr) {
    reset();
    if (n == 0) return;
    a = current_allocator();
    st = s;
    if (a.alloc) {
      p = a.alloc(n, s, a.ctx);
      if (!p)
        throw Error(SPT_E_OOM, "the allocator hook returned NULL for " + std::to_string(n) +
                                   " bytes");
    } else {
      hipError_t e = hipMalloc(&p, n);
      if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw Error(SPT_E_OOM, "hipMalloc(" + std::to_string(n) + " bytes) failed: " +
                                   hipGetErrorString(e));
      }
    }
    bytes = n;
  }
  void ensure(size_t n) {
    if (n > bytes) alloc(n);
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

template <typename T>
void upload(DevBuf& b, const std::vector<T>& h, hipStream_t s) {
  b.alloc(h.size() * sizeof(T), s);
  if (!h.empty()) {
    SPT_HIP(hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    SPT_HIP(hipStreamSynchronize(s));
  }
}

struct DevBlock {
  BlockGeom g;
  int P = 0;
  FftPlan fft;
  // the fused computation-stage FFT: its plan (P, or P / 2 when the transform
  // is split by output parity), the split, and 2^lbw right-hand sides per
  // workgroup
  FftPlan fftw;
  int half = 0, lbw = 0;
  DevBuf winv64, winv32, tw64, post64, post32, posttw;
  DevBuf k0, kw, off;   // per tile
  bool big = false;  // the transform does not fit one workgroup (four steps)
  // the computation stage's forward FFT is fused (one workgroup per transform
  // or split part; every block of a plan with !big, and split blocks up to
  // FUSED_FWD_MAX_P)
  bool fwd = false;
  // transposed product: the segments of row tiles per TCHUNK spectrum columns
  std::vector<int32_t> h_tptr;  // chunk c's tiles are h_tent[h_tptr[c] .. h_tptr[c + 1])
  std::vector<TChunkEnt> h_tent;
  DevBuf val64, val32;  // tile boxes
  DevBuf valbf, soff;   // pre-split tile boxes of the split-bf16 path, their offsets
  int64_t nnz = 0, stored = 0;
  int max_band = 0;
  double maxabs = 0.0;
  double kappa = 0.0;
  std::vector<int32_t> h_k0, h_kw;
  std::vector<int64_t> h_off, h_soff;
  int ldz4 = 0;  // P + 1 rounded up to a multiple of 4 (pre-split spectra)
  // persistent executor: one workgroup per batch of transforms (four == 0) or
  // a four-step transform P = P1 * P2 (COL and ROW items)
  int four = 0, P1 = 0, P2 = 0, lcw = 0, lgp = 0, n_col = 0, n_row = 0;
  FftPlan f1, f2;
};

// launch description of the persistent executor for one plan or one batch
struct ExecCtx {
  std::vector<int64_t> key;
  DevBuf plans, blocks, items, sync;
  int n_items = 0, n_sync = 0, grid = 0;
  // persistent launches: a host-visible word that the launch's last workgroup
  // sets when a dependency wait gave up, and an event after the launch; the
  // next launch on the context reports it
  uint32_t* herr = nullptr;
  uint32_t* derr = nullptr;
  hipEvent_t done = nullptr;
  bool pending = false;
  ExecCtx() = default;
  ExecCtx(const ExecCtx&) = delete;
  ExecCtx& operator=(const ExecCtx&) = delete;
  ~ExecCtx() {
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    if (herr) (void)hipHostFree(herr);
  }
  DevBuf items2;  // staged FFT: the row items (second launch)
  int n_items2 = 0;
  int ntw = 0;     // largest twiddle table (entries) of the blocks
  DevBuf sargs, sitems;  // staged batch: product arguments per plan, product items
  int n_sitems = 0;
  DevBuf witems;         // split-bf16 staged batch: chunked-product items of windowed plans
  int n_witems = 0;
  size_t wlds = 0;
  bool fft64 = false;    // plans and blocks describe float64 transforms
  bool xf = false;       // ... of float32 right-hand sides (the float32 paths)
};

bool is_jacobi(int f) { return f == SPT_LEGENDRE || f == SPT_JACOBI; }

// A complex plan's one block (Algorithm 1): full-spectrum tile boxes, the
// columns k0 .. k0 + kw - 1 of a box in 0 .. L + pad - 1 (past L - 1: the
// spectrum's first columns again), the transposed product's chunk lists.
struct CplxState {
  int L = 0, pad = 0, m_off = 0, c_lo = 0, c_hi = 0, n_chunks = 0;
  FftPlan fp;
  DevBuf winv, tw, meta, val64, val32, tptr, tents;
  std::vector<double> angles;  // row angles theta_j (SPT_CEXP) or phases phi_j
  int64_t nnz = 0, stored = 0;
  int max_band = 0;
  int max_kw = 0;    // widest tile box (columns)
  int max_list = 0;  // longest tile list of a transposed chunk
  double maxabs = 0.0, kappa = 0.0;
};

}  // namespace
}  // namespace spt

struct spt_plan {
  int family = 0;
  spt_params p{};
  int64_t N = 0;
  double eps1 = 0, eps2 = 0, zeta = 0;
  int mode = SPT_MODE_ROW;  // resolved mode
  int requested_mode = 0;
  std::vector<spt::BlockGeom> geom;
  int64_t tail = 0;
  std::vector<double> user_nodes;
  int device = 0;
  bool precomputed = false;
  uint32_t prepared = 0;
  int n_tiles = 0;
  // device state
  spt::DevBuf nodes, rowscale, ca, cb;
  double p0 = 0.0;
  std::vector<std::unique_ptr<spt::DevBlock>> blk;
  spt::DevBuf tail64, tail32, tailbf;
  // execute workspaces (half spectra, four-step intermediates): one per stream
  // that executed the plan, so that executes on different streams overlap
  struct Work {
    hipStream_t stream = nullptr;
    spt::DevBuf buf;
  };
  std::vector<std::unique_ptr<Work>> works;
  spt::DevBuf* work = nullptr;  // the workspace of the call in progress
  spt::DevBuf fftdesc64, fftdesc32;  // FftDesc per block for the fused FFT launch
  spt::DevBuf tilemeta;              // TileMeta per (tile, block)
  spt::DevBuf spmmblk64, spmmblk32;  // SpmmBlock per block
  spt::DevBuf tilemeta_bf, spmmblk_bf;  // the same for the pre-split boxes
  int64_t zper4 = 0;                    // sum of ldz4 over the blocks
  // windowed split-bf16 product: WinMeta per (tile group, block); used when
  // every group's windows fit the LDS of a workgroup
  spt::DevBuf winmeta;
  spt::DevBuf tseg, tent, tblk;  // the transposed product's segments, tile lists, blocks
  spt::DevBuf tred;              // its chunks of several segments
  int n_tseg = 0, n_tred = 0, n_tslot = 0, tseglen = 0;
  spt::DevBuf invdesc64, invdesc32;  // its single-workgroup inverse transforms
  int n_inv = 0, inv_threads = 64, inv_maxP = 1;
  int n_groups = 0;
  size_t win_lds = 0;
  int64_t win_cols = 0;
  int win_rg = 4;                  // groups of 16 right-hand sides per workgroup
  int win_waves = 1;               // waves per row tile of the windowed product
  int win_xlds = 0, win_tpad = 0;  // x of the direct tail in LDS (16-byte units), its pitch
  bool win_ok = false;
  bool win_chunked = false;  // the windows pass through LDS in chunks (too wide to fit)
  int fft_threads = 64, fft_maxP = 1;
  int fft_wgP = 1;  // most points of one workgroup of the fused FFT
  bool fwd_fused = false;  // every block's forward FFT is fused (DevBlock::fwd)
  int64_t serial = 0;  // changes with every precompute (keys of executor contexts)
  std::vector<std::unique_ptr<spt::ExecCtx>> ctx;  // executor contexts of spt_execute
  uint32_t exec_wait = spt::EXEC_WAIT_DEFAULT;      // persistent executor: wait bound, ticks
  std::unique_ptr<spt::CplxState> cx;  // complex generators (is_complex_family)
  spt_tuning tune{};                    // launch choices (spt_plan_set_tuning)
  // the float32 and split-bf16 paths' x-side FFTs in float64 arithmetic
  // (spt_params.reduced_fft)
  bool reduced_fft64 = false;
  double reduced_fft32_err = 0.0;
};

namespace spt {
namespace {

int64_t tiles_of(int64_t N) { return (N + TILE_ROWS - 1) / TILE_ROWS; }

void check_plan(spt_plan_t plan) {
  if (!plan) throw Error(SPT_E_INVALID_ARG, "plan is NULL");
}

void set_device(spt_plan_t plan) { SPT_HIP(hipSetDevice(plan->device)); }

// recurrence tables for the family, degrees 0 .. K
void family_tables(spt_plan_t plan, int64_t K, hipStream_t s) {
  const int f = plan->family;
  std::vector<double> a(K + 2, 0.0), b(K + 2, 0.0);
  if (is_jacobi(f)) {
    const double al = plan->p.alpha, be = plan->p.beta, ab = al + be;
    // orthonormal Jacobi recurrence x p_k = a_{k+1} p_{k+1} + b_k p_k + a_k p_{k-1}
    b[0] = (be - al) / (ab + 2.0);
    for (int64_t k = 1; k <= K + 1; ++k) {
      const double kk = (double)k;
      b[k] = (be * be - al * al) / ((2 * kk + ab) * (2 * kk + ab + 2));
    }
    a[1] = std::sqrt(4.0 * (1 + al) * (1 + be) / ((2 + ab) * (2 + ab) * (3 + ab)));
    for (int64_t k = 2; k <= K + 1; ++k) {
      const double kk = (double)k;
      const double num = 4.0 * kk * (kk + al) * (kk + be) * (kk + ab);
      const double den = (2 * kk + ab) * (2 * kk + ab) * (2 * kk + ab + 1) * (2 * kk + ab - 1);
      a[k] = std::sqrt(num / den);
    }
    const double log_mu0 = (ab + 1.0) * std::log(2.0) + std::lgamma(al + 1.0) +
                           std::lgamma(be + 1.0) - std::lgamma(ab + 2.0);
    plan->p0 = std::exp(-0.5 * log_mu0);
  } else if (f == SPT_HERMITE_FN) {
    for (int64_t k = 0; k <= K + 1; ++k) {
      a[k] = std::sqrt(2.0 / (double)(k + 1));
      b[k] = std::sqrt((double)k / (double)(k + 1));
    }
  }
  upload(plan->ca, a, s);
  upload(plan->cb, b, s);
}

FamilyArgs family_args(spt_plan_t plan, bool with_scale) {
  FamilyArgs f{};
  f.family = plan->family;
  f.power = plan->p.power;
  f.N = plan->N;
  f.unweighted = plan->p.unweighted;
  f.x = plan->nodes.as<double>();
  f.rowscale = with_scale ? plan->rowscale.as<double>() : nullptr;
  f.ca = plan->ca.as<double>();
  f.cb = plan->cb.as<double>();
  f.p0 = plan->p0;
  return f;
}

void compute_nodes(spt_plan_t plan, hipStream_t s) {
  const int64_t N = plan->N;
  const int f = plan->family;
  plan->nodes.alloc(N * sizeof(double));
  if (!plan->user_nodes.empty()) {
    SPT_HIP(hipMemcpyAsync(plan->nodes.p, plan->user_nodes.data(), N * sizeof(double),
                           hipMemcpyHostToDevice, s));
    return;
  }
  std::vector<double> d(N, 0.0), e2(N, 0.0);
  if (is_jacobi(f)) {
    const double al = plan->p.alpha, be = plan->p.beta, ab = al + be;
    d[0] = (be - al) / (ab + 2.0);
    for (int64_t k = 1; k < N; ++k) {
      const double kk = (double)k;
      d[k] = (be * be - al * al) / ((2 * kk + ab) * (2 * kk + ab + 2));
    }
    if (N > 1) e2[1] = 4.0 * (1 + al) * (1 + be) / ((2 + ab) * (2 + ab) * (3 + ab));
    for (int64_t k = 2; k < N; ++k) {
      const double kk = (double)k;
      e2[k] = 4.0 * kk * (kk + al) * (kk + be) * (kk + ab) /
              ((2 * kk + ab) * (2 * kk + ab) * (2 * kk + ab + 1) * (2 * kk + ab - 1));
    }
  } else if (f == SPT_LAGUERRE_FN) {
    for (int64_t k = 0; k < N; ++k) {
      d[k] = 2.0 * k + 1.0;
      e2[k] = (double)k * (double)k;
    }
  } else if (f == SPT_HERMITE_FN) {
    for (int64_t k = 0; k < N; ++k) e2[k] = 0.5 * (double)k;
  }
  double lo = 1e300, hi = -1e300;
  for (int64_t k = 0; k < N; ++k) {
    const double r = (k > 0 ? std::sqrt(e2[k]) : 0.0) + (k + 1 < N ? std::sqrt(e2[k + 1]) : 0.0);
    lo = std::min(lo, d[k] - r);
    hi = std::max(hi, d[k] + r);
  }
  const double pad = 1e-10 * std::max(1.0, std::max(std::fabs(lo), std::fabs(hi)));
  lo -= pad;
  hi += pad;
  DevBuf dd, de;
  upload(dd, d, s);
  upload(de, e2, s);
  launch_nodes(family_args(plan, false), dd.as<double>(), de.as<double>(), lo, hi,
               plan->nodes.as<double>(), s);
  SPT_HIP(hipStreamSynchronize(s));
}

template <typename C, typename T>
std::vector<C> to_vec2(const std::vector<long double>& re, const std::vector<long double>& im) {
  std::vector<C> out(re.size());
  for (size_t i = 0; i < re.size(); ++i) out[i] = C{(T)re[i], (T)im[i]};
  return out;
}

// Pass twiddles as two tables (exp(+2 pi i q/P), q < 128, then
// exp(+2 pi i 128 q/P), q <= P/128) and the unpack twiddles exp(+i pi k/P),
// k <= P, in long double
void twiddles(int P, std::vector<long double>& twr, std::vector<long double>& twi,
              std::vector<long double>& por, std::vector<long double>& poi) {
  const long double pi = 3.141592653589793238462643383279502884L;
  const int lo = 128, nhi = P / lo + 1;
  twr.resize(lo + nhi);
  twi.resize(lo + nhi);
  for (int q = 0; q < lo; ++q) {
    const long double a = 2.0L * pi * (long double)q / (long double)P;
    twr[q] = cosl(a);
    twi[q] = sinl(a);
  }
  for (int q = 0; q < nhi; ++q) {
    const long double a = 2.0L * pi * (long double)(q * lo) / (long double)P;
    twr[lo + q] = cosl(a);
    twi[lo + q] = sinl(a);
  }
  por.resize(P + 1);
  poi.resize(P + 1);
  for (int k = 0; k <= P; ++k) {
    const long double a = pi * (long double)k / (long double)P;
    por[k] = cosl(a);
    poi[k] = sinl(a);
  }
}

// two-level table of exp(i pi k / P), k <= P (the unpack twiddles):
// lo[q] = exp(i pi q / P), q < 128; hi[q] = exp(i pi 128 q / P), q <= P / 128
std::vector<double2> post_table(int P) {
  const long double pi = 3.141592653589793238462643383279502884L;
  const int lo = 128, nhi = P / lo + 1;
  std::vector<double2> t(lo + nhi);
  for (int q = 0; q < lo; ++q) {
    const long double a = pi * (long double)q / (long double)P;
    t[q] = double2{(double)cosl(a), (double)sinl(a)};
  }
  for (int q = 0; q < nhi; ++q) {
    const long double a = pi * (long double)(q * lo) / (long double)P;
    t[lo + q] = double2{(double)cosl(a), (double)sinl(a)};
  }
  return t;
}

size_t max_lds_bytes(int device) {
  int v = 0;
  SPT_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
  return (size_t)v;
}

// ---------------------------------------------------------------- precompute
// Executor geometry of a block: transforms with P <= split_points() run in one
// workgroup (several right-hand sides at a time when they fit); longer ones as
// four-step transforms P = P1 * P2, P1 the divisor nearest sqrt(P) for which a
// column item holds >= 8 columns and a row item >= 1 pair of rows.
int split_points() { return EXEC_POINTS; }

int log2_floor(int v) {
  int l = 0;
  while ((2 << l) <= v) ++l;
  return l;
}

uint32_t magic_of(int d) {
  return (uint32_t)((((uint64_t)1 << 32) + (uint64_t)d - 1) / (uint64_t)d);
}

// log2 of the most right-hand sides per workgroup of a short block's fused
// FFT (spt_tuning.fft_batch; 4 by default)
int fft_max_lb(spt_plan_t plan) {
  const int b = plan->tune.fft_batch;
  return b == 1 ? 0 : b == 2 ? 1 : 2;
}

// The split-bf16 product (spt_tuning.product): windowed unless the per-tile
// one is asked for; windows that do not fit LDS, or all windows when asked
// for, in chunks.
bool window_product_enabled(spt_plan_t plan) { return plan->tune.product != SPT_PRODUCT_TILE; }
bool window_chunks_forced(spt_plan_t plan) { return plan->tune.product == SPT_PRODUCT_CHUNKED; }

void exec_geometry(DevBlock& B) {
  const int P = B.P;
  B.four = P > split_points();
  if (!B.four) {
    B.f1 = make_fft_plan(P);
    return;
  }
  int best = 0;
  double best_score = 1e300;
  for (int p1 = 2; p1 <= 1024 && p1 < P; ++p1) {
    if (P % p1) continue;
    const int p2 = P / p1;
    if (2 * p2 > EXEC_POINTS) continue;
    int cw = 1;
    while (p2 % (2 * cw) == 0 && 2 * cw * p1 <= EXEC_POINTS && 2 * cw <= 64) cw *= 2;
    if (cw * p1 > EXEC_POINTS) continue;
    const double score = std::fabs(std::log((double)p1) - 0.5 * std::log((double)P)) +
                         (cw < 8 ? 10.0 : 0.0);
    if (score < best_score) {
      best_score = score;
      best = p1;
    }
  }
  if (!best) throw Error(SPT_E_UNSUPPORTED, "no four-step split of FFT length half " +
                                                std::to_string(P));
  B.P1 = best;
  B.P2 = P / best;
  int cw = 1;
  while (B.P2 % (2 * cw) == 0 && 2 * cw * B.P1 <= EXEC_POINTS && 2 * cw <= 64) cw *= 2;
  B.lcw = log2_floor(cw);
  const int npairs = B.P1 / 2 + 1;
  int gp = 1;
  while (4 * gp * B.P2 <= EXEC_POINTS && gp < npairs) gp *= 2;
  B.lgp = log2_floor(gp);
  B.n_col = B.P2 >> B.lcw;
  B.n_row = (npairs + gp - 1) / gp;
  B.f1 = make_fft_plan(B.P1);
  B.f2 = make_fft_plan(B.P2);
}

// The fused FFT's split of a transform of P points (FftDesc::half, by the
// plan's launch choice): by output parity by default for P >= 4096; by output
// residue mod 8 when asked for and 4 divides P; none when asked for and the
// whole transform fits one workgroup.
int fused_split(spt_plan_t plan, int P, size_t lds_max) {
  if (P < FUSED_HALF_MIN_P || P % 2) return FFT_SPLIT_NONE;
  const int t = plan->tune.fft_half;
  if (t == SPT_FFT_EIGHT && P % 4 == 0) return FFT_SPLIT_EIGHT;
  const bool whole_fits = fused_lds_bytes<double>(P, 128 + P / 128 + 1) <= lds_max;
  if (t == SPT_TUNE_OFF && whole_fits) return FFT_SPLIT_NONE;
  return FFT_SPLIT_PARITY;
}

// points of one workgroup's transform under a split
int fused_points(int P, int split) {
  return split == FFT_SPLIT_EIGHT ? P / 4 : split == FFT_SPLIT_PARITY ? P / 2 : P;
}

// Build the compressed block B (three passes over row panels).  With
// `estimate`, only 8 panels of 64 rows spread over the rows are transformed
// (maximum and tile boxes from those rows) and the return value is the
// estimated number of stored entries; nothing is packed.
int64_t build_block(spt_plan_t plan, DevBlock& B, hipStream_t s, size_t lds_max,
                    bool estimate = false) {
  const int L = B.g.L, P = L / 2;
  if (L % 2) throw Error(SPT_E_UNSUPPORTED, "odd block length " + std::to_string(L));
  B.P = P;
  // rows whose transform does not fit one workgroup's LDS go by four steps:
  // float64 points of the precomputation's row transforms and of the inverse
  // transforms (P * 16 bytes), and the fused execute FFT's points of a
  // transform or of a parity half with its two twiddle tables.  The forward
  // FFT of a four-step block stays fused while its split parts fit
  // (P <= FUSED_FWD_MAX_P).
  const int split = fused_split(plan, P, lds_max);
  const bool fits = fused_lds_bytes<double>(fused_points(P, split), 128 + P / 128 + 1) <= lds_max;
  const bool big = P > FUSED_MAX_P || (size_t)P * sizeof(double2) > lds_max || !fits;
  B.big = big;
  B.fwd = fits && (!big || (P <= FUSED_FWD_MAX_P && split != FFT_SPLIT_NONE));
  if (!big) B.fft = make_fft_plan(P);
  if (B.fwd) {
    B.half = split;
    B.fftw = make_fft_plan(fused_points(P, split), true);
  }
  exec_geometry(B);
  if (big && !B.four)
    throw Error(SPT_E_UNSUPPORTED, "no four-step split of FFT length " + std::to_string(L));
  // window over the L columns and its reciprocal
  std::vector<double> w(L), winv(L);
  std::vector<float> winv32(L);
  double sw = 0.0, swi = 0.0;
  for (int c = 0; c < L; ++c) {
    w[c] = kaiser((double)c, (double)(L - 1), plan->zeta);
    winv[c] = 1.0 / w[c];
    winv32[c] = (float)winv[c];
    sw += w[c] * w[c];
    if (c >= B.g.c_lo && c < B.g.c_hi) swi += winv[c] * winv[c];
  }
  B.kappa = std::sqrt(sw / L) * std::sqrt(swi / (B.g.c_hi - B.g.c_lo));
  DevBuf dw;
  upload(dw, w, s);
  upload(B.winv64, winv, s);
  upload(B.winv32, winv32, s);
  std::vector<long double> twr, twi, por, poi;
  twiddles(P, twr, twi, por, poi);
  upload(B.tw64, to_vec2<double2, double>(twr, twi), s);
  upload(B.post64, to_vec2<double2, double>(por, poi), s);
  upload(B.post32, to_vec2<float2, float>(por, poi), s);
  upload(B.posttw, post_table(P), s);

  const int64_t N = plan->N;
  const int64_t ntiles = plan->n_tiles;
  // rows per panel: A_e W rows (8 L bytes) + their half spectra (16 (P+1)
  // bytes) + the four-step intermediate (16 P bytes)
  int64_t budget = (int64_t)8 << 30;
  const int64_t row_bytes = 8 * (int64_t)L + 16 * (int64_t)(P + 1) + (big ? 16 * (int64_t)P : 0);
  int64_t rows = plan->p.panel_rows > 0 ? plan->p.panel_rows : budget / row_bytes;
  if (estimate) rows = 64;
  rows = std::max<int64_t>(TILE_ROWS, (rows / TILE_ROWS) * TILE_ROWS);
  rows = std::min<int64_t>(rows, ntiles * TILE_ROWS);
  const int64_t npanel = (N + rows - 1) / rows;
  DevBuf rowbuf, spec, maxbits, klo, khi, kcnt;
  rowbuf.alloc((size_t)rows * L * sizeof(double));
  spec.alloc((size_t)rows * (P + 1) * sizeof(double2));
  // four-step row transforms: one block descriptor, column and row items of
  // every panel row (row-major, so a shorter panel takes a prefix)
  DevBuf wbuf, fplan, fblock, fcol, frow;
  ExecArgs<double> fa4{};
  if (big) {
    wbuf.alloc((size_t)rows * P * sizeof(double2));
    ExecBlock<double> e{};
    e.tw = B.tw64.as<double2>();
    e.tw2 = B.posttw.as<double2>();
    e.ntw = 128 + P / 128 + 1;
    e.winv = nullptr;
    e.P = P;
    e.m_off = 0;
    e.c_lo = 0;
    e.c_hi = L;
    e.scale = 1.0 / std::sqrt((double)L);
    e.magic = magic_of(P);
    e.magic1 = magic_of(P + 1);
    e.magic2 = magic_of(B.P2);
    e.four = 1;
    e.P1 = B.P1;
    e.P2 = B.P2;
    e.lcw = B.lcw;
    e.lgp = B.lgp;
    e.n_col = B.n_col;
    e.n_row = B.n_row;
    e.f1 = B.f1;
    e.f2 = B.f2;
    upload(fblock, std::vector<ExecBlock<double>>{e}, s);
    ExecPlan<double> pl{};
    pl.Z = spec.as<double2>();
    pl.W = wbuf.as<double2>();
    pl.blocks = fblock.as<ExecBlock<double>>();
    pl.N = L;
    pl.R = (int)rows;
    pl.nblk = 1;
    upload(fplan, std::vector<ExecPlan<double>>{pl}, s);
    std::vector<int4> ic, ir;
    for (int r = 0; r < (int)rows; ++r) {
      for (int g = 0; g < B.n_col; ++g) ic.push_back(make_int4(item_head(ITEM_COL, 0), 0, r, g));
      for (int q = 0; q < B.n_row; ++q) ir.push_back(make_int4(item_head(ITEM_ROW, 0), 0, r, q));
    }
    upload(fcol, ic, s);
    upload(frow, ir, s);
    init_exec_kernels();
    if (exec_lds_bytes<double>(e.ntw) + 256 > lds_max)
      throw Error(SPT_E_UNSUPPORTED, "FFT twiddle tables exceed the LDS of a workgroup");
    fa4.plans = fplan.as<ExecPlan<double>>();
    fa4.ntw = e.ntw;
    fa4.X[0] = rowbuf.as<double>();
  }
  maxbits.alloc(sizeof(unsigned long long));
  klo.alloc(rows * sizeof(int32_t));
  khi.alloc(rows * sizeof(int32_t));
  kcnt.alloc(rows * sizeof(int32_t));
  SPT_HIP(hipMemsetAsync(maxbits.p, 0, sizeof(unsigned long long), s));
  const FamilyArgs fa = family_args(plan, is_jacobi(plan->family) && !plan->p.unweighted);
  // Appendix A (trig_conv_q > 0): the window's spectrum near m = 0 and the
  // tones of the generator; the band half-width B reaches where the window's
  // side lobes fall below 0.1 eps1 (else the block falls back to row FFTs)
  DevBuf vtbuf;
  TrigSpecArgs ta{};
  int qa = is_trig(plan->family) ? plan->p.trig_conv_q : 0;
  if (qa > 0) {
    const int D = 2 * qa + 8;
    std::vector<double> vr(D + 1), vi(D + 1);
    // cos, sin of 2 pi r / L once per residue r, then the sums over c
    const long double two_pi = 6.283185307179586476925286766559005768L;
    std::vector<long double> ct(L), st(L);
    for (int r = 0; r < L; ++r) {
      ct[r] = cosl(two_pi * (long double)r / (long double)L);
      st[r] = sinl(two_pi * (long double)r / (long double)L);
    }
    for (int m = 0; m <= D; ++m) {
      long double sr = 0.0L, si = 0.0L;
      int64_t r = 0;
      for (int c = 0; c < L; ++c) {
        sr += (long double)w[c] * ct[r];
        si -= (long double)w[c] * st[r];
        r += m;
        if (r >= L) r -= L;
      }
      vr[m] = (double)(sr / sqrtl((long double)L));
      vi[m] = (double)(si / sqrtl((long double)L));
    }
    const double v0 = std::hypot(vr[0], vi[0]);
    int bw = -1;
    for (int d = D; d >= 1; --d) {
      if (std::hypot(vr[d], vi[d]) >= 0.1 * plan->eps1 * v0) break;
      bw = d;
    }
    if (bw < 0 || bw > D - 2) {
      qa = 0;  // side lobes too high within D bins: row FFTs
    } else {
      // the window is real: vt_{-m} = conj(vt_m)
      std::vector<double2> vt(2 * qa + 1);
      for (int m = -qa; m <= qa; ++m)
        vt[m + qa] = m >= 0 ? double2{vr[m], vi[m]} : double2{vr[-m], -vi[-m]};
      upload(vtbuf, vt, s);
      ta.N = N;
      ta.L = L;
      ta.P = P;
      ta.m_off = B.g.m_off;
      ta.q = qa;
      ta.B = bw + 2;
      ta.vt = vtbuf.as<double2>();
      ta.sine = plan->family == SPT_SINE ? 1 : 0;
      if (plan->family == SPT_COS_POWER) {
        const int sp = plan->p.power;
        auto binom = [](int n, int k) {
          double r = 1.0;
          for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
          return r;
        };
        for (int k = 0; 2 * k < sp; ++k) {
          ta.tone[ta.ntones] = sp - 2 * k;
          ta.coef[ta.ntones++] = std::ldexp(binom(sp, k), 1 - sp);
        }
        if (sp % 2 == 0) {
          ta.tone[ta.ntones] = 0;
          ta.coef[ta.ntones++] = std::ldexp(binom(sp, sp / 2), -sp);
        }
      } else {
        ta.tone[0] = 1;
        ta.coef[0] = 1.0;
        ta.ntones = 1;
      }
    }
  }
  RowFftArgs ra{};
  ra.rows = rowbuf.as<double>();
  ra.spec = spec.as<double2>();
  ra.tw = B.tw64.as<double2>();
  ra.post = B.post64.as<double2>();
  ra.L = L;
  ra.P = P;
  ra.scale = 1.0 / std::sqrt((double)L);
  auto spectrum = [&](int64_t row0, int nr) {
    if (qa > 0) {
      SPT_HIP(hipMemsetAsync(spec.p, 0, (size_t)nr * (P + 1) * sizeof(double2), s));
      ta.row0 = row0;
      ta.nrows = nr;
      ta.spec = spec.as<double2>();
      launch_trig_spec(ta, s);
      return;
    }
    launch_rec_rows(fa, row0, nr, B.g.m_off, L, dw.as<double>(), rowbuf.as<double>(), s);
    if (!big) {
      ra.nrows = nr;
      launch_row_fft(ra, B.fft, s);
      return;
    }
    fa4.items = fcol.as<int4>();
    fa4.n_items = nr * B.n_col;
    launch_row_fft4(fa4, s);
    fa4.items = frow.as<int4>();
    fa4.n_items = nr * B.n_row;
    launch_row_fft4(fa4, s);
  };
  // the row panels: all rows, or the sample
  std::vector<std::pair<int64_t, int>> panels;
  if (estimate) {
    for (int i = 0; i < 8; ++i) {
      const int64_t r0 = ((int64_t)i * N / 8) & ~(int64_t)(TILE_ROWS - 1);
      if (panels.empty() || r0 >= panels.back().first + panels.back().second)
        panels.push_back({r0, (int)std::min<int64_t>(rows, N - r0)});
    }
  } else {
    for (int64_t p = 0; p < npanel; ++p)
      panels.push_back({p * rows, (int)std::min<int64_t>(rows, N - p * rows)});
  }
  const bool multi = panels.size() > 1;

  // pass 1: max |A_e W F| over the block (Alg. 1 step 1.3)
  for (const auto& pn : panels) {
    const int nr = pn.second;
    spectrum(pn.first, nr);
    launch_maxabs(spec.as<double2>(), (int64_t)nr * (P + 1), maxbits.as<unsigned long long>(), s);
  }
  unsigned long long bits = 0;
  SPT_HIP(hipMemcpyAsync(&bits, maxbits.p, sizeof(bits), hipMemcpyDeviceToHost, s));
  SPT_HIP(hipStreamSynchronize(s));
  double m2;
  std::memcpy(&m2, &bits, sizeof(m2));
  if (!std::isfinite(m2))
    throw Error(SPT_E_NUMERIC, "non-finite entries in the compressed block of length " +
                                   std::to_string(L));
  B.maxabs = std::sqrt(m2);
  const double thr = plan->eps1 * B.maxabs;

  // pass 2: band of every row, tile boxes on the host
  std::vector<int32_t> hlo(N), hhi(N, -1), hcnt(N);
  for (const auto& pn : panels) {
    const int nr = pn.second;
    if (multi) spectrum(pn.first, nr);
    launch_extents(spec.as<double2>(), nr, P, thr, klo.as<int32_t>(), khi.as<int32_t>(),
                   kcnt.as<int32_t>(), s);
    SPT_HIP(hipMemcpyAsync(hcnt.data() + pn.first, kcnt.p, nr * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    SPT_HIP(hipMemcpyAsync(hlo.data() + pn.first, klo.p, nr * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    SPT_HIP(hipMemcpyAsync(hhi.data() + pn.first, khi.p, nr * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    SPT_HIP(hipStreamSynchronize(s));
  }
  if (estimate) {
    // boxes of the sampled tiles, scaled to all tiles
    int64_t sum = 0, ntile_s = 0;
    for (const auto& pn : panels)
      for (int64_t t = pn.first / TILE_ROWS; t * TILE_ROWS < pn.first + pn.second; ++t) {
        int lo = 0x7FFFFFFF, hi = -1;
        for (int64_t q = 0; q < TILE_ROWS; ++q) {
          const int64_t n = t * TILE_ROWS + q;
          if (n >= N || hhi[n] < 0) continue;
          lo = std::min(lo, hlo[n]);
          hi = std::max(hi, hhi[n]);
        }
        if (hi >= 0) sum += (int64_t)(hi - (lo & ~3) + 1) * TILE_ROWS;
        ++ntile_s;
      }
    return ntile_s ? (int64_t)((double)sum * (double)ntiles / (double)ntile_s) : 0;
  }
  B.h_k0.assign(ntiles, 0);
  B.h_kw.assign(ntiles, 0);
  B.h_off.assign(ntiles, 0);
  int64_t total = 0;
  B.max_band = 0;
  for (int64_t t = 0; t < ntiles; ++t) {
    int lo = 0x7FFFFFFF, hi = -1;
    for (int64_t q = 0; q < TILE_ROWS; ++q) {
      const int64_t n = t * TILE_ROWS + q;
      if (n >= N || hhi[n] < 0) continue;
      lo = std::min(lo, hlo[n]);
      hi = std::max(hi, hhi[n]);
      B.max_band = std::max(B.max_band, hhi[n] - hlo[n] + 1);
    }
    // boxes start at a multiple of 4 columns (16-byte loads of pre-split spectra)
    B.h_k0[t] = hi < 0 ? 0 : (lo & ~3);
    B.h_kw[t] = hi < 0 ? 0 : hi - B.h_k0[t] + 1;
    B.h_off[t] = total;
    total += (int64_t)B.h_kw[t] * TILE_ROWS;
  }
  B.stored = total;
  upload(B.k0, B.h_k0, s);
  upload(B.kw, B.h_kw, s);
  upload(B.off, B.h_off, s);
  {
    // the row tiles whose boxes meet each TCHUNK columns of the half spectrum
    const int nch = (P + 1 + TCHUNK - 1) / TCHUNK;
    std::vector<int32_t> ptr(nch + 1, 0);
    auto chunks = [&](int64_t t, int& c0, int& c1) {
      c0 = B.h_k0[t] / TCHUNK;
      c1 = std::min(nch - 1, (B.h_k0[t] + B.h_kw[t] - 1) / TCHUNK);
    };
    for (int64_t t = 0; t < ntiles; ++t) {
      if (B.h_kw[t] <= 0) continue;
      int c0, c1;
      chunks(t, c0, c1);
      for (int c = c0; c <= c1; ++c) ++ptr[c + 1];
    }
    for (int c = 0; c < nch; ++c) ptr[c + 1] += ptr[c];
    std::vector<TChunkEnt> ents(ptr[nch]);
    std::vector<int32_t> pos(ptr.begin(), ptr.end() - 1);
    for (int64_t t = 0; t < ntiles; ++t) {
      if (B.h_kw[t] <= 0) continue;
      int c0, c1;
      chunks(t, c0, c1);
      for (int c = c0; c <= c1; ++c)
        ents[pos[c]++] = TChunkEnt{B.h_off[t], (int32_t)t, B.h_k0[t], B.h_kw[t], 0};
    }
    B.h_tptr = std::move(ptr);
    B.h_tent = std::move(ents);
  }
  const bool want64 = plan->prepared & (1u << SPT_F64);
  const bool want32 = plan->prepared & ((1u << SPT_F32) | (1u << SPT_SPLIT_BF16));
  B.val64.reset();
  B.val32.reset();
  if (want64) B.val64.alloc(std::max<int64_t>(total, 1) * sizeof(double2));
  if (want32) B.val32.alloc(std::max<int64_t>(total, 1) * sizeof(float2));

  // pass 3: pack the kept entries (times c_k) into the tiles
  for (const auto& pn : panels) {
    const int nr = pn.second;
    if (multi) spectrum(pn.first, nr);
    launch_pack(spec.as<double2>(), pn.first, nr, N, P, thr, B.k0.as<int32_t>(),
                B.kw.as<int32_t>(), B.off.as<int64_t>(), (int)(pn.first / TILE_ROWS),
                want64 ? B.val64.as<double2>() : nullptr, want32 ? B.val32.as<float2>() : nullptr,
                s);
  }
  // pre-split boxes of the split-bf16 path (3 pieces x 512 bfloat16 per step)
  B.valbf.reset();
  B.ldz4 = ((P + 1) + 3) & ~3;
  B.h_soff.assign(ntiles, 0);
  int64_t soff = 0;
  for (int64_t t = 0; t < ntiles; ++t) {
    B.h_soff[t] = soff;
    soff += (int64_t)((B.h_kw[t] + 15) / 16) * 3 * 512;
  }
  if (plan->prepared & (1u << SPT_SPLIT_BF16)) {
    upload(B.soff, B.h_soff, s);
    B.valbf.alloc((size_t)std::max<int64_t>(soff, 1) * sizeof(uint16_t));
    launch_split_pack(B.val32.as<float2>(), B.kw.as<int32_t>(), B.off.as<int64_t>(),
                      B.soff.as<int64_t>(), (int)ntiles, B.valbf.as<uint16_t>(), s);
  }
  SPT_HIP(hipStreamSynchronize(s));
  int64_t nnz = 0;
  for (int64_t n = 0; n < N; ++n) nnz += hcnt[n];
  B.nnz = nnz;
  return B.stored;
}

void build_tail(spt_plan_t plan, hipStream_t s) {
  plan->tail64.reset();
  plan->tail32.reset();
  plan->tailbf.reset();
  const int64_t t = plan->tail;
  if (t <= 0) return;
  const int64_t ldt = (int64_t)plan->n_tiles * TILE_ROWS;
  plan->tail64.alloc((size_t)t * ldt * sizeof(double));
  launch_rec_tail(family_args(plan, is_jacobi(plan->family) && !plan->p.unweighted), (int)t,
                  plan->tail64.as<double>(), s);
  if (plan->prepared & ((1u << SPT_F32) | (1u << SPT_SPLIT_BF16))) {
    plan->tail32.alloc((size_t)t * ldt * sizeof(float));
    launch_to_f32(plan->tail64.as<double>(), plan->tail32.as<float>(), t * ldt, s);
  }
  if (plan->prepared & (1u << SPT_SPLIT_BF16)) {
    const int64_t tsteps = (t + 31) / 32;
    plan->tailbf.alloc((size_t)plan->n_tiles * tsteps * 3 * 512 * sizeof(uint16_t));
    launch_split_tail(plan->tail32.as<float>(), ldt, (int)t, plan->n_tiles,
                      plan->tailbf.as<uint16_t>(), s);
  }
  SPT_HIP(hipStreamSynchronize(s));
}

// right-hand sides per ITEM_FFT of a block (a power of two <= 64)
int fft_batch(int P, int64_t R) {
  int nb = 1;
  while (2 * nb * P <= EXEC_POINTS && 2 * nb <= 64 && nb < R) nb *= 2;
  return nb;
}

int cu_count(int device) {
  int v = 0;
  SPT_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device));
  return v;
}

// executor workspace per right-hand side, in complex values: the half spectra
// of every block, then the four-step intermediates
int64_t z_per_rhs(spt_plan_t plan) {
  int64_t n = 0;
  for (auto& B : plan->blk) n += B->P + 1;
  return n;
}
int64_t w_per_rhs(spt_plan_t plan) {
  int64_t n = 0;
  for (auto& B : plan->blk)
    if (B->four) n += B->P;
  return n;
}
// the transposed product's partial sums, after the four-step intermediates
int64_t t_per_rhs(spt_plan_t plan) { return (int64_t)plan->n_tslot * TCHUNK; }

int engine_of(int prec) { return prec == SPT_F64 ? 0 : prec == SPT_F32 ? 1 : 2; }

// Build the items, descriptors and counters of one launch over `count` plans
// (persistent executor), or the two FFT launches of one plan (staged; with
// split, the spectra go to the pre-split planes and the four-step
// intermediates follow them in the workspace).
template <typename T>
void build_exec_ctx(ExecCtx& c, const spt_plan_t* plans, const int64_t* R, int count, int prec,
                    hipStream_t s, bool staged = false) {
  const bool split = staged && prec == SPT_SPLIT_BF16;
  using C = cplx_t<T>;
  const bool dbl = std::is_same<T, double>::value;
  std::vector<ExecPlan<T>> ep(count);
  std::vector<ExecBlock<T>> eb;
  std::vector<size_t> first(count);
  std::vector<int4> spmm;
  std::vector<std::vector<FftItemBlock>> fblk(count);
  std::vector<int64_t> fR(R, R + count);
  int nsync = EXEC_SYNC_BASE;
  for (int i = 0; i < count; ++i) {
    spt_plan_t plan = plans[i];
    const int r = (int)R[i];
    const int groups = (r + 15) / 16;
    first[i] = eb.size();
    int64_t zoff = 0, woff = 0, zoff4 = 0;
    for (size_t b = 0; b < plan->blk.size(); ++b) {
      const DevBlock& B = *plan->blk[b];
      ExecBlock<T> e{};
      e.winv = (const T*)(dbl ? B.winv64.p : B.winv32.p);
      e.tw = B.tw64.as<double2>();
      e.tw2 = B.posttw.as<double2>();
      e.ntw = 128 + B.P / 128 + 1;
      c.ntw = std::max(c.ntw, e.ntw);
      e.post = (const C*)(dbl ? B.post64.p : B.post32.p);
      e.val = (const C*)(dbl ? B.val64.p : B.val32.p);
      e.zoff = zoff;
      e.zoff4 = zoff4;
      e.ldz4 = B.ldz4;
      e.P = B.P;
      e.m_off = B.g.m_off;
      e.c_lo = B.g.c_lo;
      e.c_hi = B.g.c_hi;
      e.scale = (T)(1.0 / std::sqrt((double)B.g.L));
      e.magic = magic_of(B.P);
      e.magic1 = magic_of(B.P + 1);
      e.four = B.four;
      e.f1 = B.f1;
      e.ctr = nsync;
      nsync += groups;
      if (B.four) {
        e.woff = woff;
        woff += B.P;
        e.P1 = B.P1;
        e.P2 = B.P2;
        e.magic2 = magic_of(B.P2);
        e.lcw = B.lcw;
        e.lgp = B.lgp;
        e.n_col = B.n_col;
        e.n_row = B.n_row;
        e.f2 = B.f2;
        e.cctr = nsync;
        nsync += r;
        e.parts = B.n_row;
      } else {
        e.parts = 1;
      }
      fblk[i].push_back(FftItemBlock{B.P, B.four, B.n_col, B.n_row, fft_batch(B.P, r)});
      eb.push_back(e);
      zoff += B.P + 1;
      zoff4 += B.ldz4;
    }
    ExecPlan<T>& P = ep[i];
    P.Z = plan->work->as<C>();
    P.W = P.Z + (int64_t)r * zoff;
    if (split) {
      P.Zs = plan->work->as<uint32_t>();
      P.zplane = (int64_t)r * zoff4;
      P.W = reinterpret_cast<C*>(P.Zs + 3 * P.zplane);
    } else if (dbl && prec == SPT_F32) {
      // float32 spectra of float64 transforms; the float64 intermediate sits
      // behind them (at twice their size)
      P.Zf = plan->work->as<float2>();
    }
    P.meta = plan->tilemeta.as<TileMeta>();
    P.tailmat = (const T*)(dbl ? plan->tail64.p : plan->tail32.p);
    P.N = plan->N;
    P.R = r;
    P.nblk = (int)plan->blk.size();
    P.n_tiles = plan->n_tiles;
    P.tail = (int)plan->tail;
    if (!staged)
      for (int t = 0; t < plan->n_tiles; t += 2)
        for (int r0 = 0; r0 < r; r0 += 64)
          spmm.push_back(make_int4(item_head(ITEM_SPMM, i), t, r0, 0));
  }
  upload(c.blocks, eb, s);
  for (int i = 0; i < count; ++i) ep[i].blocks = c.blocks.as<ExecBlock<T>>() + first[i];
  upload(c.plans, ep, s);
  // FFT items: staged, the column and single-workgroup items in a first
  // launch, the row items in a second; persistent, one queue with the product
  // items last
  FftItemLists fl;
  build_fft_item_lists(fblk, fR, fl);
  std::string why;
  if (!check_fft_item_lists(fblk, fR, fl, &why))
    throw Error(SPT_E_UNSUPPORTED, "FFT work lists failed their check: " + why);
  auto as_int4 = [](const std::vector<WorkItem>& v) {
    std::vector<int4> o(v.size());
    for (size_t k = 0; k < v.size(); ++k) o[k] = make_int4(v[k].x, v[k].y, v[k].z, v[k].w);
    return o;
  };
  std::vector<int4> items = as_int4(fl.first);
  if (staged) {
    upload(c.items2, as_int4(fl.second), s);
    c.n_items2 = (int)fl.second.size();
  } else {
    const std::vector<int4> rows = as_int4(fl.second);
    items.insert(items.end(), rows.begin(), rows.end());
    items.insert(items.end(), spmm.begin(), spmm.end());
  }
  upload(c.items, items, s);
  c.n_items = (int)items.size();
  c.n_sync = nsync;
  c.sync.alloc((size_t)nsync * sizeof(uint32_t));
  SPT_HIP(hipMemsetAsync(c.sync.p, 0, c.sync.bytes, s));
  const uint32_t wait = plans[0]->exec_wait;
  SPT_HIP(hipMemcpyAsync(c.sync.as<uint32_t>() + EXEC_SYNC_WAIT, &wait, sizeof(wait),
                         hipMemcpyHostToDevice, s));
  SPT_HIP(hipStreamSynchronize(s));
  init_exec_kernels();
  if (exec_lds_bytes<T>(c.ntw) + 256 > max_lds_bytes(plans[0]->device))
    throw Error(SPT_E_UNSUPPORTED, "FFT twiddle tables exceed the LDS of a workgroup");
  const int occ = std::max(1, exec_occupancy(engine_of(prec), c.ntw));
  c.grid = std::max(1, std::min(c.n_items, occ * cu_count(plans[0]->device)));
}

template <typename T>
std::vector<FftDesc<T>> fft_descs(spt_plan_t plan) {
  using C = cplx_t<T>;
  const bool dbl = std::is_same<T, double>::value;
  std::vector<FftDesc<T>> d;
  int64_t zoff = 0, zoff4 = 0;
  for (auto& Bp : plan->blk) {
    DevBlock& B = *Bp;
    FftDesc<T> e{};
    e.winv = (const T*)(dbl ? B.winv64.p : B.winv32.p);
    e.tw = B.tw64.as<double2>();
    e.post = (const C*)(dbl ? B.post64.p : B.post32.p);
    e.zoff = zoff;
    e.fp = B.fftw;
    e.L = B.g.L;
    e.m_off = B.g.m_off;
    e.c_lo = B.g.c_lo;
    e.c_hi = B.g.c_hi;
    e.ldz = B.P + 1;
    e.scale = (T)(1.0 / std::sqrt((double)B.g.L));
    e.zoff4 = zoff4;
    e.ldz4 = B.ldz4;
    e.tw2 = B.posttw.as<double2>();
    e.ntw = 128 + B.P / 128 + 1;
    // up to 4 right-hand sides per workgroup of a short block: 2^lb transforms
    // interleaved put 64 / 2^lb consecutive points of a row in a wave's
    // loads and stores.  A batched workgroup stays below the launch's largest
    // transform: its interleaved passes take longer than a single transform
    // of the same points, and it would become the launch's last workgroup.
    e.half = B.half;
    e.lb = 0;
    while (!B.half && e.lb < fft_max_lb(plan) && ((int64_t)B.fftw.P << (e.lb + 1)) < plan->fft_wgP)
      ++e.lb;
    B.lbw = e.lb;
    d.push_back(e);
    zoff += B.P + 1;
    zoff4 += B.ldz4;
  }
  return d;
}

// Windows of the windowed split-bf16 product: for each group of WIN_TILES row
// tiles and each block, the union of the tiles' boxes (columns k0 .. k0 +
// ceil4(kw) - 1, which is what a step reads) and its place in LDS.
void build_windows(spt_plan_t plan, hipStream_t s) {
  plan->win_ok = false;
  plan->win_chunked = false;
  plan->win_lds = 0;
  const int nblk = (int)plan->blk.size();
  plan->n_groups = (plan->n_tiles + WIN_TILES - 1) / WIN_TILES;
  if (nblk == 0 || nblk > 64 || !window_product_enabled(plan)) return;
  for (auto& B : plan->blk)
    if (B->h_soff.empty()) return;
  // union of the boxes of each (group, block): [lo, hi) columns
  std::vector<std::pair<int, int>> span((size_t)plan->n_groups * nblk, {0, 0});
  for (int gi = 0; gi < plan->n_groups; ++gi)
    for (int b = 0; b < nblk; ++b) {
      const DevBlock& B = *plan->blk[b];
      int lo = INT32_MAX, hi = 0;
      for (int t = gi * WIN_TILES; t < std::min(plan->n_tiles, (gi + 1) * WIN_TILES); ++t)
        if (B.h_kw[t] > 0) {
          lo = std::min(lo, B.h_k0[t]);
          hi = std::max(hi, B.h_k0[t] + ((B.h_kw[t] + 3) & ~3));
        }
      if (lo < hi) span[(size_t)gi * nblk + b] = {lo, hi};
    }
  const int tpad = plan->tail > 0 ? 32 * (int)((plan->tail + 31) / 32) + 4 : 0;
  const size_t lds_max = max_lds_bytes(plan->device);
  // layout for rg groups of 16 right-hand sides: windows, then the tail's x
  auto layout = [&](int rg, std::vector<WinMeta>* win, int64_t* cols) {
    const int nr = 16 * rg;
    int64_t most = 0, c = 0;
    for (int gi = 0; gi < plan->n_groups; ++gi) {
      int64_t units = 0;
      for (int b = 0; b < nblk; ++b) {
        const auto sp = span[(size_t)gi * nblk + b];
        WinMeta w{};
        w.pitch = 3;
        if (sp.first < sp.second) {
          w.k0 = sp.first;
          w.w4 = (sp.second - sp.first) / 4;
          w.pitch = std::max(w.w4 | 1, 3);
          w.magic = magic_of(w.pitch);
          w.units = (3 * nr * w.pitch + 63) & ~63;
          w.lds = (int32_t)units;
          units += w.units;
          c += sp.second - sp.first;
        }
        if (win) (*win)[(size_t)gi * nblk + b] = w;
      }
      most = std::max(most, units);
    }
    if (cols) *cols = c;
    return std::make_pair(most, (size_t)most * 16 + (size_t)tpad * nr * sizeof(float));
  };
  // 64 right-hand sides per workgroup (more reuse of each matrix piece) when
  // two such workgroups still fit a CU's LDS, else 32, which leaves room for
  // the FFTs of other streams beside the product (spt_tuning.window_rhs)
  int rg = 2 * layout(4, nullptr, nullptr).second <= lds_max ? 4 : 2;
  if (plan->tune.window_rhs == 64) rg = 4;
  if (plan->tune.window_rhs == 32) rg = 2;
  plan->win_waves = 1;
  if (plan->tune.product == SPT_PRODUCT_WINDOW_2W) {
    rg = 4;
    plan->win_waves = 2;
  }
  std::vector<WinMeta> win((size_t)plan->n_groups * nblk);
  int64_t cols = 0;
  const auto lay = layout(rg, &win, &cols);
  if (lay.second > lds_max || window_chunks_forced(plan)) {
    // the windows pass through LDS in chunks (64 right-hand sides per workgroup)
    if (spmm_chunk_lds_bytes(tpad) > lds_max) return;
    upload(plan->winmeta, win, s);
    plan->win_rg = 4;
    plan->win_tpad = tpad;
    plan->win_lds = spmm_chunk_lds_bytes(tpad);
    plan->win_cols = cols;
    plan->win_chunked = true;
    plan->win_ok = true;
    return;
  }
  upload(plan->winmeta, win, s);
  plan->win_rg = rg;
  plan->win_xlds = (int)lay.first;
  plan->win_tpad = tpad;
  plan->win_lds = lay.second;
  plan->win_cols = cols;
  plan->win_ok = true;
}

void build_fft_descs(spt_plan_t plan, hipStream_t s) {
  plan->fft_threads = 64;
  plan->fft_maxP = 1;
  for (auto& B : plan->blk) exec_geometry(*B);
  plan->fft_wgP = 1;
  plan->fwd_fused = true;
  for (auto& B : plan->blk) {
    plan->fwd_fused = plan->fwd_fused && B->fwd;
    plan->fft_threads = std::max(plan->fft_threads, B->fftw.threads);
    plan->fft_maxP = std::max(plan->fft_maxP, B->P);
    plan->fft_wgP = std::max(plan->fft_wgP, B->fftw.P);
  }
  upload(plan->fftdesc64, fft_descs<double>(plan), s);
  upload(plan->fftdesc32, fft_descs<float>(plan), s);
  // banded product tables: tile boxes of every block, tile-major
  const int nblk = (int)plan->blk.size();
  std::vector<TileMeta> meta((size_t)plan->n_tiles * std::max(nblk, 1));
  std::vector<SpmmBlock<double>> b64;
  std::vector<SpmmBlock<float>> b32;
  int64_t zoff = 0;
  for (int b = 0; b < nblk; ++b) {
    const DevBlock& B = *plan->blk[b];
    for (int t = 0; t < plan->n_tiles; ++t)
      meta[(size_t)t * nblk + b] = TileMeta{B.h_k0[t], B.h_kw[t], B.h_off[t]};
    b64.push_back(SpmmBlock<double>{B.val64.as<double2>(), zoff, B.P + 1, 0});
    b32.push_back(SpmmBlock<float>{B.val32.as<float2>(), zoff, B.P + 1, 0});
    zoff += B.P + 1;
  }
  upload(plan->tilemeta, meta, s);
  upload(plan->spmmblk64, b64, s);
  upload(plan->spmmblk32, b32, s);
  // pre-split boxes: the same tiles, offsets into the bfloat16 pieces
  std::vector<TileMeta> meta_bf((size_t)plan->n_tiles * std::max(nblk, 1));
  std::vector<SpmmSplitBlock> bbf;
  int64_t zoff4 = 0;
  for (int b = 0; b < nblk; ++b) {
    const DevBlock& B = *plan->blk[b];
    if (!B.h_soff.empty())
      for (int t = 0; t < plan->n_tiles; ++t)
        meta_bf[(size_t)t * nblk + b] = TileMeta{B.h_k0[t], B.h_kw[t], B.h_soff[t]};
    bbf.push_back(SpmmSplitBlock{B.valbf.as<uint16_t>(), zoff4, B.ldz4, 0});
    zoff4 += B.ldz4;
  }
  plan->zper4 = zoff4;
  upload(plan->tilemeta_bf, meta_bf, s);
  upload(plan->spmmblk_bf, bbf, s);
  build_windows(plan, s);
  // the transposed product's segments of every block, in one list: a chunk
  // whose tiles fit one segment stores, the segments of the others get slots of
  // partial sums.  Segments hold TSEG tiles, or more where the slots would need
  // more memory than 4 times the half spectra (nearly dense plans: every chunk
  // meets most tiles).
  static_assert(MAX_BLOCKS <= (1 << TSEG_BLOCK_BITS), "segment block field");
  int seglen = TSEG;
  {
    const int64_t budget = std::max<int64_t>(256, z_per_rhs(plan) / 8);
    auto count_slots = [&](int len) {
      int64_t n = 0;
      for (auto& Bp : plan->blk)
        for (size_t c = 0; c + 1 < Bp->h_tptr.size(); ++c) {
          const int cnt = Bp->h_tptr[c + 1] - Bp->h_tptr[c];
          if (cnt > len) n += (cnt + len - 1) / len;
        }
      return n;
    };
    while (count_slots(seglen) > budget && seglen < (1 << 24)) seglen *= 2;
  }
  std::vector<int4> tseg, tred;
  std::vector<TChunkEnt> tent;
  std::vector<TBlkInfo> tblk;
  int64_t uoff = 0;
  int slots = 0;
  for (int b = 0; b < nblk; ++b) {
    const DevBlock& B = *plan->blk[b];
    const int base = (int)tent.size();
    for (size_t c = 0; c + 1 < B.h_tptr.size(); ++c) {
      const int e0 = B.h_tptr[c], e1 = B.h_tptr[c + 1];
      if (e1 == e0) {
        tred.push_back(int4{b, (int)c, 0, 0});  // no tile meets the chunk: zeros
      } else if (e1 - e0 <= seglen) {
        tseg.push_back(int4{(int)c, e0 + base, e1 + base, (b << 1) | 1});
      } else {
        tred.push_back(int4{b, (int)c, slots, 0});
        for (int e = e0; e < e1; e += seglen) {
          ++tred.back().w;
          tseg.push_back(int4{(int)c, e + base, std::min(e + seglen, e1) + base,
                              (slots++ << (TSEG_BLOCK_BITS + 1)) | (b << 1)});
        }
      }
    }
    tent.insert(tent.end(), B.h_tent.begin(), B.h_tent.end());
    tblk.push_back(TBlkInfo{B.val64.p, B.val32.p, uoff, B.P, 0});
    uoff += B.P + 1;
  }
  if ((int64_t)slots >= ((int64_t)1 << (31 - TSEG_BLOCK_BITS - 1)))
    throw Error(SPT_E_UNSUPPORTED, "too many transposed-product segments");
  plan->n_tseg = (int)tseg.size();
  plan->n_tred = (int)tred.size();
  plan->n_tslot = slots;
  plan->tseglen = seglen;
  if (tseg.empty()) tseg.push_back(int4{0, 0, 0, 0});
  if (tred.empty()) tred.push_back(int4{0, 0, 0, 0});
  upload(plan->tred, tred, s);
  if (tent.empty()) tent.push_back(TChunkEnt{});
  if (tblk.empty()) tblk.push_back(TBlkInfo{});
  upload(plan->tseg, tseg, s);
  upload(plan->tent, tent, s);
  upload(plan->tblk, tblk, s);
  // the single-workgroup inverse transforms of the transposed product
  std::vector<InvFftDesc<double>> inv64;
  std::vector<InvFftDesc<float>> inv32;
  plan->inv_threads = 64;
  plan->inv_maxP = 1;
  uoff = 0;
  for (int b = 0; b < nblk; ++b) {
    const DevBlock& B = *plan->blk[b];
    if (!B.big) {
      const double sc = 1.0 / std::sqrt((double)B.g.L);
      inv64.push_back(InvFftDesc<double>{B.winv64.as<double>(), B.tw64.as<double2>(),
                                         B.post64.as<double2>(), uoff, B.P, (int)B.g.m_off,
                                         (int)B.g.c_lo, (int)B.g.c_hi, sc, B.fft});
      inv32.push_back(InvFftDesc<float>{B.winv32.as<float>(), B.tw64.as<double2>(),
                                        B.post32.as<float2>(), uoff, B.P, (int)B.g.m_off,
                                        (int)B.g.c_lo, (int)B.g.c_hi, (float)sc, B.fft});
      plan->inv_threads = std::max(plan->inv_threads, B.fft.threads);
      plan->inv_maxP = std::max(plan->inv_maxP, B.P);
    }
    uoff += B.P + 1;
  }
  plan->n_inv = (int)inv64.size();
  if (inv64.empty()) {
    inv64.push_back(InvFftDesc<double>{});
    inv32.push_back(InvFftDesc<float>{});
  }
  upload(plan->invdesc64, inv64, s);
  upload(plan->invdesc32, inv32, s);
}

void choose_reduced_fft(spt_plan_t plan, hipStream_t s);
bool inv_four_step(spt_plan_t plan, const DevBlock& B);
template <typename T>
void execute_transposed_t(spt_plan_t plan, const T* F, T* Y, int64_t R, hipStream_t s);

void precompute_complex(spt_plan_t plan, hipStream_t s);

void precompute(spt_plan_t plan, hipStream_t s) {
  set_device(plan);
  if (is_complex_family(plan->family)) {
    plan->precomputed = false;
    plan->serial = next_serial();
    plan->prepared = plan->p.precisions ? plan->p.precisions : 3u;
    plan->n_tiles = (int)tiles_of(plan->N);
    plan->works.clear();
    plan->work = nullptr;
    precompute_complex(plan, s);
    plan->precomputed = true;
    return;
  }
  const size_t lds_max = max_lds_bytes(plan->device);
  init_fft_kernels(lds_max);
  init_spmm_kernels(lds_max);
  plan->precomputed = false;
  plan->ctx.clear();
  plan->serial = next_serial();
  plan->prepared = plan->p.precisions ? plan->p.precisions : 7u;
  plan->n_tiles = (int)tiles_of(plan->N);
  int64_t K = plan->N;
  for (auto& g : plan->geom) K = std::max<int64_t>(K, g.L + std::max(0, g.m_off));
  family_tables(plan, K + 2, s);
  compute_nodes(plan, s);
  if (is_jacobi(plan->family) && !plan->p.unweighted) {
    plan->rowscale.alloc(plan->N * sizeof(double));
    launch_weights(family_args(plan, false), plan->rowscale.as<double>(), s);
  }
  SPT_HIP(hipStreamSynchronize(s));
  plan->blk.clear();
  plan->mode = plan->requested_mode == SPT_MODE_DIRECT ? SPT_MODE_DIRECT : SPT_MODE_ROW;
  // AUTO: fewest stored reals, the compressed blocks (complex = 2 reals, plus
  // the direct tail) against the dense matrix; decided on the built blocks up
  // to N = AUTO_EXACT_N, from sampled rows above
  const bool autom = plan->requested_mode == SPT_MODE_AUTO;
  if (plan->mode == SPT_MODE_ROW && autom && plan->N > AUTO_EXACT_N) {
    int64_t est = plan->tail * plan->N;
    for (auto& g : plan->geom) {
      DevBlock tmp;
      tmp.g = g;
      est += 2 * build_block(plan, tmp, s, lds_max, true);
    }
    if (est > plan->N * plan->N) plan->mode = SPT_MODE_DIRECT;
  }
  if (plan->mode == SPT_MODE_ROW) {
    for (auto& g : plan->geom) {
      auto B = std::make_unique<DevBlock>();
      B->g = g;
      build_block(plan, *B, s, lds_max);
      plan->blk.push_back(std::move(B));
    }
    if (autom && plan->N <= AUTO_EXACT_N) {
      int64_t stored = 0;
      for (auto& B : plan->blk) stored += 2 * B->stored;
      stored += plan->tail * plan->N;
      if (stored > plan->N * plan->N) {
        plan->blk.clear();
        plan->mode = SPT_MODE_DIRECT;
      }
    }
  }
  if (plan->mode == SPT_MODE_DIRECT) plan->tail = plan->N;
  build_tail(plan, s);
  build_fft_descs(plan, s);
  choose_reduced_fft(plan, s);
  plan->precomputed = true;
}

template <typename T>
void execute_staged_t(spt_plan_t plan, const T* X, T* Y, int64_t R, int prec, hipStream_t s,
                      void* ws = nullptr);

// Arithmetic of the float32 and split-bf16 paths' x-side FFTs
// (spt_params.reduced_fft).  The automatic choice runs 4 right-hand sides
// x ~ N(0, 1) (a fixed seed) through the split-bf16 path (the float32 path
// when only that is prepared) with float32 FFTs and keeps them when the result
// is within REDUCED_TOTAL_BUDGET of the float64 path's (relative 2-norm, max
// over the right-hand sides): 70% of the 1e-6 target, the rest a margin for
// other inputs.  Without a float64 path the float32 FFTs are compared with
// float64 ones and kept within REDUCED_FFT32_BUDGET.  What float32 FFTs add is
// their rounding of the half spectra, amplified in the product by kappa.
constexpr double REDUCED_TOTAL_BUDGET = 7e-7;
constexpr double REDUCED_FFT32_BUDGET = 5e-7;

void choose_reduced_fft(spt_plan_t plan, hipStream_t s) {
  plan->reduced_fft64 = plan->p.reduced_fft == 2;
  plan->reduced_fft32_err = 0.0;
  const bool sp = plan->prepared & (1u << SPT_SPLIT_BF16);
  const bool f32 = plan->prepared & (1u << SPT_F32);
  const bool f64 = plan->prepared & (1u << SPT_F64);
  if (plan->p.reduced_fft != 0 || plan->blk.empty() || !(sp || f32)) return;
  const int prec = sp ? SPT_SPLIT_BF16 : SPT_F32;
  const int R = 4;
  const int64_t N = plan->N;
  const size_t n = (size_t)R * N;
  std::vector<double> hx(n);
  std::mt19937_64 gen(0x5eed2004116ull);
  std::normal_distribution<double> nd;
  for (double& v : hx) v = nd(gen);
  std::vector<float> hx32(hx.begin(), hx.end());
  DevBuf x, y32, yref;
  upload(x, hx32, s);
  y32.alloc(n * sizeof(float), s);
  plan->reduced_fft64 = false;
  execute_staged_t<float>(plan, x.as<float>(), y32.as<float>(), R, prec, s);
  std::vector<float> h32(n);
  std::vector<double> href(n);
  if (f64) {
    DevBuf x64;
    upload(x64, hx, s);
    yref.alloc(n * sizeof(double), s);
    execute_staged_t<double>(plan, x64.as<double>(), yref.as<double>(), R, SPT_F64, s);
    SPT_HIP(hipMemcpyAsync(href.data(), yref.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
  } else {
    yref.alloc(n * sizeof(float), s);
    plan->reduced_fft64 = true;
    execute_staged_t<float>(plan, x.as<float>(), yref.as<float>(), R, prec, s);
    std::vector<float> h(n);
    SPT_HIP(hipMemcpyAsync(h.data(), yref.p, n * sizeof(float), hipMemcpyDeviceToHost, s));
    SPT_HIP(hipStreamSynchronize(s));
    href.assign(h.begin(), h.end());
  }
  SPT_HIP(hipMemcpyAsync(h32.data(), y32.p, n * sizeof(float), hipMemcpyDeviceToHost, s));
  SPT_HIP(hipStreamSynchronize(s));
  // worst relative 2-norm error over the right-hand sides
  auto worst_err = [&] {
    double w = 0.0;
    for (int r = 0; r < R; ++r) {
      double num = 0.0, den = 0.0;
      for (int64_t j = 0; j < N; ++j) {
        const double a = h32[(size_t)r * N + j], b = href[(size_t)r * N + j];
        num += (a - b) * (a - b);
        den += b * b;
      }
      if (!(den > 0.0) || !std::isfinite(num))
        throw Error(SPT_E_NUMERIC, "non-finite or zero result while choosing the FFT arithmetic");
      w = std::max(w, std::sqrt(num / den));
    }
    return w;
  };
  double worst = worst_err();
  // the transposed product (float32 against float64) on the same inputs: its
  // inverse transforms take the same choice, and its error can exceed the
  // forward product's on long blocks
  bool tr = f32 && f64;
  for (auto& B : plan->blk)
    if (inv_four_step(plan, *B) && !B->four) tr = false;
  if (tr) {
    execute_transposed_t<float>(plan, x.as<float>(), y32.as<float>(), R, s);
    DevBuf x64;
    upload(x64, hx, s);
    execute_transposed_t<double>(plan, x64.as<double>(), yref.as<double>(), R, s);
    SPT_HIP(hipMemcpyAsync(href.data(), yref.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    SPT_HIP(hipMemcpyAsync(h32.data(), y32.p, n * sizeof(float), hipMemcpyDeviceToHost, s));
    SPT_HIP(hipStreamSynchronize(s));
    worst = std::max(worst, worst_err());
  }
  plan->reduced_fft32_err = worst;
  plan->reduced_fft64 = worst > (f64 ? REDUCED_TOTAL_BUDGET : REDUCED_FFT32_BUDGET);
}

// ---------------------------------------------------------------- execute
// bytes of an execute's workspace for R right-hand sides: complex float64
// spectra (and four-step intermediates; the transposed product also keeps its
// partial sums after them), or the three bfloat16-pair planes of the
// split-bf16 path
size_t work_bytes(spt_plan_t plan, int64_t R, bool transposed) {
  if (plan->cx)  // complex spectra (or transposed sums) of L + pad columns, float64
    return (size_t)std::max<int64_t>(R, 1) * (size_t)(plan->cx->L + plan->cx->pad) *
           sizeof(double2);
  const int64_t per = z_per_rhs(plan) + w_per_rhs(plan) + (transposed ? t_per_rhs(plan) : 0);
  return std::max((size_t)std::max<int64_t>(per, 1) * (size_t)R * sizeof(double2),
                  ((size_t)plan->zper4 * 3 * sizeof(uint32_t) +
                   (size_t)w_per_rhs(plan) * sizeof(float2)) * (size_t)R);
}

// select (and size) the workspace of stream s
void ensure_work(spt_plan_t plan, int64_t R, hipStream_t s, bool transposed = false) {
  spt_plan::Work* w = nullptr;
  for (auto& e : plan->works)
    if (e->stream == s) w = e.get();
  if (!w) {
    if (plan->works.size() >= 8) {
      // take over the oldest stream's workspace once the device is idle
      SPT_HIP(hipDeviceSynchronize());
      std::rotate(plan->works.begin(), plan->works.begin() + 1, plan->works.end());
      w = plan->works.back().get();
    } else {
      plan->works.push_back(std::make_unique<spt_plan::Work>());
      w = plan->works.back().get();
    }
    w->stream = s;
  }
  plan->work = &w->buf;
  const size_t bytes = work_bytes(plan, R, transposed);
  if (bytes > plan->work->bytes) {
    // work lists hold the old workspace address; work in flight may use them
    SPT_HIP(hipDeviceSynchronize());
    plan->ctx.clear();
    plan->work->alloc(bytes, s);
  }
}

void check_exec(spt_plan_t plan, const void* X, const void* Y, int64_t R, int prec) {
  check_plan(plan);
  if (!plan->precomputed) throw Error(SPT_E_NOT_PRECOMPUTED, "plan is not precomputed");
  if (!X || !Y) throw Error(SPT_E_INVALID_ARG, "X or Y is NULL");
  if (R < 1 || R > 65535 * 64) throw Error(SPT_E_INVALID_ARG, "nrhs out of range");
  if (prec < 0 || prec > 2) throw Error(SPT_E_INVALID_ARG, "unknown precision");
  if (!(plan->prepared & (1u << prec)))
    throw Error(SPT_E_UNSUPPORTED, "precision " + std::to_string(prec) + " was not prepared");
  const size_t es = (prec == SPT_F64 ? 8 : 4) * (is_complex_family(plan->family) ? 2 : 1);
  if (is_complex_family(plan->family) && prec == SPT_SPLIT_BF16)
    throw Error(SPT_E_UNSUPPORTED, "complex plans execute in F64 or F32");
  const char* x0 = static_cast<const char*>(X);
  const char* y0 = static_cast<const char*>(Y);
  const size_t n = (size_t)R * plan->N * es;
  if (x0 < y0 + n && y0 < x0 + n) throw Error(SPT_E_INVALID_ARG, "X and Y overlap");
}

ExecCtx& plan_ctx(spt_plan_t plan, int64_t R, int prec, hipStream_t s, bool staged);

// The staged FFT items of context c (two launches: single-workgroup transforms
// and column halves, then row halves), in the context's arithmetic: float64
// when c.fft64 (a split-bf16 context of float64 FFTs, or a float64 one).
template <typename T>
void fft_items_of(ExecCtx& c, const void* const* X, int count, bool split, hipStream_t s) {
  ExecArgs<T> a{};
  a.plans = c.plans.as<ExecPlan<T>>();
  a.ntw = c.ntw;
  for (int i = 0; i < count; ++i) a.X[i] = X[i];
  a.items = c.items.as<int4>();
  a.n_items = c.n_items;
  launch_fft_items<T>(a, split, c.xf, s);
  a.items = c.items2.as<int4>();
  a.n_items = c.n_items2;
  launch_fft_items<T>(a, split, c.xf, s);
}

void run_fft_items(ExecCtx& c, const void* const* X, int count, bool split, hipStream_t s) {
  if (c.fft64)
    fft_items_of<double>(c, X, count, split, s);
  else
    fft_items_of<float>(c, X, count, split, s);
}

// Staged execution in stream order.  FFTs: when every block's transform fits
// one workgroup (P <= 10240, the fused kernel's LDS bound in float64), one
// launch with a workgroup per (block, rhs); otherwise the FFT items, i.e. the
// single-workgroup transforms and the column halves of the four-step ones, in
// one launch and the row halves in a second.  Then the banded product.  The
// split-bf16 path writes and reads the pre-split spectra.
// ws: the workspace (work_bytes(plan, R, false) bytes) when the caller brings
// one; then only fused-FFT plans are accepted (the FFT items need work lists)
template <typename T>
void execute_staged_t(spt_plan_t plan, const T* X, T* Y, int64_t R, int prec, hipStream_t s,
                      void* ws) {
  using C = cplx_t<T>;
  const bool own_ws = ws == nullptr;
  if (own_ws) {
    ensure_work(plan, R, s);
    ws = plan->work->p;
  }
  const int nblk = (int)plan->blk.size();
  const bool split = std::is_same<T, float>::value && prec == SPT_SPLIT_BF16;
  const bool fused = nblk > 0 && plan->fwd_fused;
  const FftDesc<T>* d = std::is_same<T, double>::value ? (const FftDesc<T>*)plan->fftdesc64.p
                                                       : (const FftDesc<T>*)plan->fftdesc32.p;
  // fused FFT launch of blocks b0 .. b0 + nb - 1 on stream st
  auto fft_fused = [&](int b0, int nb, hipStream_t st) {
    int threads = 64;
    size_t lds = 16;
    if (nb > FFT_GRID_MAX)
      throw Error(SPT_E_UNSUPPORTED, "more than " + std::to_string(FFT_GRID_MAX) +
                                         " blocks in one fused FFT launch");
    FftGrid g{};
    g.nblk = nb;
    int64_t wgs = 0;
    for (int b = b0; b < b0 + nb; ++b) {
      const DevBlock& B = *plan->blk[b];
      threads = std::max(threads, B.fftw.threads);
      lds = std::max(lds, fused_lds_bytes<T>(B.fftw.P << B.lbw, 128 + B.P / 128 + 1));
      g.wg0[b - b0] = (int)wgs;
      wgs += B.half ? fft_split_wgs(B.half) * R : (R + (1 << B.lbw) - 1) >> B.lbw;
    }
    if (wgs > INT32_MAX) throw Error(SPT_E_UNSUPPORTED, "FFT grid too large");
    g.wg0[nb] = (int)wgs;
    if constexpr (std::is_same<T, float>::value) {
      if (plan->reduced_fft64) {
        size_t lds64 = 16;
        for (int b = b0; b < b0 + nb; ++b) {
          const DevBlock& B = *plan->blk[b];
          lds64 = std::max(lds64, fused_lds_bytes<double>(B.fftw.P << B.lbw, 128 + B.P / 128 + 1));
        }
        launch_exec_fft_multi_x32(plan->fftdesc64.as<FftDesc<double>>() + b0, g, threads, lds64,
                                  X, split ? nullptr : static_cast<float2*>(ws),
                                  split ? static_cast<uint32_t*>(ws) : nullptr,
                                  (int64_t)R * plan->zper4, (int)R, plan->N, st);
        return;
      }
      if (split) {
        launch_exec_fft_multi_split(d + b0, g, threads, lds, X, static_cast<uint32_t*>(ws),
                                    (int64_t)R * plan->zper4, (int)R, plan->N, st);
        return;
      }
    }
    launch_exec_fft_multi<T>(d + b0, g, threads, lds, X, static_cast<C*>(ws), (int)R, plan->N,
                             st);
  };
  // banded product of every block and the tail
  auto product = [&](hipStream_t st) {
    if constexpr (std::is_same<T, float>::value) {
      if (split) {
        SpmmSplitArgs pa{};
        pa.meta = plan->tilemeta_bf.as<TileMeta>();
        pa.blocks = plan->spmmblk_bf.as<SpmmSplitBlock>();
        pa.nblk = nblk;
        pa.n_tiles = plan->n_tiles;
        pa.Zs = static_cast<uint32_t*>(ws);
        pa.zplane = (int64_t)R * plan->zper4;
        pa.tail = (int)plan->tail;
        pa.tailmat = plan->tailbf.as<uint16_t>();
        pa.X = X;
        pa.Y = Y;
        pa.R = (int)R;
        pa.N = plan->N;
        // the windowed kernel forms byte offsets within the three spectrum
        // planes in 32 bits
        if (plan->win_ok && plan->win_chunked)
          launch_spmm_chunk(pa, plan->winmeta.as<WinMeta>(), plan->n_groups, plan->win_tpad, st);
        else if (plan->win_ok && 12.0 * (double)R * (double)plan->zper4 < 4294967296.0)
          launch_spmm_window(pa, plan->winmeta.as<WinMeta>(), plan->n_groups, plan->win_rg,
                             plan->win_waves, plan->win_xlds, plan->win_tpad, plan->win_lds,
                             st);
        else
          launch_spmm_presplit(pa, st);
        return;
      }
    }
    SpmmArgs<T> sa{};
    sa.nblk = nblk;
    sa.n_tiles = plan->n_tiles;
    sa.meta = plan->tilemeta.as<TileMeta>();
    sa.blocks = std::is_same<T, double>::value ? (const SpmmBlock<T>*)plan->spmmblk64.p
                                               : (const SpmmBlock<T>*)plan->spmmblk32.p;
    sa.Z = static_cast<C*>(ws);
    sa.tail = (int)plan->tail;
    sa.tailmat = std::is_same<T, double>::value ? (const T*)plan->tail64.p
                                                : (const T*)plan->tail32.p;
    sa.X = X;
    sa.Y = Y;
    sa.R = (int)R;
    sa.N = plan->N;
    if constexpr (std::is_same<T, double>::value) {
      // windows too wide for LDS: the chunked float64 product
      if (plan->win_ok && plan->win_chunked) {
        launch_spmm_chunk_f64(sa, plan->winmeta.as<WinMeta>(), plan->n_groups, st);
        return;
      }
    }
    launch_spmm<T>(sa, st);
  };

  if (fused) {
    // one launch per FFT_GRID_MAX blocks (a plan has more only for eps2 near 1)
    staged(SPT_STAGE_FFT, s, [&] {
      for (int b0 = 0; b0 < nblk; b0 += FFT_GRID_MAX)
        fft_fused(b0, std::min(FFT_GRID_MAX, nblk - b0), s);
    });
  } else if (nblk > 0) {
    if (!own_ws)
      throw Error(SPT_E_UNSUPPORTED, "a block's FFT exceeds one workgroup: the caller's workspace "
                                     "serves fused-FFT plans only");
    ExecCtx& c = plan_ctx(plan, R, prec, s, true);
    const void* xs[1] = {X};
    staged(SPT_STAGE_FFT, s, [&] { run_fft_items(c, xs, 1, split, s); });
  }
  staged(SPT_STAGE_SPMM, s, [&] { product(s); });
}

// Blocks of the transposed product whose inverse transform runs in four steps:
// those longer than one workgroup's FFT, and (spt_tuning.inv_four) every block
// with a four-step geometry.
bool inv_four_forced(spt_plan_t plan) { return plan->tune.inv_four == 2; }
bool inv_four_step(spt_plan_t plan, const DevBlock& B) {
  return B.big || (B.four && inv_four_forced(plan));
}

// log2 of the transforms of n points per workgroup of a four-step inverse
// pass (at most 64, at most `count`, about 4096 points per workgroup)
int inv_four_lb(int n, int count) {
  int lb = 0;
  while (lb < 6 && (n << (lb + 1)) <= 4096 && (2 << lb) <= count) ++lb;
  return lb;
}

template <typename T>
void execute_transposed_t(spt_plan_t plan, const T* F, T* Y, int64_t R, hipStream_t s) {
  using C = cplx_t<T>;
  for (auto& B : plan->blk)
    if (inv_four_step(plan, *B) && !B->four)
      throw Error(SPT_E_UNSUPPORTED, "block of FFT length half " + std::to_string(B->P) +
                                         " has no four-step split");
  ensure_work(plan, R, s, true);
  int64_t per = 0;
  for (auto& B : plan->blk) per += B->P + 1;
  // four-step intermediates after the half spectra (w_per_rhs); the float32
  // path's float64 intermediates (reduced_fft64) behind everything it uses,
  // 16-byte aligned: the workspace holds (z + w + t) R float64 complex values
  // and the float32 path uses half of that, and z > w
  C* wbuf = plan->work->as<C>() + per * R;
  C* u = plan->work->as<C>();
  const size_t used32 = (size_t)(z_per_rhs(plan) + w_per_rhs(plan) + t_per_rhs(plan)) * R *
                        sizeof(float2);
  double2* wbuf64 = reinterpret_cast<double2*>(static_cast<char*>(plan->work->p) +
                                               ((used32 + 15) & ~(size_t)15));
  SpmmTArgs<T> ta{};
  ta.segs = plan->tseg.as<int4>();
  ta.ents = plan->tent.as<TChunkEnt>();
  ta.blk = plan->tblk.as<TBlkInfo>();
  ta.u = u;
  ta.part = u + (z_per_rhs(plan) + w_per_rhs(plan)) * R;
  ta.red = plan->tred.as<int4>();
  ta.n_segs = plan->n_tseg;
  ta.n_red = plan->n_tred;
  ta.F = F;
  ta.R = (int)R;
  ta.N = plan->N;
  staged(SPT_STAGE_SPMM_T, s, [&] { launch_spmm_transposed<T>(ta, plan->reduced_fft64, s); });
  // the blocks that fit one workgroup in one launch (per block when four
  // steps are forced, a diagnostic)
  const bool multi = !inv_four_forced(plan);
  if (multi && plan->n_inv > 0)
    staged(SPT_STAGE_INV_FFT, s, [&] {
      if constexpr (std::is_same<T, float>::value) {
        if (plan->reduced_fft64) {
          launch_inv_fft_multi_x32(plan->invdesc64.as<InvFftDesc<double>>(), plan->n_inv,
                                   plan->inv_threads, sizeof(double2) * (size_t)plan->inv_maxP,
                                   u, Y, (int)R, plan->N, s);
          return;
        }
      }
      launch_inv_fft_multi<T>(
          std::is_same<T, double>::value ? (const InvFftDesc<T>*)plan->invdesc64.p
                                         : (const InvFftDesc<T>*)plan->invdesc32.p,
          plan->n_inv, plan->inv_threads, sizeof(C) * (size_t)plan->inv_maxP, u, Y, (int)R,
          plan->N, s);
    });
  for (auto& Bp : plan->blk) {
    DevBlock& B = *Bp;
    InvFftArgs<T> ia{};
    ia.U = u;
    ia.Y = Y;
    ia.winv = std::is_same<T, double>::value ? (const T*)B.winv64.p : (const T*)B.winv32.p;
    ia.tw = B.tw64.as<double2>();
    ia.post = std::is_same<T, double>::value ? (const C*)B.post64.p : (const C*)B.post32.p;
    ia.N = plan->N;
    ia.R = (int)R;
    ia.L = B.g.L;
    ia.P = B.P;
    ia.ldu = B.P + 1;
    ia.m_off = B.g.m_off;
    ia.c_lo = B.g.c_lo;
    ia.c_hi = B.g.c_hi;
    ia.scale = (T)(1.0 / std::sqrt((double)B.g.L));
    if (inv_four_step(plan, B)) {
      InvFft4Args<T> fa{};
      fa.U = u;
      fa.W = wbuf;
      fa.Y = Y;
      fa.winv = ia.winv;
      fa.tw = ia.tw;
      fa.post = ia.post;
      fa.N = ia.N;
      fa.R = ia.R;
      fa.P = B.P;
      fa.P1 = B.P1;
      fa.P2 = B.P2;
      fa.ldu = ia.ldu;
      fa.m_off = ia.m_off;
      fa.c_lo = ia.c_lo;
      fa.c_hi = ia.c_hi;
      fa.lb1 = inv_four_lb(B.P2, B.P1);
      fa.lb2 = inv_four_lb(B.P1, B.P2);
      fa.f1 = B.f1;
      fa.f2 = B.f2;
      fa.scale = ia.scale;
      bool done = false;
      if constexpr (std::is_same<T, float>::value) {
        if (plan->reduced_fft64) {
          // float64 arithmetic on float32 data (as the single-workgroup inverse
          // transforms): the intermediate in float64, in the second half of
          // the workspace, which is sized for float64 spectra
          InvFft4Args<double, float> fx{};
          fx.U = fa.U;
          fx.W = wbuf64;
          fx.Y = fa.Y;
          fx.winv = B.winv64.as<double>();
          fx.tw = fa.tw;
          fx.post = B.post64.as<double2>();
          fx.N = fa.N;
          fx.R = fa.R;
          fx.P = fa.P;
          fx.P1 = fa.P1;
          fx.P2 = fa.P2;
          fx.ldu = fa.ldu;
          fx.m_off = fa.m_off;
          fx.c_lo = fa.c_lo;
          fx.c_hi = fa.c_hi;
          fx.lb1 = fa.lb1;
          fx.lb2 = fa.lb2;
          fx.f1 = fa.f1;
          fx.f2 = fa.f2;
          fx.scale = 1.0 / std::sqrt((double)B.g.L);
          staged(SPT_STAGE_INV_FFT, s, [&] { launch_inv_fft4<double, float>(fx, s); });
          wbuf64 += (size_t)R * B.P;
          done = true;
        }
      }
      if (!done) staged(SPT_STAGE_INV_FFT, s, [&] { launch_inv_fft4<T>(fa, s); });
      wbuf += (size_t)R * B.P;
    } else if (!multi) {
      staged(SPT_STAGE_INV_FFT, s, [&] { launch_inv_fft<T>(ia, B.fft, s); });
    }
    u += (size_t)R * (B.P + 1);
  }
  if (plan->tail > 0)
    staged(SPT_STAGE_TAIL_T, s, [&] {
      launch_tail_transposed<T>(std::is_same<T, double>::value ? (const T*)plan->tail64.p
                                                               : (const T*)plan->tail32.p,
                                (int)plan->tail, F, Y, (int)R, plan->N, s);
    });
}

// ---------------------------------------------------------------- complex generators
template <typename F>
void staged(int stage, hipStream_t s, F&& fn);

// The compressed block of a complex plan: rows of A_e W by their closed forms
// and their transforms F on the device in panels, then on the host the
// threshold (eps1 times the block's maximum, Alg. 1 step 1.3), each row's kept
// entries as one circular arc of the spectrum (a row is one tone), and the
// tile boxes (union of their rows' arcs, unwrapped next to the first row's).
void precompute_complex(spt_plan_t plan, hipStream_t s) {
  if (plan->geom.size() != 1 || plan->tail != 0)
    throw Error(SPT_E_UNSUPPORTED, "complex plans take Algorithm 1's single block");
  auto cx = std::make_unique<CplxState>();
  const BlockGeom g = plan->geom[0];
  const int L = g.L;
  const int64_t N = plan->N;
  if (L > FUSED_MAX_P)
    throw Error(SPT_E_UNSUPPORTED, "complex plans need L <= " + std::to_string(FUSED_MAX_P) +
                                       " (one workgroup's transform); L = " + std::to_string(L));
  cx->L = L;
  cx->m_off = g.m_off;
  cx->c_lo = g.c_lo;
  cx->c_hi = g.c_hi;
  cx->fp = make_fft_plan(L);
  // window, its reciprocal, kappa
  std::vector<double> w(L), winv(L);
  double sw = 0.0, swi = 0.0;
  for (int c = 0; c < L; ++c) {
    w[c] = kaiser((double)c, (double)(L - 1), plan->zeta);
    winv[c] = 1.0 / w[c];
    sw += w[c] * w[c];
    if (c >= g.c_lo && c < g.c_hi) swi += winv[c] * winv[c];
  }
  cx->kappa = std::sqrt(sw / L) * std::sqrt(swi / (g.c_hi - g.c_lo));
  DevBuf dw;
  upload(dw, w, s);
  upload(cx->winv, winv, s);
  std::vector<long double> twr, twi, por, poi;
  twiddles(L, twr, twi, por, poi);
  upload(cx->tw, to_vec2<double2, double>(twr, twi), s);
  // row angles; for the Laguerre matrix C the phases phi_j and the factors
  // 1 / (eta/2 - i k_j), k_j = 2 pi j / T
  const long double pi = 3.141592653589793238462643383279502884L;
  cx->angles.resize(N);
  std::vector<double2> rowf;
  if (plan->family == SPT_CEXP) {
    for (int64_t j = 0; j < N; ++j)
      cx->angles[j] = (double)(pi * (long double)(2 * j + 1) / (long double)(2 * N));
  } else {
    const double eta = plan->p.eta, T = plan->p.period;
    rowf.resize(N);
    for (int64_t j = 0; j < N; ++j) {
      const double k = 2.0 * (double)pi * (double)j / T;
      cx->angles[j] = plan->user_nodes.empty() ? 2.0 * std::atan(2.0 * k / eta) - (double)pi
                                               : plan->user_nodes[j];
      const double a = 0.5 * eta, d = a * a + k * k;
      rowf[j] = double2{a / d, k / d};
    }
  }
  DevBuf dphi, drowf;
  if (!rowf.empty()) {
    upload(dphi, cx->angles, s);
    upload(drowf, rowf, s);
  }
  // spectra of all rows, panel by panel, to the host
  const int64_t panel = std::max<int64_t>(1, std::min<int64_t>(N, (int64_t)(256 << 20) / (16 * L)));
  DevBuf rows;
  rows.alloc((size_t)panel * L * sizeof(double2), s);
  std::vector<double2> S((size_t)N * L);
  for (int64_t r0 = 0; r0 < N; r0 += panel) {
    const int nr = (int)std::min<int64_t>(panel, N - r0);
    CplxRowsArgs ra{rows.as<double2>(), dw.as<double>(), dphi.as<double>(), drowf.as<double2>(),
                    N, r0, L, g.m_off, plan->family};
    launch_cplx_rows(ra, nr, s);
    launch_cplx_row_fft(rows.as<double2>(), nr, L, cx->fp, cx->tw.as<double2>(), s);
    SPT_HIP(hipMemcpyAsync(S.data() + (size_t)r0 * L, rows.p, (size_t)nr * L * sizeof(double2),
                           hipMemcpyDeviceToHost, s));
  }
  SPT_HIP(hipStreamSynchronize(s));
  double mx2 = 0.0;
  for (const double2& v : S) mx2 = std::max(mx2, v.x * v.x + v.y * v.y);
  if (!std::isfinite(mx2))
    throw Error(SPT_E_NUMERIC, "non-finite entries in the compressed complex block");
  cx->maxabs = std::sqrt(mx2);
  const double thr = plan->eps1 * cx->maxabs, thr2 = thr * thr;
  auto kept = [&](int64_t n, int k) {
    const double2 v = S[(size_t)n * L + k];
    return v.x * v.x + v.y * v.y > thr2;
  };
  // each row's kept entries: the arc that leaves out the longest circular run
  // of dropped columns; lo in [0, L), len columns (len 0: none kept)
  std::vector<int> lo(N, 0), len(N, 0);
  for (int64_t n = 0; n < N; ++n) {
    std::vector<int> ks;
    for (int k = 0; k < L; ++k)
      if (kept(n, k)) ks.push_back(k);
    if (ks.empty()) continue;
    int gap = -1, at = 0;
    for (size_t i = 0; i < ks.size(); ++i) {
      const int nxt = i + 1 < ks.size() ? ks[i + 1] : ks[0] + L;
      if (nxt - ks[i] > gap) {
        gap = nxt - ks[i];
        at = (int)((i + 1) % ks.size());
      }
    }
    lo[n] = ks[at];
    len[n] = L - gap + 1;
    cx->nnz += (int64_t)ks.size();
    cx->max_band = std::max(cx->max_band, len[n]);
  }
  // tile boxes
  const int nt = plan->n_tiles;
  std::vector<TileMeta> meta(nt);
  std::vector<int64_t> k0s(nt, 0), kws(nt, 0);
  int64_t off = 0;
  for (int t = 0; t < nt; ++t) {
    int64_t b0 = 0, b1 = -1;
    bool first = true;
    for (int q = 0; q < TILE_ROWS; ++q) {
      const int64_t n = (int64_t)t * TILE_ROWS + q;
      if (n >= N || len[n] == 0) continue;
      int64_t a0 = lo[n], a1 = lo[n] + len[n] - 1;
      if (first) {
        b0 = a0;
        b1 = a1;
        first = false;
        continue;
      }
      // unwrap next to the box so far (the rows of a tile are neighbouring tones)
      const int64_t mid = (b0 + b1) / 2;
      while (a0 - mid > L / 2) { a0 -= L; a1 -= L; }
      while (mid - a0 > L / 2) { a0 += L; a1 += L; }
      b0 = std::min(b0, a0);
      b1 = std::max(b1, a1);
    }
    if (first) continue;  // nothing kept in the tile
    int64_t kw = b1 - b0 + 1;
    if (kw >= L) {
      b0 = 0;
      kw = L;
    }
    b0 = ((b0 % L) + L) % L;
    k0s[t] = b0;
    kws[t] = kw;
    cx->pad = std::max<int>(cx->pad, (int)std::max<int64_t>(0, b0 + kw - L));
    meta[t] = TileMeta{(int)b0, (int)kw, off};
    off += kw * TILE_ROWS;
    cx->max_kw = std::max<int>(cx->max_kw, (int)kw);
  }
  cx->stored = off;
  std::vector<double2> v64((size_t)std::max<int64_t>(off, 1), double2{0.0, 0.0});
  for (int t = 0; t < nt; ++t)
    for (int64_t kk = 0; kk < kws[t]; ++kk)
      for (int q = 0; q < TILE_ROWS; ++q) {
        const int64_t n = (int64_t)t * TILE_ROWS + q;
        if (n >= N) continue;
        const int k = (int)((k0s[t] + kk) % L);
        if (kept(n, k)) v64[(size_t)(meta[t].off + kk * TILE_ROWS + q)] = S[(size_t)n * L + k];
      }
  S.clear();
  S.shrink_to_fit();
  upload(cx->meta, meta, s);
  if (plan->prepared & (1u << SPT_F64)) upload(cx->val64, v64, s);
  if (plan->prepared & (1u << SPT_F32)) {
    std::vector<float2> v32(v64.size());
    for (size_t i = 0; i < v64.size(); ++i) v32[i] = float2{(float)v64[i].x, (float)v64[i].y};
    upload(cx->val32, v32, s);
  }
  // the transposed product's lists: the tiles whose boxes meet each 32 columns
  // of 0 .. L + pad - 1
  const int ldu = L + cx->pad;
  cx->n_chunks = (ldu + 31) / 32;
  std::vector<int32_t> tptr(cx->n_chunks + 1, 0), tents;
  for (int c = 0; c < cx->n_chunks; ++c) {
    for (int t = 0; t < nt; ++t)
      if (kws[t] > 0 && k0s[t] < 32 * (c + 1) && k0s[t] + kws[t] > 32 * c) tents.push_back(t);
    tptr[c + 1] = (int32_t)tents.size();
    cx->max_list = std::max(cx->max_list, tptr[c + 1] - tptr[c]);
  }
  if (tents.empty()) tents.push_back(0);
  upload(cx->tptr, tptr, s);
  upload(cx->tents, tents, s);
  plan->cx = std::move(cx);
}

template <typename T>
void execute_complex(spt_plan_t plan, const void* X, void* Y, int64_t R, hipStream_t s) {
  using C = cplx_t<T>;
  const CplxState& cx = *plan->cx;
  ensure_work(plan, R, s);
  const int ldz = cx.L + cx.pad;
  CplxExecArgs<T> ea{static_cast<const C*>(X), plan->work->as<C>(), cx.winv.as<double>(),
                     cx.tw.as<double2>(), plan->N, cx.L, ldz, cx.m_off, cx.c_lo, cx.c_hi,
                     1.0 / std::sqrt((double)cx.L)};
  staged(SPT_STAGE_FFT, s, [&] { launch_cplx_exec_fft<T>(ea, cx.fp, (int)R, s); });
  CplxSpmmArgs<T> pa{cx.meta.as<TileMeta>(),
                     std::is_same<T, double>::value ? (const C*)cx.val64.p : (const C*)cx.val32.p,
                     plan->work->as<C>(), static_cast<C*>(Y), plan->N, (int)R, ldz};
  staged(SPT_STAGE_SPMM, s, [&] { launch_cplx_spmm<T>(pa, plan->n_tiles, cx.max_kw, s); });
}

template <typename T>
void execute_complex_transposed(spt_plan_t plan, const void* F, void* Y, int64_t R,
                                hipStream_t s) {
  using C = cplx_t<T>;
  const CplxState& cx = *plan->cx;
  ensure_work(plan, R, s, true);
  const int ldu = cx.L + cx.pad;
  CplxSpmmTArgs<T> ta{cx.meta.as<TileMeta>(),
                      std::is_same<T, double>::value ? (const C*)cx.val64.p : (const C*)cx.val32.p,
                      cx.tptr.as<int32_t>(), cx.tents.as<int32_t>(), static_cast<const C*>(F),
                      plan->work->as<C>(), plan->N, (int)R, ldu};
  staged(SPT_STAGE_SPMM_T, s, [&] { launch_cplx_spmm_t<T>(ta, cx.n_chunks, cx.max_list, s); });
  CplxInvArgs<T> ia{plan->work->as<C>(), static_cast<C*>(Y), cx.winv.as<double>(),
                    cx.tw.as<double2>(), plan->N, cx.L, ldu, cx.m_off, cx.c_lo, cx.c_hi,
                    1.0 / std::sqrt((double)cx.L)};
  staged(SPT_STAGE_INV_FFT, s, [&] { launch_cplx_inv_fft<T>(ia, cx.fp, (int)R, s); });
}

// ---------------------------------------------------------------- stage timing
struct Profiler {
  bool on = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    SPT_HIP(hipEventCreate(&e));
    return e;
  }
};
Profiler g_prof;

// set while a call must not create anything (spt_execute_noalloc): no
// profiling events then
thread_local bool t_noalloc = false;

// records an event pair around fn() on stream s when profiling is on
template <typename F>
void staged(int stage, hipStream_t s, F&& fn) {
  if (!g_prof.on || t_noalloc) {
    fn();
    return;
  }
  Profiler::Rec r{stage, g_prof.get(), g_prof.get()};
  SPT_HIP(hipEventRecord(r.a, s));
  fn();
  SPT_HIP(hipEventRecord(r.b, s));
  g_prof.recs.push_back(r);
}

// ---------------------------------------------------------------- persistent executor
bool uses_staged(spt_plan_t plan) { return plan->p.executor != SPT_EXECUTOR_PERSISTENT; }

// Report a dependency wait that gave up in the previous persistent launch on
// context c (its outputs hold NaN).  Waits for that launch: launches on one
// context run in stream order anyway, and the word is reused by the next one.
void check_exec_error(ExecCtx& c) {
  if (!c.pending) return;
  SPT_HIP(hipEventSynchronize(c.done));
  c.pending = false;
  if (__atomic_load_n(c.herr, __ATOMIC_ACQUIRE) != 0) {
    *c.herr = 0;
    throw Error(SPT_E_HIP,
                "persistent executor: a dependency wait of the previous launch on these plans "
                "and sizes gave up (its outputs hold NaN); this call did not run");
  }
}

template <typename T>
void run_exec(ExecCtx& c, const void* const* X, void* const* Y, int count, int prec,
              hipStream_t s) {
  check_exec_error(c);
  if (!c.herr) {
    SPT_HIP(hipHostMalloc((void**)&c.herr, sizeof(uint32_t),
                          hipHostMallocMapped | hipHostMallocCoherent));
    *c.herr = 0;
    SPT_HIP(hipHostGetDevicePointer((void**)&c.derr, c.herr, 0));
    SPT_HIP(hipEventCreateWithFlags(&c.done, hipEventDisableTiming));
  }
  ExecArgs<T> a{};
  a.plans = c.plans.as<ExecPlan<T>>();
  a.items = c.items.as<int4>();
  a.sync = c.sync.as<uint32_t>();
  a.err_out = c.derr;
  a.n_items = c.n_items;
  a.n_sync = c.n_sync;
  a.ntw = c.ntw;
  for (int i = 0; i < count; ++i) {
    a.X[i] = X[i];
    a.Y[i] = static_cast<T*>(Y[i]);
  }
  staged(SPT_STAGE_EXEC, s, [&] { launch_exec<T>(a, engine_of(prec), c.grid, s); });
  SPT_HIP(hipEventRecord(c.done, s));
  c.pending = true;
}


// Product arguments and items of a staged batch (items of a plan's chunk of 64
// right-hand sides start at a multiple of 8, tiles in XCD order).
template <typename T>
void build_batch_products(ExecCtx& c, const spt_plan_t* plans, const int64_t* R, int count,
                          int prec, hipStream_t s) {
  const bool dbl = std::is_same<T, double>::value;
  // split-bf16: plans with windows take the chunked product (groups of 4 row
  // tiles), the others the per-tile product; float64: plans whose windows are
  // too wide for LDS take the chunked float64 product (as a single execute
  // does), the others the per-tile one
  const bool chunked = prec == SPT_SPLIT_BF16 || prec == SPT_F64;
  auto windowed = [&](const spt_plan_t plan) {
    return prec == SPT_SPLIT_BF16 ? plan->win_ok
                                  : prec == SPT_F64 && plan->win_ok && plan->win_chunked;
  };
  std::vector<BatchProductPlan> bp(count);
  c.wlds = 0;
  for (int i = 0; i < count; ++i) {
    const spt_plan_t plan = plans[i];
    bp[i] = BatchProductPlan{windowed(plan) ? 1 : 0, plan->n_groups, plan->n_tiles, R[i]};
    if (prec == SPT_SPLIT_BF16 && plan->win_ok)
      c.wlds = std::max(c.wlds, spmm_chunk_lds_bytes(plan->win_tpad));
  }
  BatchProductLists bl;
  build_batch_product_lists(bp.data(), count, chunked, bl);
  std::string why;
  for (const BatchProductLaunch* l : {&bl.tile_launch, &bl.win_launch})
    if (!check_batch_product_launch(bp.data(), count, *l, &why))
      throw Error(SPT_E_UNSUPPORTED, "product work lists failed their check: " + why);
  auto upload_items = [&](DevBuf& b, const std::vector<WorkItem>& v) {
    std::vector<int4> o(std::max<size_t>(v.size(), 1), make_int4(0, -1, 0, 0));
    for (size_t k = 0; k < v.size(); ++k) o[k] = make_int4(v[k].x, v[k].y, v[k].z, v[k].w);
    upload(b, o, s);
  };
  upload_items(c.sitems, bl.tile_items);
  upload_items(c.witems, bl.win_items);
  // each launch reads its own list, as many items as the list holds
  c.n_sitems = bl.tile_launch.count;
  c.n_witems = bl.win_launch.count;
  if (prec == SPT_SPLIT_BF16) {
    std::vector<SpmmSplitArgs> a(count);
    for (int i = 0; i < count; ++i) {
      const spt_plan_t plan = plans[i];
      a[i].meta = plan->tilemeta_bf.as<TileMeta>();
      a[i].blocks = plan->spmmblk_bf.as<SpmmSplitBlock>();
      a[i].nblk = (int)plan->blk.size();
      a[i].n_tiles = plan->n_tiles;
      a[i].Zs = plan->work->as<uint32_t>();
      a[i].zplane = R[i] * plan->zper4;
      a[i].tail = (int)plan->tail;
      a[i].tailmat = plan->tailbf.as<uint16_t>();
      a[i].R = (int)R[i];
      a[i].N = plan->N;
      if (plan->win_ok) {
        a[i].win = plan->winmeta.as<WinMeta>();
        a[i].n_groups = plan->n_groups;
        a[i].tpad = plan->win_tpad;
      }
    }
    upload(c.sargs, a, s);
    return;
  }
  std::vector<SpmmArgs<T>> a(count);
  for (int i = 0; i < count; ++i) {
    const spt_plan_t plan = plans[i];
    a[i].meta = plan->tilemeta.as<TileMeta>();
    a[i].blocks = dbl ? (const SpmmBlock<T>*)plan->spmmblk64.p
                      : (const SpmmBlock<T>*)plan->spmmblk32.p;
    a[i].nblk = (int)plan->blk.size();
    a[i].n_tiles = plan->n_tiles;
    a[i].Z = plan->work->as<cplx_t<T>>();
    a[i].tail = (int)plan->tail;
    a[i].tailmat = dbl ? (const T*)plan->tail64.p : (const T*)plan->tail32.p;
    a[i].R = (int)R[i];
    a[i].N = plan->N;
    a[i].win = windowed(plan) ? plan->winmeta.as<WinMeta>() : nullptr;
  }
  upload(c.sargs, a, s);
}

// Staged batch: FFT items of every plan (two launches), then one product launch.
template <typename T>
void run_batch_staged(ExecCtx& c, const void* const* X, void* const* Y, int count, int prec,
                      hipStream_t s) {
  const bool split = std::is_same<T, float>::value && prec == SPT_SPLIT_BF16;
  staged(SPT_STAGE_FFT, s, [&] { run_fft_items(c, X, count, split, s); });
  staged(SPT_STAGE_SPMM, s, [&] {
    if (split) {
      SpmmSplitBatch b{};
      b.plans = c.sargs.as<SpmmSplitArgs>();
      for (int i = 0; i < count; ++i) {
        b.X[i] = static_cast<const float*>(X[i]);
        b.Y[i] = static_cast<float*>(Y[i]);
      }
      // each launch reads its own item list (n items each)
      b.items = c.witems.as<int4>();
      launch_spmm_chunk_items(b, c.n_witems, c.wlds, s);
      b.items = c.sitems.as<int4>();
      launch_spmm_presplit_items(b, c.n_sitems, s);
      return;
    }
    SpmmBatch<T> b{};
    b.plans = c.sargs.as<SpmmArgs<T>>();
    for (int i = 0; i < count; ++i) {
      b.X[i] = static_cast<const T*>(X[i]);
      b.Y[i] = static_cast<T*>(Y[i]);
    }
    // each launch reads its own item list (n items each)
    if constexpr (std::is_same<T, double>::value) {
      b.items = c.witems.as<int4>();
      launch_spmm_chunk_f64_items(b, c.n_witems, s);
    }
    b.items = c.sitems.as<int4>();
    launch_spmm_items<T>(b, c.n_sitems, s);
  });
}

// Staged transforms of the float32 paths in float64 arithmetic: when any plan
// of the set asks for them (a batch then runs all its plans' transforms that
// way).
bool wants_fft64(const spt_plan_t* plans, int count, int prec, bool staged) {
  if (prec == SPT_F64 || !staged) return false;
  for (int i = 0; i < count; ++i)
    if (plans[i]->reduced_fft64) return true;
  return false;
}

std::unique_ptr<ExecCtx> new_ctx(const std::vector<int64_t>& key, const spt_plan_t* plans,
                                 const int64_t* R, int count, int prec, hipStream_t s,
                                 bool staged = false, bool batch = false) {
  auto c = std::make_unique<ExecCtx>();
  c->key = key;
  c->fft64 = prec == SPT_F64 || wants_fft64(plans, count, prec, staged);
  c->xf = c->fft64 && prec != SPT_F64;
  if (c->fft64)
    build_exec_ctx<double>(*c, plans, R, count, prec, s, staged);
  else
    build_exec_ctx<float>(*c, plans, R, count, prec, s, staged);
  if (staged && batch) {
    if (prec == SPT_F64)
      build_batch_products<double>(*c, plans, R, count, prec, s);
    else
      build_batch_products<float>(*c, plans, R, count, prec, s);
  }
  return c;
}

ExecCtx& plan_ctx(spt_plan_t plan, int64_t R, int prec, hipStream_t s, bool staged) {
  const std::vector<int64_t> key{prec, R, plan->serial, (int64_t)(intptr_t)plan->work->p, staged,
                                 plan->reduced_fft64};
  for (auto& c : plan->ctx)
    if (c->key == key) return *c;
  if (plan->ctx.size() >= 8) {
    SPT_HIP(hipDeviceSynchronize());  // the oldest work list may be in flight
    plan->ctx.erase(plan->ctx.begin());
  }
  plan->ctx.push_back(new_ctx(key, &plan, &R, 1, prec, s, staged));
  return *plan->ctx.back();
}

// contexts of batched launches (a few recent sets of plans)
std::mutex g_batch_mu;
std::vector<std::unique_ptr<ExecCtx>> g_batch_ctx;

// new bound of the persistent executor's dependency waits of this plan: its
// own contexts and the batch contexts that it leads (plans[0] of the batch)
void set_exec_wait(spt_plan_t plan, uint32_t ticks) {
  plan->exec_wait = ticks;
  std::vector<ExecCtx*> cs;
  for (auto& c : plan->ctx) cs.push_back(c.get());
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto& c : g_batch_ctx)
      if (c->key.size() > 3 && c->key[3] == plan->serial) cs.push_back(c.get());
  }
  if (cs.empty()) return;
  set_device(plan);
  SPT_HIP(hipDeviceSynchronize());  // launches in flight read the old bound
  for (ExecCtx* c : cs)
    SPT_HIP(hipMemcpy(c->sync.as<uint32_t>() + EXEC_SYNC_WAIT, &ticks, sizeof(ticks),
                      hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------- launch choices
void check_tuning(const spt_tuning& t) {
  if (t.product < SPT_PRODUCT_DEFAULT || t.product > SPT_PRODUCT_WINDOW_2W)
    throw Error(SPT_E_INVALID_ARG, "unknown product choice");
  if (t.window_rhs != 0 && t.window_rhs != 32 && t.window_rhs != 64)
    throw Error(SPT_E_INVALID_ARG, "window_rhs must be 0, 32 or 64");
  if (t.fft_batch != 0 && t.fft_batch != 1 && t.fft_batch != 2 && t.fft_batch != 4)
    throw Error(SPT_E_INVALID_ARG, "fft_batch must be 0, 1, 2 or 4");
  if (t.inv_four < SPT_TUNE_DEFAULT || t.inv_four > SPT_TUNE_ON)
    throw Error(SPT_E_INVALID_ARG, "unknown on/off choice");
  if (t.fft_half < SPT_TUNE_DEFAULT || t.fft_half > SPT_FFT_EIGHT)
    throw Error(SPT_E_INVALID_ARG, "unknown FFT split choice");
}

// the batch contexts that refer to a plan's buffers (keyed by its serial)
void drop_batch_contexts(spt_plan_t plan) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  auto uses = [&](const std::unique_ptr<ExecCtx>& c) {
    for (size_t i = 3; i < c->key.size(); i += 3)  // key: prec, n, staged, (serial, R, work)...
      if (c->key[i] == plan->serial) return true;
    return false;
  };
  g_batch_ctx.erase(std::remove_if(g_batch_ctx.begin(), g_batch_ctx.end(), uses),
                    g_batch_ctx.end());
}

// Rebuild what the launch choices shape on a precomputed plan: each block's
// parity split, the fused FFT descriptors (batching), the windows.
void apply_tuning(spt_plan_t plan, hipStream_t s) {
  if (!plan->precomputed || plan->cx) return;
  SPT_HIP(hipDeviceSynchronize());  // launches in flight read the old descriptions
  plan->ctx.clear();
  drop_batch_contexts(plan);
  const size_t lds_max = max_lds_bytes(plan->device);
  for (auto& Bp : plan->blk) {
    DevBlock& B = *Bp;
    if (!B.fwd) continue;
    const int P = B.P;
    const int split = fused_split(plan, P, lds_max);
    if (fused_lds_bytes<double>(fused_points(P, split), 128 + P / 128 + 1) > lds_max)
      throw Error(SPT_E_UNSUPPORTED, "FFT split does not fit one workgroup");
    B.half = split;
    B.fftw = make_fft_plan(fused_points(P, split), true);
  }
  build_fft_descs(plan, s);
  plan->serial = next_serial();  // keys of the executor contexts
}

// seconds of `reps` executes after `warm` ones, HIP events on s (median of reps)
template <typename T>
double time_executes(spt_plan_t plan, const T* X, T* Y, int64_t R, int prec, hipStream_t s,
                     int warm, int reps) {
  for (int i = 0; i < warm; ++i) execute_staged_t<T>(plan, X, Y, R, prec, s);
  std::vector<hipEvent_t> ev(reps + 1);
  for (auto& e : ev) SPT_HIP(hipEventCreate(&e));
  SPT_HIP(hipEventRecord(ev[0], s));
  for (int i = 0; i < reps; ++i) {
    execute_staged_t<T>(plan, X, Y, R, prec, s);
    SPT_HIP(hipEventRecord(ev[i + 1], s));
  }
  SPT_HIP(hipEventSynchronize(ev[reps]));
  std::vector<float> ms(reps);
  for (int i = 0; i < reps; ++i) SPT_HIP(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
  for (auto& e : ev) (void)hipEventDestroy(e);
  std::sort(ms.begin(), ms.end());
  return 1e-3 * ms[reps / 2];
}

std::string tuning_key(spt_plan_t plan, int64_t R, int prec) {
  int ln = 0, lr = 0;
  while (((int64_t)1 << ln) < plan->N) ++ln;
  while (((int64_t)1 << lr) < R) ++lr;
  char buf[160];
  std::snprintf(buf, sizeof(buf), "family=%d alpha=%.17g beta=%.17g log2N=%d log2R=%d prec=%d",
                plan->family, plan->p.alpha, plan->p.beta, ln, lr, prec);
  return buf;
}

// The autotuner's cache: one line per key, "key": {fields}, inside { }.
bool cache_lookup(const char* path, const std::string& key, spt_tuning& t) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  const size_t at = text.find("\"" + key + "\"");
  if (at == std::string::npos) return false;
  const size_t b = text.find('{', at), e = text.find('}', at);
  if (b == std::string::npos || e == std::string::npos || e < b) return false;
  const std::string body = text.substr(b, e - b);
  auto field = [&](const char* name, int32_t& out) {
    const size_t p = body.find(std::string("\"") + name + "\":");
    if (p == std::string::npos) return false;
    out = (int32_t)std::strtol(body.c_str() + p + std::strlen(name) + 3, nullptr, 10);
    return true;
  };
  spt_tuning c{};
  if (!field("product", c.product) || !field("window_rhs", c.window_rhs) ||
      !field("fft_batch", c.fft_batch) || !field("fft_half", c.fft_half) ||
      !field("inv_four", c.inv_four))
    return false;
  check_tuning(c);
  t = c;
  return true;
}

void cache_store(const char* path, const std::string& key, const spt_tuning& t, double us) {
  if (!path) return;
  std::vector<std::string> lines;
  if (FILE* f = std::fopen(path, "r")) {
    char buf[1024];
    while (std::fgets(buf, sizeof(buf), f)) {
      std::string l(buf);
      while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
      if (l.size() > 2 && l[0] == ' ' && l.find("\"" + key + "\"") == std::string::npos)
        lines.push_back(l);
    }
    std::fclose(f);
  }
  char rec[512];
  std::snprintf(rec, sizeof(rec),
                "  \"%s\": {\"product\": %d, \"window_rhs\": %d, \"fft_batch\": %d, "
                "\"fft_half\": %d, \"inv_four\": %d, \"us\": %.3f}",
                key.c_str(), t.product, t.window_rhs, t.fft_batch, t.fft_half, t.inv_four, us);
  lines.push_back(rec);
  FILE* f = std::fopen(path, "w");
  if (!f) throw Error(SPT_E_INVALID_ARG, std::string("cannot write the tuning cache ") + path);
  std::fputs("{\n", f);
  for (size_t i = 0; i < lines.size(); ++i)
    std::fprintf(f, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
  std::fputs("}\n", f);
  std::fclose(f);
}

template <typename T>
void autotune_t(spt_plan_t plan, int64_t R, int prec, hipStream_t s, spt_tuning& best,
                double& best_s) {
  const int64_t N = plan->N;
  std::vector<double> hx((size_t)R * N);
  std::mt19937_64 gen(0x70e5eed);
  std::normal_distribution<double> nd;
  for (double& v : hx) v = nd(gen);
  std::vector<T> h(hx.begin(), hx.end());
  DevBuf x, y;
  upload(x, h, s);
  y.alloc(h.size() * sizeof(T), s);
  const bool split = prec == SPT_SPLIT_BF16;
  const size_t lds_max = max_lds_bytes(plan->device);
  // the FFT splits worth timing: parity (the default), none where a whole
  // transform fits one workgroup, eight-way where 4 divides P
  bool can_split = false, can_off = false, can_eight = false;
  for (auto& B : plan->blk)
    if (B->fwd && B->P >= FUSED_HALF_MIN_P && B->P % 2 == 0) {
      can_split = true;
      can_off |= fused_lds_bytes<double>(B->P, 128 + B->P / 128 + 1) <= lds_max;
      can_eight |= B->P % 4 == 0;
    }
  std::vector<int> halves{SPT_TUNE_DEFAULT};
  if (can_split) {
    halves = {SPT_TUNE_ON};
    if (can_off) halves.push_back(SPT_TUNE_OFF);
    if (can_eight) halves.push_back(SPT_FFT_EIGHT);
  }
  std::vector<spt_tuning> cand;
  const std::vector<int> prods = split ? std::vector<int>{SPT_PRODUCT_TILE, SPT_PRODUCT_WINDOW,
                                                          SPT_PRODUCT_CHUNKED,
                                                          SPT_PRODUCT_WINDOW_2W}
                                       : std::vector<int>{SPT_PRODUCT_DEFAULT};
  for (int pr : prods)
    for (int rhs : (pr == SPT_PRODUCT_WINDOW ? std::vector<int>{32, 64} : std::vector<int>{0}))
      for (int fb : {1, 2, 4})
        for (int hf : halves) cand.push_back(spt_tuning{pr, rhs, fb, hf, plan->tune.inv_four});
  // two sweeps, so that a choice timed during a slow moment gets a second
  // chance: the smaller of its two medians counts
  std::vector<double> tc(cand.size(), 1e30);
  for (int sweep = 0; sweep < 2; ++sweep)
    for (size_t i = 0; i < cand.size(); ++i) {
      plan->tune = cand[i];
      apply_tuning(plan, s);
      tc[i] = std::min(tc[i], time_executes<T>(plan, x.as<T>(), y.as<T>(), R, prec, s, 3, 20));
    }
  best_s = 1e30;
  for (size_t i = 0; i < cand.size(); ++i)
    if (tc[i] < best_s) {
      best_s = tc[i];
      best = cand[i];
    }
  plan->tune = best;
  apply_tuning(plan, s);
  SPT_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------- no-allocation execute
// The workspace of spt_execute_noalloc: one static array per device, resident
// from the library's load until the process ends.  Host code uses the address
// that hipGetSymbolAddress gives on each device, never the array's name.
static __device__ __align__(256) unsigned char scratch[SPT_NOALLOC_MAX_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// the array's address on the current device (looked up once per device)
void* scratch_on(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES)
    throw Error(SPT_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      throw Error(SPT_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                 hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

template <typename F>
spt_status guard(F&& fn) {
  try {
    fn();
    g_last_error.clear();
    return SPT_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return SPT_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return SPT_E_HIP;
  }
}

}  // namespace
}  // namespace spt

using namespace spt;

extern "C" {

const char* spt_last_error(void) { return g_last_error.c_str(); }

const char* spt_version(void) { return "spt 0.1 (gfx950)"; }

spt_status spt_plan_create(spt_plan_t* out, int32_t family, const spt_params* p, int64_t N,
                           double eps) {
  return guard([&] {
    if (!out) throw Error(SPT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (family < SPT_CHEBYSHEV_T || family > SPT_LAGUERRE_SPECTRAL)
      throw Error(SPT_E_INVALID_ARG, "unknown family " + std::to_string(family));
    if (N < 2 || N > (int64_t)1 << 24) throw Error(SPT_E_INVALID_ARG, "N out of range");
    spt_params prm{};
    if (p) prm = *p;
    const double eps2 = prm.eps2 == 0.0 ? 1e-2 : prm.eps2;
    if (!(eps > 0.0 && eps < 1.0)) throw Error(SPT_E_INVALID_ARG, "eps must lie in (0, 1)");
    if (!(eps2 > eps && eps2 < 1.0)) throw Error(SPT_E_INVALID_ARG, "need eps < eps2 < 1");
    if (family == SPT_JACOBI && !(prm.alpha > -1.0 && prm.beta > -1.0))
      throw Error(SPT_E_INVALID_ARG, "Jacobi needs alpha, beta > -1");
    if (family == SPT_LEGENDRE) prm.alpha = prm.beta = 0.0;
    if (family == SPT_COS_POWER && (prm.power < 2 || prm.power > 5))
      throw Error(SPT_E_INVALID_ARG, "cos power s must be 2, 3, 4 or 5");
    if (prm.trig_conv_q < 0 || prm.trig_conv_q > 64)
      throw Error(SPT_E_INVALID_ARG, "trig_conv_q must lie in 0..64");
    if (prm.trig_conv_q > 0 && !is_trig(family))
      throw Error(SPT_E_INVALID_ARG, "Appendix A covers the trigonometric generators only");
    if (prm.mode != SPT_MODE_AUTO && prm.mode != SPT_MODE_ROW && prm.mode != SPT_MODE_DIRECT)
      throw Error(SPT_E_INVALID_ARG, "unknown mode");
    if (prm.precisions & ~7u) throw Error(SPT_E_INVALID_ARG, "unknown precision bits");
    if (prm.executor < SPT_EXECUTOR_AUTO || prm.executor > SPT_EXECUTOR_PERSISTENT)
      throw Error(SPT_E_INVALID_ARG, "unknown executor");
    if (prm.min_block < 0 || prm.panel_rows < 0) throw Error(SPT_E_INVALID_ARG, "negative size");
    if (family == SPT_LAGUERRE_SPECTRAL && !(prm.eta > 0.0 && prm.period > 0.0))
      throw Error(SPT_E_INVALID_ARG, "the Laguerre spectral matrix needs eta > 0 and period > 0");
    if (is_complex_family(family) && prm.mode == SPT_MODE_DIRECT)
      throw Error(SPT_E_UNSUPPORTED, "complex plans run the compressed method only");
    if (is_complex_family(family) && (prm.precisions & (1u << SPT_SPLIT_BF16)))
      throw Error(SPT_E_UNSUPPORTED, "complex plans execute in F64 or F32");
    if (family == SPT_CEXP && prm.nodes)
      throw Error(SPT_E_INVALID_ARG, "the exp(i m theta) generator takes the Chebyshev-Gauss angles");
    if (prm.reduced_fft < 0 || prm.reduced_fft > 2)
      throw Error(SPT_E_INVALID_ARG, "reduced_fft must be 0 (automatic), 1 or 2");
    auto plan = std::make_unique<spt_plan>();
    plan->family = family;
    plan->N = N;
    plan->eps1 = eps;
    plan->eps2 = eps2;
    plan->requested_mode = prm.mode;
    if (prm.nodes) {
      plan->user_nodes.assign(prm.nodes, prm.nodes + N);
      for (double v : plan->user_nodes)
        if (!std::isfinite(v)) throw Error(SPT_E_INVALID_ARG, "non-finite node");
    }
    prm.nodes = nullptr;
    plan->p = prm;
    plan->zeta = zeta_of_eps(eps);
    const int64_t min_block = prm.min_block > 0 ? prm.min_block : 32;
    const bool round_fft = prm.exact_fft_len == 0;
    if (prm.mode == SPT_MODE_DIRECT) {
      plan->geom.clear();
      plan->tail = N;
    } else if (is_trig(family) || is_complex_family(family)) {
      partition_two_sided(N, plan->zeta, eps2, round_fft, plan->geom, plan->tail);
    } else {
      partition_one_sided(N, plan->zeta, eps2, min_block, round_fft, plan->geom, plan->tail);
    }
    if ((int)plan->geom.size() > MAX_BLOCKS) throw Error(SPT_E_UNSUPPORTED, "too many blocks");
    plan->mode = prm.mode == SPT_MODE_DIRECT ? SPT_MODE_DIRECT : SPT_MODE_ROW;
    // plan creation is host-only; the device is the current one (0 when HIP
    // reports none, in which case the first device call fails with SPT_E_HIP)
    if (hipGetDevice(&plan->device) != hipSuccess) {
      (void)hipGetLastError();
      plan->device = 0;
    }
    *out = plan.release();
  });
}

spt_status spt_plan_blocks(spt_plan_t plan, int32_t* L, int32_t* m_offset, int32_t* c_lo,
                           int32_t* c_hi, int32_t cap, int32_t* n_blocks) {
  return guard([&] {
    check_plan(plan);
    const bool built = plan->precomputed && !plan->cx;  // complex plans keep geom
    const int n = built ? (int)plan->blk.size() : (int)plan->geom.size();
    if (n_blocks) *n_blocks = n;
    for (int i = 0; i < n && i < cap; ++i) {
      const BlockGeom& g = built ? plan->blk[i]->g : plan->geom[i];
      if (L) L[i] = g.L;
      if (m_offset) m_offset[i] = g.m_off;
      if (c_lo) c_lo[i] = g.c_lo;
      if (c_hi) c_hi[i] = g.c_hi;
    }
  });
}

spt_status spt_precompute(spt_plan_t plan, void* stream) {
  return guard([&] {
    check_plan(plan);
    try {
      precompute(plan, static_cast<hipStream_t>(stream));
    } catch (...) {
      plan->precomputed = false;
      plan->blk.clear();
      plan->cx.reset();
      throw;
    }
  });
}

spt_status spt_execute(spt_plan_t plan, const void* X, void* Y, int64_t nrhs, int32_t prec,
                       void* stream) {
  return guard([&] {
    check_exec(plan, X, Y, nrhs, prec);
    set_device(plan);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (plan->cx) {
      if (prec == SPT_F64)
        execute_complex<double>(plan, X, Y, nrhs, s);
      else
        execute_complex<float>(plan, X, Y, nrhs, s);
      return;
    }
    if (uses_staged(plan)) {
      if (prec == SPT_F64)
        execute_staged_t<double>(plan, (const double*)X, (double*)Y, nrhs, prec, s);
      else
        execute_staged_t<float>(plan, (const float*)X, (float*)Y, nrhs, prec, s);
      return;
    }
    ensure_work(plan, nrhs, s);
    ExecCtx& c = plan_ctx(plan, nrhs, prec, s, false);
    const void* xs[1] = {X};
    void* ys[1] = {Y};
    if (prec == SPT_F64)
      run_exec<double>(c, xs, ys, 1, prec, s);
    else
      run_exec<float>(c, xs, ys, 1, prec, s);
  });
}

spt_status spt_execute_noalloc(spt_plan_t plan, const void* X, void* Y, int64_t nrhs,
                               int32_t prec, void* stream) {
  return guard([&] {
    check_exec(plan, X, Y, nrhs, prec);
    if (!uses_staged(plan) || plan->cx)
      throw Error(SPT_E_UNSUPPORTED,
                  "spt_execute_noalloc runs the staged executor of real plans only");
    if (!plan->blk.empty() && !plan->fwd_fused)
      throw Error(SPT_E_UNSUPPORTED, "a block's FFT exceeds one workgroup (it needs work lists)");
    const size_t need = work_bytes(plan, nrhs, false);
    if (need > (size_t)SPT_NOALLOC_MAX_BYTES)
      throw Error(SPT_E_INVALID_ARG, "the workspace of " + std::to_string(nrhs) +
                                         " right-hand sides (" + std::to_string(need) +
                                         " bytes) exceeds SPT_NOALLOC_MAX_BYTES (" +
                                         std::to_string((size_t)SPT_NOALLOC_MAX_BYTES) + ")");
    set_device(plan);
    void* ws = scratch_on(plan->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    t_noalloc = true;
    try {
      if (prec == SPT_F64)
        execute_staged_t<double>(plan, (const double*)X, (double*)Y, nrhs, prec, s, ws);
      else
        execute_staged_t<float>(plan, (const float*)X, (float*)Y, nrhs, prec, s, ws);
    } catch (...) {
      t_noalloc = false;
      throw;
    }
    t_noalloc = false;
  });
}

spt_status spt_execute_transposed(spt_plan_t plan, const void* X, void* Y, int64_t nrhs,
                                  int32_t prec, void* stream) {
  return guard([&] {
    check_exec(plan, X, Y, nrhs, prec);
    if (prec == SPT_SPLIT_BF16)
      throw Error(SPT_E_UNSUPPORTED, "the transposed product runs in F64 or F32");
    set_device(plan);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (plan->cx) {
      if (prec == SPT_F64)
        execute_complex_transposed<double>(plan, X, Y, nrhs, s);
      else
        execute_complex_transposed<float>(plan, X, Y, nrhs, s);
      return;
    }
    if (prec == SPT_F64)
      execute_transposed_t<double>(plan, (const double*)X, (double*)Y, nrhs, s);
    else
      execute_transposed_t<float>(plan, (const float*)X, (float*)Y, nrhs, s);
  });
}

spt_status spt_execute_batched(const spt_plan_t* plans, const void* const* X, void* const* Y,
                               const int64_t* nrhs, int32_t count, int32_t prec, void* stream) {
  return guard([&] {
    if (count < 0 || (count > 0 && (!plans || !X || !Y || !nrhs)))
      throw Error(SPT_E_INVALID_ARG, "bad batch arrays");
    if (count == 0) return;
    for (int i = 0; i < count; ++i) {
      check_exec(plans[i], X[i], Y[i], nrhs[i], prec);
      if (plans[i]->device != plans[0]->device)
        throw Error(SPT_E_INVALID_ARG, "batched plans live on different devices");
      for (int j = 0; j < i; ++j)
        if (plans[j] == plans[i])
          throw Error(SPT_E_INVALID_ARG, "a plan appears twice in one batch");
      if (plans[i]->cx) throw Error(SPT_E_UNSUPPORTED, "complex plans do not run in batches");
    }
    set_device(plans[0]);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (count == 1 && uses_staged(plans[0])) {
      // one plan: its own staged launches (fused FFT, windowed or chunked
      // product in every precision), as spt_execute
      if (prec == SPT_F64)
        execute_staged_t<double>(plans[0], (const double*)X[0], (double*)Y[0], nrhs[0], prec, s);
      else
        execute_staged_t<float>(plans[0], (const float*)X[0], (float*)Y[0], nrhs[0], prec, s);
      return;
    }
    for (int i = 0; i < count; ++i) ensure_work(plans[i], nrhs[i], s);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    // persistent when the first plan asks for it, staged launches otherwise
    const bool staged = plans[0]->p.executor != SPT_EXECUTOR_PERSISTENT;
    for (int i0 = 0; i0 < count; i0 += EXEC_MAX_PLANS) {
      const int n = std::min(count - i0, EXEC_MAX_PLANS);
      std::vector<int64_t> key{prec, n, staged};
      for (int i = i0; i < i0 + n; ++i) {
        key.push_back(plans[i]->serial);
        key.push_back(nrhs[i]);
        key.push_back((int64_t)(intptr_t)plans[i]->work->p);
      }
      ExecCtx* c = nullptr;
      for (auto& e : g_batch_ctx)
        if (e->key == key) c = e.get();
      if (!c) {
        if (g_batch_ctx.size() >= 4) {
          SPT_HIP(hipDeviceSynchronize());  // the oldest work list may be in flight
          g_batch_ctx.erase(g_batch_ctx.begin());
        }
        g_batch_ctx.push_back(new_ctx(key, plans + i0, nrhs + i0, n, prec, s, staged, true));
        c = g_batch_ctx.back().get();
      }
      if (staged) {
        if (prec == SPT_F64)
          run_batch_staged<double>(*c, X + i0, Y + i0, n, prec, s);
        else
          run_batch_staged<float>(*c, X + i0, Y + i0, n, prec, s);
      } else if (prec == SPT_F64) {
        run_exec<double>(*c, X + i0, Y + i0, n, prec, s);
      } else {
        run_exec<float>(*c, X + i0, Y + i0, n, prec, s);
      }
    }
  });
}

spt_status spt_set_allocator(spt_alloc_fn alloc, spt_free_fn free_, void* ctx) {
  return guard([&] {
    if ((alloc == nullptr) != (free_ == nullptr))
      throw Error(SPT_E_INVALID_ARG, "give both hooks or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free = free_;
    g_alloc.ctx = alloc ? ctx : nullptr;
  });
}

spt_status spt_plan_set_tuning(spt_plan_t plan, const spt_tuning* t) {
  return guard([&] {
    check_plan(plan);
    if (!t) throw Error(SPT_E_INVALID_ARG, "t is NULL");
    check_tuning(*t);
    plan->tune = *t;
    if (plan->precomputed) {
      set_device(plan);
      apply_tuning(plan, nullptr);
    }
  });
}

spt_status spt_plan_get_tuning(spt_plan_t plan, spt_tuning* t) {
  return guard([&] {
    check_plan(plan);
    if (!t) throw Error(SPT_E_INVALID_ARG, "t is NULL");
    *t = plan->tune;
  });
}

spt_status spt_autotune(spt_plan_t plan, int64_t nrhs, int32_t prec, void* stream,
                        const char* cache_path, spt_tuning* chosen, double* us) {
  return guard([&] {
    check_plan(plan);
    if (!plan->precomputed) throw Error(SPT_E_NOT_PRECOMPUTED, "plan is not precomputed");
    if (nrhs < 1 || nrhs > 65535 * 64) throw Error(SPT_E_INVALID_ARG, "nrhs out of range");
    if (prec < 0 || prec > 2) throw Error(SPT_E_INVALID_ARG, "unknown precision");
    if (!(plan->prepared & (1u << prec)))
      throw Error(SPT_E_UNSUPPORTED, "precision " + std::to_string(prec) + " was not prepared");
    if (us) *us = 0.0;
    if (plan->cx || !uses_staged(plan)) {
      if (chosen) *chosen = plan->tune;
      return;
    }
    set_device(plan);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::string key = tuning_key(plan, nrhs, prec);
    spt_tuning t{};
    if (cache_lookup(cache_path, key, t)) {
      plan->tune = t;
      apply_tuning(plan, s);
    } else {
      double best = 0.0;
      if (prec == SPT_F64)
        autotune_t<double>(plan, nrhs, prec, s, t, best);
      else
        autotune_t<float>(plan, nrhs, prec, s, t, best);
      cache_store(cache_path, key, t, 1e6 * best);
      if (us) *us = 1e6 * best;
    }
    if (chosen) *chosen = plan->tune;
  });
}

spt_status spt_plan_set_exec_wait(spt_plan_t plan, int64_t ticks) {
  return guard([&] {
    check_plan(plan);
    if (ticks < 0 || ticks > 0xffffffffll) throw Error(SPT_E_INVALID_ARG, "ticks out of range");
    set_exec_wait(plan, ticks == 0 ? EXEC_WAIT_DEFAULT : (uint32_t)ticks);
  });
}

spt_status spt_plan_query(spt_plan_t plan, spt_plan_info* info) {
  return guard([&] {
    check_plan(plan);
    if (!info) throw Error(SPT_E_INVALID_ARG, "info is NULL");
    std::memset(info, 0, sizeof(*info));
    info->family = plan->family;
    info->mode = plan->mode;
    info->N = plan->N;
    info->eps1 = plan->eps1;
    info->eps2 = plan->eps2;
    info->zeta = plan->zeta;
    info->tail = (int32_t)plan->tail;
    info->precomputed = plan->precomputed;
    info->is_complex = is_complex_family(plan->family) ? 1 : 0;
    info->n_blocks = plan->precomputed && !plan->cx ? (int)plan->blk.size()
                                                    : (int)plan->geom.size();
    if (plan->precomputed) {
      int64_t ldt = (int64_t)plan->n_tiles * TILE_ROWS;
      int64_t tiles_bytes = 0;
      for (size_t i = 0; i < plan->blk.size(); ++i) {
        const DevBlock& B = *plan->blk[i];
        info->nnz += B.nnz;
        info->stored += B.stored;
        info->max_band = std::max(info->max_band, B.max_band);
        tiles_bytes += (int64_t)plan->n_tiles * 16;
        if (i < 16) info->max_abs[i] = B.maxabs;
        if (i < 16) info->nnz_blk[i] = B.nnz;
        info->kappa = std::max(info->kappa, B.kappa);
      }
      info->matrix_bytes_f64 = info->stored * 16 + tiles_bytes + plan->tail * ldt * 8;
      info->matrix_bytes_f32 = info->stored * 8 + tiles_bytes + plan->tail * ldt * 4;
      if (plan->win_ok) {
        info->window_lds = (int64_t)plan->win_lds;
        info->window_cols = plan->win_cols;
        info->window_chunked = plan->win_chunked ? 1 : 0;
      }
      info->transposed_segment = plan->tseglen;
      if (plan->cx) {
        const CplxState& cx = *plan->cx;
        info->nnz = cx.nnz;
        info->stored = cx.stored;
        info->max_band = cx.max_band;
        info->max_abs[0] = cx.maxabs;
        info->nnz_blk[0] = cx.nnz;
        info->kappa = cx.kappa;
        const int64_t tb = (int64_t)plan->n_tiles * 16;
        info->matrix_bytes_f64 = cx.stored * 16 + tb;
        info->matrix_bytes_f32 = cx.stored * 8 + tb;
      }
      info->reduced_fft_f64 = plan->reduced_fft64 ? 1 : 0;
      info->reduced_fft_f32_err = plan->reduced_fft32_err;
    }
  });
}

spt_status spt_plan_nodes(spt_plan_t plan, double* out) {
  return guard([&] {
    check_plan(plan);
    if (!out) throw Error(SPT_E_INVALID_ARG, "out is NULL");
    if (!plan->precomputed) throw Error(SPT_E_NOT_PRECOMPUTED, "plan is not precomputed");
    if (plan->cx) {
      std::copy(plan->cx->angles.begin(), plan->cx->angles.end(), out);
      return;
    }
    set_device(plan);
    SPT_HIP(hipMemcpy(out, plan->nodes.p, plan->N * sizeof(double), hipMemcpyDeviceToHost));
  });
}

spt_status spt_plan_compressed_rows(spt_plan_t plan, int32_t blk, int64_t row0, int64_t nrows,
                                    double* out) {
  return guard([&] {
    check_plan(plan);
    if (!plan->precomputed) throw Error(SPT_E_NOT_PRECOMPUTED, "plan is not precomputed");
    if (plan->cx) throw Error(SPT_E_UNSUPPORTED, "complex plans: rows are not exported");
    if (blk < 0 || blk >= (int)plan->blk.size()) throw Error(SPT_E_INVALID_ARG, "bad block");
    if (!out || row0 < 0 || nrows < 0 || row0 + nrows > plan->N)
      throw Error(SPT_E_INVALID_ARG, "bad row range");
    const DevBlock& B = *plan->blk[blk];
    if (!B.val64.p) throw Error(SPT_E_UNSUPPORTED, "F64 values were not prepared");
    set_device(plan);
    const int64_t P1 = B.P + 1;
    std::fill(out, out + 2 * nrows * P1, 0.0);
    if (nrows == 0) return;
    const int64_t t0 = row0 / TILE_ROWS, t1 = (row0 + nrows - 1) / TILE_ROWS;
    for (int64_t t = t0; t <= t1; ++t) {
      const int kw = B.h_kw[t];
      if (kw == 0) continue;
      std::vector<double2> box((size_t)kw * TILE_ROWS);
      SPT_HIP(hipMemcpy(box.data(), B.val64.as<double2>() + B.h_off[t],
                        box.size() * sizeof(double2), hipMemcpyDeviceToHost));
      for (int kk = 0; kk < kw; ++kk)
        for (int q = 0; q < TILE_ROWS; ++q) {
          const int64_t n = t * TILE_ROWS + q;
          if (n < row0 || n >= row0 + nrows) continue;
          const int64_t k = B.h_k0[t] + kk;
          out[2 * ((n - row0) * P1 + k)] = box[(size_t)kk * TILE_ROWS + q].x;
          out[2 * ((n - row0) * P1 + k) + 1] = box[(size_t)kk * TILE_ROWS + q].y;
        }
    }
  });
}

spt_status spt_profile_begin(void) {
  return guard([&] {
    for (auto& r : g_prof.recs) {
      g_prof.pool.push_back(r.a);
      g_prof.pool.push_back(r.b);
    }
    g_prof.recs.clear();
    g_prof.on = true;
  });
}

spt_status spt_profile_end(double* ms, int64_t* launches) {
  return guard([&] {
    g_prof.on = false;
    if (ms) std::fill(ms, ms + SPT_NUM_STAGES, 0.0);
    if (launches) std::fill(launches, launches + SPT_NUM_STAGES, (int64_t)0);
    for (auto& r : g_prof.recs) {
      SPT_HIP(hipEventSynchronize(r.b));
      float t = 0.f;
      SPT_HIP(hipEventElapsedTime(&t, r.a, r.b));
      if (ms) ms[r.stage] += t;
      if (launches) launches[r.stage] += 1;
      g_prof.pool.push_back(r.a);
      g_prof.pool.push_back(r.b);
    }
    g_prof.recs.clear();
  });
}

spt_status spt_plan_destroy(spt_plan_t plan) {
  return guard([&] {
    if (!plan) return;
    (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    drop_batch_contexts(plan);  // batched contexts refer to its buffers
    delete plan;
  });
}

}  // extern "C"
