// Shared host/device definitions of the spt library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "spt.h"

namespace spt {

// Rows per compressed tile: every block of a plan is cut into the same row
// tiles of TILE_ROWS consecutive nodes, so that one workgroup owns the same
// output rows in every block and sums the blocks in registers.
constexpr int TILE_ROWS = 16;
// Tiles per workgroup of the banded product (one wave per tile).
constexpr int SPMM_GROUP = 4;
// Largest number of blocks a plan may have (the recursion stops long before).
constexpr int MAX_BLOCKS = 24;
// Largest FFT radix pass count.
constexpr int MAX_PASSES = 16;
// longest FFT half-length of the fused one-workgroup-per-transform kernel: a
// float64 transform of P points fills P * 16 bytes of the 160 KiB LDS
constexpr int FUSED_MAX_P = 10240;
// the fused FFT splits transforms of an even number of points, at least
// this many, into two workgroups (by the parity of the outputs)
constexpr int FUSED_HALF_MIN_P = 4096;
// longest FFT half-length of the fused computation-stage FFT when it is split
// (parity halves or the eight-way split): a float64 parity half of 8192
// points and its tables fill 136 KiB of LDS.  Longer blocks go by four steps.
constexpr int FUSED_FWD_MAX_P = 16384;
// AUTO mode compares built blocks with the dense matrix up to this N, and an
// estimate from sampled rows above it
constexpr int64_t AUTO_EXACT_N = 8192;

struct Error : std::runtime_error {
  spt_status code;
  Error(spt_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SPT_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::spt::Error(e_ == hipErrorOutOfMemory ? SPT_E_OOM : SPT_E_HIP,             \
                         std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

// load through a global-memory pointer: a pointer loaded from memory or rebuilt
// from an integer is generic, and a generic (flat) load also waits for and is
// waited on by LDS traffic
template <typename V>
__device__ __forceinline__ V gload(const V* p) {
  return *(const __attribute__((address_space(1))) V*)p;
}
// HIP's float2 / double2 are classes: load their native vector
__device__ __forceinline__ float2 gload(const float2* p) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const __attribute__((address_space(1))) v2*)p;
  return float2{v.x, v.y};
}
__device__ __forceinline__ double2 gload(const double2* p) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const __attribute__((address_space(1))) v2*)p;
  return double2{v.x, v.y};
}

// A raw buffer over `bytes` bytes at p (gfx9 buffer resource, 32-bit
// elements): a load whose offset is at or past the end, a negative offset
// included (it wraps past the end), returns zeros.  Offsets are in bytes and
// all go in the lane's offset register, which is what the range check sees.
typedef __amdgpu_buffer_rsrc_t buf_t;
__device__ __forceinline__ buf_t buf_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float buf_f32(buf_t r, int off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ float2 buf_f32x2(buf_t r, int off) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  return float2{v.x, v.y};
}
__device__ __forceinline__ float4 buf_f32x4(buf_t r, int off) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 v = __builtin_bit_cast(v4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  return float4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ double buf_f64(buf_t r, int off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ double2 buf_f64x2(buf_t r, int off) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  return double2{v.x, v.y};
}
// typed forms: buf_ld<float>, buf_ld<float2>, buf_ld<double>, buf_ld<double2>
template <typename V> __device__ __forceinline__ V buf_ld(buf_t r, int off);
template <> __device__ __forceinline__ float buf_ld<float>(buf_t r, int off) { return buf_f32(r, off); }
template <> __device__ __forceinline__ float2 buf_ld<float2>(buf_t r, int off) { return buf_f32x2(r, off); }
template <> __device__ __forceinline__ double buf_ld<double>(buf_t r, int off) { return buf_f64(r, off); }
template <> __device__ __forceinline__ double2 buf_ld<double2>(buf_t r, int off) { return buf_f64x2(r, off); }

template <typename T> struct cplx;
template <> struct cplx<double> { using type = double2; };
template <> struct cplx<float> { using type = float2; };
template <typename T> using cplx_t = typename cplx<T>::type;

// FFT radix schedule for one length P (complex points): P = prod(radix[i]).
struct FftPlan {
  int P = 1;
  int npass = 0;
  int radix[MAX_PASSES] = {};
  int threads = 64;
};

// radix10: the plan may merge a radix 2 and a radix 5 into one radix-10 pass,
// which only the fused FFT kernels take (run_fft<..., R10 = true>)
FftPlan make_fft_plan(int P, bool radix10 = false);

// ---------------------------------------------------------------- kernel launch API
// (implemented in the .hip files; all take device pointers and a stream)

template <typename T>
struct ExecFftArgs {
  const T* X;         // R x N input (RHS-major)
  cplx_t<T>* Z;       // R x ldz output half spectrum
  const T* winv;      // 1/w over the block's L columns
  const double2* tw;      // P twiddles e^{+2 pi i q/P} (float64 for every precision)
  const cplx_t<T>* post;  // P+1 twiddles e^{+i pi k/P}
  int64_t N;
  int R, L, P, ldz, m_off, c_lo, c_hi;
  T scale;            // 1/sqrt(L)
};

template <typename T>
void launch_exec_fft(const ExecFftArgs<T>& a, const FftPlan& fp, hipStream_t s);

// One block of the fused x-side FFT launch (all blocks of a plan, all
// right-hand sides in one grid); lives in device memory.
template <typename T>
struct FftDesc {
  const T* winv;
  const double2* tw;
  const cplx_t<T>* post;
  int64_t zoff;  // block spectra start at Z + R * zoff; right-hand side r at + r * ldz
  FftPlan fp;
  int L, m_off, c_lo, c_hi, ldz;
  T scale;
  int64_t zoff4;  // the same for the split planes (ldz4 = ldz rounded up to 4)
  int ldz4;
  const double2* tw2;  // two-level table of exp(i pi k / P), k <= P
  int ntw;             // entries of tw and of tw2: 128 + P / 128 + 1
  // the fused launch gives each workgroup 2^lb right-hand sides of this block
  // (2^lb fp.P <= the launch's largest fp.P)
  int lb;
  // FFT_SPLIT_PARITY: the transform of P = L/2 points is split by the parity
  // of its outputs into two halves of fp.P = P/2 points, one workgroup each;
  // FFT_SPLIT_EIGHT: the real transform of L points is split by the residue
  // of its outputs mod 8 into five workgroups of fp.P = L/8 points
  int half;
};

enum { FFT_SPLIT_NONE = 0, FFT_SPLIT_PARITY = 1, FFT_SPLIT_EIGHT = 2 };

// workgroups per right-hand side of a split transform
inline int fft_split_wgs(int half) {
  return half == FFT_SPLIT_EIGHT ? 5 : half == FFT_SPLIT_PARITY ? 2 : 1;
}

// The fused FFT launch's one-dimensional grid: block b takes workgroups
// wg0[b] .. wg0[b + 1] - 1 (no idle workgroups); at most FFT_GRID_MAX blocks
// per launch.
constexpr int FFT_GRID_MAX = 16;
struct FftGrid {
  int nblk;
  int wg0[FFT_GRID_MAX + 1];
};

// grid: the g.wg0[g.nblk] workgroups of `threads` that g assigns to the
// blocks; lds: bytes of the largest workgroup (fused_lds_bytes)
template <typename T>
void launch_exec_fft_multi(const FftDesc<T>* descs, const FftGrid& g, int threads, size_t lds,
                           const T* X, cplx_t<T>* Z, int R, int64_t N, hipStream_t s);
// LDS of a fused FFT workgroup of pts points whose block has two-level
// twiddle tables of ntw entries (tw and tw2, float64)
template <typename T>
inline size_t fused_lds_bytes(int pts, int ntw) {
  const size_t data = ((size_t)pts * sizeof(cplx_t<T>) + 15) & ~(size_t)15;
  return data + 2 * (size_t)ntw * sizeof(double2);
}

template <typename T>
struct InvFftArgs {      // transposed execute: half spectrum -> real, /w, keep retained
  const cplx_t<T>* U;   // R x ldu half spectrum
  T* Y;                 // R x N output, written at degrees c + m_off, c in [c_lo, c_hi)
  const T* winv;
  const double2* tw;
  const cplx_t<T>* post;
  int64_t N;
  int R, L, P, ldu, m_off, c_lo, c_hi;
  T scale;
};

template <typename T>
void launch_inv_fft(const InvFftArgs<T>& a, const FftPlan& fp, hipStream_t s);

// The single-workgroup inverse transforms of every block in one launch:
// workgroup (r, b) takes right-hand side r of block descs[b] (half spectra at
// uoff R complex values into U).
template <typename T>
struct InvFftDesc {
  const T* winv;
  const double2* tw;
  const cplx_t<T>* post;
  int64_t uoff;
  int P, m_off, c_lo, c_hi;
  T scale;
  FftPlan fp;
};

template <typename T>
void launch_inv_fft_multi(const InvFftDesc<T>* descs, int nblk, int threads, size_t lds,
                          const cplx_t<T>* U, T* Y, int R, int64_t N, hipStream_t s);
// the float32 path's single-workgroup inverse transforms in float64 arithmetic
// (float32 U and Y, the float64 descriptors and tables; lds for double2 points)
void launch_inv_fft_multi_x32(const InvFftDesc<double>* descs, int nblk, int threads, size_t lds,
                              const float2* U, float* Y, int R, int64_t N, hipStream_t s);

// T: arithmetic, tables and intermediate; TI: type of U and Y (float with T =
// double: the float32 path's transform in float64 arithmetic)
template <typename T, typename TI = T>
struct InvFft4Args {      // transposed execute of a block with P = P1 P2 (four steps)
  const cplx_t<TI>* U;    // R x ldu half spectrum
  cplx_t<T>* W;           // R x P intermediate, W[j2 P1 + k1]
  TI* Y;                  // R x N output, written at degrees c + m_off, c in [c_lo, c_hi)
  const T* winv;
  const double2* tw;      // two-level table of the length P
  const cplx_t<T>* post;
  int64_t N;
  int R, P, P1, P2, ldu, m_off, c_lo, c_hi;
  int lb1, lb2;           // 2^lb1 transforms over k2, 2^lb2 over k1, per workgroup
  FftPlan f1, f2;         // passes of the P1- and P2-point transforms
  T scale;
};

template <typename T, typename TI = T>
void launch_inv_fft4(const InvFft4Args<T, TI>& a, hipStream_t s);

struct RowFftArgs {      // precompute: forward F of windowed rows, float64
  const double* rows;    // nrows x L
  double2* spec;         // nrows x (P+1)
  const double2* tw;
  const double2* post;
  int nrows, L, P;
  double scale;
};
void launch_row_fft(const RowFftArgs& a, const FftPlan& fp, hipStream_t s);

// banded product, all blocks + tail, y = sum_i Re(A_i z_i) + B_tail x_tail
struct TileMeta {      // one (tile, block): box columns k0 .. k0+kw-1 at val + off
  int32_t k0, kw;
  int64_t off;
};
template <typename T>
struct SpmmBlock {     // one block: its tile boxes and where its half spectra live
  const cplx_t<T>* val;
  int64_t zoff;        // spectra of the block start at Z + R * zoff
  int32_t ldz;         // P + 1
  int32_t pad;
};
template <typename T>
struct SpmmArgs {
  const TileMeta* meta;        // n_tiles x nblk, tile-major
  const SpmmBlock<T>* blocks;  // nblk
  int nblk;
  int n_tiles;
  const cplx_t<T>* Z;          // half spectra written by the FFT stage
  int tail;
  const T* tailmat;   // tail x (n_tiles * TILE_ROWS): column m of the tail over rows
  const T* X;
  T* Y;
  int R;
  int64_t N;
  const struct WinMeta* win;  // batches: the windows of a plan the chunked float64
                              // product takes (n_groups x nblk), else null
};

template <typename T>
void launch_spmm(const SpmmArgs<T>& a, hipStream_t s);
void launch_spmm_split_bf16(const SpmmArgs<float>& a, hipStream_t s);

// Pre-split storage of the split-bf16 path.  Every value f is kept as three
// bfloat16 pieces p0 + p1 + p2 (p0 = bf16(f), p1 = bf16(f - p0),
// p2 = bf16(f - p0 - p1), round to nearest even).
//  * Tile box of (tile, block), 16-column steps s: piece p of step s is 64
//    lanes x 8 bfloat16 at val + off + (3 s + p) * 512 + 8 lane; lane l holds
//    row l % 16, complex columns 16 s + 4 (l / 16) + j / 2 (j < 8), as
//    (Re, -Im) pairs; columns past kw are zero.
//  * Half spectra: three planes (plane stride zplane, in complex values);
//    rhs r of a block at plane + zoff * R + r * ldz, ldz = P + 1 rounded up to
//    a multiple of 4 (zeros past P); a complex value is a (Re, Im) bfloat16 pair.
//  * Direct tail: per tile, 32-column steps s, piece p at
//    tail + ((tile * tsteps + s) * 3 + p) * 512 + 8 lane, lane l holding row
//    l % 16, tail columns 32 s + 8 (l / 16) + j.
struct SpmmSplitBlock {
  const uint16_t* val;
  int64_t zoff;
  int32_t ldz;
  int32_t pad;
};

struct WinMeta;
struct SpmmSplitArgs {
  const TileMeta* meta;          // n_tiles x nblk (off in bfloat16 units)
  const SpmmSplitBlock* blocks;  // nblk
  int nblk;
  int n_tiles;
  const uint32_t* Zs;            // spectra planes of (Re, Im) bfloat16 pairs
  int64_t zplane;
  int tail;
  const uint16_t* tailmat;       // pre-split tail
  const float* X;
  float* Y;
  int R;
  int64_t N;
  const WinMeta* win;            // staged batches: the plan's windows (chunked product),
  int n_groups, tpad;            // or null for the per-tile product
};
void launch_spmm_presplit(const SpmmSplitArgs& a, hipStream_t s);

// Windowed pre-split product: a workgroup takes WIN_TILES consecutive row
// tiles and NR = 16 rg right-hand sides (rg = 4 or 2), and the half spectra
// its tiles' boxes need in each block (the union of the boxes, a window of
// consecutive columns) are staged in LDS once for all of them.  Window of
// (tile group, block) in LDS: row q = NR p + i (piece p, right-hand side
// r0 + i) at lds + q * pitch, pitch 16-byte units (4 complex columns each)
// from column k0.
constexpr int WIN_TILES = 4;
struct WinMeta {
  int32_t k0;      // first column of the window (multiple of 4)
  int32_t w4;      // width in groups of 4 columns (0: no box of the block in the group)
  int32_t pitch;   // LDS row pitch in 16-byte units: odd, >= max(w4, 3)
  int32_t lds;     // offset of the window in LDS, 16-byte units
  uint32_t magic;  // ceil(2^32 / pitch): q = umulhi(u, magic) = u / pitch for u * pitch < 2^32
  int32_t units;   // 16-byte units of the window, 3 * NR * pitch rounded up to 64
  int32_t pad[2];
};
// win: n_groups x nblk, group-major.  LDS: the windows (the largest sum of a
// group's windows), then from 16-byte unit xlds the direct tail's x of the NR
// right-hand sides, tpad = 32 * ceil(tail / 32) + 4 floats apart (0: no tail).
// Plans whose windows do not fit: the same windows (k0, w4 only) staged in
// chunks; LDS bytes of a workgroup for a tail pitch tpad.
size_t spmm_chunk_lds_bytes(int tpad);
// the float64 matrix-core product through the same chunked windows
void launch_spmm_chunk_f64(const SpmmArgs<double>& a, const WinMeta* win, int n_groups,
                           hipStream_t s);
void launch_spmm_chunk(const SpmmSplitArgs& a, const WinMeta* win, int n_groups, int tpad,
                       hipStream_t s);
// waves: per row tile (2: 8-wave workgroups over 64 right-hand sides, rg 4)
void launch_spmm_window(const SpmmSplitArgs& a, const WinMeta* win, int n_groups, int rg,
                        int waves, int xlds, int tpad, size_t lds_bytes, hipStream_t s);
void init_spmm_kernels(size_t max_lds);

// Products of several plans in one launch: items (plan, row tile or -1, first
// rhs) index per-plan argument blocks in device memory; X and Y of each plan
// travel in the kernel arguments.
constexpr int BATCH_MAX_PLANS = 64;
template <typename T>
struct SpmmBatch {
  const SpmmArgs<T>* plans;
  const int4* items;
  const T* X[BATCH_MAX_PLANS];
  T* Y[BATCH_MAX_PLANS];
};
struct SpmmSplitBatch {
  const SpmmSplitArgs* plans;
  const int4* items;
  const float* X[BATCH_MAX_PLANS];
  float* Y[BATCH_MAX_PLANS];
};
template <typename T>
void launch_spmm_items(const SpmmBatch<T>& b, int n_items, hipStream_t s);
// items {plan, tile group, first right-hand side, 0} of the chunked float64
// product (group < 0: padding); the plans' SpmmArgs carry their windows
void launch_spmm_chunk_f64_items(const SpmmBatch<double>& b, int n_items, hipStream_t s);
void launch_spmm_presplit_items(const SpmmSplitBatch& b, int n_items, hipStream_t s);
// items {plan, tile group, first right-hand side, 0} of the chunked product
// (group < 0: padding); lds: the largest spmm_chunk_lds_bytes of the plans
void launch_spmm_chunk_items(const SpmmSplitBatch& b, int n_items, size_t lds, hipStream_t s);

// split-bf16 staged FFT: the half spectra go out as the three planes above
void launch_exec_fft_multi_split(const FftDesc<float>* descs, const FftGrid& g, int threads,
                                 size_t lds, const float* X, uint32_t* Zs, int64_t zplane, int R,
                                 int64_t N, hipStream_t s);
// the float32 paths' transforms in float64 arithmetic (float32 X, the float64
// descriptors and tables; lds from fused_lds_bytes<double>): each spectrum
// value is rounded once to float32, then split into the three planes Zs
// (split-bf16) or stored in Z (float32 path, Zs null)
void launch_exec_fft_multi_x32(const FftDesc<double>* descs, const FftGrid& g, int threads,
                               size_t lds, const float* X, float2* Z, uint32_t* Zs,
                               int64_t zplane, int R, int64_t N, hipStream_t s);

// transposed banded product: u_i = A_i^T f (half spectrum), per block
// The transposed product gathers by columns of the half spectrum: the row
// tiles whose boxes meet columns [TCHUNK c, TCHUNK c + TCHUNK) of a block.
constexpr int TCHUNK = 32;
constexpr int TSEG = 8;    // row tiles per segment (one workgroup each), at least
constexpr int TSEG_BLOCK_BITS = 5;  // block field of a segment (MAX_BLOCKS <= 32)
struct TChunkEnt {
  int64_t off;             // the tile's first stored value
  int32_t tile, k0, kw, pad;
};

// per block: its stored values and where its half spectra start in the
// workspace (uoff R complex values in)
struct TBlkInfo {
  const void* val64;
  const void* val32;
  int64_t uoff;
  int32_t P, pad;
};

template <typename T>
struct SpmmTArgs {
  const int4* segs;        // n_segs segments of every block: {chunk c, first entry, end entry,
                           // slot << 6 | block << 1 | (1 if the only segment of c)}
  const TChunkEnt* ents;   // per block and chunk, the row tiles meeting it
  const TBlkInfo* blk;
  cplx_t<T>* u;            // the workspace: block b's R x (P + 1) half spectra at uoff R
  cplx_t<T>* part;         // R x TCHUNK partial sums per slot (chunks of several segments)
  const int4* red;         // n_red chunks of several segments: {block, chunk, first slot, slots}
  int n_segs, n_red;
  const T* F;              // R x N
  int R;
  int64_t N;
};
// products64: a tile's rows summed in float64 as well (float32 plans with
// float64 spectra-side arithmetic)
template <typename T>
void launch_spmm_transposed(const SpmmTArgs<T>& a, bool products64, hipStream_t s);

// tail of the transposed product: fhat[:, m] += sum_j A[j, m] f_j, m < tail
template <typename T>
void launch_tail_transposed(const T* tailmat, int tail, const T* F, T* Y, int R, int64_t N,
                            hipStream_t s);

// ---------------------------------------------------------------- precompute kernels
// the trigonometric generators: closed-form entries at the Chebyshev-Gauss
// angles, extras on both sides (Algorithm 1)
__host__ __device__ inline bool is_trig(int family) {
  return family == SPT_CHEBYSHEV_T || family == SPT_SINE || family == SPT_COS_POWER;
}
// the complex generators (Algorithm 1, complex data, full spectrum; cplx.hip)
__host__ __device__ inline bool is_complex_family(int family) {
  return family == SPT_CEXP || family == SPT_LAGUERRE_SPECTRAL;
}

// ---------------------------------------------------------------- complex generators (cplx.hip)
// rows row0 .. of A_e W (degrees m = c + m_off, c < L), complex float64, row
// stride L: exp(i m theta_j) at the exact angle (SPT_CEXP), or exp(i m phi_j)
// rowf_j (SPT_LAGUERRE_SPECTRAL, rowf_j = 1 / (eta/2 - i k_j))
struct CplxRowsArgs {
  double2* out;
  const double* w;      // window, L entries
  const double* phi;    // row phases (SPT_LAGUERRE_SPECTRAL)
  const double2* rowf;  // row factors (SPT_LAGUERRE_SPECTRAL)
  int64_t N, row0;
  int L, m_off, family;
};
void launch_cplx_rows(const CplxRowsArgs& a, int nrows, hipStream_t s);
// F (unitary, SIGN -1) of nrows rows of L points in place (L <= 10240)
void launch_cplx_row_fft(double2* rows, int nrows, int L, const FftPlan& fp, const double2* tw,
                         hipStream_t s);
template <typename TI>
struct CplxExecArgs {
  const cplx_t<TI>* X;  // R x N complex
  cplx_t<TI>* Z;        // R x ldz spectra (ldz = L + pad)
  const double* winv;   // 1 / w_c, c < L
  const double2* tw;    // two-level table of exp(2 pi i q / L)
  int64_t N;
  int L, ldz, m_off, c_lo, c_hi;
  double scale;         // 1 / sqrt(L)
};
template <typename TI>
void launch_cplx_exec_fft(const CplxExecArgs<TI>& a, const FftPlan& fp, int R, hipStream_t s);
template <typename T>
struct CplxSpmmArgs {
  const TileMeta* meta;  // per tile: box columns k0 .. k0 + kw - 1 (k0 < L), values at off
  const cplx_t<T>* val;  // val[off + kk * 16 + q]
  const cplx_t<T>* Z;
  cplx_t<T>* Y;
  int64_t N;
  int R, ldz;
};
template <typename T>
void launch_cplx_spmm(const CplxSpmmArgs<T>& a, int n_tiles, int max_kw, hipStream_t s);
template <typename T>
struct CplxSpmmTArgs {
  const TileMeta* meta;
  const cplx_t<T>* val;
  const int32_t* tptr;   // tiles of the 32-column chunk c: tents[tptr[c] .. tptr[c + 1])
  const int32_t* tents;
  const cplx_t<T>* F;    // R x N
  cplx_t<T>* U;          // R x ldu (ldu = L + pad)
  int64_t N;
  int R, ldu;
};
template <typename T>
void launch_cplx_spmm_t(const CplxSpmmTArgs<T>& a, int n_chunks, int max_list, hipStream_t s);
template <typename TI>
struct CplxInvArgs {
  const cplx_t<TI>* U;
  cplx_t<TI>* Y;
  const double* winv;
  const double2* tw;
  int64_t N;
  int L, ldu, m_off, c_lo, c_hi;
  double scale;
};
template <typename TI>
void launch_cplx_inv_fft(const CplxInvArgs<TI>& a, const FftPlan& fp, int R, hipStream_t s);

struct FamilyArgs {
  int family;
  int power;              // s of SPT_COS_POWER
  int64_t N;
  int unweighted;
  const double* x;        // nodes
  const double* rowscale; // sqrt(lambda_j) (Jacobi family) or NULL
  const double* ca;       // recurrence coefficient tables (family specific)
  const double* cb;
  const double* cc;
  int ncoef;              // entries in the tables
  double p0;              // p_0 for the Jacobi family
};

void launch_nodes(const FamilyArgs& f, const double* diag, const double* off2, double lo,
                  double hi, double* x_out, hipStream_t s);
void launch_weights(const FamilyArgs& f, double* rowscale, hipStream_t s);

// Appendix A: compressed rows of a trigonometric generator without a row FFT.
// Row j's entry k of the half spectrum is L^{-1/2} sum_{|m| <= q} vt_m
// U_{(k-m) mod L}, with vt the window's spectrum (2q+1 coefficients) and U the
// closed-form DFT of the row's tones (eq. y3 and its cos / sin halves); only
// the bins within B of each tone are evaluated, the rest of the panel is zero.
constexpr int TRIG_MAX_TONES = 4;
struct TrigSpecArgs {
  int64_t N;
  int L, P, m_off, q, B;
  int sine;                       // 1: the sine generator (tones are sines)
  int ntones;
  int tone[TRIG_MAX_TONES];       // t >= 0: the tone pair exp(+-i t m theta_j)
  double coef[TRIG_MAX_TONES];
  const double2* vt;              // window spectrum, m = -q .. q
  int64_t row0;
  int nrows;
  double2* spec;                  // nrows x (P+1), zero elsewhere (caller clears)
};
void launch_trig_spec(const TrigSpecArgs& a, hipStream_t s);
// rows [row0, row0+nrows) x degrees [m0, m0+L), times window w (NULL = 1),
// row-major into out (ld = L)
void launch_rec_rows(const FamilyArgs& f, int64_t row0, int nrows, int m0, int L,
                     const double* w, double* out, hipStream_t s);
// tail matrix: out[m * N + j] = A[j, m], m < t (float64)
void launch_rec_tail(const FamilyArgs& f, int t, double* out, hipStream_t s);

void launch_maxabs(const double2* spec, int64_t count, unsigned long long* max_bits,
                   hipStream_t s);
void launch_extents(const double2* spec, int nrows, int P, double thr, int32_t* klo,
                    int32_t* khi, int32_t* cnt, hipStream_t s);
void init_fft_kernels(size_t max_lds);
void launch_pack(const double2* spec, int64_t row0, int nrows, int64_t N, int P, double thr,
                 const int32_t* tile_k0, const int32_t* tile_kw, const int64_t* tile_off,
                 int tile0, double2* val64, float2* val32, hipStream_t s);
void launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
// pre-split tile boxes from the float32 ones (layout above)
void launch_split_pack(const float2* val32, const int32_t* tile_kw, const int64_t* tile_off,
                       const int64_t* tile_soff, int ntiles, uint16_t* valbf, hipStream_t s);
// pre-split direct tail from the float32 one (column m at tail32 + m * ldt)
void launch_split_tail(const float* tail32, int64_t ldt, int tail, int ntiles, uint16_t* tailbf,
                       hipStream_t s);
void launch_nonfinite(const double* p, int64_t n, int* flag, hipStream_t s);

}  // namespace spt
