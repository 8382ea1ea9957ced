// Persistent executor of the computation stage (Alg. 1 steps 2.1-2.2 with the
// block version of sec. 3): one launch runs every step of one plan, or of a
// batch of plans, as a queue of work items.
//
// Items (taken in queue order by a persistent grid, one item per workgroup at
// a time):
//   ITEM_FFT   extend, divide by the window and F* for up to 64 right-hand
//              sides of a block whose packed length P fits one workgroup;
//   ITEM_COL   first half of a four-step F* (P = P1 * P2): length-P1
//              transforms over a group of columns, times the twiddles
//              exp(2 pi i n2 k1 / P), into the intermediate W;
//   ITEM_ROW   second half: length-P2 transforms over pairs of rows (k1 and
//              P1 - k1, which the real-to-half-spectrum unpacking couples);
//   ITEM_SPMM  two tiles of 16 output rows x 64 right-hand sides: the direct
//              tail, then every block's banded product (smallest blocks first),
//              each after that block's spectra of those right-hand sides are
//              complete.
// Dependencies are counters in device memory: a producer publishes its writes
// (agent-scope release) and adds to its counter; a consumer waits for the count
// it needs, then acquires.  Items only wait for items earlier in the queue, and
// the queue is taken in order, so every awaited item is held by a running
// workgroup: the grid cannot deadlock, whatever the number of resident
// workgroups.  The last workgroup to finish returns every counter to zero for
// the next launch.
#pragma once

#include "common.hpp"
#include "worklist.hpp"

namespace spt {

constexpr int EXEC_THREADS = 512;
constexpr int EXEC_EPT = 8;                           // FFT points per thread
constexpr int EXEC_POINTS = EXEC_THREADS * EXEC_EPT;  // complex points of one workgroup's FFTs
constexpr int EXEC_MAX_PLANS = 64;  // plans of one launch (X, Y travel as arguments)
constexpr int EXEC_SYNC_HEAD = 0;   // next item
constexpr int EXEC_SYNC_DONE = 1;   // finished workgroups
constexpr int EXEC_SYNC_ERR = 2;    // set by a wait that gave up (sticky within a launch)
constexpr int EXEC_SYNC_WAIT = 3;   // bound of a dependency wait, 100 MHz ticks (host-set)
constexpr int EXEC_SYNC_BASE = 4;   // dependency counters start here
constexpr uint32_t EXEC_WAIT_DEFAULT = 100000000u;  // 1 s


template <typename T>
struct ExecBlock {
  const T* winv;             // 1 / w_c, c < L
  const double2* tw;         // two-level table of exp(2 pi i q / P)
  const double2* tw2;        // two-level table of exp(i pi k / P), k <= P
  int ntw;                   // entries of either table: 128 + P / 128 + 1
  const cplx_t<T>* post;     // exp(i pi k / P), k <= P
  const cplx_t<T>* val;      // tile boxes of the compressed block
  int64_t zoff;              // spectra of rhs r: Z + R * zoff + r * (P + 1)
  int64_t woff;              // four-step intermediate of rhs r: W + R * woff + r * P
  int64_t zoff4;             // pre-split spectra of rhs r: plane + R * zoff4 + r * ldz4
  int ldz4;                  // P + 1 rounded up to a multiple of 4
  int P, m_off, c_lo, c_hi;
  T scale;                   // 1 / sqrt(L)
  uint32_t magic;            // ceil(2^32 / P): u / P = umulhi(u, magic) for u * P < 2^32
  uint32_t magic1;           // the same for P + 1
  uint32_t magic2;           // the same for P2
  int four;                  // 1: four-step F*, 0: ITEM_FFT
  int P1, P2, lcw, lgp;      // 2^lcw columns per COL item, 2^lgp row pairs per ROW item
  int n_col, n_row;          // COL / ROW items per right-hand side
  int ctr;                   // counter of (block, rhs group of 16) g: sync[ctr + g]
  int cctr;                  // COL items done for rhs r: sync[cctr + r]
  int parts;                 // count of a complete rhs in sync[ctr + g]
  FftPlan f1;                // passes of P (ITEM_FFT) or of P1 (COL)
  FftPlan f2;                // passes of P2 (ROW)
};

template <typename T>
struct ExecPlan {
  cplx_t<T>* Z;              // half spectra of every block
  cplx_t<T>* W;              // four-step intermediates
  uint32_t* Zs;              // pre-split spectra (three planes, staged split-bf16 path)
  float2* Zf;                // float32 spectra of a float64 transform (staged F32 path
                             // with float64 FFTs; replaces Z as the output), or null
  int64_t zplane;            // plane stride, in (Re, Im) bfloat16 pairs
  const TileMeta* meta;      // tile box of (tile, block) at meta[tile * nblk + block]
  const ExecBlock<T>* blocks;
  const T* tailmat;          // direct tail, column m at tailmat + m * n_tiles * 16
  int64_t N;
  int R, nblk, n_tiles, tail;
};

template <typename T>
struct ExecArgs {
  const ExecPlan<T>* plans;
  const int4* items;
  uint32_t* sync;
  uint32_t* err_out;         // host-visible word: the launch's EXEC_SYNC_ERR at its end
  int n_items, n_sync;
  int ntw;                   // entries of the largest twiddle table (LDS copies)
  // right-hand sides: T, except float for the split-bf16 FFT items in float64
  // arithmetic (T = double, launch_fft_items with split)
  const void* X[EXEC_MAX_PLANS];
  T* Y[EXEC_MAX_PLANS];
};

// dynamic LDS of the item kernels: the transform points, then the two twiddle
// tables of the block being transformed
template <typename T>
inline size_t exec_lds_bytes(int ntw) {
  return (size_t)EXEC_POINTS * sizeof(cplx_t<T>) + 2 * (size_t)ntw * sizeof(double2);
}

// engine: 0 = float64, 1 = float32, 2 = split bfloat16 (T = float)
template <typename T>
void launch_exec(const ExecArgs<T>& a, int engine, int grid, hipStream_t s);
// The FFT items without the queue and the counters (items of one launch do
// not depend on each other): one workgroup per item of a.items[0 .. n_items).
// split: spectra go out as the three bfloat16 planes.  With T = double and
// split or xf the right-hand sides are float (a.X) and the transforms run in
// float64 arithmetic, each spectrum value rounded once to float32 (before its
// split, or into ExecPlan::Zf).
template <typename T>
void launch_fft_items(const ExecArgs<T>& a, bool split, bool xf, hipStream_t s);
// Precomputation: F of the rows of a panel by four-step items (float64);
// a.plans[0] describes the panel: X[0] = the rows (stride N = L), Z = the half
// spectra (stride P + 1), W = the intermediate (stride P), R = rows; the
// block's winv is null.
void launch_row_fft4(const ExecArgs<double>& a, hipStream_t s);
// resident workgroups per CU of the executor kernel of this engine
int exec_occupancy(int engine, int ntw);
void init_exec_kernels();

}  // namespace spt
