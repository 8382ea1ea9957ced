/*
 * spt.h -- fast special-function transforms by the extra-component method
 * (A. V. Terekhov, "An extra-component method for evaluating fast
 * matrix-vector multiplication with special functions", arXiv 2004.11610),
 * on AMD Instinct MI355X (gfx950).
 *
 * The library computes y = A x for a fixed N x N matrix A of special-function
 * values at quadrature nodes, for many right-hand sides x, in O(N log N) per
 * right-hand side after an O(N^2 log N) precomputation:
 *
 *   precomputation (Alg. 1 steps 1.1-1.3; sec. 3 for the block version)
 *     zeta(eps1) and the extra-component counts s_i (sec. 2.2), the block
 *     partition (sec. 3, Table 1), the compressed blocks A_e W F (eq. A_comp)
 *     thresholded at eps1 * max|A_e W F| and stored as banded tiles.
 *   computation (Alg. 1 steps 2.1-2.2; sec. 3)
 *     extend x with zero extra components and divide by the window (eq. Fe1),
 *     real-to-half-complex FFT (F*, sec. 5.1), banded product with every block
 *     and the direct tail, summed into y (eq. comp1).
 *   transposed computation (Alg. 2 steps 2.1-2.2; sec. 3)
 *     banded product with the transposed blocks, inverse FFT, divide by the
 *     window and discard the extra components (eq. Fe2).
 *
 * Matrices (row j = node x_j, column m = degree):
 *   SPT_CHEBYSHEV_T  A[j,m] = T_m(x_j) = cos(m theta_j), Chebyshev-Gauss nodes
 *                    theta_j = pi (j+1/2)/N (eq. cheb_matrix); Algorithm 1 with
 *                    extras on both sides.
 *   SPT_LEGENDRE     A[j,m] = sqrt(lambda_j) p_m(x_j), orthonormal Legendre
 *                    polynomials, Gauss-Legendre nodes (x descending) and
 *                    Christoffel weights lambda_j, so A is orthogonal (sec. 5.2).
 *   SPT_JACOBI       the same for Jacobi (alpha, beta), alpha, beta > -1.
 *   SPT_LAGUERRE_FN  A[j,m] = exp(-x_j/2) L_m(x_j), Gauss-Laguerre nodes
 *                    ascending (sec. 4).
 *   SPT_HERMITE_FN   A[j,m] = psi_m(x_j), Hermite functions, Gauss-Hermite
 *                    nodes ascending.
 *   SPT_SINE         A[j,m] = sin(m theta_j) at the Chebyshev-Gauss angles: a
 *                    generator Algorithms 1 and 2 compress as they do the
 *                    cosine one (sec. 2, after Algorithm 2).
 *   SPT_COS_POWER    A[j,m] = cos(m theta_j)^s, s = spt_params.power in 2..5
 *                    (eq. cosd2), at the Chebyshev-Gauss angles.
 *   SPT_CEXP         A[j,m] = exp(i m theta_j) at the Chebyshev-Gauss angles: the
 *                    complex generator of sec. 2 (after Algorithm 2).
 *   SPT_LAGUERRE_SPECTRAL  A[j,m] = C[j,m] = (-eta/2 - i k_j)^m / (eta/2 - i k_j)^(m+1)
 *                    (sec. 4.1, eqs. main_formula2 and lag_matrix), k_j = 2 pi j / T
 *                    (spt_params.eta, .period): row j is exp(i m phi_j) /
 *                    (eta/2 - i k_j) with phi_j = 2 atan(2 k_j / eta) - pi (the
 *                    row phases; spt_params.nodes may give them instead); the
 *                    Laguerre coefficients of the spectral method are
 *                    V = C^T F (spt_execute_transposed).
 *   The complex generators (SPT_CEXP, SPT_LAGUERRE_SPECTRAL) use Algorithm 1 with
 *   extras on both sides and the full spectrum; X and Y are complex (interleaved
 *   re, im), float64 for SPT_F64 and float32 for SPT_F32 (transforms in float64
 *   arithmetic; SPT_SPLIT_BF16 unsupported); plans need L <= 10240 (one
 *   workgroup's transform); staged executor, no batches.
 *   The trigonometric generators (SPT_CHEBYSHEV_T, SPT_SINE, SPT_COS_POWER)
 *   use Algorithm 1, extras on both sides (the generator continues to m < 0);
 *   the others use the block method (sec. 3): extras on the right only,
 *   recursion on the first s_i columns, the last columns direct.
 *
 * Conventions for every call:
 *   - Every function returns spt_status: SPT_OK (0) or a negative error code;
 *     spt_last_error() then returns a message (thread-local, valid until the
 *     next call on the same thread).
 *   - A failed call leaves its plan valid (spt_plan_create leaves *out NULL).
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls that take a stream enqueue their work and return; device outputs
 *     are ready when the stream is synchronised.
 *   - Device pointers are HIP device memory of the device that was current
 *     when the plan was created.  Matrices of right-hand sides are RHS-major:
 *     X[r*N + m] is component m of right-hand side r (R x N, contiguous).
 *   - A plan owns its device memory (compressed blocks, tables, workspace)
 *     and frees it in spt_plan_destroy.  One plan must not execute on two
 *     streams at once (its workspace is shared).
 */
#ifndef SPT_H
#define SPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t spt_status;
enum {
  SPT_OK = 0,
  SPT_E_INVALID_ARG = -1,    /* a NULL, out-of-range or inconsistent argument */
  SPT_E_NOT_PRECOMPUTED = -2,/* execute before a successful spt_precompute    */
  SPT_E_HIP = -3,            /* a HIP runtime call failed (message has the text) */
  SPT_E_OOM = -4,            /* device memory allocation failed               */
  SPT_E_UNSUPPORTED = -5,    /* precision not prepared, size beyond a kernel  */
  SPT_E_NUMERIC = -6         /* non-finite values met in the precomputation   */
};

typedef enum {
  SPT_CHEBYSHEV_T = 1,
  SPT_LEGENDRE = 2,
  SPT_JACOBI = 3,
  SPT_LAGUERRE_FN = 4,
  SPT_HERMITE_FN = 5,
  SPT_SINE = 6,
  SPT_COS_POWER = 7,
  SPT_CEXP = 8,              /* complex: exp(i m theta_j), Chebyshev-Gauss angles */
  SPT_LAGUERRE_SPECTRAL = 9  /* complex: the matrix C of the spectral-domain
                                Laguerre transform (sec. 4.1, eq. lag_matrix) */
} spt_family;

/* Arithmetic of the execute path.  The precomputation is always float64. */
typedef enum {
  SPT_F64 = 0,        /* X, Y float64; FFT and banded product in float64          */
  SPT_F32 = 1,        /* X, Y float32; FFT and banded product in float32          */
  SPT_SPLIT_BF16 = 2  /* X, Y float32; FFT float32; banded product on the matrix
                         cores: both operands split into three bfloat16 pieces,
                         the six products of total order <= 2 accumulated in
                         float32                                               */
} spt_precision;

typedef enum {
  SPT_MODE_AUTO = 0,   /* ROW unless the compressed form stores more than dense
                          (decided on the built blocks for N <= 8192, from 8
                          panels of 64 sampled rows per block above)          */
  SPT_MODE_ROW = 1,    /* row compression (Alg. 1 / block Alg. 3)              */
  SPT_MODE_DIRECT = 3  /* dense product with A (no compression)                */
} spt_mode;

/* How spt_execute runs the computation stage. */
typedef enum {
  SPT_EXECUTOR_AUTO = 0,       /* STAGED (the faster one on MI355X)             */
  SPT_EXECUTOR_STAGED = 1,     /* launches in stream order: the FFTs of every
                                  block (four-step ones in two launches), then
                                  all banded products                          */
  SPT_EXECUTOR_PERSISTENT = 2  /* one launch: a persistent grid takes work items
                                  (FFTs of every block, four-step FFTs of long
                                  blocks, banded-product tiles) from a queue, a
                                  tile's product of a block starting once that
                                  block's spectra are complete                 */
} spt_executor;

/* Plan parameters.  A zero-filled struct selects every default. */
typedef struct {
  double alpha, beta;     /* SPT_JACOBI only; alpha, beta > -1                    */
  double eps2;            /* extra-component level eps2 (sec. 2.2); 0 -> 1e-2;
                             must satisfy eps < eps2 < 1                          */
  int32_t mode;           /* spt_mode                                             */
  int32_t unweighted;     /* LEGENDRE/JACOBI: 1 drops the sqrt(lambda_j) factor   */
  uint32_t precisions;    /* bit (1 << spt_precision) per execute precision to
                             prepare in spt_precompute; 0 -> all three            */
  int32_t min_block;      /* block recursion stops at width <= min_block; 0 -> 32 */
  int32_t exact_fft_len;  /* 0: L_i rounded up to the smallest even length whose
                             half is 2^a 3^b 5^c; 1: L_i = W_i + s_i as computed
                             (for geometry queries: spt_precompute then fails
                             with SPT_E_UNSUPPORTED unless every L_i has that
                             form)                                                 */
  int32_t executor;       /* spt_executor of spt_execute                          */
  int64_t panel_rows;     /* rows per precompute panel; 0 -> automatic            */
  const double* nodes;    /* optional host array of the N nodes, in the family's
                             order (see above); NULL -> computed on the device.
                             Copied during spt_plan_create.  The trigonometric
                             generators take their angles from the node index
                             and ignore it.                                       */
  int32_t power;          /* SPT_COS_POWER: s in 2..5 (others ignore it)          */
  int32_t trig_conv_q;    /* trigonometric generators only: 0 -> compressed rows
                             by row FFTs (eq. A_comp); q in 1..64 -> by the fast
                             precomputation of Appendix A: the closed-form DFT
                             of each row convolved with the 2q+1 window
                             coefficients m = -q..q (eq. conv_appendix), only
                             near each tone of the row.  The window's side
                             lobes make this an approximation: q = 12 moves an
                             entry by < 0.25 eps max|A_e W F|                     */
  double eta;             /* SPT_LAGUERRE_SPECTRAL: the Laguerre scale eta > 0    */
  double period;          /* SPT_LAGUERRE_SPECTRAL: the interval length T > 0 of
                             the Fourier series (k_j = 2 pi j / T)               */
  int32_t reduced_fft;    /* arithmetic of the x-side FFTs (and of the transposed
                             product's inverse FFTs) of the SPT_F32 and
                             SPT_SPLIT_BF16 paths, staged executor:
                             0 -> chosen at spt_precompute from 4 seeded N(0,1)
                             right-hand sides through the split-bf16 path (the
                             float32 path if only that is prepared) with float32
                             FFTs: kept when within 7e-7 of the float64 path
                             (relative 2-norm), the transposed float32 product
                             too when F32 and F64 are prepared, or, without a
                             float64 path, within 5e-7 of the same path with
                             float64 FFTs;
                             1 -> float32; 2 -> float64 (float32 in and out,
                             each spectrum value rounded once to float32).  The
                             spectra's rounding is amplified by kappa
                             (spt_plan_info) in the product, so long blocks and
                             two-sided plans can exceed 1e-6 with float32 FFTs.
                             The persistent executor always runs float32 FFTs. */
} spt_params;

typedef struct spt_plan* spt_plan_t;

/* Launch choices of a plan's staged execute (none changes what is computed;
 * the banded-product and FFT-batching choices give the same bits, the parity
 * split of a transform rounds differently).  Zero-filled: the defaults. */
enum {
  SPT_PRODUCT_DEFAULT = 0,  /* split-bf16 product: windowed, chunked where the
                               windows do not fit LDS                            */
  SPT_PRODUCT_TILE = 1,     /* per row tile, spectra read from memory             */
  SPT_PRODUCT_WINDOW = 2,   /* the default's choice, asked for explicitly         */
  SPT_PRODUCT_CHUNKED = 3,  /* windows through LDS in chunks of 32 columns        */
  SPT_PRODUCT_WINDOW_2W = 4,  /* windowed over 64 right-hand sides, two waves per row
                                 tile (32 right-hand sides each, 8 waves)         */
  SPT_TUNE_DEFAULT = 0, SPT_TUNE_OFF = 1, SPT_TUNE_ON = 2,
  SPT_FFT_EIGHT = 3         /* fft_half: split by output residue mod 8 instead      */
};
typedef struct {
  int32_t product;     /* SPT_PRODUCT_*                                          */
  int32_t window_rhs;  /* right-hand sides per windowed-product workgroup: 0 (64
                          when two such workgroups fit a CU's LDS, else 32), 32, 64 */
  int32_t fft_batch;   /* most right-hand sides per workgroup of a short block's
                          fused FFT: 0 (4), 1, 2 or 4                            */
  int32_t fft_half;    /* SPT_TUNE_* or SPT_FFT_EIGHT: split transforms of at least
                          4096 points by output parity into two workgroups (ON,
                          and DEFAULT), or the real transform by output residue
                          mod 8 into five (SPT_FFT_EIGHT, when 4 divides P),
                          or not at all (OFF: only where the whole transform
                          fits one workgroup)                                   */
  int32_t inv_four;    /* SPT_TUNE_*: transposed product, four-step inverse
                          transforms also for blocks that fit one workgroup (ON) */
} spt_tuning;

/* Plan summary (spt_plan_query). */
typedef struct {
  int32_t family, mode, n_blocks, tail;  /* tail = columns multiplied directly  */
  int64_t N;
  double eps1, eps2, zeta;
  int32_t precomputed;
  int32_t max_band;                      /* widest per-row band (half spectrum) */
  int64_t nnz;                           /* kept half-spectrum entries, all blocks */
  int64_t stored;                        /* stored (tile-padded) entries        */
  int64_t matrix_bytes_f64;              /* device bytes read per execute (F64) */
  int64_t matrix_bytes_f32;              /* same for F32 / SPLIT_BF16           */
  double max_abs[16];                    /* max |A_e W F| per block (first 16)  */
  double kappa;                          /* max over blocks of rms(w) rms(1/w on the
                                            retained columns): the factor by which
                                            rounding of the half spectra grows in
                                            the product (sec. 2.2 error growth)  */
  int64_t nnz_blk[16];                   /* kept half-spectrum entries per block  */
  int64_t window_lds;                    /* SPLIT_BF16 product: LDS bytes of a workgroup
                                            of the windowed kernel, 0 when the plan
                                            uses the per-tile kernel              */
  int64_t window_cols;                   /* sum over groups of 4 row tiles and over
                                            blocks of the spectrum columns that the
                                            windowed kernel stages in LDS          */
  int64_t window_chunked;                /* 1: the windows are too wide for LDS and
                                            pass through it in chunks of 32 columns
                                            (window_lds is then the chunked
                                            kernel's)                              */
  int64_t transposed_segment;            /* row tiles per segment of the transposed
                                            product (8, more for nearly dense plans,
                                            whose partial sums would otherwise need
                                            more than 4x the half spectra's memory) */
  int64_t reduced_fft_f64;               /* 1: the F32 and SPLIT_BF16 paths' FFTs run
                                            in float64 arithmetic (spt_params.reduced_fft) */
  int64_t is_complex;                    /* 1: complex matrix, data and spectra      */
  double reduced_fft_f32_err;            /* the measurement behind an automatic choice
                                            (spt_params.reduced_fft): relative error
                                            with float32 FFTs against the float64 path
                                            (or the same path with float64 FFTs); 0
                                            when not measured                        */
} spt_plan_info;

/* Create a plan for the N x N matrix of `family` with threshold eps (= eps1 of
 * sec. 2.2: entries of A_e W F with |.| <= eps * max|.| are dropped, and
 * 1/I0(zeta) = eps).  Host only: computes zeta, s_i and the block partition.
 * N >= 2, 0 < eps < eps2 < 1.  p may be NULL (all defaults). */
spt_status spt_plan_create(spt_plan_t* out, int32_t family, const spt_params* p,
                           int64_t N, double eps);

/* Block geometry (host, valid after create): for block i, its FFT length L[i],
 * the degree of its column 0 (m_offset[i]) and its retained columns
 * [c_lo[i], c_hi[i]).  Arrays hold `cap` entries; *n_blocks gets the count. */
spt_status spt_plan_blocks(spt_plan_t plan, int32_t* L, int32_t* m_offset, int32_t* c_lo,
                           int32_t* c_hi, int32_t cap, int32_t* n_blocks);

/* Precomputation on `stream` (nodes, weights, A_e W F by panels, threshold,
 * banded tiles).  Synchronises `stream` before returning.  May be called
 * again (it rebuilds the compressed form). */
spt_status spt_precompute(spt_plan_t plan, void* stream);

/* Y = A X^T for nrhs right-hand sides: Y[r*N + j] = sum_m A[j,m] X[r*N + m].
 * X, Y: device, nrhs x N, float64 for SPT_F64 and float32 otherwise, must not
 * overlap.  nrhs >= 1.  The precision must have been prepared.
 * Asynchronous on `stream`.  The plan keeps one workspace per stream (up to 8
 * streams; a ninth takes over the oldest after a device synchronisation), so
 * executes of one plan on different streams may run at the same time; the
 * host calls on one plan must not be made from several threads at once. */
spt_status spt_execute(spt_plan_t plan, const void* X, void* Y, int64_t nrhs, int32_t prec,
                       void* stream);

/* spt_execute for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * arguments, kernels and results, with the workspace in a static device array
 * of SPT_NOALLOC_MAX_BYTES per device (resident from the library's load until
 * the process ends) instead of the plan's workspace.  Calls no hipMalloc,
 * hipFree or allocating routine.  Every call on a device shares that device's
 * array: calls that overlap on one device (two streams, two threads) race and
 * must be ordered by the caller; nothing in the array needs clearing between
 * calls (each call writes all it reads).  SPT_E_INVALID_ARG when the workspace
 * of nrhs right-hand sides (complex float64 half spectra of every block, or the
 * split-bf16 pieces) exceeds the array; SPT_E_UNSUPPORTED for plans with the
 * persistent executor or with a block whose forward FFT does not run fused
 * (half length above 16384, or above 10240 and odd: such blocks go by work
 * lists). */
#define SPT_NOALLOC_MAX_BYTES (32u << 20)
spt_status spt_execute_noalloc(spt_plan_t plan, const void* X, void* Y, int64_t nrhs, int32_t prec,
                               void* stream);

/* Transposed product (Alg. 2 / block Alg. 4): Y[r*N + m] = sum_j A[j,m] X[r*N + j].
 * Same arguments and rules as spt_execute; F64 or F32 (SPT_E_UNSUPPORTED for
 * split-bf16).  Blocks with an FFT half-length above 10240 take a four-step
 * inverse transform (the workspace then holds P complex values per right-hand
 * side for each such block). */
spt_status spt_execute_transposed(spt_plan_t plan, const void* X, void* Y, int64_t nrhs,
                                  int32_t prec, void* stream);

/* Execute `count` plans (any families and sizes, each precomputed with `prec`)
 * on `stream`: Y[i] = A_i X[i]^T with nrhs[i] right-hand sides.  X, Y, nrhs
 * are host arrays of `count` entries holding device pointers / counts.  Every
 * 64 plans run together: with the executor of plans[0] PERSISTENT, as one
 * launch of the persistent executor; otherwise as the FFT items of every plan
 * in two launches, then the banded products (split-bf16: one launch for the
 * plans with windows, one for the others; a batch of a single plan runs that
 * plan's own launches, as spt_execute).  The
 * first call for a set of plans and sizes builds the work lists (host work and
 * a stream synchronisation), later calls reuse them.  A plan may appear once
 * per batch.  Batches of the same plans on different streams use each plan's
 * workspace of that stream and their own work lists, and may overlap. */
spt_status spt_execute_batched(const spt_plan_t* plans, const void* const* X, void* const* Y,
                               const int64_t* nrhs, int32_t count, int32_t prec, void* stream);

/* Device memory of the library (compressed blocks, tables, workspaces, work
 * lists).  With a hook pair set, every later allocation calls
 * alloc(bytes, stream, ctx), which returns device memory of the current device
 * aligned to 256 bytes, or NULL when it has none (the call that needed it then
 * returns SPT_E_OOM and leaves its plan valid: a later call allocates again);
 * stream is the stream of the call that allocates (NULL for the null stream).
 * Each buffer is freed through the hook that allocated it, with the same
 * stream and ctx, once no launch uses it (plans free theirs in
 * spt_plan_destroy, after a device synchronisation).  Both NULL restores
 * hipMalloc / hipFree for later allocations; giving one hook alone is
 * SPT_E_INVALID_ARG.  Process-wide; buffers allocated before the call keep
 * their allocator.  Lets a framework's caching allocator (PyTorch's, say)
 * own the memory. */
typedef void* (*spt_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*spt_free_fn)(void* ptr, void* stream, void* ctx);
spt_status spt_set_allocator(spt_alloc_fn alloc, spt_free_fn free_, void* ctx);

/* Bound of a dependency wait of the persistent executor (SPT_EXECUTOR_PERSISTENT)
 * for this plan's launches and the batches it leads (plans[0]), in ticks of
 * the 100 MHz wall clock; 0 restores the default of 1e8 (1 s).  A wait that
 * reaches the bound gives up: the launch drains, the outputs that waited hold
 * NaN, and the next persistent execute on the same plans and sizes returns
 * SPT_E_HIP without running (the call after it runs normally).  For tests of
 * that path; waits end without it, since items only wait for items taken
 * before them.  Synchronises the device when contexts exist. */
spt_status spt_plan_set_exec_wait(spt_plan_t plan, int64_t ticks);

/* Set / read a plan's launch choices (host struct).  Set after spt_precompute,
 * the device-side descriptions are rebuilt (a device synchronisation first);
 * before, spt_precompute applies them.  SPT_E_INVALID_ARG for unknown values. */
spt_status spt_plan_set_tuning(spt_plan_t plan, const spt_tuning* t);
spt_status spt_plan_get_tuning(spt_plan_t plan, spt_tuning* t);

/* Autotuner: time spt_execute of nrhs right-hand sides (x ~ N(0,1), a fixed
 * seed) in precision prec on `stream` with HIP events for every launch choice
 * that applies to the plan (split-bf16: the four products and both window
 * widths; every precision: FFT batching 1, 2, 4 and, where a block qualifies,
 * the parity split on and off and the eight-way split): two sweeps over the
 * choices, each the median of 20 executes after 3 warm-up executes, the
 * smaller of a choice's two medians kept, and keep the fastest
 * (spt_plan_set_tuning).  cache_path (may be
 * NULL): a JSON file of earlier results keyed by family, Jacobi parameters,
 * ceil(log2 N), ceil(log2 nrhs) and precision; a key found there is applied
 * without timing, a new result is added to the file.  *chosen (may be NULL)
 * gets the choice, *us (may be NULL) its time per execute in microseconds (0
 * when taken from the cache).  Complex plans have nothing to tune (their
 * current choice is returned).  Allocates the right-hand sides and outputs
 * through the library's allocator; synchronises the device. */
spt_status spt_autotune(spt_plan_t plan, int64_t nrhs, int32_t prec, void* stream,
                        const char* cache_path, spt_tuning* chosen, double* us);

/* Plan summary; info is a host struct filled by the call. */
spt_status spt_plan_query(spt_plan_t plan, spt_plan_info* info);

/* Copy the N nodes (after spt_precompute) to the host array `out`. */
spt_status spt_plan_nodes(spt_plan_t plan, double* out);

/* Copy one dense row block of the compressed matrix of block `blk` (after
 * spt_precompute) to the host: out[(row - row0) * (L/2+1) + k] for rows
 * [row0, row0 + nrows) and k in [0, L/2], as interleaved (re, im) float64
 * pairs, entries that are not stored read as zero.  The values are the stored
 * ones, i.e. already multiplied by c_k (1 at k = 0 and k = L/2, else 2). */
spt_status spt_plan_compressed_rows(spt_plan_t plan, int32_t blk, int64_t row0, int64_t nrows,
                                    double* out);

/* Kernel timing with HIP events (for measurement): between spt_profile_begin
 * and spt_profile_end every execute records an event pair on its stream around
 * each stage below; spt_profile_end synchronises those events and returns,
 * per stage, the summed milliseconds and the number of timed launches
 * (host arrays of SPT_NUM_STAGES entries).  Process-wide; not thread-safe. */
enum {
  SPT_STAGE_FFT = 0,        /* extend, divide by the window, F* (all blocks)     */
  SPT_STAGE_SPMM = 1,       /* banded product of every block and the tail       */
  SPT_STAGE_SPMM_T = 2,     /* transposed banded product (all blocks)           */
  SPT_STAGE_INV_FFT = 3,    /* F*, divide by the window, discard the extras     */
  SPT_STAGE_TAIL_T = 4,     /* transposed direct tail                           */
  SPT_STAGE_EXEC = 5,       /* persistent executor launch (the whole stage)     */
  SPT_NUM_STAGES = 6
};
spt_status spt_profile_begin(void);
spt_status spt_profile_end(double* ms, int64_t* launches);

/* Destroy a plan (NULL is allowed).  Waits for the device to finish. */
spt_status spt_plan_destroy(spt_plan_t plan);

/* Message of the last failed call on this thread ("" if none). */
const char* spt_last_error(void);

/* Library version string. */
const char* spt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPT_H */
