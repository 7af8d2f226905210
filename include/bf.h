/*
 * bf.h -- C ABI of the MI355X (gfx950) randomized butterfly library.
 *
 * The library builds the hybrid butterfly factorization of an m x n complex
 * operator A that it sees only through products with A and A^H (Liu, Xing,
 * Guo, Michielssen, Ghysels, Li, "Butterfly factorization via randomized
 * matrix-vector multiplications", arXiv:2002.03400, Alg. 2), and applies the
 * result.  Output form (Alg. 2 output, eq. hybrid_butterfly_mat):
 *
 *     A ~ (U^L R^{L-1} ... R^{l_m}) B^{l_m} (W^{l_m} ... W^1 V^0),
 *     l_m = floor(L/2).
 *
 * Conventions shared by every call:
 *   - complex numbers are interleaved (re, im); bf_c64 = two floats,
 *     bf_c128 = two doubles;
 *   - matrices are column-major with an explicit leading dimension (ld >=
 *     rows); all device pointers are HIP device (HBM) addresses;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     calls enqueue work on it and return; results are valid once the stream
 *     has reached the call;
 *   - every call returns BF_OK (0) or a negative error code and never aborts;
 *     on failure nothing is leaked and output handles are left untouched;
 *   - transposes of the paper are conjugate transposes (Sec. 2.1 extends the
 *     real algorithms to complex matrices): "rmatvec" is Y = A^H X.
 */
#ifndef BF_H
#define BF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } bf_c64;
typedef struct { double re, im; } bf_c128;

enum {
  BF_OK = 0,
  BF_EINVAL = -1,     /* bad argument: sizes <= 0, tol not in (0,1), leaf < 1, NULL */
  BF_ENOMEM = -2,     /* device or pinned host allocation failed */
  BF_ECALLBACK = -3,  /* a black-box callback returned nonzero */
  BF_ERANK = -4,      /* rank estimate passed opts.max_rank, or a block exceeds the
                         kernels' size limits (BF_MAX_BLOCK_ROWS / _COLS) */
  BF_EHIP = -5,       /* a HIP runtime call failed */
  BF_ENOTSUP = -6     /* no usable GPU / wrong architecture */
};

/* Largest Z block the batched QR and least-squares kernels accept (rows x
 * columns).  Blocks whose working set fits in the 160 KB LDS are factored
 * there; larger ones in device scratch (at most 1 GiB per launch, blocks
 * processed in as many launches as that takes). */
#define BF_MAX_BLOCK_ROWS 2048
#define BF_MAX_BLOCK_COLS 2048

/*
 * Black-box product (Alg. 2, input: products of A and of A^H with any block
 * of columns the algorithm chooses).  Writes Y = op(A) X on
 * `stream`, op = A for the matvec callback (X has n rows, Y has m rows) and
 * op = A^H for the rmatvec callback (X has m rows, Y has n rows).
 *
 *   seg == NULL : plain product of the ncols columns of X.
 *   seg != NULL : structured samples of Sec. 4.1.  `seg` is a HOST array of
 *                 nseg+1 nondecreasing row offsets within the rows of X;
 *                 group g is the row range [seg[g], seg[g+1]).  Y has
 *                 nseg*ncols columns and its columns [g*ncols, (g+1)*ncols)
 *                 receive op(A)(:, seg_g) * X(seg_g, :) -- the product with
 *                 the random matrix that is zero outside node g.  Rows of X
 *                 outside [seg[0], seg[nseg]) are not used: a level's nodes
 *                 may come in several calls (see bf_opts.work_bytes).
 *
 * X and Y are device buffers owned by the library for the duration of the
 * call; the callback must not keep them, nor write X.  Return 0 on success; any nonzero
 * value aborts the construction with BF_ECALLBACK.
 */
typedef int (*bf_op_fn)(void* user, const bf_c64* X, int64_t ldx, int64_t ncols,
                        bf_c64* Y, int64_t ldy, const int64_t* seg, int32_t nseg,
                        void* stream);

/* A black box with both products (built-in operators fill this in). */
typedef struct {
  bf_op_fn matvec;
  bf_op_fn rmatvec;
  void* user;
  int64_t m, n;
} bf_operator;

/* Knobs of Alg. 2.  Pass NULL for the defaults p = 2, r0 = 4 (the values of
   Sec. 6.1 and 6.2), seed = 0, no rank cap, 8 GiB of sweep workspace. */
typedef struct {
  int32_t p;          /* over-sampling (Alg. 1 input), >= 0 */
  int32_t r0;         /* initial rank guess of the adaptive loops, >= 1 */
  int32_t max_rank;   /* 0 = none; else BF_ERANK when a rank estimate passes it */
  int32_t flags;      /* BF_OPT_* bits, or 0 */
  uint64_t seed;      /* key of the counter-based random matrices */
  int64_t work_bytes; /* device bytes a sweep level's samples may occupy at once
                         (black-box output and partial-factor products); the
                         level's samples are processed in groups under this
                         bound (at least one sample per group).  0 = 8 GiB.
                         Only the summation order inside black-box products
                         can change with it. */
  /* Optional progress report: called on the host, from the thread that runs
     the construction, after each adaptive leaf-loop iteration and each sweep
     level, with phase BF_PHASE_* and the iteration (leaf loops, from 1) or
     level.  The level's ranks are known then (its samples have been
     factored).  NULL = none. */
  void (*progress)(void* user, int32_t phase, int32_t level);
  void* progress_user;
  /* With BF_OPT_CENTER_LEVEL in flags: the level l_m of the centre factor B
     (eq. hybrid_butterfly_mat), in [0, L]; negative values count from L + 1
     (-1 is L).  0 builds the column-wise factorization of Sec. 3.3.1
     (E^0 = B^0 V^0), L the row-wise one of Sec. 3.3.2 (F^L = U^L B^L); both
     need far more black-box columns and partial products than the hybrid
     (an R level l has 2^(L-l) samples, a W level 2^l).  With l_m = L the
     centre blocks use the leaf column bases directly and the last progress
     report is (BF_PHASE_R, L).  Default l_m = floor(L/2) (Sec. 3.3.3).
     bf_import always assumes the default. */
  int32_t center_level;
  int32_t reserved;   /* 0 */
} bf_opts;

/* BF_OPT_CENTER_LEVEL: use center_level.
 * BF_OPT_SEQUENTIAL_LEAF: one black-box call per pass of the adaptive leaf
 *   loops.  By default consecutive passes (each with its own fixed random
 *   block) share one call while their widths add up to at most 80 columns,
 *   which returns the same products in fewer calls; when the loop stops
 *   before a merged pass, that pass's columns are wasted (and counted in
 *   bf_info's column totals).
 * BF_OPT_SEQUENTIAL_SWEEP: one black-box call per sweep level.  By default,
 *   for the built-in operators that evaluate every kernel entry once per call
 *   (bf_op_segkernel, bf_op_helmholtz3d, bf_op_fio, bf_op_dense) and the
 *   default centre level, a W or R level whose samples leave room in one
 *   80-column tile also draws the next level's samples (as wide as that room,
 *   the next level's exact widths needing this level's ranks; not from the
 *   first level when the leaf bases have full rank) and makes one call over
 *   the next level's segments for both: the next level's
 *   products are those of its own call bit for bit, this level's are the
 *   sums of the halves over each node's two children (one more rounding).
 *   A guess that proves too small costs the next level its own call; the
 *   drawn columns are counted in bf_info's column totals either way.
 * BF_OPT_ONE_STREAM: run the whole construction on `stream` from the calling
 *   thread.  By default, for the built-in operators (and compositions of
 *   them) with no progress callback and outside cross-request solve rounds,
 *   the row side of Alg. 2 (leaf V loop, W levels 1..l_m) runs on a second
 *   stream driven by a second host thread while the calling thread runs the
 *   column side (leaf U loop, R levels L-1..l_m+1); the two meet at the
 *   centre level.  The sides enqueue the same work either way, so the factors
 *   are the same bit for bit; each side's samples count against work_bytes
 *   separately, so up to twice that may be in use at once.  The second
 *   stream waits for the work enqueued on `stream` before the call, and
 *   `stream` waits for the second stream before the centre level. */
enum {
  BF_OPT_CENTER_LEVEL = 1,
  BF_OPT_SEQUENTIAL_LEAF = 2,
  BF_OPT_SEQUENTIAL_SWEEP = 4,
  BF_OPT_ONE_STREAM = 8
};

enum { BF_PHASE_LEAF_V = 0, BF_PHASE_LEAF_U = 1, BF_PHASE_W = 2, BF_PHASE_R = 3 };

typedef struct bf_factors bf_factors;

/*
 * Device-memory provider of a call, e.g. a framework's caching allocator
 * (the Python binding passes one backed by torch's).  alloc returns `bytes`
 * of device memory on the current device for use in stream order on `stream`
 * (NULL on failure: the call then fails with BF_ENOMEM); free returns a block
 * once the work enqueued on `stream` before the call no longer needs it
 * (stream-ordered, like hipFreeAsync).  With an allocator, every device block
 * the call needs comes from it: sample, product and solver workspace, and for
 * bf_construct / bf_import the factor storage, which goes back to it at
 * bf_free, so ctx and both functions must stay valid until every handle built
 * with them is freed.  Blocks from an allocator are never kept by the library.
 * Not covered: the private buffers of captured apply graphs
 * (bf_set_apply_graph_cols) and pinned host staging.  NULL = the library's
 * own stream-ordered pool, with device blocks kept for reuse across calls.
 */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
} bf_alloc;

/*
 * Alg. 2: adaptive randomized hybrid butterfly construction.
 *   matvec, rmatvec, user : the black box (see bf_op_fn); both required.
 *   m, n                  : operator size (rows = targets T, cols = sources S).
 *   tol                   : truncation tolerance eps of Alg. 1, in (0, 1);
 *                           read as the relative Frobenius tail of each
 *                           sample, ||R[k:,k:]||_F <= eps ||Y||_F.
 *   leaf                  : leaf size n0 of the bisection trees (Sec. 3.1);
 *                           L is the smallest level count with
 *                           ceil(max(m,n)/2^L) <= leaf.
 *   opts                  : NULL or knobs above.
 *   alloc                 : NULL or the device-memory provider (bf_alloc).
 *   stream                : all device work and callbacks use this stream.
 *   out                   : receives the factor handle (owned by the caller,
 *                           release with bf_free).
 * The random matrices are drawn in complex64 from Philox4x64-10 keyed by
 * (seed, phase, level, node, row, col); black-box products are complex64;
 * every pivoted QR and least-squares solve runs in FP64 on the device.
 * Blocks on the host: syncs once per adaptive iteration and per level.
 */
int bf_construct(bf_op_fn matvec, bf_op_fn rmatvec, void* user, int64_t m, int64_t n,
                 double tol, int64_t leaf, const bf_opts* opts, const bf_alloc* alloc,
                 void* stream, bf_factors** out);

/*
 * Apply the factorization (eq. hybrid_butterfly_mat, right to left):
 *   trans = 0 : Y = F X,   X is n x ncols (ldx >= n), Y is m x ncols (ldy >= m)
 *   trans = 1 : Y = F^H X, X is m x ncols,            Y is n x ncols
 * complex64 data (arithmetic: bf_set_apply_precision).  X, Y are caller-owned device buffers
 * and must not overlap.  alloc: NULL or the provider of the intermediates
 * (bf_alloc).  Reentrant across streams for one handle.
 */
int bf_apply(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
             bf_c64* Y, int64_t ldy, const bf_alloc* alloc, void* stream);

/*
 * bf_apply without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, kernels and results as bf_apply
 * (launched stage by stage, never through a cached graph, never profiled).
 * The intermediates live in a fixed scratch array of
 * bf_apply_noalloc_scratch_bytes() bytes (64 MiB) per device, which the
 * library holds on every device it runs on until the process ends.  A call is
 * accepted when the stage-by-stage apply's two ping-pong intermediates fit
 * (2 x (largest level rank sum) x ncols complex64 values); it then runs like
 * bf_apply (fused stages for up to 4 columns when their larger intermediate
 * also fits, else stage by stage).  Larger requests return BF_EINVAL
 * (nothing is launched).  Every call on a device uses that
 * device's one array: calls that overlap on one GPU (other streams, other
 * threads) race and give wrong results, so callers serialize them.  F must
 * live on the current device.  The first call on a device looks up the
 * array's address (no allocation).
 */
int bf_apply_noalloc(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx,
                     int64_t ncols, bf_c64* Y, int64_t ldy, void* stream);
int64_t bf_apply_noalloc_scratch_bytes(void);

/* Applies of at most max_cols columns (0 = off, the default) run their L+3
 * stage launches as one captured HIP graph: bf_apply copies X into a private
 * buffer, launches the graph and copies the result out (two device copies
 * instead of L+2 launch gaps, which bound few-column applies at n <= 65536).
 * Graphs are cached per direction, column count, apply precision and stream
 * (at most 16 per factorization; the first call of a key captures it, beyond
 * 16 keys bf_apply launches the stages directly) and freed with the factors.
 * Same kernels, same results.  Not to be called while applies of F run. */
int bf_set_apply_graph_cols(bf_factors* F, int64_t max_cols);

/* Applies of 1 to 4 columns may run fused: consecutive stages share one
 * launch, each workgroup taking a group of blocks that depend only on each
 * other (about 4 launches instead of L + 3 at L = 10; planned only where a
 * launch keeps at least 256 groups and its stages are small enough to be
 * bound by latency; the autotuner then picks fused or staged, same bits).
 * enable = 0 runs every stage as its own launch (the path used above 4
 * columns).  Default 1.  Not synchronized with applies in flight on F. */
int bf_set_apply_fusion(bf_factors* F, int enable);

/* Summary of a factorization. */
typedef struct {
  int64_t m, n;
  int32_t L, lm;
  int32_t max_rank;          /* over every block of every level */
  int32_t v_iters, u_iters;  /* passes of the two adaptive leaf loops */
  int32_t apply_graphs;      /* captured apply graphs held (bf_set_apply_graph_cols) */
  int64_t matvec_cols;       /* black-box columns used: products with A ... */
  int64_t rmatvec_cols;      /* ... and with A^H (structured samples count s each) */
  int64_t factor_entries;    /* complex entries stored over all factors */
  int64_t device_bytes;      /* device memory held by the handle */
  int32_t fused_launches;    /* launches of a fused 1-4 column apply (0: every stage
                                is its own launch, L + 3 of them) */
  int32_t merged_levels;     /* sweep levels whose products came from the previous
                                level's black-box call (BF_OPT_SEQUENTIAL_SWEEP) */
  int32_t merge_misses;      /* sweep levels drawn ahead whose guessed width proved
                                too small (they made their own call) */
  int32_t reserved;
} bf_info;
int bf_stats(const bf_factors* F, bf_info* info);

/*
 * Ranks of every block.  kU receives (L - lm + 1) * 2^L ints: level l in
 * lm..L, block (l, i, j) at [(l - lm) * 2^L + i * 2^(L-l) + j].  kV receives
 * (lm + 1) * 2^L ints: level l in 0..lm at [l * 2^L + i * 2^(L-l) + j].
 * Host buffers; either may be NULL.
 */
int bf_ranks(const bf_factors* F, int32_t* kU, int32_t* kV);

/*
 * Factor data exchange in FP64 (host buffers).  Canonical order, each block
 * column-major with ld = its row count:
 *   U_{L,i} (i = 0..2^L-1), then R^{l} for l = L-1 down to lm (blocks (i, j)
 *   i-major), then B (i, j), then W^{l} for l = lm down to 1, then V_{0,j}.
 * Shapes follow from the ranks (bf_ranks layout): U_{L,i}: m_i x kU(L,i,0);
 * R_{l,i,j}: (kU(l+1,2i,j>>1) + kU(l+1,2i+1,j>>1)) x kU(l,i,j);
 * B_{i,j}: kU(lm,i,j) x kV(lm,i,j);
 * W_{l,i,j}: (kV(l-1,i>>1,2j) + kV(l-1,i>>1,2j+1)) x kV(l,i,j);
 * V_{0,j}: n_j x kV(0,0,j).
 * bf_export writes `count` entries (query with data == NULL to get count).
 * bf_import builds a handle from ranks + data (used for exact-butterfly black
 * boxes and for applying externally built factors); alloc as for bf_construct.
 */
int bf_export(const bf_factors* F, bf_c128* data, int64_t* count);
int bf_import(int64_t m, int64_t n, int64_t leaf, const int32_t* kU, const int32_t* kV,
              const bf_c128* data, int64_t count, const bf_alloc* alloc, void* stream,
              bf_factors** out);

/* Release a handle.  Its device blocks are reused only after the work
 * enqueued on `stream` before this call has finished; with stream NULL the
 * call first waits for all work on the handle's device (the null stream does
 * not order non-blocking streams).  Blocks from a caller's bf_alloc go back to
 * it; the library's own are kept for later requests on the same device (up to
 * 16 GB per device), as is the pinned host memory of descriptor uploads;
 * bf_release_cached_memory gives both back. */
int bf_free(bf_factors* F, void* stream);

/* Return every device block and pinned host block the library keeps for
 * reuse: waits for the work that last used them, frees them and trims each
 * device's stream-ordered memory pool to what is still allocated, so the
 * memory is available to other allocators again.  Live factor handles,
 * operators and servers are unaffected.  Must not overlap with other calls
 * into the library (it synchronizes every device it has used). */
int bf_release_cached_memory(void);

/* Text for an error code (static storage). */
const char* bf_strerror(int code);

/* Detail message of the calling thread's last failed call (thread-local storage,
   valid until that thread's next failing call). */
const char* bf_last_error(void);

/* ---------------------------------------------------------------------------
 * Request engine (serving): constructions and applies of many requests run
 * concurrently on `slots` device streams, each driven by a host worker
 * thread.  A request is admitted when a slot is idle and its estimated device
 * footprint fits under `hbm_budget` next to the requests in flight (first fit
 * in arrival order; a request passed over 8 times holds back later ones until
 * it fits; a request larger than the budget runs when the device is otherwise
 * idle).  An apply waits for the construction it references.  Factors stay on
 * the device until their ticket is released.  Results are independent of the
 * mix: every random matrix is keyed by its own request's seed, and every
 * reduction has a fixed order.  The calls are thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct bf_server bf_server;
typedef struct {
  int32_t slots;        /* concurrent requests (streams); 0 = 4 */
  int32_t batch_cols;   /* 0: every apply is its own product.  > 0: continuous
                           batching -- a slot that admits an apply also takes the
                           queued applies against the same factors and direction,
                           up to this many columns in all, gathers their columns
                           into one block, applies once and scatters the result
                           (one launch sequence instead of one per request).
                           Merged results are those of the merged product: the
                           same accuracy, but the arithmetic follows the merged
                           width (a 1-column apply alone runs on the vector
                           ALUs, merged with 4+ others on the matrix cores), so
                           they can differ from a lone apply in the last bits. */
  int64_t hbm_budget;   /* bytes; 0 = 64 GiB */
  const bf_alloc* alloc;  /* NULL or the device-memory provider of every request
                             (bf_alloc; copied at creation, must outlive the
                             server and every factor it holds) */
  int32_t solve_rounds; /* 0: every construction launches its own level solves.
                           1: cross-request solve rounds -- the batched
                           truncated QRs (Alg. 1 step 3) and centre-block least
                           squares (Sec. 4.4) that in-flight constructions reach
                           within a short window (60 us, or until every
                           construction in flight has joined) run as one
                           persistent launch over a device work list of
                           (request, block) items, replayed from a captured
                           HIP graph (one per LDS size class); blocks too large
                           for the LDS keep their own launches.  Each block runs
                           the code of its own launch: results are bitwise
                           those without rounds. */
  int32_t max_constructs; /* 0: every slot may run a construction.  > 0: at most
                           this many constructions run at once; further ones
                           wait in the queue while applies still take the idle
                           slots.  Constructions that share the device each take
                           proportionally longer, so a cap below `slots` trades
                           some throughput for tail latency under light load
                           (n = 65536, 4 slots, Poisson arrivals at half the
                           capacity: p99 359 ms uncapped, 268 ms with at most 2
                           constructions; at full load the cap costs 4% of the
                           throughput and the queue grows). */
} bf_server_opts;
typedef struct {
  int32_t status;       /* BF_OK or the request's error code */
  int32_t batch;        /* applies merged into this request's product (1 = alone) */
  int64_t arrival_ns;   /* submit, start, completion: ns since server creation */
  int64_t start_ns;
  int64_t finish_ns;
  int64_t footprint;    /* device bytes reserved for admission */
} bf_request_info;
int bf_server_create(const bf_server_opts* opts, bf_server** out);
/* Finishes every request that can still run, then frees all resident factors. */
int bf_server_destroy(bf_server* S);
/* Queue a construction; the operator (its callbacks and user data) must stay
   valid until the request completes.  Writes the request's ticket.  With
   more than one slot the engine runs every construction on its slot's one
   stream (it adds BF_OPT_ONE_STREAM to opts): the slots already overlap
   requests. */
int bf_server_submit_construct(bf_server* S, const bf_operator* op, double tol, int64_t leaf,
                               const bf_opts* opts, int64_t* ticket);
/* Queue Y = F X (trans 0) or F^H X (trans 1) with the factors of construction
   `factors_ticket`; X, Y are device buffers that must stay valid until done. */
int bf_server_submit_apply(bf_server* S, int64_t factors_ticket, int trans, const bf_c64* X,
                           int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy, int64_t* ticket);
/* Block until the request is done; returns its status (info may be NULL). */
int bf_server_wait(bf_server* S, int64_t ticket, bf_request_info* info);
/* Borrow the factors of a completed construction (valid until released). */
int bf_server_factors(bf_server* S, int64_t ticket, const bf_factors** F);
/* Forget a finished request; for a construction, free its factors (refused
   while applies that reference it are queued or running). */
int bf_server_release(bf_server* S, int64_t ticket);
/* Solve rounds launched so far and the blocks they held (0, 0 without
   solve_rounds). */
int bf_server_rounds(bf_server* S, int64_t* rounds, int64_t* items);

/* ---------------------------------------------------------------------------
 * Profiling: while enabled, every launch of the library's kernels is
 * bracketed by HIP events recorded on the stream the kernel runs on, and
 * its algorithmic work is counted (flops of the complex multiply-adds, bytes
 * of the operands the algorithm must move).  Per kernel class:
 * ------------------------------------------------------------------------ */
enum {
  BF_KC_MATFREE = 0,   /* black-box products of the built-in operators */
  BF_KC_APPLY = 1,     /* butterfly apply stages */
  BF_KC_CPQR = 2,      /* batched truncated pivoted QR */
  BF_KC_CHAIN = 3,     /* partial-factor products of the sweeps */
  BF_KC_LSQ = 4,       /* centre-block least squares */
  BF_KC_OTHER = 5,     /* random blocks, packing, reductions */
  BF_KC_COUNT = 6
};
typedef struct {
  int64_t launches;
  double ms;      /* summed event time of the launches */
  double flops;   /* algorithmic flops (complex MAC = 8) */
  double bytes;   /* algorithmic bytes */
} bf_kernel_stats;
/* Reset the counters and start recording (process-wide). */
int bf_profile_start(void);
/* Stop recording; waits for the recorded events and writes BF_KC_COUNT
   entries to `out` (HOST). */
int bf_profile_stop(bf_kernel_stats* out);

/* ---------------------------------------------------------------------------
 * Kernel-level entry points: the batched building blocks of Alg. 2 exposed
 * on their own so that each can be checked against a reference.  All buffers
 * are device buffers unless marked HOST.
 * ------------------------------------------------------------------------ */

/* Complex Gaussians of the random matrices of Alg. 2: out[r + c*rows] =
 * g(seed, tag, row0 + r, c) for r < rows, c < cols, in FP64, where
 * g = sqrt(-2 ln u0) (cos 2 pi u1 + i sin 2 pi u1) / sqrt(2),
 * u_q = ((o_q >> 12) + 1/2) 2^-52 and (o_0, o_1, ..) = Philox4x64-10 of
 * counter (row, col, tag, 0) under key (seed, 0) (Salmon et al., SC'11). */
int bf_gauss(uint64_t seed, uint64_t tag, int64_t row0, int64_t rows, int64_t cols,
             bf_c128* out, void* stream);

/* Alg. 1 step 3 on a batch: block b is M[b] x N[b] (HOST arrays), stored
 * column-major (ld = M[b]) at Z + zoff[b] (HOST offsets, in elements).  Its
 * truncated pivoted-QR basis Q_k (M[b] x k, ld = M[b]) is written at
 * Q + qoff[b] (room for M[b] x min(M[b], N[b]) entries) and k into
 * ranks[b] (HOST).  Rank rule: first k >= 1 with ||R[k:,k:]||_F <= tol ||Z||_F,
 * else min(M, N); 0 for an empty block.  Synchronizes `stream`. */
int bf_cpqr_batched(int32_t nblk, const int32_t* M, const int32_t* N, const bf_c128* Z,
                    const int64_t* zoff, double tol, bf_c128* Q, const int64_t* qoff,
                    int32_t* ranks, void* stream);

/* Centre blocks by least squares (Sec. 4.4, eq. Bij read from its argmin):
 * B_b = argmin ||C_b - B X_b||_F with C_b kU[b] x s[b] at C + coff[b],
 * X_b kV[b] x s[b] at X + xoff[b], B_b kU[b] x kV[b] at B + boff[b]
 * (column-major, ld = row count; HOST shape/offset arrays; s[b] >= kV[b];
 * kU, kV, s up to BF_MAX_BLOCK_COLS). */
int bf_lsq_batched(int32_t nblk, const int32_t* kU, const int32_t* kV, const int32_t* s,
                   const bf_c128* C, const int64_t* coff, const bf_c128* X, const int64_t* xoff,
                   bf_c128* B, const int64_t* boff, void* stream);

/* ---------------------------------------------------------------------------
 * Built-in black boxes.  Each fills a bf_operator whose callbacks run HIP
 * kernels on the stream they are given; release with bf_operator_destroy.
 * ------------------------------------------------------------------------ */

/* A_ij = exp(i k r_ij) / r_ij, r_ij = |x_i - y_j| (2D points), evaluated on the
 * fly: phase k r reduced in FP64, sin/cos and 1/r in FP32, complex64 products
 * with FP32 accumulation.  targets: m x 2 row-major doubles (host), sources:
 * n x 2 (host); copied to the device.  The kernel family of Sec. 3 on the
 * parallel-line geometry of Sec. 6.2. */
int bf_op_segkernel(const double* targets, int64_t m, const double* sources, int64_t n,
                    double k, bf_operator* out);

/* The same kernel on 3D points (eq. 3dkernel of Sec. 6.3, there between two
 * adjacent semi-spheres; written exp(i k r)/r here, k the wavenumber):
 * targets m x 3 and sources n x 3 row-major doubles (host), copied to the
 * device; same arithmetic as bf_op_segkernel.  Coincident points give
 * non-finite entries (the kernel is singular there): the point sets must be
 * disjoint. */
int bf_op_helmholtz3d(const double* targets, int64_t m, const double* sources, int64_t n,
                      double k, bf_operator* out);

/* A_jk = exp(2 pi i (x_j xi_k + c(x_j) |xi_k|)), x_j = j/n, xi_k = k - n/2,
 * c(x) = (2 + sin 2 pi x)/16: a 1D Fourier integral operator (Sec. 4.4.1,
 * "low-dimensional Fourier operators").  x_j xi_k is reduced modulo 1 exactly
 * in integers.  n even. */
int bf_op_fio(int64_t n, bf_operator* out);

/* Explicit matrix: A is a device m x n complex64 matrix with leading
 * dimension lda (>= m); the operator keeps the pointer, the caller keeps the
 * memory alive while the operator is used. */
int bf_op_dense(const bf_c64* A, int64_t m, int64_t n, int64_t lda, bf_operator* out);

/* A built factorization as a black box (category (ii) of Sec. 1: operators
 * applied in quasi-linear time).  Keeps a reference to F.  Structured
 * samples (seg != NULL) whose segments are consecutive nodes of one level of
 * the input-side tree (the source tree for matvec, the target tree for
 * rmatvec; what bf_construct passes) run the apply stages that keep the
 * segments apart once on X itself, for a whole level with split-BF16 applies
 * the next merging stages on per-node windows of the segments below each
 * node, and the rest on the block-diagonal expansion (up to 16 GiB of
 * intermediates at once); other segments are expanded first.  All give the product
 * the callback contract defines (bitwise the same for 5 or more columns). */
int bf_op_factors(const bf_factors* F, bf_operator* out);

/* Composition A = A1 A2 (A1: m x k, A2: k x n), e.g. the product of two
 * butterflies to be recompressed.  Keeps references to both. */
int bf_op_compose(const bf_operator* a1, const bf_operator* a2, bf_operator* out);

int bf_operator_destroy(bf_operator* op);

/* Arithmetic of the built-in matrix-free products (segment kernel, FIO,
 * dense).  Entries are FP32-accurate in both modes (FP64 phase reduction);
 * the complex multiply-adds run
 *   BF_PREC_FP64   : on the FP64 matrix cores, FP64 accumulation;
 *   BF_PREC_BF16X3 : on the BF16 matrix cores with every entry and input
 *                    split into three BF16 terms (products kept to 2^-24
 *                    relative; inputs exact in BF16, such as the random
 *                    blocks of the construction, need only their first
 *                    term), 32-term FP32 sums folded into FP64.  The BF16
 *                    matrix cores run beside the vector ALUs that evaluate the
 *                    entries, so this mode is the faster one.
 * Default: BF_PREC_BF16X3.  Returns BF_EINVAL for other operators or values. */
enum { BF_PREC_FP64 = 0, BF_PREC_BF16X3 = 1, BF_PREC_FP32 = 2 };
int bf_op_set_precision(bf_operator* op, int precision);

/* Launch-shape autotuner (on by default).  For each kernel family and shape
 * class it keeps the fastest of a few launch variants that give bitwise the
 * same results, timed on the first launch of the class (which then runs
 * every candidate four times on its stream -- once to warm caches, then three
 * interleaved timed rounds, keeping each candidate's fastest -- and
 * synchronizes it once; launches
 * under HIP graph capture and bf_apply_noalloc never time, they use the
 * table or the default rule):
 *   black-box column tile : 48, 64 or 80 columns, split-BF16 products of more
 *                           than 48 columns (class: operator kind, column
 *                           count, powers of two above the row count, inner
 *                           length and segment count);
 *   chain tile height     : 8, 16, 20, 24, 32, 40, 48 or 64 rows, at least the
 *                           launch's largest block (class: input type,
 *                           largest block, powers of two above the block and
 *                           column counts);
 *   CPQR workgroup        : 256 or 512 threads for blocks held in LDS (class:
 *                           input type, powers of two above the largest
 *                           block's rows and columns and the block count);
 *   few-column apply      : fused stages or one launch per stage, 1 to 4
 *                           columns (class: direction, columns, powers of two
 *                           above m and n, L, apply precision);
 *   few-column stage      : a block kernel (1, 2 or 4 row groups per load,
 *                           inputs in registers or LDS, and below 4096 blocks
 *                           one, two or four waves per block) or one 8-lane
 *                           group per row record, stages whose rows have at
 *                           most 96 terms and blocks at most 128 rows (class:
 *                           columns, 32-term chunks per row, powers of two
 *                           above the block count and rows); stages of more
 *                           than 64 MB are not timed (repeated launches would
 *                           find part of their factors in the last-level
 *                           cache) and take one row group per load with the
 *                           inputs in registers (1-2 columns) or LDS (4);
 *   matrix-core stage     : one workgroup per block and 64 columns, or one
 *                           wave per block and 1, 2, 4 ... or all of its
 *                           16-column tiles, blocks of 17 to 64 rows (class:
 *                           power of two above the column count, 16-row tiles,
 *                           powers of two above the block count and terms).
 * Without the tuner every family uses its rule (80-column tiles, the
 * smallest tile height, 256 threads, fused applies, one wave per block; for
 * matrix-core stages all tiles per wave from 4096 blocks, else one).  The table is
 * process-wide; the first lookup loads the file named by the environment
 * variable BF_TUNE_FILE or, if unset, tune_gfx950.tsv beside libbf.so (when
 * present).  bf_autotune_save writes the table (path NULL or "": that same
 * default file), bf_autotune_load merges a file into it, bf_autotune_clear
 * empties it, bf_autotune_entries counts its classes. */
int bf_set_autotune(int enable);
int bf_autotune_entries(int64_t* entries);
int bf_autotune_save(const char* path);
int bf_autotune_load(const char* path);
int bf_autotune_clear(void);

/* Arithmetic of bf_apply (and of the factors as a black box, bf_op_factors)
 * for F (eq. hybrid_butterfly_mat, complex64 data in both modes):
 *   BF_PREC_FP32   : FP32 multiply-adds and sums on the vector ALUs;
 *   BF_PREC_BF16X3 : (default) stages with 5 or more right-hand sides on the
 *                    BF16 matrix cores, factor entries and inputs split into
 *                    three BF16 terms (products kept to 2^-24 relative),
 *                    FP32 sums rounded once per 32-term matrix instruction
 *                    (faster than FP32 and about twice as accurate); 1 to 4
 *                    on the vector ALUs with FP32 sums, as in BF_PREC_FP32.
 * Not synchronized with applies in flight on F: set it before applying.
 * Returns BF_EINVAL for a null F or another value. */
int bf_set_apply_precision(bf_factors* F, int precision);

#ifdef __cplusplus
}
#endif
#endif /* BF_H */
