// Internal declarations shared by the HIP sources of libbf (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bf.h"

namespace bf {

// ---------------------------------------------------------------- errors --

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

#define BF_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::bf::Error(e_ == hipErrorOutOfMemory ? BF_ENOMEM : BF_EHIP,          \
                        std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define BF_CHECK(cond, code, msg)                    \
  do {                                               \
    if (!(cond)) throw ::bf::Error((code), (msg));   \
  } while (0)

void set_last_error(const std::string& msg);

// Host-side bounds validation of device accesses (enabled by the environment
// variable BF_VALIDATE=1): the library records its own live allocations and
// checks every descriptor's extent against them before a launch, so an
// indexing error surfaces as BF_EINVAL instead of a GPU memory fault.
bool validating();
void check_extent(const void* p, size_t bytes, const char* what);

// -------------------------------------------------------------- profiling --
// RAII bracket of one launch: records a start event now and a stop event at
// scope exit on the same stream, when profiling is enabled.
bool profiling();
struct ProfScope {
  int cls;
  hipStream_t s;
  double flops, bytes;
  hipEvent_t a = nullptr;
  ProfScope(int c, hipStream_t st, double fl, double by);
  ~ProfScope();
};

// ------------------------------------------------------- device buffers --
// Stream-ordered device memory (hipMallocAsync from the device's default pool,
// whose release threshold is raised at first use so freed memory is reused).

void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

// A caller's device-memory provider (bf_alloc).  While a UseAllocator is
// alive on a thread, every device block the thread allocates comes from it
// (recycled within an AllocScope like pool blocks) and goes back to it when
// freed, whenever that is (factor storage at bf_free); such blocks are never
// kept by the library.  A null bf_alloc leaves the library's own pool in use.
struct UserAlloc {
  void* ctx = nullptr;
  void* (*alloc)(void*, size_t, void*) = nullptr;
  void (*free)(void*, void*, void*) = nullptr;
};
class UseAllocator {
 public:
  explicit UseAllocator(const bf_alloc* a);
  // the same provider on another thread (nullptr: none)
  explicit UseAllocator(const UserAlloc* ua);
  ~UseAllocator();
  UseAllocator(const UseAllocator&) = delete;
  UseAllocator& operator=(const UseAllocator&) = delete;

 private:
  UserAlloc ua_{};
  const UserAlloc* prev_ = nullptr;
  bool set_ = false;
};

struct Staging;
// Recycling scope of one request.  While an AllocScope is alive on a thread,
// device blocks the thread allocates and frees on the scope's stream are kept
// and handed out again (best fit, at most twice the request, sizes rounded
// to 1/8 of their power of two) instead of going through the pool's
// allocation calls, whose host cost (tens of microseconds each) would
// otherwise sit between dependent launches; uploads share the scope's pinned
// staging.  Reuse is safe because every use of a block is ordered on the one
// stream.  The scope returns its free blocks to the pool when it ends (blocks
// still in use, such as factor storage, are freed to the pool by their
// owners).  A scope opened while one for the same stream is active on the
// thread joins it.
class AllocScope {
 public:
  explicit AllocScope(hipStream_t s);
  ~AllocScope();
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
  struct Cache;

 private:
  Cache* c_ = nullptr;
  bool owner_ = false;
};
// Pinned staging of the active scope on stream s of this thread, or nullptr.
// Its users reset it only after synchronizing s.
Staging* scope_staging(hipStream_t s);

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(size_t count, hipStream_t st) : n(count), s(st) {
    p = count ? static_cast<T*>(dev_alloc(count * sizeof(T), st)) : nullptr;
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { reset(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { reset(); }
  void reset() {
    if (p) dev_free(p, s);
    p = nullptr;
    n = 0;
  }
  T* release() { T* q = p; p = nullptr; n = 0; return q; }
};

// Pinned host staging for descriptor uploads: a bump allocator whose space is
// recycled only after the owning stream has been synchronized (reset()), so
// in-flight host-to-device copies never see their source overwritten.  Its
// blocks come from a process-wide set of pinned blocks and go back to it (with
// an event marking the end of their copies) when the staging grows or ends.
struct Staging {
  char* h = nullptr;
  size_t cap = 0, off = 0;
  hipStream_t last = nullptr;                  // stream of the latest copy out of h
  ~Staging();
  void* alloc(size_t bytes, hipStream_t s);   // may synchronize s to grow
  void reset() { off = 0; }                    // caller has synchronized the stream
};

template <typename T>
DevBuf<T> upload(const std::vector<T>& v, hipStream_t s, Staging& st) {
  DevBuf<T> d(v.size(), s);
  if (!v.empty()) {
    void* h = st.alloc(v.size() * sizeof(T), s);
    std::memcpy(h, v.data(), v.size() * sizeof(T));
    BF_HIP(hipMemcpyAsync(d.p, h, v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  return d;
}

// ---------------------------------------------------------------- kernels --

// Philox4x64-10 complex Gaussians for structured samples (Alg. 2, random
// matrix lines; Sec. 4.1).  Fills X (rows x ncols, ld = rows) in complex64:
// row r belongs to node g = the level-`level` node of a bisection tree over
// `rows` points; entry (r, c) = gauss(seed, tags[g], r, c) if c < widths[g],
// else 0.
void launch_gauss_samples(bf_c64* X, int64_t rows, int64_t ncols, int32_t level,
                          const uint64_t* tags_dev, const int32_t* widths_dev,
                          uint64_t seed, hipStream_t s);

// FP64 variant used by the self-test of the generator.
void launch_gauss_f64(bf_c128* X, int64_t rows, int64_t ncols, int64_t row0, uint64_t tag,
                      uint64_t seed, hipStream_t s);

// Batched small complex GEMM with up to two terms:
//   out[r, c] = sum_t sum_k op_t(F_t)[r, k] * in_t[k, c],   r < M, c < ncols,
// op = 0: F is M x K column-major (ld f_ld); op = 1: F^H with F K x M.
// Strided operands: element (row k, column c) of `in` is in[c * in_ld +
// k * in_rs] and output (r, c) is out[c * out_ld + r * out_rs]; column-major
// operands have a row stride of 1, the row-major intermediates of the sweeps
// a column stride of 1.
// (Row strides are sample widths or column counts, so 32 bits hold them; the
// descriptors stay at 40 / 112 bytes, millions of them per construction.)
struct GemmTerm {
  const bf_c128* F;
  const void* in;    // bf_c64* or bf_c128* (kernel template parameter)
  int64_t in_ld;
  int32_t f_ld;
  int32_t K;
  int32_t op;
  int32_t in_rs = 1;
};
struct GemmDesc {
  bf_c128* out;
  int64_t out_ld;
  int32_t M;
  int32_t ncols;
  int32_t nterm;
  int32_t out_rs = 1;
  GemmTerm t[2];
};
// in_c64: the inputs are complex64 (samples straight from the black box);
// max_M and max_Ksum bound every descriptor's M and summed terms' K.
void launch_chain_gemm(const GemmDesc* d_dev, int32_t ndesc, int32_t max_ncols, int32_t max_M,
                       int32_t max_Ksum, bool in_c64, hipStream_t s);

// Batched truncated column-pivoted QR (Alg. 1 step 3) on FP64.
struct QRDesc {
  const void* in;    // bf_c64* or bf_c128*; element (i, j) at in[j * in_ld + i * in_rs]
  bf_c128* q;        // M x min(M,N) capacity, ld = M; first k columns written
  int64_t in_ld;
  int32_t M;
  int32_t N;
  int64_t in_rs = 1;
};
void launch_cpqr(const QRDesc* d_dev, int32_t nblk, int32_t maxM, int32_t maxN, double tol,
                 bool in_c64, int32_t* ranks_dev, hipStream_t s);

// Batched centre blocks: B = C X^+ (least squares, eq. Bij read from its argmin).
struct LSDesc {
  const bf_c128* C;  // kU x s, ld = ldc
  const bf_c128* X;  // kV x s: element (j, i) at X[i * ldx + j * rsx]
  bf_c128* B;        // kU x kV, ld = kU
  int64_t ldc, ldx;
  int32_t kU, kV, s;
  int32_t rsx = 1;
};
void launch_lsq(const LSDesc* d_dev, int32_t nblk, int32_t maxS, int32_t maxK, hipStream_t s);

// Cross-request solve rounds: one persistent launch over a work list of
// blocks from several requests' batched QRs and least squares (LDS path
// only: each block's need, solve_lds_qr / solve_lds_lsq, must be at most
// solve_lds_limit()).  nitems is a device int read by the kernel.
enum { kSolveQR = 0, kSolveLSQ = 1 };
struct SolveWork {
  const void* descs;   // QRDesc* or LSDesc* (device)
  int32_t* ranks;      // QR: rank of block b at ranks[b] (device)
  double tol;
  int32_t kind;
  int32_t in_c64;
};
struct SolveItem {
  int32_t work, block;
};
size_t solve_lds_qr(int32_t maxM, int32_t maxN);
size_t solve_lds_lsq(int32_t maxS, int32_t maxK);
size_t solve_lds_limit();
void launch_solve_round(const SolveWork* works, const SolveItem* items, const int32_t* nitems,
                        int32_t grid, size_t lds, hipStream_t s);
// Hands a level's batched solves to the solve rounds of the calling thread's
// request engine, if it has them (blocks until the round is launched; the
// stream s then waits for it); false: the caller launches them itself.
// cost[b]: estimated work of block b (orders the round's work list).
bool round_solve(int kind, const void* descs_dev, int32_t n, const std::vector<double>& cost,
                 double tol, bool in_c64, int32_t* ranks_dev, size_t lds, hipStream_t s);

class SolveRounds;
SolveRounds* new_solve_rounds(int device);
void delete_solve_rounds(SolveRounds* R);
void solve_rounds_stats(const SolveRounds* R, int64_t* rounds, int64_t* items);
// While alive, the calling thread's constructions hand their level solves to
// R (round_solve) and count as in flight for its round windows.
// true while this thread takes part in cross-request solve rounds
bool solve_rounds_active();
class RoundsScope {
 public:
  explicit RoundsScope(SolveRounds* R);
  ~RoundsScope();
  RoundsScope(const RoundsScope&) = delete;
  RoundsScope& operator=(const RoundsScope&) = delete;

 private:
  SolveRounds* R_;
  SolveRounds* prev_;
};

// complex128 -> complex64 copy (contiguous)
void launch_c128_to_c64(const bf_c128* in, bf_c64* out, int64_t n, hipStream_t s);

// Apply stage (complex64 factors, FP32 accumulation).  Every output block of
// a stage is out = [G_0 G_1] [in_0; in_1]: one packed row-major M x (K0+K1)
// factor block and two input row ranges.  Buffer ids select among 4 base
// pointers given at launch (0: caller input, 1/2: ping-pong intermediates,
// 3: caller output); row offsets are fixed when the plan is built.
struct ApplyBlk {
  int64_t g_off;      // element offset of the packed block (row-major, M x (K0+K1))
  int64_t out_row;
  int64_t in_row0, in_row1;
  int64_t row_rec;    // index of the block's first row record
  int32_t M, K0, K1;
  int8_t out_buf, in_buf0, in_buf1, pad;
};
// One output row of a stage with every address it needs (few right-hand sides).
struct ApplyRowRec {
  int64_t g;          // element offset of the row in the packed arena
  int64_t in0, in1;   // input row offsets (in1 already shifted by -K0)
  int64_t out;        // output row
  int32_t K0, KK;
  int8_t out_buf, in_buf0, in_buf1, pad[5];
};
// Writes the row records of every block (rows[b.row_rec + r], r < b.M).
void launch_expand_rows(const ApplyBlk* blks_dev, int32_t nblk, ApplyRowRec* rows_dev,
                        hipStream_t s);
// Up to this many right-hand sides a stage runs the few-column kernel, whose
// row records address column-major buffers.
constexpr int kApplyFewCols = 4;
// Up to this many right-hand sides an apply runs its stages fused (several
// stages per launch, launch_apply_fused), column-major throughout.
constexpr int kApplyFusedCols = kApplyFewCols;
// Rows of one group and stage in a fused launch of several stages.  Such a
// group's intermediates stay in its workgroup's LDS: row records with buffer
// index kFusedLdsBuf address a column-major LDS matrix of 2 kFusedLdsRows
// rows per column, a stage writing the half (stage - first stage) & 1 and
// the next stage reading it there.
constexpr int kFusedLdsRows = 128;
constexpr int kFusedLdsBuf = 4;
// maxMK / maxKK / maxM: largest M*(K0+K1), K0+K1 and M over the stage's
// blocks.  Buffer i holds element (r, c) at bufs[i][r * rss[i] + c * lds[i]]
// (column-major: rss = 1; with at most kApplyFewCols columns every buffer must be).
// prec: BF_PREC_BF16X3 runs stages of >= 5 right-hand sides on the BF16
// matrix cores (split operands), anything else on the vector ALUs.
void launch_apply_stage(const ApplyBlk* blks_dev, int32_t nblk, const ApplyRowRec* rows_dev,
                        int32_t nrows, int32_t maxMK, int32_t maxKK, int32_t maxM, const bf_c64* G,
                        const bf_c64* const bufs[4], const int64_t lds[4], const int64_t rss[4],
                        int64_t ncols, int prec, hipStream_t s, bool may_time = true);
// A merging stage on windowed intermediates of a structured sample (split-BF16
// matrix cores, blocks of at most 64 rows): output columns [0, win) of a
// block come from its first term and its first input's columns, columns
// [win, ncols) from its second term and its second input's columns
// [0, ncols - win).
void launch_apply_window_stage(const ApplyBlk* blks_dev, int32_t nblk, int32_t maxM,
                               const bf_c64* G, const bf_c64* const bufs[4],
                               const int64_t lds[4], const int64_t rss[4], int64_t ncols,
                               int64_t win, hipStream_t s);

// Fused stages: workgroup w runs the row records [off[w*(nstage+1)+t],
// off[w*(nstage+1)+t+1]) of stage t for t = 0..nstage-1, with a barrier
// between stages; buffers column-major (element (r, c) at bufs[i][r + c*lds[i]]).
// ncols <= kApplyFusedCols; FP32 sums whatever prec.
// max_rows: the most rows one workgroup has in one stage (sizes the workgroup).
void launch_apply_fused(const ApplyRowRec* rows_dev, const int32_t* off_dev, int32_t nwg,
                        int32_t nstage, int32_t max_rows, const bf_c64* G,
                        const bf_c64* const bufs[4], const int64_t lds[4], int64_t ncols,
                        int prec, hipStream_t s);

// Gather (and optionally conjugate-transpose) factor sub-blocks into an
// arena: element (r, k) of the M x K result goes to
//   dst[dst_off + r * dst_rs + k * dst_cs],
// taken from conjT ? conj(src[(row0 + k) + r*src_ld]) : src[(row0 + r) + k*src_ld].
struct PackDesc {
  const bf_c128* src;
  int64_t dst_off;
  int32_t src_ld;
  int32_t row0;
  int32_t M;
  int32_t K;
  int32_t conjT;
  int32_t dst_rs;    // destination stride between rows
  int32_t dst_cs;    // destination stride between columns
  int32_t pad;
};
void launch_pack_c64(const PackDesc* d_dev, int32_t ndesc, bf_c64* dst, hipStream_t s);
void launch_pack_c128(const PackDesc* d_dev, int32_t ndesc, bf_c128* dst, hipStream_t s);

// Segment-stacked expansion: out[:, g*ncols + c] = X restricted to rows seg_g,
// zero elsewhere (rows x nseg*ncols, ld = ldo).
void launch_expand_segments(const bf_c64* X, int64_t ldx, int64_t rows, int64_t ncols,
                            const int64_t* seg_dev, int32_t nseg, bf_c64* out, int64_t ldo,
                            hipStream_t s);

// E(r, (g - g0) s + c) = C(r, c) for rows r of segment g (rowseg[r] = g, -1:
// none), zero in every other column of E (rows x ng s); element (r, c) of C
// at C[r crs + c cld], of E at E[r ers + col eld].
void launch_expand_by_segment(const bf_c64* C, int64_t crs, int64_t cld, const int32_t* rowseg,
                              int64_t rows, int32_t s, int32_t g0, int32_t ng, bf_c64* E,
                              int64_t ers, int64_t eld, hipStream_t st);

// -------------------------------------------------------------- autotuner --
// Family, then kTuneKeyFields class fields (powers of two of the sizes that
// matter, column counts, flags).  tune_choose runs run(c) for the class's
// chosen candidate c -- or, the first time a class is seen (tuner on, stream
// not capturing), every candidate in turn, timed, keeping the fastest -- and
// returns it; with the tuner off or a single candidate it runs `fallback`,
// and so it does for an unknown class under capture or when may_time is
// false (callers that must not create events).  Candidates must give bitwise
// the same results.
enum { kTuneMatfreeWidth = 0, kTuneChainRows = 1, kTuneCpqrThreads = 2, kTuneApplyFused = 3,
       kTuneApplyRows = 4, kTuneApplyMfma = 5, kTuneFamilies = 6 };
constexpr int kTuneKeyFields = 5;
using TuneKey = std::array<int64_t, 1 + kTuneKeyFields>;
int64_t pow2_ceil(int64_t v);
bool autotune_on();
int64_t tune_choose(const TuneKey& key, const std::vector<int64_t>& cand, int64_t fallback,
                    hipStream_t s, const std::function<void(int64_t)>& run,
                    bool may_time = true);
int tune_save(const char* path);
int tune_load(const char* path);
void tune_clear();

// ------------------------------------------------- matrix-free operators --
struct PointSet {     // structure-of-arrays FP64 coordinates on the device
  const double* x;
  const double* y;
  const double* z;    // nullptr for 2D points
};
// Y[:, g*ncols + c] = sum_{j in seg_g} E(i, j) X[j, c], E = kernel entries of
// op(A) (sign = +1: A, sign = -1: A^H, points swapped by the caller).
// The autotuner's switch and table size (tune.cpp); process-wide.
void set_autotune(int on);
int64_t autotune_entries();
void launch_segkernel(int prec, PointSet out_pts, int64_t nout, PointSet in_pts, int64_t nin,
                      double k_over_2pi, int sign, const bf_c64* X, int64_t ldx, int64_t ncols,
                      bf_c64* Y, int64_t ldy, const int64_t* seg_host, int32_t nseg,
                      hipStream_t s);
void launch_fio(int prec, int64_t n, const double* cx_dev, int adjoint, const bf_c64* X, int64_t ldx,
                int64_t ncols, bf_c64* Y, int64_t ldy, const int64_t* seg_host, int32_t nseg,
                hipStream_t s);
void launch_dense(int prec, const bf_c64* A, int64_t m, int64_t n, int64_t lda, int adjoint,
                  const bf_c64* X, int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy,
                  const int64_t* seg_host, int32_t nseg, hipStream_t s);
// Y0 (rows x nseg*s0) = the sums of the column pairs of Yb (rows x 2 nseg*w)
// that hold the two halves of every node's product: Y0(:, g s0 + c) =
// Yb(:, 2g w + off + c) + Yb(:, (2g+1) w + off + c).
void launch_sum_halves(const bf_c64* Yb, int64_t rows, int64_t nseg, int32_t w, int32_t off,
                       int32_t s0, bf_c64* Y0, hipStream_t s);
// Built-in operators whose black-box call evaluates every kernel entry once
// per call (its cost nearly independent of the column count up to the widest
// column tile): the construction may then merge sweep levels.
bool entrywise_operator(bf_op_fn mv, bf_op_fn rmv);
// true for the library's own operators (entrywise ones, factors as a black
// box, and compositions of those): their products may be requested from two
// host threads on two streams at once
bool builtin_operator(bf_op_fn mv, bf_op_fn rmv, void* user);
// the caller's provider in force on this thread (nullptr: the library's pool)
const UserAlloc* current_user_alloc();
// Black-box inputs known to be exact in BF16: the construction driver marks
// the random block it passes to the operator, for the duration of the call
// and on its own thread; a built-in operator handed that very buffer (not a
// copy or a transform of it, which a user callback wrapping it might pass)
// launches only its kernel variant for BF16-exact inputs.
struct ExactInputScope {
  explicit ExactInputScope(const void* x);
  ~ExactInputScope();
  const void* prev;
};
bool input_known_exact(const void* x);

}  // namespace bf
