// Factor store of a hybrid butterfly (output of Alg. 2) and its apply plan.
#pragma once

#include "bf_internal.h"

namespace bf {

// Node (l, i) of a bisection tree over N sorted points covers
// [floor(i N / 2^l), floor((i+1) N / 2^l)) (Sec. 3.1; exact nesting for any N).
inline int64_t node_lo(int64_t N, int l, int64_t i) { return (i * N) >> l; }
inline int64_t node_hi(int64_t N, int l, int64_t i) { return ((i + 1) * N) >> l; }
inline int64_t node_size(int64_t N, int l, int64_t i) { return node_hi(N, l, i) - node_lo(N, l, i); }

inline int num_levels(int64_t m, int64_t n, int64_t leaf) {
  int64_t big = m > n ? m : n;
  int L = 0;
  while ((big + (int64_t(1) << L) - 1) >> L > leaf) ++L;
  return L;
}

// A factor block: column-major, ld = rows, FP64.
struct Block {
  bf_c128* p = nullptr;
  int32_t rows = 0, cols = 0;
};

// One apply stage: output blocks [blk_off, blk_off + nblk) of the plan.
struct Stage {
  int64_t blk_off = 0;
  int32_t nblk = 0;
  int64_t row_off = 0;
  int32_t nrows = 0;
  int32_t maxMK = 0, maxKK = 0, maxM = 0;
  double macs = 0;   // complex multiply-adds per right-hand side
  // level of the input-side tree node each output block belongs to (the
  // source tree for the forward apply, the target tree for the adjoint; the
  // node indices are ApplyPlan::node): a structured sample whose segments are
  // nodes at level tl stays within its segments through every stage with
  // level >= tl.  -1: the output rows mix all of them (the last stage).
  int32_t level = -1;
  int32_t out_buf = 0;   // buffer the stage writes (1, 2: intermediates; 3: output)
};

// Consecutive stages run as one launch (launch_apply_fused): workgroup w
// takes records foff[off_off + w*(nstage+1) + t] .. +1 of stage t.
struct FusedSeg {
  int64_t off_off = 0;
  int32_t nwg = 0, nstage = 0;
  int32_t first_stage = 0;
  int32_t max_rows = 0;   // most rows one group has in one stage
  double macs = 0;        // complex multiply-adds per right-hand side
};

struct ApplyPlan {
  DevBuf<bf_c64> G;              // packed blocks of every stage (row-major per block)
  DevBuf<ApplyBlk> blks;         // output blocks of all stages, stage after stage
  DevBuf<ApplyRowRec> rows;      // output rows of all stages (few right-hand sides)
  std::vector<Stage> stages;     // in execution order
  int64_t tmp_rows = 0;          // rows of each ping-pong intermediate
  // host copies of every block's output rows and input-side tree node (see
  // Stage::level), for applies to structured samples
  std::vector<int64_t> out_row;
  std::vector<int32_t> out_m;
  std::vector<int64_t> node;
  // fused schedule (few right-hand sides): every stage but the last writes its
  // own rows of one tall intermediate of fused_rows rows
  DevBuf<ApplyRowRec> frows;     // row records grouped by segment, workgroup, stage
  DevBuf<int32_t> foff;
  std::vector<FusedSeg> segs;
  int64_t fused_rows = 0;
};

}  // namespace bf

struct bf_factors;
namespace bf {
struct ApplyGraphCache;
ApplyGraphCache* new_apply_graph_cache();
int apply_graph_count(const bf_factors* F);
void free_apply_graphs(ApplyGraphCache* c);
}

struct bf_factors {
  int64_t m = 0, n = 0, leaf = 0;
  int L = 0, lm = 0;
  std::vector<bf::DevBuf<bf_c128>> store;   // owning FP64 level buffers
  std::vector<bf::Block> U, V, B;           // U_{L,i}, V_{0,j}, B_{i,j} (i * 2^(L-lm) + j)
  std::vector<std::vector<bf::Block>> R;    // R[l - lm][i * 2^(L-l) + j], lm <= l < L
  std::vector<std::vector<bf::Block>> W;    // W[l][i * 2^(L-l) + j], 1 <= l <= lm
  std::vector<int32_t> kU, kV;              // ranks, layout of bf_ranks
  bf::ApplyPlan fwd, adj;
  int apply_prec = BF_PREC_BF16X3;          // bf_set_apply_precision
  int apply_fuse = 1;                       // bf_set_apply_fusion
  bf_info info{};
  int device = 0;
  int64_t graph_cols = 0;                   // bf_set_apply_graph_cols
  bf::ApplyGraphCache* graphs = nullptr;    // captured apply graphs (plan.cpp)
  bf_factors() = default;
  bf_factors(const bf_factors&) = delete;
  bf_factors& operator=(const bf_factors&) = delete;
  ~bf_factors();

  int32_t ku(int l, int64_t i, int64_t j) const {
    return kU[(size_t)(l - lm) * ((size_t)1 << L) + (size_t)(i << (L - l)) + (size_t)j];
  }
  int32_t kv(int l, int64_t i, int64_t j) const {
    return kV[(size_t)l * ((size_t)1 << L) + (size_t)(i << (L - l)) + (size_t)j];
  }
  int32_t& ku_ref(int l, int64_t i, int64_t j) {
    return kU[(size_t)(l - lm) * ((size_t)1 << L) + (size_t)(i << (L - l)) + (size_t)j];
  }
  int32_t& kv_ref(int l, int64_t i, int64_t j) {
    return kV[(size_t)l * ((size_t)1 << L) + (size_t)(i << (L - l)) + (size_t)j];
  }
};

namespace bf {
// Build the forward and adjoint apply plans (packs the complex64 blocks).
void build_apply_plans(bf_factors* F, hipStream_t s);
// Device bytes of intermediates an apply of ncols columns uses: the fused
// schedule's tall buffer for up to kApplyFusedCols columns, else (or with
// staged = true) two ping-pong buffers of plan.tmp_rows rows.
size_t apply_scratch_bytes(const bf_factors* F, int trans, int64_t ncols, bool staged = false);
// One apply with caller-provided intermediates (scratch, scratch_bytes): the
// fused schedule when ncols allows it and the scratch holds it, else the L+3
// stage launches (BF_EINVAL if neither fits).  prof brackets each launch for
// bf_profile_* (creates events; off for callers that must not allocate).
void run_apply(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
               bf_c64* Y, int64_t ldy, void* scratch, size_t scratch_bytes, hipStream_t s,
               bool prof);
// Apply (Y = F X or F^H X), complex64.
void apply_factors(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
                   bf_c64* Y, int64_t ldy, hipStream_t s);
// Structured samples (Sec. 4.1) through the factors: Y[:, g ncols + c] =
// op(F)(:, seg_g) X(seg_g, c) for the nseg row segments of X.  When the
// segments are consecutive nodes of one level of the input-side tree, the
// stages that keep every segment apart run once on X itself (ncols columns:
// each of their output rows belongs to one segment), and only the later
// stages run on the block-diagonal expansion (nseg ncols columns, in chunks
// of at most max_cols).  Returns false (nothing launched) for other segments.
bool apply_structured(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx,
                      int64_t ncols, bf_c64* Y, int64_t ldy, const int64_t* seg, int32_t nseg,
                      int64_t max_cols, hipStream_t s);
// bf_apply_noalloc: run_apply with the intermediates in the library's fixed
// per-device scratch array (noalloc.hip); BF_EINVAL if they do not fit.
void apply_noalloc(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
                   bf_c64* Y, int64_t ldy, hipStream_t s);
size_t noalloc_scratch_bytes();
// Canonical-order block list (U, R^{L-1..lm}, B, W^{lm..1}, V).
std::vector<Block> canonical_blocks(const bf_factors* F);
}  // namespace bf
