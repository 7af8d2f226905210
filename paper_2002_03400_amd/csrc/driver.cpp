// Host driver of Alg. 2 (adaptive randomized hybrid butterfly construction).
//
// Per adaptive iteration / per level the driver
//   1. draws the structured random block of every sample of the level in one
//      launch (segment-stacked: the samples' supports partition the rows),
//   2. hands it to the black box once (one callback for the whole level),
//   3. applies the already-built factors to all samples (batched GEMMs of the
//      partial chains: V-chain^H, U-chain^H, X-chain),
//   4. runs the truncated pivoted QR of every block of the level in one
//      batched launch (FP64) and reads the ranks back (the one host sync of
//      the level: the next level's widths depend on them).
// The W sweep (row side) and the R sweep (column side) follow the paper's
// order; B is computed with the last R level (l = l_m), or, when the centre
// sits on the row leaves (l_m = L), from one full-height sample afterwards.
// The passes of the adaptive leaf loops are merged into shared black-box
// calls where their widths allow (same products, fewer entry sweeps).
//
// Readings of the paper taken here (the CPU oracle takes the same ones):
// conjugate transposes for complex data; Alg. 1's tolerance is the relative
// Frobenius tail of each sample; the adaptive loops draw a fresh random block
// per pass, stop without doubling once r > max rank, and restart from r0 for
// the U loop; the R sweep's tau ranges over T-level l; eq. (Bij) is read from
// its argmin, B = (R^H Z) X^+; at l = l_m the sample width also covers the
// V-side ranks; every sample has its own width.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <memory>
#include <mutex>
#include <thread>

#include "factors.h"

namespace bf {

namespace {

constexpr uint64_t PHASE_V0 = 1, PHASE_U0 = 2, PHASE_W = 3, PHASE_R = 4;
inline uint64_t make_tag(uint64_t phase, uint64_t level, uint64_t node) {
  return (phase << 56) | (level << 40) | node;
}

// A stack of blocks of one sample ("tall matrix"): block b occupies rows
// [roff[b], roff[b] + k_b) of a column-major matrix with leading dimension ld;
// `base` already points at the sample's first column.
template <typename T>
struct Tall {
  const T* base = nullptr;
  int64_t ld = 0;      // column stride
  int64_t rs = 1;      // row stride (row-major views: the sample's width)
  std::vector<int64_t> roff;
  const T* at(int64_t row) const { return base + row * rs; }
  T* out_at(int64_t row) const { return const_cast<T*>(base + row * rs); }
};

// Chain-product operands on a view: rows [row, row + K) of every column.
inline GemmTerm view_term(const bf_c128* F, const Tall<bf_c128>& v, int64_t row, int32_t f_ld,
                          int32_t K) {
  GemmTerm t{F, v.at(row), v.ld, f_ld, K, 1};
  t.in_rs = (int32_t)v.rs;
  return t;
}
inline void view_out(GemmDesc& g, const Tall<bf_c128>& v, int64_t row) {
  g.out = v.out_at(row);
  g.out_ld = v.ld;
  g.out_rs = (int32_t)v.rs;
}

// Second streams for the row side of constructions, kept for reuse (one per
// construction running its two sides at once; default priority).
std::mutex g_side_mu;
std::vector<hipStream_t> g_side_free[64];

struct SideStream {
  int dev;
  hipStream_t s = nullptr;
  explicit SideStream(int d) : dev(d) {
    BF_CHECK(dev >= 0 && dev < 64, BF_EINVAL, "device index out of range");
    {
      std::lock_guard<std::mutex> lk(g_side_mu);
      if (!g_side_free[dev].empty()) {
        s = g_side_free[dev].back();
        g_side_free[dev].pop_back();
      }
    }
    if (!s) BF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  }
  ~SideStream() {
    std::lock_guard<std::mutex> lk(g_side_mu);
    g_side_free[dev].push_back(s);
  }
  SideStream(const SideStream&) = delete;
  SideStream& operator=(const SideStream&) = delete;
};

// `to` waits on the device for the work enqueued on `from` so far
void stream_after(hipStream_t to, hipStream_t from) {
  hipEvent_t e = nullptr;
  BF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipError_t r = hipEventRecord(e, from);
  if (r == hipSuccess) r = hipStreamWaitEvent(to, e, 0);
  (void)hipEventDestroy(e);
  BF_HIP(r);
}

class Builder {
 public:
  Builder(bf_op_fn mv, bf_op_fn rmv, void* user, int64_t m, int64_t n, double tol, int64_t leaf,
          const bf_opts* o, hipStream_t s)
      : mv_(mv), rmv_(rmv), user_(user), tol_(tol), s_(s) {
    F_ = new bf_factors();
    F_->m = m;
    F_->n = n;
    F_->leaf = leaf;
    if (o) {
      p_ = o->p;
      r0_ = o->r0;
      cap_ = o->max_rank;
      seed_ = o->seed;
      if (o->work_bytes > 0) work_ = o->work_bytes;
      progress_ = o->progress;
      progress_user_ = o->progress_user;
      merge_leaf_ = (o->flags & BF_OPT_SEQUENTIAL_LEAF) == 0;
    }
    merge_sweeps_ = entrywise_operator(mv, rmv) &&
                    !(o && (o->flags & (BF_OPT_SEQUENTIAL_SWEEP | BF_OPT_CENTER_LEVEL)));
    BF_CHECK(p_ >= 0 && r0_ >= 1 && cap_ >= 0 && (!o || o->work_bytes >= 0), BF_EINVAL,
             "bad bf_opts");
    BF_CHECK(!o || (o->flags & ~(BF_OPT_CENTER_LEVEL | BF_OPT_SEQUENTIAL_LEAF |
                                 BF_OPT_SEQUENTIAL_SWEEP | BF_OPT_ONE_STREAM)) == 0,
             BF_EINVAL, "unknown bf_opts flags");
    F_->L = num_levels(m, n, leaf);
    F_->lm = F_->L / 2;
    if (o && (o->flags & BF_OPT_CENTER_LEVEL)) {
      const int c = o->center_level < 0 ? o->center_level + F_->L + 1 : o->center_level;
      BF_CHECK(c >= 0 && c <= F_->L, BF_EINVAL, "centre level outside [0, L]");
      F_->lm = c;
    }
    BF_CHECK(F_->L <= 24, BF_EINVAL, "too many levels");
    BF_HIP(hipGetDevice(&F_->device));
    const size_t nb = size_t(1) << F_->L;
    F_->kU.assign((size_t)(F_->L - F_->lm + 1) * nb, 0);
    F_->kV.assign((size_t)(F_->lm + 1) * nb, 0);
    F_->R.resize(F_->L - F_->lm);
    F_->W.resize(F_->lm + 1);
    two_sides_ = F_->L >= 2 && !progress_ && !(o && (o->flags & BF_OPT_ONE_STREAM)) &&
                 !solve_rounds_active() && builtin_operator(mv, rmv, user);
  }
  // The row side's builder (leaf V loop and W levels) of `main`, for its own
  // stream: the same parameters, factors of the same shape.
  Builder(const Builder& main, hipStream_t s)
      : mv_(main.mv_), rmv_(main.rmv_), user_(main.user_), tol_(main.tol_), s_(s) {
    p_ = main.p_;
    r0_ = main.r0_;
    cap_ = main.cap_;
    seed_ = main.seed_;
    work_ = main.work_;
    merge_leaf_ = main.merge_leaf_;
    merge_sweeps_ = main.merge_sweeps_;
    stop_ = &main.stop_side_;
    const bf_factors* G = main.F_;
    F_ = new bf_factors();
    F_->m = G->m;
    F_->n = G->n;
    F_->leaf = G->leaf;
    F_->L = G->L;
    F_->lm = G->lm;
    F_->device = G->device;
    F_->kU.assign(G->kU.size(), 0);
    F_->kV.assign(G->kV.size(), 0);
    F_->R.resize(G->R.size());
    F_->W.resize(G->W.size());
  }
  ~Builder() { delete F_; }

  bf_factors* run() {
    if (two_sides_) {
      run_sides();
    } else {
      leaf_loop(false);
      leaf_loop(true);
      for (int l = 1; l <= F_->lm; ++l) {
        w_level(l);
        report(BF_PHASE_W, l);
      }
      for (int l = F_->L - 1; l > F_->lm; --l) {
        r_level(l);
        report(BF_PHASE_R, l);
      }
    }
    if (F_->lm < F_->L) {
      r_level(F_->lm);
      report(BF_PHASE_R, F_->lm);
    }
    if (F_->lm == F_->L) {
      centre_at_leaves();
      if (F_->L > 0) report(BF_PHASE_R, F_->L);
    }
    finalize();
    bf_factors* out = F_;
    F_ = nullptr;
    return out;
  }

 private:
  // What the row side hands back: its factors, ranks, storage and counts.
  struct RowSide {
    std::vector<Block> V;
    std::vector<std::vector<Block>> W;
    std::vector<int32_t> kV;
    std::vector<DevBuf<bf_c128>> store;
    int v_iters = 0, merged = 0, misses = 0;
    int64_t rmv_cols = 0;
  };

  // The two sides of Alg. 2 meet only at the centre level: the row side
  // (leaf V loop, W levels 1..l_m) needs the black box's A^H products and
  // its own ranks, the column side (leaf U loop, R levels L-1..l_m+1) A's
  // products and its ranks.  The row side runs on a second stream, driven
  // by a second host thread, while this thread drives the column side; each
  // side's partial products, solves and rank reads then overlap the other
  // side's black-box products.  Both enqueue exactly the work they would
  // enqueue one after the other, so the factors are the same bit for bit.
  void run_sides() {
    SideStream side(F_->device);
    stream_after(side.s, s_);   // the caller's earlier work on s_ comes first
    const UserAlloc* ua = current_user_alloc();
    std::exception_ptr err;
    RowSide rs;
    std::thread th([&] {
      try {
        BF_HIP(hipSetDevice(F_->device));
        UseAllocator use(ua);
        AllocScope scope(side.s);
        Builder vb(*this, side.s);
        vb.leaf_loop(false);
        for (int l = 1; l <= vb.lm(); ++l) vb.w_level(l);
        rs.V = std::move(vb.F_->V);
        rs.W = std::move(vb.F_->W);
        rs.kV = std::move(vb.F_->kV);
        rs.store = std::move(vb.F_->store);
        rs.v_iters = vb.v_iters_;
        rs.merged = vb.merged_levels_;
        rs.misses = vb.merge_misses_;
        rs.rmv_cols = vb.rmv_cols_;
      } catch (...) {
        err = std::current_exception();
      }
    });
    struct Joiner {
      std::thread& t;
      std::atomic<bool>& stop;
      ~Joiner() {
        if (t.joinable()) {
          stop = true;   // this side failed: the other stops at its next level
          t.join();
        }
      }
    } joiner{th, stop_side_};
    leaf_loop(true);
    for (int l = F_->L - 1; l > F_->lm; --l) r_level(l);
    th.join();
    if (err) std::rethrow_exception(err);
    stream_after(s_, side.s);
    F_->V = std::move(rs.V);
    F_->W = std::move(rs.W);
    F_->kV = std::move(rs.kV);
    for (auto& b : rs.store) F_->store.push_back(std::move(b));
    v_iters_ = rs.v_iters;
    merged_levels_ += rs.merged;
    merge_misses_ += rs.misses;
    rmv_cols_ += rs.rmv_cols;
  }
  void check_stop() const {
    if (stop_ && stop_->load()) throw Error(BF_EINVAL, "construction stopped: the other side failed");
  }

  bf_op_fn mv_, rmv_;
  void* user_;
  double tol_;
  hipStream_t s_;
  int p_ = 2, r0_ = 4, cap_ = 0;
  uint64_t seed_ = 0;
  int64_t work_ = int64_t(8) << 30;   // sweep workspace bound (bf_opts.work_bytes)
  bf_factors* F_;
  Staging own_st_;
  // uploads go through the request scope's pinned staging when there is one
  Staging& st_ = scope_staging(s_) ? *scope_staging(s_) : own_st_;
  int64_t mv_cols_ = 0, rmv_cols_ = 0;
  int v_iters_ = 0, u_iters_ = 0;
  int merged_levels_ = 0, merge_misses_ = 0;
  bool merge_leaf_ = true;
  bool two_sides_ = false;                  // run_sides() (else one stream, one thread)
  std::atomic<bool> stop_side_{false};      // set when the column side fails
  const std::atomic<bool>* stop_ = nullptr; // the row side's view of it
  // Sweep levels two at a time.  For a built-in operator that evaluates the
  // kernel entries on the fly, a black-box call costs about the same for 40
  // columns as for 80 (its vector ALUs evaluate every entry once per call;
  // the matrix cores multiplying them have room).  A sweep level then draws
  // the next level's samples too (twice as many nodes, each one of its nodes'
  // children), at a width guessed from its own (the next level's widths need
  // its ranks), and makes one call over the next level's segments with both
  // blocks side by side: the next level's products come out as its own call
  // would give them (the same random columns -- Philox counters keyed by row
  // and column -- and sums that do not depend on the other columns), this
  // level's as the sums of the halves over each node's two children.  When
  // the next level comes and every node's width fits the guess, its call is
  // skipped; otherwise it makes its own and the early columns are wasted
  // (both are counted in bf_info's column totals).
  bool merge_sweeps_ = false;
  static constexpr int32_t kMergeCols = 80;   // the widest column tile of the black boxes
  struct Ahead {
    int level = -1;            // sweep level the products belong to (-1: none)
    int32_t width = 0;         // every node's sample width
    DevBuf<bf_c64> Y;          // out rows x (nodes * width), node-major
    DevBuf<bf_c64> Om;         // in rows x width (ld in rows): the random block first
  };
  Ahead ahead_;
  void (*progress_)(void*, int32_t, int32_t) = nullptr;
  void* progress_user_ = nullptr;
  void report(int32_t phase, int32_t level) const {
    if (progress_) progress_(progress_user_, phase, level);
  }

  int L() const { return F_->L; }
  int lm() const { return F_->lm; }
  int64_t nb() const { return int64_t(1) << F_->L; }

  void check_cap(int64_t r) {
    if (cap_ > 0 && r > cap_)
      throw Error(BF_ERANK, "rank estimate " + std::to_string(r) + " exceeds max_rank " +
                                std::to_string(cap_));
  }

  // X is always one of this construction's random blocks (gauss, gauss_into:
  // Gaussians stored rounded to BF16, zero padding), hence exact in BF16
  void call_op(bool adjoint, const bf_c64* X, int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy,
               const std::vector<int64_t>* seg) {
    bf_op_fn fn = adjoint ? rmv_ : mv_;
    ExactInputScope ex(X);
    int rc = fn(user_, X, ldx, ncols, Y, ldy, seg ? seg->data() : nullptr,
                seg ? (int32_t)(seg->size() - 1) : 0, (void*)s_);
    if (rc != 0)
      throw Error(BF_ECALLBACK, std::string(adjoint ? "rmatvec" : "matvec") +
                                    " callback returned " + std::to_string(rc));
  }

  DevBuf<bf_c64> gauss(int64_t rows, int64_t ncols, int level, const std::vector<uint64_t>& tags,
                       const std::vector<int32_t>& widths) {
    DevBuf<bf_c64> X((size_t)rows * ncols, s_);
    gauss_at(X.p, rows, ncols, level, tags, widths);
    return X;
  }
  // The structured random block of a level into rows x ncols at X (ld rows).
  void gauss_at(bf_c64* X, int64_t rows, int64_t ncols, int level,
                const std::vector<uint64_t>& tags, const std::vector<int32_t>& widths) {
    if (validating()) {
      BF_CHECK(tags.size() == (size_t(1) << level) && widths.size() == tags.size(), BF_EINVAL,
               "bounds check failed: sample tags");
      for (auto w : widths) BF_CHECK(w <= ncols, BF_EINVAL, "bounds check failed: sample width");
    }
    auto dt = upload(tags, s_, st_);
    auto dw = upload(widths, s_, st_);
    launch_gauss_samples(X, rows, ncols, level, dt.p, dw.p, seed_, s_);
  }

  // The guess for the next level's widths is all the room the 80-column tile
  // leaves beside this level's, taken when it is at least this level's
  // width.  Leaf bases of full rank (rank = leaf size: the FIO at leaf 16)
  // mean the ranks still grow after the leaves, so the first sweep level
  // does not guess.
  bool leaves_saturated(bool col_side) const {
    const int64_t N = col_side ? F_->m : F_->n;
    for (int64_t j = 0; j < nb(); ++j) {
      const int32_t k = col_side ? F_->ku(L(), j, 0) : F_->kv(0, 0, j);
      if (k > 0 && k >= node_lo(N, L(), j + 1) - node_lo(N, L(), j)) return true;
    }
    return false;
  }

  // One black-box call for a sweep level's samples (nseg nodes of input-tree
  // level tl, widths `width`, at most s0) and the next level's (2 nseg nodes
  // of level tl + 1, all spec wide, tags ntags): X = [next level's block |
  // this level's block] over the next level's segments.  Returns this level's
  // products (out_rows x nseg s0, node-major); the next level's go to ahead_.
  DevBuf<bf_c64> merged_call(bool adjoint, int64_t in_rows, int64_t out_rows, int tl,
                             int64_t nseg, const std::vector<uint64_t>& tags,
                             const std::vector<int32_t>& width, int32_t s0, int32_t spec,
                             int next_level, const std::vector<uint64_t>& ntags) {
    const int64_t n2 = 2 * nseg;
    const int32_t w = spec + s0;
    DevBuf<bf_c64> X((size_t)in_rows * w, s_);
    gauss_at(X.p, in_rows, spec, tl + 1, ntags, std::vector<int32_t>((size_t)n2, spec));
    gauss_at(X.p + (size_t)in_rows * spec, in_rows, s0, tl, tags, width);
    std::vector<int64_t> seg((size_t)n2 + 1);
    for (int64_t i = 0; i <= n2; ++i) seg[(size_t)i] = node_lo(in_rows, tl + 1, i);
    DevBuf<bf_c64> Yb((size_t)out_rows * n2 * w, s_);
    call_op(adjoint, X.p, in_rows, w, Yb.p, out_rows, &seg);
    DevBuf<bf_c64> Y0((size_t)out_rows * nseg * s0, s_);
    launch_sum_halves(Yb.p, out_rows, nseg, w, spec, s0, Y0.p, s_);
    ahead_.level = next_level;
    ahead_.width = spec;
    ahead_.Y = DevBuf<bf_c64>((size_t)out_rows * n2 * spec, s_);
    const size_t blk = (size_t)out_rows * spec;
    for (int64_t g = 0; g < n2; ++g)
      BF_HIP(hipMemcpyAsync(ahead_.Y.p + (size_t)g * blk, Yb.p + (size_t)g * out_rows * w,
                            blk * sizeof(bf_c64), hipMemcpyDeviceToDevice, s_));
    ahead_.Om = std::move(X);
    return Y0;
  }

  void gemm(const std::vector<GemmDesc>& d, bool in_c64) {
    if (d.empty()) return;
    int maxc = 0, maxm = 0, maxk = 0;
    for (auto& x : d) {
      maxc = std::max(maxc, x.ncols);
      maxm = std::max(maxm, x.M);
      int ks = 0;
      for (int t = 0; t < x.nterm; ++t) ks += x.t[t].K;
      maxk = std::max(maxk, ks);
    }
    if (validating()) {
      const size_t isz = in_c64 ? sizeof(bf_c64) : sizeof(bf_c128);
      for (auto& x : d) {
        if (x.M <= 0 || x.ncols <= 0) continue;
        check_extent(x.out, ((size_t)(x.ncols - 1) * x.out_ld + (size_t)(x.M - 1) * x.out_rs + 1) *
                                sizeof(bf_c128), "gemm out");
        for (int t = 0; t < x.nterm; ++t) {
          const GemmTerm& T = x.t[t];
          if (T.K <= 0) continue;
          size_t fe = T.op == 0 ? (size_t)(T.K - 1) * T.f_ld + x.M : (size_t)(x.M - 1) * T.f_ld + T.K;
          check_extent(T.F, fe * sizeof(bf_c128), "gemm factor");
          check_extent(T.in, ((size_t)(x.ncols - 1) * T.in_ld + (size_t)(T.K - 1) * T.in_rs + 1) * isz,
                       "gemm input");
        }
      }
    }
    auto dd = upload(d, s_, st_);
    launch_chain_gemm(dd.p, (int32_t)d.size(), maxc, maxm, maxk, in_c64, s_);
  }

  // Batched Alg. 1 step 3; Q blocks go to a fresh capacity buffer that becomes
  // the factor storage of the level.  Returns ranks (host) and fills `out`.
  std::vector<int32_t> cpqr(const std::vector<QRDesc>& in, bool in_c64, std::vector<Block>& out) {
    const size_t nblk = in.size();
    std::vector<int64_t> off(nblk);
    int64_t tot = 0;
    int maxM = 0, maxN = 0;
    for (size_t b = 0; b < nblk; ++b) {
      off[b] = tot;
      tot += (int64_t)in[b].M * std::min(in[b].M, in[b].N);
      maxM = std::max(maxM, in[b].M);
      maxN = std::max(maxN, in[b].N);
    }
    DevBuf<bf_c128> store((size_t)std::max<int64_t>(tot, 1), s_);
    std::vector<QRDesc> d = in;
    for (size_t b = 0; b < nblk; ++b) d[b].q = store.p + off[b];
    if (validating())
      for (auto& x : d) {
        if (x.M <= 0 || x.N <= 0) continue;
        check_extent(x.in, ((size_t)(x.N - 1) * x.in_ld + (size_t)(x.M - 1) * x.in_rs + 1) *
                               (in_c64 ? sizeof(bf_c64) : sizeof(bf_c128)),
                     "cpqr input");
        check_extent(x.q, (size_t)x.M * std::min(x.M, x.N) * sizeof(bf_c128), "cpqr output");
      }
    auto dd = upload(d, s_, st_);
    DevBuf<int32_t> rk(nblk, s_);
    // in a request engine with solve rounds, this level's QRs join the other
    // in-flight constructions' in one launch (same per-block code)
    std::vector<double> cost(nblk);
    for (size_t b = 0; b < nblk; ++b)
      cost[b] = (double)in[b].M * in[b].N * std::min(in[b].M, in[b].N);
    if (!round_solve(kSolveQR, dd.p, (int32_t)nblk, cost, tol_, in_c64, rk.p,
                     solve_lds_qr(maxM, maxN), s_))
      launch_cpqr(dd.p, (int32_t)nblk, maxM, maxN, tol_, in_c64, rk.p, s_);
    std::vector<int32_t> ranks(nblk);
    int32_t* hr = static_cast<int32_t*>(st_.alloc(nblk * sizeof(int32_t), s_));
    BF_HIP(hipMemcpyAsync(hr, rk.p, nblk * sizeof(int32_t), hipMemcpyDeviceToHost, s_));
    BF_HIP(hipStreamSynchronize(s_));
    std::memcpy(ranks.data(), hr, nblk * sizeof(int32_t));
    st_.reset();
    // keep only the k leading columns of every Q (the capacity holds
    // min(M, N) of them): factor storage becomes sum M k instead of
    // sum M min(M, N)
    std::vector<int64_t> coff(nblk);
    int64_t ctot = 0;
    for (size_t b = 0; b < nblk; ++b) {
      coff[b] = ctot;
      ctot += (int64_t)in[b].M * std::max(ranks[b], 0);
    }
    DevBuf<bf_c128> compact((size_t)std::max<int64_t>(ctot, 1), s_);
    std::vector<PackDesc> pd;
    pd.reserve(nblk);
    for (size_t b = 0; b < nblk; ++b)
      if (in[b].M > 0 && ranks[b] > 0)
        pd.push_back(PackDesc{store.p + off[b], coff[b], in[b].M, 0, in[b].M, ranks[b], 0, 1,
                              in[b].M, 0});
    for (size_t o = 0; o < pd.size(); o += 60000) {
      const size_t cnt = std::min<size_t>(60000, pd.size() - o);
      std::vector<PackDesc> part(pd.begin() + o, pd.begin() + o + cnt);
      auto dd = upload(part, s_, st_);
      launch_pack_c128(dd.p, (int32_t)cnt, compact.p, s_);
    }
    store.reset();
    out.resize(nblk);
    for (size_t b = 0; b < nblk; ++b) out[b] = Block{compact.p + coff[b], in[b].M, ranks[b]};
    F_->store.push_back(std::move(compact));
    return ranks;
  }

  // ---- adaptive leaf loops (first two loops of Alg. 2) ---------------------
  // Every pass draws a fresh random block whose values are fixed in advance
  // (its own tag), so consecutive passes are merged into one black-box call
  // while their widths add up to at most LEAF_BATCH_COLS (the widest tile of
  // the built-in split-BF16 products, which evaluate each matrix entry once
  // per call up to that width; r = 4, 8, 16, 32 at p = 2 take 68 columns).  Merging
  // changes only how the products are grouped into calls, not their values;
  // a pass the loop does not reach wastes its columns (counted in the stats).
  // BF_OPT_SEQUENTIAL_LEAF makes one call per pass.
  static constexpr int64_t LEAF_BATCH_COLS = 80;

  void leaf_loop(bool col_side) {
    const int64_t rows_in = col_side ? F_->n : F_->m;   // rows of the random block
    const int64_t rows_out = col_side ? F_->m : F_->n;  // rows of the sample
    int64_t r = r0_;
    DevBuf<bf_c64> Y;                  // samples of the current batch of passes
    std::vector<int64_t> boff;         // column offset of each pass in the batch
    int bstart = 0, bend = 0;          // passes [bstart, bend) are in Y
    for (int it = 0;; ++it) {
      check_stop();
      check_cap(r);
      const int64_t s = r + p_;
      BF_CHECK(s <= 65535, BF_ERANK, "sample width too large");
      if (it == bend) {
        // passes it, it+1, ... (stopping at the rank cap and the width bound)
        std::vector<int64_t> widths{s};
        int64_t tot = s;
        for (int64_t rr = 2 * r; merge_leaf_; rr *= 2) {
          if ((cap_ > 0 && rr > cap_) || tot + rr + p_ > LEAF_BATCH_COLS) break;
          widths.push_back(rr + p_);
          tot += rr + p_;
        }
        DevBuf<bf_c64> G((size_t)rows_in * tot, s_);
        boff.assign(widths.size(), 0);
        for (size_t q = 0; q < widths.size(); ++q) {
          boff[q] = q ? boff[q - 1] + widths[q - 1] : 0;
          gauss_into(G.p + boff[q] * rows_in, rows_in, widths[q],
                     make_tag(col_side ? PHASE_U0 : PHASE_V0, it + (int)q, 0));
        }
        Y = DevBuf<bf_c64>((size_t)rows_out * tot, s_);
        call_op(!col_side, G.p, rows_in, tot, Y.p, rows_out, nullptr);
        (col_side ? mv_cols_ : rmv_cols_) += tot;
        bstart = it;
        bend = it + (int)widths.size();
      }
      const bf_c64* Yp = Y.p + boff[(size_t)(it - bstart)] * rows_out;
      std::vector<QRDesc> d(nb());
      for (int64_t b = 0; b < nb(); ++b) {
        const int64_t lo = node_lo(rows_out, L(), b);
        d[b] = QRDesc{Yp + lo, nullptr, rows_out, (int32_t)node_size(rows_out, L(), b),
                      (int32_t)s};
      }
      // the previous iteration's store is superseded
      size_t nstore = F_->store.size();
      std::vector<Block> blocks;
      auto ranks = cpqr(d, true, blocks);
      int32_t kmax = *std::max_element(ranks.begin(), ranks.end());
      (col_side ? u_iters_ : v_iters_)++;
      report(col_side ? BF_PHASE_LEAF_U : BF_PHASE_LEAF_V, col_side ? u_iters_ : v_iters_);
      if (col_side) {
        F_->U = blocks;
        for (int64_t i = 0; i < nb(); ++i) F_->ku_ref(L(), i, 0) = ranks[i];
      } else {
        F_->V = blocks;
        for (int64_t j = 0; j < nb(); ++j) F_->kv_ref(0, 0, j) = ranks[j];
      }
      if (it > 0) {
        // drop the superseded store of the previous pass
        F_->store.erase(F_->store.begin() + (nstore - 1));
      }
      if (r > kmax) break;
      r *= 2;
    }
  }

  // One pass's random block (level 0, one tag) into rows x ncols at X.
  void gauss_into(bf_c64* X, int64_t rows, int64_t ncols, uint64_t tag) {
    auto dt = upload(std::vector<uint64_t>{tag}, s_, st_);
    auto dw = upload(std::vector<int32_t>{(int32_t)ncols}, s_, st_);
    launch_gauss_samples(X, rows, ncols, 0, dt.p, dw.p, seed_, s_);
  }

  int64_t group_size(int64_t nsamples, double bytes_per_sample) const {
    const double g = std::floor((double)work_ / std::max(bytes_per_sample, 1.0));
    return std::max<int64_t>(1, std::min<int64_t>(nsamples, (int64_t)std::min(g, 1e15)));
  }

  // ---- W sweep, level l (Sec. 4.3) ------------------------------------------
  void w_level(int l) {
    check_stop();
    const int64_t m = F_->m, n = F_->n;
    const int64_t nT = int64_t(1) << l, nS = int64_t(1) << (L() - l);
    std::vector<int32_t> width(nT);
    std::vector<uint64_t> tags(nT);
    int32_t smax = 0;
    for (int64_t i = 0; i < nT; ++i) {
      int32_t w = 0;
      for (int64_t j = 0; j < nS; ++j)
        w = std::max(w, F_->kv(l - 1, i >> 1, 2 * j) + F_->kv(l - 1, i >> 1, 2 * j + 1));
      width[i] = w + p_;
      check_cap(w);
      tags[i] = make_tag(PHASE_W, l, i);
      smax = std::max(smax, width[i]);
    }
    int64_t rows0 = 0;
    std::vector<int64_t> roff0(nb());
    for (int64_t j = 0; j < nb(); ++j) { roff0[j] = rows0; rows0 += F_->kv(0, 0, j); }
    // per sample: Y' (n x smax c64), the leaf stage and two chain stages (FP64)
    auto sample_bytes = [&](int32_t w) { return (double)w * (8.0 * n + 48.0 * (double)rows0); };
    // the whole level's products, when they come from a merged call
    DevBuf<bf_c64> G, Ypre;
    Ahead ah = std::move(ahead_);
    ahead_ = Ahead{};
    bool use_ahead = ah.level == l && group_size(nT, sample_bytes(ah.width)) == nT;
    for (auto w : width) use_ahead = use_ahead && w <= ah.width;
    if (ah.level == l) (use_ahead ? merged_levels_ : merge_misses_)++;
    if (use_ahead) {
      smax = ah.width;
      Ypre = std::move(ah.Y);
    } else {
      const int32_t spec = merge_sweeps_ && l < lm() && !(l == 1 && leaves_saturated(false))
                               ? kMergeCols - smax : 0;
      if (spec >= smax && group_size(nT, sample_bytes(smax)) == nT &&
          group_size(2 * nT, sample_bytes(spec)) == 2 * nT) {
        std::vector<uint64_t> ntags((size_t)(2 * nT));
        for (int64_t i = 0; i < 2 * nT; ++i) ntags[(size_t)i] = make_tag(PHASE_W, l + 1, i);
        Ypre = merged_call(true, m, n, l, nT, tags, width, smax, spec, l + 1, ntags);
        rmv_cols_ += 2 * nT * spec;
      } else {
        G = gauss(m, smax, l, tags, width);
      }
      for (auto w : width) rmv_cols_ += w;
    }
    const int64_t gsz = group_size(nT, sample_bytes(smax));
    BF_CHECK(!Ypre.p || gsz == nT, BF_EINVAL, "internal: merged sweep level split in groups");
    F_->W[l].assign((size_t)nb(), Block{});
    for (int64_t i0 = 0; i0 < nT; i0 += gsz) {
      const int64_t i1 = std::min(nT, i0 + gsz), ng = i1 - i0;
      std::vector<int64_t> seg(ng + 1);
      for (int64_t i = 0; i <= ng; ++i) seg[i] = node_lo(m, l, i0 + i);
      const int64_t ycols = ng * smax;
      DevBuf<bf_c64> Yp;
      if (Ypre.p) {
        Yp = std::move(Ypre);
      } else {
        Yp = DevBuf<bf_c64>((size_t)n * ycols, s_);
        call_op(true, G.p, m, smax, Yp.p, n, &seg);
      }

      // V stage (shared by the group's samples): P0 = V^H Y', rows by leaf j,
      // stored row-major (row stride ycols) so that a block's rows are
      // contiguous for every later product
      DevBuf<bf_c128> P0buf((size_t)std::max<int64_t>(rows0, 1) * ycols, s_);
      {
        std::vector<GemmDesc> d;
        for (int64_t j = 0; j < nb(); ++j) {
          const Block& V = F_->V[j];
          GemmDesc g{};
          g.out = P0buf.p + roff0[j] * ycols;
          g.out_ld = 1;
          g.out_rs = ycols;
          g.M = V.cols;
          g.ncols = (int32_t)ycols;
          g.nterm = 1;
          g.t[0] = GemmTerm{V.p, Yp.p + node_lo(n, L(), j), n, V.rows, V.rows, 1};
          if (g.M > 0) d.push_back(g);
        }
        gemm(d, true);
      }
      Yp.reset();
      // per-sample views of level l' (starting from the shared level 0);
      // view[q] is sample i0 + q
      std::vector<Tall<bf_c128>> view(ng);
      for (int64_t q = 0; q < ng; ++q) {
        view[q].base = P0buf.p + q * smax;
        view[q].ld = 1;
        view[q].rs = ycols;
        view[q].roff = roff0;
      }
      std::vector<DevBuf<bf_c128>> keep;
      for (int lp = 1; lp < l; ++lp) {
        const int64_t nSl = int64_t(1) << (L() - lp);
        // the samples of one node ip of this stage share its W blocks and its
        // output rows: they sit side by side (smax columns each, zero beyond a
        // sample's width), so each block is one product over all of them
        const int sh = l - lp;
        std::vector<int64_t> base(ng);
        std::vector<Tall<bf_c128>> next(ng);
        int64_t tot = 0;
        for (int64_t qa = 0; qa < ng;) {
          const int64_t ip = (i0 + qa) >> sh;
          int64_t qe = qa;
          while (qe < ng && ((i0 + qe) >> sh) == ip) ++qe;
          int64_t rows = 0;
          std::vector<int64_t> roff((size_t)nSl);
          for (int64_t j = 0; j < nSl; ++j) { roff[(size_t)j] = rows; rows += F_->kv(lp, ip, j); }
          const int64_t gw = (qe - qa) * smax;
          for (int64_t q = qa; q < qe; ++q) {
            next[q].roff = roff;
            next[q].ld = 1;                  // row-major, rows x (group width)
            next[q].rs = gw;
            base[q] = tot + (q - qa) * smax;
          }
          tot += std::max<int64_t>(rows, 1) * gw;
          qa = qe;
        }
        DevBuf<bf_c128> buf((size_t)std::max<int64_t>(tot, 1), s_);
        for (int64_t q = 0; q < ng; ++q) next[q].base = buf.p + base[q];
        std::vector<GemmDesc> d;
        for (int64_t qa = 0; qa < ng;) {
          const int64_t ip = (i0 + qa) >> sh;
          int64_t qe = qa;
          while (qe < ng && ((i0 + qe) >> sh) == ip) ++qe;
          for (int64_t j = 0; j < nSl; ++j) {
            const Block& Wb = F_->W[lp][(size_t)((ip << (L() - lp)) + j)];
            const int32_t ka = F_->kv(lp - 1, ip >> 1, 2 * j);
            const int32_t kb = F_->kv(lp - 1, ip >> 1, 2 * j + 1);
            GemmDesc g{};
            view_out(g, next[qa], next[qa].roff[j]);
            g.M = Wb.cols;
            g.ncols = (int32_t)((qe - qa) * smax);
            g.nterm = 2;
            g.t[0] = view_term(Wb.p, view[qa], view[qa].roff[2 * j], Wb.rows, ka);
            g.t[1] = view_term(Wb.p + ka, view[qa], view[qa].roff[2 * j + 1], Wb.rows, kb);
            if (g.M > 0) d.push_back(g);
          }
          qa = qe;
        }
        gemm(d, false);
        if (keep.size() >= 1) keep.erase(keep.begin());   // two stages alive at most
        keep.push_back(std::move(buf));
        view.swap(next);
        if (lp == 1) P0buf.reset();
      }
      // Z_{l,i,j} = [P_{2j}; P_{2j+1}] of sample i  ->  W_{l,i,j}
      std::vector<QRDesc> q((size_t)(ng * nS));
      for (int64_t a = 0; a < ng; ++a)
        for (int64_t j = 0; j < nS; ++j) {
          const int64_t i = i0 + a;
          const int32_t M = F_->kv(l - 1, i >> 1, 2 * j) + F_->kv(l - 1, i >> 1, 2 * j + 1);
          QRDesc qd{view[a].at(view[a].roff[2 * j]), nullptr, view[a].ld, M, width[i]};
          qd.in_rs = view[a].rs;
          q[(size_t)(a * nS + j)] = qd;
        }
      std::vector<Block> blocks;
      auto ranks = cpqr(q, false, blocks);
      for (int64_t a = 0; a < ng; ++a)
        for (int64_t j = 0; j < nS; ++j) {
          const size_t b = (size_t)(((i0 + a) << (L() - l)) + j);
          F_->W[l][b] = blocks[(size_t)(a * nS + j)];
          F_->kv_ref(l, i0 + a, j) = ranks[(size_t)(a * nS + j)];
        }
    }
  }

  // ---- R sweep, level l (Sec. 4.2) and B at l_m (Sec. 4.4) -----------------
  void r_level(int l) {
    const int64_t m = F_->m, n = F_->n;
    const int64_t nT = int64_t(1) << l, nS = int64_t(1) << (L() - l);
    std::vector<int32_t> width(nS);
    std::vector<uint64_t> tags(nS);
    int32_t smax = 0;
    for (int64_t j = 0; j < nS; ++j) {
      int32_t w = 0;
      for (int64_t i = 0; i < nT; ++i)
        w = std::max(w, F_->ku(l + 1, 2 * i, j >> 1) + F_->ku(l + 1, 2 * i + 1, j >> 1));
      if (l == lm())
        for (int64_t i = 0; i < nT; ++i) w = std::max(w, F_->kv(lm(), i, j));
      check_cap(w);
      width[j] = w + p_;
      tags[j] = make_tag(PHASE_R, l, j);
      smax = std::max(smax, width[j]);
    }
    int64_t rowsL = 0;
    std::vector<int64_t> roffL(nb());
    for (int64_t i = 0; i < nb(); ++i) { roffL[i] = rowsL; rowsL += F_->ku(L(), i, 0); }
    // per sample: Y (m x smax c64), the leaf stage and two chain stages (FP64)
    auto sample_bytes = [&](int32_t w) { return (double)w * (8.0 * m + 48.0 * (double)rowsL); };
    // the whole level's products, when they come from a merged call (the
    // random block Om is kept for the centre level)
    DevBuf<bf_c64> Om, Ypre;
    Ahead ah = std::move(ahead_);
    ahead_ = Ahead{};
    bool use_ahead = ah.level == l && group_size(nS, sample_bytes(ah.width)) == nS;
    for (auto w : width) use_ahead = use_ahead && w <= ah.width;
    if (ah.level == l) (use_ahead ? merged_levels_ : merge_misses_)++;
    if (use_ahead) {
      smax = ah.width;
      Ypre = std::move(ah.Y);
      Om = std::move(ah.Om);
    } else {
      const int32_t spec = merge_sweeps_ && l > lm() && !(l == L() - 1 && leaves_saturated(true))
                               ? kMergeCols - smax : 0;
      if (spec >= smax && group_size(nS, sample_bytes(smax)) == nS &&
          group_size(2 * nS, sample_bytes(spec)) == 2 * nS) {
        std::vector<uint64_t> ntags((size_t)(2 * nS));
        for (int64_t j = 0; j < 2 * nS; ++j) ntags[(size_t)j] = make_tag(PHASE_R, l - 1, j);
        Ypre = merged_call(false, n, m, L() - l, nS, tags, width, smax, spec, l - 1, ntags);
        mv_cols_ += 2 * nS * spec;
      } else {
        Om = gauss(n, smax, L() - l, tags, width);
      }
      for (auto w : width) mv_cols_ += w;
    }
    const int64_t gsz = group_size(nS, sample_bytes(smax));
    BF_CHECK(!Ypre.p || gsz == nS, BF_EINVAL, "internal: merged sweep level split in groups");
    F_->R[l - lm()].assign((size_t)nb(), Block{});
    if (l == lm()) F_->B.assign((size_t)nb(), Block{});
    for (int64_t j0 = 0; j0 < nS; j0 += gsz) {
      const int64_t j1 = std::min(nS, j0 + gsz), ng = j1 - j0;
      std::vector<int64_t> seg(ng + 1);
      for (int64_t q = 0; q <= ng; ++q) seg[q] = node_lo(n, L() - l, j0 + q);
      const int64_t ycols = ng * smax;
      DevBuf<bf_c64> Y;
      if (Ypre.p) {
        Y = std::move(Ypre);
      } else {
        Y = DevBuf<bf_c64>((size_t)m * ycols, s_);
        call_op(false, Om.p, n, smax, Y.p, m, &seg);
      }

      // U^H stage (shared by the group's samples): PL rows by leaf i, stored
      // row-major (row stride ycols)
      DevBuf<bf_c128> PL((size_t)std::max<int64_t>(rowsL, 1) * ycols, s_);
      {
        std::vector<GemmDesc> d;
        for (int64_t i = 0; i < nb(); ++i) {
          const Block& U = F_->U[i];
          GemmDesc g{};
          g.out = PL.p + roffL[i] * ycols;
          g.out_ld = 1;
          g.out_rs = ycols;
          g.M = U.cols;
          g.ncols = (int32_t)ycols;
          g.nterm = 1;
          g.t[0] = GemmTerm{U.p, Y.p + node_lo(m, L(), i), m, U.rows, U.rows, 1};
          if (g.M > 0) d.push_back(g);
        }
        gemm(d, true);
      }
      Y.reset();
      // view[q] is sample j0 + q
      std::vector<Tall<bf_c128>> view(ng);
      for (int64_t q = 0; q < ng; ++q) {
        view[q].base = PL.p + q * smax;
        view[q].ld = 1;
        view[q].rs = ycols;
        view[q].roff = roffL;
      }
      std::vector<DevBuf<bf_c128>> keep;
      for (int lp = L() - 1; lp > l; --lp) {
        const int64_t nTl = int64_t(1) << lp;
        // the samples of one node jp of this stage share its R blocks and its
        // output rows: side by side as in the W sweep
        const int sh = lp - l;
        std::vector<int64_t> base(ng);
        std::vector<Tall<bf_c128>> next(ng);
        int64_t tot = 0;
        for (int64_t qa = 0; qa < ng;) {
          const int64_t jp = (j0 + qa) >> sh;
          int64_t qe = qa;
          while (qe < ng && ((j0 + qe) >> sh) == jp) ++qe;
          int64_t rows = 0;
          std::vector<int64_t> roff((size_t)nTl);
          for (int64_t i = 0; i < nTl; ++i) { roff[(size_t)i] = rows; rows += F_->ku(lp, i, jp); }
          const int64_t gw = (qe - qa) * smax;
          for (int64_t q = qa; q < qe; ++q) {
            next[q].roff = roff;
            next[q].ld = 1;                  // row-major, rows x (group width)
            next[q].rs = gw;
            base[q] = tot + (q - qa) * smax;
          }
          tot += std::max<int64_t>(rows, 1) * gw;
          qa = qe;
        }
        DevBuf<bf_c128> buf((size_t)std::max<int64_t>(tot, 1), s_);
        for (int64_t q = 0; q < ng; ++q) next[q].base = buf.p + base[q];
        std::vector<GemmDesc> d;
        for (int64_t qa = 0; qa < ng;) {
          const int64_t jp = (j0 + qa) >> sh;
          int64_t qe = qa;
          while (qe < ng && ((j0 + qe) >> sh) == jp) ++qe;
          for (int64_t i = 0; i < nTl; ++i) {
            const Block& Rb = F_->R[lp - lm()][(size_t)((i << (L() - lp)) + jp)];
            const int32_t k1 = F_->ku(lp + 1, 2 * i, jp >> 1);
            const int32_t k2 = F_->ku(lp + 1, 2 * i + 1, jp >> 1);
            GemmDesc g{};
            view_out(g, next[qa], next[qa].roff[i]);
            g.M = Rb.cols;
            g.ncols = (int32_t)((qe - qa) * smax);
            g.nterm = 2;
            g.t[0] = view_term(Rb.p, view[qa], view[qa].roff[2 * i], Rb.rows, k1);
            g.t[1] = view_term(Rb.p + k1, view[qa], view[qa].roff[2 * i + 1], Rb.rows, k2);
            if (g.M > 0) d.push_back(g);
          }
          qa = qe;
        }
        gemm(d, false);
        if (!keep.empty()) keep.erase(keep.begin());   // two stages alive at most
        keep.push_back(std::move(buf));
        view.swap(next);
        if (lp == L() - 1) PL.reset();
      }
      // Z_{l,i,j} = [P_{2i}; P_{2i+1}] of sample j  ->  R_{l,i,j}; local order
      // i * ng + (j - j0)
      std::vector<QRDesc> zq((size_t)(nT * ng));
      for (int64_t i = 0; i < nT; ++i)
        for (int64_t q = 0; q < ng; ++q) {
          const int64_t j = j0 + q;
          const int32_t M = F_->ku(l + 1, 2 * i, j >> 1) + F_->ku(l + 1, 2 * i + 1, j >> 1);
          QRDesc qd{view[q].at(view[q].roff[2 * i]), nullptr, view[q].ld, M, width[j]};
          qd.in_rs = view[q].rs;
          zq[(size_t)(i * ng + q)] = qd;
        }
      std::vector<Block> blocks;
      auto ranks = cpqr(zq, false, blocks);
      for (int64_t i = 0; i < nT; ++i)
        for (int64_t q = 0; q < ng; ++q) {
          const size_t b = (size_t)((i << (L() - l)) + j0 + q);
          F_->R[l - lm()][b] = blocks[(size_t)(i * ng + q)];
          F_->ku_ref(l, i, j0 + q) = ranks[(size_t)(i * ng + q)];
        }
      if (l == lm()) centre_blocks(Om, width, j0, j1, zq);
    }
  }

  // X_{lm,i,j} = V_{tau,nu}^H Omega_nu for the samples j in [j0, j1) of the
  // centre level, by the nested row bases: V^0 on the leaves under nu, then
  // W^1..W^{lm} restricted to nu's subtree.  view[j - j0] holds sample j's
  // X blocks (rows by i); keep owns the buffers.
  void x_chain(const DevBuf<bf_c64>& Om, const std::vector<int32_t>& width, int64_t j0, int64_t j1,
               std::vector<Tall<bf_c128>>& view, std::vector<DevBuf<bf_c128>>& keep) {
    const int64_t n = F_->n;
    const int lmv = lm();
    const int64_t ng = j1 - j0;
    // level 0 (leaves under nu): per-sample tall, blocks j' local in [0, 2^lm)
    const int64_t nl0 = int64_t(1) << lmv;
    view.assign(ng, Tall<bf_c128>{});
    std::vector<int64_t> base(ng);
    int64_t tot = 0;
    for (int64_t q = 0; q < ng; ++q) {
      const int64_t j = j0 + q;
      int64_t rows = 0;
      view[q].roff.resize(nl0);
      for (int64_t t = 0; t < nl0; ++t) {
        view[q].roff[t] = rows;
        rows += F_->kv(0, 0, (j << lmv) + t);
      }
      view[q].ld = 1;                        // row-major, rows x width
      view[q].rs = width[j];
      base[q] = tot;
      tot += std::max<int64_t>(rows, 1) * width[j];
    }
    DevBuf<bf_c128> buf0((size_t)std::max<int64_t>(tot, 1), s_);
    {
      std::vector<GemmDesc> d;
      for (int64_t q = 0; q < ng; ++q) {
        const int64_t j = j0 + q;
        view[q].base = buf0.p + base[q];
        for (int64_t t = 0; t < nl0; ++t) {
          const int64_t jl = (j << lmv) + t;
          const Block& V = F_->V[jl];
          GemmDesc g{};
          view_out(g, view[q], view[q].roff[t]);
          g.M = V.cols;
          g.ncols = width[j];
          g.nterm = 1;
          g.t[0] = GemmTerm{V.p, Om.p + node_lo(n, L(), jl), n, V.rows, V.rows, 1};
          if (g.M > 0) d.push_back(g);
        }
      }
      gemm(d, true);
    }
    keep.clear();
    keep.push_back(std::move(buf0));
    for (int lp = 1; lp <= lmv; ++lp) {
      const int64_t nTl = int64_t(1) << lp;
      const int64_t nSub = int64_t(1) << (lmv - lp);       // S-nodes of nu's subtree at S-level L-lp
      const int64_t nSubPrev = int64_t(1) << (lmv - lp + 1);
      std::vector<Tall<bf_c128>> next(ng);
      tot = 0;
      for (int64_t q = 0; q < ng; ++q) {
        const int64_t j = j0 + q;
        int64_t rows = 0;
        next[q].roff.resize(nTl * nSub);
        for (int64_t i = 0; i < nTl; ++i)
          for (int64_t t = 0; t < nSub; ++t) {
            next[q].roff[i * nSub + t] = rows;
            rows += F_->kv(lp, i, (j << (lmv - lp)) + t);
          }
        next[q].ld = 1;                      // row-major, rows x width
        next[q].rs = width[j];
        base[q] = tot;
        tot += std::max<int64_t>(rows, 1) * width[j];
      }
      DevBuf<bf_c128> buf((size_t)std::max<int64_t>(tot, 1), s_);
      std::vector<GemmDesc> d;
      for (int64_t q = 0; q < ng; ++q) {
        const int64_t j = j0 + q;
        next[q].base = buf.p + base[q];
        for (int64_t i = 0; i < nTl; ++i)
          for (int64_t t = 0; t < nSub; ++t) {
            const int64_t jj = (j << (lmv - lp)) + t;   // global S-node at S-level L-lp
            const Block& Wb = F_->W[lp][(size_t)((i << (L() - lp)) + jj)];
            const int32_t ka = F_->kv(lp - 1, i >> 1, 2 * jj);
            const int32_t kb = F_->kv(lp - 1, i >> 1, 2 * jj + 1);
            // previous level's local indices: (i >> 1, 2t) and (i >> 1, 2t + 1)
            const int64_t pa = (lp == 1) ? 2 * t : (i >> 1) * nSubPrev + 2 * t;
            GemmDesc g{};
            view_out(g, next[q], next[q].roff[i * nSub + t]);
            g.M = Wb.cols;
            g.ncols = width[j];
            g.nterm = 2;
            g.t[0] = view_term(Wb.p, view[q], view[q].roff[pa], Wb.rows, ka);
            g.t[1] = view_term(Wb.p + ka, view[q], view[q].roff[pa + 1], Wb.rows, kb);
            if (g.M > 0) d.push_back(g);
          }
      }
      gemm(d, false);
      keep.push_back(std::move(buf));
      view.swap(next);
    }
  }

  // Samples j in [j0, j1) of level l_m: X by the x-chain, then C = R^H Z and
  // B = C X^+ for the blocks (i, j).  zq holds the Z blocks in the local order
  // i * (j1 - j0) + (j - j0).
  void centre_blocks(const DevBuf<bf_c64>& Om, const std::vector<int32_t>& width, int64_t j0,
                     int64_t j1, const std::vector<QRDesc>& zq) {
    const int lmv = lm();
    const int64_t nT = int64_t(1) << lmv, ng = j1 - j0;
    std::vector<Tall<bf_c128>> view;
    std::vector<DevBuf<bf_c128>> keep;
    x_chain(Om, width, j0, j1, view, keep);
    std::vector<int64_t> coff((size_t)(nT * ng));
    int64_t tot = 0;
    // C = R^H Z (kU x s) for every block (i, j) of the group
    for (int64_t i = 0; i < nT; ++i)
      for (int64_t q = 0; q < ng; ++q) {
        coff[(size_t)(i * ng + q)] = tot;
        tot += (int64_t)F_->ku(lmv, i, j0 + q) * width[j0 + q];
      }
    DevBuf<bf_c128> C((size_t)std::max<int64_t>(tot, 1), s_);
    {
      std::vector<GemmDesc> d;
      for (int64_t i = 0; i < nT; ++i)
        for (int64_t q = 0; q < ng; ++q) {
          const size_t b = (size_t)((i << (L() - lmv)) + j0 + q);
          const size_t lb = (size_t)(i * ng + q);
          const Block& Rb = F_->R[0][b];
          GemmDesc g{};
          g.out = C.p + coff[lb];
          g.out_ld = std::max(Rb.cols, 1);
          g.M = Rb.cols;
          g.ncols = width[j0 + q];
          g.nterm = 1;
          g.t[0] = GemmTerm{Rb.p, zq[lb].in, zq[lb].in_ld, Rb.rows, Rb.rows, 1};
          g.t[0].in_rs = (int32_t)zq[lb].in_rs;
          if (g.M > 0) d.push_back(g);
        }
      gemm(d, false);
    }
    solve_b(C.p, coff, view, width, j0, j1, [&](int64_t i, int64_t) { return i; });
  }

  // B = C X^+ for the blocks (i, j), j in [j0, j1), of level l_m; C and xview
  // use the group's local order (C block i * (j1 - j0) + (j - j0), xview[j - j0]).
  template <typename IdxFn>
  void solve_b(const bf_c128* C, const std::vector<int64_t>& coff,
               const std::vector<Tall<bf_c128>>& xview, const std::vector<int32_t>& width,
               int64_t j0, int64_t j1, IdxFn xblock) {
    const int lmv = lm();
    const int64_t nT = int64_t(1) << lmv, ng = j1 - j0;
    std::vector<int64_t> boff((size_t)(nT * ng));
    int64_t tot = 0;
    for (int64_t i = 0; i < nT; ++i)
      for (int64_t q = 0; q < ng; ++q) {
        boff[(size_t)(i * ng + q)] = tot;
        tot += (int64_t)F_->ku(lmv, i, j0 + q) * F_->kv(lmv, i, j0 + q);
      }
    DevBuf<bf_c128> Bst((size_t)std::max<int64_t>(tot, 1), s_);
    std::vector<LSDesc> d;
    int32_t maxS = 0, maxK = 0;
    for (int64_t i = 0; i < nT; ++i)
      for (int64_t q = 0; q < ng; ++q) {
        const int64_t j = j0 + q;
        const size_t b = (size_t)((i << (L() - lmv)) + j), lb = (size_t)(i * ng + q);
        const int32_t ku = F_->ku(lmv, i, j), kv = F_->kv(lmv, i, j);
        F_->B[b] = Block{Bst.p + boff[lb], ku, kv};
        if (ku == 0 || kv == 0) continue;
        BF_CHECK(width[j] >= kv, BF_EINVAL, "centre sample narrower than the row rank");
        const Tall<bf_c128>& xv = xview[q];
        LSDesc ls{C + coff[lb], xv.at(xv.roff[xblock(i, j)]), Bst.p + boff[lb],
                  (int64_t)std::max(ku, 1), xv.ld, ku, kv, width[j]};
        ls.rsx = (int32_t)xv.rs;
        d.push_back(ls);
        maxS = std::max(maxS, width[j]);
        maxK = std::max(maxK, std::max(ku, kv));
      }
    if (validating())
      for (auto& x : d) {
        check_extent(x.C, ((size_t)(x.s - 1) * x.ldc + x.kU) * sizeof(bf_c128), "lsq C");
        check_extent(x.X, ((size_t)(x.s - 1) * x.ldx + (size_t)(x.kV - 1) * x.rsx + 1) *
                              sizeof(bf_c128), "lsq X");
        check_extent(x.B, (size_t)x.kU * x.kV * sizeof(bf_c128), "lsq B");
      }
    if (!d.empty()) {
      auto dd = upload(d, s_, st_);
      std::vector<double> cost(d.size());
      for (size_t b = 0; b < d.size(); ++b)
        cost[b] = (double)d[b].s * d[b].kV * (d[b].kU + d[b].kV);
      if (!round_solve(kSolveLSQ, dd.p, (int32_t)d.size(), cost, 0.0, false, nullptr,
                       solve_lds_lsq(maxS, maxK), s_))
        launch_lsq(dd.p, (int32_t)d.size(), maxS, maxK, s_);
    }
    F_->store.push_back(std::move(Bst));
  }

  // l_m = L (the row-wise factorization, and L = 0): the centre blocks sit on
  // the row leaves, B_{i,0} = (U_i^H A Omega)(V_{i,0}^H Omega)^+ with the leaf
  // column bases themselves (no R level) and the full-height row bases of the
  // x-chain.  One sample over all of S, max_i max(k_U, k_V) + p wide.
  void centre_at_leaves() {
    const int64_t m = F_->m, n = F_->n, nT = nb();
    int32_t w = 0;
    for (int64_t i = 0; i < nT; ++i) w = std::max(w, std::max(F_->ku(L(), i, 0), F_->kv(L(), i, 0)));
    check_cap(w);
    const int32_t s = w + p_;
    std::vector<int32_t> width{s};
    auto Om = gauss(n, s, 0, {make_tag(PHASE_R, L(), 0)}, width);
    DevBuf<bf_c64> Y((size_t)m * s, s_);
    call_op(false, Om.p, n, s, Y.p, m, nullptr);
    mv_cols_ += s;
    std::vector<Tall<bf_c128>> xv;
    std::vector<DevBuf<bf_c128>> keep;
    x_chain(Om, width, 0, 1, xv, keep);
    std::vector<int64_t> coff((size_t)nT);
    int64_t tot = 0;
    for (int64_t i = 0; i < nT; ++i) {
      coff[(size_t)i] = tot;
      tot += (int64_t)F_->ku(L(), i, 0) * s;
    }
    DevBuf<bf_c128> C((size_t)std::max<int64_t>(tot, 1), s_);
    std::vector<GemmDesc> d;
    for (int64_t i = 0; i < nT; ++i) {
      const Block& U = F_->U[(size_t)i];
      GemmDesc g{};
      g.out = C.p + coff[(size_t)i];
      g.out_ld = std::max(U.cols, 1);
      g.M = U.cols;
      g.ncols = s;
      g.nterm = 1;
      g.t[0] = GemmTerm{U.p, Y.p + node_lo(m, L(), i), m, U.rows, U.rows, 1};
      if (g.M > 0) d.push_back(g);
    }
    gemm(d, true);
    F_->B.assign((size_t)nT, Block{});
    solve_b(C.p, coff, xv, width, 0, 1, [](int64_t i, int64_t) { return i; });
  }

  void finalize() {
    int32_t kmax = 0;
    int64_t entries = 0;
    for (auto k : F_->kU) kmax = std::max(kmax, k);
    for (auto k : F_->kV) kmax = std::max(kmax, k);
    for (auto& b : canonical_blocks(F_)) entries += (int64_t)b.rows * b.cols;
    build_apply_plans(F_, s_);
    BF_HIP(hipStreamSynchronize(s_));
    st_.reset();
    int64_t bytes = 0;
    for (auto& b : F_->store) bytes += (int64_t)(b.n * sizeof(bf_c128));
    bytes += (int64_t)(F_->fwd.G.n + F_->adj.G.n) * (int64_t)sizeof(bf_c64);
    bf_info& I = F_->info;
    I.m = F_->m;
    I.n = F_->n;
    I.L = F_->L;
    I.lm = F_->lm;
    I.max_rank = kmax;
    I.v_iters = v_iters_;
    I.u_iters = u_iters_;
    I.merged_levels = merged_levels_;
    I.merge_misses = merge_misses_;
    I.matvec_cols = mv_cols_;
    I.rmatvec_cols = rmv_cols_;
    I.factor_entries = entries;
    I.device_bytes = bytes;
  }
};

}  // namespace

std::vector<Block> canonical_blocks(const bf_factors* F) {
  std::vector<Block> out;
  const int L = F->L, lm = F->lm;
  for (auto& b : F->U) out.push_back(b);
  for (int l = L - 1; l >= lm; --l)
    for (auto& b : F->R[l - lm]) out.push_back(b);
  for (auto& b : F->B) out.push_back(b);
  for (int l = lm; l >= 1; --l)
    for (auto& b : F->W[l]) out.push_back(b);
  for (auto& b : F->V) out.push_back(b);
  return out;
}

thread_local const void* t_exact_input = nullptr;

ExactInputScope::ExactInputScope(const void* x) : prev(t_exact_input) { t_exact_input = x; }
ExactInputScope::~ExactInputScope() { t_exact_input = prev; }
bool input_known_exact(const void* x) { return x != nullptr && x == t_exact_input; }

bf_factors* construct(bf_op_fn mv, bf_op_fn rmv, void* user, int64_t m, int64_t n, double tol,
                      int64_t leaf, const bf_opts* o, hipStream_t s) {
  Builder b(mv, rmv, user, m, n, tol, leaf, o, s);
  return b.run();
}

}  // namespace bf
