// C ABI of libbf: argument checks, error codes, memory utilities, factor
// import/export and the built-in black-box operators.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdlib>
#include <map>
#include <unordered_map>
#include <mutex>

#include "factors.h"

namespace bf {

bf_factors* construct(bf_op_fn mv, bf_op_fn rmv, void* user, int64_t m, int64_t n, double tol,
                      int64_t leaf, const bf_opts* o, hipStream_t s);

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

// ---- profiling --------------------------------------------------------------
namespace {
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double flops, bytes;
};
std::mutex g_prof_mu;
std::vector<ProfRec> g_prof;
std::atomic<bool> g_prof_on{false};
}  // namespace

bool profiling() { return g_prof_on.load(std::memory_order_relaxed); }

ProfScope::ProfScope(int c, hipStream_t st, double fl, double by)
    : cls(c), s(st), flops(fl), bytes(by) {
  if (!profiling()) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventRecord(a, s) != hipSuccess) a = nullptr;
}

ProfScope::~ProfScope() {
  if (!a) return;
  hipEvent_t b = nullptr;
  if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s) != hipSuccess) {
    (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(ProfRec{cls, a, b, flops, bytes});
}

// ---- memory ---------------------------------------------------------------
static std::once_flag g_pool_once[64];

bool validating() {
  static const bool on = [] {
    const char* v = std::getenv("BF_VALIDATE");
    return v && v[0] && v[0] != '0';
  }();
  return on;
}

static std::mutex g_reg_mu;
static std::map<uintptr_t, size_t> g_reg;   // live allocations (validation mode)

void check_extent(const void* p, size_t bytes, const char* what) {
  if (!validating() || bytes == 0) return;
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  std::lock_guard<std::mutex> lk(g_reg_mu);
  auto it = g_reg.upper_bound(a);
  if (it != g_reg.begin()) {
    --it;
    if (a >= it->first && a + bytes <= it->first + it->second) return;
  }
  throw Error(BF_EINVAL, std::string("bounds check failed: ") + what);
}

static std::atomic<bool> g_dev_used[64];   // devices whose pool dev_alloc has used

static void ensure_pool(int dev) {
  if (dev < 0 || dev >= 64) return;
  g_dev_used[dev].store(true);
  std::call_once(g_pool_once[dev], [dev]() {
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
}

// Device blocks that outlive the request scope that made them (factor
// storage, freed with its factors) and the spare blocks a scope holds when it
// ends are kept per device for later requests instead of going back through
// hipFreeAsync: giving back a block of ~100 MB took 3-4 ms of host time per
// call, which sat between consecutive requests.  A kept block carries an event
// recorded on the stream that freed it, waited for before the block is handed
// out again (by the new user's stream on the device, so the host never waits).
// At most kDevKeepBytes are kept per device; an allocation that fails gives
// them all back and retries, and bf_release_cached_memory gives them back on
// request.
namespace {
struct BlockInfo {
  size_t cap;
  int dev;
  UserAlloc ua;   // ua.alloc != nullptr: the block came from a caller's bf_alloc
};
std::mutex g_cap_mu;
std::unordered_map<void*, BlockInfo> g_cap;   // every block dev_alloc made
struct KeptBlock {
  void* p;
  hipEvent_t ev;   // recorded on the freeing stream, which may be gone by now
};
struct DevKeep {
  std::mutex mu;
  std::multimap<size_t, KeptBlock> blocks;   // capacity -> block
  size_t bytes = 0;
};
DevKeep g_keep[64];
constexpr size_t kDevKeepBytes = size_t(16) << 30;

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

BlockInfo block_info(void* p) {
  std::lock_guard<std::mutex> lk(g_cap_mu);
  auto it = g_cap.find(p);
  return it == g_cap.end() ? BlockInfo{0, -1, UserAlloc{}} : it->second;
}

// return p to where it came from: the caller's allocator or the device pool
void give_back(void* p, hipStream_t s) {
  UserAlloc ua{};
  {
    std::lock_guard<std::mutex> lk(g_cap_mu);
    auto it = g_cap.find(p);
    if (it != g_cap.end()) {
      ua = it->second.ua;
      g_cap.erase(it);
    }
  }
  if (ua.alloc)
    ua.free(ua.ctx, p, (void*)s);
  else
    (void)hipFreeAsync(p, s);
}

// keep p (last used on s) for reuse; false: the caller gives it back
// (blocks of a caller's allocator always go back to it)
bool keep_block(void* p, hipStream_t s) {
  const BlockInfo bi = block_info(p);
  if (bi.cap == 0 || bi.dev < 0 || bi.dev >= 64 || bi.ua.alloc || capturing(s)) return false;
  DevKeep& k = g_keep[bi.dev];
  {
    std::lock_guard<std::mutex> lk(k.mu);
    if (k.bytes + bi.cap > kDevKeepBytes) return false;
  }
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return false;
  if (hipEventRecord(ev, s) != hipSuccess) {
    (void)hipEventDestroy(ev);
    return false;
  }
  std::lock_guard<std::mutex> lk(k.mu);
  k.blocks.emplace(bi.cap, KeptBlock{p, ev});
  k.bytes += bi.cap;
  return true;
}

// Events of kept blocks handed out while their work was still pending: the
// new user's stream waits for them on the device, and they are destroyed
// once complete.
std::mutex g_retired_mu;
std::vector<hipEvent_t> g_retired;

void retire_event(hipEvent_t ev) {
  std::lock_guard<std::mutex> lk(g_retired_mu);
  for (size_t i = 0; i < g_retired.size();) {
    if (hipEventQuery(g_retired[i]) == hipSuccess) {
      (void)hipEventDestroy(g_retired[i]);
      g_retired[i] = g_retired.back();
      g_retired.pop_back();
    } else {
      ++i;
    }
  }
  if (ev) g_retired.push_back(ev);
}

// a kept block of capacity in [want, 2 want], made safe for use on s: if the
// work that last used it may still run, s waits for its event on the device
// (the host never blocks here)
void* take_kept(int dev, size_t want, hipStream_t s, size_t* cap) {
  if (dev < 0 || dev >= 64) return nullptr;
  DevKeep& k = g_keep[dev];
  KeptBlock b{nullptr, nullptr};
  {
    std::lock_guard<std::mutex> lk(k.mu);
    auto it = k.blocks.lower_bound(want);
    if (it == k.blocks.end() || it->first > 2 * want) return nullptr;
    b = it->second;
    *cap = it->first;
    k.bytes -= it->first;
    k.blocks.erase(it);
  }
  if (hipEventQuery(b.ev) == hipSuccess) {
    (void)hipEventDestroy(b.ev);
    retire_event(nullptr);
  } else if (hipStreamWaitEvent(s, b.ev, 0) == hipSuccess) {
    retire_event(b.ev);
  } else {   // no device-side wait: wait on the host rather than lose the block
    (void)hipGetLastError();
    (void)hipEventSynchronize(b.ev);
    (void)hipEventDestroy(b.ev);
  }
  return b.p;
}

// gives every kept block of dev back to the pool on stream s (live; the
// blocks' own freeing streams may have been destroyed since)
void release_kept(int dev, hipStream_t s) {
  if (dev < 0 || dev >= 64) return;
  std::multimap<size_t, KeptBlock> all;
  {
    std::lock_guard<std::mutex> lk(g_keep[dev].mu);
    all.swap(g_keep[dev].blocks);
    g_keep[dev].bytes = 0;
  }
  for (auto& kv : all) {
    (void)hipEventSynchronize(kv.second.ev);
    (void)hipEventDestroy(kv.second.ev);
    give_back(kv.second.p, s);
  }
}
}  // namespace

struct AllocScope::Cache {
  hipStream_t s = nullptr;
  std::multimap<size_t, void*> free_;          // capacity -> block
  std::unordered_map<void*, size_t> cap_;      // every block this scope allocated
  size_t free_bytes = 0;
  Staging st;
  Cache* prev = nullptr;
  void trim() {
    for (auto& kv : free_) {
      if (!keep_block(kv.second, s)) give_back(kv.second, s);
      cap_.erase(kv.second);
    }
    free_.clear();
    free_bytes = 0;
  }
};
static thread_local AllocScope::Cache* t_cache = nullptr;
static thread_local const UserAlloc* t_user = nullptr;

UseAllocator::UseAllocator(const bf_alloc* a) : prev_(t_user) {
  if (!a) return;
  BF_CHECK(a->alloc && a->free, BF_EINVAL, "bf_alloc: alloc and free are both required");
  ua_ = UserAlloc{a->ctx, a->alloc, a->free};
  t_user = &ua_;
  set_ = true;
}
UseAllocator::UseAllocator(const UserAlloc* ua) : prev_(t_user) {
  if (!ua) return;
  ua_ = *ua;
  t_user = &ua_;
  set_ = true;
}
const UserAlloc* current_user_alloc() { return t_user; }
UseAllocator::~UseAllocator() {
  if (set_) t_user = prev_;
}
// free blocks a scope may hold before it returns them to the pool
static constexpr size_t kScopeFreeLimit = size_t(8) << 30;

static size_t round_block(size_t b) {
  if (b <= 4096) return (b + 255) & ~size_t(255);
  const int e = 63 - __builtin_clzll(b);
  const size_t step = size_t(1) << (e - 3);
  return (b + step - 1) / step * step;
}

AllocScope::AllocScope(hipStream_t s) {
  if (t_cache && t_cache->s == s) return;   // join the active scope
  c_ = new Cache();
  c_->s = s;
  c_->prev = t_cache;
  t_cache = c_;
  owner_ = true;
}

AllocScope::~AllocScope() {
  if (!owner_) return;
  c_->trim();
  t_cache = c_->prev;
  delete c_;
}

Staging* scope_staging(hipStream_t s) {
  return (t_cache && t_cache->s == s) ? &t_cache->st : nullptr;
}

void* dev_alloc(size_t bytes, hipStream_t s) {
  int dev = 0;
  BF_HIP(hipGetDevice(&dev));
  ensure_pool(dev);
  void* p = nullptr;
  const size_t want = round_block(bytes);
  AllocScope::Cache* c = t_cache;
  const bool scoped = c && c->s == s;
  if (scoped) {
    auto it = c->free_.lower_bound(want);
    if (it != c->free_.end() && it->first <= 2 * want) {
      p = it->second;
      c->free_bytes -= it->first;
      c->free_.erase(it);
    }
  }
  if (!p && t_user) {   // the caller's allocator (bf_alloc) instead of the pool
    p = t_user->alloc(t_user->ctx, want, (void*)s);
    BF_CHECK(p != nullptr, BF_ENOMEM,
             "bf_alloc: the caller's allocator returned NULL for " + std::to_string(want) +
                 " bytes");
    {
      std::lock_guard<std::mutex> lk(g_cap_mu);
      g_cap[p] = BlockInfo{want, dev, *t_user};
    }
    if (scoped) c->cap_[p] = want;
  }
  if (!p && !capturing(s)) {
    size_t cap = 0;
    p = take_kept(dev, want, s, &cap);
    if (p && scoped) c->cap_[p] = cap;
  }
  if (!p) {
    if (scoped && c->free_bytes > kScopeFreeLimit) c->trim();
    hipError_t e = hipMallocAsync(&p, want, s);
    if (e != hipSuccess) {   // give the pool every spare block, retry
      (void)hipGetLastError();
      if (scoped) c->trim();
      release_kept(dev, s);
      e = hipMallocAsync(&p, want, s);
    }
    BF_HIP(e);
    {
      std::lock_guard<std::mutex> lk(g_cap_mu);
      g_cap[p] = BlockInfo{want, dev, UserAlloc{}};
    }
    if (scoped) c->cap_[p] = want;
  }
  if (validating()) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_reg[reinterpret_cast<uintptr_t>(p)] = bytes;
  }
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  if (validating()) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_reg.erase(reinterpret_cast<uintptr_t>(p));
  }
  AllocScope::Cache* c = t_cache;
  if (c && c->s == s) {
    auto it = c->cap_.find(p);
    if (it != c->cap_.end()) {
      c->free_.emplace(it->second, p);
      c->free_bytes += it->second;
      return;
    }
  }
  if (!keep_block(p, s)) give_back(p, s);
}

// Pinned host blocks shared by every Staging of the process.  A staging area
// that ends or grows hands its block back here, tagged with an event that
// completes once the copies issued from it have, and later stagings reuse the
// blocks: pinning and unpinning many MB costs milliseconds per call
// (hipHostFree also waits for the device), which would otherwise sit between
// consecutive requests.  At most kPinnedKeep blocks are kept; they stay
// pinned until bf_release_cached_memory or the end of the process.
namespace {
struct PinnedBlock {
  char* h;
  size_t cap;
  hipEvent_t done;   // null: no copy from the block can be pending
};
std::mutex g_pin_mu;
std::vector<PinnedBlock> g_pinned;
constexpr size_t kPinnedKeep = 8;

void release_pinned(char* h, size_t cap, hipStream_t s, bool synced) {
  hipEvent_t ev = nullptr;
  if (!synced) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    // a capture would make the graph read the block at replay time: keep it
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamSynchronize(s);
      ev = nullptr;
    } else if (hipEventRecord(ev, s) != hipSuccess) {
      (void)hipEventDestroy(ev);
      (void)hipStreamSynchronize(s);
      ev = nullptr;
    }
  }
  PinnedBlock drop{nullptr, 0, nullptr};
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pinned.push_back(PinnedBlock{h, cap, ev});
    if (g_pinned.size() > kPinnedKeep) {
      auto it = std::min_element(g_pinned.begin(), g_pinned.end(),
                                 [](const PinnedBlock& a, const PinnedBlock& b) { return a.cap < b.cap; });
      drop = *it;
      g_pinned.erase(it);
    }
  }
  if (drop.h) {
    if (drop.done) {
      (void)hipEventSynchronize(drop.done);
      (void)hipEventDestroy(drop.done);
    }
    (void)hipHostFree(drop.h);
  }
}

void release_all_pinned() {
  std::vector<PinnedBlock> all;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    all.swap(g_pinned);
  }
  for (auto& b : all) {
    if (b.done) {
      (void)hipEventSynchronize(b.done);
      (void)hipEventDestroy(b.done);
    }
    (void)hipHostFree(b.h);
  }
}

// the smallest kept block of at least `need` bytes, else a new one of `want`
char* acquire_pinned(size_t need, size_t want, size_t* cap) {
  PinnedBlock got{nullptr, 0, nullptr};
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    // only blocks whose copies have finished: the host writes into it next,
    // and waiting here would stall the host behind the device
    auto best = g_pinned.end();
    for (auto it = g_pinned.begin(); it != g_pinned.end(); ++it)
      if (it->cap >= need && (best == g_pinned.end() || it->cap < best->cap) &&
          (!it->done || hipEventQuery(it->done) == hipSuccess))
        best = it;
    if (best != g_pinned.end()) {
      got = *best;
      g_pinned.erase(best);
    }
  }
  if (got.h) {
    if (got.done) (void)hipEventDestroy(got.done);   // complete (queried above)
    *cap = got.cap;
    return got.h;
  }
  void* p = nullptr;
  BF_HIP(hipHostMalloc(&p, want, hipHostMallocDefault));
  *cap = want;
  return static_cast<char*>(p);
}
}  // namespace

Staging::~Staging() {
  if (h) release_pinned(h, cap, last, false);
}

void* Staging::alloc(size_t bytes, hipStream_t s) {
  const size_t need = (bytes + 255) & ~size_t(255);
  if (off + need > cap) {
    if (h) {
      // earlier copies from the old block may still be in flight
      BF_HIP(hipStreamSynchronize(last));
      release_pinned(h, cap, last, true);
      h = nullptr;
    }
    h = acquire_pinned(need, std::max<size_t>(std::max<size_t>(2 * cap, need), 1 << 20), &cap);
    off = 0;
  }
  last = s;
  void* r = h + off;
  off += need;
  return r;
}

// ---- operators --------------------------------------------------------------
struct SegCtx {
  DevBuf<double> tx, ty, tz, sx, sy, sz;   // tz, sz empty for 2D points
  int64_t m, n;
  double kk;
  int prec = BF_PREC_BF16X3;
};
struct FioCtx {
  DevBuf<double> cx;
  int64_t n;
  int prec = BF_PREC_BF16X3;
};
struct DenseCtx {
  const bf_c64* A;
  int64_t m, n, lda;
  int prec = BF_PREC_BF16X3;
};
struct FactorsCtx {
  const bf_factors* F;
};
struct ComposeCtx {
  bf_operator a1, a2;
};

enum OpKind { OP_SEG = 1, OP_FIO, OP_DENSE, OP_FACTORS, OP_COMPOSE };
struct OpHeader {
  int kind;
  void* ctx;
};

template <typename Fn>
static int guarded(Fn&& fn) {
  try {
    fn();
    return BF_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return BF_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return BF_EHIP;
  }
}

static int seg_apply(void* user, bool adj, const bf_c64* X, int64_t ldx, int64_t ncols, bf_c64* Y,
                     int64_t ldy, const int64_t* seg, int32_t nseg, void* stream) {
  return guarded([&] {
    auto* c = static_cast<SegCtx*>(static_cast<OpHeader*>(user)->ctx);
    PointSet T{c->tx.p, c->ty.p, c->tz.p}, S{c->sx.p, c->sy.p, c->sz.p};
    if (!adj)
      launch_segkernel(c->prec, T, c->m, S, c->n, c->kk, +1, X, ldx, ncols, Y, ldy, seg, nseg,
                       (hipStream_t)stream);
    else
      launch_segkernel(c->prec, S, c->n, T, c->m, c->kk, -1, X, ldx, ncols, Y, ldy, seg, nseg,
                       (hipStream_t)stream);
  });
}
static int seg_mv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                  const int64_t* seg, int32_t nseg, void* st) {
  return seg_apply(u, false, X, ldx, nc, Y, ldy, seg, nseg, st);
}
static int seg_rmv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                   const int64_t* seg, int32_t nseg, void* st) {
  return seg_apply(u, true, X, ldx, nc, Y, ldy, seg, nseg, st);
}

static int fio_apply(void* user, int adj, const bf_c64* X, int64_t ldx, int64_t ncols, bf_c64* Y,
                     int64_t ldy, const int64_t* seg, int32_t nseg, void* stream) {
  return guarded([&] {
    auto* c = static_cast<FioCtx*>(static_cast<OpHeader*>(user)->ctx);
    launch_fio(c->prec, c->n, c->cx.p, adj, X, ldx, ncols, Y, ldy, seg, nseg, (hipStream_t)stream);
  });
}
static int fio_mv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                  const int64_t* seg, int32_t nseg, void* st) {
  return fio_apply(u, 0, X, ldx, nc, Y, ldy, seg, nseg, st);
}
static int fio_rmv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                   const int64_t* seg, int32_t nseg, void* st) {
  return fio_apply(u, 1, X, ldx, nc, Y, ldy, seg, nseg, st);
}

static int dense_apply(void* user, int adj, const bf_c64* X, int64_t ldx, int64_t ncols,
                       bf_c64* Y, int64_t ldy, const int64_t* seg, int32_t nseg, void* stream) {
  return guarded([&] {
    auto* c = static_cast<DenseCtx*>(static_cast<OpHeader*>(user)->ctx);
    launch_dense(c->prec, c->A, c->m, c->n, c->lda, adj, X, ldx, ncols, Y, ldy, seg, nseg,
                 (hipStream_t)stream);
  });
}
static int dense_mv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                    const int64_t* seg, int32_t nseg, void* st) {
  return dense_apply(u, 0, X, ldx, nc, Y, ldy, seg, nseg, st);
}
static int dense_rmv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                     const int64_t* seg, int32_t nseg, void* st) {
  return dense_apply(u, 1, X, ldx, nc, Y, ldy, seg, nseg, st);
}

// Segment-stacked input for an operator that only has plain products: expand
// X into the block-diagonal nrows x (nseg*ncols) matrix, then multiply.
static void expand(const bf_c64* X, int64_t ldx, int64_t rows, int64_t ncols, const int64_t* seg,
                   int32_t nseg, DevBuf<bf_c64>& out, hipStream_t s) {
  std::vector<int64_t> sv(seg, seg + nseg + 1);
  DevBuf<int64_t> sd(sv.size(), s);
  if (Staging* st = scope_staging(s)) {   // pinned: no wait for the stream to drain
    void* h = st->alloc(sv.size() * sizeof(int64_t), s);
    std::memcpy(h, sv.data(), sv.size() * sizeof(int64_t));
    BF_HIP(hipMemcpyAsync(sd.p, h, sv.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  } else {
    BF_HIP(hipMemcpyAsync(sd.p, sv.data(), sv.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  }
  out = DevBuf<bf_c64>((size_t)rows * nseg * ncols, s);
  launch_expand_segments(X, ldx, rows, ncols, sd.p, nseg, out.p, rows, s);
}

static int factors_apply(void* user, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
                         bf_c64* Y, int64_t ldy, const int64_t* seg, int32_t nseg, void* stream) {
  return guarded([&] {
    auto* c = static_cast<FactorsCtx*>(static_cast<OpHeader*>(user)->ctx);
    hipStream_t s = (hipStream_t)stream;
    const int64_t rows_in = trans ? c->F->m : c->F->n;
    if (!seg) {
      apply_factors(c->F, trans, X, ldx, ncols, Y, ldy, s);
      return;
    }
    const ApplyPlan& P = trans ? c->F->adj : c->F->fwd;
    // segments that are nodes of the input-side tree: the stages that keep
    // them apart run once on X, later ones on windows of the segments below
    // each node, the rest on the expansion (each phase two intermediates of
    // 8 tmp_rows bytes per column, at most 8 GiB; both phases' buffers are
    // alive at the end)
    const int64_t tree_cols =
        std::max<int64_t>(ncols, (int64_t)((double)(int64_t(8) << 30) / (16.0 * (double)P.tmp_rows)));
    if (apply_structured(c->F, trans, X, ldx, ncols, Y, ldy, seg, nseg, tree_cols, s))
      return;
    // other segments in chunks: the expanded input and the apply's two
    // intermediates take 8 (rows_in + 2 tmp_rows) bytes per expanded column;
    // keep them under 4 GiB per chunk
    const double per_col = 8.0 * (double)(rows_in + 2 * P.tmp_rows);
    const int64_t max_cols = std::max<int64_t>(ncols, (int64_t)((double)(int64_t(4) << 30) / per_col));
    const int32_t per_chunk = (int32_t)std::max<int64_t>(1, max_cols / std::max<int64_t>(ncols, 1));
    for (int32_t g0 = 0; g0 < nseg; g0 += per_chunk) {
      const int32_t ng = std::min(per_chunk, nseg - g0);
      DevBuf<bf_c64> Xe;
      expand(X, ldx, rows_in, ncols, seg + g0, ng, Xe, s);
      apply_factors(c->F, trans, Xe.p, rows_in, (int64_t)ng * ncols, Y + (int64_t)g0 * ncols * ldy,
                    ldy, s);
    }
  });
}
static int factors_mv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                      const int64_t* seg, int32_t nseg, void* st) {
  return factors_apply(u, 0, X, ldx, nc, Y, ldy, seg, nseg, st);
}
static int factors_rmv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                       const int64_t* seg, int32_t nseg, void* st) {
  return factors_apply(u, 1, X, ldx, nc, Y, ldy, seg, nseg, st);
}

static int compose_apply(void* user, int adj, const bf_c64* X, int64_t ldx, int64_t ncols,
                         bf_c64* Y, int64_t ldy, const int64_t* seg, int32_t nseg, void* stream) {
  auto* c = static_cast<ComposeCtx*>(static_cast<OpHeader*>(user)->ctx);
  int rc = BF_OK;
  int rc2 = guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    const int64_t k = c->a1.n;   // inner dimension
    const int64_t tcols = seg ? (int64_t)nseg * ncols : ncols;
    DevBuf<bf_c64> T((size_t)k * tcols, s);
    if (!adj) {
      rc = c->a2.matvec(c->a2.user, X, ldx, ncols, T.p, k, seg, nseg, stream);
      if (rc) return;
      rc = c->a1.matvec(c->a1.user, T.p, k, tcols, Y, ldy, nullptr, 0, stream);
    } else {
      rc = c->a1.rmatvec(c->a1.user, X, ldx, ncols, T.p, k, seg, nseg, stream);
      if (rc) return;
      rc = c->a2.rmatvec(c->a2.user, T.p, k, tcols, Y, ldy, nullptr, 0, stream);
    }
  });
  return rc2 != BF_OK ? rc2 : rc;
}
static int compose_mv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                      const int64_t* seg, int32_t nseg, void* st) {
  return compose_apply(u, 0, X, ldx, nc, Y, ldy, seg, nseg, st);
}
static int compose_rmv(void* u, const bf_c64* X, int64_t ldx, int64_t nc, bf_c64* Y, int64_t ldy,
                       const int64_t* seg, int32_t nseg, void* st) {
  return compose_apply(u, 1, X, ldx, nc, Y, ldy, seg, nseg, st);
}

bool entrywise_operator(bf_op_fn mv, bf_op_fn rmv) {
  return (mv == seg_mv && rmv == seg_rmv) || (mv == fio_mv && rmv == fio_rmv) ||
         (mv == dense_mv && rmv == dense_rmv);
}

bool builtin_operator(bf_op_fn mv, bf_op_fn rmv, void* user) {
  if (entrywise_operator(mv, rmv) || (mv == factors_mv && rmv == factors_rmv)) return true;
  if (mv == compose_mv && rmv == compose_rmv) {
    auto* c = static_cast<ComposeCtx*>(static_cast<OpHeader*>(user)->ctx);
    return builtin_operator(c->a1.matvec, c->a1.rmatvec, c->a1.user) &&
           builtin_operator(c->a2.matvec, c->a2.rmatvec, c->a2.user);
  }
  return false;
}

static void check_device() {
  int dev = 0;
  hipDeviceProp_t prop;
  BF_CHECK(hipGetDevice(&dev) == hipSuccess, BF_ENOTSUP, "no HIP device");
  BF_HIP(hipGetDeviceProperties(&prop, dev));
  BF_CHECK(std::string(prop.gcnArchName).rfind("gfx950", 0) == 0, BF_ENOTSUP,
           std::string("libbf is built for gfx950, device is ") + prop.gcnArchName);
}

}  // namespace bf

using namespace bf;

extern "C" {

const char* bf_strerror(int code) {
  switch (code) {
    case BF_OK: return "success";
    case BF_EINVAL: return "invalid argument";
    case BF_ENOMEM: return "out of memory";
    case BF_ECALLBACK: return "black-box callback failed";
    case BF_ERANK: return "rank cap exceeded or block too large";
    case BF_EHIP: return "HIP runtime error";
    case BF_ENOTSUP: return "unsupported device";
    default: return "unknown error";
  }
}

const char* bf_last_error(void) { return g_last_error.c_str(); }

int bf_profile_start(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof) {
    (void)hipEventSynchronize(r.b);
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  g_prof_on = true;
  return BF_OK;
}

int bf_profile_stop(bf_kernel_stats* out) {
  g_prof_on = false;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  bf_kernel_stats acc[BF_KC_COUNT] = {};
  int rc = BF_OK;
  for (auto& r : g_prof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      rc = BF_EHIP;
    if (r.cls >= 0 && r.cls < BF_KC_COUNT) {
      acc[r.cls].launches += 1;
      acc[r.cls].ms += ms;
      acc[r.cls].flops += r.flops;
      acc[r.cls].bytes += r.bytes;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  if (out)
    for (int k = 0; k < BF_KC_COUNT; ++k) out[k] = acc[k];
  return rc;
}

int bf_construct(bf_op_fn matvec, bf_op_fn rmatvec, void* user, int64_t m, int64_t n, double tol,
                 int64_t leaf, const bf_opts* opts, const bf_alloc* alloc, void* stream,
                 bf_factors** out) {
  if (!matvec || !rmatvec || !out || m <= 0 || n <= 0 || !(tol > 0.0 && tol < 1.0) || leaf < 1 ||
      (alloc && (!alloc->alloc || !alloc->free))) {
    set_last_error("bf_construct: invalid argument");
    return BF_EINVAL;
  }
  bf_factors* F = nullptr;
  int rc = guarded([&] {
    check_device();
    UseAllocator ua(alloc);
    AllocScope scope((hipStream_t)stream);
    F = construct(matvec, rmatvec, user, m, n, tol, leaf, opts, (hipStream_t)stream);
  });
  if (rc == BF_OK) *out = F;
  return rc;
}

int bf_apply(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx, int64_t ncols,
             bf_c64* Y, int64_t ldy, const bf_alloc* alloc, void* stream) {
  if (!F || !X || !Y || ncols < 0 || (trans != 0 && trans != 1)) return BF_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->free)) return BF_EINVAL;
  const int64_t rin = trans ? F->m : F->n, rout = trans ? F->n : F->m;
  if (ldx < rin || ldy < rout) return BF_EINVAL;
  return guarded([&] {
    UseAllocator ua(alloc);
    AllocScope scope((hipStream_t)stream);
    apply_factors(F, trans, X, ldx, ncols, Y, ldy, (hipStream_t)stream);
  });
}

int bf_apply_noalloc(const bf_factors* F, int trans, const bf_c64* X, int64_t ldx,
                     int64_t ncols, bf_c64* Y, int64_t ldy, void* stream) {
  if (!F || !X || !Y || ncols < 0 || (trans != 0 && trans != 1)) return BF_EINVAL;
  const int64_t rin = trans ? F->m : F->n, rout = trans ? F->n : F->m;
  if (ldx < rin || ldy < rout) return BF_EINVAL;
  return guarded([&] { apply_noalloc(F, trans, X, ldx, ncols, Y, ldy, (hipStream_t)stream); });
}

int64_t bf_apply_noalloc_scratch_bytes(void) { return (int64_t)noalloc_scratch_bytes(); }

int bf_set_apply_fusion(bf_factors* F, int enable) {
  if (!F || (enable != 0 && enable != 1)) return BF_EINVAL;
  F->apply_fuse = enable;
  return BF_OK;
}

int bf_set_apply_precision(bf_factors* F, int precision) {
  if (!F || (precision != BF_PREC_FP32 && precision != BF_PREC_BF16X3)) return BF_EINVAL;
  F->apply_prec = precision;
  return BF_OK;
}

int bf_set_apply_graph_cols(bf_factors* F, int64_t max_cols) {
  if (!F || max_cols < 0) return BF_EINVAL;
  return guarded([&] {
    if (max_cols > 0 && !F->graphs) F->graphs = new_apply_graph_cache();
    F->graph_cols = max_cols;
  });
}

int bf_stats(const bf_factors* F, bf_info* info) {
  if (!F || !info) return BF_EINVAL;
  *info = F->info;
  info->apply_graphs = apply_graph_count(F);
  info->fused_launches = (int32_t)F->fwd.segs.size();
  return BF_OK;
}

int bf_ranks(const bf_factors* F, int32_t* kU, int32_t* kV) {
  if (!F) return BF_EINVAL;
  if (kU) std::copy(F->kU.begin(), F->kU.end(), kU);
  if (kV) std::copy(F->kV.begin(), F->kV.end(), kV);
  return BF_OK;
}

int bf_export(const bf_factors* F, bf_c128* data, int64_t* count) {
  if (!F || !count) return BF_EINVAL;
  auto blocks = canonical_blocks(F);
  int64_t tot = 0;
  for (auto& b : blocks) tot += (int64_t)b.rows * b.cols;
  if (!data) {
    *count = tot;
    return BF_OK;
  }
  if (*count < tot) return BF_EINVAL;
  int rc = guarded([&] {
    hipStream_t s = nullptr;
    BF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    try {
      std::vector<PackDesc> d;
      int64_t off = 0;
      for (auto& b : blocks) {
        if ((int64_t)b.rows * b.cols > 0)
          d.push_back(PackDesc{b.p, off, b.rows, 0, b.rows, b.cols, 0, 1, b.rows, 0});
        off += (int64_t)b.rows * b.cols;
      }
      {
        DevBuf<bf_c128> arena((size_t)std::max<int64_t>(tot, 1), s);
        Staging st;
        for (size_t o = 0; o < d.size(); o += 60000) {
          size_t cnt = std::min<size_t>(60000, d.size() - o);
          std::vector<PackDesc> part(d.begin() + o, d.begin() + o + cnt);
          auto dd = upload(part, s, st);
          launch_pack_c128(dd.p, (int32_t)cnt, arena.p, s);
        }
        if (tot > 0)
          BF_HIP(hipMemcpyAsync(data, arena.p, tot * sizeof(bf_c128), hipMemcpyDeviceToHost, s));
        BF_HIP(hipStreamSynchronize(s));
      }
      BF_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
      throw;
    }
    BF_HIP(hipStreamDestroy(s));
  });
  if (rc == BF_OK) *count = tot;
  return rc;
}

int bf_import(int64_t m, int64_t n, int64_t leaf, const int32_t* kU, const int32_t* kV,
              const bf_c128* data, int64_t count, const bf_alloc* alloc, void* stream,
              bf_factors** out) {
  if (m <= 0 || n <= 0 || leaf < 1 || !kU || !kV || !out || (count > 0 && !data)) return BF_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->free)) return BF_EINVAL;
  bf_factors* F = new (std::nothrow) bf_factors();
  if (!F) return BF_ENOMEM;
  int rc = guarded([&] {
    check_device();
    UseAllocator ua(alloc);
    hipStream_t s = (hipStream_t)stream;
    F->m = m;
    F->n = n;
    F->leaf = leaf;
    F->L = num_levels(m, n, leaf);
    F->lm = F->L / 2;
    BF_CHECK(F->L <= 24, BF_EINVAL, "too many levels");
    BF_HIP(hipGetDevice(&F->device));
    const int L = F->L, lm = F->lm;
    const size_t nb = size_t(1) << L;
    F->kU.assign(kU, kU + (size_t)(L - lm + 1) * nb);
    F->kV.assign(kV, kV + (size_t)(lm + 1) * nb);
    for (auto k : F->kU) BF_CHECK(k >= 0, BF_EINVAL, "negative rank");
    for (auto k : F->kV) BF_CHECK(k >= 0, BF_EINVAL, "negative rank");
    // shapes in canonical order
    std::vector<std::pair<int32_t, int32_t>> shp;
    for (size_t i = 0; i < nb; ++i) shp.push_back({(int32_t)node_size(m, L, i), F->ku(L, i, 0)});
    for (int l = L - 1; l >= lm; --l)
      for (int64_t i = 0; i < (int64_t(1) << l); ++i)
        for (int64_t j = 0; j < (int64_t(1) << (L - l)); ++j)
          shp.push_back({F->ku(l + 1, 2 * i, j >> 1) + F->ku(l + 1, 2 * i + 1, j >> 1), F->ku(l, i, j)});
    for (int64_t i = 0; i < (int64_t(1) << lm); ++i)
      for (int64_t j = 0; j < (int64_t(1) << (L - lm)); ++j) shp.push_back({F->ku(lm, i, j), F->kv(lm, i, j)});
    for (int l = lm; l >= 1; --l)
      for (int64_t i = 0; i < (int64_t(1) << l); ++i)
        for (int64_t j = 0; j < (int64_t(1) << (L - l)); ++j)
          shp.push_back({F->kv(l - 1, i >> 1, 2 * j) + F->kv(l - 1, i >> 1, 2 * j + 1), F->kv(l, i, j)});
    for (size_t j = 0; j < nb; ++j) shp.push_back({(int32_t)node_size(n, L, j), F->kv(0, 0, j)});
    int64_t tot = 0;
    for (auto& p : shp) tot += (int64_t)p.first * p.second;
    BF_CHECK(tot == count, BF_EINVAL, "data size does not match the ranks");
    DevBuf<bf_c128> buf((size_t)std::max<int64_t>(tot, 1), s);
    if (tot > 0) BF_HIP(hipMemcpyAsync(buf.p, data, tot * sizeof(bf_c128), hipMemcpyHostToDevice, s));
    BF_HIP(hipStreamSynchronize(s));
    std::vector<Block> blocks;
    int64_t off = 0;
    for (auto& p : shp) {
      blocks.push_back(Block{buf.p + off, p.first, p.second});
      off += (int64_t)p.first * p.second;
    }
    size_t q = 0;
    F->U.assign(blocks.begin(), blocks.begin() + nb);
    q = nb;
    F->R.assign(L - lm, {});
    for (int l = L - 1; l >= lm; --l) {
      size_t cnt = nb;
      F->R[l - lm].assign(blocks.begin() + q, blocks.begin() + q + cnt);
      q += cnt;
    }
    F->B.assign(blocks.begin() + q, blocks.begin() + q + nb);
    q += nb;
    F->W.assign(lm + 1, {});
    for (int l = lm; l >= 1; --l) {
      F->W[l].assign(blocks.begin() + q, blocks.begin() + q + nb);
      q += nb;
    }
    F->V.assign(blocks.begin() + q, blocks.begin() + q + nb);
    F->store.push_back(std::move(buf));
    build_apply_plans(F, s);
    int32_t kmax = 0;
    for (auto k : F->kU) kmax = std::max(kmax, k);
    for (auto k : F->kV) kmax = std::max(kmax, k);
    F->info.m = m;
    F->info.n = n;
    F->info.L = L;
    F->info.lm = lm;
    F->info.max_rank = kmax;
    F->info.factor_entries = tot;
    F->info.device_bytes = tot * (int64_t)sizeof(bf_c128) +
                           (int64_t)(F->fwd.G.n + F->adj.G.n) * (int64_t)sizeof(bf_c64);
  });
  if (rc != BF_OK) {
    delete F;
    return rc;
  }
  *out = F;
  return BF_OK;
}

int bf_release_cached_memory(void) {
  return guarded([&] {
    int cur = 0;
    BF_HIP(hipGetDevice(&cur));
    int ndev = 0;
    BF_HIP(hipGetDeviceCount(&ndev));
    for (int dev = 0; dev < ndev && dev < 64; ++dev) {
      if (!g_dev_used[dev].load()) continue;
      BF_HIP(hipSetDevice(dev));
      release_kept(dev, nullptr);
      BF_HIP(hipDeviceSynchronize());
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) BF_HIP(hipMemPoolTrimTo(pool, 0));
    }
    BF_HIP(hipSetDevice(cur));
    release_all_pinned();
  });
}

int bf_free(bf_factors* F, void* stream) {
  if (!F) return BF_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (!s) {
    // the null stream does not order work on non-blocking streams: wait for
    // everything on the factors' device before their blocks can be reused
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(F->device) == hipSuccess) {
      (void)hipDeviceSynchronize();
      (void)hipSetDevice(cur);
    }
  }
  for (auto& b : F->store) b.s = s;
  for (auto* P : {&F->fwd, &F->adj}) {
    P->G.s = s;
    P->blks.s = s;
    P->rows.s = s;
  }
  delete F;
  return BF_OK;
}

int bf_gauss(uint64_t seed, uint64_t tag, int64_t row0, int64_t rows, int64_t cols,
             bf_c128* out, void* stream) {
  if (rows < 0 || cols < 0 || cols > 65535 || row0 < 0 || (!out && rows * cols > 0)) return BF_EINVAL;
  return guarded([&] { launch_gauss_f64(out, rows, cols, row0, tag, seed, (hipStream_t)stream); });
}

int bf_cpqr_batched(int32_t nblk, const int32_t* M, const int32_t* N, const bf_c128* Z,
                    const int64_t* zoff, double tol, bf_c128* Q, const int64_t* qoff,
                    int32_t* ranks, void* stream) {
  if (nblk < 0 || (nblk > 0 && (!M || !N || !Z || !zoff || !Q || !qoff || !ranks)) ||
      !(tol >= 0.0 && tol < 1.0))
    return BF_EINVAL;
  return guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    std::vector<QRDesc> d(nblk);
    int maxM = 0, maxN = 0;
    for (int b = 0; b < nblk; ++b) {
      BF_CHECK(M[b] >= 0 && N[b] >= 0, BF_EINVAL, "negative block size");
      d[b] = QRDesc{Z + zoff[b], Q + qoff[b], std::max(M[b], 1), M[b], N[b]};
      maxM = std::max(maxM, M[b]);
      maxN = std::max(maxN, N[b]);
    }
    Staging st;
    auto dd = upload(d, s, st);
    DevBuf<int32_t> rk((size_t)std::max(nblk, 1), s);
    launch_cpqr(dd.p, nblk, maxM, maxN, tol, false, rk.p, s);
    if (nblk > 0)
      BF_HIP(hipMemcpyAsync(ranks, rk.p, nblk * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BF_HIP(hipStreamSynchronize(s));
  });
}

int bf_lsq_batched(int32_t nblk, const int32_t* kU, const int32_t* kV, const int32_t* s_,
                   const bf_c128* C, const int64_t* coff, const bf_c128* X, const int64_t* xoff,
                   bf_c128* B, const int64_t* boff, void* stream) {
  if (nblk < 0 || (nblk > 0 && (!kU || !kV || !s_ || !C || !coff || !X || !xoff || !B || !boff)))
    return BF_EINVAL;
  return guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    std::vector<LSDesc> d;
    int maxS = 0, maxK = 0;
    for (int b = 0; b < nblk; ++b) {
      BF_CHECK(kU[b] >= 0 && kV[b] >= 0 && s_[b] >= kV[b], BF_EINVAL, "bad least-squares block");
      if (kU[b] == 0 || kV[b] == 0) continue;
      d.push_back(LSDesc{C + coff[b], X + xoff[b], B + boff[b], kU[b], kV[b], kU[b], kV[b], s_[b]});
      maxS = std::max(maxS, s_[b]);
      maxK = std::max(maxK, std::max(kU[b], kV[b]));
    }
    Staging st;
    auto dd = upload(d, s, st);
    launch_lsq(dd.p, (int32_t)d.size(), maxS, maxK, s);
    BF_HIP(hipStreamSynchronize(s));
  });
}

// ---- built-in operators -----------------------------------------------------

// One coordinate of `dim`-dimensional row-major host points -> device array.
static DevBuf<double> coord_to_device(const double* pts, int64_t npts, int dim, int d) {
  std::vector<double> v(npts);
  for (int64_t i = 0; i < npts; ++i) v[i] = pts[dim * i + d];
  DevBuf<double> b(npts, nullptr);
  BF_HIP(hipMemcpy(b.p, v.data(), npts * 8, hipMemcpyHostToDevice));
  return b;
}

static int op_pointkernel(const double* targets, int64_t m, const double* sources, int64_t n,
                          double k, int dim, bf_operator* out) {
  if (!targets || !sources || m <= 0 || n <= 0 || !out || !std::isfinite(k)) return BF_EINVAL;
  return guarded([&] {
    check_device();
    auto* c = new SegCtx();
    try {
      c->tx = coord_to_device(targets, m, dim, 0);
      c->ty = coord_to_device(targets, m, dim, 1);
      c->sx = coord_to_device(sources, n, dim, 0);
      c->sy = coord_to_device(sources, n, dim, 1);
      if (dim == 3) {
        c->tz = coord_to_device(targets, m, dim, 2);
        c->sz = coord_to_device(sources, n, dim, 2);
      }
      c->m = m;
      c->n = n;
      c->kk = k / (2.0 * M_PI);
    } catch (...) {
      delete c;
      throw;
    }
    out->matvec = seg_mv;
    out->rmatvec = seg_rmv;
    out->user = new OpHeader{OP_SEG, c};
    out->m = m;
    out->n = n;
  });
}

int bf_op_segkernel(const double* targets, int64_t m, const double* sources, int64_t n, double k,
                    bf_operator* out) {
  return op_pointkernel(targets, m, sources, n, k, 2, out);
}

int bf_op_helmholtz3d(const double* targets, int64_t m, const double* sources, int64_t n,
                      double k, bf_operator* out) {
  return op_pointkernel(targets, m, sources, n, k, 3, out);
}

int bf_op_fio(int64_t n, bf_operator* out) {
  if (n <= 0 || (n & 1) || !out) return BF_EINVAL;
  return guarded([&] {
    check_device();
    auto* c = new FioCtx();
    std::vector<double> cx(n);
    for (int64_t j = 0; j < n; ++j) cx[j] = (2.0 + std::sin(2.0 * M_PI * (double)j / (double)n)) / 16.0;
    c->cx = DevBuf<double>(n, nullptr);
    BF_HIP(hipMemcpy(c->cx.p, cx.data(), n * 8, hipMemcpyHostToDevice));
    c->n = n;
    out->matvec = fio_mv;
    out->rmatvec = fio_rmv;
    out->user = new OpHeader{OP_FIO, c};
    out->m = out->n = n;
  });
}

int bf_op_dense(const bf_c64* A, int64_t m, int64_t n, int64_t lda, bf_operator* out) {
  if (!A || m <= 0 || n <= 0 || lda < m || !out) return BF_EINVAL;
  out->matvec = dense_mv;
  out->rmatvec = dense_rmv;
  out->user = new OpHeader{OP_DENSE, new DenseCtx{A, m, n, lda, BF_PREC_BF16X3}};
  out->m = m;
  out->n = n;
  return BF_OK;
}

int bf_op_factors(const bf_factors* F, bf_operator* out) {
  if (!F || !out) return BF_EINVAL;
  out->matvec = factors_mv;
  out->rmatvec = factors_rmv;
  out->user = new OpHeader{OP_FACTORS, new FactorsCtx{F}};
  out->m = F->m;
  out->n = F->n;
  return BF_OK;
}

int bf_op_compose(const bf_operator* a1, const bf_operator* a2, bf_operator* out) {
  if (!a1 || !a2 || !out || a1->n != a2->m) return BF_EINVAL;
  out->matvec = compose_mv;
  out->rmatvec = compose_rmv;
  out->user = new OpHeader{OP_COMPOSE, new ComposeCtx{*a1, *a2}};
  out->m = a1->m;
  out->n = a2->n;
  return BF_OK;
}

int bf_set_autotune(int enable) {
  set_autotune(enable);
  return BF_OK;
}

int bf_autotune_entries(int64_t* entries) {
  if (!entries) return BF_EINVAL;
  *entries = autotune_entries();
  return BF_OK;
}

int bf_autotune_save(const char* path) {
  return guarded([&] {
    BF_CHECK(tune_save(path) == BF_OK, BF_EINVAL, "bf_autotune_save: cannot write the table");
  });
}

int bf_autotune_load(const char* path) {
  return guarded([&] {
    BF_CHECK(tune_load(path) == BF_OK, BF_EINVAL, "bf_autotune_load: cannot read the table");
  });
}

int bf_autotune_clear(void) {
  tune_clear();
  return BF_OK;
}

int bf_op_set_precision(bf_operator* op, int precision) {
  if (!op || !op->user || (precision != BF_PREC_FP64 && precision != BF_PREC_BF16X3))
    return BF_EINVAL;
  auto* h = static_cast<OpHeader*>(op->user);
  switch (h->kind) {
    case OP_SEG: static_cast<SegCtx*>(h->ctx)->prec = precision; return BF_OK;
    case OP_FIO: static_cast<FioCtx*>(h->ctx)->prec = precision; return BF_OK;
    case OP_DENSE: static_cast<DenseCtx*>(h->ctx)->prec = precision; return BF_OK;
    default: return BF_EINVAL;
  }
}

int bf_operator_destroy(bf_operator* op) {
  if (!op || !op->user) return BF_EINVAL;
  auto* h = static_cast<OpHeader*>(op->user);
  switch (h->kind) {
    case OP_SEG: delete static_cast<SegCtx*>(h->ctx); break;
    case OP_FIO: delete static_cast<FioCtx*>(h->ctx); break;
    case OP_DENSE: delete static_cast<DenseCtx*>(h->ctx); break;
    case OP_FACTORS: delete static_cast<FactorsCtx*>(h->ctx); break;
    case OP_COMPOSE: delete static_cast<ComposeCtx*>(h->ctx); break;
    default: return BF_EINVAL;
  }
  delete h;
  op->user = nullptr;
  return BF_OK;
}

}  // extern "C"
