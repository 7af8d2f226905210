// Cross-request solve rounds of the request engine: the batched truncated
// pivoted QRs (Alg. 1 step 3) and centre-block least squares (Sec. 4.4) that
// the in-flight constructions reach at about the same time run as one
// persistent launch (solve_round_kernel) over a device work list of
// (request, block) items, replayed from a captured HIP graph.
//
// A construction thread that reaches a level's solves records an event on its
// stream (its inputs are then enqueued) and hands the work to the rounds
// thread, which waits a short window for the other in-flight constructions
// (at most until every registered one has handed in work), sorts the items by
// estimated cost, uploads the work list, makes its stream wait for every
// contributor's event, launches the graph of the round's LDS class and records
// each contributor's completion event; the contributor's stream waits for
// that event and goes on.  Each block runs the code of its own kernel, so
// results do not depend on the mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <thread>

#include "bf_internal.h"

namespace bf {

namespace {
thread_local SolveRounds* t_rounds = nullptr;
}

class SolveRounds {
 public:
  explicit SolveRounds(int device);
  ~SolveRounds();
  void enter();
  void leave();
  bool submit(int kind, const void* descs, int32_t n, const std::vector<double>& cost, double tol,
              bool in_c64, int32_t* ranks, size_t lds, hipStream_t s);
  int64_t rounds() const { return rounds_.load(); }
  int64_t items() const { return items_.load(); }

 private:
  struct Req {
    SolveWork w;
    int32_t n;
    const std::vector<double>* cost;
    size_t lds;
    hipEvent_t ready, done;
    bool launched = false, failed = false;
  };
  // LDS classes of the captured graphs (bytes per workgroup) and the
  // workgroups each keeps per compute unit
  static constexpr size_t kClass[4] = {32 * 1024, 64 * 1024, 96 * 1024, 160 * 1024};
  static constexpr int kPerCU[4] = {5, 2, 1, 1};
  static constexpr auto kWindow = std::chrono::microseconds(60);

  void run();
  bool ensure(size_t nworks, size_t nitems);
  void release_graphs();
  bool capture(int c);

  int device_ = 0, cus_ = 256;
  std::mutex mu_;
  std::condition_variable cv_, cv_done_;
  std::vector<Req*> pending_;
  int active_ = 0;
  bool stop_ = false;
  hipStream_t bs_ = nullptr;
  hipEvent_t up_ = nullptr;          // end of the previous round's upload
  SolveWork* works_d_ = nullptr;
  SolveItem* items_d_ = nullptr;
  int32_t* n_d_ = nullptr;
  char* host_ = nullptr;             // pinned staging of the work list
  size_t cap_works_ = 0, cap_items_ = 0;
  hipGraphExec_t exec_[4] = {nullptr, nullptr, nullptr, nullptr};
  std::atomic<int64_t> rounds_{0}, items_{0};
  std::thread th_;
};

constexpr size_t SolveRounds::kClass[4];
constexpr int SolveRounds::kPerCU[4];

SolveRounds::SolveRounds(int device) : device_(device) {
  BF_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  BF_HIP(hipGetDeviceProperties(&prop, device));
  cus_ = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  BF_HIP(hipStreamCreateWithFlags(&bs_, hipStreamNonBlocking));
  BF_HIP(hipEventCreateWithFlags(&up_, hipEventDisableTiming));
  BF_HIP(hipEventRecord(up_, bs_));
  th_ = std::thread([this] { run(); });
}

SolveRounds::~SolveRounds() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  if (th_.joinable()) th_.join();
  (void)hipStreamSynchronize(bs_);
  release_graphs();
  if (works_d_) (void)hipFree(works_d_);
  if (items_d_) (void)hipFree(items_d_);
  if (n_d_) (void)hipFree(n_d_);
  if (host_) (void)hipHostFree(host_);
  (void)hipEventDestroy(up_);
  (void)hipStreamDestroy(bs_);
}

void SolveRounds::enter() {
  std::lock_guard<std::mutex> lk(mu_);
  ++active_;
}
void SolveRounds::leave() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    --active_;
  }
  cv_.notify_all();   // a round waiting for this construction need not
}

void SolveRounds::release_graphs() {
  for (auto& e : exec_)
    if (e) {
      (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
}

// One graph per LDS class: the persistent kernel reading the fixed work-list
// buffers (so a round only refreshes their contents).
bool SolveRounds::capture(int c) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(bs_, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  bool ok = true;
  try {
    launch_solve_round(works_d_, items_d_, n_d_, cus_ * kPerCU[c], kClass[c], bs_);
  } catch (...) {
    ok = false;
  }
  if (hipStreamEndCapture(bs_, &g) != hipSuccess || !g) ok = false;
  if (ok && hipGraphInstantiate(&exec_[c], g, nullptr, nullptr, 0) != hipSuccess) {
    exec_[c] = nullptr;
    ok = false;
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  return ok;
}

// Work-list buffers of at least this capacity (reallocated, graphs recaptured
// when they grow; the previous round has finished with them by then).
bool SolveRounds::ensure(size_t nworks, size_t nitems) {
  if (nworks <= cap_works_ && nitems <= cap_items_) return true;
  if (hipStreamSynchronize(bs_) != hipSuccess) return false;
  release_graphs();
  if (works_d_) (void)hipFree(works_d_);
  if (items_d_) (void)hipFree(items_d_);
  if (host_) (void)hipHostFree(host_);
  works_d_ = nullptr;
  items_d_ = nullptr;
  host_ = nullptr;
  cap_works_ = std::max<size_t>(64, 2 * nworks);
  cap_items_ = std::max<size_t>(1 << 16, 2 * nitems);
  const size_t hb = cap_works_ * sizeof(SolveWork) + cap_items_ * sizeof(SolveItem) + 64;
  if (hipMalloc((void**)&works_d_, cap_works_ * sizeof(SolveWork)) != hipSuccess ||
      hipMalloc((void**)&items_d_, cap_items_ * sizeof(SolveItem)) != hipSuccess ||
      (!n_d_ && hipMalloc((void**)&n_d_, sizeof(int32_t)) != hipSuccess) ||
      hipHostMalloc((void**)&host_, hb, 0) != hipSuccess) {
    (void)hipGetLastError();
    cap_works_ = cap_items_ = 0;
    return false;
  }
  for (int c = 0; c < 4; ++c)
    if (!capture(c)) return false;
  return true;
}

void SolveRounds::run() {
  (void)hipSetDevice(device_);
  for (;;) {
    std::vector<Req*> batch;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || !pending_.empty(); });
      if (pending_.empty()) return;
      // let the other in-flight constructions join this round
      cv_.wait_for(lk, kWindow, [&] { return stop_ || (int)pending_.size() >= active_; });
      batch.swap(pending_);
    }
    size_t nitems = 0, lds = 0;
    for (Req* r : batch) {
      nitems += (size_t)r->n;
      lds = std::max(lds, r->lds);
    }
    int c = 0;
    while (c < 3 && kClass[c] < lds) ++c;
    bool ok = lds <= kClass[3] && nitems < (size_t)INT32_MAX && ensure(batch.size(), nitems);
    if (ok) {
      // items by estimated cost, largest first; ties in request order
      std::vector<std::pair<double, SolveItem>> order;
      order.reserve(nitems);
      for (size_t w = 0; w < batch.size(); ++w)
        for (int32_t b = 0; b < batch[w]->n; ++b)
          order.push_back({(*batch[w]->cost)[(size_t)b], SolveItem{(int32_t)w, b}});
      std::stable_sort(order.begin(), order.end(),
                       [](const auto& x, const auto& y) { return x.first > y.first; });
      ok = hipEventSynchronize(up_) == hipSuccess;   // staging free again
      if (ok) {
        SolveWork* hw = reinterpret_cast<SolveWork*>(host_);
        SolveItem* hi = reinterpret_cast<SolveItem*>(hw + cap_works_);
        int32_t* hn = reinterpret_cast<int32_t*>(hi + cap_items_);
        for (size_t w = 0; w < batch.size(); ++w) hw[w] = batch[w]->w;
        for (size_t i = 0; i < nitems; ++i) hi[i] = order[i].second;
        *hn = (int32_t)nitems;
        ok = hipMemcpyAsync(works_d_, hw, batch.size() * sizeof(SolveWork),
                            hipMemcpyHostToDevice, bs_) == hipSuccess &&
             hipMemcpyAsync(items_d_, hi, nitems * sizeof(SolveItem), hipMemcpyHostToDevice,
                            bs_) == hipSuccess &&
             hipMemcpyAsync(n_d_, hn, sizeof(int32_t), hipMemcpyHostToDevice, bs_) == hipSuccess &&
             hipEventRecord(up_, bs_) == hipSuccess;
        for (Req* r : batch) ok = ok && hipStreamWaitEvent(bs_, r->ready, 0) == hipSuccess;
        if (ok) {
          ProfScope ps(BF_KC_CPQR, bs_, 0.0, 0.0);   // the round's QRs and least squares
          ok = hipGraphLaunch(exec_[c], bs_) == hipSuccess;
        }
        for (Req* r : batch) ok = ok && hipEventRecord(r->done, bs_) == hipSuccess;
      }
    }
    if (!ok) {
      // nothing of this round may have run: make sure, then let every
      // contributor launch its own solves
      (void)hipGetLastError();
      (void)hipStreamSynchronize(bs_);
    } else {
      ++rounds_;
      items_ += (int64_t)nitems;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (Req* r : batch) {
        r->launched = ok;
        r->failed = !ok;
      }
    }
    cv_done_.notify_all();
  }
}

bool SolveRounds::submit(int kind, const void* descs, int32_t n, const std::vector<double>& cost,
                         double tol, bool in_c64, int32_t* ranks, size_t lds, hipStream_t s) {
  Req r;
  r.w = SolveWork{descs, ranks, tol, kind, in_c64 ? 1 : 0};
  r.n = n;
  r.cost = &cost;
  r.lds = lds;
  if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess) return false;
  if (hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(r.ready);
    return false;
  }
  bool ok = hipEventRecord(r.ready, s) == hipSuccess;
  if (ok) {
    std::unique_lock<std::mutex> lk(mu_);
    pending_.push_back(&r);
    cv_.notify_all();
    cv_done_.wait(lk, [&] { return r.launched || r.failed; });
    ok = r.launched;
  }
  if (ok) ok = hipStreamWaitEvent(s, r.done, 0) == hipSuccess;
  (void)hipEventDestroy(r.ready);
  (void)hipEventDestroy(r.done);
  return ok;
}

bool solve_rounds_active() { return t_rounds != nullptr; }

bool round_solve(int kind, const void* descs_dev, int32_t n, const std::vector<double>& cost,
                 double tol, bool in_c64, int32_t* ranks_dev, size_t lds, hipStream_t s) {
  SolveRounds* R = t_rounds;
  if (!R || n <= 0 || lds > solve_lds_limit() || (size_t)n > cost.size()) return false;
  return R->submit(kind, descs_dev, n, cost, tol, in_c64, ranks_dev, lds, s);
}

SolveRounds* new_solve_rounds(int device) { return new SolveRounds(device); }
void delete_solve_rounds(SolveRounds* R) { delete R; }
void solve_rounds_stats(const SolveRounds* R, int64_t* rounds, int64_t* items) {
  *rounds = R ? R->rounds() : 0;
  *items = R ? R->items() : 0;
}

RoundsScope::RoundsScope(SolveRounds* R) : R_(R), prev_(t_rounds) {
  if (!R_) return;
  R_->enter();
  t_rounds = R_;
}
RoundsScope::~RoundsScope() {
  if (!R_) return;
  t_rounds = prev_;
  R_->leave();
}

}  // namespace bf
