// Request engine: constructions (Alg. 2) and applies against resident factors,
// run concurrently on a fixed set of device slots.
//
// * Each slot is a host worker thread with its own HIP stream; a request runs
//   on the stream of the slot that admitted it, so the kernels of different
//   requests overlap on the device while each request's host-side level syncs
//   only block its own slot.
// * Admission: a request enters a slot when one is idle and its estimated
//   device footprint fits under the budget next to the requests in flight
//   (first fit in arrival order; a request passed over 8 times blocks later
//   ones until it fits, so large requests are not starved).
// * Applies wait for the construction they reference; factors stay resident
//   until their ticket is released.
// * Results do not depend on the mix: the random matrices are keyed by the
//   request's own seed and every reduction has a fixed order.  With
//   continuous batching on (batch_cols > 0), queued applies against the same
//   factors share one product: their results follow the merged width.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "factors.h"

namespace bf {
bf_factors* construct(bf_op_fn mv, bf_op_fn rmv, void* user, int64_t m, int64_t n, double tol,
                      int64_t leaf, const bf_opts* o, hipStream_t s);
}

using namespace bf;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  int kind = 0;   // 0 construct, 1 apply
  // construct
  bf_operator op{};
  double tol = 0;
  int64_t leaf = 0;
  bf_opts opts{};
  bool has_opts = false;
  // apply
  int64_t target = 0;
  int trans = 0;
  const bf_c64* X = nullptr;
  bf_c64* Y = nullptr;
  int64_t ldx = 0, ldy = 0, ncols = 0;
  // bookkeeping
  int64_t footprint = 0;
  int skipped = 0;
  Clock::time_point arrival, start, finish;
  int status = 1;          // 1 pending, 2 running, 0 / <0 done
  int batch = 1;           // applies merged into this request's product
  bf_factors* F = nullptr; // construct result
  std::string error;
};

// Device bytes a construction may hold at its peak: the factors plus the
// widest level's samples, black-box output and chain buffers.  Ranks are not
// known before the run; 40 is above every rank the built-in operators show at
// 4..16 points per wavelength and tolerances >= 1e-7.
int64_t construct_footprint(int64_t m, int64_t n, int64_t leaf) {
  const int L = num_levels(m, n, leaf);
  const double big = (double)std::max(m, n);
  const double r = 40.0, s = 2.0 * r + 2.0;
  const double half = std::ldexp(1.0, (L + 1) / 2);          // samples of the widest level
  const double samples = big * s * 8.0 * (1.0 + half);       // random block + black-box output
  const double chains = 2.0 * r * (double)(int64_t(1) << L) * half * s * 16.0 / 2.0;
  const double factors = 16.0 * r * big * (2.0 + 2.0 * (L + 1));
  return (int64_t)(samples + chains + factors);
}

}  // namespace

struct bf_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> queue;
  std::unordered_map<int64_t, Request*> all;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  int64_t budget = 0, reserved = 0, next_id = 1;
  int64_t batch_cols = 0;
  int32_t max_constructs = 0;   // bf_server_opts.max_constructs (0: no cap)
  int32_t running_constructs = 0;
  bf_alloc alloc{};          // the caller's allocator (bf_server_opts.alloc), if any
  bool has_alloc = false;
  SolveRounds* rounds = nullptr;   // cross-request solve rounds (bf_server_opts.solve_rounds)
  int device = 0;
  bool stopping = false;
  Clock::time_point t0 = Clock::now();

  // a construction is always ready; an apply once its construction finished
  // (successfully or not: a failed target fails the apply when it runs)
  bool ready(const Request* r) const {
    if (r->kind == 0) return true;
    auto it = all.find(r->target);
    return it == all.end() || it->second->status <= 0;
  }

  // a construction waits while max_constructs others run (applies do not)
  bool capped(const Request* r) const {
    return r->kind == 0 && max_constructs > 0 && running_constructs >= max_constructs;
  }

  Request* admit() {   // called with mu held
    for (size_t q = 0; q < queue.size(); ++q) {
      Request* r = queue[q];
      if (capped(r)) continue;
      const bool fits = reserved + r->footprint <= budget || reserved == 0;
      if (ready(r) && fits) {
        queue.erase(queue.begin() + q);
        for (size_t e = 0; e < q; ++e) queue[e]->skipped++;
        return r;
      }
      if (r->skipped >= 8 && ready(r)) return nullptr;   // hold the line for it
    }
    return nullptr;
  }

  // Continuous batching (called with mu held, r just admitted): the queued
  // applies against the same factors and direction, up to batch_cols columns
  // with r, leave the queue with it.
  std::vector<Request*> take_batch(Request* r) {
    std::vector<Request*> b{r};
    if (r->kind != 1 || batch_cols <= 0) return b;
    int64_t cols = r->ncols;
    for (size_t q = 0; q < queue.size();) {
      Request* o = queue[q];
      if (o->kind == 1 && o->target == r->target && o->trans == r->trans &&
          cols + o->ncols <= batch_cols && reserved + o->footprint <= budget) {
        cols += o->ncols;
        reserved += o->footprint;
        b.push_back(o);
        queue.erase(queue.begin() + q);
      } else {
        ++q;
      }
    }
    return b;
  }

  // The applies of a batch as one product: columns gathered into one block,
  // one bf_apply, results scattered back.
  int apply_batch(const bf_factors* T, const std::vector<Request*>& b, hipStream_t s) {
    const bf_alloc* al = has_alloc ? &alloc : nullptr;
    if (b.size() == 1) {
      const Request* r = b[0];
      int rc = bf_apply(T, r->trans, r->X, r->ldx, r->ncols, r->Y, r->ldy, al, (void*)s);
      if (rc == BF_OK && hipStreamSynchronize(s) != hipSuccess) rc = BF_EHIP;
      return rc;
    }
    bf_info I{};
    if (bf_stats(T, &I) != BF_OK) return BF_EINVAL;
    const int trans = b[0]->trans;
    const int64_t rin = trans ? I.m : I.n, rout = trans ? I.n : I.m;
    int64_t cols = 0;
    for (auto* r : b) cols += r->ncols;
    // gathered columns: from the caller's allocator if one was given, else the pool
    UseAllocator ua(al);
    DevBuf<bf_c64> xb, yb;
    try {
      xb = DevBuf<bf_c64>((size_t)std::max<int64_t>(1, rin * cols), s);
      yb = DevBuf<bf_c64>((size_t)std::max<int64_t>(1, rout * cols), s);
    } catch (const Error&) {
      xb.reset();
      (void)hipStreamSynchronize(s);
      set_last_error("apply batch: device allocation failed");
      return BF_ENOMEM;
    }
    bf_c64 *Xb = xb.p, *Yb = yb.p;
    int rc = BF_OK;
    int64_t off = 0;
    for (auto* r : b) {
      if (r->ncols > 0 &&
          hipMemcpy2DAsync(Xb + off * rin, rin * sizeof(bf_c64), r->X, r->ldx * sizeof(bf_c64),
                           rin * sizeof(bf_c64), r->ncols, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = BF_EHIP;
      off += r->ncols;
    }
    if (rc == BF_OK) rc = bf_apply(T, trans, Xb, rin, cols, Yb, rout, al, (void*)s);
    off = 0;
    for (auto* r : b) {
      if (rc == BF_OK && r->ncols > 0 &&
          hipMemcpy2DAsync(r->Y, r->ldy * sizeof(bf_c64), Yb + off * rout, rout * sizeof(bf_c64),
                           rout * sizeof(bf_c64), r->ncols, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = BF_EHIP;
      off += r->ncols;
    }
    xb.reset();
    yb.reset();
    if (hipStreamSynchronize(s) != hipSuccess && rc == BF_OK) rc = BF_EHIP;
    if (rc == BF_EHIP) set_last_error("apply batch: HIP copy or synchronization failed");
    return rc;
  }

  void run(int slot) {
    (void)hipSetDevice(device);
    hipStream_t s = streams[slot];
    for (;;) {
      Request* r = nullptr;
      std::vector<Request*> batch;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stopping || (r = admit()) != nullptr; });
        if (!r) return;
        reserved += r->footprint;
        if (r->kind == 0) ++running_constructs;
        batch = take_batch(r);
        const auto now = Clock::now();
        for (auto* q : batch) {
          q->status = 2;
          q->start = now;
          q->batch = (int)batch.size();
        }
      }
      int rc = BF_OK;
      std::string err;
      bf_factors* F = nullptr;
      if (r->kind == 0) {
        RoundsScope rs(rounds);
        rc = bf_construct(r->op.matvec, r->op.rmatvec, r->op.user, r->op.m, r->op.n, r->tol,
                          r->leaf, r->has_opts ? &r->opts : nullptr,
                          has_alloc ? &alloc : nullptr, (void*)s, &F);
      } else {
        const bf_factors* T = nullptr;
        {
          std::lock_guard<std::mutex> lk(mu);
          auto it = all.find(r->target);
          if (it != all.end()) T = it->second->F;
        }
        if (!T) {
          rc = BF_EINVAL;
          set_last_error("apply: the referenced construction failed or was released");
        } else {
          rc = apply_batch(T, batch, s);
        }
      }
      if (rc != BF_OK) err = bf_last_error();
      {
        std::lock_guard<std::mutex> lk(mu);
        const auto now = Clock::now();
        for (auto* q : batch) {
          reserved -= q->footprint;
          q->error = err;
          q->finish = now;
          q->status = rc;
        }
        if (r->kind == 0) --running_constructs;
        r->F = F;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

int bf_server_create(const bf_server_opts* o, bf_server** out) {
  if (!out) return BF_EINVAL;
  const int slots = o && o->slots > 0 ? o->slots : 4;
  if (slots > 64) return BF_EINVAL;
  auto* S = new (std::nothrow) bf_server();
  if (!S) return BF_ENOMEM;
  S->budget = o && o->hbm_budget > 0 ? o->hbm_budget : (int64_t(64) << 30);
  S->batch_cols = o && o->batch_cols > 0 ? o->batch_cols : 0;
  if (o && o->max_constructs < 0) {
    delete S;
    return BF_EINVAL;
  }
  S->max_constructs = o ? o->max_constructs : 0;
  if (o && o->alloc) {
    if (!o->alloc->alloc || !o->alloc->free) {
      delete S;
      return BF_EINVAL;
    }
    S->alloc = *o->alloc;
    S->has_alloc = true;
  }
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return BF_ENOTSUP;
  }
  if (o && o->solve_rounds) {
    try {
      S->rounds = new_solve_rounds(S->device);
    } catch (const std::exception& e) {
      set_last_error(std::string("bf_server_create: solve rounds: ") + e.what());
      delete S;
      return BF_EHIP;
    }
  }
  for (int k = 0; k < slots; ++k) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : S->streams) (void)hipStreamDestroy(x);
      delete_solve_rounds(S->rounds);
      delete S;
      return BF_EHIP;
    }
    S->streams.push_back(st);
  }
  for (int k = 0; k < slots; ++k) S->workers.emplace_back([S, k] { S->run(k); });
  *out = S;
  return BF_OK;
}

int bf_server_destroy(bf_server* S) {
  if (!S) return BF_EINVAL;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    // finish everything that can still run, then stop the workers
    S->cv_done.wait(lk, [&] {
      for (auto* r : S->queue)
        if (S->ready(r)) return false;
      for (auto& kv : S->all)
        if (kv.second->status == 2) return false;
      return true;
    });
    S->stopping = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto& kv : S->all) {
    if (kv.second->F) bf_free(kv.second->F, nullptr);
    delete kv.second;
  }
  for (auto st : S->streams) (void)hipStreamDestroy(st);
  delete_solve_rounds(S->rounds);
  delete S;
  return BF_OK;
}

int bf_server_rounds(bf_server* S, int64_t* rounds, int64_t* items) {
  if (!S || !rounds || !items) return BF_EINVAL;
  solve_rounds_stats(S->rounds, rounds, items);
  return BF_OK;
}

int bf_server_submit_construct(bf_server* S, const bf_operator* op, double tol, int64_t leaf,
                               const bf_opts* opts, int64_t* ticket) {
  if (!S || !op || !op->matvec || !op->rmatvec || !ticket || op->m <= 0 || op->n <= 0 ||
      !(tol > 0.0 && tol < 1.0) || leaf < 1)
    return BF_EINVAL;
  auto* r = new (std::nothrow) Request();
  if (!r) return BF_ENOMEM;
  r->kind = 0;
  r->op = *op;
  r->tol = tol;
  r->leaf = leaf;
  if (opts) r->opts = *opts;
  else r->opts = bf_opts{2, 4, 0, 0, 0, 0, nullptr, nullptr, 0, 0};
  // one stream per construction when there are several slots: they already
  // overlap requests, and a second stream per request measured 1-2% fewer
  // constructions per second; a single slot keeps the two sides apart
  if (S->streams.size() > 1) r->opts.flags |= BF_OPT_ONE_STREAM;
  r->has_opts = true;
  r->footprint = construct_footprint(op->m, op->n, leaf);
  r->arrival = Clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->id = S->next_id++;
    S->all[r->id] = r;
    S->queue.push_back(r);
  }
  S->cv_work.notify_all();
  *ticket = r->id;
  return BF_OK;
}

int bf_server_submit_apply(bf_server* S, int64_t factors_ticket, int trans, const bf_c64* X,
                           int64_t ldx, int64_t ncols, bf_c64* Y, int64_t ldy, int64_t* ticket) {
  if (!S || !X || !Y || !ticket || ncols < 0 || (trans != 0 && trans != 1)) return BF_EINVAL;
  auto* r = new (std::nothrow) Request();
  if (!r) return BF_ENOMEM;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(factors_ticket);
    if (it == S->all.end() || it->second->kind != 0) {
      delete r;
      return BF_EINVAL;
    }
    const bf_operator& op = it->second->op;
    if (ldx < (trans ? op.m : op.n) || ldy < (trans ? op.n : op.m)) {
      delete r;
      return BF_EINVAL;
    }
    r->kind = 1;
    r->target = factors_ticket;
    r->trans = trans;
    r->X = X;
    r->Y = Y;
    r->ldx = ldx;
    r->ldy = ldy;
    r->ncols = ncols;
    r->footprint = 2 * 8 * ncols * 4 * std::max(op.m, op.n);
    r->arrival = Clock::now();
    r->id = S->next_id++;
    S->all[r->id] = r;
    S->queue.push_back(r);
  }
  S->cv_work.notify_all();
  *ticket = r->id;
  return BF_OK;
}

int bf_server_wait(bf_server* S, int64_t ticket, bf_request_info* info) {
  if (!S) return BF_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return BF_EINVAL;
  Request* r = it->second;
  S->cv_done.wait(lk, [&] { return r->status <= 0; });
  if (info) {
    using ns = std::chrono::nanoseconds;
    info->status = r->status;
    info->arrival_ns = std::chrono::duration_cast<ns>(r->arrival - S->t0).count();
    info->start_ns = std::chrono::duration_cast<ns>(r->start - S->t0).count();
    info->finish_ns = std::chrono::duration_cast<ns>(r->finish - S->t0).count();
    info->footprint = r->footprint;
    info->batch = r->batch;
  }
  if (r->status < 0) set_last_error(r->error);
  return r->status;
}

int bf_server_factors(bf_server* S, int64_t ticket, const bf_factors** F) {
  if (!S || !F) return BF_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end() || it->second->kind != 0 || it->second->status != 0) return BF_EINVAL;
  *F = it->second->F;
  return BF_OK;
}

int bf_server_release(bf_server* S, int64_t ticket) {
  if (!S) return BF_EINVAL;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end() || it->second->status > 0) return BF_EINVAL;
    for (auto* q : S->queue)   // applies still waiting on these factors keep them
      if (q->kind == 1 && q->target == ticket) return BF_EINVAL;
    for (auto& kv : S->all)
      if (kv.second->kind == 1 && kv.second->target == ticket && kv.second->status == 2)
        return BF_EINVAL;
    r = it->second;
    S->all.erase(it);
  }
  if (r->F) bf_free(r->F, nullptr);
  delete r;
  return BF_OK;
}

}  // extern "C"
