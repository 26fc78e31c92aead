// Serving loop: resident graphs, a request queue, footprint-bounded
// continuous batching.
//
// A server has `workers` step threads, each with its own context (stream
// and workspace; the first is the caller's).  Every step a worker (1) admits
// queued requests into free running slots, (2) hands running requests the
// next chunks of their canonical edge-id ranges, the chunks together fitting
// the step's HBM work-list budget and work target, (3) runs all chunks in one
// launch sequence, (4) adds each chunk's exact 128-bit accumulators into its
// request and finalises requests whose range is exhausted and whose chunks
// have all returned.  Requests that arrive during a step join at the next
// step, and with two workers one step's set-up, host round trips and tail
// overlap the other step's kernels on the device.  Because the sampler is
// keyed by edge id and the sums are exact integers, a request's result is
// independent of how its range was chunked, of the order chunks return in and
// of what ran beside it.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lge.h"
#include "lge_internal.h"
#include "lge_runtime.h"

using namespace lge;

namespace {

constexpr int32_t kMaxWorkers = 4;

struct Request {
  uint64_t ticket = 0;
  int32_t gid = 0;
  double p = 1.0;
  uint64_t seed = 0;
  int64_t cursor = 0;  // next canonical edge id to hand out
  int64_t m = 0;
  int32_t inflight = 0;  // chunks running on some worker
  bool canceled = false;
  bool done = false;
  int status = LGE_OK;
  int error = LGE_OK;  // first failed chunk
  unsigned long long acc[kAccSlots * 2] = {};
  lge_result result{};
};

// scheduling weight of canonical edge ids [0, x) of g: the graph's work
// profile, linear inside a profile block
double work_at(const lge_graph *g, int64_t x) {
  const std::vector<double> &P = g->work_pref;
  if (P.size() < 2) return (double)x * g->work_per_id;
  const int64_t k = x / kWorkBlock;
  if (k >= (int64_t)P.size() - 1) return P.back();
  const int64_t b0 = k * kWorkBlock, b1 = std::min(b0 + kWorkBlock, g->m);
  return P[(size_t)k] + (P[(size_t)k + 1] - P[(size_t)k]) * (double)(x - b0) / (double)(b1 - b0);
}

// the smallest x in (c, m] with work_at(x) - work_at(c) >= units (m if none)
int64_t ids_for_work(const lge_graph *g, int64_t c, double units) {
  const std::vector<double> &P = g->work_pref;
  if (P.size() < 2) return std::min(g->m, c + std::max<int64_t>(1, (int64_t)std::min(units / std::max(g->work_per_id, 1e-9), 9.0e15)));
  const double target = work_at(g, c) + units;
  if (target >= P.back()) return g->m;
  const int64_t k = (int64_t)(std::lower_bound(P.begin(), P.end(), target) - P.begin());  // P[k-1] < target <= P[k]
  const int64_t b0 = (k - 1) * kWorkBlock, b1 = std::min(k * kWorkBlock, g->m);
  const double span = P[(size_t)k] - P[(size_t)k - 1];
  const double f = span > 0 ? (target - P[(size_t)k - 1]) / span : 1.0;
  const int64_t x = b0 + (int64_t)std::ceil(f * (double)(b1 - b0));
  return std::min(g->m, std::max(x, c + 1));
}

void add_acc(unsigned long long *dst, const unsigned long long *src) {
  for (int k = 0; k < kAccSlots; ++k) {
    const unsigned long long lo = dst[2 * k] + src[2 * k];
    const unsigned long long carry = lo < dst[2 * k] ? 1ull : 0ull;
    dst[2 * k] = lo;
    dst[2 * k + 1] += src[2 * k + 1] + carry;
  }
}

}  // namespace

struct lge_server {
  struct Worker {
    lge_ctx *ctx = nullptr;
    bool owned = false;  // opened by the server
    std::thread th;
  };
  lge_ctx *ctx = nullptr;
  lge_server_cfg cfg{};
  std::vector<const lge_graph *> graphs;
  std::mutex mu;
  std::condition_variable cv_work;  // workers wait for assignable work
  std::condition_variable cv_done;  // waiters wait for results
  std::deque<Request *> queue;
  std::vector<Request *> running;
  std::unordered_map<uint64_t, Request *> all;
  uint64_t next_ticket = 1;
  size_t rotate = 0;
  double rate = 5e8;  // work units per second and worker, updated after every step
  bool stop = false;
  int waiters = 0;
  lge_server_stats stats{};
  Worker workers[kMaxWorkers];
  int nworkers = 0;

  void finish(Request *r, int status) {
    r->status = status;
    r->done = true;
    if (status == LGE_OK) ++stats.completed;
    else if (status == LGE_ECANCELED) ++stats.canceled;
  }

  // resolve a running request once it has nothing left to hand out and no
  // chunk in flight; true if it finished
  bool try_complete(Request *r) {
    if (r->done || r->inflight > 0) return r->done;
    if (r->error != LGE_OK) {
      finish(r, r->error);
    } else if (r->canceled) {
      finish(r, LGE_ECANCELED);
    } else if (r->cursor >= r->m) {
      const lge_graph *g = graphs[(size_t)r->gid];
      lge_finalize(g->n, g->m, r->p, r->seed, r->acc, &r->result);
      finish(r, LGE_OK);
    }
    return r->done;
  }

  bool has_short_lane() const { return cfg.short_us >= 0 && nworkers >= 3; }

  // expected seconds of r's remaining range on one worker
  double remaining_s(const Request *r) const {
    const lge_graph *g = graphs[(size_t)r->gid];
    return r->p * (work_at(g, r->m) - work_at(g, r->cursor)) / rate;
  }

  // may a worker of this lane step r now?
  bool eligible(const Request *r, bool short_lane) const {
    if (r->canceled || r->error != LGE_OK || r->cursor >= r->m) return false;
    if (!has_short_lane()) return true;
    return short_lane == (remaining_s(r) * 1e6 < (double)cfg.short_us);
  }

  bool assignable(bool short_lane) const {
    if (!queue.empty() && (int32_t)running.size() < cfg.max_inflight) return true;
    for (const Request *r : running)
      if (eligible(r, short_lane)) return true;
    return false;
  }

  void loop(lge_ctx *wctx, bool short_lane) {
    std::vector<Job> jobs;
    std::vector<Request *> in_step;
    for (;;) {
      double step_work = 0.0;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || assignable(short_lane); });
        if (stop) return;
        // admission: running slots free up as requests finish
        bool admitted = false;
        while (!queue.empty() && (int32_t)running.size() < cfg.max_inflight) {
          running.push_back(queue.front());
          queue.pop_front();
          admitted = true;
        }
        if (admitted) cv_work.notify_all();  // the other lane may own some of them
        // chunks for this step, starting at a rotating request
        jobs.clear();
        in_step.clear();
        // half of the HBM budget for the per-id arrays of the step's ids, half
        // for its split-class lists (the launch sequence runs in pieces
        // rather than exceed that)
        int64_t budget = std::max<int64_t>(cfg.hbm_budget_bytes / 2 / lge_ws_bytes_per_id(), 1);  // edge ids
        const double step_us = short_lane ? (double)std::min<int64_t>(cfg.short_us, cfg.target_step_us)
                                          : (double)cfg.target_step_us;
        double wbudget = std::max(rate * step_us * 1e-6, 1.0);  // work units
        std::vector<Request *> open;
        for (Request *r : running)
          if (eligible(r, short_lane)) open.push_back(r);
        const size_t nr = open.size();
        if (nr == 0) continue;
        rotate %= nr;
        for (size_t k = 0; k < nr && budget > 0; ++k) {
          Request *r = open[(rotate + k) % nr];
          const lge_graph *g = graphs[(size_t)r->gid];
          const int64_t left = r->m - r->cursor;
          // the ids whose expected work (the graph's profile times p) is
          // this request's share of the step
          const double wshare = wbudget / (double)(nr - k);
          const int64_t by_work = ids_for_work(g, r->cursor, wshare / std::max(r->p, 1e-300)) - r->cursor;
          const int64_t want = std::max<int64_t>(cfg.min_chunk_edges, by_work);
          const int64_t len = std::min(left, std::min(want, budget));
          const double wk = r->p * (work_at(g, r->cursor + len) - work_at(g, r->cursor));
          jobs.push_back(Job{g, r->p, r->seed, r->cursor, r->cursor + len, -1, -1, 0});
          in_step.push_back(r);
          r->cursor += len;
          r->inflight += 1;
          budget -= std::max<int64_t>(len, 1);
          wbudget -= std::min(wbudget, wk);
          step_work += wk;
        }
        rotate += 1;
        ++stats.steps;
        if (assignable(short_lane) || assignable(!short_lane)) cv_work.notify_all();  // work for idle workers
      }
      const auto t0 = std::chrono::steady_clock::now();
      lge_opts o = wctx->opts;
      o.max_list_mib = (int32_t)std::max<int64_t>(1, std::min<int64_t>(cfg.hbm_budget_bytes / 2 >> 20, INT32_MAX));
      const int rc = lge_run_jobs(wctx, jobs.data(), (int)jobs.size(), &o);
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      {
        std::lock_guard<std::mutex> lk(mu);
        stats.busy_s += dt;
        stats.workspace_bytes = std::max<uint64_t>(stats.workspace_bytes, (uint64_t)lge_ws_bytes(wctx));
        // work rate of the steps that were long enough to measure it
        if (rc == LGE_OK && dt > 2e-3 && step_work > 0) rate = 0.7 * rate + 0.3 * (step_work / dt);
        for (size_t j = 0; j < in_step.size(); ++j) {
          Request *r = in_step[j];
          r->inflight -= 1;
          if (rc != LGE_OK) {
            if (r->error == LGE_OK) r->error = rc;
          } else {
            add_acc(r->acc, wctx->ws.h_acc + (int64_t)j * kAccSlots * 2);
          }
        }
        // cancelled requests and finished ranges resolve once nothing is in flight
        for (Request *r : running) try_complete(r);
        running.erase(std::remove_if(running.begin(), running.end(), [](Request *r) { return r->done; }),
                      running.end());
        cv_done.notify_all();
        cv_work.notify_all();
      }
    }
  }
};

extern "C" int lge_server_cfg_default(lge_server_cfg *c) {
  if (!c) return LGE_EINVAL;
  memset(c, 0, sizeof(*c));
  c->max_inflight = 64;
  c->queue_capacity = 4096;
  c->hbm_budget_bytes = (int64_t)8 << 30;
  c->min_chunk_edges = 4096;
  c->target_step_us = 20000;
  c->workers = 3;
  c->short_us = 20000;
  return LGE_OK;
}

extern "C" int lge_server_create(lge_ctx *ctx, const lge_server_cfg *cfg, lge_server **out) {
  if (!ctx || !out) return LGE_EINVAL;
  *out = nullptr;
  lge_server_cfg c;
  lge_server_cfg_default(&c);
  if (cfg) {
    if (cfg->max_inflight < 0 || cfg->queue_capacity < 0 || cfg->hbm_budget_bytes < 0 || cfg->min_chunk_edges < 0 ||
        cfg->target_step_us < 0 || cfg->workers < 0 || cfg->workers > kMaxWorkers)
      return LGE_EINVAL;
    if (cfg->target_step_us) c.target_step_us = cfg->target_step_us;
    if (cfg->max_inflight) c.max_inflight = cfg->max_inflight;
    if (cfg->queue_capacity) c.queue_capacity = cfg->queue_capacity;
    if (cfg->hbm_budget_bytes) c.hbm_budget_bytes = cfg->hbm_budget_bytes;
    if (cfg->min_chunk_edges) c.min_chunk_edges = cfg->min_chunk_edges;
    if (cfg->workers) c.workers = cfg->workers;
    if (cfg->short_us) c.short_us = cfg->short_us;
  }
  if (c.hbm_budget_bytes < 2 * lge_ws_bytes_per_id()) return LGE_EINVAL;
  lge_server *s = new (std::nothrow) lge_server();
  if (!s) return LGE_ENOMEM;
  s->ctx = ctx;
  s->cfg = c;
  // worker 0 steps on the caller's context, the others on contexts of their
  // own (same device, own stream and workspace); a context that cannot be
  // opened leaves fewer workers
  s->workers[0].ctx = ctx;
  s->nworkers = 1;
  for (int k = 1; k < c.workers; ++k) {
    lge_ctx *wc = nullptr;
    if (lge_open(ctx->device, &wc) != LGE_OK) break;
    wc->opts = ctx->opts;
    s->workers[k].ctx = wc;
    s->workers[k].owned = true;
    s->nworkers = k + 1;
  }
  s->cfg.workers = s->nworkers;
  try {
    for (int k = 0; k < s->nworkers; ++k) {
      lge_ctx *wc = s->workers[k].ctx;
      const bool short_lane = s->has_short_lane() && k == s->nworkers - 1;
      s->workers[k].th = std::thread([s, wc, short_lane] {
        (void)hipSetDevice(wc->device);
        s->loop(wc, short_lane);
      });
    }
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
      s->cv_work.notify_all();
    }
    for (int k = 0; k < s->nworkers; ++k) {
      if (s->workers[k].th.joinable()) s->workers[k].th.join();
      if (s->workers[k].owned) lge_close(s->workers[k].ctx);
    }
    delete s;
    return LGE_ENOMEM;
  }
  *out = s;
  return LGE_OK;
}

extern "C" int lge_server_add_graph(lge_server *srv, const lge_graph *g, int32_t *gid) {
  if (!srv || !g || !gid) return LGE_EINVAL;
  if (g->ctx != srv->ctx) return LGE_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return LGE_ECANCELED;
  *gid = (int32_t)srv->graphs.size();
  srv->graphs.push_back(g);
  return LGE_OK;
}

extern "C" int lge_submit(lge_server *srv, int32_t gid, double p, uint64_t seed, uint64_t *ticket) {
  if (!(p > 0.0 && p <= 1.0)) return LGE_EINVAL;
  if (!srv || !ticket) return LGE_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return LGE_ECANCELED;
  if (gid < 0 || (size_t)gid >= srv->graphs.size()) return LGE_ENOTFOUND;
  if ((int64_t)(srv->queue.size() + srv->running.size()) >= srv->cfg.queue_capacity) {
    ++srv->stats.rejected;
    return LGE_EBUSY;
  }
  Request *r = new (std::nothrow) Request();
  if (!r) return LGE_ENOMEM;
  r->ticket = srv->next_ticket++;
  r->gid = gid;
  r->p = p;
  r->seed = seed;
  r->m = srv->graphs[(size_t)gid]->m;
  if (r->m == 0) {  // nothing to sample: result is immediate
    const lge_graph *g = srv->graphs[(size_t)gid];
    lge_finalize(g->n, g->m, p, seed, r->acc, &r->result);
    srv->finish(r, LGE_OK);
  } else {
    srv->queue.push_back(r);
  }
  srv->all[r->ticket] = r;
  ++srv->stats.submitted;
  *ticket = r->ticket;
  srv->cv_work.notify_all();
  if (r->done) srv->cv_done.notify_all();
  return LGE_OK;
}

extern "C" int lge_wait(lge_server *srv, uint64_t ticket, int64_t timeout_us, lge_result *out) {
  if (!srv || !out) return LGE_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return LGE_ENOTFOUND;
  Request *r = it->second;
  ++srv->waiters;
  bool ok = true;
  if (timeout_us < 0) {
    srv->cv_done.wait(lk, [&] { return r->done; });
  } else {
    ok = srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; });
  }
  --srv->waiters;
  srv->cv_done.notify_all();
  if (!ok) return LGE_ETIMEDOUT;
  const int st = r->status;
  if (st == LGE_OK) *out = r->result;
  srv->all.erase(ticket);
  delete r;
  return st;
}

extern "C" int lge_cancel(lge_server *srv, uint64_t ticket) {
  if (!srv) return LGE_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) return LGE_ENOTFOUND;
  Request *r = it->second;
  if (r->done) return LGE_OK;
  r->canceled = true;
  auto q = std::find(srv->queue.begin(), srv->queue.end(), r);
  if (q != srv->queue.end()) {  // never admitted: resolve now
    srv->queue.erase(q);
    srv->finish(r, LGE_ECANCELED);
  } else if (srv->try_complete(r)) {  // running, no chunk in flight
    srv->running.erase(std::remove(srv->running.begin(), srv->running.end(), r), srv->running.end());
  }
  if (r->done) srv->cv_done.notify_all();
  srv->cv_work.notify_all();
  return LGE_OK;
}

extern "C" int lge_server_get_stats(lge_server *srv, lge_server_stats *out) {
  if (!srv || !out) return LGE_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->stats;
  out->queued = srv->queue.size();
  out->running = srv->running.size();
  return LGE_OK;
}

extern "C" int lge_server_destroy(lge_server *srv) {
  if (!srv) return LGE_EINVAL;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  for (int k = 0; k < srv->nworkers; ++k)  // steps in flight complete first
    if (srv->workers[k].th.joinable()) srv->workers[k].th.join();
  for (int k = 0; k < srv->nworkers; ++k)
    if (srv->workers[k].owned) lge_close(srv->workers[k].ctx);
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    for (auto &kv : srv->all)
      if (!kv.second->done) srv->finish(kv.second, LGE_ECANCELED);
    srv->queue.clear();
    srv->running.clear();
    srv->cv_done.notify_all();
    // let threads blocked in lge_wait observe their result before freeing
    srv->cv_done.wait(lk, [&] { return srv->waiters == 0; });
    for (auto &kv : srv->all) delete kv.second;
    srv->all.clear();
  }
  delete srv;
  return LGE_OK;
}
