// Serving: continuous batching of sieve queries over resident graphs.
//
// A worker thread owns a HIP stream (default priority) and loops:
//   1. admit queued queries in arrival order while the HBM footprint of the
//      admitted set stays within the budget and fewer than max_inflight are
//      admitted (a query that has to wait counts once as deferred);
//   2. build an epoch: every admitted query contributes its next range of
//      64-iteration chunks, oldest first, until the epoch's edge-update
//      target is reached (each query gets at least one chunk);
//   3. run the epoch as one batched persistent launch and XOR each slice's
//      partial fingerprint into its query (F over disjoint iteration ranges
//      XOR to F over their union); finished queries complete and wake pollers.
// Queries arriving while an epoch runs are admitted for the next epoch, so
// long queries do not hold back short ones and the device always runs a mix.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "rs_internal.h"

namespace rs {

rs_status plan_query(const rs_graph* g, const rs_query* q, QueryPlan& qp);
rs_status run_batch_impl(const rs_graph* const* graphs, const rs_query* queries, uint32_t nq,
                         rs_result* results, const rs_tuning* tune, hipStream_t st, bool use_graph,
                         uint64_t slot_budget);

using Clock = std::chrono::steady_clock;

struct SQuery {
  uint64_t ticket;
  uint32_t graph_id;
  rs_query q;
  uint8_t motif[RS_MAX_COLOURS];
  bool has_motif;
  QueryPlan plan;
  uint64_t next_chunk;  // next 64-iteration chunk to schedule
  uint64_t F = 0;
  uint64_t footprint;
  uint64_t work_per_chunk;  // edge-updates
  Clock::time_point t_submit;
  bool deferred_counted = false;
  bool done = false, cancelled = false;
  rs_result result{};
};

}  // namespace rs

struct rs_server {
  uint64_t budget;
  rs_server_opts opts;
  std::vector<const rs_graph*> graphs;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<rs::SQuery>> queued;
  std::vector<std::shared_ptr<rs::SQuery>> active;
  std::map<uint64_t, std::shared_ptr<rs::SQuery>> by_ticket;
  std::vector<double> latencies_ms;
  uint64_t next_ticket = 1;
  uint64_t used_bytes = 0;
  bool stop = false;
  std::thread worker;
  hipStream_t stream = nullptr;
  int device = 0;
  rs::Clock::time_point t_create;
  rs_server_stats st{};
};

namespace rs {

static uint64_t footprint_of(const rs_graph* g, const QueryPlan& qp) {
  const uint64_t m = g->g.m, n = g->g.n;
  const uint64_t per_query = 4 * m + 8 * n * qp.kq + 8 * m * qp.kq * (qp.k - 1) + 8 * (1ull << qp.k) + 2 * m + 5 * n;
  const uint64_t slot = 2ull * (m + n) * 64 * 8 + 2ull * ((m + 15) / 16) * 1024;  // one chunk's buffers
  return per_query + slot;
}

static void worker_loop(rs_server* S) {
  (void)hipSetDevice(S->device);
  while (true) {
    std::vector<std::shared_ptr<SQuery>> epoch_q;
    std::vector<rs_query> slices;
    std::vector<const rs_graph*> gl;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop) {
        for (auto& a : S->active) a->cancelled = true;
        if (S->active.empty()) break;
      }
      // admission
      while (!S->stop && !S->queued.empty()) {
        auto& f = S->queued.front();
        if (f->cancelled) {
          S->queued.pop_front();
          continue;
        }
        if (S->active.size() >= S->opts.max_inflight || S->used_bytes + f->footprint > S->budget) {
          if (!f->deferred_counted) {
            f->deferred_counted = true;
            S->st.deferred++;
          }
          break;
        }
        S->used_bytes += f->footprint;
        S->active.push_back(f);
        S->queued.pop_front();
        S->st.admitted++;
      }
      if (S->active.empty()) {
        if (S->stop) break;
        S->cv_work.wait(lk, [&] { return S->stop || !S->queued.empty(); });
        continue;
      }
      // epoch: oldest first, at least one chunk each
      uint64_t budget = S->opts.epoch_edge_updates;
      for (auto& a : S->active) {
        if (a->cancelled) continue;
        const uint64_t left = a->plan.chunk_last - a->next_chunk;
        uint64_t take = 1;
        if (a->work_per_chunk) {
          const uint64_t fit = budget / a->work_per_chunk;
          take = std::max<uint64_t>(1, std::min(left, fit));
        }
        take = std::min(take, left);
        const uint64_t b = std::max(a->plan.it_begin, a->next_chunk * 64);
        const uint64_t e = std::min(a->plan.it_end, (a->next_chunk + take) * 64);
        rs_query sq = a->q;
        sq.motif_count = a->has_motif ? a->motif : nullptr;
        sq.it_begin = b;
        sq.it_end = e;
        slices.push_back(sq);
        gl.push_back(S->graphs[a->graph_id]);
        epoch_q.push_back(a);
        a->next_chunk += take;
        const uint64_t w = take * a->work_per_chunk;
        budget = budget > w ? budget - w : 0;
      }
    }
    // run the epoch (outside the lock: submissions and polls continue)
    std::vector<rs_result> res(slices.size());
    const auto t0 = Clock::now();
    rs_status s = slices.empty() ? RS_OK
                                 : run_batch_impl(gl.data(), slices.data(), (uint32_t)slices.size(), res.data(),
                                                  nullptr, S->stream, false, S->budget / 2);
    const double busy = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st.busy_ms += busy;
      S->st.epochs++;
      const auto now = Clock::now();
      for (size_t i = 0; i < epoch_q.size(); ++i) {
        auto& a = epoch_q[i];
        if (s != RS_OK || res[i].status != RS_OK) {
          a->result.status = res[i].status != RS_OK ? res[i].status : s;
          a->done = true;
        } else {
          a->F ^= res[i].fingerprint;
          if (a->next_chunk >= a->plan.chunk_last) {
            a->result.fingerprint = a->F;
            a->result.yes = a->F != 0;
            a->result.status = RS_OK;
            a->done = true;
          }
        }
        if (a->done) {
          const double lat = std::chrono::duration<double, std::milli>(now - a->t_submit).count();
          a->result.device_ms = (float)lat;
          if (a->result.status == RS_OK) {
            S->latencies_ms.push_back(lat);
            S->st.completed++;
          }
        }
      }
      // retire finished and cancelled queries, free their footprint
      std::vector<std::shared_ptr<SQuery>> keep;
      for (auto& a : S->active) {
        if (a->done || a->cancelled) {
          S->used_bytes -= a->footprint;
          if (a->cancelled && !a->done) {
            a->result.status = RS_ECANCELED;
            a->done = true;
          }
        } else {
          keep.push_back(a);
        }
      }
      S->active.swap(keep);
    }
    S->cv_done.notify_all();
  }
  // cancel what is left
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto& a : S->queued) {
    a->cancelled = true;
    a->result.status = RS_ECANCELED;
    a->done = true;
    S->st.cancelled++;
  }
  S->queued.clear();
  S->cv_done.notify_all();
}

static double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double idx = p * (double)(v.size() - 1);
  const size_t lo = (size_t)idx, hi = std::min(v.size() - 1, lo + 1);
  const double f = idx - (double)lo;
  return v[lo] * (1 - f) + v[hi] * f;
}

}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_server_create(uint64_t hbm_budget, const rs_server_opts* opts, rs_server** out) {
  if (!out || hbm_budget == 0) return RS_EINVAL;
  try {
    rs_server* S = new rs_server();
    S->budget = hbm_budget;
    S->opts = opts ? *opts : rs_server_opts{0, 0, 0};
    if (!S->opts.max_inflight) S->opts.max_inflight = 64;
    if (!S->opts.epoch_edge_updates) S->opts.epoch_edge_updates = 4000000000ull;
    if (!S->opts.streams) S->opts.streams = 1;
    if (hipGetDevice(&S->device) != hipSuccess || hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
      delete S;
      return RS_EDEVICE;
    }
    S->t_create = Clock::now();
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return RS_OK;
  } catch (...) {
    return RS_ENOMEM;
  }
}

rs_status rs_server_add_graph(rs_server* s, const rs_graph* g, uint32_t* graph_id) {
  if (!s || !g || !graph_id) return RS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->graphs.push_back(g);
  *graph_id = (uint32_t)(s->graphs.size() - 1);
  return RS_OK;
}

rs_status rs_server_submit(rs_server* s, uint32_t graph_id, const rs_query* q, uint64_t* ticket) {
  if (!s || !q || !ticket) return RS_EINVAL;
  try {
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id >= s->graphs.size()) return RS_ENOTFOUND;
    const rs_graph* g = s->graphs[graph_id];
    auto a = std::make_shared<SQuery>();
    rs_status st = plan_query(g, q, a->plan);
    s->st.submitted++;
    if (st != RS_OK) {
      s->st.rejected++;
      return st;
    }
    a->footprint = footprint_of(g, a->plan);
    if (a->footprint > s->budget) {
      s->st.rejected++;
      return RS_ENOMEM;
    }
    a->ticket = s->next_ticket++;
    a->graph_id = graph_id;
    a->q = *q;
    a->has_motif = q->motif_count != nullptr;
    if (a->has_motif) {
      memset(a->motif, 0, sizeof(a->motif));
      for (uint32_t c = 0; c < g->info.n_colours; ++c) a->motif[c] = q->motif_count[c];
    }
    a->next_chunk = a->plan.chunk_first;
    a->work_per_chunk = 64ull * (a->plan.k - 1) * g->g.m;
    a->t_submit = Clock::now();
    const bool trivial = g->g.m == 0 || a->plan.k > g->g.n || a->plan.it_end == a->plan.it_begin;
    if (trivial) {  // F = 0 exactly, nothing to run
      a->done = true;
      a->result = rs_result{0, 0, RS_OK, 0.0f};
      s->latencies_ms.push_back(0.0);
      s->st.completed++;
    } else {
      s->queued.push_back(a);
    }
    s->by_ticket[a->ticket] = a;
    *ticket = a->ticket;
  } catch (...) {
    return RS_ENOMEM;
  }
  s->cv_work.notify_one();
  s->cv_done.notify_all();
  return RS_OK;
}

rs_status rs_server_poll(rs_server* s, uint64_t ticket, rs_result* r, int32_t wait_ms) {
  if (!s || !r) return RS_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return RS_ENOTFOUND;
  auto a = it->second;
  auto ready = [&] { return a->done; };
  if (!ready()) {
    if (wait_ms == 0) return RS_ETIMEOUT;
    if (wait_ms < 0)
      s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready))
      return RS_ETIMEOUT;
  }
  *r = a->result;
  s->by_ticket.erase(ticket);
  return RS_OK;
}

rs_status rs_server_cancel(rs_server* s, uint64_t ticket) {
  if (!s) return RS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->by_ticket.find(ticket);
  if (it == s->by_ticket.end()) return RS_ENOTFOUND;
  auto a = it->second;
  if (a->done) return RS_OK;
  a->cancelled = true;
  s->st.cancelled++;
  // queued queries finish at once; admitted ones when the current epoch ends
  for (auto q = s->queued.begin(); q != s->queued.end(); ++q) {
    if (*q == a) {
      s->queued.erase(q);
      a->result.status = RS_ECANCELED;
      a->done = true;
      break;
    }
  }
  s->cv_done.notify_all();
  return RS_OK;
}

rs_status rs_server_stats_get(rs_server* s, rs_server_stats* out) {
  if (!s || !out) return RS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queued = s->queued.size();
  out->inflight = s->active.size();
  const double secs = std::chrono::duration<double>(Clock::now() - s->t_create).count();
  out->qps = secs > 0 ? (double)s->st.completed / secs : 0.0;
  out->p50_ms = percentile(s->latencies_ms, 0.50);
  out->p99_ms = percentile(s->latencies_ms, 0.99);
  return RS_OK;
}

rs_status rs_server_destroy(rs_server* s) {
  if (!s) return RS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (auto& a : s->active) a->cancelled = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamDestroy(s->stream);
  delete s;
  return RS_OK;
}

}  // extern "C"
