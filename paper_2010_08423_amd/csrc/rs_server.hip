// Serving: continuous batching of sieve queries over resident graphs.
//
// A pool of worker threads, each with its own HIP stream (default priority),
// takes queued queries in arrival order:
//   * a query on a large graph (its launches fill the GPU by themselves) runs
//     alone through the plain level kernels, in a plain workspace taken from
//     a pool of workspaces kept resident per graph;
//   * queries on small graphs that wait together are taken as one group (up
//     to a work cap) and evaluated by the batched path in shared level
//     launches, which removes their per-query launch and setup overhead;
//     while a group runs, small-graph arrivals queue for the next group and
//     idle workers take large-graph queries;
//   * a query whose remaining work exceeds what is left of the cap joins a
//     group with a slice of whole 64-iteration chunks (an iteration range:
//     the sieve sums over iterations, so slice fingerprints XOR to the
//     query's) and its rest rejoins the queue in arrival order. Queries thus
//     enter and leave groups at chunk boundaries: an arrival waits for at
//     most one group, not for the longest query of the one running.
// Workers run concurrently, so queries overlap on the device. Admission is
// by HBM: the resident plain workspaces, the group workspace and the growth
// a job needs must stay within the budget; idle workspaces are freed when a
// job needs their room. A query that has to wait for memory or for an
// in-flight slot counts once as deferred. Every result is the one the query
// gives alone (same kernels, same arithmetic).
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "rs_internal.h"

namespace rs {

using Clock = std::chrono::steady_clock;

constexpr uint64_t kGroupMaxEdges = 262144;  // default: graphs this small are grouped
constexpr uint64_t kGroupEdgeUpdates = 4000000000ull;  // about 20 ms of level work
constexpr uint32_t kMaxGroup = 64;
constexpr uint32_t kMaxWorkers = 16;

struct SQuery {
  uint64_t ticket;
  uint32_t graph_id;
  rs_query q;
  uint8_t motif[RS_MAX_COLOURS];
  bool has_motif;
  QueryPlan plan;
  Tuning tu;
  PlainSizes sizes;    // plain workspace buffers it needs
  uint64_t group_bytes;  // its per-query tables in a group
  uint64_t work;         // edge-updates of the remaining iterations
  uint64_t per_it;       // edge-updates per iteration: (k-1) m
  uint64_t next_it;      // first iteration not yet run
  uint64_t acc_F = 0;    // XOR of the fingerprints of the slices run so far
  bool admitted_once = false;
  bool split = false;    // runs in more than one piece
  Clock::time_point t_submit;
  bool deferred_counted = false;
  bool done = false, cancelled = false;
  rs_result result{};
};

// A plain workspace kept resident for one graph.
struct PoolEntry {
  uint32_t graph_id;
  PlainWorkspace ws;
  uint64_t bytes = 0;  // device bytes held (as of the last run)
  bool busy = false;
};

struct Job {
  std::vector<std::shared_ptr<SQuery>> qs;
  std::vector<uint64_t> it_end;  // per query: end of the iterations this job runs
  PoolEntry* entry = nullptr;  // plain job
  uint64_t reserved = 0;       // bytes added to the held total for this job
  bool group = false;
};

}  // namespace rs

struct rs_server {
  uint64_t budget;
  rs_server_opts opts;
  std::vector<const rs_graph*> graphs;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<rs::SQuery>> queued;
  std::map<uint64_t, std::shared_ptr<rs::SQuery>> by_ticket;
  std::vector<double> latencies_ms;
  uint64_t next_ticket = 1;
  uint64_t inflight = 0;
  // device memory held: resident plain workspaces and the group workspace
  std::vector<std::unique_ptr<rs::PoolEntry>> pool;
  rs::BatchWorkspace* bws = nullptr;
  uint64_t plain_held = 0, batch_held = 0;
  bool group_running = false;
  bool stop = false;
  std::vector<std::thread> workers;
  int device = 0;
  rs::Clock::time_point t_create;
  rs_server_stats st{};
};

namespace rs {

static bool is_small(const rs_server* S, const SQuery& a) {
  return S->graphs[a.graph_id]->g.m <= S->opts.group_max_edges;
}

// Bytes a workspace grows by to run a query of the given sizes (a buffer
// that is too small is replaced by one of the needed size).
static uint64_t growth(const PlainWorkspace& w, const PlainSizes& z) {
  auto g = [](const DevBuf& b, uint64_t need) { return need > b.bytes ? need - b.bytes : 0; };
  return g(w.lo, z.lo) + g(w.z, z.z) + g(w.q, z.q) + g(w.p0, z.p) + g(w.p1, z.p) + g(w.partial, z.partial) +
         g(w.fsum, z.fsum) + g(w.out, 64) + g(w.ref, z.ref) + g(w.need, z.need) + g(w.cov_diff, z.cover) +
         g(w.agg, z.records) + g(w.incl, z.records) + g(w.run_pre, z.run_pre) + g(w.run_bsum, z.run_bsum) +
         g(w.run_boff, z.run_boff) + g(w.run_bounds, z.run_bounds) + g(w.lists, z.lists) + g(w.rr, z.rr) + g(w.grp, z.grp);
}

// Puts a query back in the queue before the first query that arrived after
// it (queries that have run slices keep their place in arrival order).
static void requeue(rs_server* S, const std::shared_ptr<SQuery>& a) {
  auto it = S->queued.begin();
  while (it != S->queued.end() && (*it)->t_submit <= a->t_submit) ++it;
  S->queued.insert(it, a);
}

// Iterations [next_it, end) of a that fit `room` edge-updates, ending at a
// chunk boundary or at the query's end; end == next_it if no chunk fits.
static uint64_t slice_end(const SQuery& a, uint64_t room) {
  const uint64_t its = room / std::max<uint64_t>(a.per_it, 1);
  if (a.next_it + its >= a.plan.it_end) return a.plan.it_end;
  const uint64_t e = (a.next_it + its) / 64 * 64;  // 64-iteration chunks
  return e > a.next_it ? e : a.next_it;
}

static uint64_t held(const rs_server* S) { return S->plain_held + S->batch_held; }

static void defer(rs_server* S, SQuery& a) {
  if (!a.deferred_counted) {
    a.deferred_counted = true;
    S->st.deferred++;
  }
}

// Frees idle resident workspaces (other graphs first, never `keep`), and the
// group workspace when no group runs, until `need` more bytes fit the budget.
// Freeing synchronises the device; it happens only under memory pressure.
static void make_room(rs_server* S, uint64_t need, const PoolEntry* keep, uint32_t graph_id) {
  for (int pass = 0; pass < 2 && held(S) + need > S->budget; ++pass) {
    for (size_t i = 0; i < S->pool.size() && held(S) + need > S->budget;) {
      PoolEntry* e = S->pool[i].get();
      const bool other = e->graph_id != graph_id;
      if (e == keep || e->busy || (pass == 0 && !other)) {
        ++i;
        continue;
      }
      e->ws.release();
      S->plain_held -= e->bytes;
      S->pool.erase(S->pool.begin() + i);
    }
    if (pass == 0 && held(S) + need > S->budget && !S->group_running && S->batch_held) {
      batch_ws_release(S->bws);
      S->batch_held = 0;
    }
  }
}

// Reserves a plain workspace for query a: an idle one of its graph if the
// growth fits, else a new one. False if the memory is not there yet.
static bool reserve_plain(rs_server* S, SQuery& a, Job& job) {
  PoolEntry* best = nullptr;
  uint64_t best_gr = 0;
  for (auto& e : S->pool) {
    if (e->busy || e->graph_id != a.graph_id) continue;
    const uint64_t gr = growth(e->ws, a.sizes);
    if (!best || gr < best_gr) {
      best = e.get();
      best_gr = gr;
    }
  }
  const uint64_t need = best ? best_gr : a.sizes.total();
  if (held(S) + need > S->budget) make_room(S, need, best, a.graph_id);
  if (held(S) + need > S->budget) return false;
  if (!best) {
    S->pool.emplace_back(new PoolEntry());
    best = S->pool.back().get();
    best->graph_id = a.graph_id;
  }
  best->busy = true;
  S->plain_held += need;
  job.entry = best;
  job.reserved = need;
  return true;
}

// Takes the next job under the lock; false if nothing can start now.
static bool take_job(rs_server* S, Job& job) {
  while (!S->queued.empty() && S->queued.front()->cancelled) S->queued.pop_front();
  if (S->queued.empty()) return false;
  // while a group runs, small-graph queries wait for the next group
  auto it = S->queued.begin();
  if (S->group_running)
    while (it != S->queued.end() && is_small(S, **it)) ++it;
  if (it == S->queued.end()) return false;
  auto& a = *it;
  if (S->inflight >= S->opts.max_inflight) {
    defer(S, *a);
    return false;
  }
  if (is_small(S, *a) && slice_end(*a, S->opts.group_edge_updates) > a->next_it) {
    // a group: small-graph queries in arrival order while work, slots and
    // memory allow, each with all its remaining iterations or a slice of them
    const uint64_t slot_share = S->budget / 4;  // prefix-state arena of the group's rounds
    uint64_t work = 0, bytes = slot_share;
    const uint64_t slots = S->opts.max_inflight - S->inflight;
    std::vector<size_t> pick;     // queue positions, ascending
    std::vector<uint64_t> ends;   // iterations each picked query runs up to
    for (size_t j = (size_t)(it - S->queued.begin());
         j < S->queued.size() && pick.size() < std::min<uint64_t>(kMaxGroup, slots); ++j) {
      SQuery& b = *S->queued[j];
      if (b.cancelled || !is_small(S, b)) continue;
      const uint64_t end = slice_end(b, S->opts.group_edge_updates - work);
      if (end == b.next_it) break;  // not one chunk of it fits what is left
      const uint64_t nb = bytes + b.group_bytes;
      if (S->plain_held + std::max(S->batch_held, nb) > S->budget) {
        make_room(S, nb > S->batch_held ? nb - S->batch_held : 0, nullptr, UINT32_MAX);
        if (S->plain_held + std::max(S->batch_held, nb) > S->budget) {
          if (!pick.empty()) defer(S, b);  // waits for a later group
          break;
        }
      }
      work += (end - b.next_it) * b.per_it;
      bytes = nb;
      pick.push_back(j);
      ends.push_back(end);
      if (work >= S->opts.group_edge_updates) break;
    }
    if (pick.size() >= 2) {
      for (size_t i = 0; i < pick.size(); ++i) {
        auto& b = S->queued[pick[i]];
        job.qs.push_back(b);
        job.it_end.push_back(ends[i]);
        if (!b->admitted_once) {
          b->admitted_once = true;
          S->st.admitted++;
        }
      }
      for (auto j = pick.rbegin(); j != pick.rend(); ++j) S->queued.erase(S->queued.begin() + *j);
      job.group = true;
      job.reserved = bytes > S->batch_held ? bytes - S->batch_held : 0;
      S->batch_held += job.reserved;
      S->group_running = true;
      S->inflight += job.qs.size();
      return true;
    }
  }
  // one query through the plain kernels
  if (!reserve_plain(S, *a, job)) {
    defer(S, *a);
    return false;
  }
  job.qs.push_back(a);
  // a small-graph query runs alone a slice within the group cap, so that
  // arrivals behind it join at its next chunk boundary (all of it when not
  // one chunk fits the cap)
  const uint64_t end = is_small(S, *a) ? slice_end(*a, S->opts.group_edge_updates) : a->plan.it_end;
  job.it_end.push_back(end > a->next_it ? end : a->plan.it_end);
  if (!a->admitted_once) {
    a->admitted_once = true;
    S->st.admitted++;
  }
  S->queued.erase(it);
  S->inflight++;
  return true;
}

static void worker_loop(rs_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  while (true) {
    Job job;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while (!S->stop && !take_job(S, job)) S->cv_work.wait(lk);
      if (job.qs.empty()) break;  // stopping
    }
    const auto t0 = Clock::now();
    std::vector<rs_result> res(job.qs.size());
    rs_status s = have_stream ? RS_OK : RS_EDEVICE;
    if (s == RS_OK && !job.group) {
      SQuery& a = *job.qs[0];
      rs_graph* g = const_cast<rs_graph*>(S->graphs[a.graph_id]);
      QueryPlan plan = a.plan;  // the iterations of this piece
      if (a.next_it != plan.it_begin || job.it_end[0] != plan.it_end) {
        rs_query q = a.q;
        q.motif_count = a.has_motif ? a.motif : nullptr;
        q.it_begin = a.next_it;
        q.it_end = job.it_end[0];
        s = plan_query(g, &q, plan);
      }
      if (s == RS_OK) s = run_plain(g, job.entry->ws, plan, a.tu, nullptr, &res[0], st);
      res[0].status = s;
    } else if (s == RS_OK) {
      std::vector<const rs_graph*> gl;
      std::vector<rs_query> qs;
      for (size_t i = 0; i < job.qs.size(); ++i) {
        const SQuery& a = *job.qs[i];
        rs_query q = a.q;
        q.motif_count = a.has_motif ? a.motif : nullptr;
        q.it_begin = a.next_it;
        q.it_end = job.it_end[i];
        qs.push_back(q);
        gl.push_back(S->graphs[a.graph_id]);
      }
      s = run_batch_impl(gl.data(), qs.data(), (uint32_t)qs.size(), res.data(), nullptr, st, false, S->budget / 4,
                         S->bws);
    }
    const double busy = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st.busy_ms += busy;
      S->st.jobs++;
      if (job.group) {
        S->batch_held = batch_ws_bytes(S->bws);
        S->group_running = false;
        if (held(S) > S->budget) {  // buffers kept from earlier groups overshoot: give them back
          batch_ws_release(S->bws);
          S->batch_held = 0;
        }
      } else if (job.entry) {
        const uint64_t now_bytes = job.entry->ws.bytes();
        S->plain_held = S->plain_held + now_bytes - (job.entry->bytes + job.reserved);
        job.entry->bytes = now_bytes;
        job.entry->busy = false;
      }
      const auto now = Clock::now();
      for (size_t i = 0; i < job.qs.size(); ++i) {
        auto& ap = job.qs[i];
        SQuery& a = *ap;
        rs_result r = res[i];
        if (s != RS_OK && r.status == RS_OK) r.status = s;
        S->inflight--;
        if (a.split || job.it_end[i] < a.plan.it_end) {
          a.split = true;
          S->st.slices++;
        }
        a.acc_F ^= r.fingerprint;
        a.next_it = job.it_end[i];
        a.work = (a.plan.it_end - a.next_it) * a.per_it;
        if (r.status == RS_OK && !a.cancelled && a.next_it < a.plan.it_end) {
          requeue(S, ap);  // the rest of its iterations joins a later group
          continue;
        }
        a.result = r;
        a.result.fingerprint = a.acc_F;
        a.result.yes = a.acc_F != 0;
        if (a.cancelled) a.result.status = RS_ECANCELED;
        const double lat = std::chrono::duration<double, std::milli>(now - a.t_submit).count();
        a.result.device_ms = (float)lat;
        if (a.result.status == RS_OK) {
          S->latencies_ms.push_back(lat);
          S->st.completed++;
        }
        a.done = true;
      }
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  if (have_stream) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
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
    S->opts = opts ? *opts : rs_server_opts{0, 0, 0, 0};
    if (!S->opts.max_inflight) S->opts.max_inflight = 256;
    if (!S->opts.group_edge_updates) S->opts.group_edge_updates = kGroupEdgeUpdates;
    if (!S->opts.streams) S->opts.streams = 2;
    S->opts.streams = std::min(S->opts.streams, kMaxWorkers);
    if (!S->opts.group_max_edges) S->opts.group_max_edges = kGroupMaxEdges;
    if (hipGetDevice(&S->device) != hipSuccess) {
      delete S;
      return RS_EDEVICE;
    }
    S->bws = batch_ws_create();
    S->t_create = Clock::now();
    for (uint32_t i = 0; i < S->opts.streams; ++i) S->workers.emplace_back(worker_loop, S);
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
    const uint64_t m = g->g.m, n = g->g.n;
    a->tu = resolve_tuning(g, a->plan.k, nullptr);
    a->sizes = plain_sizes(m, n, a->plan, a->tu);
    // the wider launches of large queries are taken only where every worker
    // can hold such a workspace at once, within three quarters of the budget:
    // else idle workspaces would be freed and reallocated job after job
    while (a->tu.chunks_per_launch > Tuning{}.chunks_per_launch &&
           a->sizes.total() * s->opts.streams > s->budget / 4 * 3) {
      a->tu.chunks_per_launch /= 2;
      a->sizes = plain_sizes(m, n, a->plan, a->tu);
    }
    if (a->sizes.total() > s->budget) {  // can never run alone
      s->st.rejected++;
      return RS_ENOMEM;
    }
    a->group_bytes = batch_query_bytes(m, n, a->plan);
    a->ticket = s->next_ticket++;
    a->graph_id = graph_id;
    a->q = *q;
    a->has_motif = q->motif_count != nullptr;
    if (a->has_motif) {
      memset(a->motif, 0, sizeof(a->motif));
      for (uint32_t c = 0; c < g->info.n_colours; ++c) a->motif[c] = q->motif_count[c];
    }
    a->per_it = (uint64_t)(a->plan.k - 1) * m;
    a->next_it = a->plan.it_begin;
    a->work = (a->plan.it_end - a->plan.it_begin) * a->per_it;
    a->t_submit = Clock::now();
    const bool trivial = m == 0 || a->plan.k > n || a->plan.it_end == a->plan.it_begin;
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
  // a queued query finishes at once; a running one when its job completes
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
  out->inflight = s->inflight;
  out->held_bytes = s->plain_held + s->batch_held;
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
    for (auto& a : s->queued) {
      a->cancelled = true;
      a->result.status = RS_ECANCELED;
      a->done = true;
      s->st.cancelled++;
    }
    s->queued.clear();
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  for (auto& w : s->workers)
    if (w.joinable()) w.join();
  for (auto& e : s->pool) e->ws.release();
  if (s->bws) batch_ws_destroy(s->bws);
  delete s;
  return RS_OK;
}

}  // extern "C"
