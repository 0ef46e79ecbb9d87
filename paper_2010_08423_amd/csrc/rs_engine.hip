// Query engine and C ABI: graph lifetime, query validation, the plain
// level-by-level launch sequence, device workspaces and kernel timing.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rs_internal.h"

namespace rs {

rs_status graph_build(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                      const uint32_t* t, const uint8_t* colour, uint32_t n_colours, bool host_ptrs,
                      hipStream_t st, rs_graph** out);

// Launch trace of the plain path (rs_trace_enable; initially on when the
// environment variable RS_TRACE is set to anything but "0"): each launch is
// followed by a stream synchronisation and one line on stderr with its wall
// time and, for a prefix level, the look-back counters (predecessors
// recomputed, probe rounds without an answer). Meant for diagnosing large
// queries; it serialises the launches with the host.
static std::atomic<int> g_trace{-1};
static bool trace_on() {
  int v = g_trace.load(std::memory_order_relaxed);
  if (v < 0) {
    const char* e = getenv("RS_TRACE");
    int want = e && *e && strcmp(e, "0") != 0 ? 1 : 0;
    g_trace.compare_exchange_strong(v, want);
    v = g_trace.load(std::memory_order_relaxed);
  }
  return v > 0;
}

static std::atomic<bool> g_lb_on{false};
static std::atomic<uint64_t> g_lb_recomputes{0}, g_lb_unanswered{0};
bool lookback_counting() { return g_lb_on.load(std::memory_order_relaxed); }
void lookback_add(uint64_t recomputes, uint64_t unanswered) {
  g_lb_recomputes.fetch_add(recomputes);
  g_lb_unanswered.fetch_add(unanswered);
}

static thread_local std::string g_last_error;
void set_last_error(const std::string& s) { g_last_error = s; }

// ---------------------------------------------------------------------------
// DevBuf
// ---------------------------------------------------------------------------
rs_status DevBuf::reserve(size_t need, hipStream_t st, bool zero) {
  if (need <= bytes && p) return RS_OK;
  release();
  if (need == 0) need = 8;
  void* q = nullptr;
  if (hipMalloc(&q, need) != hipSuccess) {
    (void)hipGetLastError();
    return RS_ENOMEM;
  }
  p = q;
  bytes = need;
  if (zero) {
    hipError_t e = launch_fill64(static_cast<uint64_t*>(p), 0, need / 8, st);
    if (e == hipSuccess && need % 8) e = hipMemsetAsync(static_cast<char*>(p) + (need & ~size_t(7)), 0, need % 8, st);
    if (e != hipSuccess) return RS_EDEVICE;
  }
  return RS_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

// ---------------------------------------------------------------------------
// Kernel timing
// ---------------------------------------------------------------------------
static const char* kClassNames[KC_COUNT] = {"level_scan", "level_first", "level_top", "qtable",
                                            "ztable",     "window",      "batch",     "literal_level"};
static std::mutex g_prof_mu;
static std::atomic<bool> g_prof_on{false};
struct PendingEv {
  KernelClass kc;
  hipEvent_t e0, e1;
  double bytes;
};
static std::vector<PendingEv> g_pending;
static uint64_t g_launches[KC_COUNT];
static double g_ms[KC_COUNT];
static double g_bytes[KC_COUNT];

bool profiling_on() { return g_prof_on.load(std::memory_order_relaxed); }

ProfScope::ProfScope(KernelClass k, hipStream_t s, double b, bool allowed) : kc(k), st(s), bytes(b) {
  if (!allowed || !profiling_on()) return;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    e0 = e1 = nullptr;
    return;
  }
  (void)hipEventRecord(e0, st);
}

ProfScope::~ProfScope() {
  if (!e0) return;
  (void)hipEventRecord(e1, st);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_pending.push_back({kc, e0, e1, bytes});
}

void profile_flush() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<PendingEv> keep;
  for (auto& p : g_pending) {
    if (hipEventQuery(p.e1) != hipSuccess) {
      keep.push_back(p);
      continue;
    }
    float ms = 0;
    if (hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
      g_launches[p.kc]++;
      g_ms[p.kc] += ms;
      g_bytes[p.kc] += p.bytes;
    }
    (void)hipEventDestroy(p.e0);
    (void)hipEventDestroy(p.e1);
  }
  g_pending.swap(keep);
}

// ---------------------------------------------------------------------------
// Query planning
// ---------------------------------------------------------------------------
static uint32_t round_kq(uint32_t k) { return (k + 3) / 4 * 4; }

rs_status plan_query(const rs_graph* g, const rs_query* q, QueryPlan& qp) {
  if (!g || !q) return RS_EINVAL;
  if (q->k < 2 || q->k > RS_MAX_K) return RS_EINVAL;
  const uint64_t total = 1ull << q->k;
  qp = QueryPlan();
  qp.k = q->k;
  qp.kq = round_kq(q->k);
  qp.delta = q->delta;
  qp.seed = q->seed;
  qp.it_begin = q->it_begin;
  qp.it_end = q->it_end;
  if (qp.it_begin == 0 && qp.it_end == 0) qp.it_end = total;
  if (qp.it_begin > qp.it_end || qp.it_end > total) return RS_EINVAL;
  if (q->motif_count) {
    const uint32_t nc = g->info.n_colours;
    if (nc == 0) return RS_EINVAL;
    uint32_t s = 0;
    for (uint32_t c = 0; c < nc; ++c) {
      qp.mu[c] = q->motif_count[c];
      qp.shade_off[c] = (uint8_t)s;
      s += q->motif_count[c];
    }
    if (s != q->k) return RS_EINVAL;
    qp.motif = true;
  }
  qp.chunk_first = qp.it_begin / 64;
  qp.chunk_last = (qp.it_end + 63) / 64;
  return RS_OK;
}

Tuning resolve_tuning(const rs_graph* g, uint32_t k, const rs_tuning* t) {
  Tuning tu;
  if (g && g->has_tuned[k]) {
    tu = g->tuned[k];
  } else if (g && k >= 10 && 16ull * (g->g.m + g->g.n) * 512 <= (96ull << 30)) {
    // at least 16 chunks: groups of 8 halve the launches and their tails
    // (10^7-edge motif query, k = 10: 92.7 ms against 96.9 ms with groups of
    // 4; one group of all 16 ran 110 ms), while the prefix state of a group
    // stays within 96 GiB
    tu.chunks_per_launch = 8;
  }
  if (t) {
    if (t->edges_per_tile) tu.edges_per_tile = t->edges_per_tile;
    if (t->top_edges_per_tile) tu.top_edges_per_tile = t->top_edges_per_tile;
    if (t->chunks_per_launch) tu.chunks_per_launch = t->chunks_per_launch;
    if (t->waves_per_block) tu.waves_per_block = tu.top_waves_per_block = t->waves_per_block;
    if (t->max_slots) tu.max_slots = t->max_slots;
    if (t->chunks_per_wave) tu.chunks_per_wave = t->chunks_per_wave;
  }
  if (tu.chunks_per_wave != 1 && tu.chunks_per_wave != 2) tu.chunks_per_wave = 2;
  if (tu.edges_per_tile != 8 && tu.edges_per_tile != 16) tu.edges_per_tile = 16;
  tu.top_edges_per_tile = std::min(std::max(tu.top_edges_per_tile, 1u), 4096u);
  if (tu.waves_per_block != 1 && tu.waves_per_block != 2 && tu.waves_per_block != 4) tu.waves_per_block = 4;
  if (tu.top_waves_per_block != 1 && tu.top_waves_per_block != 2 && tu.top_waves_per_block != 4)
    tu.top_waves_per_block = 2;
  if (tu.chunks_per_launch < 1) tu.chunks_per_launch = 1;
  return tu;
}

static uint64_t chunks_of(const QueryPlan& qp) { return qp.chunk_last - qp.chunk_first; }

// The launch shape a plain query runs with. The last level runs two chunks
// per wave when every chunk group holds an even number of chunks from an even
// chunk (so a pair's iterations differ only in bit 6) and the rows have at
// least 7 entries (k >= 7, which two chunks imply for a full range); the
// fine-grained last level reads one chunk per wave. (Two chunks per wave in
// the prefix levels measured slower.) Idempotent.
static Tuning query_tuning(Tuning tu, const QueryPlan& qp, bool fine) {
  const uint64_t nch = chunks_of(qp);
  const uint64_t cpl = std::min<uint64_t>(tu.chunks_per_launch, nch);
  const bool pairs = tu.chunks_per_wave == 2 && !fine && qp.k >= 7 && nch >= 2 && nch % 2 == 0 &&
                     qp.chunk_first % 2 == 0 && cpl % 2 == 0;
  if (!pairs) tu.chunks_per_wave = 1;
  return tu;
}

// Algorithmic HBM bytes of one level launch over `chunks` 64-iteration
// chunks: what the exact computation has to move once edges whose window is
// empty, or whose product reaches no read slot, are skipped and only read
// slots are stored. Per chunk: two 512-byte window rows per gathered edge and
// one 512-byte row per stored slot; per launch: the entries of the level's
// compacted list (slot, window bounds and flags, 13 bytes each) and the
// kq-entry rows of the entries that form a product (at level 2 also their
// substitution rows). k = 2 reads every edge.
double scan_bytes(const NeedCounts& nc, uint64_t m, uint32_t kq, uint64_t chunks, bool first) {
  const double stores = 512.0 * (double)(nc.ref_slots + nc.ref_lead);
  if (first)  // level 2: no gathers; product and substitution rows of needed edges
    return stores * (double)chunks + 9.0 * (double)nc.kept + 16.0 * kq * (double)nc.needed;
  return (1024.0 * (double)nc.live_needed + stores) * (double)chunks + 13.0 * (double)nc.kept +
         8.0 * kq * (double)nc.live_needed;
}
// Level 3 from window rows: no gathers; the q, D and source z rows of the
// product entries.
double drows_bytes(const NeedCounts& nc, uint32_t kq, uint64_t chunks) {
  const double stores = 512.0 * (double)(nc.ref_slots + nc.ref_lead);
  return stores * (double)chunks + 13.0 * (double)nc.kept + 24.0 * kq * (double)nc.live_needed;
}
// units: the entries the last level runs over (its windows, grouped or not;
// 0 = every non-empty window).
double top_bytes(const NeedCounts& nc, uint64_t m, uint32_t kq, uint64_t chunks, bool first, uint64_t units = 0) {
  if (first) return 8.0 * (double)m + 16.0 * kq * (double)m;
  const double u = units ? (double)units : (double)nc.live;
  return 1024.0 * u * (double)chunks + 8.0 * u + 8.0 * kq * u;
}

uint64_t table_lo_bytes(uint64_t m) { return 4 * (m + kEdgePad); }
uint64_t table_z_bytes(uint64_t n, uint32_t kq) { return 8 * n * kq; }
uint64_t table_q_bytes(uint64_t m, uint32_t k, uint32_t kq) { return 8 * (m * (k - 1) + kEdgePad) * kq; }
uint64_t table_need_bytes(uint64_t m, uint32_t k) { return (uint64_t)need_levels(k) * need_stride(m); }

// ---------------------------------------------------------------------------
// Plain path: setup kernels, then per chunk group levels 2..k.
// ---------------------------------------------------------------------------
// Buffer sizes (bytes) one query needs in a plain workspace.
PlainSizes plain_sizes(uint64_t m, uint64_t n, const QueryPlan& qp, const Tuning& tu_in, const QueryExtras* ex) {
  const Tuning tu = query_tuning(tu_in, qp, ex && ex->fine);
  PlainSizes s;
  const uint32_t k = qp.k, kq = qp.kq;
  const uint64_t nchunks = std::max<uint64_t>(chunks_of(qp), 1);
  const uint64_t cpl = std::max<uint64_t>(std::min<uint64_t>(tu.chunks_per_launch, nchunks), 1);
  const uint64_t tiles = (m + tu.edges_per_tile - 1) / tu.edges_per_tile;
  TopArgs ta{};
  ta.m = (uint32_t)m;
  ta.edges_per_wave = tu.top_edges_per_tile;
  // Rows per chunk of the last level's partial sums; the single-chunk launch
  // bounds every group: gc * blocks(gc) <= cpl * blocks(1).
  const uint32_t tblocks = top_blocks(ta, k == 2, kq, 1, tu);
  s.lo = table_lo_bytes(m);
  s.z = table_z_bytes(n, kq);
  // k = 2 reads the product rows of every edge; deeper queries read the rows
  // of their compacted lists
  s.q = k == 2 ? table_q_bytes(m, k, kq) : 0;
  s.lists = k >= 3 ? compact_bytes(m, k, kq) : 0;
  s.rr = k >= 4 && m ? rrows_bytes(m, kq) : 0;
  // the last level by distinct windows pays for its sort (once per query)
  // when the last level runs for at least two groups of chunks
  const uint64_t groups = (nchunks + cpl - 1) / cpl;
  s.grp = k >= 3 && m && groups >= 2 && !(ex && ex->fine) ? group_bytes(m, n, kq) : 0;
  s.p = 8 * (m + n) * 64 * cpl;
  s.partial = 8 * 64 * cpl * (uint64_t)tblocks + 4 * cpl;  // block rows, then one range ticket per chunk
  s.fsum = 8 * (1ull << k);
  s.ref = 2 * flag_ref_bytes(m, n);  // two levels' read marks, alternating
  s.need = table_need_bytes(m, k);
  s.cover = 8 * (m + n + 1) + 8 * ((m + n + 1 + 1023) / 1024);  // two difference arrays and block sums
  s.records = 1024 * cpl * tiles;
  // work-balanced runs, cut for the grid width of a full chunk group
  s.run_w2 = s.run_w3 = s.run_w4 = s.run_stride = 0;
  s.run_pre = s.run_bsum = s.run_boff = s.run_bounds = 0;
  if (k >= 3 && m) {
    const uint32_t E = tu.edges_per_tile;
    s.run_w2 = scan_waves(kq, E, true, (uint32_t)tiles, (uint32_t)cpl, tu.waves_per_block);
    // level 3 is formed from window rows when level 2 is folded (k >= 4); its
    // kernel holds fewer registers than the gathering one of levels >= 4, so
    // more of its waves fit
    s.run_w3 = scan_waves(kq, E, false, (uint32_t)tiles, (uint32_t)cpl, tu.waves_per_block, s.rr != 0);
    s.run_w4 = scan_waves(kq, E, false, (uint32_t)tiles, (uint32_t)cpl, tu.waves_per_block);
    s.run_stride = std::max(std::max(s.run_w2, s.run_w3), s.run_w4) + 1;
    const uint64_t levels = k - 2, nb = (tiles + 1023) / 1024;
    s.run_pre = 4 * tiles * levels;
    s.run_bsum = s.run_boff = 4 * nb * levels;
    s.run_bounds = 4ull * s.run_stride * levels;
  }
  s.dv = ex && ex->delta_v ? 4 * n : 0;
  s.smask = ex && ex->smask ? n : 0;
  s.tmask = ex && ex->tmask ? n : 0;
  s.rmask = ex && ex->rmask ? n : 0;
  const bool fine = ex && ex->fine;
  s.fine_t = fine ? 8 * m : 0;
  s.fine_z = fine ? 8 * m : 0;
  s.fine_r = fine ? 4 * n : 0;
  return s;
}

uint64_t PlainSizes::total() const {
  return lo + z + q + 2 * p + partial + fsum + 64 + ref + need + cover + 2 * records + run_pre + run_bsum + run_boff +
         run_bounds + lists + rr + grp + dv + smask + tmask + rmask + fine_t + fine_z + fine_r;
}

uint64_t plain_footprint(const rs_graph* g, const QueryPlan& qp, const Tuning& tu) {
  return plain_sizes(g->g.m, g->g.n, qp, tu).total();
}

// The buffers of one query in ws: reserved (grown) in an allocating
// workspace, carved from the borrowed scratch region otherwise. p_elems is
// the prefix-state size of one chunk of this graph.
static rs_status acquire_buffers(PlainWorkspace& ws, const PlainSizes& sz, uint64_t p_elems, hipStream_t st) {
  if (ws.scratch) {
    uint64_t off = 0;
    bool fits = true;
    auto carve = [&](DevBuf& b, uint64_t bytes) {
      bytes = std::max<uint64_t>((bytes + 255) & ~255ull, 256);
      if (off + bytes > ws.scratch_bytes) fits = false;
      b.p = fits ? ws.scratch + off : nullptr;
      b.bytes = fits ? bytes : 0;
      off += bytes;
    };
    carve(ws.agg, sz.records);
    carve(ws.incl, sz.records);
    carve(ws.lo, sz.lo);
    carve(ws.z, sz.z);
    carve(ws.q, sz.q);
    carve(ws.p0, sz.p);
    carve(ws.p1, sz.p);
    carve(ws.partial, sz.partial);
    carve(ws.fsum, sz.fsum);
    carve(ws.out, 64);
    carve(ws.ref, sz.ref);
    carve(ws.need, sz.need);
    carve(ws.cov_diff, sz.cover);
    carve(ws.run_pre, sz.run_pre);
    carve(ws.run_bsum, sz.run_bsum);
    carve(ws.run_boff, sz.run_boff);
    carve(ws.run_bounds, sz.run_bounds);
    carve(ws.lists, sz.lists);
    carve(ws.rr, sz.rr);
    carve(ws.grp, sz.grp);
    carve(ws.dv, sz.dv);
    carve(ws.smask, sz.smask);
    carve(ws.tmask, sz.tmask);
    carve(ws.rmask, sz.rmask);
    carve(ws.fine_t, sz.fine_t);
    carve(ws.fine_z, sz.fine_z);
    carve(ws.fine_r, sz.fine_r);
    if (!fits) {
      set_last_error("query workspace of " + std::to_string(off) + " bytes exceeds the " +
                     std::to_string(ws.scratch_bytes) + "-byte scratch of the no-allocation entry point");
      return RS_ENOMEM;
    }
    // The region keeps the previous call's contents: tagged look-back records
    // must start at tag 0, which no launch uses (epochs restart at 1). The
    // prefix states need no clearing (every slot a window reads is written
    // before it is read, leading slots included).
    RS_HIP(launch_fill64(ws.agg.as<uint64_t>(), 0, 2 * ws.agg.bytes / 8, st));  // agg and incl are adjacent
    ws.epoch = 0;
    ws.p_elems_per_chunk = p_elems;
    return RS_OK;
  }
  if (ws.p_elems_per_chunk != p_elems) {  // slot layout differs: rezero
    ws.p0.release();
    ws.p1.release();
    ws.p_elems_per_chunk = p_elems;
  }
  if (ws.lo.reserve(sz.lo, st, false) || ws.z.reserve(sz.z, st, false) || ws.q.reserve(sz.q, st, false) ||
      ws.p0.reserve(sz.p, st, true) || ws.p1.reserve(sz.p, st, true) || ws.partial.reserve(sz.partial, st, false) ||
      ws.fsum.reserve(sz.fsum, st, false) || ws.out.reserve(64, st, false) || ws.ref.reserve(sz.ref, st, false) ||
      ws.need.reserve(sz.need, st, false) || ws.cov_diff.reserve(sz.cover, st, false) ||
      ws.run_pre.reserve(sz.run_pre, st, false) || ws.run_bsum.reserve(sz.run_bsum, st, false) ||
      ws.run_boff.reserve(sz.run_boff, st, false) || ws.run_bounds.reserve(sz.run_bounds, st, false) ||
      (sz.lists && ws.lists.reserve(sz.lists, st, false)) || (sz.rr && ws.rr.reserve(sz.rr, st, false)) ||
      (sz.grp && ws.grp.reserve(sz.grp, st, false)) || (sz.dv && ws.dv.reserve(sz.dv, st, false)) ||
      (sz.smask && ws.smask.reserve(sz.smask, st, false)) || (sz.tmask && ws.tmask.reserve(sz.tmask, st, false)) ||
      (sz.rmask && ws.rmask.reserve(sz.rmask, st, false)) ||
      (sz.fine_t && ws.fine_t.reserve(sz.fine_t, st, false)) || (sz.fine_z && ws.fine_z.reserve(sz.fine_z, st, false)) ||
      (sz.fine_r && ws.fine_r.reserve(sz.fine_r, st, false)))
    return RS_ENOMEM;
  if (ws.agg.bytes < sz.records || ws.incl.bytes < sz.records) {
    // tagged records start at epoch 0, which no launch uses
    if (ws.agg.reserve(sz.records, st, true) || ws.incl.reserve(sz.records, st, true)) return RS_ENOMEM;
    ws.epoch = 0;
  }
  return RS_OK;
}

rs_status run_plain(rs_graph* g, PlainWorkspace& ws, const QueryPlan& qp, const Tuning& tu_in, uint64_t* per_it_host,
                    rs_result* r, hipStream_t st, QueryExtras* ex) {
  const GraphDev& G = g->g;
  const bool fine = ex && ex->fine;
  const Tuning tu = query_tuning(tu_in, qp, fine);
  const uint64_t m = G.m, n = G.n;
  const uint64_t span = qp.it_end - qp.it_begin;
  const bool timed = !ws.scratch;  // the no-allocation workspace records no events
  if (timed && !ws.ev0) {
    RS_HIP(hipEventCreate(&ws.ev0));
    RS_HIP(hipEventCreate(&ws.ev1));
  }
  if (timed) RS_HIP(hipEventRecord(ws.ev0, st));
  uint64_t F = 0;
  // No path with k distinct vertices can exist: F is exactly 0.
  const bool trivial = m == 0 || qp.k > n || span == 0;
  if (!trivial) {
    const uint32_t k = qp.k, kq = qp.kq;
    const uint64_t nchunks = chunks_of(qp);
    const uint64_t cpl = std::min<uint64_t>(tu.chunks_per_launch, nchunks);
    const uint32_t E = tu.edges_per_tile;
    const uint64_t tiles = (m + E - 1) / E;
    const uint64_t p_elems = (m + n) * 64;
    const PlainSizes sz = plain_sizes(m, n, qp, tu, ex);
    const bool fold2 = sz.rr != 0;  // k >= 4: level 2 folded into level 3 (rs_rrows.hip)
    GroupView gv{};                  // the last level by distinct windows (rs_group.hip)
    bool grouped = false;
    uint64_t top_units = 0;          // the last level's entries, when counted (profiling)
    RS_TRY(acquire_buffers(ws, sz, p_elems, st));
    // constraints (host arrays, copied in) and fine-grained output buffers
    const uint32_t* dv = nullptr;
    EdgeFilter filt;
    if (ex) filt.t_max = ex->t_max;
    if (sz.dv) {
      RS_HIP(hipMemcpyAsync(ws.dv.p, ex->delta_v, 4 * n, hipMemcpyHostToDevice, st));
      dv = ws.dv.as<uint32_t>();
    }
    if (sz.smask) {
      RS_HIP(hipMemcpyAsync(ws.smask.p, ex->smask, n, hipMemcpyHostToDevice, st));
      filt.smask = ws.smask.as<uint8_t>();
    }
    if (sz.tmask) {
      RS_HIP(hipMemcpyAsync(ws.tmask.p, ex->tmask, n, hipMemcpyHostToDevice, st));
      filt.tmask = ws.tmask.as<uint8_t>();
    }
    if (sz.rmask) {
      RS_HIP(hipMemcpyAsync(ws.rmask.p, ex->rmask, n, hipMemcpyHostToDevice, st));
      filt.rmask = ws.rmask.as<uint8_t>();
    }
    if (fine) {
      RS_HIP(launch_fill64(ws.fine_t.as<uint64_t>(), 0, m, st));
      RS_HIP(launch_fill32(ws.fine_r.as<uint32_t>(), 0xFFFFFFFFu, n, st));
    }
    auto need_of = [&](uint32_t l) { return ws.need.as<uint8_t>() + (uint64_t)(l - 2) * need_stride(m); };
    const bool tr = timed && trace_on();
    const bool count_lb = !tr && timed && lookback_counting();  // totals for the query, read at its end
    if ((tr || count_lb) && ws.lb_stats.reserve(16, st, true)) return RS_ENOMEM;
    if (count_lb) RS_HIP(launch_fill64(ws.lb_stats.as<uint64_t>(), 0, 2, st));
    auto t_last = std::chrono::steady_clock::now();
    // one trace line: waits for the launches so far, reads the counters
    auto trace = [&](const char* what, uint32_t l, uint64_t c0, uint32_t gc, bool counters) -> rs_status {
      RS_HIP(hipStreamSynchronize(st));
      unsigned long long h[2] = {0, 0};
      if (counters) RS_HIP(hipMemcpy(h, ws.lb_stats.p, sizeof(h), hipMemcpyDeviceToHost));
      if (counters && lookback_counting()) lookback_add(h[0], h[1]);
      const auto now = std::chrono::steady_clock::now();
      fprintf(stderr, "[rs-trace] %s level %u chunks %llu..%llu: %.3f ms", what, l, (unsigned long long)c0,
              (unsigned long long)(c0 + gc), std::chrono::duration<double, std::milli>(now - t_last).count());
      if (counters) fprintf(stderr, ", look-back recomputes %llu, unanswered probe rounds %llu", h[0], h[1]);
      fprintf(stderr, "\n");
      fflush(stderr);
      t_last = std::chrono::steady_clock::now();
      return RS_OK;
    };
    if (tr) {
      const rs_status ts = trace("workspace", 0, 0, 0, false);
      if (ts != RS_OK) return ts;
    }
    {
      ProfScope ps(KC_ZTABLE, st, 8.0 * n * kq, timed);
      RS_HIP(launch_ztable(ws.z.as<uint64_t>(), (uint32_t)n, qp, G.colour.as<uint8_t>(), st));
    }
    const uint32_t run_w2 = sz.run_w2, run_w3 = sz.run_w3, run_w4 = sz.run_w4, run_stride = sz.run_stride;
    CompactArgs ca{};
    if (k >= 3) {
      const uint64_t L = k - 1, lst = list_stride(m);
      ca.e_src = G.e_src.as<uint32_t>();
      ca.e_dst = G.e_dst.as<uint32_t>();
      ca.e_t = G.e_t.as<uint32_t>();
      ca.e_out = G.e_out.as<uint32_t>();
      ca.hi = G.hi.as<uint32_t>();
      ca.lo = ws.lo.as<uint32_t>();
      ca.need = need_of(2);
      ca.need_stride = need_stride(m);
      ca.m = (uint32_t)m;
      ca.k = k;
      ca.kq = kq;
      ca.nb = (uint32_t)((m + kCostBlock - 1) / kCostBlock);
      ca.list_stride = lst;
      ca.rows = ws.lists.as<uint64_t>();
      ca.u32 = (uint32_t*)(ca.rows + L * lst * kq);
      ca.u8 = (uint8_t*)(ca.u32 + L * 4 * lst);
      ca.bsum = (uint32_t*)(((uintptr_t)(ca.u8 + L * lst) + 3) & ~(uintptr_t)3);
      ca.boff = ca.bsum + L * ca.nb;
      ca.count = ca.boff + L * ca.nb;
    }
    {
      ProfScope ps(KC_WINDOW, st, 16.0 * m, timed);
      RS_HIP(launch_window(G.e_src.as<uint32_t>(), G.e_t.as<uint32_t>(), G.in_off.as<uint32_t>(),
                           ws.lo.as<uint32_t>(), (uint32_t)m, qp.delta, dv, st));
      // Flags per prefix level, from the last one down: level l stores the
      // slots the windows of level l+1's product edges read, and forms a
      // product only for edges inside one of those windows (level k-1: the
      // windows of every last-level edge).
      RS_HIP(launch_flags(G.e_out.as<uint32_t>(), G.hi.as<uint32_t>(), ws.lo.as<uint32_t>(), (uint32_t)m,
                          (uint32_t)n, k, need_of(2), need_stride(m), ws.ref.as<uint8_t>(), ws.cov_diff.as<uint32_t>(),
                          st));
      // compacted edge lists of levels 2..k and the work-balanced runs of
      // the prefix lists, cut for the grid width of the first chunk group
      // (later groups launch the same width)
      if (k >= 3) {
        RS_HIP(launch_compact(ca, st));
        const uint32_t wpb = tu.waves_per_block;
        RS_HIP(launch_compact_bounds(ca, E, (uint32_t)tiles, run_w2, run_w3, run_w4, run_skew(run_w2, wpb),
                                     run_skew(run_w3, wpb), run_skew(run_w4, wpb), ws.run_pre.as<uint32_t>(),
                                     ws.run_bsum.as<uint32_t>(), ws.run_boff.as<uint32_t>(),
                                     ws.run_bounds.as<uint32_t>(), run_stride, st));
      }
    }
    if (tr) {
      const rs_status ts = trace("setup (z table, windows, flags, runs)", 0, 0, 0, false);
      if (ts != RS_OK) return ts;
    }
    // Counts for the byte accounting of timed launches: measured once per
    // (delta, k) (a synchronising read-back), only while kernel timing is on.
    std::vector<NeedCounts> ncs(k + 1);
    if (timed && profiling_on()) {
      std::lock_guard<std::mutex> lk(g->counts_mu);
      auto it = g->need_counts.find({qp.delta, k});
      if (it == g->need_counts.end()) {
        if (g->counts_dev.reserve(64, st, true)) return RS_ENOMEM;
        for (uint32_t l = 2; l < k; ++l) {
          unsigned long long h[6] = {0, 0, 0, 0, 0, 0};
          RS_HIP(launch_fill64(g->counts_dev.as<uint64_t>(), 0, 8, st));
          RS_HIP(launch_need_counts(G.hi.as<uint32_t>(), ws.lo.as<uint32_t>(), need_of(l), (uint32_t)m,
                                    g->counts_dev.as<unsigned long long>(), st));
          RS_HIP(hipMemcpyAsync(h, g->counts_dev.p, sizeof(h), hipMemcpyDeviceToHost, st));
          RS_HIP(hipStreamSynchronize(st));
          ncs[l].live = h[0];
          ncs[l].live_needed = h[1];
          ncs[l].needed = h[2];
          ncs[l].ref_slots = h[3];
          ncs[l].ref_lead = h[4];
          ncs[l].kept = h[5];
        }
        ncs[k] = ncs[k > 2 ? k - 1 : k];  // the last level needs only the window count
        if (k == 2) {  // no prefix level: count the windows alone
          unsigned long long h[6] = {0, 0, 0, 0, 0, 0};
          RS_HIP(launch_fill64(g->counts_dev.as<uint64_t>(), 0, 8, st));
          RS_HIP(launch_need_counts(G.hi.as<uint32_t>(), ws.lo.as<uint32_t>(), need_of(2), (uint32_t)m,
                                    g->counts_dev.as<unsigned long long>(), st));
          RS_HIP(hipMemcpyAsync(h, g->counts_dev.p, sizeof(h), hipMemcpyDeviceToHost, st));
          RS_HIP(hipStreamSynchronize(st));
          ncs[2].live = h[0];
        }
        g->need_counts[{qp.delta, k}] = ncs;
      } else {
        ncs = it->second;
      }
    }
    {
      // product rows: of the compacted lists' product entries (k >= 3), else
      // of every edge, with the source and target constraints applied
      ProfScope ps(KC_QTABLE, st, (double)m * (12.0 + 8.0 * kq * (k - 1)), timed);
      if (k >= 3) {
        // (level 2's own rows are not used when it is folded into level 3)
        RS_HIP(launch_compact_rows(ca, ws.z.as<uint64_t>(), qp.seed, nullptr, filt, kq, st, fold2 ? 1 : 0));
        // level 2 as iteration-independent prefix rows, level 3's window rows
        if (fold2) RS_HIP(launch_rrows(ca, G.in_off.as<uint32_t>(), ws.z.as<uint64_t>(), qp.seed, nullptr, filt, kq,
                                       ws.rr.as<uint8_t>(), st));
        // the last level's entries grouped by window
        if (sz.grp) {
          uint32_t n_last = 0, n_groups = 0;
          RS_HIP(hipMemcpyAsync(&n_last, ca.count + (k - 2), 4, hipMemcpyDeviceToHost, st));
          RS_HIP(hipStreamSynchronize(st));
          gv = group_view(ws.grp.as<uint8_t>(), m, kq);
          RS_HIP(launch_group(ca.list(k - 2), ca.count + (k - 2), n_last, m + n, kq, gv, group_temp_bytes(m, n), st));
          grouped = true;
          if (profiling_on() && timed) {
            RS_HIP(hipMemcpyAsync(&n_groups, gv.gcount, 4, hipMemcpyDeviceToHost, st));
            RS_HIP(hipStreamSynchronize(st));
            top_units = n_groups;
          }
        }
      } else {
        RS_HIP(launch_qtable(G.e_src.as<uint32_t>(), G.e_dst.as<uint32_t>(), G.e_t.as<uint32_t>(),
                             ws.z.as<uint64_t>(), ws.q.as<uint64_t>(), (uint32_t)m, qp, st));
        if (filt.any())
          RS_HIP(launch_mask_rows(ws.q.as<uint64_t>(), G.e_src.as<uint32_t>(), G.e_dst.as<uint32_t>(),
                                  G.e_t.as<uint32_t>(), filt, (uint32_t)m, kq, st));
      }
    }
    if (tr) {
      const rs_status ts = trace("product rows", 0, 0, 0, false);
      if (ts != RS_OK) return ts;
    }
    RS_HIP(launch_fill64(ws.fsum.as<uint64_t>(), 0, 1ull << k, st));
    for (uint64_t c0 = qp.chunk_first; c0 < qp.chunk_last; c0 += cpl) {
      const uint32_t gc = (uint32_t)std::min<uint64_t>(cpl, qp.chunk_last - c0);
      uint64_t* prev = ws.p0.as<uint64_t>();
      uint64_t* cur = ws.p1.as<uint64_t>();
      for (uint32_t l = 2; l <= k; ++l) {
        const bool first = l == 2;
        if (fold2 && first) continue;  // folded into level 3's window rows
        const bool drows = fold2 && l == 3;
        if (l < k) {
          if (++ws.epoch >= (1u << 30)) {
            RS_HIP(launch_fill64(ws.agg.as<uint64_t>(), 0, ws.agg.bytes / 8, st));
            RS_HIP(launch_fill64(ws.incl.as<uint64_t>(), 0, ws.incl.bytes / 8, st));
            ws.epoch = 1;
          }
          const LevelList Lc = ca.list(l - 2);
          ScanArgs a;
          a.e_src = Lc.chi;  // level 2, and level 3 from window rows: the source of each entry
          a.e_out = Lc.cslot;
          a.hi = Lc.chi;
          a.lo = Lc.clo;
          a.q = Lc.cq;
          a.z = ws.z.as<uint64_t>();
          a.p_prev = prev;
          a.p_cur = cur;
          a.p_stride = p_elems;
          a.chunk_base = c0 * 64;
          a.m = (uint32_t)m;
          a.n_tiles = (uint32_t)tiles;
          a.k = k;
          a.epoch = ws.epoch;
          a.agg = ws.agg.as<uint64_t>();
          a.incl = ws.incl.as<uint64_t>();
          a.need = Lc.cflag;
          a.bounds = ws.run_bounds.as<uint32_t>() + (uint64_t)(l - 2) * run_stride;
          a.waves = first ? run_w2 : (l == 3 ? run_w3 : run_w4);
          a.count = ca.count + (l - 2);
          if (drows) a.d = ca.list(0).cq;  // the D rows, indexed like level 3's entries
          if (tr) RS_HIP(launch_fill64(ws.lb_stats.as<uint64_t>(), 0, 2, st));
          if (tr || count_lb) a.lb_stats = ws.lb_stats.as<unsigned long long>();
          {
            ProfScope ps(first || drows ? KC_FIRST : KC_SCAN, st,
                         drows ? drows_bytes(ncs[l], kq, gc) : scan_bytes(ncs[l], m, kq, gc, first), timed);
            RS_HIP(launch_scan(a, first, kq, gc, tu, st));
          }
          if (tr) {
            const rs_status ts = trace("prefix", l, c0, gc, true);
            if (ts != RS_OK) return ts;
          }
          std::swap(prev, cur);
        } else {
          TopArgs a;
          a.e_src = G.e_src.as<uint32_t>();
          if (grouped) {  // one entry per distinct window, its rows summed
            a.hi = gv.ghi;
            a.lo = gv.glo;
            a.q = gv.gq;
            a.count = gv.gcount;
            a.ce = nullptr;
          } else if (k >= 3) {  // the compacted list of non-empty windows
            const LevelList Lc = ca.list(k - 2);
            a.hi = Lc.chi;
            a.lo = Lc.clo;
            a.q = Lc.cq;
            a.count = ca.count + (k - 2);
            a.ce = Lc.ce;
          } else {
            a.hi = G.hi.as<uint32_t>();
            a.lo = ws.lo.as<uint32_t>();
            a.q = ws.q.as<uint64_t>();
          }
          a.z = ws.z.as<uint64_t>();
          a.p_prev = prev;
          a.p_stride = p_elems;
          a.chunk_base = c0 * 64;
          a.it_begin = qp.it_begin;
          a.it_end = qp.it_end;
          a.m = (uint32_t)m;
          a.edges_per_wave = tu.top_edges_per_tile;
          a.k = k;
          a.partial = ws.partial.as<uint64_t>();
          a.fsum = ws.fsum.as<uint64_t>();
          // Ranges by tickets when a wave has many of them (the 10^7-edge motif
          // query: about 270 per wave, 6.47 -> 6.28 ms per launch); with few
          // per wave the atomics cost more than the balance gains (10^6-edge
          // path query, about 14 per wave: 0.42 -> 0.47 ms). The tickets follow
          // the block rows of a full chunk group.
          const uint64_t t1 = top_blocks(a, first, kq, 1, tu);
          const uint64_t top_waves = (uint64_t)top_blocks(a, first, kq, gc, tu) * tu.top_waves_per_block;
          if (!fine && (m + tu.top_edges_per_tile - 1) / tu.top_edges_per_tile >= 32 * top_waves) {
            a.ticket = reinterpret_cast<uint32_t*>(ws.partial.as<uint8_t>() + 8 * 64 * cpl * t1);
            RS_HIP(launch_fill32(a.ticket, 0, gc, st));
          }
          {
            ProfScope ps(KC_TOP, st, top_bytes(ncs[k], m, kq, gc, first, top_units), timed);
            if (fine)
              RS_HIP(launch_top_fine(a, first, kq, gc, tu, ws.fine_t.as<uint64_t>(), st));
            else
              RS_HIP(launch_top(a, first, kq, gc, tu, st));
          }
          if (tr) {
            const rs_status ts = trace("last", l, c0, gc, false);
            if (ts != RS_OK) return ts;
          }
        }
      }
    }
    if (fine) {
      // zeta per slot, reach times; F = the XOR of the per-edge sums
      RS_HIP(launch_fine_slots(G.e_dst.as<uint32_t>(), G.e_t.as<uint32_t>(), ws.fine_t.as<uint64_t>(), (uint32_t)m,
                               ws.fine_z.as<uint64_t>(), ws.fine_r.as<uint32_t>(), st));
      RS_HIP(launch_xor_reduce(ws.fine_t.as<uint64_t>(), 0, m, ws.out.as<uint64_t>(), st));
      RS_HIP(hipMemcpyAsync(&F, ws.out.p, 8, hipMemcpyDeviceToHost, st));
      RS_HIP(hipMemcpyAsync(ex->reach, ws.fine_r.p, 4 * n, hipMemcpyDeviceToHost, st));
      if (ex->zeta) RS_HIP(hipMemcpyAsync(ex->zeta, ws.fine_z.p, 8 * m, hipMemcpyDeviceToHost, st));
      if (timed) RS_HIP(hipEventRecord(ws.ev1, st));
      RS_HIP(hipStreamSynchronize(st));
      if (count_lb) {
        unsigned long long h[2] = {0, 0};
        RS_HIP(hipMemcpy(h, ws.lb_stats.p, sizeof(h), hipMemcpyDeviceToHost));
        lookback_add(h[0], h[1]);
      }
      ex->reached = 0;
      for (uint64_t u = 0; u < n; ++u) ex->reached += ex->reach[u] != 0xFFFFFFFFu;
      float ms = 0;
      if (timed) (void)hipEventElapsedTime(&ms, ws.ev0, ws.ev1);
      if (profiling_on()) profile_flush();
      r->fingerprint = F;
      r->yes = ex->reached != 0;
      r->status = RS_OK;
      r->device_ms = ms;
      return RS_OK;
    }
    RS_HIP(launch_xor_reduce(ws.fsum.as<uint64_t>(), qp.it_begin, qp.it_end, ws.out.as<uint64_t>(), st));
    RS_HIP(hipMemcpyAsync(&F, ws.out.p, 8, hipMemcpyDeviceToHost, st));
    if (per_it_host)
      RS_HIP(hipMemcpyAsync(per_it_host, ws.fsum.as<uint64_t>() + qp.it_begin, 8 * span,
                            hipMemcpyDeviceToHost, st));
    if (timed) RS_HIP(hipEventRecord(ws.ev1, st));
    RS_HIP(hipStreamSynchronize(st));
    if (count_lb) {
      unsigned long long h[2] = {0, 0};
      RS_HIP(hipMemcpy(h, ws.lb_stats.p, sizeof(h), hipMemcpyDeviceToHost));
      lookback_add(h[0], h[1]);
    }
  } else {
    if (per_it_host)
      for (uint64_t i = 0; i < span; ++i) per_it_host[i] = 0;
    if (fine) {  // nothing reaches anything
      for (uint64_t u = 0; u < n; ++u) ex->reach[u] = 0xFFFFFFFFu;
      if (ex->zeta)
        for (uint64_t e = 0; e < m; ++e) ex->zeta[e] = 0;
      ex->reached = 0;
    }
    if (timed) RS_HIP(hipEventRecord(ws.ev1, st));
    RS_HIP(hipStreamSynchronize(st));
  }
  float ms = 0;
  if (timed) (void)hipEventElapsedTime(&ms, ws.ev0, ws.ev1);
  if (profiling_on()) profile_flush();
  r->fingerprint = F;
  r->yes = F != 0;
  r->status = RS_OK;
  r->device_ms = ms;
  return RS_OK;
}

// ---------------------------------------------------------------------------
// No-allocation workspace: one file-scope device array per GPU. In host code
// `scratch` names a host-side stand-in, not device memory; its address on a
// device comes from hipGetSymbolAddress with that device current, taken once
// per device and kept, and only that address is ever handed to kernels or
// fills. The array keeps the last call's contents.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

struct NoAllocDevice {
  std::mutex mu;            // one query at a time per device (each call syncs its stream)
  uint8_t* base = nullptr;  // this device's copy of scratch
  PlainWorkspace ws;        // buffers borrowed from base
};
static std::mutex g_noalloc_mu;
static std::map<int, NoAllocDevice*> g_noalloc;  // by device; lives until process end

static rs_status noalloc_device(int dev, NoAllocDevice** out) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc.find(dev);
  if (it != g_noalloc.end()) {
    *out = it->second;
    return RS_OK;
  }
  int cur = 0;
  RS_HIP(hipGetDevice(&cur));
  if (cur != dev) RS_HIP(hipSetDevice(dev));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p) {
    set_last_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return RS_EDEVICE;
  }
  NoAllocDevice* d = new (std::nothrow) NoAllocDevice();
  if (!d) return RS_ENOMEM;
  d->base = static_cast<uint8_t*>(p);
  d->ws.scratch = d->base;
  d->ws.scratch_bytes = kNoAllocScratchBytes;
  g_noalloc[dev] = d;
  *out = d;
  return RS_OK;
}

}  // namespace rs

using namespace rs;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* rs_status_str(rs_status s) {
  switch (s) {
    case RS_OK: return "RS_OK";
    case RS_EINVAL: return "RS_EINVAL: invalid argument";
    case RS_ENOMEM: return "RS_ENOMEM: out of memory or over budget";
    case RS_EDEVICE: return "RS_EDEVICE: device error";
    case RS_EBUSY: return "RS_EBUSY: busy";
    case RS_ECANCELED: return "RS_ECANCELED: cancelled";
    case RS_ENOTFOUND: return "RS_ENOTFOUND: not found";
    case RS_ETIMEOUT: return "RS_ETIMEOUT: timed out";
    default: return "unknown rs_status";
  }
}

const char* rs_version(void) { return "librestless_sieve 0.1 (gfx950)"; }

const char* rs_last_error(void) { return g_last_error.c_str(); }

rs_status rs_graph_create(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                          const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                          void* hip_stream, rs_graph** out) {
  try {
    return graph_build(n, m, src, dst, t, colour, n_colours, true, (hipStream_t)hip_stream, out);
  } catch (...) {
    return RS_ENOMEM;
  }
}

rs_status rs_graph_create_device(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                                 const uint32_t* t, const uint8_t* colour, uint32_t n_colours,
                                 void* hip_stream, rs_graph** out) {
  try {
    return graph_build(n, m, src, dst, t, colour, n_colours, false, (hipStream_t)hip_stream, out);
  } catch (...) {
    return RS_ENOMEM;
  }
}

rs_status rs_graph_get_info(const rs_graph* g, rs_graph_info* out) {
  if (!g || !out) return RS_EINVAL;
  *out = g->info;
  return RS_OK;
}

rs_status rs_graph_edges(const rs_graph* g, uint32_t* src, uint32_t* dst, uint32_t* t) {
  if (!g) return RS_EINVAL;
  const uint64_t m = g->g.m;
  if (!m) return RS_OK;
  if (src) RS_HIP(hipMemcpy(src, g->g.e_src.p, 4 * m, hipMemcpyDeviceToHost));
  if (dst) RS_HIP(hipMemcpy(dst, g->g.e_dst.p, 4 * m, hipMemcpyDeviceToHost));
  if (t) RS_HIP(hipMemcpy(t, g->g.e_t.p, 4 * m, hipMemcpyDeviceToHost));
  return RS_OK;
}

rs_status rs_graph_destroy(rs_graph* g) {
  if (!g) return RS_OK;
  (void)hipDeviceSynchronize();
  for (DevBuf* b : {&g->g.e_src, &g->g.e_dst, &g->g.e_t, &g->g.e_out, &g->g.hi, &g->g.in_off, &g->g.colour,
                    &g->counts_dev})
    b->release();
  g->ws.release();
  g->lit.release();
  delete g;
  return RS_OK;
}

rs_status rs_query_footprint(const rs_graph* g, const rs_query* q, uint64_t* bytes) {
  if (!bytes) return RS_EINVAL;
  QueryPlan qp;
  RS_TRY(plan_query(g, q, qp));
  *bytes = plain_footprint(g, qp, resolve_tuning(g, qp.k, nullptr));
  return RS_OK;
}

rs_status rs_run_ex(const rs_graph* gc, const rs_query* q, const rs_tuning* tune,
                    uint64_t* per_iteration, rs_result* r, void* hip_stream) {
  if (!r) return RS_EINVAL;
  QueryPlan qp;
  rs_status s = plan_query(gc, q, qp);
  if (s != RS_OK) {
    r->status = s;
    return s;
  }
  rs_graph* g = const_cast<rs_graph*>(gc);
  if (tune && tune->edges_per_tile == 8 && g->g.m > kMaxEdgesE8) {
    set_last_error("8-edge tiles are not accepted on graphs of more than 4e6 edges");
    r->status = RS_EINVAL;
    return RS_EINVAL;
  }
  try {
    std::lock_guard<std::mutex> lk(g->mu);
    s = run_plain(g, g->ws, qp, resolve_tuning(g, qp.k, tune), per_iteration, r, (hipStream_t)hip_stream);
  } catch (...) {
    s = RS_ENOMEM;
  }
  r->status = s;
  return s;
}

rs_status rs_run(const rs_graph* g, const rs_query* q, rs_result* r, void* hip_stream) {
  return rs_run_ex(g, q, nullptr, nullptr, r, hip_stream);
}

// Host masks and per-vertex resting times of a constraint set (validated).
struct HostConstraints {
  std::vector<uint8_t> smask, tmask, rmask;
  QueryExtras ex;
};
static rs_status make_constraints(const rs_graph* g, const rs_constraints* c, HostConstraints& h) {
  h.ex = QueryExtras();
  if (!c) return RS_OK;
  const uint32_t n = g->g.n;
  if ((c->n_sources && !c->sources) || (c->n_targets && !c->targets) || (c->n_removed && !c->removed))
    return RS_EINVAL;
  h.ex.delta_v = c->delta_per_vertex;
  h.ex.t_max = c->t_max;
  if (c->n_removed) {
    h.rmask.assign(std::max<uint32_t>(n, 1), 0);
    for (uint32_t i = 0; i < c->n_removed; ++i) {
      if (c->removed[i] >= n) return RS_EINVAL;
      h.rmask[c->removed[i]] = 1;
    }
    h.ex.rmask = h.rmask.data();
  }
  if (c->n_sources) {
    h.smask.assign(std::max<uint32_t>(n, 1), 0);
    for (uint32_t i = 0; i < c->n_sources; ++i) {
      if (c->sources[i] >= n) return RS_EINVAL;
      h.smask[c->sources[i]] = 1;
    }
    h.ex.smask = h.smask.data();
  }
  if (c->n_targets) {
    h.tmask.assign(std::max<uint32_t>(n, 1), 0);
    for (uint32_t i = 0; i < c->n_targets; ++i) {
      if (c->targets[i] >= n) return RS_EINVAL;
      h.tmask[c->targets[i]] = 1;
    }
    h.ex.tmask = h.tmask.data();
  }
  return RS_OK;
}

rs_status rs_run_constrained(const rs_graph* gc, const rs_query* q, const rs_constraints* c, uint64_t* per_iteration,
                             rs_result* r, void* hip_stream) {
  if (!r) return RS_EINVAL;
  QueryPlan qp;
  rs_status s = plan_query(gc, q, qp);
  rs_graph* g = const_cast<rs_graph*>(gc);
  try {
    HostConstraints h;
    if (s == RS_OK) s = make_constraints(g, c, h);
    if (s == RS_OK) {
      std::lock_guard<std::mutex> lk(g->mu);
      s = run_plain(g, g->ws, qp, resolve_tuning(g, qp.k, nullptr), per_iteration, r, (hipStream_t)hip_stream, &h.ex);
    }
  } catch (...) {
    s = RS_ENOMEM;
  }
  r->status = s;
  return s;
}

rs_status rs_run_fine(const rs_graph* gc, const rs_query* q, const rs_constraints* c, uint32_t* reach_time,
                      uint64_t* slot_zeta, rs_result* r, void* hip_stream) {
  if (!r || !reach_time) return RS_EINVAL;
  QueryPlan qp;
  rs_status s = plan_query(gc, q, qp);
  rs_graph* g = const_cast<rs_graph*>(gc);
  try {
    HostConstraints h;
    if (s == RS_OK) s = make_constraints(g, c, h);
    if (s == RS_OK) {
      h.ex.fine = true;
      h.ex.reach = reach_time;
      h.ex.zeta = slot_zeta;
      std::lock_guard<std::mutex> lk(g->mu);
      s = run_plain(g, g->ws, qp, resolve_tuning(g, qp.k, nullptr), nullptr, r, (hipStream_t)hip_stream, &h.ex);
    }
  } catch (...) {
    s = RS_ENOMEM;
  }
  r->status = s;
  return s;
}

rs_status rs_reach_at_most(const rs_graph* gc, const rs_query* q, const rs_constraints* c, uint32_t* reach_time,
                           uint32_t* reach_vertices, rs_result* r, void* hip_stream) {
  if (!r || !reach_time || !q || q->motif_count || q->it_begin || q->it_end) return RS_EINVAL;
  rs_graph* g = const_cast<rs_graph*>(gc);
  rs_status s = RS_OK;
  try {
    const uint32_t n = gc ? gc->g.n : 0;
    std::vector<uint32_t> rk(std::max<uint32_t>(n, 1));
    for (uint32_t u = 0; u < n; ++u) {
      reach_time[u] = 0xFFFFFFFFu;
      if (reach_vertices) reach_vertices[u] = 0;
    }
    uint64_t F = 0;
    float ms = 0;
    uint64_t reached = 0;
    for (uint32_t kk = 2; kk <= q->k && s == RS_OK; ++kk) {
      rs_query qk = *q;
      qk.k = kk;
      rs_result rr{};
      s = rs_run_fine(g, &qk, c, rk.data(), nullptr, &rr, hip_stream);
      if (s != RS_OK) break;
      F ^= rr.fingerprint;
      ms += rr.device_ms;
      for (uint32_t u = 0; u < n; ++u) {
        if (rk[u] == 0xFFFFFFFFu) continue;
        if (reach_vertices && reach_vertices[u] == 0) reach_vertices[u] = kk;
        if (reach_time[u] == 0xFFFFFFFFu) ++reached;
        reach_time[u] = std::min(reach_time[u], rk[u]);
      }
    }
    if (s == RS_OK) {
      r->fingerprint = F;
      r->yes = reached != 0;
      r->device_ms = ms;
    }
  } catch (...) {
    s = RS_ENOMEM;
  }
  r->status = s;
  return s;
}

rs_status rs_run_noalloc(const rs_graph* gc, const rs_query* q, uint64_t* per_iteration, rs_result* r,
                         void* hip_stream) {
  if (!r) return RS_EINVAL;
  QueryPlan qp;
  rs_status s = plan_query(gc, q, qp);
  if (s != RS_OK) {
    r->status = s;
    return s;
  }
  rs_graph* g = const_cast<rs_graph*>(gc);
  try {
    NoAllocDevice* d = nullptr;
    s = noalloc_device(g->device, &d);
    if (s == RS_OK) {
      // one 64-iteration chunk per launch keeps the prefix state smallest
      Tuning tu = resolve_tuning(g, qp.k, nullptr);
      tu.chunks_per_launch = 1;
      std::lock_guard<std::mutex> lk(d->mu);
      s = run_plain(g, d->ws, qp, tu, per_iteration, r, (hipStream_t)hip_stream);
    }
  } catch (...) {
    s = RS_ENOMEM;
  }
  r->status = s;
  return s;
}

rs_status rs_trace_enable(int on) {
  g_trace.store(on != 0 ? 1 : 0);
  return RS_OK;
}

rs_status rs_lookback_count(int on) {
  if (on) {
    g_lb_recomputes = 0;
    g_lb_unanswered = 0;
  }
  g_lb_on.store(on != 0);
  return RS_OK;
}

rs_status rs_lookback_get(uint64_t* recomputes, uint64_t* unanswered_rounds) {
  if (!recomputes || !unanswered_rounds) return RS_EINVAL;
  *recomputes = g_lb_recomputes.load();
  *unanswered_rounds = g_lb_unanswered.load();
  return RS_OK;
}

rs_status rs_profile_enable(int on) {
  g_prof_on.store(on != 0);
  return RS_OK;
}

rs_status rs_profile_reset(void) {
  (void)hipDeviceSynchronize();
  profile_flush();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int i = 0; i < KC_COUNT; ++i) {
    g_launches[i] = 0;
    g_ms[i] = 0;
    g_bytes[i] = 0;
  }
  return RS_OK;
}

rs_status rs_profile_get(const char* kernel_class, uint64_t* launches, double* total_ms,
                         double* algorithmic_bytes) {
  if (!kernel_class) return RS_EINVAL;
  profile_flush();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (int i = 0; i < KC_COUNT; ++i) {
    if (strcmp(kernel_class, kClassNames[i]) == 0) {
      if (launches) *launches = g_launches[i];
      if (total_ms) *total_ms = g_ms[i];
      if (algorithmic_bytes) *algorithmic_bytes = g_bytes[i];
      return RS_OK;
    }
  }
  return RS_ENOTFOUND;
}

}  // extern "C"
