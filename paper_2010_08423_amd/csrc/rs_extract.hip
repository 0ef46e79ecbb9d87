// Extraction of an optimal solution with k fine-grained queries (Sec. 4.7).
//
// Host orchestration over the fine-grained sieve: the path is peeled from its
// last vertex. The first query (k vertices) gives zeta_{u,k,i} per slot; the
// slot with the least time i (then the least u) ends the path, and its time
// is the path's largest timestamp, which is therefore least. Each further
// query (j = k-1 .. 2 vertices) runs on the graph without the vertices found
// so far and without the edges later than the last time found (the
// time-truncated graph tau <- i), with the motif less the found vertices'
// colours; both are constraints of the same sieve (excluded edges get zero
// product rows), so the graph is never rebuilt. A non-zero zeta_{v,j,i}
// proves a restless path with j vertices ending at v at time i that avoids
// the found vertices, so an edge (v, u, t) into the last found vertex u with
// t - delta(v) <= i <= t extends it.
//
// The paper takes the next pair from the reach set R of the smaller query;
// the least reach time of a vertex can lie more than delta(v) before t, so
// the choice here is made among the non-zero slots inside v's waiting
// window. Ties go to the least vertex id, then the least time.
#include <algorithm>
#include <vector>

#include "rs_internal.h"

namespace {

struct CanonEdges {
  std::vector<uint32_t> src, dst, t;  // sorted by (dst, t, src)
  // [first, last) of the edges with the given dst and t in [t0, t1]
  std::pair<uint64_t, uint64_t> range(uint32_t d, uint32_t t0, uint32_t t1) const {
    const uint64_t m = dst.size();
    auto before = [&](uint64_t e, uint32_t dd, uint32_t tt) { return dst[e] < dd || (dst[e] == dd && t[e] < tt); };
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      if (before(mid, d, t0)) lo = mid + 1; else hi = mid;
    }
    uint64_t a = lo;
    hi = m;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) / 2;
      if (before(mid, d, t1 + 1)) lo = mid + 1; else hi = mid;
    }
    return {a, lo};
  }
};

}  // namespace

rs_status rs_extract(const rs_graph* gc, const rs_query* q, const rs_constraints* c, uint32_t* path_vertices,
                     uint32_t* path_times, rs_result* r, void* hip_stream) {
  if (!gc || !q || !r || !path_vertices || !path_times) return RS_EINVAL;
  if (q->it_begin || q->it_end) return RS_EINVAL;
  if (c && (c->n_removed || c->removed || c->t_max)) return RS_EINVAL;
  if (q->k < 2 || q->k > RS_MAX_K) return RS_EINVAL;
  rs_graph* g = const_cast<rs_graph*>(gc);
  const uint32_t n = g->g.n, k = q->k;
  const uint64_t m = g->g.m;
  rs_status s = RS_OK;
  try {
    // the first query decides; it also validates the query and constraints
    std::vector<uint32_t> reach(std::max<uint32_t>(n, 1));
    rs_result first{};
    s = rs_run_fine(g, q, c, reach.data(), nullptr, &first, hip_stream);
    if (s != RS_OK) {
      r->status = s;
      return s;
    }
    r->fingerprint = first.fingerprint;
    r->device_ms = first.device_ms;
    uint32_t best_i = 0xFFFFFFFFu, best_u = 0;
    auto consider = [&](uint32_t u) {
      if (reach[u] < best_i) best_i = reach[u], best_u = u;
    };
    if (c && c->n_targets) {
      for (uint32_t j = 0; j < c->n_targets; ++j) consider(c->targets[j]);
      // the least id among the targets with the least time
      for (uint32_t j = 0; j < c->n_targets; ++j)
        if (reach[c->targets[j]] == best_i) best_u = std::min(best_u, c->targets[j]);
    } else {
      for (uint32_t u = 0; u < n; ++u) consider(u);
    }
    if (best_i == 0xFFFFFFFFu) {
      r->yes = 0;
      r->status = RS_OK;
      return RS_OK;
    }
    CanonEdges E;
    E.src.resize(m);
    E.dst.resize(m);
    E.t.resize(m);
    s = rs_graph_edges(g, E.src.data(), E.dst.data(), E.t.data());
    std::vector<uint8_t> colour;
    std::vector<uint8_t> motif;
    if (s == RS_OK && q->motif_count) {
      colour.resize(std::max<uint32_t>(n, 1));
      if (hipMemcpy(colour.data(), g->g.colour.p, n, hipMemcpyDeviceToHost) != hipSuccess) s = RS_EDEVICE;
      motif.assign(q->motif_count, q->motif_count + g->g.n_colours);
    }
    std::vector<uint8_t> is_source;
    if (c && c->n_sources) {
      is_source.assign(std::max<uint32_t>(n, 1), 0);
      for (uint32_t j = 0; j < c->n_sources; ++j) is_source[c->sources[j]] = 1;
    }
    auto delta_of = [&](uint32_t v) -> uint32_t {
      return c && c->delta_per_vertex ? c->delta_per_vertex[v] : q->delta;
    };
    std::vector<uint32_t> verts{best_u}, times;
    std::vector<uint32_t> removed;
    std::vector<uint8_t> gone(std::max<uint32_t>(n, 1), 0);
    std::vector<uint64_t> zeta(std::max<uint64_t>(m, 1));
    uint32_t u = best_u, i_u = best_i;
    for (uint32_t j = k - 1; j >= 1 && s == RS_OK; --j) {
      removed.push_back(u);
      gone[u] = 1;
      if (!motif.empty()) {
        if (!motif[colour[u]]) {
          s = RS_EDEVICE;  // the found vertex's colour is not in the motif: an internal error
          break;
        }
        --motif[colour[u]];
      }
      // in-edges (v, u, i_u) of the last vertex found, by increasing v
      const auto into = E.range(u, i_u, i_u);
      if (j == 1) {
        uint32_t pick = 0xFFFFFFFFu;
        for (uint64_t e = into.first; e < into.second && pick == 0xFFFFFFFFu; ++e) {
          const uint32_t v = E.src[e];
          if (gone[v] || (!is_source.empty() && !is_source[v]) || (!motif.empty() && motif[colour[v]] != 1))
            continue;
          pick = v;
        }
        if (pick == 0xFFFFFFFFu) {
          s = RS_ERETRY;
          break;
        }
        times.push_back(i_u);
        verts.push_back(pick);
        break;
      }
      rs_query qj = *q;
      qj.k = j;
      qj.motif_count = motif.empty() ? nullptr : motif.data();
      rs_constraints cj{};
      if (c) {
        cj.delta_per_vertex = c->delta_per_vertex;
        cj.sources = c->sources;
        cj.n_sources = c->n_sources;
      }
      cj.removed = removed.data();
      cj.n_removed = (uint32_t)removed.size();
      cj.t_max = i_u;
      rs_result rj{};
      s = rs_run_fine(g, &qj, &cj, reach.data(), zeta.data(), &rj, hip_stream);
      if (s != RS_OK) break;
      r->device_ms += rj.device_ms;
      uint32_t pv = 0xFFFFFFFFu, pi = 0;
      for (uint64_t e = into.first; e < into.second && pv == 0xFFFFFFFFu; ++e) {
        const uint32_t v = E.src[e];
        if (gone[v]) continue;
        const uint32_t dv = delta_of(v);
        const uint32_t t0 = i_u > dv ? i_u - dv : 1;
        const auto win = E.range(v, std::max<uint32_t>(t0, 1), i_u);
        for (uint64_t f = win.first; f < win.second; ++f)
          if (zeta[f]) {  // every edge of a slot carries the slot's zeta
            pv = v;
            pi = E.t[f];
            break;
          }
      }
      if (pv == 0xFFFFFFFFu) {
        s = RS_ERETRY;
        break;
      }
      times.push_back(i_u);
      verts.push_back(pv);
      u = pv;
      i_u = pi;
    }
    if (s == RS_OK) {
      for (uint32_t j = 0; j < k; ++j) path_vertices[j] = verts[k - 1 - j];
      for (uint32_t j = 0; j + 1 < k; ++j) path_times[j] = times[k - 2 - j];
      r->yes = 1;
    }
  } catch (...) {
    s = RS_ENOMEM;
  }
  r->status = s;
  return s;
}
