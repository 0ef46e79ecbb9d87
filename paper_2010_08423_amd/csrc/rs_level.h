// Level-step device code shared by the per-level kernels and the persistent
// batch kernel.
//
// Layout (one query, one 64-iteration chunk):
//   * Edges are sorted by (dst, t, src); the in-edges of vertex u form the
//     segment [in_off[u], in_off[u+1]) ordered by time.
//   * The prefix state P of a level has m + n slots. Slot in_off[u] + u holds 0
//     (written by the tile holding u's first in-edge; vertices without in-edges
//     are never read through it, their windows have hi == lo); slot
//     e + dst(e) + 1 holds the XOR of the level's values over the edges of
//     dst(e)'s segment up to and including e. Each slot stores 64 uint64, one
//     per sieve iteration of the chunk (lane = iteration), 512 contiguous bytes.
//   * For edge e = (v -> u, t) the restless window of Eq. (poly-enc:1) - the
//     arrivals at v with time in [t - delta, t] - is P[hi(e)] ^ P[lo(e)], with
//     hi/lo the slots bounding that time range in v's segment.
//
// Level step (Eq. poly-enc:1 with y per edge and position): for level l and
// iteration L, c_l(e) = z^L_u * y_{e,l-1} * W where W = z^L_v at level 2 and the
// window sum at level >= 3. The factor z^L_u * y_{e,l-1} equals
// XOR_{j in L} q_j(e) with q_j(e) = z_{u,j} * y_{e,l-1} precomputed per edge and
// level; within a wavefront the edge is uniform, so the q row is one scalar
// load and each lane forms its own subset XOR (6 lane bits + chunk bits).
// One GF(2^64) product remains per edge-update, and none where the window is
// empty (hi == lo): at levels >= 3 such an edge contributes exactly zero, so
// the wave skips its gathers and product on a uniform branch.
//
// Prefix levels cut the edge list into one contiguous run of tiles (E
// consecutive edges each) per wave and keep a running XOR per lane along the
// run, so a segment receives its carry from the preceding tiles in registers.
// Only a segment that crosses into a run from the one before needs a carry
// from another wave: it comes through one decoupled look-back per run on
// self-validating per-run records (device-scope atomic stores and loads that
// bypass the per-XCD L2; no fences, no atomic read-modify-write).
#pragma once

#include "rs_device.h"
#include "rs_internal.h"

namespace rs {

// Read-only per-edge and per-vertex arrays are read through the constant
// address space so that wave-uniform accesses become scalar loads.
typedef __attribute__((address_space(4))) const uint64_t cu64;
typedef __attribute__((address_space(4))) const uint32_t cu32;
__device__ __forceinline__ cu64* as_const(const uint64_t* p) { return (cu64*)p; }
__device__ __forceinline__ cu32* as_const(const uint32_t* p) { return (cu32*)p; }

// ---------------------------------------------------------------------------
// Device-coherent accesses (bypass the per-XCD L2's non-coherent caching).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void st_dev64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev64(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// P-state accesses (kernel boundaries order the levels). Loads go through
// the global address space explicitly: a generic (flat) load would also count
// against the LDS wait counter and make every table lookup wait for the
// gathers.
typedef __attribute__((address_space(1))) const uint64_t gu64;
// Prefix-state rows are read and written once per launch at random slots of
// gigabytes of state, so they carry the non-temporal hint and leave the
// caches to the list indices and product rows, which the chunks of a run
// share: 10^7-edge motif query, levels 4..9 4.12-4.15 -> 4.02-4.06 ms and the
// last level 6.19-6.31 -> 5.97-6.09 ms per launch (same-box A/B).
__device__ __forceinline__ uint64_t p_load(const uint64_t* p) { return __builtin_nontemporal_load((gu64*)p); }
__device__ __forceinline__ void p_store(uint64_t* p, uint64_t v) { __builtin_nontemporal_store(v, p); }

// Per-lane subset XOR  XOR_{j in L} row[j]  for the iteration L = cb + lane
// (cb a multiple of 64): bits 0..5 of L come from the lane, higher bits from cb.
template <int KQ>
__device__ __forceinline__ uint64_t subset_xor(cu64* row, uint64_t cb, const uint32_t (&mk)[6]) {
  uint64_t h = 0;  // wave-uniform: chunk bits select row entries 6..KQ-1
#pragma unroll
  for (int j = 6; j < KQ; ++j) h ^= row[j] & (0ull - ((cb >> j) & 1ull));
  uint32_t lo = lo32(h), hi = hi32(h);
#pragma unroll
  for (int b = 0; b < 6 && b < KQ; ++b) {
    const uint64_t v = row[b];
    lo = and_xor(lo32(v), mk[b], lo);
    hi = and_xor(hi32(v), mk[b], hi);
  }
  return mk64(lo, hi);
}

__device__ __forceinline__ void lane_masks(uint32_t lane, uint32_t (&mk)[6]) {
#pragma unroll
  for (int b = 0; b < 6; ++b) mk[b] = ((lane >> b) & 1u) ? 0xFFFFFFFFu : 0u;
}

// Look-back records. A tile publishes, per lane, two 64-bit words each holding
// 32 bits of its 64-bit value and a 32-bit tag (epoch << 2 | state), written
// with device-scope atomic stores. A reader accepts a record only when both
// of its lane's words carry the expected tag, so no fence or separate flag
// is needed and publishing never waits.
__device__ __forceinline__ uint32_t rec_tag(uint32_t epoch, uint32_t state) { return (epoch << 2) | state; }

__device__ __forceinline__ void publish(uint64_t* rec, uint64_t fi, uint32_t lane, uint64_t v, uint32_t tag) {
  uint64_t* p = rec + (fi * kLanes + lane) * 2;
  st_dev64(p, (uint64_t)lo32(v) | ((uint64_t)tag << 32));
  st_dev64(p + 1, (uint64_t)hi32(v) | ((uint64_t)tag << 32));
}

// Lane's value of record fi if both words carry `tag`.
__device__ __forceinline__ bool read_rec(const uint64_t* rec, uint64_t fi, uint32_t lane, uint32_t tag,
                                         uint64_t* v) {
  const uint64_t* p = rec + (fi * kLanes + lane) * 2;
  const uint64_t w0 = ld_dev64(p), w1 = ld_dev64(p + 1);
  *v = mk64(lo32(w0), lo32(w1));
  return hi32(w0) == tag && hi32(w1) == tag;
}

// Everything one prefix-level tile needs; all fields wave-uniform.
struct TileCtx {
  const uint32_t* e_src;
  const uint32_t* e_out;
  const uint32_t* hi;
  const uint32_t* lo;
  const uint64_t* q;   // this level's [m][KQ] rows
  const uint64_t* z;   // [n][KQ] rows (level 2; level 3 from window rows)
  const uint64_t* d;   // level 3 from window rows: [entries][KQ] L-independent window rows
  const uint64_t* pp;  // previous level, this chunk
  uint64_t* pc;        // this level, this chunk
  uint64_t cb;         // first iteration of the chunk
  uint32_t m;
  uint32_t n_tiles;
  uint32_t epoch;
  uint64_t row0;       // record row of this (chunk, level)
  uint64_t* agg;       // [tiles][64][2] records: XOR of the tile's open segment part
  uint64_t* incl;      // [tiles][64][2] records: inclusive prefix of that segment
  const uint8_t* need; // per edge: which of its P slots some window reads (see mark_need)
  unsigned long long* lb_stats;  // null, or [2]: recomputed predecessors, unanswered probe rounds
  const uint32_t* bounds;        // null (runs of equal length), or [W+1] first tile of each run
};

// First tile of run r of a prefix level: from the bounds array when the runs
// are balanced by work, else r equal runs of `len` tiles (clamped at the end).
__device__ __forceinline__ uint32_t run_begin(const TileCtx& c, int64_t r, uint32_t len) {
  if (c.bounds) return as_const(c.bounds)[r];
  const uint64_t t = (uint64_t)r * len;
  return t < c.n_tiles ? (uint32_t)t : c.n_tiles;
}

// N consecutive entries of an index array in one scalar load (the arrays are
// padded past m, so the load stays in bounds for the last tile).
template <int N>
struct IdxN {
  uint32_t v[N];
};
template <int N>
__device__ __forceinline__ IdxN<N> load_idx(const uint32_t* p) {
  cu32* q = as_const(p);
  IdxN<N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.v[i] = q[i];
  return r;
}

// Row gathered at the last level by empty windows (and by edges past the
// range end): all zero, so both gathers of such an edge hit the same cached
// line and XOR to zero.
static __device__ const uint64_t kZeroRow[kLanes] = {0};

// The product rows (and, at level 2, the substitution rows) of a group of N
// consecutive edges, spread over the wave: lane l holds entries l*P .. l*P+P-1
// of the N x KQ block (P = N*KQ/64 rounded up; P divides KQ, so one lane's
// entries belong to one edge). They arrive by vector loads issued with the
// window gathers, so their latency overlaps; an entry is broadcast to a scalar
// register right before its use. (Scalar loads would share the wait counter
// of the LDS table accesses and be waited for at the first table read.)
template <int KQ, int N>
struct RowBlock {
  static constexpr int P = (N * KQ + 63) / 64;
  uint64_t v[P];
};

// Product rows of edges e0 .. e0+N-1: contiguous at q + e0*KQ.
template <int KQ, int N>
__device__ __forceinline__ void load_qrows(RowBlock<KQ, N>& rb, const uint64_t* q, uint32_t e0, uint32_t lane) {
  constexpr int P = RowBlock<KQ, N>::P;
  const uint32_t g = lane * P;
#pragma unroll
  for (int p = 0; p < P; ++p) rb.v[p] = 0;
  if (N * KQ >= 64 || g < N * KQ) {
#pragma unroll
    for (int p = 0; p < P; ++p) rb.v[p] = *(gu64*)(q + (uint64_t)e0 * KQ + g + p);
  }
}

// Substitution rows of the sources of edges e0 .. e0+N-1 (rows of edges at or
// past ne are not loaded).
template <int KQ, int N>
__device__ __forceinline__ void load_zrows(RowBlock<KQ, N>& rb, const uint64_t* z, const uint32_t* e_src,
                                           uint32_t e0, uint32_t ne, uint32_t lane) {
  constexpr int P = RowBlock<KQ, N>::P;
  const uint32_t g = lane * P, i = g / KQ, j = g % KQ;
#pragma unroll
  for (int p = 0; p < P; ++p) rb.v[p] = 0;
  if ((N * KQ >= 64 || g < N * KQ) && i < ne) {
    const uint32_t src = *(__attribute__((address_space(1))) const uint32_t*)(e_src + e0 + i);
#pragma unroll
    for (int p = 0; p < P; ++p) rb.v[p] = *(gu64*)(z + (uint64_t)src * KQ + j + p);
  }
}

// Entry j of edge i's row, wave-uniform.
template <int KQ, int N>
__device__ __forceinline__ uint64_t row_entry(const RowBlock<KQ, N>& rb, int i, int j) {
  constexpr int P = RowBlock<KQ, N>::P;
  const int g = i * KQ + j;
  const uint64_t v = rb.v[g % P];
  return mk64(__builtin_amdgcn_readlane(lo32(v), g / P), __builtin_amdgcn_readlane(hi32(v), g / P));
}

// Per-lane subset XOR of edge i's row (see subset_xor).
template <int KQ, int N>
__device__ __forceinline__ uint64_t subset_xor(const RowBlock<KQ, N>& rb, int i, uint64_t cb,
                                               const uint32_t (&mk)[6]) {
  uint64_t h = 0;
#pragma unroll
  for (int j = 6; j < KQ; ++j) h ^= row_entry<KQ, N>(rb, i, j) & (0ull - ((cb >> j) & 1ull));
  uint32_t lo = lo32(h), hi = hi32(h);
#pragma unroll
  for (int b = 0; b < 6 && b < KQ; ++b) {
    const uint64_t v = row_entry<KQ, N>(rb, i, b);
    lo = and_xor(lo32(v), mk[b], lo);
    hi = and_xor(hi32(v), mk[b], hi);
  }
  return mk64(lo, hi);
}

// Loads the tile's indices (three scalar loads) and issues the window gathers
// of its live edges. An edge whose window is empty (hi == lo, its sum is
// zero), whose product no read slot needs, or that lies past the tile end
// skips its gathers on a wave-uniform branch; with a sixth of the edges live
// at levels >= 3, gathering a cached zero row for the others instead cost 13 %
// of the launch (0.49 against 0.43 ms on the 10^6-edge graph; 11 % on the
// 10^7-edge motif query). The two rows of a window land in separate registers
// (w, w2) and are XORed at the product: XORed inside the branch, each live
// edge waited for its own gathers before the next edge's were issued. Kept
// apart they are all in flight together, at 115 VGPRs (four waves per SIMD):
// levels 4..9 of the motif query 4.89 -> 4.72 ms per launch.
template <int KQ, int E, bool FIRST>
__device__ __forceinline__ void tile_inputs(const TileCtx& c, uint32_t e0, uint32_t ne, uint32_t lane,
                                            const IdxN<E / 4>& need, uint32_t (&slot)[E], uint32_t (&ia)[E],
                                            uint64_t (&w)[E], uint64_t (&w2)[E]) {
  const IdxN<E> so = load_idx<E>(c.e_out + e0);
#pragma unroll
  for (int i = 0; i < E; ++i) slot[i] = so.v[i];
  if (FIRST) {
    const IdxN<E> sr = load_idx<E>(c.e_src + e0);
#pragma unroll
    for (int i = 0; i < E; ++i) ia[i] = sr.v[i];
  } else {
    const IdxN<E> h = load_idx<E>(c.hi + e0);
    const IdxN<E> l = load_idx<E>(c.lo + e0);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      // gather only where the product is needed: bit 2, which at levels >= 3
      // also requires a non-empty window and is zero past m
      const bool live = (need.v[i / 4] >> (8 * (i % 4) + 2)) & 1u;
      // wave-uniform branch: only live edges issue their two gathers
      uint64_t v = 0, v2 = 0;
      if (live) {
        v = p_load(c.pp + (uint64_t)h.v[i] * kLanes + lane);
        v2 = p_load(c.pp + (uint64_t)l.v[i] * kLanes + lane);
      }
      w[i] = v;
      w2[i] = v2;
      ia[i] = live;
    }
  }
}

// c_l(e) for edge i of the tile. DR (level 3 from window rows): the window
// is z^L_a * D^L(e), formed from the source's z row and the entry's D row.
template <int KQ, int E, bool FIRST, bool DR = false>
__device__ __forceinline__ uint64_t edge_value(const TileCtx& c, uint32_t e, uint32_t a, uint64_t w,
                                               const uint32_t (&mk)[6], uint64_t* tab) {
  const uint64_t aL = subset_xor<KQ>(as_const(c.q) + (uint64_t)e * KQ, c.cb, mk);
  uint64_t wv = w;
  if (FIRST || DR) wv = subset_xor<KQ>(as_const(c.z) + (uint64_t)a * KQ, c.cb, mk);
  if (DR) wv = gf_mul(tab, wv, subset_xor<KQ>(as_const(c.d) + (uint64_t)e * KQ, c.cb, mk));
  return gf_mul(tab, aL, wv);
}

// What tile j publishes, recomputed by a waiting successor: the XOR of the
// level values over the tile's open segment part (from the last segment start
// inside the tile, else from the tile start). *started tells whether a
// segment starts inside the tile, i.e. whether the value is inclusive. A
// rarely taken path, written edge by edge to keep register use low.
template <int KQ, int E, bool FIRST, bool DR = false>
__device__ uint64_t tile_open_part(const TileCtx& c, uint32_t j, uint32_t lane, const uint32_t (&mk)[6],
                                   uint64_t* tab, bool* started) {
  cu32* hi_idx = as_const(c.hi);
  cu32* lo_idx = as_const(c.lo);
  cu32* e_src = as_const(c.e_src);
  const uint32_t e0 = j * (uint32_t)E;
  const uint32_t e1 = min(e0 + (uint32_t)E, c.m);
  bool st = e0 == 0 || (c.need[e0] & 8u);
  uint64_t acc = 0;
#pragma unroll 1
  for (uint32_t e = e0; e < e1; ++e) {
    if (e > e0 && (c.need[e] & 8u)) {  // the running XOR restarts here
      acc = 0;
      st = true;
    }
    if (!FIRST && !DR && hi_idx[e] == lo_idx[e]) continue;  // empty window: contributes zero
    if (!(c.need[e] & 4u)) continue;                         // reaches no read slot
    const uint64_t w = (FIRST || DR) ? 0
                                     : p_load(c.pp + (uint64_t)hi_idx[e] * kLanes + lane) ^
                                           p_load(c.pp + (uint64_t)lo_idx[e] * kLanes + lane);
    acc ^= edge_value<KQ, E, FIRST, DR>(c, e, (FIRST || DR) ? e_src[e] : 0u, w, mk, tab);
  }
  *started = st;
  return acc;
}

// Spins (each a flag round trip plus a short sleep) before a waiting wave
// stops relying on its predecessor's record and recomputes that part itself.
// Records are published once per wave, when its run of tiles is done, so a
// predecessor is usually just finishing: it is waited for. The budget only
// bounds the wait (about 10 ms) for a predecessor that never got to run.
constexpr uint32_t kFallbackSpins = 4096;

// XOR of the level values of the segment part preceding run `run` (its first
// tile continues a segment). Runs publish one record each, at their last
// tile; run r covers tiles run_begin(r) .. run_begin(r + 1) - 1, and a run
// without tiles (possible when the runs are balanced by work) publishes
// nothing and is skipped. The nearest non-empty predecessor's two records are
// read first, which ends most walks in one memory round trip. After that,
// each round probes up to 64 predecessor runs at once (lane l reads the tags
// of run top - l's record, lane-0 words), then absorbs the leading run of
// published records up to and including the nearest inclusive one, every
// lane validating its own words; a carry that has to cross d runs costs about
// d/64 memory round trips. A predecessor that stays unpublished is recomputed
// here, tile by tile from the end of its run, so every wait is bounded
// whatever order the waves run in.
template <int KQ, int E, bool FIRST, bool DR = false>
__device__ uint64_t look_back(const TileCtx& c, uint32_t run, uint32_t len, uint32_t lane, const uint32_t (&mk)[6],
                              uint64_t* tab) {
  uint64_t carry = 0;
  uint32_t spins = 0, spin_total = 0;
  const uint32_t t_agg = rec_tag(c.epoch, kFlagAgg), t_inc = rec_tag(c.epoch, kFlagIncl);
  const uint32_t t0 = run_begin(c, run, len);
  // nearest non-empty predecessor run: the one holding tile t0 - 1
  int64_t top = (int64_t)run - 1;
  while (top > 0 && run_begin(c, top, len) == t0) --top;
  {
    uint64_t vi, va;
    const uint64_t fi = c.row0 + (t0 - 1);
    const bool oki = read_rec(c.incl, fi, lane, t_inc, &vi);
    const bool oka = read_rec(c.agg, fi, lane, t_agg, &va);
    if (__ballot(!oki) == 0) return vi;
    if (__ballot(!oka) == 0) {
      carry = va;
      --top;
    }
  }
  uint32_t width = 4;
  while (top >= 0) {
    const int64_t r = top - (int64_t)lane;
    bool ready = false, inc = false;
    if (r >= 0 && lane < width) {
      const uint32_t b0 = run_begin(c, r, len), b1 = run_begin(c, r + 1, len);
      if (b0 == b1) {
        ready = true;  // no tiles, no record: transparent
      } else {
        const uint64_t fi = c.row0 + (b1 - 1);
        const uint32_t ti = hi32(ld_dev64(c.incl + fi * kLanes * 2));  // both loads in flight together
        const uint32_t ta = hi32(ld_dev64(c.agg + fi * kLanes * 2));
        inc = ti == t_inc;
        ready = inc || ta == t_agg;
      }
    }
    const uint64_t ready_mask = __ballot(ready);
    const uint64_t inc_mask = __ballot(inc);
    const uint32_t lead = ready_mask == ~0ull ? 64u : (uint32_t)__builtin_ctzll(~ready_mask);
    const uint32_t first_inc = inc_mask ? (uint32_t)__builtin_ctzll(inc_mask) : 64u;
    const bool ends = first_inc < lead;
    const uint32_t take = ends ? first_inc + 1 : lead;
    if (take > 0) {
      uint64_t part = 0;
      bool ok = true;
      for (uint32_t i0 = 0; i0 < take; i0 += 4) {
#pragma unroll
        for (uint32_t d = 0; d < 4; ++d) {
          const uint32_t i = i0 + d;
          if (i < take) {
            const int64_t ri = top - (int64_t)i;
            const uint32_t b0 = run_begin(c, ri, len), b1 = run_begin(c, ri + 1, len);
            if (b0 != b1) {
              const bool use_inc = ends && i == first_inc;
              uint64_t v;
              ok &= read_rec(use_inc ? c.incl : c.agg, c.row0 + (b1 - 1), lane, use_inc ? t_inc : t_agg, &v);
              part ^= v;
            }
          }
        }
      }
      if (__ballot(!ok) == 0) {  // every lane's words were complete
        carry ^= part;
        if (ends) break;
        top -= (int64_t)take;
        spins = 0;
        width = kLanes;  // a long run of published records: probe wide
        continue;
      }
    }
    ++spin_total;
    if (++spins > kFallbackSpins) {
      // recompute the predecessor run backwards from its last tile
      if (c.lb_stats && lane == 0) atomicAdd(c.lb_stats, 1ull);
      bool started = false;
      const int64_t first = run_begin(c, top, len);
      for (int64_t j = (int64_t)run_begin(c, top + 1, len) - 1; j >= first && !started; --j)
        carry ^= tile_open_part<KQ, E, FIRST, DR>(c, (uint32_t)j, lane, mk, tab, &started);
      if (started) break;
      --top;
      spins = 0;
      continue;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  if (c.lb_stats && spin_total && lane == 0) atomicAdd(c.lb_stats + 1, (unsigned long long)spin_total);
  return carry;
}

// Inputs of one tile, loaded ahead of its compute: per edge its P slot, at
// level 2 its source vertex (ia) and at levels >= 3 its window sum (w) and
// whether that window is non-empty (ia).
template <int KQ, int E>
struct TileIn {
  uint32_t slot[E], ia[E];
  uint64_t w[E], w2[E];
  RowBlock<KQ, E> qr, zr;  // product rows; substitution rows of the sources (level 2, level 3 from D rows)
  RowBlock<KQ, E> dr;      // level 3 from window rows: the entries' D rows
  IdxN<E / 4> need;        // store flags, four edges per word
};

template <int KQ, int E, bool FIRST, bool DR = false>
__device__ __forceinline__ void load_tile(const TileCtx& c, uint32_t tile, uint32_t lane, TileIn<KQ, E>& in) {
  const uint32_t e0 = tile * (uint32_t)E;
  const uint32_t ne = min((uint32_t)E, c.m - e0);
  in.need = load_idx<E / 4>((const uint32_t*)(c.need + e0));
  load_qrows<KQ, E>(in.qr, c.q, e0, lane);
  if (FIRST || DR) load_zrows<KQ, E>(in.zr, c.z, c.e_src, e0, ne, lane);
  if (DR) load_qrows<KQ, E>(in.dr, c.d, e0, lane);
  tile_inputs<KQ, E, FIRST || DR>(c, e0, ne, lane, in.need, in.slot, in.ia, in.w, in.w2);
}

// One prefix level (2..k-1) over the run of tiles of wave w of W: the tiles
// are cut into W contiguous runs of ceil(n_tiles / W), and a wave scans its
// run in order, so the running XOR of the level values flows from tile to
// tile in registers and every read slot is stored as soon as its value is
// known. Only the segment part at the start of a run (before the run's first
// segment start) lacks the carry of the segment's part in the preceding runs:
// its slots are stored without it, and once the run is done the wave
// publishes its own record (the trailing segment part's XOR, inclusive if a
// segment starts in the run), collects the carry by one look-back and XORs it
// into those slots. A segment's leading slot (just before its first edge's
// slot) holds 0; writing it here lets P buffers be reused across graphs
// without clearing. Only slots that some window of the next level reads are
// stored; empty windows gather the zero row.
template <int KQ, int E, bool FIRST, bool DR = false>
__device__ __forceinline__ void scan_run(const TileCtx& c, uint32_t w, uint32_t W, uint32_t lane,
                                         const uint32_t (&mk)[6], uint64_t* tab) {
  const uint32_t R = (c.n_tiles + W - 1) / W;  // tiles per run when the runs are of equal length
  const uint32_t t0 = run_begin(c, w, R), t1 = run_begin(c, w + 1, R);
  if (t0 >= t1) return;
  const uint32_t m = c.m;
  const uint32_t e_begin = t0 * (uint32_t)E;
  // the run continues its predecessor's segment unless its first entry restarts
  const bool cont = e_begin > 0 && !((c.need[e_begin] >> 3) & 1u);
  bool started = !cont;        // a segment starts in the run (its own first edge included)
  uint32_t open_end = e_begin; // edges [e_begin, open_end) precede the run's first segment start
  uint64_t acc = 0;
  auto slot_ptr = [&](uint32_t slot) { return c.pc + (uint64_t)slot * kLanes + lane; };

  TileIn<KQ, E> cur;
  load_tile<KQ, E, FIRST, DR>(c, t0, lane, cur);
  for (uint32_t tile = t0;;) {
    const uint32_t e0 = tile * (uint32_t)E;
    const TileIn<KQ, E>& in = cur;
    // Wait once for all of this tile's rows and gathers. Without this the
    // compiler, which cannot count the loads issued under the per-edge
    // branches, put a full vmcnt(0) before every product, and that wait also
    // covered the slot stores issued by the edges before it: each stored slot
    // cost a store round trip before the next product. Levels 4..9 of the
    // 10^7-edge motif query: 4.48 -> 4.06 ms per launch.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt at their maxima (no wait)
    // an edge needs a product when it reaches a read slot and, at levels >= 3,
    // its window is non-empty (need bit 2 says both). The flags of the edges
    // past m are zero, so the tile's edges need no range test: a segment
    // start (bit 3) resets the running XOR, and no flag means no product and
    // no store. Keeping these tests off the scalar unit, which issues about
    // twice as many instructions as the vector units here, ran the level in
    // 0.221 ms against 0.243 ms on the 10^6-edge graph at k = 8.
    auto needs = [&](int i) {
      return ((in.need.v[i / 4] >> (8 * (i % 4) + 2)) & 1u) != 0;
    };
    auto flag = [&](int i) { return (in.need.v[i / 4] >> (8 * (i % 4))) & 3u; };
#pragma unroll
    for (int i = 0; i < E; ++i) {
      {  // edges past m carry zero flags and change nothing
        if ((in.need.v[i / 4] >> (8 * (i % 4) + 3)) & 1u) {  // a segment starts at this edge
          acc = 0;
          if (!started) {
            started = true;
            open_end = e0 + (uint32_t)i;
          }
          if (flag(i) & 2u) p_store(slot_ptr(in.slot[i] - 1u), 0);
        }
        if (needs(i)) {
          const uint64_t aL = subset_xor<KQ, E>(in.qr, i, c.cb, mk);
          uint64_t wv = in.w[i] ^ in.w2[i];
          if (FIRST || DR) wv = subset_xor<KQ, E>(in.zr, i, c.cb, mk);
          if (DR) wv = gf_mul(tab, wv, subset_xor<KQ, E>(in.dr, i, c.cb, mk));  // z^L_src * D^L
          acc ^= gf_mul(tab, aL, wv);
        }
        if (flag(i) & 1u) p_store(slot_ptr(in.slot[i]), acc);
      }
    }
    if (tile + 1 >= t1) break;
    load_tile<KQ, E, FIRST, DR>(c, tile + 1, lane, cur);
    ++tile;
  }
  if (!started) open_end = min(t1 * (uint32_t)E, m);

  const uint32_t e_end = min(t1 * (uint32_t)E, m);
  const bool next_cont = e_end < m && !((c.need[e_end] >> 3) & 1u);
  const uint64_t fi = c.row0 + (t1 - 1);
  if (next_cont)
    publish(started ? c.incl : c.agg, fi, lane, acc, rec_tag(c.epoch, started ? kFlagIncl : kFlagAgg));
  if (!cont) return;
  const uint64_t carry = look_back<KQ, E, FIRST, DR>(c, w, R, lane, mk, tab);
  if (next_cont && !started) publish(c.incl, fi, lane, carry ^ acc, rec_tag(c.epoch, kFlagIncl));
  if (!carry) return;
  // the run's leading segment part: its stored slots get the carry (same lane
  // and address as the stores above, so the XOR lands on the stored value)
  for (uint32_t e0 = e_begin; e0 < open_end; e0 += E) {
    const IdxN<E> so = load_idx<E>(c.e_out + e0);
    const IdxN<E / 4> nd = load_idx<E / 4>((const uint32_t*)(c.need + e0));
#pragma unroll
    for (int i = 0; i < E; ++i)
      if (e0 + (uint32_t)i < open_end && ((nd.v[i / 4] >> (8 * (i % 4))) & 1u))
        atomicXor((unsigned long long*)slot_ptr(so.v[i]), (unsigned long long)carry);
  }
}

// Runs per wave at level 2. Which edges need a level-2 product varies
// strongly along the edge list (hub destinations need most of theirs), so
// with one contiguous run per wave the slowest wave took 2.4x the mean time
// on the 10^6-edge Chung-Lu graph; a wave takes kRunsPerWave runs spread
// evenly over the list instead. At levels >= 3 the spread is smaller and
// interleaved runs measured slower than one run per wave.
constexpr uint32_t kRunsPerWave = 4;

// Level 2 (and any prefix level), the share of wave w of W. The tiles (E
// consecutive edges each) are cut into kRunsPerWave * W contiguous runs of
// equal length, and wave w scans runs w, w + W, w + 2W, ... in order. Along a
// run the running XOR of the level values flows from tile to tile in
// registers and every read slot is stored as soon as its value is known; a
// segment's leading slot (just before its first edge's slot) is stored as 0,
// which lets P buffers be reused across graphs without clearing. Only slots
// that some window of the next level reads are stored (empty windows gather
// the zero row).
//
// The part of a run before its first segment start lacks the carry of that
// segment's part in the preceding runs: its slots are stored without it. Each
// run publishes its record (the XOR of its trailing segment part, inclusive
// if a segment starts in the run) as soon as it is done, so the work phase
// never waits. Once all of its runs are done, the wave collects each run's
// carry by a look-back, publishes the inclusive record of a run without a
// segment start, and XORs the carry into the stored slots of the run's
// leading part.
template <int KQ, int E, bool FIRST>
__device__ __forceinline__ void scan_runs(const TileCtx& c, uint32_t w, uint32_t W, uint32_t lane,
                                          const uint32_t (&mk)[6], uint64_t* tab) {
  const uint32_t n_runs = kRunsPerWave * W;
  const uint32_t R = (c.n_tiles + n_runs - 1) / n_runs;  // tiles per run
  auto run_first = [&](uint32_t k) { return (w + k * W) * R; };
  auto has_run = [&](uint32_t k) { return k < kRunsPerWave && run_first(k) < c.n_tiles; };
  if (!has_run(0)) return;
  cu32* e_out = as_const(c.e_out);
  const uint32_t m = c.m;
  auto slot_ptr = [&](uint32_t slot) { return c.pc + (uint64_t)slot * kLanes + lane; };
  auto continues = [&](uint32_t e) { return e > 0 && e < m && e_out[e] == e_out[e - 1] + 1u; };
  const uint32_t t_agg = rec_tag(c.epoch, kFlagAgg), t_inc = rec_tag(c.epoch, kFlagIncl);

  uint32_t started_mask = 0;  // bit k: a segment starts in run k
  uint32_t k = 0;
  TileIn<KQ, E> cur;
  load_tile<KQ, E, FIRST>(c, run_first(0), lane, cur);
#pragma unroll 1
  for (;;) {
    const uint32_t t0 = run_first(k), t1 = min(t0 + R, c.n_tiles);
    const uint32_t e_begin = t0 * (uint32_t)E;
    const bool cont = continues(e_begin);
    bool started = !cont;  // a segment starts in the run (its own first edge included)
    uint64_t acc = 0;
    uint32_t last_slot = cont ? e_out[e_begin] - 1u : 0u;
#pragma unroll 1
    for (uint32_t tile = t0;;) {
      const uint32_t e0 = tile * (uint32_t)E;
      const uint32_t ne = min((uint32_t)E, m - e0);
      const TileIn<KQ, E>& in = cur;
      // an edge needs a product when it reaches a read slot (need bit 2) and,
      // at levels >= 3, its window is non-empty (an empty window contributes zero)
      auto needs = [&](int i) {
        return (uint32_t)i < ne && (FIRST ? ((in.need.v[i / 4] >> (8 * (i % 4) + 2)) & 1u) != 0 : in.ia[i] != 0);
      };
      auto flag = [&](int i) { return (in.need.v[i / 4] >> (8 * (i % 4))) & 3u; };
#pragma unroll
      for (int i = 0; i < E; ++i) {
        if ((uint32_t)i < ne) {
          if (in.slot[i] != last_slot + 1u || (tile == t0 && i == 0 && !cont)) {
            acc = 0;
            started = true;
            if (flag(i) & 2u) p_store(slot_ptr(in.slot[i] - 1u), 0);
          }
          if (needs(i)) {
            const uint64_t aL = subset_xor<KQ, E>(in.qr, i, c.cb, mk);
            const uint64_t wv = FIRST ? subset_xor<KQ, E>(in.zr, i, c.cb, mk) : in.w[i];
            acc ^= gf_mul(tab, aL, wv);
          }
          if (flag(i) & 1u) p_store(slot_ptr(in.slot[i]), acc);
          last_slot = in.slot[i];
        }
      }
      // the next tile: of this run, else the first of the wave's next run
      const bool more_here = tile + 1 < t1;
      const bool more = more_here || has_run(k + 1);
      if (more) load_tile<KQ, E, FIRST>(c, more_here ? tile + 1 : run_first(k + 1), lane, cur);
      if (!more_here) break;
      ++tile;
    }
    const uint32_t e_end = min(t1 * (uint32_t)E, m);
    if (e_end < m && e_out[e_end] == last_slot + 1u)
      publish(started ? c.incl : c.agg, c.row0 + (t1 - 1), lane, acc, started ? t_inc : t_agg);
    if (started) started_mask |= 1u << k;
    if (!has_run(k + 1)) break;
    ++k;
  }

  // carries of the runs that begin inside a segment
#pragma unroll 1
  for (uint32_t r = 0; r <= k; ++r) {
    const uint32_t t0 = run_first(r), t1 = min(t0 + R, c.n_tiles);
    const uint32_t e_begin = t0 * (uint32_t)E, e_end = min(t1 * (uint32_t)E, m);
    if (!continues(e_begin)) continue;
    const uint64_t carry = look_back<KQ, E, FIRST>(c, w + r * W, R, lane, mk, tab);
    if (!((started_mask >> r) & 1u) && continues(e_end)) {
      // no segment starts in the run: its inclusive prefix is the carry and
      // its own aggregate, published above
      uint64_t own = 0;
      (void)read_rec(c.agg, c.row0 + (t1 - 1), lane, t_agg, &own);
      publish(c.incl, c.row0 + (t1 - 1), lane, carry ^ own, t_inc);
    }
    // the run's leading segment part: its stored slots get the carry (same
    // lane and address as the stores above, so the XOR lands on the stored value)
    uint32_t prev = e_out[e_begin] - 1u;
    bool open = true;
#pragma unroll 1
    for (uint32_t e0 = e_begin; open && e0 < e_end; e0 += E) {
      const IdxN<E> so = load_idx<E>(c.e_out + e0);
      const IdxN<E / 4> nd = load_idx<E / 4>((const uint32_t*)(c.need + e0));
#pragma unroll
      for (int i = 0; i < E; ++i) {
        if (open && e0 + (uint32_t)i < e_end) {
          if (so.v[i] != prev + 1u) {
            open = false;
          } else {
            if (((nd.v[i / 4] >> (8 * (i % 4))) & 1u) && carry)
              atomicXor((unsigned long long*)slot_ptr(so.v[i]), (unsigned long long)carry);
            prev = so.v[i];
          }
        }
      }
    }
  }
}

// The schedule of a prefix level: interleaved runs at level 2 without run
// bounds, one contiguous run per wave otherwise.
template <int KQ, int E, bool FIRST, bool DR = false>
__device__ __forceinline__ void scan_level(const TileCtx& c, uint32_t w, uint32_t W, uint32_t lane,
                                           const uint32_t (&mk)[6], uint64_t* tab) {
  if constexpr (FIRST) {
    if (!c.bounds) {
      scan_runs<KQ, E, FIRST>(c, w, W, lane, mk, tab);
      return;
    }
  }
  scan_run<KQ, E, FIRST, DR>(c, w, W, lane, mk, tab);
}

// Last level k over edges [e0, e1): unreduced per-lane sum of c_k(e) into r.
// Edges go in batches of 4: one scalar load per index array and batch. Two
// batches alternate, so the next batch's gathers and rows are in flight
// during this batch's products; the two rows of a window stay apart until
// the product, so no load waits for its partner. Empty windows gather the
// zero row and skip their product. (On the 10^6-edge graph at k = 8 this
// ran the last level in 0.519 ms against 0.550 ms for one batch at a time,
// with 64 edges per wave's range.) Above level 2 the product row of an entry
// is read at its product by scalar loads instead of lane-spread vector loads
// and 24 v_readlane: 6.55 -> 6.38 ms per launch on the 10^7-edge motif query.
//
// With H = 2 the wave sums the chunk pair cb, cb + 64 (cb a multiple of 128;
// chunk 1's prefix rows `pstride` elements after chunk 0's): an entry's
// indices, product row and subset XOR serve both chunks, the second chunk's
// subset XOR being the first one's XOR row entry 6 (the two iterations of a
// lane differ only in bit 6). Last level of the 10^7-edge motif query: 12.15
// -> 10.7 ms per query; of the 10^6-edge path query 0.41 -> 0.38 ms.
template <int KQ, bool FIRST, int H = 1>
__device__ __forceinline__ void top_range(const uint32_t* e_src_p, const uint32_t* hi_p,
                                          const uint32_t* lo_p, const uint64_t* q_p,
                                          const uint64_t* z_p, const uint64_t* pp, uint64_t pstride, uint64_t cb,
                                          uint32_t e0, uint32_t e1, uint32_t lane,
                                          const uint32_t (&mk)[6], uint64_t* tab, Acc128 (&r)[H]) {
  static_assert(H == 1 || (H == 2 && KQ > 6 && !FIRST), "two chunks per wave need rows of at least 7 entries");
  if (e0 >= e1) return;
  const uint32_t base = lds_addr(tab);
  constexpr int B = 4;
  constexpr int P = RowBlock<KQ, B>::P;
  const uint64_t* zero = kZeroRow + lane;
  struct Batch {
    uint64_t wh[B][H], wl[B][H];
    IdxN<B> live;
    RowBlock<KQ, B> qr, zr;
    uint32_t eb;
  };
  // Every load is issued whatever the batch holds (edges at or past e1 read
  // the zero row, and at level 2 their product rows are clamped to edge
  // e1 - 1), so the number of loads in flight is fixed and a batch's products
  // wait only for that batch's loads while the next batch's are in flight.
  auto gather = [&](uint32_t eb, Batch& b) {
    b.eb = eb;
    if (FIRST) {  // level 2 (k = 2): product rows spread over the wave
      const uint32_t g = min(lane * P, (uint32_t)(B * KQ - P));
      const uint32_t ei = min(eb + g / KQ, e1 - 1);
#pragma unroll
      for (int p = 0; p < P; ++p) b.qr.v[p] = *(gu64*)(q_p + (uint64_t)ei * KQ + g % KQ + p);
    }
    if (FIRST) {
      load_zrows<KQ, B>(b.zr, z_p, e_src_p, eb, e1 - min(eb, e1), lane);
#pragma unroll
      for (int i = 0; i < B; ++i) b.live.v[i] = eb + (uint32_t)i < e1;
    } else {
      const IdxN<B> h = load_idx<B>(hi_p + eb);
      const IdxN<B> l = load_idx<B>(lo_p + eb);
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const bool live = eb + (uint32_t)i < e1 && h.v[i] != l.v[i];
#pragma unroll
        for (int c = 0; c < H; ++c) {
          b.wh[i][c] = p_load(live ? pp + (uint64_t)c * pstride + (uint64_t)h.v[i] * kLanes + lane : zero);
          b.wl[i][c] = p_load(live ? pp + (uint64_t)c * pstride + (uint64_t)l.v[i] * kLanes + lane : zero);
        }
        b.live.v[i] = live;
      }
    }
  };
  auto compute = [&](const Batch& b) {
#pragma unroll
    for (int i = 0; i < B; ++i) {
      if (b.live.v[i]) {
        cu64* row = as_const(q_p) + (uint64_t)(b.eb + i) * KQ;
        const uint64_t aL = FIRST ? subset_xor<KQ, B>(b.qr, i, cb, mk) : subset_xor<KQ>(row, cb, mk);
#pragma unroll
        for (int c = 0; c < H; ++c) {
          const uint64_t wv = FIRST ? subset_xor<KQ, B>(b.zr, i, cb, mk) : b.wh[i][c] ^ b.wl[i][c];
          gf_table(tab, wv);
          if constexpr (H == 2) {
            gf_comb_acc(base, c ? aL ^ row[6] : aL, r[c]);
          } else {
            gf_comb_acc(base, aL, r[c]);
          }
        }
      }
    }
  };
  // The empty asm statements are compiler barriers for memory operations
  // (no instruction): without them the compiler sank the loads of the batch
  // gathered ahead into the products that use them, so that batch's gathers
  // waited one by one. Batches of 4 keep both in flight at 79 VGPRs (batches
  // of 8 needed 112, four waves per SIMD, and ran slower): the last level of
  // the 10^7-edge motif query 6.54 -> 6.45 ms per launch, of the 10^6-edge
  // path query 0.429 -> 0.416 ms.
  Batch x, y;
  gather(e0, x);
  for (uint32_t eb = e0;; eb += 2 * B) {
    gather(eb + B, y);
    asm volatile("" ::: "memory");
    compute(x);
    if (eb + B >= e1) break;
    gather(eb + 2 * B, x);
    asm volatile("" ::: "memory");
    compute(y);
    if (eb + 2 * B >= e1) break;
  }
}

// Store and product flags of a query (they depend on the graph, delta and k).
// Per prefix level l, for the readers of level l (the windows of level
// l+1's product edges; every non-empty window when l+1 = k), need[e] says
//   bit 0: e's own slot is read;
//   bit 1: the leading slot of the segment e starts is read;
//   bit 2: e lies inside some reader's window, so its product at level l
//          enters a window sum (see mark_cover), and at levels l >= 3 its
//          own window is non-empty (an empty window contributes zero);
//   bit 3: a segment starts at e (e is the first in-edge of its destination).
// A prefix level forms the product of an edge only with bit 2 and stores only
// slots with bit 0 / bit 1. The kEdgePad bytes past m are zero.


// Work-balanced runs: bounds[w] = the first tile whose exclusive cost prefix
// reaches ceil(total * w / W), with pre[] the inclusive cost prefix within
// blocks of kCostBlock tiles and boff[] the blocks' offsets. Tile t writes
// the runs whose first tile it is; the last tile also writes bounds[w] =
// n_tiles for the runs past it (empty) and for w = W.
__device__ __forceinline__ void run_bounds_of_tile(const uint32_t* pre, const uint32_t* boff, uint32_t n_tiles,
                                                   uint32_t t, uint32_t W, uint32_t* bounds, float skew = 0.0f) {
  auto incl = [&](uint32_t i) { return (uint64_t)pre[i] + boff[i / kCostBlock]; };
  const uint64_t total = incl(n_tiles - 1);
  const uint64_t excl_t = t ? incl(t - 1) : 0;      // cost before tile t
  const uint64_t excl_p = t > 1 ? incl(t - 2) : 0;  // cost before tile t - 1
  // the run in which cost x < total falls (below W). With a skew b, run
  // u = r / W gets the share (1 - b u) / (1 - b / 2), whose cumulative
  // F(u) = (u - b u^2 / 2) / (1 - b / 2) inverts to
  // u = (1 - sqrt(1 - b (2 - b) x / total)) / b. Costs are integers below
  // 2^32, so consecutive ones move u by more than 2^-33, far above the
  // rounding error of these double operations: the runs stay monotone in x.
  auto run_of = [&](uint64_t x) -> uint64_t {
    if (skew <= 0.0f) return x * W / total;
    const double b = skew, f = (double)x / (double)total;
    const double u = (1.0 - __builtin_sqrt(1.0 - b * (2.0 - b) * f)) / b;
    const uint64_t r = (uint64_t)(u * (double)W);
    return r < W ? r : W - 1;
  };
  const uint64_t w_hi = run_of(excl_t);
  const uint64_t w_lo = t ? run_of(excl_p) + 1 : 0;
  for (uint64_t w = w_lo; w <= w_hi && w < W; ++w) bounds[w] = t;
  if (t == n_tiles - 1)
    for (uint64_t w = w_hi + 1; w <= W; ++w) bounds[w] = n_tiles;
}

// In-place inclusive prefix (modulo 2^32) of v[count] within blocks of
// kCostBlock entries (block b of a 256-thread grid); block totals to bsum[b].
__device__ __forceinline__ void block_prefix(uint32_t* v, uint64_t count, uint32_t* bsum) {
  __shared__ uint32_t part[256];
  const uint64_t base = (uint64_t)blockIdx.x * kCostBlock + threadIdx.x * 4;
  uint32_t x[4];
  uint32_t sum = 0;
  for (int j = 0; j < 4; ++j) {
    sum += base + j < count ? v[base + j] : 0u;
    x[j] = sum;
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < 256; d <<= 1) {
    const uint32_t u = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += u;
    __syncthreads();
  }
  const uint32_t before = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int j = 0; j < 4; ++j)
    if (base + j < count) v[base + j] = before + x[j];
  if (threadIdx.x == 255) bsum[blockIdx.x] = part[255];
}

// Exclusive prefix (modulo 2^32) of bs[nb] into bo, by one 1024-thread block.
__device__ __forceinline__ void block_offsets(const uint32_t* bs, uint32_t nb, uint32_t* bo) {
  __shared__ uint32_t part[1024];
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < nb ? bs[b] : 0u;
    part[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t d = 1; d < 1024; d <<= 1) {
      const uint32_t u = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
      __syncthreads();
      part[threadIdx.x] += u;
      __syncthreads();
    }
    if (b < nb) bo[b] = carry + part[threadIdx.x] - v;
    carry += part[1023];
    __syncthreads();
  }
}

// Product flags by window cover. A window reads P[hi] ^ P[lo],
// the XOR of the level values of the edges with slots in (lo, hi]; a value
// before lo enters both prefixes and cancels. So an edge's product is needed
// only when its slot lies in the window of some reader, and leaving out every
// other product leaves every window sum unchanged. Each reader adds +1 at
// slot lo + 1 and -1 at slot hi + 1 of a difference array (windows never
// leave their segment); its prefix sum at e's slot counts the readers whose
// window covers e. The two slots a reader reads are marked in ref (one byte
// per slot, zeroed beforehand).
__device__ __forceinline__ void mark_cover(const uint32_t* hi, const uint32_t* lo, const uint8_t* next, uint64_t e,
                                           uint8_t* ref, uint32_t* diff) {
  const uint32_t h = hi[e], l = lo[e];
  if (h != l && (!next || (next[e] & 4u))) {
    ref[h] = 1;
    ref[l] = 1;
    atomicAdd(&diff[l + 1], 1u);
    atomicAdd(&diff[h + 1], ~0u);  // -1 modulo 2^32
  }
}
// need[e]: bits 0, 1 and 3 as above; bit 2 when e's slot is covered, with
// cover(s) = pre[s] + boff[s / kCostBlock] (modulo 2^32) the prefix sum of
// the difference array, and (hi != null, levels >= 3) hi[e] != lo[e].
__device__ __forceinline__ void mark_need_cover(const uint32_t* e_out, const uint8_t* ref, const uint32_t* pre,
                                                const uint32_t* boff, const uint32_t* hi, const uint32_t* lo,
                                                uint64_t e, uint8_t* need) {
  const uint32_t slot = e_out[e];
  uint32_t f = ref[slot];
  if (e == 0 || e_out[e - 1] + 1u != slot) f |= 8u | ((uint32_t)ref[slot - 1] << 1);
  if (pre[slot] + boff[slot / kCostBlock] != 0u && (!hi || hi[e] != lo[e])) f |= 4u;
  need[e] = (uint8_t)f;
}

}  // namespace rs
