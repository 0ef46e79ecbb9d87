// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rs.h"  // include/ is on the include path

namespace rs {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_last_error(const std::string& s);

#define RS_HIP(expr)                                                       \
  do {                                                                     \
    hipError_t _e = (expr);                                                \
    if (_e != hipSuccess) {                                                \
      ::rs::set_last_error(std::string(#expr) + ": " + hipGetErrorString(_e)); \
      return RS_EDEVICE;                                                   \
    }                                                                      \
  } while (0)

#define RS_TRY(expr)              \
  do {                            \
    rs_status _s = (expr);        \
    if (_s != RS_OK) return _s;   \
  } while (0)

// ---------------------------------------------------------------------------
// Device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  // Grows to at least `need` bytes; new memory is zero-filled on `st`.
  rs_status reserve(size_t need, hipStream_t st, bool zero = true);
  void release();
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// ---------------------------------------------------------------------------
// Kernel launch shapes and per-query plan
// ---------------------------------------------------------------------------
// The per-edge index arrays (e_src, e_dst, e_t, e_out, hi, lo) hold this many
// readable entries past m, and the product table this many rows past its last
// level, so a level kernel can fetch a whole tile's indices and rows in one
// load; entries past m are never used.
constexpr uint32_t kEdgePad = 64;

constexpr uint32_t kFlagAgg = 1;   // record: XOR of the tile's open segment part
constexpr uint32_t kFlagIncl = 2;  // record: full prefix of that segment

// Largest graph (edges) on which 8-edge tiles are accepted: that shape ran
// for over 140 s on a 10^7-edge query under an earlier look-back schedule and
// has not been validated at that size since, so larger graphs reject it.
constexpr uint64_t kMaxEdgesE8 = 4000000;

struct Tuning {
  uint32_t edges_per_tile = 16;      // scan levels: 8 or 16
  uint32_t top_edges_per_tile = 64;  // last level: edges per wave's range
  uint32_t chunks_per_launch = 4;
  // Waves per block of the prefix levels and of the last level (one knob for
  // both when set). The gathering level kernel holds four waves per SIMD;
  // in blocks of four, one per SIMD, it ran levels 4..9 of the 10^7-edge
  // motif query in 4.49 ms per launch against 4.68 in blocks of two, while
  // the last level ran best in blocks of two (10^6-edge path query: 0.44
  // against 0.47 ms).
  uint32_t waves_per_block = 4;
  uint32_t top_waves_per_block = 2;
  uint32_t max_slots = 0;  // batched path; 0 = as many as fit
  // Plain path: chunks per wave of the last level (1 or 2; see query_tuning
  // for when 2 applies).
  uint32_t chunks_per_wave = 2;
};

struct QueryPlan {
  uint32_t k = 0, kq = 0, delta = 0;
  bool motif = false;
  uint64_t seed = 0;
  uint64_t it_begin = 0, it_end = 0;
  uint64_t chunk_first = 0, chunk_last = 0;  // 64-iteration chunks [first, last)
  uint8_t mu[RS_MAX_COLOURS] = {0};          // motif multiplicities
  uint8_t shade_off[RS_MAX_COLOURS] = {0};
};

// Arguments of the prefix levels (2..k-1).
struct ScanArgs {
  const uint32_t* e_src;
  const uint32_t* e_out;  // P slot written by edge e: e + dst(e) + 1
  const uint32_t* hi;     // P slot of the window end
  const uint32_t* lo;     // P slot of the window start
  const uint64_t* q;      // [m][kq] products z_{dst,j} * y_{e,l-1} for this level
  const uint64_t* z;      // [n][kq] (level 2, and level 3 from window rows)
  const uint64_t* d = nullptr;  // level 3 from window rows: [entries][kq] D rows (else null)
  const uint64_t* p_prev; // [(m+n)*64] per chunk
  uint64_t* p_cur;
  uint64_t p_stride;      // elements between consecutive chunks' P arrays
  uint64_t chunk_base;    // first iteration index of chunk 0 of this launch
  uint32_t m;
  uint32_t n_tiles;
  uint32_t k;
  uint32_t epoch;
  uint64_t* agg;           // [chunks][n_tiles][64][2] tagged records
  uint64_t* incl;          // [chunks][n_tiles][64][2]
  const uint8_t* need;     // [m] store flags
  unsigned long long* lb_stats = nullptr;  // null, or [2] look-back counters (see TileCtx)
  const uint32_t* bounds = nullptr;        // null, or [waves+1] work-balanced first tile of each run
  uint32_t waves = 0;                      // waves per chunk the bounds were cut for
  const uint32_t* count = nullptr;         // null, or the device-side length of a compacted edge list
                                           // (then m and n_tiles only bound it: record stride, grids)
};
// Blocks of a kernel with this block size and dynamic LDS that fit on the
// whole GPU at once (cached).
uint32_t resident_blocks(const void* kern, uint32_t threads, size_t lds);
// Waves per chunk of a prefix-level launch of this shape (grid width times
// waves per block).
uint32_t scan_waves(uint32_t kq, uint32_t E, bool first, uint32_t n_tiles, uint32_t chunks, uint32_t wpb,
                    bool drows = false);
// Arguments of the last level k.
struct TopArgs {
  const uint32_t* e_src;
  const uint32_t* hi;
  const uint32_t* lo;
  const uint64_t* q;
  const uint64_t* z;
  const uint64_t* p_prev;
  uint64_t p_stride;
  uint64_t chunk_base;
  uint64_t it_begin, it_end;
  uint32_t m;
  uint32_t edges_per_wave;
  uint32_t k;
  uint64_t* partial;  // [chunks][blocks][64] per-block sums
  uint32_t* ticket = nullptr;  // null (static ranges), or [chunks] zeroed next-range counters
  uint64_t* fsum;     // [2^k] per-iteration sums
  const uint32_t* count = nullptr;  // null, or the device-side length of the compacted last-level list
  const uint32_t* ce = nullptr;     // compacted list: original edge of each entry (fine-grained outputs)
};
// Rows of `partial` one launch_top call writes per chunk.
uint32_t top_blocks(const TopArgs& a, bool first_level, uint32_t kq, uint32_t chunks, const Tuning& tu);

// Launchers (rs_kernels.hip). All enqueue on `st` and return hipGetLastError.
hipError_t launch_ztable(uint64_t* z, uint32_t n, const QueryPlan& qp, const uint8_t* colour_d,
                         hipStream_t st);
// delta_v: per-vertex resting times [n] on the device, or null (then delta).
hipError_t launch_window(const uint32_t* e_src, const uint32_t* e_t, const uint32_t* in_off,
                         uint32_t* lo, uint32_t m, uint32_t delta, const uint32_t* delta_v, hipStream_t st);

// Entries per block of the block-wise prefix sums (tile costs, window cover,
// list compaction): 256 threads x 4.
constexpr uint32_t kCostBlock = 1024;

// Weights of the work-balanced runs, fitted to per-wave clocks: at levels
// >= 3 per tile, per product and per stored slot (per-wave clocks of the
// 10^6-edge path query and the 10^7-edge motif query, least squares per
// chunk: residual 3.8-5.8 % of a wave's time against 8-8.7 % for tile and
// product weights alone); at level 2 per tile and per product. A tile costs
// at most 2 + 16 * (7 + 1) = 130, so the level totals of any graph whose
// prefix state fits in device memory stay below 2^32.
constexpr uint32_t kTileCost = 2, kProductCost = 7, kStoreCost = 1;
constexpr uint32_t kTileCostFirst = 7, kProductCostFirst = 4;

// Waves of one launch run slower the later they were dispatched (on the
// 10^7-edge motif query the chunk whose blocks come last took 17 % longer
// than the first, and reversing the chunk order reversed the effect). The
// level kernel therefore orders its runs by dispatch order (run index = age,
// see k_scan) and the work-balanced split gives run r of W the share
// 1 - kAgeSkew * r / W, normalised: the youngest wave gets kAgeSkew less.
// (Measured there: 92.2 ms per query unskewed, 90.8 at 0.15, 90.7 at 0.2.)
constexpr float kAgeSkew = 0.2f;

// The skew of the split for a level launch of `waves` runs in blocks of wpb
// waves: k_scan orders its runs by age when its grid width is a multiple of 8.
inline float run_skew(uint32_t waves, uint32_t wpb) {
  return wpb && waves % wpb == 0 && (waves / wpb) % 8 == 0 ? kAgeSkew : 0.0f;
}

// One level's compacted edge list (rs_compact.hip): the kept edges of the
// level in edge order, with what a tile reads laid out contiguously.
struct LevelList {
  uint32_t* ce;     // original edge
  uint32_t* cslot;  // P slot of the edge (prefix levels)
  uint32_t* chi;    // window end slot (levels >= 3), or the source vertex (level 2)
  uint32_t* clo;    // window start slot (levels >= 3)
  uint8_t* cflag;   // bits 0..2 of the level's flags; bit 3: the running XOR restarts here
  uint64_t* cq;     // [entries][kq] product rows of the entries that form a product
};
// The compacted lists of levels 2..k of one query (level index y = l - 2;
// y = k - 2 is the last level), and what builds them.
struct CompactArgs {
  const uint32_t* e_src;
  const uint32_t* e_dst;
  const uint32_t* e_t;
  const uint32_t* e_out;
  const uint32_t* hi;
  const uint32_t* lo;
  const uint8_t* need;   // flags of prefix level l at need + (l - 2) * need_stride
  uint64_t need_stride;
  uint32_t m, k, kq;
  uint32_t nb;           // blocks of kCostBlock edges
  uint32_t* bsum;        // [k-1][nb] scratch: kept edges per block
  uint32_t* boff;        // [k-1][nb] scratch: their exclusive prefix
  uint32_t* count;       // [k-1] list lengths
  uint32_t* u32;         // four u32 arrays per level: ce, cslot, chi, clo, each list_stride entries
  uint8_t* u8;           // cflag per level, list_stride entries
  uint64_t* rows;        // product rows per level, list_stride * kq entries
  uint64_t list_stride;  // entries per list array (m + kEdgePad, rounded up)
  __host__ __device__ LevelList list(uint32_t y) const {
    uint32_t* b = u32 + (uint64_t)y * 4 * list_stride;
    return LevelList{b, b + list_stride, b + 2 * list_stride, b + 3 * list_stride, u8 + (uint64_t)y * list_stride,
                     rows + (uint64_t)y * list_stride * kq};
  }
};
inline uint64_t list_stride(uint64_t m) { return (m + kEdgePad + 63) & ~63ull; }
// Device bytes of the lists and their scratch for a query with k >= 3 levels.
inline uint64_t compact_bytes(uint64_t m, uint32_t k, uint32_t kq) {
  const uint64_t L = k - 1, st = list_stride(m), nb = (m + 1023) / 1024;
  return L * (st * (16 + 1 + 8ull * kq)) + 4 * L * (2 * nb + 1) + 1024;
}
// Builds the lists (counts, offsets, scatter).
hipError_t launch_compact(const CompactArgs& a, hipStream_t st);
// Restart bits and per-tile costs of the prefix lists (tiles of E entries;
// tiles_max bounds the tile count of every list): the inclusive cost prefix
// within blocks, pre [k-2][tiles_max], its block totals and offsets, bsum and
// boff [k-2][ceil(tiles_max / kCostBlock)].
hipError_t launch_compact_costs(const CompactArgs& a, uint32_t E, uint32_t tiles_max, uint32_t* pre, uint32_t* bsum,
                                uint32_t* boff, hipStream_t st);
// The same, then the work-balanced run bounds [k-2][b_stride] for w_first
// waves per chunk at level 2, w_second at level 3 and w_rest above it, each
// split with its skew (see run_skew).
hipError_t launch_compact_bounds(const CompactArgs& a, uint32_t E, uint32_t tiles_max, uint32_t w_first,
                                 uint32_t w_second, uint32_t w_rest, float skew_first, float skew_second,
                                 float skew_rest, uint32_t* pre, uint32_t* bsum, uint32_t* boff, uint32_t* bounds,
                                 uint32_t b_stride, hipStream_t st);
// Edges a query's constraints exclude (Sec. 3 and Sec. 4.7): at level 2 an
// edge whose source is not a source vertex, at the last level one whose
// destination is not a target vertex, at every level one that touches a
// removed vertex or is later than t_max (0 = no limit). Their product rows
// are 0, so they contribute nothing. Null masks exclude nothing.
struct EdgeFilter {
  const uint8_t* smask = nullptr;  // [n] source vertices
  const uint8_t* tmask = nullptr;  // [n] target vertices
  const uint8_t* rmask = nullptr;  // [n] removed vertices
  uint32_t t_max = 0;
  bool any() const { return smask || tmask || rmask || t_max; }
};
__device__ __forceinline__ bool edge_excluded(const EdgeFilter& f, uint32_t l, uint32_t k, uint32_t src, uint32_t dst,
                                              uint32_t t) {
  return (l == 2 && f.smask && !f.smask[src]) || (l == k && f.tmask && !f.tmask[dst]) ||
         (f.rmask && (f.rmask[src] | f.rmask[dst])) || (f.t_max && t > f.t_max);
}
// Level 2 folded into level 3 (k >= 4; rs_rrows.hip): the iteration-
// independent prefix rows of level 2 and, for level 3's product entries, their
// window rows D written over list(0)'s row array, with each level-3 entry's
// source written over list(1)'s window-end array. buf holds rrows_bytes(m, kq).
// The seed is *seed_p when seed_p is not null (read on the device).
uint64_t rrows_bytes(uint64_t m, uint32_t kq);
// The last level by distinct windows (rs_group.hip): the last level's list
// sorted by (hi, lo), its q rows summed per group of equal windows.
struct GroupView {
  uint64_t *key_in, *key_out;
  uint32_t *idx_in, *idx_out, *head, *gid, *gstart;
  uint32_t *ghi, *glo;   // [groups] window slots
  uint64_t* gq;          // [groups][kq] summed q rows
  uint32_t* gcount;      // number of groups (device)
  uint8_t* temp;         // sort and scan scratch
};
uint64_t group_temp_bytes(uint64_t m, uint64_t n);
uint64_t group_bytes(uint64_t m, uint64_t n, uint32_t kq);
GroupView group_view(uint8_t* buf, uint64_t m, uint32_t kq);
// n_entries: the list's length (also at *count on the device); slots = m + n.
hipError_t launch_group(const LevelList& Lk, const uint32_t* count, uint32_t n_entries, uint64_t slots, uint32_t kq,
                        const GroupView& v, uint64_t temp_bytes, hipStream_t st);
hipError_t launch_rrows(const CompactArgs& ca, const uint32_t* in_off, const uint64_t* z, uint64_t seed,
                        const uint64_t* seed_p, const EdgeFilter& f, uint32_t kq, uint8_t* buf, hipStream_t st);
// Product rows of the lists from level index y_first on (seed dependent: seed,
// or *seed_p read on the device when seed_p is not null), 0 for the edges f
// excludes.
hipError_t launch_compact_rows(const CompactArgs& a, const uint64_t* z, uint64_t seed, const uint64_t* seed_p,
                               const EdgeFilter& f, uint32_t kq, hipStream_t st, uint32_t y_first = 0);
// Fine-grained last level and slot sums (rs_fine.hip).
hipError_t launch_top_fine(const TopArgs& a, bool first_level, uint32_t kq, uint32_t chunks, const Tuning& tu,
                           uint64_t* T, hipStream_t st);
hipError_t launch_fine_slots(const uint32_t* e_dst, const uint32_t* e_t, const uint64_t* T, uint32_t m, uint64_t* zeta,
                             uint32_t* reach, hipStream_t st);
// Clears the rows [m][kq] of the one level of a k = 2 query (level 2 is
// also the last) of the edges f excludes.
hipError_t launch_mask_rows(uint64_t* rows, const uint32_t* e_src, const uint32_t* e_dst, const uint32_t* e_t,
                            const EdgeFilter& f, uint32_t m, uint32_t kq, hipStream_t st);
// Edge counts of a query's windows and flags (graph and delta only), used to
// state the algorithmic bytes of the level launches.
struct NeedCounts {
  uint64_t live = 0;         // non-empty windows
  uint64_t live_needed = 0;  // non-empty windows whose product reaches a read slot
  uint64_t needed = 0;       // edges whose product reaches a read slot
  uint64_t ref_slots = 0;    // edge slots that some window reads
  uint64_t ref_lead = 0;     // leading slots that some window reads
  uint64_t kept = 0;         // edges in the level's compacted list
};
// counts[6] on the device, zeroed beforehand: live, live_needed, needed,
// ref_slots, ref_lead, kept.
hipError_t launch_need_counts(const uint32_t* hi, const uint32_t* lo, const uint8_t* need, uint32_t m,
                              unsigned long long* counts, hipStream_t st);
// Store and product flags of prefix levels k-1 down to 2 (see mark_cover):
// the readers of level l are the windows of the edges whose level-(l+1)
// product is needed (level k-1: every non-empty window of the last level).
// Level l's flags go to need + (l - 2) * need_stride_b. Scratch: ref, two
// arrays of flag_ref_bytes(m, n); cov, two difference arrays [m+n+1] and the
// block sums and offsets [ceil((m+n+1) / 1024)] each.
inline uint64_t flag_ref_bytes(uint64_t m, uint64_t n) { return (m + n + 3) & ~3ull; }
hipError_t launch_flags(const uint32_t* e_out, const uint32_t* hi, const uint32_t* lo, uint32_t m, uint32_t n,
                        uint32_t k, uint8_t* need, uint64_t need_stride_b, uint8_t* ref, uint32_t* cov,
                        hipStream_t st);
// Flag arrays of a query: one per prefix level 2..k-1 (at least one), each
// m + kEdgePad bytes, level l at offset (l - 2) * need_stride(m); the stride
// keeps every level's array 256-byte aligned (the kernels read the flags four
// edges per 32-bit word).
inline uint32_t need_levels(uint32_t k) { return k > 3 ? k - 2 : 1; }
__host__ __device__ inline uint64_t need_stride(uint64_t m) { return (m + kEdgePad + 255) & ~255ull; }
hipError_t launch_qtable(const uint32_t* e_src, const uint32_t* e_dst, const uint32_t* e_t,
                         const uint64_t* z, uint64_t* q, uint32_t m, const QueryPlan& qp,
                         hipStream_t st);
hipError_t launch_scan(const ScanArgs& a, bool first_level, uint32_t kq, uint32_t chunks,
                       const Tuning& tu, hipStream_t st);
hipError_t launch_top(const TopArgs& a, bool first_level, uint32_t kq, uint32_t chunks,
                      const Tuning& tu, hipStream_t st);
hipError_t launch_fill32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t st);
hipError_t launch_fill64(uint64_t* p, uint64_t value, uint64_t count, hipStream_t st);
hipError_t launch_xor_reduce(const uint64_t* f, uint64_t begin, uint64_t end, uint64_t* out,
                             hipStream_t st);

// Bytes of a query's per-query tables on a graph with n vertices, m edges:
// window starts lo[m], substitution rows z[n][kq], product rows
// q[k-1][m][kq] and per-edge flags need[levels][m] (each padded past m as the level
// kernels expect).
uint64_t table_lo_bytes(uint64_t m);
uint64_t table_z_bytes(uint64_t n, uint32_t kq);
uint64_t table_q_bytes(uint64_t m, uint32_t k, uint32_t kq);
uint64_t table_need_bytes(uint64_t m, uint32_t k);
struct PlainWorkspace;
// Constraints and fine-grained outputs of one plain-path query; every array
// is host memory. Null / false: none.
struct QueryExtras {
  const uint32_t* delta_v = nullptr;  // [n] resting time per vertex (Sec. 2), replaces the scalar delta
  const uint8_t* smask = nullptr;     // [n] source vertices: walks start only there (Sec. 3)
  const uint8_t* tmask = nullptr;     // [n] target vertices: walks end only there (Sec. 3)
  const uint8_t* rmask = nullptr;     // [n] removed vertices: no walk passes through them (Sec. 4.7)
  uint32_t t_max = 0;                 // edges later than this are left out (Sec. 4.7); 0 = none
  bool fine = false;                  // keep zeta per slot (Alg. 1, Sec. 4.5)
  uint32_t* reach = nullptr;          // [n] fine: least reach time, 0xFFFFFFFF if none
  uint64_t* zeta = nullptr;           // [m] fine, may be null: zeta of each canonical edge's slot
  uint64_t reached = 0;               // fine, out: vertices with a reach time
};
// Plain path (rs_engine.hip): one query through workspace ws on stream st.
rs_status run_plain(rs_graph* g, PlainWorkspace& ws, const QueryPlan& qp, const Tuning& tu, uint64_t* per_it_host,
                    rs_result* r, hipStream_t st, QueryExtras* ex = nullptr);
rs_status plan_query(const rs_graph* g, const rs_query* q, QueryPlan& qp);
Tuning resolve_tuning(const rs_graph* g, uint32_t k, const rs_tuning* t);
// Batched path (rs_batch.hip). A batch workspace holds the device buffers and
// the captured graph of batched calls; calls through one workspace run one at
// a time. ws = nullptr uses the process-wide workspace of rs_run_batch.
struct BatchWorkspace;
BatchWorkspace* batch_ws_create();
// Per-query device bytes of a query in a batch (its tables and lists).
uint64_t batch_query_bytes(uint64_t m, uint64_t n, const QueryPlan& qp);
void batch_ws_destroy(BatchWorkspace* w);
void batch_ws_release(BatchWorkspace* w);  // frees its device memory (synchronises the device)
uint64_t batch_ws_bytes(BatchWorkspace* w);
rs_status run_batch_impl(const rs_graph* const* graphs, const rs_query* queries, uint32_t nq, rs_result* results,
                         const rs_tuning* tune, hipStream_t st, bool use_graph, uint64_t slot_budget,
                         BatchWorkspace* ws);

// Graph construction kernels (rs_graph.hip).
struct GraphDev {
  uint32_t n = 0;
  uint64_t m = 0;
  uint32_t n_colours = 0;
  DevBuf e_src, e_dst, e_t, e_out, hi, in_off, colour;
};

// ---------------------------------------------------------------------------
// Profiling (rs_engine.hip)
// ---------------------------------------------------------------------------
enum KernelClass { KC_SCAN = 0, KC_FIRST, KC_TOP, KC_QTABLE, KC_ZTABLE, KC_WINDOW, KC_BATCH, KC_LITERAL, KC_COUNT };
bool profiling_on();
// Look-back counters (rs_lookback_count / rs_lookback_get): while counting is
// on, the level kernels of both paths count predecessor runs recomputed after
// the bounded wait and probe rounds that found no record, and each query or
// batch adds its counts to the process totals.
bool lookback_counting();
void lookback_add(uint64_t recomputes, uint64_t unanswered);
struct ProfScope {
  // Records events around one launch of class `kc` on `st` when profiling is
  // on and the caller allows it (the no-allocation workspace does not).
  ProfScope(KernelClass kc, hipStream_t st, double algorithmic_bytes, bool allowed = true);
  ~ProfScope();
  KernelClass kc;
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double bytes;
};
void profile_flush();  // folds completed event pairs into the totals

}  // namespace rs

namespace rs {
// Device buffers of one plain-path query stream on one graph; they grow to
// the largest query run through them and stay allocated until release().
// A workspace with `scratch` set instead borrows every buffer from that
// device region (carved anew for each query, never allocated or freed); it
// also records no events and takes no kernel timing or launch trace.
struct PlainWorkspace {
  DevBuf lo, z, q, p0, p1, partial, agg, incl, fsum, out, ref, need;
  DevBuf lb_stats;  // look-back counters, allocated only while launches are traced
  DevBuf run_pre, run_bsum, run_boff, run_bounds;  // work-balanced runs of the prefix levels
  DevBuf cov_diff;  // window-cover scratch of the flags: difference array and block sums
  DevBuf lists;     // compacted edge lists of levels 2..k and their scratch (k >= 3)
  DevBuf rr;        // level-2 prefix rows (k >= 4)
  DevBuf grp;       // last level grouped by window
  DevBuf dv, smask, tmask, rmask;  // constraints: per-vertex resting times, source, target and removed masks
  DevBuf fine_t, fine_z, fine_r;   // fine-grained outputs: per-edge sums, per-slot zeta, reach times
  uint32_t epoch = 0;
  uint64_t p_elems_per_chunk = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  uint8_t* scratch = nullptr;  // borrowed region (no-allocation workspace), or null
  uint64_t scratch_bytes = 0;
  uint64_t bytes() const {
    uint64_t t = 0;
    for (const DevBuf* b : {&lo, &z, &q, &p0, &p1, &partial, &agg, &incl, &fsum, &out, &ref, &need, &lb_stats,
                            &run_pre, &run_bsum, &run_boff, &run_bounds, &cov_diff, &lists, &rr, &grp, &dv, &smask, &tmask, &rmask,
                            &fine_t, &fine_z, &fine_r})
      t += b->bytes;
    return t;
  }
  void release() {
    if (scratch) return;  // borrowed buffers are never freed
    for (DevBuf* b : {&lo, &z, &q, &p0, &p1, &partial, &agg, &incl, &fsum, &out, &ref, &need, &lb_stats,
                      &run_pre, &run_bsum, &run_boff, &run_bounds, &cov_diff, &lists, &rr, &grp, &dv, &smask, &tmask, &rmask, &fine_t,
                      &fine_z, &fine_r})
      b->release();
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    ev0 = ev1 = nullptr;
    epoch = 0;
    p_elems_per_chunk = 0;
  }
};
// Buffer sizes (bytes) a query needs in a plain workspace (p: each of the two
// prefix-state arrays; records: each of the two look-back record arrays;
// run_*: the work-balanced run bounds of the prefix levels).
struct PlainSizes {
  uint64_t lo, z, q, p, partial, fsum, ref, need, cover, records;
  uint64_t run_pre, run_bsum, run_boff, run_bounds;
  uint64_t lists;                  // compacted lists (k >= 3; the q table is used only at k = 2)
  uint64_t rr;                     // level 2 folded into level 3 (k >= 4): prefix rows and block carries
  uint64_t grp;                    // last level by distinct windows (k >= 3, not fine-grained)
  uint64_t dv, smask, tmask, rmask;  // constraints (0 when absent)
  uint64_t fine_t, fine_z, fine_r; // fine-grained outputs (0 when not asked)
  // waves per chunk of level 2, of level 3 and of levels >= 4; bounds stride
  uint32_t run_w2, run_w3, run_w4, run_stride;
  uint64_t total() const;
};
PlainSizes plain_sizes(uint64_t m, uint64_t n, const QueryPlan& qp, const Tuning& tu,
                       const QueryExtras* ex = nullptr);
// Largest query workspace of the no-allocation entry point (bytes of its
// per-device scratch array).
constexpr uint64_t kNoAllocScratchBytes = 256ull << 20;
}  // namespace rs

// Opaque graph handle.
namespace rs {
// State of the literal-reading fine-grained sieve on one graph (rs_literal.hip):
// the slot structure (built on first use) and the query buffers.
constexpr uint32_t kLiteralTile = 16;  // edges per wave in the literal level kernel
struct LiteralState {
  bool built = false;
  uint64_t ns = 0;                  // slots (maximal runs of equal (dst, t))
  DevBuf slot, slot_t, v_soff;      // slot of each edge [m], time of each slot [ns], first slot per vertex [n+1]
  DevBuf wlo, whi, y2, need, z, zs, out, chi0, chi1, dv, reach, zeta_edge;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  void release() {
    for (DevBuf* b : {&slot, &slot_t, &v_soff, &wlo, &whi, &y2, &need, &z, &zs, &out, &chi0, &chi1, &dv, &reach,
                      &zeta_edge})
      b->release();
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    ev0 = ev1 = nullptr;
    built = false;
  }
};
}  // namespace rs

struct rs_graph {
  int device = 0;
  rs::GraphDev g;
  rs_graph_info info{};
  // Query workspace of rs_run on this graph; guarded by mu.
  std::mutex mu;
  rs::PlainWorkspace ws;
  // Autotuned launch shapes per k (index k) for the plain path, and one for
  // the batched path.
  rs::Tuning tuned[RS_MAX_K + 1];
  bool has_tuned[RS_MAX_K + 1] = {false};
  rs::Tuning batch_tuned;
  bool has_batch_tuned = false;
  // Window and flag counts per (delta, k) and prefix level, measured when kernel timing is on;
  // guarded by counts_mu.
  std::mutex counts_mu;
  std::map<std::pair<uint32_t, uint32_t>, std::vector<rs::NeedCounts>> need_counts;  // by (delta, k), per level
  rs::DevBuf counts_dev;
  rs::LiteralState lit;  // literal-reading sieve (rs_run_literal); guarded by mu
};
