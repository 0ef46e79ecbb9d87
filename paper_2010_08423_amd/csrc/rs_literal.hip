// Fine-grained sieve under the literal reading of Eq. (poly-enc:1).
//
// The recurrence keys the y variable of a window term by the edge's end
// points, the level and the arrival time p = i - j of the predecessor at the
// edge's source v (y_{uv,l-1,p}), not by the edge's own time, and level 1 is
// z^L_v at every time. Every window term therefore has its own y: an
// edge-update costs one product per term, up to delta(v) + 1 of them (the
// evaluation-cost lemma of Sec. 4.3), where the edge-indexed form needs one.
// Paths that differ only in their last edge's time share every variable, so
// each slot (u, i) is tested on its own (Alg. 1's per-slot test).
//
// Layout. A slot is a maximal run of edges with equal (dst, t) in the
// (dst, t, src) order; slot ids follow that order, so the slots of a vertex
// are contiguous and sorted by time. chi_l holds one value per slot and
// iteration: [chunk][slot][64 lanes], 512 contiguous bytes per slot. Terms of
// times at which v has no arrival are zero at levels >= 3, so the window of
// edge e = (v -> u, i) is the contiguous slot range of v with time in
// [i - delta(v), i]; at level 2 the window sums y alone (level 1 is z^L_v at
// every time) into one per-edge constant Y2(e), formed once per query.
//
// Level kernel: one wave per tile of consecutive edges, lanes = the 64
// iterations of a chunk. The y of a term is wave-uniform (a keyed hash of
// scalars), so its product with the lane's chi uses one 16-entry table of
// multiples of y shared by the wave (lanes 0..15 write one entry each) and
// the usual comb. A slot's value z^L_u * XOR(terms) is stored once its last
// edge is reached; a slot cut by a tile boundary is summed with atomic XORs
// into an entry cleared before the launch. Levels below k skip the slots no
// window reads.
#include <rocprim/device/device_scan.hpp>

#include "rs_level.h"

namespace rs {

// As gf_comb_acc, against a table of 16 consecutive 8-byte entries that the
// whole wave shares (base 128-byte aligned, entry v at base + 8 v): lanes that
// look up different entries fall in different LDS banks.
__device__ __forceinline__ void gf_comb_acc8(uint32_t base, uint64_t a, Acc128& r) {
  const uint32_t a0 = lo32(a), a1 = hi32(a);
  uint32_t d0 = 0, d1 = 0, d2 = 0, d3 = 0;
#pragma unroll
  for (int j = 7; j >= 0; --j) {
    const uint32_t s0 = (4 * j >= 3) ? (a0 >> (4 * j - 3)) : (a0 << (3 - 4 * j));
    const uint32_t s1 = (4 * j >= 3) ? (a1 >> (4 * j - 3)) : (a1 << (3 - 4 * j));
    // base has bits 3..6 clear, so OR equals XOR
    const uint64_t x = lds_load(and_xor(s0, 0x78u, base));
    const uint64_t y = lds_load(and_xor(s1, 0x78u, base));
    d0 ^= lo32(x);
    d1 = xor3(d1, hi32(x), lo32(y));
    d2 ^= hi32(y);
    if (j) {
      d3 = funnel(d3, d2, 28);
      d2 = funnel(d2, d1, 28);
      d1 = funnel(d1, d0, 28);
      d0 <<= 4;
    }
  }
  r.d0 ^= d0;
  r.d1 ^= d1;
  r.d2 ^= d2;
  r.d3 ^= d3;
}

// acc * w through a half table: entries 0..7 of w's multiples in this lane's
// column (rows 1..7 written here, row 0 holds 0), 8 w in registers and added
// where a nibble's top bit is set. Half the LDS of gf_mul, for four more VALU
// ops per nibble.
__device__ __forceinline__ uint64_t gf_mul_half(uint64_t* tab, uint64_t a, uint64_t w) {
  uint32_t l1 = lo32(w), h1 = hi32(w);
  uint32_t l2 = l1, h2 = h1;
  gf_times_x(l2, h2);
  uint32_t l4 = l2, h4 = h2;
  gf_times_x(l4, h4);
  uint32_t l8 = l4, h8 = h4;
  gf_times_x(l8, h8);
  const uint64_t t1 = w, t2 = mk64(l2, h2), t4 = mk64(l4, h4);
  const uint64_t t3 = t1 ^ t2;
  tab[1 * kLanes] = t1;
  tab[2 * kLanes] = t2;
  tab[3 * kLanes] = t3;
  tab[4 * kLanes] = t4;
  tab[5 * kLanes] = t4 ^ t1;
  tab[6 * kLanes] = t4 ^ t2;
  tab[7 * kLanes] = t4 ^ t3;
  const uint32_t base = lds_addr(tab);
  const uint32_t a0 = lo32(a), a1 = hi32(a);
  uint32_t d0 = 0, d1 = 0, d2 = 0, d3 = 0;
#pragma unroll
  for (int j = 7; j >= 0; --j) {
    const uint32_t s0 = (4 * j >= 9) ? (a0 >> (4 * j - 9)) : (a0 << (9 - 4 * j));
    const uint32_t s1 = (4 * j >= 9) ? (a1 >> (4 * j - 9)) : (a1 << (9 - 4 * j));
    const uint64_t x = lds_load(and_xor(s0, 0x0E00u, base));
    const uint64_t y = lds_load(and_xor(s1, 0x0E00u, base));
    const uint32_t m0 = 0u - ((a0 >> (4 * j + 3)) & 1u), m1 = 0u - ((a1 >> (4 * j + 3)) & 1u);
    d0 = xor3(d0, lo32(x), l8 & m0);
    d1 = xor3(d1, hi32(x) ^ (h8 & m0), xor3(lo32(y), l8 & m1, 0u));
    d2 = xor3(d2, hi32(y), h8 & m1);
    if (j) {
      d3 = funnel(d3, d2, 28);
      d2 = funnel(d2, d1, 28);
      d1 = funnel(d1, d0, 28);
      d0 <<= 4;
    }
  }
  return gf_reduce(Acc128{d0, d1, d2, d3});
}

// y * x with y wave-uniform: the multiples y*c, c = 0..15, go to this wave's
// 128-byte region (entry c at byte offset 8 c; lane c writes entry c), then
// every lane combs its own x against it. (With the entries 512 bytes apart,
// all sixteen fell in the same two LDS banks and the lanes' lookups of
// different entries conflicted.)
__device__ __forceinline__ uint64_t gf_mul_uniform(uint64_t* region, uint32_t lane, uint64_t y, uint64_t x) {
  uint32_t l1 = lo32(y), h1 = hi32(y);
  uint32_t l2 = l1, h2 = h1;
  gf_times_x(l2, h2);
  uint32_t l4 = l2, h4 = h2;
  gf_times_x(l4, h4);
  uint32_t l8 = l4, h8 = h4;
  gf_times_x(l8, h8);
  const uint32_t c = lane & 15u;
  uint32_t lo = (c & 1u) ? l1 : 0u, hi = (c & 1u) ? h1 : 0u;
  lo ^= (c & 2u) ? l2 : 0u;
  hi ^= (c & 2u) ? h2 : 0u;
  lo ^= (c & 4u) ? l4 : 0u;
  hi ^= (c & 4u) ? h4 : 0u;
  lo ^= (c & 8u) ? l8 : 0u;
  hi ^= (c & 8u) ? h8 : 0u;
  if (lane < 16) region[c] = mk64(lo, hi);
  __builtin_amdgcn_wave_barrier();
  Acc128 r = {0, 0, 0, 0};
  gf_comb_acc8(lds_addr(region), x, r);
  __builtin_amdgcn_wave_barrier();
  return gf_reduce(r);
}

// ---------------------------------------------------------------------------
// Slot structure of a graph (once per graph).
// ---------------------------------------------------------------------------
__global__ void k_lit_marks(const uint32_t* __restrict__ e_dst, const uint32_t* __restrict__ e_t, uint64_t m,
                            uint32_t* __restrict__ mark) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  mark[e] = (e == 0 || e_dst[e] != e_dst[e - 1] || e_t[e] != e_t[e - 1]) ? 1u : 0u;
}

// scan = inclusive prefix of the marks: slot(e) = scan[e] - 1.
__global__ void k_lit_slots(const uint32_t* __restrict__ scan, const uint32_t* __restrict__ e_t, uint64_t m,
                            uint32_t* __restrict__ slot, uint32_t* __restrict__ slot_t) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t s = scan[e] - 1;
  slot[e] = s;
  if (e == 0 || scan[e - 1] != scan[e]) slot_t[s] = e_t[e];
}

// v_soff[v] = first slot of vertex v (slot of its first in-edge), v in [0, n].
__global__ void k_lit_voff(const uint32_t* __restrict__ in_off, const uint32_t* __restrict__ slot, uint64_t m,
                           uint32_t n, uint32_t ns, uint32_t* __restrict__ v_soff) {
  const uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  const uint32_t e = in_off[v];
  v_soff[v] = e < m ? slot[e] : ns;
}

// ---------------------------------------------------------------------------
// Per query: windows, the level-2 constants and the slots some window reads.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t lit_edge_key(uint64_t hp, uint32_t v, uint32_t u) {
  return mix64(hp ^ (((uint64_t)v | ((uint64_t)u << 32)) + kGolden));
}
__device__ __forceinline__ uint64_t lit_y(uint64_t h_edge, uint32_t p, uint32_t level) {
  return mix64(h_edge ^ (((uint64_t)p | ((uint64_t)level << 32)) + kGolden));
}

__global__ void k_lit_windows(const uint32_t* __restrict__ e_src, const uint32_t* __restrict__ e_dst,
                              const uint32_t* __restrict__ e_t, const uint32_t* __restrict__ slot_t,
                              const uint32_t* __restrict__ v_soff, uint64_t m, uint32_t delta,
                              const uint32_t* __restrict__ delta_v, uint64_t hp, uint32_t* __restrict__ wlo,
                              uint32_t* __restrict__ whi, uint64_t* __restrict__ y2, uint8_t* __restrict__ need) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t v = e_src[e], u = e_dst[e], i = e_t[e];
  const uint32_t dv = delta_v ? delta_v[v] : delta;
  const uint32_t t0 = i > dv ? i - dv : 1u;
  // slots of v with time in [t0, i]
  uint32_t lo = v_soff[v], hi = v_soff[v + 1];
  uint32_t a = lo, b = hi;
  while (a < b) {
    const uint32_t mid = (a + b) / 2;
    if (slot_t[mid] < t0) a = mid + 1; else b = mid;
  }
  uint32_t c = a;
  b = hi;
  while (c < b) {
    const uint32_t mid = (c + b) / 2;
    if (slot_t[mid] <= i) c = mid + 1; else b = mid;
  }
  wlo[e] = a;
  whi[e] = c;
  for (uint32_t s = a; s < c; ++s) need[s] = 1;
  // Y2(e): the level-2 window sum of y over every time i - j >= 1, j <= delta(v)
  const uint64_t h = lit_edge_key(hp, v, u);
  uint64_t acc = 0;
  for (uint64_t p = t0; p <= i; ++p) acc ^= lit_y(h, (uint32_t)p, 1);
  y2[e] = acc;
}

// Clears, in every chunk of the launch, the entries of the slots that a tile
// boundary cuts (they are summed with atomic XORs).
__global__ void k_lit_zero_split(const uint32_t* __restrict__ slot, const uint8_t* __restrict__ need, uint64_t m,
                                 uint32_t tile, uint64_t c_stride, uint64_t* __restrict__ cur) {
  const uint64_t b = (uint64_t)blockIdx.x * tile;
  if (b == 0 || b >= m) return;
  const uint32_t s = slot[b];
  if (s != slot[b - 1] || !need[s]) return;
  cur[blockIdx.y * c_stride + (uint64_t)s * kLanes + threadIdx.x] = 0;
}

struct LitArgs {
  const uint32_t *e_src, *e_dst, *slot, *wlo, *whi, *slot_t;
  const uint8_t* need;
  const uint64_t *y2, *z;
  const uint64_t* chi_prev;
  uint64_t* chi_cur;
  uint64_t* zeta;
  uint64_t c_stride;
  uint64_t hp;
  uint64_t chunk_base, it_begin, it_end;
  uint32_t m, level, tile;
};

__device__ __forceinline__ uint64_t wave_xor64(uint64_t v) {
  uint32_t lo = lo32(v), hi = hi32(v);
#pragma unroll
  for (int d = 1; d < kLanes; d <<= 1) {
    lo ^= (uint32_t)__shfl_xor((int)lo, d, kLanes);
    hi ^= (uint32_t)__shfl_xor((int)hi, d, kLanes);
  }
  return mk64(lo, hi);
}

// Level a.level of every slot touched by this wave's tile of edges.
template <int KQ, bool FIRST, bool LAST>
__global__ __launch_bounds__(256) void k_lit_level(LitArgs a) {
  // Per-lane half tables of the slot products, [wave][entry 0..7][lane]; the
  // kernel's only static LDS object, so it starts at address 0 (the comb
  // needs bits 9..11 of a table's base clear). A wave's uniform table of the
  // window terms (16 entries, bits 3..6 of its base clear) lives in entry
  // row 1 of its region: a slot product rewrites rows 1..7 before it reads
  // them, and the uniform table is rewritten for every window term, so they
  // never overlap in time. At 16 KB per block of four waves the kernel runs
  // eight waves per SIMD instead of five with full 16-entry tables (32 KB per
  // block): 6.79-6.81 -> 4.68-4.73 ms per query on the 10^6-edge path query
  // (same box, alternating runs), the half table's extra VALU work included.
  __shared__ uint64_t lds[4][8][kLanes];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint64_t* region = &lds[wv][1][0];
  uint64_t* tab = &lds[wv][0][lane];
  const uint32_t chunk = blockIdx.y;
  const uint64_t cb = a.chunk_base + (uint64_t)chunk * kLanes;
  const uint64_t e0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + wv) * a.tile;
  if (e0 >= a.m) return;
  const uint64_t e1 = e0 + a.tile < a.m ? e0 + a.tile : a.m;
  uint32_t mk[6];
  lane_masks(lane, mk);
  cu32* slot = as_const(a.slot);
  cu32* src = as_const(a.e_src);
  cu32* dst = as_const(a.e_dst);
  cu32* wlo = as_const(a.wlo);
  cu32* whi = as_const(a.whi);
  cu32* slot_t = as_const(a.slot_t);
  const uint64_t* prev = a.chi_prev + chunk * a.c_stride;
  uint64_t* cur = LAST ? nullptr : a.chi_cur + chunk * a.c_stride;
  const bool in_range = cb + lane >= a.it_begin && cb + lane < a.it_end;
  // a slot that began before this tile is shared with the tile before
  const uint32_t cut_lo = (e0 > 0 && slot[e0 - 1] == slot[e0]) ? slot[e0] : 0xFFFFFFFFu;
  uint64_t acc = 0;
  for (uint64_t e = e0; e < e1; ++e) {
    const uint32_t sl = slot[e];
    // no window reads this slot at the next level. The flag byte is read with
    // a scalar load of its word: a vector byte load here made every edge wait
    // (vmcnt) for the slot stores of the edges before it.
    if (!LAST && !((*(const __attribute__((address_space(4))) uint32_t*)(a.need + (sl & ~3u)) >> (8 * (sl & 3u))) & 0xFFu))
      continue;
    const uint32_t v = src[e];
    if (FIRST) {
      const uint64_t zv = subset_xor<KQ>(as_const(a.z) + (uint64_t)v * KQ, cb, mk);
      acc ^= gf_mul_uniform(region, lane, as_const(a.y2)[e], zv);
    } else {
      const uint32_t lo = wlo[e], hi = whi[e];
      if (lo != hi) {
        const uint64_t h = lit_edge_key(a.hp, v, dst[e]);
        // the next window slot's row is in flight during this slot's product
        // (the last slot's row is loaded twice)
        uint64_t xn = p_load(prev + (uint64_t)lo * kLanes + lane);
        for (uint32_t s = lo; s < hi; ++s) {
          const uint64_t x = xn;
          xn = p_load(prev + (uint64_t)(s + 1 < hi ? s + 1 : s) * kLanes + lane);
          const uint64_t y = lit_y(h, slot_t[s], a.level - 1);
          acc ^= gf_mul_uniform(region, lane, y, x);
        }
      }
    }
    const bool last_edge = e + 1 == e1 || slot[e + 1] != sl;
    if (!last_edge) continue;
    uint64_t val = 0;
    if (__ballot(acc != 0)) {
      const uint64_t zu = subset_xor<KQ>(as_const(a.z) + (uint64_t)dst[e] * KQ, cb, mk);
      tab[0] = 0;
      val = gf_mul_half(tab, acc, zu);
    }
    acc = 0;
    if (LAST) {
      const uint64_t w = wave_xor64(in_range ? val : 0);
      if (lane == 0 && w) atomicXor((unsigned long long*)&a.zeta[sl], (unsigned long long)w);
    } else {
      const bool cut = sl == cut_lo || (e + 1 == e1 && e1 < a.m && slot[e1] == sl);
      uint64_t* p = cur + (uint64_t)sl * kLanes + lane;
      if (cut) {
        if (val) atomicXor((unsigned long long*)p, (unsigned long long)val);
      } else {
        p_store(p, val);
      }
    }
  }
}

// Per canonical edge: the zeta of its slot; the first edge of each slot with
// a non-zero zeta lowers its vertex's reach time.
__global__ void k_lit_outputs(const uint32_t* __restrict__ slot, const uint32_t* __restrict__ e_dst,
                              const uint32_t* __restrict__ e_t, const uint64_t* __restrict__ zs, uint64_t m,
                              uint64_t* __restrict__ zeta_edge, uint32_t* __restrict__ reach) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t s = slot[e];
  const uint64_t z = zs[s];
  if (zeta_edge) zeta_edge[e] = z;
  if (z && (e == 0 || slot[e - 1] != s)) atomicMin(&reach[e_dst[e]], e_t[e]);
}

static inline uint32_t blocks_for(uint64_t count, uint32_t per) { return (uint32_t)((count + per - 1) / per); }

static rs_status lit_build_slots(const GraphDev& G, LiteralState& L, hipStream_t st) {
  const uint64_t m = G.m;
  const uint32_t n = G.n;
  const size_t mb = (size_t)std::max<uint64_t>(m, 1);
  DevBuf scan, tmp;
  struct Free {
    DevBuf &a, &b;
    ~Free() {
      a.release();
      b.release();
    }
  } free_temps{scan, tmp};
  if (L.slot.reserve((mb + kEdgePad) * 4, st, true) || scan.reserve(mb * 4, st, false) ||
      L.slot_t.reserve(mb * 4, st, false) || L.v_soff.reserve(((size_t)n + 2) * 4, st, true))
    return RS_ENOMEM;
  L.ns = 0;
  if (m) {
    hipLaunchKernelGGL(k_lit_marks, dim3(blocks_for(m, 256)), dim3(256), 0, st, G.e_dst.as<uint32_t>(),
                       G.e_t.as<uint32_t>(), m, L.slot.as<uint32_t>());
    RS_HIP(hipGetLastError());
    size_t need = 0;
    RS_HIP(rocprim::inclusive_scan(nullptr, need, L.slot.as<uint32_t>(), scan.as<uint32_t>(), (size_t)m,
                                   rocprim::plus<uint32_t>(), st));
    if (tmp.reserve(need + 256, st, false)) return RS_ENOMEM;
    size_t sz = tmp.bytes;
    RS_HIP(rocprim::inclusive_scan(tmp.p, sz, L.slot.as<uint32_t>(), scan.as<uint32_t>(), (size_t)m,
                                   rocprim::plus<uint32_t>(), st));
    hipLaunchKernelGGL(k_lit_slots, dim3(blocks_for(m, 256)), dim3(256), 0, st, scan.as<uint32_t>(),
                       G.e_t.as<uint32_t>(), m, L.slot.as<uint32_t>(), L.slot_t.as<uint32_t>());
    RS_HIP(hipGetLastError());
    uint32_t last = 0;
    RS_HIP(hipMemcpyAsync(&last, scan.as<uint32_t>() + (m - 1), 4, hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    L.ns = last;
  }
  hipLaunchKernelGGL(k_lit_voff, dim3(blocks_for((uint64_t)n + 1, 256)), dim3(256), 0, st, G.in_off.as<uint32_t>(),
                     L.slot.as<uint32_t>(), m, n, (uint32_t)L.ns, L.v_soff.as<uint32_t>());
  RS_HIP(hipGetLastError());
  RS_HIP(hipStreamSynchronize(st));  // the temporaries are freed on return
  L.built = true;
  return RS_OK;
}

hipError_t lit_windows(const GraphDev& G, LiteralState& L, uint32_t delta, const uint32_t* delta_v, uint64_t hp,
                       hipStream_t st) {
  if (!G.m) return hipSuccess;
  hipLaunchKernelGGL(k_lit_windows, dim3(blocks_for(G.m, 256)), dim3(256), 0, st, G.e_src.as<uint32_t>(),
                     G.e_dst.as<uint32_t>(), G.e_t.as<uint32_t>(), L.slot_t.as<uint32_t>(),
                     L.v_soff.as<uint32_t>(), G.m, delta, delta_v, hp, L.wlo.as<uint32_t>(), L.whi.as<uint32_t>(),
                     L.y2.as<uint64_t>(), L.need.as<uint8_t>());
  return hipGetLastError();
}

template <int KQ>
static void lit_level_kq(const LitArgs& a, bool first, bool last, uint32_t chunks, hipStream_t st) {
  const uint32_t tiles = blocks_for(a.m, a.tile);
  const dim3 g(blocks_for(tiles, 4), chunks), b(256);
  if (first && last)
    hipLaunchKernelGGL((k_lit_level<KQ, true, true>), g, b, 0, st, a);
  else if (first)
    hipLaunchKernelGGL((k_lit_level<KQ, true, false>), g, b, 0, st, a);
  else if (last)
    hipLaunchKernelGGL((k_lit_level<KQ, false, true>), g, b, 0, st, a);
  else
    hipLaunchKernelGGL((k_lit_level<KQ, false, false>), g, b, 0, st, a);
}

hipError_t lit_level(const LitArgs& a, uint32_t kq, bool first, bool last, uint32_t chunks, hipStream_t st) {
  if (!a.m) return hipSuccess;
  if (!last) {
    const uint32_t tiles = blocks_for(a.m, a.tile);
    hipLaunchKernelGGL(k_lit_zero_split, dim3(tiles, chunks), dim3(kLanes), 0, st, a.slot, a.need, (uint64_t)a.m,
                       a.tile, a.c_stride, a.chi_cur);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  switch (kq) {
    case 4: lit_level_kq<4>(a, first, last, chunks, st); break;
    case 8: lit_level_kq<8>(a, first, last, chunks, st); break;
    case 12: lit_level_kq<12>(a, first, last, chunks, st); break;
    case 16: lit_level_kq<16>(a, first, last, chunks, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t lit_outputs(const GraphDev& G, const LiteralState& L, uint64_t* zeta_edge, uint32_t* reach,
                       hipStream_t st) {
  if (!G.m) return hipSuccess;
  hipLaunchKernelGGL(k_lit_outputs, dim3(blocks_for(G.m, 256)), dim3(256), 0, st, L.slot.as<uint32_t>(),
                     G.e_dst.as<uint32_t>(), G.e_t.as<uint32_t>(), L.zs.as<uint64_t>(), G.m, zeta_edge, reach);
  return hipGetLastError();
}

// SplitMix64 output finalizer on the host (the query's hash prefix).
static uint64_t mix64_host(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

static rs_status run_literal(rs_graph* g, const QueryPlan& qp, const uint32_t* delta_per_vertex,
                             uint32_t* reach_time, uint64_t* slot_zeta, rs_result* r, hipStream_t st) {
  const GraphDev& G = g->g;
  LiteralState& L = g->lit;
  const uint64_t m = G.m;
  const uint32_t n = G.n, k = qp.k, kq = qp.kq;
  if (!L.built) RS_TRY(lit_build_slots(G, L, st));
  if (!L.ev0) {
    RS_HIP(hipEventCreate(&L.ev0));
    RS_HIP(hipEventCreate(&L.ev1));
  }
  const uint64_t ns = L.ns;
  const size_t mb = (size_t)std::max<uint64_t>(m, 1), nsb = (size_t)std::max<uint64_t>(ns, 1);
  const uint64_t nchunks = qp.chunk_last - qp.chunk_first;
  // chunks per launch: the two slot-state buffers of a group within 8 GiB
  const uint64_t per_chunk = 2ull * nsb * kLanes * 8;
  const uint32_t group =
      (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(std::min<uint64_t>(nchunks, 16), (8ull << 30) / per_chunk));
  if (L.wlo.reserve((mb + kEdgePad) * 4, st, false) || L.whi.reserve((mb + kEdgePad) * 4, st, false) ||
      L.y2.reserve((mb + kEdgePad) * 8, st, false) || L.need.reserve(nsb + 8, st, false) ||
      L.z.reserve(((size_t)n + 1) * kq * 8, st, false) || L.zs.reserve(nsb * 8, st, false) ||
      L.out.reserve(64, st, false) || L.chi0.reserve((size_t)group * nsb * kLanes * 8, st, false) ||
      L.chi1.reserve((size_t)group * nsb * kLanes * 8, st, false) ||
      (delta_per_vertex && L.dv.reserve(((size_t)n + 1) * 4, st, false)) ||
      L.reach.reserve(((size_t)n + 1) * 4, st, false) || (slot_zeta && L.zeta_edge.reserve(mb * 8, st, false)))
    return RS_ENOMEM;
  const uint32_t* dv = nullptr;
  if (delta_per_vertex) {
    RS_HIP(hipMemcpyAsync(L.dv.p, delta_per_vertex, 4ull * n, hipMemcpyHostToDevice, st));
    dv = L.dv.as<uint32_t>();
  }
  RS_HIP(hipEventRecord(L.ev0, st));
  const uint64_t hp = mix64_host(qp.seed + (uint64_t)'P' * 0x9E3779B97F4A7C15ull);
  RS_HIP(launch_ztable(L.z.as<uint64_t>(), n, qp, G.colour.as<uint8_t>(), st));
  RS_HIP(launch_fill64(L.need.as<uint64_t>(), 0, (nsb + 7) / 8, st));
  RS_HIP(lit_windows(G, L, qp.delta, dv, hp, st));
  RS_HIP(launch_fill64(L.zs.as<uint64_t>(), 0, nsb, st));
  LitArgs a{};
  a.e_src = G.e_src.as<uint32_t>();
  a.e_dst = G.e_dst.as<uint32_t>();
  a.slot = L.slot.as<uint32_t>();
  a.wlo = L.wlo.as<uint32_t>();
  a.whi = L.whi.as<uint32_t>();
  a.slot_t = L.slot_t.as<uint32_t>();
  a.need = L.need.as<uint8_t>();
  a.y2 = L.y2.as<uint64_t>();
  a.z = L.z.as<uint64_t>();
  a.zeta = L.zs.as<uint64_t>();
  a.c_stride = nsb * kLanes;
  a.hp = hp;
  a.it_begin = qp.it_begin;
  a.it_end = qp.it_end;
  a.m = (uint32_t)m;
  a.tile = kLiteralTile;
  for (uint64_t c0 = qp.chunk_first; c0 < qp.chunk_last; c0 += group) {
    const uint32_t gc = (uint32_t)std::min<uint64_t>(group, qp.chunk_last - c0);
    a.chunk_base = c0 * kLanes;
    uint64_t* prev = L.chi0.as<uint64_t>();
    uint64_t* cur = L.chi1.as<uint64_t>();
    for (uint32_t l = 2; l <= k; ++l) {
      a.level = l;
      a.chi_prev = prev;
      a.chi_cur = cur;
      {
        ProfScope ps(KC_LITERAL, st, 0.0);
        RS_HIP(lit_level(a, kq, l == 2, l == k, gc, st));
      }
      std::swap(prev, cur);
    }
  }
  RS_HIP(launch_fill32(L.reach.as<uint32_t>(), 0xFFFFFFFFu, n, st));
  RS_HIP(lit_outputs(G, L, slot_zeta ? L.zeta_edge.as<uint64_t>() : nullptr, L.reach.as<uint32_t>(), st));
  RS_HIP(launch_xor_reduce(L.zs.as<uint64_t>(), 0, ns, L.out.as<uint64_t>(), st));
  RS_HIP(hipEventRecord(L.ev1, st));
  uint64_t F = 0;
  RS_HIP(hipMemcpyAsync(&F, L.out.p, 8, hipMemcpyDeviceToHost, st));
  if (n) RS_HIP(hipMemcpyAsync(reach_time, L.reach.p, 4ull * n, hipMemcpyDeviceToHost, st));
  if (slot_zeta && m) RS_HIP(hipMemcpyAsync(slot_zeta, L.zeta_edge.p, 8 * m, hipMemcpyDeviceToHost, st));
  RS_HIP(hipStreamSynchronize(st));
  float ms = 0;
  RS_HIP(hipEventElapsedTime(&ms, L.ev0, L.ev1));
  uint32_t reached = 0;
  for (uint32_t u = 0; u < n; ++u) reached |= reach_time[u] != 0xFFFFFFFFu;
  r->fingerprint = F;
  r->yes = reached;
  r->device_ms = ms;
  return RS_OK;
}

}  // namespace rs

using namespace rs;

rs_status rs_run_literal(const rs_graph* gc, const rs_query* q, const uint32_t* delta_per_vertex,
                         uint32_t* reach_time, uint64_t* slot_zeta, rs_result* r, void* hip_stream) {
  if (!r || !reach_time) return RS_EINVAL;
  QueryPlan qp;
  rs_status s = plan_query(gc, q, qp);
  rs_graph* g = const_cast<rs_graph*>(gc);
  try {
    if (s == RS_OK) {
      std::lock_guard<std::mutex> lk(g->mu);
      s = run_literal(g, qp, delta_per_vertex, reach_time, slot_zeta, r, (hipStream_t)hip_stream);
    }
  } catch (...) {
    s = RS_ENOMEM;
  }
  r->status = s;
  return s;
}
