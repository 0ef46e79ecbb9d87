// Sieve kernels for gfx950.
//
// Layout (one query, one 64-iteration chunk):
//   * Edges are sorted by (dst, t, src); the in-edges of vertex u form the
//     segment [in_off[u], in_off[u+1]) ordered by time.
//   * The prefix state P of a level has m + n slots. Slot in_off[u] + u holds 0;
//     slot e + dst(e) + 1 holds the XOR of the level's values over the edges of
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
// level; within a wavefront the edge is uniform, so q_j is loaded once per
// wave and each lane forms its own subset XOR (6 lane bits + chunk bits).
// One GF(2^64) product remains per edge-update.
//
// Prefix levels keep a running XOR per lane along a tile of E consecutive
// edges; a segment that crosses tiles receives its carry through a decoupled
// look-back on per-tile flags (cache-bypassing device-scope stores and loads,
// ordered with s_waitcnt, no L2 writeback fence).
#include "rs_device.h"
#include "rs_internal.h"

namespace rs {

// ---------------------------------------------------------------------------
// Device-coherent accesses for the look-back state.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void st_dev64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_dev64(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev32(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_dev32(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Orders this wave's earlier memory operations before later ones by waiting
// for them to complete (vmcnt = 0); no cache writeback or invalidation.
__device__ __forceinline__ void order_release() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0xF70);
}
__device__ __forceinline__ void order_acquire() {
  __builtin_amdgcn_s_waitcnt(0xF70);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Per-lane subset XOR  XOR_{j in L} row[j]  for the iteration L = cb + lane
// (cb a multiple of 64): bits 0..5 of L come from the lane, higher bits from cb.
template <int KQ>
__device__ __forceinline__ uint64_t subset_xor(const uint64_t* __restrict__ row, uint64_t cb,
                                               const uint32_t (&mk)[6]) {
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

__device__ __forceinline__ void publish(uint64_t* __restrict__ vals, uint32_t* __restrict__ flags,
                                        uint64_t fi, uint32_t lane, uint64_t v, uint32_t state,
                                        uint32_t epoch) {
  st_dev64(&vals[fi * kLanes + lane], v);
  order_release();
  if (lane == 0) st_dev32(&flags[fi], (epoch << 2) | state);
}

// XOR of the level values of the segment part preceding tile `tile`.
__device__ uint64_t look_back(uint32_t tile, uint64_t row0, uint32_t lane, uint32_t epoch,
                              uint32_t* __restrict__ flags, uint64_t* __restrict__ agg,
                              uint64_t* __restrict__ incl, uint32_t* __restrict__ err) {
  uint64_t carry = 0;
  uint32_t j = tile - 1;
  uint32_t spins = 0;
  while (true) {
    const uint64_t fi = row0 + j;
    const uint32_t f = uniform(ld_dev32(&flags[fi]));
    if ((f >> 2) == epoch) {
      order_acquire();
      if ((f & 3u) == kFlagIncl) {
        carry ^= ld_dev64(&incl[fi * kLanes + lane]);
        break;
      }
      carry ^= ld_dev64(&agg[fi * kLanes + lane]);
      if (j == 0) {  // tile 0 always starts a segment; reaching here is a bug
        if (lane == 0) atomicOr(err, 2u);
        break;
      }
      --j;
      spins = 0;
      continue;
    }
    if (++spins > kSpinLimit) {
      if (lane == 0) atomicOr(err, 1u);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return carry;
}

// ---------------------------------------------------------------------------
// Prefix levels 2..k-1.
// ---------------------------------------------------------------------------
template <int KQ, int E, bool FIRST>
__global__ __launch_bounds__(256) void k_scan(
    const uint32_t* __restrict__ e_src, const uint32_t* __restrict__ e_out,
    const uint32_t* __restrict__ hi_idx, const uint32_t* __restrict__ lo_idx,
    const uint64_t* __restrict__ q, const uint64_t* __restrict__ z,
    const uint64_t* __restrict__ p_prev, uint64_t* __restrict__ p_cur, uint64_t p_stride,
    uint64_t chunk_base, uint32_t m, uint32_t n_tiles, uint32_t epoch,
    uint32_t* __restrict__ tile_counter, uint32_t* __restrict__ flags, uint64_t* __restrict__ agg,
    uint64_t* __restrict__ incl, uint32_t* __restrict__ err) {
  extern __shared__ uint64_t dyn_lds[];  // [waves][16][64]
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = threadIdx.x >> 6;
  uint64_t* tab = dyn_lds + wv * 16 * kLanes + lane;
  tab[0] = 0;

  const uint32_t chunk = blockIdx.y;
  uint32_t tile = 0;
  if (lane == 0) tile = atomicAdd(&tile_counter[chunk], 1u);
  tile = uniform(tile);
  if (tile >= n_tiles) return;

  const uint64_t cb = chunk_base + (uint64_t)chunk * kLanes;
  uint32_t mk[6];
  lane_masks(lane, mk);
  const uint64_t* __restrict__ pp = p_prev + (uint64_t)chunk * p_stride;
  uint64_t* __restrict__ pc = p_cur + (uint64_t)chunk * p_stride;

  const uint32_t e0 = tile * (uint32_t)E;
  const uint32_t ne = min((uint32_t)E, m - e0);
  const bool cont = e0 > 0 && e_out[e0] == e_out[e0 - 1] + 1u;

  uint64_t pref[E];
  uint32_t slot[E];
  uint64_t acc = 0;
  uint32_t first_len = 0;
  bool started = !cont;
  uint32_t last_slot = 0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    pref[i] = 0;
    slot[i] = 0;
    if ((uint32_t)i < ne) {
      const uint32_t e = e0 + (uint32_t)i;
      const uint32_t s = e_out[e];
      if (i > 0 && s != last_slot + 1u) {
        acc = 0;
        started = true;
      }
      if (!started) first_len = (uint32_t)i + 1u;
      const uint64_t aL = subset_xor<KQ>(q + (uint64_t)e * KQ, cb, mk);
      uint64_t w;
      if (FIRST) {
        w = subset_xor<KQ>(z + (uint64_t)e_src[e] * KQ, cb, mk);
      } else {
        w = pp[(uint64_t)hi_idx[e] * kLanes + lane] ^ pp[(uint64_t)lo_idx[e] * kLanes + lane];
      }
      acc ^= gf_mul(tab, aL, w);
      pref[i] = acc;
      slot[i] = s;
      last_slot = s;
    }
  }

  const uint32_t e_end = e0 + ne;
  const bool next_cont = e_end < m && e_out[e_end] == last_slot + 1u;
  const uint64_t row0 = (uint64_t)chunk * n_tiles;
  const uint64_t fi = row0 + tile;
  if (next_cont) publish(started ? incl : agg, flags, fi, lane, acc, started ? kFlagIncl : kFlagAgg, epoch);
  uint64_t carry = 0;
  if (cont) {
    carry = look_back(tile, row0, lane, epoch, flags, agg, incl, err);
    if (next_cont && !started) publish(incl, flags, fi, lane, carry ^ acc, kFlagIncl, epoch);
  }
#pragma unroll
  for (int i = 0; i < E; ++i)
    if ((uint32_t)i < ne) pc[(uint64_t)slot[i] * kLanes + lane] = pref[i] ^ ((uint32_t)i < first_len ? carry : 0);
}

// ---------------------------------------------------------------------------
// Last level k: per-lane XOR of all edge values, one atomic per lane per wave.
// ---------------------------------------------------------------------------
template <int KQ, bool FIRST>
__global__ __launch_bounds__(256) void k_top(
    const uint32_t* __restrict__ e_src, const uint32_t* __restrict__ hi_idx,
    const uint32_t* __restrict__ lo_idx, const uint64_t* __restrict__ q,
    const uint64_t* __restrict__ z, const uint64_t* __restrict__ p_prev, uint64_t p_stride,
    uint64_t chunk_base, uint64_t it_begin, uint64_t it_end, uint32_t m, uint32_t edges_per_wave,
    uint64_t* __restrict__ fsum) {
  extern __shared__ uint64_t dyn_lds[];  // [waves][16][64]
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = threadIdx.x >> 6;
  uint64_t* tab = dyn_lds + wv * 16 * kLanes + lane;
  tab[0] = 0;
  const uint32_t chunk = blockIdx.y;
  const uint64_t wave_id = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wv;
  const uint64_t e0 = wave_id * edges_per_wave;
  if (e0 >= m) return;
  const uint32_t e1 = (uint32_t)min((uint64_t)m, e0 + edges_per_wave);
  const uint64_t cb = chunk_base + (uint64_t)chunk * kLanes;
  uint32_t mk[6];
  lane_masks(lane, mk);
  const uint64_t* __restrict__ pp = p_prev + (uint64_t)chunk * p_stride;
  Acc128 r = {0, 0, 0, 0};
  for (uint32_t e = (uint32_t)e0; e < e1; ++e) {
    const uint64_t aL = subset_xor<KQ>(q + (uint64_t)e * KQ, cb, mk);
    uint64_t w;
    if (FIRST) {
      w = subset_xor<KQ>(z + (uint64_t)e_src[e] * KQ, cb, mk);
    } else {
      w = pp[(uint64_t)hi_idx[e] * kLanes + lane] ^ pp[(uint64_t)lo_idx[e] * kLanes + lane];
    }
    gf_table(tab, w);
    gf_comb_acc(lds_addr(tab), aL, r);
  }
  const uint64_t f = gf_reduce(r);
  const uint64_t it = cb + lane;
  if (it >= it_begin && it < it_end && f) atomicXor((unsigned long long*)&fsum[it], (unsigned long long)f);
}

// ---------------------------------------------------------------------------
// Per-query setup.
// ---------------------------------------------------------------------------
struct ShadeTable {
  uint8_t mu[RS_MAX_COLOURS];
  uint8_t off[RS_MAX_COLOURS];
};

// z_{u,j} (Sec. 4.3) or the shade sum of Eq. (multilinear:3); rows padded to kq.
__global__ __launch_bounds__(256) void k_ztable(uint64_t* __restrict__ z, uint32_t n, uint32_t k,
                                                uint32_t kq, uint64_t seed, int motif,
                                                const uint8_t* __restrict__ colour, ShadeTable sh) {
  __shared__ uint64_t lds[4][16][kLanes];
  const uint32_t lane = threadIdx.x & 63u;
  uint64_t* tab = &lds[threadIdx.x >> 6][0][lane];
  tab[0] = 0;
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)n * kq) return;
  const uint32_t u = (uint32_t)(idx / kq), j = (uint32_t)(idx % kq);
  uint64_t v = 0;
  if (j < k) {
    const uint64_t jj = (uint64_t)(j + 1) << 32;
    if (!motif) {
      v = hash1(seed, 'Z', (uint64_t)u | jj);
    } else {
      const uint32_t s = colour[u];
      for (uint32_t r = 0; r < sh.mu[s]; ++r) {
        const uint64_t d = (uint64_t)sh.off[s] + r;
        v ^= gf_mul(tab, hash1(seed, 'G', (uint64_t)u | (d << 32)), hash1(seed, 'W', d | jj));
      }
    }
  }
  z[idx] = v;
}

// lo(e): slot of the first arrival at v = src(e) with time >= t(e) - delta.
__global__ __launch_bounds__(256) void k_window(const uint32_t* __restrict__ e_src,
                                                const uint32_t* __restrict__ e_t,
                                                const uint32_t* __restrict__ in_off,
                                                uint32_t* __restrict__ lo, uint32_t m,
                                                uint32_t delta) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t v = e_src[e];
  const uint32_t t = e_t[e];
  const uint32_t thr = t > delta ? t - delta : 0u;
  uint32_t a = in_off[v], b = in_off[v + 1];
  while (a < b) {
    const uint32_t mid = a + ((b - a) >> 1);
    if (e_t[mid] < thr)
      a = mid + 1;
    else
      b = mid;
  }
  lo[e] = a + v;
}

// q[l-2][e][j] = z_{dst(e),j} * y_{e,l-1} for l = 2..k.
template <int KQ>
__global__ __launch_bounds__(256) void k_qtable(const uint32_t* __restrict__ e_src,
                                                const uint32_t* __restrict__ e_dst,
                                                const uint32_t* __restrict__ e_t,
                                                const uint64_t* __restrict__ z,
                                                uint64_t* __restrict__ q, uint32_t m, uint32_t k,
                                                uint64_t seed) {
  __shared__ uint64_t lds[4][16][kLanes];
  const uint32_t lane = threadIdx.x & 63u;
  uint64_t* tab = &lds[threadIdx.x >> 6][0][lane];
  tab[0] = 0;
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t src = e_src[e], dst = e_dst[e], t = e_t[e];
  uint64_t zr[KQ];
#pragma unroll
  for (int j = 0; j < KQ; ++j) zr[j] = z[(uint64_t)dst * KQ + j];
  const uint64_t w0 = (uint64_t)src | ((uint64_t)dst << 32);
  for (uint32_t p = 1; p < k; ++p) {
    const uint64_t y = hash2(seed, 'Y', w0, (uint64_t)t | ((uint64_t)p << 32));
    gf_table(tab, y);
    uint64_t* out = q + ((uint64_t)(p - 1) * m + e) * KQ;
#pragma unroll
    for (int j = 0; j < KQ; ++j) {
      Acc128 r = {0, 0, 0, 0};
      gf_comb_acc(lds_addr(tab), zr[j], r);
      out[j] = gf_reduce(r);
    }
  }
}

__global__ void k_fill32(uint32_t* __restrict__ p, uint32_t v, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill64(uint64_t* __restrict__ p, uint64_t v, uint64_t count) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// out[0] = XOR of f[begin, end); one block.
__global__ __launch_bounds__(1024) void k_xor_reduce(const uint64_t* __restrict__ f, uint64_t begin,
                                                     uint64_t end, uint64_t* __restrict__ out) {
  __shared__ uint64_t part[1024];
  uint64_t acc = 0;
  for (uint64_t i = begin + threadIdx.x; i < end; i += blockDim.x) acc ^= f[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] ^= part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_ztable(uint64_t* z, uint32_t n, const QueryPlan& qp, const uint8_t* colour_d,
                         hipStream_t st) {
  ShadeTable sh;
  for (int i = 0; i < RS_MAX_COLOURS; ++i) {
    sh.mu[i] = qp.mu[i];
    sh.off[i] = qp.shade_off[i];
  }
  const uint64_t cnt = (uint64_t)n * qp.kq;
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ztable, dim3(div_up(cnt, 256)), dim3(256), 0, st, z, n, qp.k, qp.kq, qp.seed,
                     qp.motif ? 1 : 0, colour_d, sh);
  return hipGetLastError();
}

hipError_t launch_window(const uint32_t* e_src, const uint32_t* e_t, const uint32_t* in_off,
                         uint32_t* lo, uint32_t m, uint32_t delta, hipStream_t st) {
  if (!m) return hipSuccess;
  hipLaunchKernelGGL(k_window, dim3(div_up(m, 256)), dim3(256), 0, st, e_src, e_t, in_off, lo, m, delta);
  return hipGetLastError();
}

hipError_t launch_qtable(const uint32_t* e_src, const uint32_t* e_dst, const uint32_t* e_t,
                         const uint64_t* z, uint64_t* q, uint32_t m, const QueryPlan& qp,
                         hipStream_t st) {
  if (!m) return hipSuccess;
  dim3 g(div_up(m, 256)), b(256);
  switch (qp.kq) {
    case 4: hipLaunchKernelGGL(k_qtable<4>, g, b, 0, st, e_src, e_dst, e_t, z, q, m, qp.k, qp.seed); break;
    case 8: hipLaunchKernelGGL(k_qtable<8>, g, b, 0, st, e_src, e_dst, e_t, z, q, m, qp.k, qp.seed); break;
    case 12: hipLaunchKernelGGL(k_qtable<12>, g, b, 0, st, e_src, e_dst, e_t, z, q, m, qp.k, qp.seed); break;
    case 16: hipLaunchKernelGGL(k_qtable<16>, g, b, 0, st, e_src, e_dst, e_t, z, q, m, qp.k, qp.seed); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KQ, int E, bool FIRST>
static void scan_one(const ScanArgs& a, uint32_t chunks, uint32_t wpb, hipStream_t st) {
  dim3 g(div_up(a.n_tiles, wpb), chunks), b(64 * wpb);
  hipLaunchKernelGGL((k_scan<KQ, E, FIRST>), g, b, wpb * 16 * kLanes * 8, st, a.e_src, a.e_out, a.hi, a.lo, a.q, a.z,
                     a.p_prev, a.p_cur, a.p_stride, a.chunk_base, a.m, a.n_tiles, a.epoch,
                     a.tile_counter, a.flags, a.agg, a.incl, a.err);
}

template <int KQ>
static bool scan_kq(const ScanArgs& a, bool first, uint32_t E, uint32_t chunks, uint32_t wpb,
                    hipStream_t st) {
  if (E == 8) {
    if (first) scan_one<KQ, 8, true>(a, chunks, wpb, st); else scan_one<KQ, 8, false>(a, chunks, wpb, st);
  } else if (E == 16) {
    if (first) scan_one<KQ, 16, true>(a, chunks, wpb, st); else scan_one<KQ, 16, false>(a, chunks, wpb, st);
  } else {
    return false;
  }
  return true;
}

hipError_t launch_scan(const ScanArgs& a, bool first_level, uint32_t kq, uint32_t chunks,
                       const Tuning& tu, hipStream_t st) {
  if (!a.n_tiles) return hipSuccess;
  const uint32_t E = tu.edges_per_tile, wpb = tu.waves_per_block;
  bool ok = false;
  switch (kq) {
    case 4: ok = scan_kq<4>(a, first_level, E, chunks, wpb, st); break;
    case 8: ok = scan_kq<8>(a, first_level, E, chunks, wpb, st); break;
    case 12: ok = scan_kq<12>(a, first_level, E, chunks, wpb, st); break;
    case 16: ok = scan_kq<16>(a, first_level, E, chunks, wpb, st); break;
  }
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int KQ>
static void top_kq(const TopArgs& a, bool first, uint32_t chunks, uint32_t wpb, hipStream_t st) {
  const uint32_t waves = div_up(a.m, a.edges_per_wave);
  dim3 g(div_up(waves, wpb), chunks), b(64 * wpb);
  if (first)
    hipLaunchKernelGGL((k_top<KQ, true>), g, b, wpb * 16 * kLanes * 8, st, a.e_src, a.hi, a.lo, a.q, a.z, a.p_prev,
                       a.p_stride, a.chunk_base, a.it_begin, a.it_end, a.m, a.edges_per_wave, a.fsum);
  else
    hipLaunchKernelGGL((k_top<KQ, false>), g, b, wpb * 16 * kLanes * 8, st, a.e_src, a.hi, a.lo, a.q, a.z, a.p_prev,
                       a.p_stride, a.chunk_base, a.it_begin, a.it_end, a.m, a.edges_per_wave, a.fsum);
}

hipError_t launch_top(const TopArgs& a, bool first_level, uint32_t kq, uint32_t chunks,
                      const Tuning& tu, hipStream_t st) {
  if (!a.m) return hipSuccess;
  const uint32_t wpb = tu.waves_per_block;
  switch (kq) {
    case 4: top_kq<4>(a, first_level, chunks, wpb, st); break;
    case 8: top_kq<8>(a, first_level, chunks, wpb, st); break;
    case 12: top_kq<12>(a, first_level, chunks, wpb, st); break;
    case 16: top_kq<16>(a, first_level, chunks, wpb, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t st) {
  if (!count) return hipSuccess;
  hipLaunchKernelGGL(k_fill32, dim3(min(div_up(count, 256), 4096u)), dim3(256), 0, st, p, value, count);
  return hipGetLastError();
}
hipError_t launch_fill64(uint64_t* p, uint64_t value, uint64_t count, hipStream_t st) {
  if (!count) return hipSuccess;
  hipLaunchKernelGGL(k_fill64, dim3(min(div_up(count, 256), 4096u)), dim3(256), 0, st, p, value, count);
  return hipGetLastError();
}
hipError_t launch_xor_reduce(const uint64_t* f, uint64_t begin, uint64_t end, uint64_t* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_xor_reduce, dim3(1), dim3(1024), 0, st, f, begin, end, out);
  return hipGetLastError();
}

}  // namespace rs
