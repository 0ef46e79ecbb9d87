// Per-level sieve kernels for gfx950 (the plain path): setup tables, the
// prefix levels 2..k-1, the last level k and small utilities. The level-step
// arithmetic and data layout are described in rs_level.h.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "rs_level.h"

namespace rs {

// ---------------------------------------------------------------------------
// Prefix levels 2..k-1. The grid holds about as many waves as fit on the GPU;
// at levels >= 3 wave w of W scans the w-th of W contiguous runs of tiles
// (scan_run), at level 2 a few runs spread over the edge list (scan_runs), so
// carries flow in registers along a run and the waves meet only at the run
// ends, through the look-back records. A run whose predecessor has not
// published after a bounded wait recomputes that run's tail (see look_back).
// ---------------------------------------------------------------------------
template <int KQ, int E, bool FIRST, bool DR = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((FIRST || DR || E == 8) ? 5 : 4))) void k_scan(
    const uint32_t* __restrict__ e_src, const uint32_t* __restrict__ e_out,
    const uint32_t* __restrict__ hi_idx, const uint32_t* __restrict__ lo_idx,
    const uint64_t* __restrict__ q, const uint64_t* __restrict__ z, const uint64_t* __restrict__ d,
    const uint64_t* __restrict__ p_prev, uint64_t* __restrict__ p_cur, uint64_t p_stride,
    uint64_t chunk_base, uint32_t m, uint32_t n_tiles, uint32_t epoch,
    uint64_t* __restrict__ agg, uint64_t* __restrict__ incl, const uint8_t* __restrict__ need,
    unsigned long long* __restrict__ lb_stats, const uint32_t* __restrict__ bounds, const uint32_t* __restrict__ count) {
  extern __shared__ uint64_t dyn_lds[];  // [waves][16][64]; starts at LDS address 0
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform for the compiler
  uint64_t* tab = dyn_lds + wv * 16 * kLanes + lane;
  tab[0] = 0;

  // Blocks start in linear order (x fastest) and alternate over the eight
  // XCDs. With a grid width that is a multiple of 8, block L = (8 k + d) takes
  // run block x = 8 (k / C) + d of chunk k mod C (C chunks): a run's chunks
  // share an XCD (and its L2 copy of the run's indices and rows), and runs are
  // in dispatch order, which the skewed split of the runs counts on.
  uint32_t bx = blockIdx.x, chunk = blockIdx.y;
  if ((gridDim.x & 7u) == 0) {
    const uint32_t L = blockIdx.y * gridDim.x + blockIdx.x, k = L >> 3;
    chunk = k % gridDim.y;
    bx = (k / gridDim.y) * 8 + (L & 7u);
  }
  uint32_t mk[6];
  lane_masks(lane, mk);
  TileCtx c;
  c.e_src = e_src;
  c.e_out = e_out;
  c.hi = hi_idx;
  c.lo = lo_idx;
  c.q = q;
  c.z = z;
  c.d = d;
  c.pp = p_prev + (uint64_t)chunk * p_stride;
  c.pc = p_cur + (uint64_t)chunk * p_stride;
  c.cb = chunk_base + (uint64_t)chunk * kLanes;
  // a compacted list's length is on the device; n_tiles stays the record stride
  c.m = count ? __builtin_amdgcn_readfirstlane(*as_const(count)) : m;
  c.n_tiles = count ? (c.m + E - 1) / E : n_tiles;
  c.epoch = epoch;
  c.row0 = (uint64_t)chunk * n_tiles;
  c.agg = agg;
  c.incl = incl;
  c.need = need;
  c.lb_stats = lb_stats;
  c.bounds = bounds;
  const uint32_t waves = gridDim.x * (blockDim.x >> 6);
  scan_level<KQ, E, FIRST, DR>(c, bx * (blockDim.x >> 6) + wv, waves, lane, mk, tab);
}

// ---------------------------------------------------------------------------
// Last level k: grid-stride over edge ranges, per-lane sums XORed across the
// block in LDS, one partial row per block (no contended atomics); k_top_fold
// folds the rows into the per-iteration sums. With H = 2 a wave sums a chunk
// pair (gridDim.y counts pairs) and writes both chunks' rows.
// ---------------------------------------------------------------------------
template <int KQ, bool FIRST, int H = 1>
__global__ __launch_bounds__(256) void k_top(
    const uint32_t* __restrict__ e_src, const uint32_t* __restrict__ hi_idx,
    const uint32_t* __restrict__ lo_idx, const uint64_t* __restrict__ q,
    const uint64_t* __restrict__ z, const uint64_t* __restrict__ p_prev, uint64_t p_stride,
    uint64_t chunk_base, uint32_t m_max, uint32_t edges_per_wave, uint64_t* __restrict__ partial,
    const uint32_t* __restrict__ count, uint32_t* __restrict__ ticket) {
  extern __shared__ uint64_t dyn_lds[];  // [waves][16][64]; starts at LDS address 0
  const uint32_t m = count ? __builtin_amdgcn_readfirstlane(*as_const(count)) : m_max;  // compacted list length
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform for the compiler
  const uint32_t nw = blockDim.x >> 6;
  uint64_t* tab = dyn_lds + wv * 16 * kLanes + lane;
  tab[0] = 0;
  const uint32_t chunk = blockIdx.y;  // chunk pair when H = 2
  const uint64_t chunk0 = (uint64_t)chunk * H;
  const uint64_t cb = chunk_base + chunk0 * kLanes;
  const uint64_t* pp = p_prev + chunk0 * p_stride;
  uint32_t mk[6];
  lane_masks(lane, mk);
  const uint64_t waves = (uint64_t)gridDim.x * nw;
  Acc128 r[H];
#pragma unroll
  for (int h = 0; h < H; ++h) r[h] = Acc128{0, 0, 0, 0};
  if (ticket) {
    // ranges handed out in arrival order: waves dispatched later run slower,
    // and a wave that finishes early takes the next range (the sum is an XOR,
    // so the assignment does not change the result)
    for (;;) {
      uint32_t rid = 0;
      if (lane == 0) rid = atomicAdd(ticket + chunk, 1u);
      rid = __builtin_amdgcn_readfirstlane(rid);
      const uint64_t e0 = (uint64_t)rid * edges_per_wave;
      if (e0 >= m) break;
      const uint32_t e1 = (uint32_t)min((uint64_t)m, e0 + edges_per_wave);
      top_range<KQ, FIRST, H>(e_src, hi_idx, lo_idx, q, z, pp, p_stride, cb, (uint32_t)e0, e1, lane, mk, tab, r);
    }
  } else {
    for (uint64_t wave_id = (uint64_t)blockIdx.x * nw + wv; wave_id * edges_per_wave < m; wave_id += waves) {
      const uint64_t e0 = wave_id * edges_per_wave;
      const uint32_t e1 = (uint32_t)min((uint64_t)m, e0 + edges_per_wave);
      top_range<KQ, FIRST, H>(e_src, hi_idx, lo_idx, q, z, pp, p_stride, cb, (uint32_t)e0, e1, lane, mk, tab, r);
    }
  }
  // XOR the block's waves through LDS entry T[1] of each wave's table, one
  // chunk at a time.
#pragma unroll
  for (int h = 0; h < H; ++h) {
    const uint64_t f = gf_reduce(r[h]);
    __syncthreads();
    tab[kLanes] = f;
    __syncthreads();
    if (wv == 0) {
      uint64_t s = 0;
      for (uint32_t k2 = 0; k2 < nw; ++k2) s ^= dyn_lds[k2 * 16 * kLanes + kLanes + lane];
      partial[((chunk0 + h) * gridDim.x + blockIdx.x) * kLanes + lane] = s;
    }
  }
}

// fsum[cb + lane] = XOR over blocks of partial[chunk][block][lane], for the
// iterations of [it_begin, it_end). One block of 1024 threads per chunk: 16
// groups of 64 lanes stride over the rows with four independent loads in
// flight each, then the groups are XORed in LDS.
__global__ __launch_bounds__(1024) void k_top_fold(const uint64_t* __restrict__ partial, uint32_t blocks,
                                                   uint64_t chunk_base, uint64_t it_begin, uint64_t it_end,
                                                   uint64_t* __restrict__ fsum) {
  __shared__ uint64_t part[16][kLanes];
  const uint32_t chunk = blockIdx.x, lane = threadIdx.x & 63u, grp = threadIdx.x >> 6;
  const uint64_t* rows = partial + (uint64_t)chunk * blocks * kLanes + lane;
  uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  uint32_t b = grp;
  for (; b + 48 < blocks; b += 64) {
    s0 ^= rows[(uint64_t)b * kLanes];
    s1 ^= rows[(uint64_t)(b + 16) * kLanes];
    s2 ^= rows[(uint64_t)(b + 32) * kLanes];
    s3 ^= rows[(uint64_t)(b + 48) * kLanes];
  }
  for (; b < blocks; b += 16) s0 ^= rows[(uint64_t)b * kLanes];
  part[grp][lane] = s0 ^ s1 ^ s2 ^ s3;
  __syncthreads();
  if (grp == 0) {
    uint64_t s = 0;
    for (uint32_t g = 0; g < 16; ++g) s ^= part[g][lane];
    const uint64_t it = chunk_base + (uint64_t)chunk * kLanes + lane;
    if (it >= it_begin && it < it_end) fsum[it] = s;
  }
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

// lo(e): slot of the first arrival at v = src(e) with time >= t(e) - delta(v)
// (delta(v) from delta_v when given, else the scalar delta).
__global__ __launch_bounds__(256) void k_window(const uint32_t* __restrict__ e_src,
                                                const uint32_t* __restrict__ e_t,
                                                const uint32_t* __restrict__ in_off,
                                                uint32_t* __restrict__ lo, uint32_t m,
                                                uint32_t delta, const uint32_t* __restrict__ delta_v) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t v = e_src[e];
  const uint32_t t = e_t[e];
  const uint32_t dv = delta_v ? delta_v[v] : delta;
  const uint32_t thr = t > dv ? t - dv : 0u;
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

// LDS a CU gives to resident blocks, as measured on MI355X: with 8 KB of LDS
// per wave, 18 waves per CU started at once and the 19th and 20th only when
// others had finished (16 with 32 KB blocks), although the occupancy query
// counts 20. Grids sized by the query left a tenth of their waves to start
// late, after the launch had run for about half its time.
constexpr size_t kUsableLdsPerCu = 144 * 1024;

// Blocks of `kern` that fit on the whole GPU at once (cached per kernel and
// block shape).
uint32_t resident_blocks(const void* kern, uint32_t threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, uint32_t, size_t>, uint32_t> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_tuple(kern, threads, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, (int)threads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (lds > 0) per_cu = std::max(1, std::min(per_cu, (int)(kUsableLdsPerCu / lds)));
  const uint32_t v = (uint32_t)std::max(cus, 1) * (uint32_t)per_cu;
  cache[key] = v;
  return v;
}

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

// Exclusive prefix of the block totals of each level (one block per level).
__global__ __launch_bounds__(1024) void k_cost_block_offsets(const uint32_t* __restrict__ bsum, uint32_t nb,
                                                             uint32_t* __restrict__ boff) {
  block_offsets(bsum + (uint64_t)blockIdx.x * nb, nb, boff + (uint64_t)blockIdx.x * nb);
}

__global__ __launch_bounds__(256) void k_need_counts(const uint32_t* __restrict__ hi, const uint32_t* __restrict__ lo,
                                                     const uint8_t* __restrict__ need, uint32_t m,
                                                     unsigned long long* __restrict__ counts) {
  __shared__ unsigned long long part[6];
  if (threadIdx.x < 6) part[threadIdx.x] = 0;
  __syncthreads();
  uint32_t c[6] = {0, 0, 0, 0, 0, 0};
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t f = need[e];
    const bool live = hi[e] != lo[e];
    c[0] += live;
    c[1] += live && (f & 4u);
    c[2] += (f >> 2) & 1u;
    c[3] += f & 1u;
    c[4] += (f >> 1) & 1u;
    c[5] += (f & 7u) != 0;  // kept in the level's compacted list
  }
  for (int j = 0; j < 6; ++j) atomicAdd(&part[j], (unsigned long long)c[j]);
  __syncthreads();
  if (threadIdx.x < 6) atomicAdd(&counts[threadIdx.x], part[threadIdx.x]);
}

hipError_t launch_need_counts(const uint32_t* hi, const uint32_t* lo, const uint8_t* need, uint32_t m,
                              unsigned long long* counts, hipStream_t st) {
  if (!m) return hipSuccess;
  hipLaunchKernelGGL(k_need_counts, dim3(std::min(div_up(m, 256), 512u)), dim3(256), 0, st, hi, lo, need, m, counts);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mark_cover(const uint32_t* __restrict__ hi, const uint32_t* __restrict__ lo,
                                                    const uint8_t* __restrict__ next, uint32_t m,
                                                    uint8_t* __restrict__ ref, uint32_t* __restrict__ diff) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) mark_cover(hi, lo, next, e, ref, diff);
}

// In-place block-wise inclusive prefix of this level's cover difference
// array (see block_prefix). When a lower level follows, the grid also zeroes
// the other pair of scratch arrays (ref_o, diff_o): the flag kernel of the
// level above, their last reader, has finished, and this level's flag kernel
// marks the lower level's windows into them.
__global__ __launch_bounds__(256) void k_cover_prefix(uint32_t* __restrict__ diff, uint64_t slots,
                                                      uint32_t* __restrict__ bsum, uint32_t* __restrict__ diff_o,
                                                      uint32_t* __restrict__ ref_o, uint64_t ref_words) {
  block_prefix(diff, slots, bsum);
  if (!diff_o) return;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < slots; i += stride) diff_o[i] = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ref_words; i += stride) ref_o[i] = 0;
}

// The flags of level l (window emptiness folded into the product bit when
// hi != null), the zero padding past m, and, when ref_n != null, the windows
// of level l's product edges marked for level l - 1 (its readers).
__global__ __launch_bounds__(256) void k_flags_and_marks(const uint32_t* __restrict__ e_out,
                                                         const uint8_t* __restrict__ ref,
                                                         const uint32_t* __restrict__ pre,
                                                         const uint32_t* __restrict__ boff,
                                                         const uint32_t* __restrict__ hi,
                                                         const uint32_t* __restrict__ hi_all,
                                                         const uint32_t* __restrict__ lo, uint32_t m,
                                                         uint8_t* __restrict__ need, uint8_t* __restrict__ ref_n,
                                                         uint32_t* __restrict__ diff_n) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) {
    mark_need_cover(e_out, ref, pre, boff, hi, lo, e, need);
    if (ref_n) mark_cover(hi_all, lo, need, e, ref_n, diff_n);  // reads back this thread's own flag byte
  } else if (e < (uint64_t)m + kEdgePad) {
    need[e] = 0;  // the padding a level's last tile reads
  }
}

hipError_t launch_flags(const uint32_t* e_out, const uint32_t* hi, const uint32_t* lo, uint32_t m, uint32_t n,
                        uint32_t k, uint8_t* need, uint64_t need_stride_b, uint8_t* ref, uint32_t* cov,
                        hipStream_t st) {
  if (!m || k < 3) return hipSuccess;
  const uint64_t slots = (uint64_t)m + n + 1;  // slots 0 .. m+n-1, and one past the last window end
  const uint32_t nb = (uint32_t)((slots + kCostBlock - 1) / kCostBlock);
  const uint64_t ref_bytes = flag_ref_bytes(m, n);
  uint8_t* refs[2] = {ref, ref + ref_bytes};
  uint32_t* diffs[2] = {cov, cov + slots};
  uint32_t* bsum = cov + 2 * slots;
  uint32_t* boff = bsum + nb;
  // level k-1: its readers are every non-empty window of the last level
  {
    const uint32_t b = (k - 1) & 1u;
    hipError_t e = launch_fill32((uint32_t*)refs[b], 0, ref_bytes / 4, st);
    if (e == hipSuccess) e = launch_fill32(diffs[b], 0, slots, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mark_cover, dim3(div_up(m, 256)), dim3(256), 0, st, hi, lo, nullptr, m, refs[b], diffs[b]);
  }
  for (uint32_t l = k - 1; l >= 2; --l) {
    const uint32_t b = l & 1u, o = b ^ 1u;
    const bool lower = l > 2;
    hipLaunchKernelGGL(k_cover_prefix, dim3(nb), dim3(256), 0, st, diffs[b], slots, bsum, lower ? diffs[o] : nullptr,
                       (uint32_t*)refs[o], ref_bytes / 4);
    hipLaunchKernelGGL(k_cost_block_offsets, dim3(1), dim3(1024), 0, st, bsum, nb, boff);
    hipLaunchKernelGGL(k_flags_and_marks, dim3(div_up((uint64_t)m + kEdgePad, 256)), dim3(256), 0, st, e_out,
                       refs[b], diffs[b], boff, l >= 3 ? hi : nullptr, hi, lo, m,
                       need + (uint64_t)(l - 2) * need_stride_b, lower ? refs[o] : nullptr,
                       lower ? diffs[o] : nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_window(const uint32_t* e_src, const uint32_t* e_t, const uint32_t* in_off,
                         uint32_t* lo, uint32_t m, uint32_t delta, const uint32_t* delta_v, hipStream_t st) {
  if (!m) return hipSuccess;
  hipLaunchKernelGGL(k_window, dim3(div_up(m, 256)), dim3(256), 0, st, e_src, e_t, in_off, lo, m, delta, delta_v);
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

template <int KQ, int E, bool FIRST, bool DR = false>
static uint32_t scan_blocks_one(uint32_t n_tiles, uint32_t chunks, uint32_t wpb) {
  const size_t lds = (size_t)wpb * 16 * kLanes * 8;
  const uint32_t fit =
      std::max(1u, resident_blocks((const void*)k_scan<KQ, E, FIRST, DR>, 64 * wpb, lds) / chunks);
  return std::min(div_up(n_tiles, wpb), fit);
}

template <int KQ, int E, bool FIRST, bool DR = false>
static void scan_one(const ScanArgs& a, uint32_t chunks, uint32_t wpb, hipStream_t st) {
  const size_t lds = (size_t)wpb * 16 * kLanes * 8;
  // with run bounds the grid is the one the bounds were cut for
  const uint32_t gx = a.bounds ? a.waves / wpb : scan_blocks_one<KQ, E, FIRST, DR>(a.n_tiles, chunks, wpb);
  dim3 g(gx, chunks), b(64 * wpb);
  hipLaunchKernelGGL((k_scan<KQ, E, FIRST, DR>), g, b, lds, st, a.e_src, a.e_out, a.hi, a.lo, a.q, a.z, a.d,
                     a.p_prev, a.p_cur, a.p_stride, a.chunk_base, a.m, a.n_tiles, a.epoch, a.agg,
                     a.incl, a.need, a.lb_stats, a.bounds, a.count);
}

uint32_t scan_waves(uint32_t kq, uint32_t E, bool first, uint32_t n_tiles, uint32_t chunks, uint32_t wpb,
                    bool drows) {
  uint32_t b = 0;
  auto pick = [&](auto kqc) {
    constexpr int K = decltype(kqc)::value;
    if (E == 8)
      b = first ? scan_blocks_one<K, 8, true>(n_tiles, chunks, wpb)
                : (drows ? scan_blocks_one<K, 8, false, true>(n_tiles, chunks, wpb)
                         : scan_blocks_one<K, 8, false>(n_tiles, chunks, wpb));
    else
      b = first ? scan_blocks_one<K, 16, true>(n_tiles, chunks, wpb)
                : (drows ? scan_blocks_one<K, 16, false, true>(n_tiles, chunks, wpb)
                         : scan_blocks_one<K, 16, false>(n_tiles, chunks, wpb));
  };
  switch (kq) {
    case 4: pick(std::integral_constant<int, 4>{}); break;
    case 8: pick(std::integral_constant<int, 8>{}); break;
    case 12: pick(std::integral_constant<int, 12>{}); break;
    default: pick(std::integral_constant<int, 16>{}); break;
  }
  return b * wpb;
}

template <int KQ>
static bool scan_kq(const ScanArgs& a, bool first, uint32_t E, uint32_t chunks, uint32_t wpb,
                    hipStream_t st) {
  if (E == 8) {
    if (first) scan_one<KQ, 8, true>(a, chunks, wpb, st);
    else if (a.d) scan_one<KQ, 8, false, true>(a, chunks, wpb, st);
    else scan_one<KQ, 8, false>(a, chunks, wpb, st);
  } else if (E == 16) {
    if (first) scan_one<KQ, 16, true>(a, chunks, wpb, st);
    else if (a.d) scan_one<KQ, 16, false, true>(a, chunks, wpb, st);
    else scan_one<KQ, 16, false>(a, chunks, wpb, st);
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

// Blocks of the last-level launch (also the number of partial rows per chunk).
// With two chunks per wave the grid has a row per chunk pair.
template <int KQ>
static uint32_t top_blocks_kq(const TopArgs& a, bool first, uint32_t chunks, uint32_t wpb, uint32_t cpw) {
  const uint32_t waves = div_up(a.m, a.edges_per_wave);
  const size_t lds = (size_t)wpb * 16 * kLanes * 8;
  const void* kern = first ? (const void*)k_top<KQ, true> : (const void*)k_top<KQ, false>;
  if constexpr (KQ > 6) {
    if (cpw == 2 && !first) kern = (const void*)k_top<KQ, false, 2>;
  }
  const uint32_t rows = std::max(1u, cpw == 2 && !first ? chunks / 2 : chunks);
  const uint32_t fit = std::max(1u, resident_blocks(kern, 64 * wpb, lds) / rows);
  return std::min(div_up(waves, wpb), fit);
}

template <int KQ>
static bool top_kq(const TopArgs& a, bool first, uint32_t chunks, uint32_t wpb, uint32_t cpw, uint32_t blocks,
                   hipStream_t st) {
  const size_t lds = (size_t)wpb * 16 * kLanes * 8;
  dim3 b(64 * wpb);
  if (cpw == 2) {
    if constexpr (KQ > 6) {
      if (first || chunks % 2) return false;
      hipLaunchKernelGGL((k_top<KQ, false, 2>), dim3(blocks, chunks / 2), b, lds, st, a.e_src, a.hi, a.lo, a.q,
                         a.z, a.p_prev, a.p_stride, a.chunk_base, a.m, a.edges_per_wave, a.partial, a.count,
                         a.ticket);
      return true;
    }
    return false;
  }
  dim3 g(blocks, chunks);
  if (first)
    hipLaunchKernelGGL((k_top<KQ, true>), g, b, lds, st, a.e_src, a.hi, a.lo, a.q, a.z, a.p_prev,
                       a.p_stride, a.chunk_base, a.m, a.edges_per_wave, a.partial, a.count, a.ticket);
  else
    hipLaunchKernelGGL((k_top<KQ, false>), g, b, lds, st, a.e_src, a.hi, a.lo, a.q, a.z, a.p_prev,
                       a.p_stride, a.chunk_base, a.m, a.edges_per_wave, a.partial, a.count, a.ticket);
  return true;
}

uint32_t top_blocks(const TopArgs& a, bool first, uint32_t kq, uint32_t chunks, const Tuning& tu) {
  const uint32_t wpb = tu.top_waves_per_block, cpw = tu.chunks_per_wave;
  switch (kq) {
    case 4: return top_blocks_kq<4>(a, first, chunks, wpb, cpw);
    case 8: return top_blocks_kq<8>(a, first, chunks, wpb, cpw);
    case 12: return top_blocks_kq<12>(a, first, chunks, wpb, cpw);
    default: return top_blocks_kq<16>(a, first, chunks, wpb, cpw);
  }
}

hipError_t launch_top(const TopArgs& a, bool first_level, uint32_t kq, uint32_t chunks,
                      const Tuning& tu, hipStream_t st) {
  if (!a.m) return hipSuccess;
  const uint32_t wpb = tu.top_waves_per_block, cpw = tu.chunks_per_wave;
  const uint32_t blocks = top_blocks(a, first_level, kq, chunks, tu);
  bool ok = false;
  switch (kq) {
    case 4: ok = top_kq<4>(a, first_level, chunks, wpb, cpw, blocks, st); break;
    case 8: ok = top_kq<8>(a, first_level, chunks, wpb, cpw, blocks, st); break;
    case 12: ok = top_kq<12>(a, first_level, chunks, wpb, cpw, blocks, st); break;
    case 16: ok = top_kq<16>(a, first_level, chunks, wpb, cpw, blocks, st); break;
  }
  if (!ok) return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_top_fold, dim3(chunks), dim3(1024), 0, st, a.partial, blocks, a.chunk_base, a.it_begin,
                     a.it_end, a.fsum);
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
