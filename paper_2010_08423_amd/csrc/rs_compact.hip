// Per-level compacted edge lists of the plain path.
//
// A prefix level touches only the edges whose product reaches some window of
// the level above (flag bit 2) or whose slots such a window reads (bits 0 and
// 1); every other edge adds nothing to the running XOR and stores nothing,
// so skipping it leaves every window sum unchanged. The last level touches
// only edges with a non-empty window. Each level therefore gets the list of
// its kept edges, in edge order, with everything a tile reads laid out
// contiguously:
//   ce[j]    original edge id;
//   cslot[j] P slot of the edge (prefix levels);
//   chi[j]   window end slot (levels >= 3), or the edge's source (level 2);
//   clo[j]   window start slot (levels >= 3);
//   cflag[j] bits 0, 1, 2 of the level's flags, and bit 3 when a segment
//            starts between the previous kept edge and this one (the two
//            belong to different destinations), which is where the running
//            XOR restarts; the 64 entries past the list are 0;
//   cq[j]    the edge's product row z_{dst,j'} * y_{e,l-1} (kq entries), for
//            edges that form a product (written by k_compact_rows).
// The list lengths stay in device memory (count[y]); the level kernels read
// them, so no host round trip separates the setup from the levels.
//
// Level index y = l - 2 for l = 2..k; y = k - 2 is the last level (k >= 3).
#include "rs_level.h"

namespace rs {

// Kept edge e at level index y of a query with k levels (y < k - 2: flags of
// prefix level l = y + 2; y = k - 2: the last level).
__device__ __forceinline__ bool kept_at(const CompactArgs& a, uint32_t y, uint64_t e) {
  if (y + 2 == a.k) return a.hi[e] != a.lo[e];
  return (a.need[(uint64_t)y * a.need_stride + e] & 7u) != 0;
}

// Block totals of kept edges, 1024 edges per block (blockIdx.y = level index).
__global__ __launch_bounds__(256) void k_compact_count(CompactArgs a) {
  __shared__ uint32_t part[256];
  const uint32_t y = blockIdx.y;
  const uint64_t base = (uint64_t)blockIdx.x * kCostBlock + threadIdx.x * 4;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (base + i < a.m) c += kept_at(a, y, base + i);
  part[threadIdx.x] = c;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.bsum[(uint64_t)y * a.nb + blockIdx.x] = part[0];
}

// Writes the kept edges of each 1024-edge block at their list positions
// (block offset from boff plus the position inside the block), then the list
// length and the zero flags past the list.
__global__ __launch_bounds__(256) void k_compact_scatter(CompactArgs a) {
  __shared__ uint32_t part[256];
  const uint32_t y = blockIdx.y;
  const uint32_t l = y + 2;
  const bool top = l == a.k;
  const uint64_t base = (uint64_t)blockIdx.x * kCostBlock + threadIdx.x * 4;
  bool kp[4];
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    kp[i] = base + i < a.m && kept_at(a, y, base + i);
    c += kp[i];
  }
  part[threadIdx.x] = c;
  __syncthreads();
  for (uint32_t d = 1; d < 256; d <<= 1) {  // inclusive scan of the thread counts
    const uint32_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  const LevelList L = a.list(y);
  uint64_t p = (uint64_t)a.boff[(uint64_t)y * a.nb + blockIdx.x] + part[threadIdx.x] - c;
  const uint8_t* need = a.need + (uint64_t)y * a.need_stride;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!kp[i]) continue;
    const uint64_t e = base + i;
    L.ce[p] = (uint32_t)e;
    if (top) {
      L.chi[p] = a.hi[e];
      L.clo[p] = a.lo[e];
      L.cflag[p] = 4;
    } else {
      L.cslot[p] = a.e_out[e];
      if (l == 2) {
        L.chi[p] = a.e_src[e];
      } else {
        L.chi[p] = a.hi[e];
        L.clo[p] = a.lo[e];
      }
      L.cflag[p] = (uint8_t)(need[e] & 7u);
    }
    ++p;
  }
  if (blockIdx.x == 0) {
    const uint64_t last = (uint64_t)y * a.nb + a.nb - 1;
    const uint32_t total = a.boff[last] + a.bsum[last];
    if (threadIdx.x < kEdgePad) L.cflag[(uint64_t)total + threadIdx.x] = 0;
    if (threadIdx.x == 0) a.count[y] = total;
  }
}

// Restart bits of the prefix lists: entry j gets bit 3 when it is the first
// entry or its edge's destination differs from the previous entry's (a new
// segment, so the running XOR restarts). One thread per entry.
__global__ __launch_bounds__(256) void k_compact_restart(CompactArgs a) {
  const uint32_t y = blockIdx.y;
  const LevelList L = a.list(y);
  const uint32_t n = a.count[y];
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const uint32_t d = a.e_dst[L.ce[j]];
    if (j == 0 || a.e_dst[L.ce[j - 1]] != d) L.cflag[j] |= 8u;
  }
}

// Per compacted tile of E entries: its cost (a weight per tile and per
// product, the products being a population count of bit 2 over the tile's
// flag words; the flags past the list are 0) and the inclusive cost prefix
// within blocks of kCostBlock tiles (pre, bsum), as the run bounds need.
// Tiles past the list cost nothing.
template <int E>
__global__ __launch_bounds__(256) void k_compact_tiles(CompactArgs a, uint32_t tile_cost, uint32_t product_cost,
                                                       uint32_t store_cost, uint32_t tile_cost_first,
                                                       uint32_t product_cost_first,
                                                       uint32_t* __restrict__ pre, uint32_t* __restrict__ bsum,
                                                       uint32_t tiles_max) {
  __shared__ uint32_t part[256];
  const uint32_t y = blockIdx.y;
  const LevelList L = a.list(y);
  const uint32_t n = a.count[y];
  const uint32_t n_tiles = (n + E - 1) / E;
  const uint32_t t_base = blockIdx.x * kCostBlock + threadIdx.x * 4;
  uint32_t cost[4];
  uint32_t sum = 0;
  for (int jt = 0; jt < 4; ++jt) {
    const uint32_t t = t_base + jt;
    uint32_t cst = 0;
    if (t < n_tiles) {
      const uint32_t* wds = reinterpret_cast<const uint32_t*>(L.cflag + (uint64_t)t * E);
      uint32_t np = 0, ns = 0;
#pragma unroll
      for (int q = 0; q < E / 4; ++q) {
        np += __popc(wds[q] & 0x04040404u);  // products (bit 2)
        ns += __popc(wds[q] & 0x01010101u);  // stored slots (bit 0)
      }
      cst = y == 0 ? tile_cost_first + product_cost_first * np : tile_cost + product_cost * np + store_cost * ns;
    }
    sum += cst;
    cost[jt] = sum;
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < 256; d <<= 1) {
    const uint32_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  const uint32_t before = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  uint32_t* pl = pre + (uint64_t)y * tiles_max;
  for (int jt = 0; jt < 4; ++jt)
    if (t_base + jt < tiles_max) pl[t_base + jt] = before + cost[jt];
  if (threadIdx.x == 255) bsum[(uint64_t)y * gridDim.x + blockIdx.x] = part[255];
}

// Work-balanced run bounds of the compacted prefix levels (one row of threads
// per level, the tile count read from the level's list length): run w starts
// at the first tile whose preceding cost reaches its share (run_bounds_of_tile).
template <int E>
__global__ __launch_bounds__(256) void k_compact_bounds(const uint32_t* __restrict__ count,
                                                        const uint32_t* __restrict__ pre,
                                                        const uint32_t* __restrict__ boff, uint32_t nb,
                                                        uint32_t tiles_max, uint32_t w_first, uint32_t w_second,
                                                        uint32_t w_rest, float skew_first, float skew_second,
                                                        float skew_rest, uint32_t b_stride,
                                                        uint32_t* __restrict__ bounds) {
  const uint32_t y = blockIdx.y;
  const uint32_t n_tiles = (count[y] + E - 1) / E;
  const uint32_t W = y == 0 ? w_first : (y == 1 ? w_second : w_rest);
  uint32_t* b = bounds + (uint64_t)y * b_stride;
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (n_tiles == 0) {  // an empty level: every run is empty
    if (t == 0)
      for (uint32_t w = 0; w <= W; ++w) b[w] = 0;
    return;
  }
  if (t < n_tiles)
    run_bounds_of_tile(pre + (uint64_t)y * tiles_max, boff + (uint64_t)y * nb, n_tiles, t, W, b,
                       y == 0 ? skew_first : (y == 1 ? skew_second : skew_rest));
}

// Product rows of the kept edges that form a product (bit 2; every entry of
// the last level): cq[j][i] = z_{dst,i} * y_{e,l-1}. A row of an edge that the
// query's constraints exclude is 0, so the edge contributes nothing.
// Grid-stride over the entries of every level.
template <int KQ>
__global__ __launch_bounds__(256) void k_compact_rows(CompactArgs a, const uint64_t* __restrict__ z, uint64_t seed_v,
                                                      const uint64_t* __restrict__ seed_p, EdgeFilter f,
                                                      uint32_t y_first) {
  const uint64_t seed = seed_p ? *seed_p : seed_v;  // from a batch descriptor, read at run time
  __shared__ uint64_t lds[4][16][kLanes];
  const uint32_t lane = threadIdx.x & 63u;
  uint64_t* tab = &lds[threadIdx.x >> 6][0][lane];
  tab[0] = 0;
  const uint32_t y = blockIdx.y + y_first;
  const uint32_t l = y + 2;
  const LevelList L = a.list(y);
  const uint32_t n = a.count[y];
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    if (!(L.cflag[j] & 4u)) continue;
    const uint32_t e = L.ce[j];
    const uint32_t src = a.e_src[e], dst = a.e_dst[e], t = a.e_t[e];
    uint64_t* out = L.cq + (uint64_t)j * KQ;
    if (edge_excluded(f, l, a.k, src, dst, t)) {
#pragma unroll
      for (int i = 0; i < KQ; ++i) out[i] = 0;
      continue;
    }
    const uint64_t yv = hash2(seed, 'Y', (uint64_t)src | ((uint64_t)dst << 32), (uint64_t)t | ((uint64_t)(l - 1) << 32));
    gf_table(tab, yv);
#pragma unroll
    for (int i = 0; i < KQ; ++i) {
      Acc128 r = {0, 0, 0, 0};
      gf_comb_acc(lds_addr(tab), z[(uint64_t)dst * KQ + i], r);
      out[i] = gf_reduce(r);
    }
  }
}

// Exclusive prefix of the block totals of each level (one block per level).
__global__ __launch_bounds__(1024) void k_compact_offsets(const uint32_t* __restrict__ bsum, uint32_t nb,
                                                          uint32_t* __restrict__ boff) {
  block_offsets(bsum + (uint64_t)blockIdx.x * nb, nb, boff + (uint64_t)blockIdx.x * nb);
}

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

hipError_t launch_compact(const CompactArgs& a, hipStream_t st) {
  if (!a.m || a.k < 3) return hipSuccess;
  const uint32_t levels = a.k - 1;
  hipLaunchKernelGGL(k_compact_count, dim3(a.nb, levels), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_compact_offsets, dim3(levels), dim3(1024), 0, st, a.bsum, a.nb, a.boff);
  hipLaunchKernelGGL(k_compact_scatter, dim3(a.nb, levels), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_compact_costs(const CompactArgs& a, uint32_t E, uint32_t tiles_max, uint32_t* pre, uint32_t* bsum,
                                uint32_t* boff, hipStream_t st) {
  if (!a.m || a.k < 3) return hipSuccess;
  const uint32_t levels = a.k - 2;  // prefix levels only
  const uint32_t nbt = cdiv(tiles_max, kCostBlock);
  hipLaunchKernelGGL(k_compact_restart, dim3(std::min<uint32_t>(cdiv(a.m, 256), 4096), levels), dim3(256), 0, st, a);
  if (E == 8)
    hipLaunchKernelGGL(k_compact_tiles<8>, dim3(nbt, levels), dim3(256), 0, st, a, kTileCost, kProductCost,
                       kStoreCost, kTileCostFirst, kProductCostFirst, pre, bsum, tiles_max);
  else
    hipLaunchKernelGGL(k_compact_tiles<16>, dim3(nbt, levels), dim3(256), 0, st, a, kTileCost, kProductCost,
                       kStoreCost, kTileCostFirst, kProductCostFirst, pre, bsum, tiles_max);
  hipLaunchKernelGGL(k_compact_offsets, dim3(levels), dim3(1024), 0, st, bsum, nbt, boff);
  return hipGetLastError();
}

hipError_t launch_compact_bounds(const CompactArgs& a, uint32_t E, uint32_t tiles_max, uint32_t w_first,
                                 uint32_t w_second, uint32_t w_rest, float skew_first, float skew_second,
                                 float skew_rest, uint32_t* pre, uint32_t* bsum, uint32_t* boff, uint32_t* bounds,
                                 uint32_t b_stride, hipStream_t st) {
  if (!a.m || a.k < 3) return hipSuccess;
  hipError_t err = launch_compact_costs(a, E, tiles_max, pre, bsum, boff, st);
  if (err != hipSuccess) return err;
  const uint32_t levels = a.k - 2;
  const uint32_t nbt = cdiv(tiles_max, kCostBlock);
  const dim3 g(cdiv((uint64_t)tiles_max + 1, 256), levels);
  if (E == 8)
    hipLaunchKernelGGL(k_compact_bounds<8>, g, dim3(256), 0, st, a.count, pre, boff, nbt, tiles_max, w_first, w_second,
                       w_rest, skew_first, skew_second, skew_rest, b_stride, bounds);
  else
    hipLaunchKernelGGL(k_compact_bounds<16>, g, dim3(256), 0, st, a.count, pre, boff, nbt, tiles_max, w_first,
                       w_second, w_rest, skew_first, skew_second, skew_rest, b_stride, bounds);
  return hipGetLastError();
}

hipError_t launch_compact_rows(const CompactArgs& a, const uint64_t* z, uint64_t seed, const uint64_t* seed_p,
                               const EdgeFilter& f, uint32_t kq, hipStream_t st, uint32_t y_first) {
  if (!a.m || a.k < 3 || y_first >= a.k - 1) return hipSuccess;
  const dim3 g(std::min<uint32_t>(cdiv(a.m, 256), 2048), a.k - 1 - y_first), b(256);
  switch (kq) {
    case 4: hipLaunchKernelGGL(k_compact_rows<4>, g, b, 0, st, a, z, seed, seed_p, f, y_first); break;
    case 8: hipLaunchKernelGGL(k_compact_rows<8>, g, b, 0, st, a, z, seed, seed_p, f, y_first); break;
    case 12: hipLaunchKernelGGL(k_compact_rows<12>, g, b, 0, st, a, z, seed, seed_p, f, y_first); break;
    case 16: hipLaunchKernelGGL(k_compact_rows<16>, g, b, 0, st, a, z, seed, seed_p, f, y_first); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rs

