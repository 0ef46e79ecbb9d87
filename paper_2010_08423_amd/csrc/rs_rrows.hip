// Level 2 by iteration-independent prefix rows.
//
// At level 2 the window term is z^L_v itself (level 1 holds z^L at every time),
// so the prefix state of level 2 at the slot of edge e in u's segment is
//   P_2(e) = z^L_u * XOR_{e' <= e in the segment} y_{e',1} z^L_{src(e')}
//          = z^L_u * XOR_{j in L} R_j(e),  R_j(e) = XOR_{e' <= e} y_{e',1} z_{src(e'),j},
// and the level-3 window of an edge out of v, P_2[hi] ^ P_2[lo] over v's
// segment, is
//   z^L_v * XOR_{j in L} D_j,  D_j = R_j(hi) ^ R_j(lo)
// (a leading slot holds 0). R and D do not depend on L: they are formed once
// per query, k products per edge and a segmented XOR prefix over the edge
// list, after which level 2 needs no launch and level 3 forms each window
// from the D row of its entry and the z row of its source (two products per
// entry instead of two 512-byte gathers and one product).
//
// The prefix runs in three steps: per block of 4096 edges (16 per thread),
// local prefixes with the carries between the block's threads; the carries
// between blocks (one block, 256 threads); and, folded into the D rows, the
// block carry of every edge before its block's first segment start.
#include "rs_level.h"

namespace rs {

constexpr uint32_t kREdgesPerThread = 16;
constexpr uint32_t kRBlockEdges = 256 * kREdgesPerThread;

static inline uint32_t blocks_of(uint64_t count, uint64_t per) { return (uint32_t)((count + per - 1) / per); }

// Per block: R rows of its edges with the carries inside the block, and the
// block's summary: XOR of its trailing open segment part (btail [nb][KQ]),
// whether a segment starts in it (bhead), the offset of the first start
// (bfirst, kRBlockEdges if none).
// The product tables (8 KB per wave, at LDS offset 0) and, once the products
// are done, the threads' tail rows share one buffer.
struct RLocalShared {
  uint64_t buf[4 * 16 * kLanes];
  uint32_t heads[256], firsts[256];
};

// Only the terms of edges whose level-2 slot lies inside some level-3
// product window (level-2 flag bit 2) are formed: every other term cancels
// between the two ends of each window that is read.
template <int KQ>
__global__ __launch_bounds__(256) void k_r_local(const uint32_t* __restrict__ e_src, const uint32_t* __restrict__ e_dst,
                                                 const uint32_t* __restrict__ e_t, const uint8_t* __restrict__ need2,
                                                 const uint64_t* __restrict__ z, uint64_t seed_v,
                                                 const uint64_t* __restrict__ seed_p, EdgeFilter f,
                                                 uint32_t k, uint64_t m, uint64_t* __restrict__ R,
                                                 uint64_t* __restrict__ btail, uint32_t* __restrict__ bhead,
                                                 uint32_t* __restrict__ bfirst) {
  static_assert(256 * KQ <= 4 * 16 * kLanes, "tail rows fit the table buffer");
  const uint64_t seed = seed_p ? *seed_p : seed_v;  // from a batch descriptor, read at run time
  __shared__ RLocalShared sh;  // the only static LDS of the kernel, so it starts at address 0
  auto& heads = sh.heads;
  auto& firsts = sh.firsts;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  uint64_t* tab = sh.buf + wv * 16 * kLanes + lane;
  tab[0] = 0;
  const uint64_t e0 = (uint64_t)blockIdx.x * kRBlockEdges + (uint64_t)tid * kREdgesPerThread;
  uint64_t run[KQ];
#pragma unroll
  for (int j = 0; j < KQ; ++j) run[j] = 0;
  uint32_t has_head = 0, first = kREdgesPerThread;
  for (uint32_t i = 0; i < kREdgesPerThread && e0 + i < m; ++i) {
    const uint64_t e = e0 + i;
    const uint32_t src = e_src[e], dst = e_dst[e], t = e_t[e];
    if (e == 0 || e_dst[e - 1] != dst) {  // a segment (dst's in-edges) starts here
#pragma unroll
      for (int j = 0; j < KQ; ++j) run[j] = 0;
      if (!has_head) {
        has_head = 1;
        first = i;
      }
    }
    if (((need2[e] >> 2) & 1u) && !edge_excluded(f, 2, k, src, dst, t)) {
      gf_table(tab, hash2(seed, 'Y', (uint64_t)src | ((uint64_t)dst << 32), (uint64_t)t | (1ull << 32)));
#pragma unroll
      for (int j = 0; j < KQ; ++j) {
        Acc128 r = {0, 0, 0, 0};
        gf_comb_acc(lds_addr(tab), z[(uint64_t)src * KQ + j], r);
        run[j] ^= gf_reduce(r);
      }
    }
#pragma unroll
    for (int j = 0; j < KQ; ++j) R[e * KQ + j] = run[j];
  }
  __syncthreads();  // the tables are done with: the buffer holds the tails from here
  uint64_t(*tail)[KQ] = reinterpret_cast<uint64_t(*)[KQ]>(sh.buf);
#pragma unroll
  for (int j = 0; j < KQ; ++j) tail[tid][j] = run[j];
  heads[tid] = has_head;
  firsts[tid] = first;
  __syncthreads();
  if (tid < KQ) {  // column tid: the carry into each thread, in place of its tail
    uint64_t running = 0;
    for (uint32_t u = 0; u < 256; ++u) {
      const uint64_t v = tail[u][tid];
      tail[u][tid] = running;
      running = heads[u] ? v : running ^ v;
    }
    btail[(uint64_t)blockIdx.x * KQ + tid] = running;
  }
  if (tid == 64) {  // a wave other than the columns' one
    uint32_t bh = 0, bf = kRBlockEdges;
    for (uint32_t u = 0; u < 256 && !bh; ++u)
      if (heads[u]) {
        bh = 1;
        bf = u * kREdgesPerThread + firsts[u];
      }
    bhead[blockIdx.x] = bh;
    bfirst[blockIdx.x] = bf;
  }
  __syncthreads();
  bool any = false;
#pragma unroll
  for (int j = 0; j < KQ; ++j) any |= tail[tid][j] != 0;
  if (!any) return;
  for (uint32_t i = 0; i < first && e0 + i < m; ++i)  // edges before this thread's first segment start
#pragma unroll
    for (int j = 0; j < KQ; ++j) R[(e0 + i) * KQ + j] ^= tail[tid][j];
}

// The carry into every block (in place of btail): one block of 256 threads,
// each over a contiguous range of block summaries.
template <int KQ>
__global__ __launch_bounds__(256) void k_r_blocks(uint64_t* __restrict__ btail, const uint32_t* __restrict__ bhead,
                                                  uint32_t nb) {
  __shared__ uint64_t tail[256][KQ];
  __shared__ uint32_t heads[256];
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (nb + 255) / 256, b0 = min(tid * per, nb), b1 = min(b0 + per, nb);
  uint64_t run[KQ];
#pragma unroll
  for (int j = 0; j < KQ; ++j) run[j] = 0;
  uint32_t hh = 0;
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t h = bhead[b];
    hh |= h;
#pragma unroll
    for (int j = 0; j < KQ; ++j) run[j] = h ? btail[(uint64_t)b * KQ + j] : run[j] ^ btail[(uint64_t)b * KQ + j];
  }
#pragma unroll
  for (int j = 0; j < KQ; ++j) tail[tid][j] = run[j];
  heads[tid] = hh;
  __syncthreads();
  if (tid < KQ) {
    uint64_t running = 0;
    for (uint32_t u = 0; u < 256; ++u) {
      const uint64_t v = tail[u][tid];
      tail[u][tid] = running;
      running = heads[u] ? v : running ^ v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < KQ; ++j) run[j] = tail[tid][j];
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t h = bhead[b];
#pragma unroll
    for (int j = 0; j < KQ; ++j) {
      const uint64_t v = btail[(uint64_t)b * KQ + j];
      btail[(uint64_t)b * KQ + j] = run[j];  // carry into block b
      run[j] = h ? v : run[j] ^ v;
    }
  }
}

// R row of edge e, with its block's carry when e precedes the block's first
// segment start.
template <int KQ>
__device__ __forceinline__ uint64_t r_entry(const uint64_t* R, const uint64_t* bcarry, const uint32_t* bfirst,
                                            uint64_t e, int j) {
  const uint64_t b = e / kRBlockEdges;
  uint64_t v = R[e * KQ + j];
  if (e - b * kRBlockEdges < bfirst[b]) v ^= bcarry[b * KQ + j];
  return v;
}

// Level 3's entries: D rows of the product entries (bit 2), D_j = R_j(hi) ^
// R_j(lo) over the source's segment (its leading slot holds 0), written to
// d [entries][KQ]; and the source vertex of every entry, written over the
// list's window-end array, from which level 3 loads the source's z row.
template <int KQ>
__global__ __launch_bounds__(256) void k_r_drows(LevelList L3, const uint32_t* __restrict__ count3,
                                                 const uint32_t* __restrict__ e_src,
                                                 const uint32_t* __restrict__ in_off, const uint64_t* __restrict__ R,
                                                 const uint64_t* __restrict__ bcarry,
                                                 const uint32_t* __restrict__ bfirst, uint64_t* __restrict__ d) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *count3) return;
  const uint32_t v = e_src[L3.ce[j]];
  if (L3.cflag[j] & 4u) {
    const uint32_t lead = in_off[v] + v, hi = L3.chi[j], lo = L3.clo[j];
#pragma unroll
    for (int jj = 0; jj < KQ; ++jj) {
      uint64_t x = 0;
      if (hi != lead) x ^= r_entry<KQ>(R, bcarry, bfirst, (uint64_t)hi - v - 1, jj);
      if (lo != lead) x ^= r_entry<KQ>(R, bcarry, bfirst, (uint64_t)lo - v - 1, jj);
      d[j * KQ + jj] = x;
    }
  }
  L3.chi[j] = v;
}

uint64_t rrows_bytes(uint64_t m, uint32_t kq) {
  const uint64_t nb = (m + kRBlockEdges - 1) / kRBlockEdges;
  return 8ull * (m + kEdgePad) * kq + 8ull * nb * kq + 8ull * nb + 1024;
}

template <int KQ>
static hipError_t rrows_kq(const CompactArgs& ca, const uint32_t* in_off, const uint64_t* z, uint64_t seed,
                           const uint64_t* seed_p, const EdgeFilter& f, uint8_t* buf, hipStream_t st) {
  const uint64_t m = ca.m;
  const uint32_t nb = blocks_of(m, kRBlockEdges);
  uint64_t* R = (uint64_t*)buf;
  uint64_t* btail = R + (m + kEdgePad) * KQ;
  uint32_t* bhead = (uint32_t*)(btail + (uint64_t)nb * KQ);
  uint32_t* bfirst = bhead + nb;
  hipLaunchKernelGGL(k_r_local<KQ>, dim3(nb), dim3(256), 0, st, ca.e_src, ca.e_dst, ca.e_t, ca.need, z, seed, seed_p, f,
                     ca.k, m, R, btail, bhead, bfirst);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_r_blocks<KQ>, dim3(1), dim3(256), 0, st, btail, bhead, nb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const LevelList L3 = ca.list(1);
  hipLaunchKernelGGL(k_r_drows<KQ>, dim3(blocks_of(m, 256)), dim3(256), 0, st, L3, ca.count + 1, ca.e_src, in_off,
                     R, btail, bfirst, ca.list(0).cq);
  return hipGetLastError();
}

hipError_t launch_rrows(const CompactArgs& ca, const uint32_t* in_off, const uint64_t* z, uint64_t seed,
                        const uint64_t* seed_p, const EdgeFilter& f, uint32_t kq, uint8_t* buf, hipStream_t st) {
  if (!ca.m || ca.k < 4) return hipSuccess;
  switch (kq) {
    case 4: return rrows_kq<4>(ca, in_off, z, seed, seed_p, f, buf, st);
    case 8: return rrows_kq<8>(ca, in_off, z, seed, seed_p, f, buf, st);
    case 12: return rrows_kq<12>(ca, in_off, z, seed, seed_p, f, buf, st);
    case 16: return rrows_kq<16>(ca, in_off, z, seed, seed_p, f, buf, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rs
