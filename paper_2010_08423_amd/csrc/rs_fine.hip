// Fine-grained outputs of the sieve (Alg. 1, FineGrainedOracle; Sec. 4.5):
// instead of one sum over every end vertex and end time, the last level's
// values are summed over the iterations L per slot (u, i), giving
// zeta_{u,k,i}; zeta_{u,k,i} != 0 says a restless path with k vertices ends at
// u at time i. R_u is the least such i and D the vertices that have one.
//
// The last level keeps, per edge e = (v -> u, i), T(e) = XOR over the
// iterations of the range of c_k(e): each wave forms c_k(e) for one edge in
// its 64 lanes (one iteration each), XORs the lanes together and adds the
// result into T(e) (one atomic XOR per edge and chunk). The edges of a slot
// (u, i) are consecutive in the (dst, t, src) order, so zeta_{u,k,i} is the
// XOR of T over that run of edges, formed by the slot kernel, which also
// lowers R_u.
#include "rs_level.h"

namespace rs {

// XOR of v over the 64 lanes of the wave (every lane receives it).
__device__ __forceinline__ uint64_t wave_xor(uint64_t v) {
  uint32_t lo = lo32(v), hi = hi32(v);
#pragma unroll
  for (int d = 1; d < kLanes; d <<= 1) {
    lo ^= (uint32_t)__shfl_xor((int)lo, d, kLanes);
    hi ^= (uint32_t)__shfl_xor((int)hi, d, kLanes);
  }
  return mk64(lo, hi);
}

// Last level k, per edge: T[e] ^= XOR over the lanes whose iteration lies in
// [it_begin, it_end) of c_k(e). One edge per wave step (grid-stride over the
// entries); an edge whose window is empty (levels >= 3) contributes zero.
// With a compacted list (count != null) entry j is edge ce[j], with its
// window slots and product row at j.
template <int KQ, bool FIRST>
__global__ __launch_bounds__(256) void k_top_fine(const uint32_t* __restrict__ e_src, const uint32_t* __restrict__ hi_idx,
                                                  const uint32_t* __restrict__ lo_idx, const uint64_t* __restrict__ q,
                                                  const uint64_t* __restrict__ z, const uint64_t* __restrict__ p_prev,
                                                  uint64_t p_stride, uint64_t chunk_base, uint64_t it_begin,
                                                  uint64_t it_end, uint32_t m_max, uint64_t* __restrict__ T,
                                                  const uint32_t* __restrict__ count, const uint32_t* __restrict__ ce) {
  const uint32_t m = count ? __builtin_amdgcn_readfirstlane(*as_const(count)) : m_max;
  extern __shared__ uint64_t dyn_lds[];  // [waves][16][64]
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t nw = blockDim.x >> 6;
  uint64_t* tab = dyn_lds + wv * 16 * kLanes + lane;
  tab[0] = 0;
  const uint32_t chunk = blockIdx.y;
  const uint64_t cb = chunk_base + (uint64_t)chunk * kLanes;
  const bool in_range = cb + lane >= it_begin && cb + lane < it_end;
  uint32_t mk[6];
  lane_masks(lane, mk);
  const uint64_t* pp = p_prev + (uint64_t)chunk * p_stride;
  cu32* hs = as_const(hi_idx);
  cu32* ls = as_const(lo_idx);
  cu32* ss = as_const(e_src);
  const uint32_t waves = gridDim.x * nw;
  for (uint32_t e = blockIdx.x * nw + wv; e < m; e += waves) {
    uint64_t w;
    if (FIRST) {
      w = subset_xor<KQ>(as_const(z) + (uint64_t)ss[e] * KQ, cb, mk);
    } else {
      const uint32_t h = hs[e], l = ls[e];
      if (h == l) continue;  // empty window: c_k(e) = 0 (wave-uniform)
      w = p_load(pp + (uint64_t)h * kLanes + lane) ^ p_load(pp + (uint64_t)l * kLanes + lane);
    }
    const uint64_t aL = subset_xor<KQ>(as_const(q) + (uint64_t)e * KQ, cb, mk);
    uint64_t v = gf_mul(tab, aL, w);
    if (!in_range) v = 0;
    v = wave_xor(v);
    if (lane == 0 && v) atomicXor((unsigned long long*)&T[ce ? ce[e] : e], (unsigned long long)v);
  }
}

// Per slot (u, i) (a maximal run of edges with equal dst and t, starting at an
// edge e whose predecessor differs): zeta = XOR of T over the run, written
// to every edge of the run; a non-zero zeta lowers reach[u] to i.
__global__ __launch_bounds__(256) void k_fine_slots(const uint32_t* __restrict__ e_dst, const uint32_t* __restrict__ e_t,
                                                    const uint64_t* __restrict__ T, uint32_t m,
                                                    uint64_t* __restrict__ zeta, uint32_t* __restrict__ reach) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t u = e_dst[e], t = e_t[e];
  if (e > 0 && e_dst[e - 1] == u && e_t[e - 1] == t) return;  // not the first edge of its slot
  uint64_t acc = 0;
  uint64_t f = e;
  for (; f < m && e_dst[f] == u && e_t[f] == t; ++f) acc ^= T[f];
  for (uint64_t g = e; g < f; ++g) zeta[g] = acc;
  if (acc) atomicMin(&reach[u], t);
}

// Product rows [m][kq] of the one level of a k = 2 query with the query's
// constraints applied: the rows of the edges they exclude are cleared, so
// those edges contribute nothing (Sec. 3: paths from a source, paths to a
// destination; Sec. 4.7: removed vertices, a last time).
__global__ __launch_bounds__(256) void k_mask_rows(uint64_t* __restrict__ rows, const uint32_t* __restrict__ e_src,
                                                   const uint32_t* __restrict__ e_dst, const uint32_t* __restrict__ e_t,
                                                   EdgeFilter f, uint32_t m, uint32_t kq) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint64_t)m * kq) return;
  const uint64_t e = i / kq;
  if (edge_excluded(f, 2, 2, e_src[e], e_dst[e], e_t[e])) rows[i] = 0;
}

static inline uint32_t div_up32(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

template <int KQ>
static void top_fine_kq(const TopArgs& a, bool first, uint32_t chunks, uint32_t wpb, uint64_t* T, hipStream_t st) {
  const size_t lds = (size_t)wpb * 16 * kLanes * 8;
  const void* kern = first ? (const void*)k_top_fine<KQ, true> : (const void*)k_top_fine<KQ, false>;
  const uint32_t fit = std::max(1u, resident_blocks(kern, 64 * wpb, lds) / chunks);
  const uint32_t blocks = std::min(div_up32(a.m, wpb), fit);
  dim3 g(blocks, chunks), b(64 * wpb);
  if (first)
    hipLaunchKernelGGL((k_top_fine<KQ, true>), g, b, lds, st, a.e_src, a.hi, a.lo, a.q, a.z, a.p_prev, a.p_stride,
                       a.chunk_base, a.it_begin, a.it_end, a.m, T, a.count, a.ce);
  else
    hipLaunchKernelGGL((k_top_fine<KQ, false>), g, b, lds, st, a.e_src, a.hi, a.lo, a.q, a.z, a.p_prev, a.p_stride,
                       a.chunk_base, a.it_begin, a.it_end, a.m, T, a.count, a.ce);
}

hipError_t launch_top_fine(const TopArgs& a, bool first_level, uint32_t kq, uint32_t chunks, const Tuning& tu,
                           uint64_t* T, hipStream_t st) {
  if (!a.m) return hipSuccess;
  const uint32_t wpb = tu.top_waves_per_block;
  switch (kq) {
    case 4: top_fine_kq<4>(a, first_level, chunks, wpb, T, st); break;
    case 8: top_fine_kq<8>(a, first_level, chunks, wpb, T, st); break;
    case 12: top_fine_kq<12>(a, first_level, chunks, wpb, T, st); break;
    case 16: top_fine_kq<16>(a, first_level, chunks, wpb, T, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fine_slots(const uint32_t* e_dst, const uint32_t* e_t, const uint64_t* T, uint32_t m, uint64_t* zeta,
                             uint32_t* reach, hipStream_t st) {
  if (!m) return hipSuccess;
  hipLaunchKernelGGL(k_fine_slots, dim3(div_up32(m, 256)), dim3(256), 0, st, e_dst, e_t, T, m, zeta, reach);
  return hipGetLastError();
}

hipError_t launch_mask_rows(uint64_t* rows, const uint32_t* e_src, const uint32_t* e_dst, const uint32_t* e_t,
                            const EdgeFilter& f, uint32_t m, uint32_t kq, hipStream_t st) {
  const uint64_t count = (uint64_t)m * kq;
  if (!count) return hipSuccess;
  hipLaunchKernelGGL(k_mask_rows, dim3(div_up32(count, 256)), dim3(256), 0, st, rows, e_src, e_dst, e_t, f, m, kq);
  return hipGetLastError();
}

}  // namespace rs
