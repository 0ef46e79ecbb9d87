// Graph upload: validation, dedupe, (dst, t, src) ordering and window indices,
// all on the device.
//
// A directed temporal graph is a SET of triples (u, v, j), j >= 1 (Sec. 2), so
// repeated triples collapse to one; self-loops are dropped (they lie on no
// path, and every walk through one cancels in the sieve). The kept edges are
// sorted by (dst, t, src): the in-edges of a vertex then form a time-ordered
// segment, which is what the per-level prefix XOR and the restless window
// need.
#include <string.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <new>

#include "rs_internal.h"

namespace rs {

__global__ void k_validate(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                           const uint32_t* __restrict__ t, uint64_t m, uint32_t n,
                           uint32_t* __restrict__ stats /* [0]=err [1]=tmin [2]=tmax */,
                           unsigned long long* __restrict__ loops) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t s = src[i], d = dst[i], ti = t[i];
  if (s >= n || d >= n || ti < 1) atomicOr(&stats[0], 1u);
  if (s == d) atomicAdd(loops, 1ull);
  atomicMin(&stats[1], ti);
  atomicMax(&stats[2], ti);
}

__global__ void k_iota(uint32_t* __restrict__ p, uint64_t m) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = (uint32_t)i;
}

// key2[i] = dst << 32 | t of the edge perm[i].
__global__ void k_key2(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ dst,
                       const uint32_t* __restrict__ t, uint64_t* __restrict__ key, uint64_t m) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    const uint32_t e = perm[i];
    key[i] = ((uint64_t)dst[e] << 32) | t[e];
  }
}

// keep[i] = not a self-loop and not equal to the previous sorted triple.
__global__ void k_mark(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ src,
                       const uint64_t* __restrict__ key, uint32_t* __restrict__ keep, uint64_t m) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t s = src[perm[i]];
  const uint32_t d = (uint32_t)(key[i] >> 32);
  bool k = s != d;
  if (k && i > 0) k = !(key[i] == key[i - 1] && src[perm[i - 1]] == s);
  keep[i] = k ? 1u : 0u;
}

__global__ void k_scatter(const uint32_t* __restrict__ perm, const uint32_t* __restrict__ src,
                          const uint64_t* __restrict__ key, const uint32_t* __restrict__ keep,
                          const uint32_t* __restrict__ pos, uint32_t* __restrict__ o_src,
                          uint32_t* __restrict__ o_dst, uint32_t* __restrict__ o_t, uint64_t m) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m || !keep[i]) return;
  const uint32_t p = pos[i];
  o_src[p] = src[perm[i]];
  o_dst[p] = (uint32_t)(key[i] >> 32);
  o_t[p] = (uint32_t)key[i];
}

// in_off[u] = first edge with dst >= u, u in [0, n].
__global__ void k_in_off(const uint32_t* __restrict__ e_dst, uint32_t m, uint32_t n,
                         uint32_t* __restrict__ in_off) {
  const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u > n) return;
  uint32_t a = 0, b = m;
  while (a < b) {
    const uint32_t mid = a + ((b - a) >> 1);
    if (e_dst[mid] < u)
      a = mid + 1;
    else
      b = mid;
  }
  in_off[u] = a;
}

// hi(e): slot just past the last arrival at v = src(e) with time <= t(e);
// e_out(e): slot holding the prefix through e.
__global__ void k_hi(const uint32_t* __restrict__ e_src, const uint32_t* __restrict__ e_dst,
                     const uint32_t* __restrict__ e_t, const uint32_t* __restrict__ in_off,
                     uint32_t* __restrict__ hi, uint32_t* __restrict__ e_out, uint32_t m,
                     uint32_t* __restrict__ max_deg) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint32_t v = e_src[e], t = e_t[e];
  uint32_t a = in_off[v], b = in_off[v + 1];
  while (a < b) {
    const uint32_t mid = a + ((b - a) >> 1);
    if (e_t[mid] <= t)
      a = mid + 1;
    else
      b = mid;
  }
  hi[e] = a + v;
  const uint32_t u = e_dst[e];
  e_out[e] = (uint32_t)e + u + 1u;
  if (e == in_off[u]) atomicMax(max_deg, in_off[u + 1] - in_off[u]);
}

static inline uint32_t grid_for(uint64_t n, uint32_t b = 256) { return (uint32_t)((n + b - 1) / b); }

// Temporary device buffers of one upload; released on every exit path.
struct UploadTemps {
  DevBuf in_src, in_dst, in_t, stats, loops, perm_a, perm_b, key_a, key_b, k1a, k1b, keep, pos, tmp;
  ~UploadTemps() {
    for (DevBuf* b : {&in_src, &in_dst, &in_t, &stats, &loops, &perm_a, &perm_b, &key_a, &key_b, &k1a, &k1b, &keep,
                      &pos, &tmp})
      b->release();
  }
};

// Fills g (already allocated) from the input edges; on failure the caller
// destroys g.
static rs_status graph_fill(rs_graph* g, uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                            const uint32_t* t, const uint8_t* colour, uint32_t n_colours, bool host_ptrs,
                            hipStream_t st) {
  RS_HIP(hipGetDevice(&g->device));
  GraphDev& G = g->g;
  G.n = n;
  G.n_colours = n_colours;
  UploadTemps T;
  DevBuf &in_src = T.in_src, &in_dst = T.in_dst, &in_t = T.in_t, &stats = T.stats, &loops = T.loops,
         &perm_a = T.perm_a, &perm_b = T.perm_b, &key_a = T.key_a, &key_b = T.key_b, &k1a = T.k1a, &k1b = T.k1b,
         &keep = T.keep, &pos = T.pos, &tmp = T.tmp;

  // Inputs on the device.
  const uint32_t *d_src = src, *d_dst = dst, *d_t = t;
  const size_t mb = (size_t)std::max<uint64_t>(m, 1);
  if (host_ptrs && m) {
    if (in_src.reserve(mb * 4, st, false) || in_dst.reserve(mb * 4, st, false) ||
        in_t.reserve(mb * 4, st, false)) return RS_ENOMEM;
    RS_HIP(hipMemcpyAsync(in_src.p, src, m * 4, hipMemcpyHostToDevice, st));
    RS_HIP(hipMemcpyAsync(in_dst.p, dst, m * 4, hipMemcpyHostToDevice, st));
    RS_HIP(hipMemcpyAsync(in_t.p, t, m * 4, hipMemcpyHostToDevice, st));
    d_src = in_src.as<uint32_t>();
    d_dst = in_dst.as<uint32_t>();
    d_t = in_t.as<uint32_t>();
  }
  if (stats.reserve(16, st) || loops.reserve(8, st)) return RS_ENOMEM;
  uint32_t init[4] = {0, 0xFFFFFFFFu, 0, 0};
  RS_HIP(hipMemcpyAsync(stats.p, init, 16, hipMemcpyHostToDevice, st));
  if (m) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(m)), dim3(256), 0, st, d_src, d_dst, d_t, m, n,
                       stats.as<uint32_t>(), loops.as<unsigned long long>());
    RS_HIP(hipGetLastError());
  }
  uint32_t hstats[4];
  unsigned long long hloops = 0;
  RS_HIP(hipMemcpyAsync(hstats, stats.p, 16, hipMemcpyDeviceToHost, st));
  RS_HIP(hipMemcpyAsync(&hloops, loops.p, 8, hipMemcpyDeviceToHost, st));
  RS_HIP(hipStreamSynchronize(st));
  if (hstats[0]) return RS_EINVAL;

  uint64_t mk = 0;
  if (m) {
    // Pass 1: order by src; pass 2 (stable): order by (dst, t).
    if (perm_a.reserve(mb * 4, st, false) || perm_b.reserve(mb * 4, st, false) ||
        key_a.reserve(mb * 8, st, false) || key_b.reserve(mb * 8, st, false) ||
        k1a.reserve(mb * 4, st, false) || k1b.reserve(mb * 4, st, false) ||
        keep.reserve(mb * 4, st, false) || pos.reserve(mb * 4, st, false)) return RS_ENOMEM;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(m)), dim3(256), 0, st, perm_a.as<uint32_t>(), m);
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(k1a.p, d_src, m * 4, hipMemcpyDeviceToDevice, st));
    unsigned nbits = 1;
    while (nbits < 32 && (1ull << nbits) < n) ++nbits;
    size_t need1 = 0, need2 = 0, need3 = 0;
    RS_HIP(rocprim::radix_sort_pairs(nullptr, need1, k1a.as<uint32_t>(), k1b.as<uint32_t>(),
                                     perm_a.as<uint32_t>(), perm_b.as<uint32_t>(), (size_t)m, 0, nbits, st));
    RS_HIP(rocprim::radix_sort_pairs(nullptr, need2, key_a.as<uint64_t>(), key_b.as<uint64_t>(),
                                     perm_b.as<uint32_t>(), perm_a.as<uint32_t>(), (size_t)m, 0, 32 + nbits, st));
    RS_HIP(rocprim::exclusive_scan(nullptr, need3, keep.as<uint32_t>(), pos.as<uint32_t>(), 0u, (size_t)m,
                                   rocprim::plus<uint32_t>(), st));
    if (tmp.reserve(std::max(need1, std::max(need2, need3)) + 256, st, false)) return RS_ENOMEM;
    size_t sz = tmp.bytes;
    RS_HIP(rocprim::radix_sort_pairs(tmp.p, sz, k1a.as<uint32_t>(), k1b.as<uint32_t>(),
                                     perm_a.as<uint32_t>(), perm_b.as<uint32_t>(), (size_t)m, 0, nbits, st));
    hipLaunchKernelGGL(k_key2, dim3(grid_for(m)), dim3(256), 0, st, perm_b.as<uint32_t>(), d_dst, d_t,
                       key_a.as<uint64_t>(), m);
    RS_HIP(hipGetLastError());
    sz = tmp.bytes;
    RS_HIP(rocprim::radix_sort_pairs(tmp.p, sz, key_a.as<uint64_t>(), key_b.as<uint64_t>(),
                                     perm_b.as<uint32_t>(), perm_a.as<uint32_t>(), (size_t)m, 0, 32 + nbits, st));
    hipLaunchKernelGGL(k_mark, dim3(grid_for(m)), dim3(256), 0, st, perm_a.as<uint32_t>(), d_src,
                       key_b.as<uint64_t>(), keep.as<uint32_t>(), m);
    RS_HIP(hipGetLastError());
    sz = tmp.bytes;
    RS_HIP(rocprim::exclusive_scan(tmp.p, sz, keep.as<uint32_t>(), pos.as<uint32_t>(), 0u, (size_t)m,
                                   rocprim::plus<uint32_t>(), st));
    uint32_t last_pos = 0, last_keep = 0;
    RS_HIP(hipMemcpyAsync(&last_pos, pos.as<uint32_t>() + (m - 1), 4, hipMemcpyDeviceToHost, st));
    RS_HIP(hipMemcpyAsync(&last_keep, keep.as<uint32_t>() + (m - 1), 4, hipMemcpyDeviceToHost, st));
    RS_HIP(hipStreamSynchronize(st));
    mk = (uint64_t)last_pos + last_keep;
    const size_t kb = (size_t)std::max<uint64_t>(mk, 1) + kEdgePad;
    if (G.e_src.reserve(kb * 4, st, false) || G.e_dst.reserve(kb * 4, st, false) ||
        G.e_t.reserve(kb * 4, st, false) || G.e_out.reserve(kb * 4, st, false) ||
        G.hi.reserve(kb * 4, st, false)) return RS_ENOMEM;
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(m)), dim3(256), 0, st, perm_a.as<uint32_t>(), d_src,
                       key_b.as<uint64_t>(), keep.as<uint32_t>(), pos.as<uint32_t>(),
                       G.e_src.as<uint32_t>(), G.e_dst.as<uint32_t>(), G.e_t.as<uint32_t>(), m);
    RS_HIP(hipGetLastError());
  }
  G.m = mk;
  if (G.in_off.reserve(((size_t)n + 1) * 4, st, true)) return RS_ENOMEM;
  uint32_t max_deg = 0;
  if (mk) {
    hipLaunchKernelGGL(k_in_off, dim3(grid_for((uint64_t)n + 1)), dim3(256), 0, st,
                       G.e_dst.as<uint32_t>(), (uint32_t)mk, n, G.in_off.as<uint32_t>());
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemsetAsync(stats.p, 0, 4, st));
    hipLaunchKernelGGL(k_hi, dim3(grid_for(mk)), dim3(256), 0, st, G.e_src.as<uint32_t>(),
                       G.e_dst.as<uint32_t>(), G.e_t.as<uint32_t>(), G.in_off.as<uint32_t>(),
                       G.hi.as<uint32_t>(), G.e_out.as<uint32_t>(), (uint32_t)mk, stats.as<uint32_t>());
    RS_HIP(hipGetLastError());
    RS_HIP(hipMemcpyAsync(&max_deg, stats.p, 4, hipMemcpyDeviceToHost, st));
  }
  if (colour) {
    if (G.colour.reserve(std::max<size_t>(n, 1), st, false)) return RS_ENOMEM;
    RS_HIP(hipMemcpyAsync(G.colour.p, colour, n, host_ptrs ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
  }
  RS_HIP(hipStreamSynchronize(st));

  rs_graph_info& I = g->info;
  I.n = n;
  I.m_input = m;
  I.m = mk;
  I.self_loops = hloops;
  I.duplicates = m - hloops - mk;
  I.t_min = mk ? hstats[1] : 0;
  I.t_max = mk ? hstats[2] : 0;
  I.n_colours = n_colours;
  I.max_in_degree = max_deg;
  I.device_bytes = G.e_src.bytes + G.e_dst.bytes + G.e_t.bytes + G.e_out.bytes + G.hi.bytes +
                   G.in_off.bytes + G.colour.bytes;
  return RS_OK;
}


rs_status graph_build(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst,
                      const uint32_t* t, const uint8_t* colour, uint32_t n_colours, bool host_ptrs,
                      hipStream_t st, rs_graph** out) {
  if (!out || (m && (!src || !dst || !t))) return RS_EINVAL;
  if (n >= (1u << 31) || (uint64_t)m + n >= (1ull << 32)) return RS_EINVAL;
  if ((colour == nullptr) != (n_colours == 0) || n_colours > RS_MAX_COLOURS) return RS_EINVAL;
  rs_graph* g = new (std::nothrow) rs_graph();
  if (!g) return RS_ENOMEM;
  const rs_status s = graph_fill(g, n, m, src, dst, t, colour, n_colours, host_ptrs, st);
  if (s != RS_OK) {
    rs_graph_destroy(g);
    return s;
  }
  *out = g;
  return RS_OK;
}

}  // namespace rs
