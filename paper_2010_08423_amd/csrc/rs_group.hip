// The last level by distinct windows.
//
// The last level sums c_k(e) = (XOR_{j in L} q_j(e)) * W(e) over its entries,
// with W(e) = P[hi(e)] ^ P[lo(e)]: entries with the same window slots (hi, lo)
// share W, so their sum is (XOR_{j in L} Q_j) * W with Q_j the XOR of their
// q_j rows, which does not depend on L. The entries of the last level's list
// are sorted by (hi, lo) once per query and their rows summed per group; the
// last level then runs over the groups: one pair of gathers and one product
// per distinct window instead of per edge. (On the 10^7-edge motif query the
// 3.8 million last-level entries have 2.1 million distinct windows.)
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "rs_internal.h"

namespace rs {

static inline uint32_t gblocks(uint64_t count, uint32_t per) { return (uint32_t)((count + per - 1) / per); }

__global__ void k_group_keys(const uint32_t* __restrict__ hi, const uint32_t* __restrict__ lo,
                             const uint32_t* __restrict__ count, uint64_t* __restrict__ key,
                             uint32_t* __restrict__ idx) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *count) return;
  key[j] = ((uint64_t)hi[j] << 32) | lo[j];
  idx[j] = j;
}

// head[j] = 1 where a new (hi, lo) starts in the sorted order.
__global__ void k_group_heads(const uint64_t* __restrict__ key, const uint32_t* __restrict__ count,
                              uint32_t* __restrict__ head) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *count) return;
  head[j] = (j == 0 || key[j] != key[j - 1]) ? 1u : 0u;
}

// gid = inclusive prefix of the heads: the group of sorted position j is
// gid[j] - 1. Group starts, window slots, and the group count.
__global__ void k_group_starts(const uint64_t* __restrict__ key, const uint32_t* __restrict__ gid,
                               const uint32_t* __restrict__ count, uint32_t* __restrict__ gstart,
                               uint32_t* __restrict__ ghi, uint32_t* __restrict__ glo,
                               uint32_t* __restrict__ gcount) {
  const uint32_t n = *count;
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (j == 0 || gid[j] != gid[j - 1]) {
    const uint32_t g = gid[j] - 1;
    gstart[g] = j;
    ghi[g] = (uint32_t)(key[j] >> 32);
    glo[g] = (uint32_t)key[j];
  }
  if (j == n - 1) {
    *gcount = gid[j];
    gstart[gid[j]] = n;
  }
}

// Row of each group: XOR of its members' q rows (one thread per group entry).
__global__ void k_group_rows(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ gcount,
                             const uint32_t* __restrict__ idx, const uint64_t* __restrict__ q, uint32_t kq,
                             uint64_t* __restrict__ gq) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t g = i / kq, jj = i % kq;
  if (g >= *gcount) return;
  uint64_t acc = 0;
  for (uint32_t p = gstart[g]; p < gstart[g + 1]; ++p) acc ^= q[(uint64_t)idx[p] * kq + jj];
  gq[g * kq + jj] = acc;
}

static uint32_t key_bits(uint64_t slots) {
  uint32_t b = 1;
  while (b < 32 && (1ull << b) <= slots) ++b;
  return 32 + b;
}

uint64_t group_temp_bytes(uint64_t m, uint64_t n) {
  size_t a = 0, b = 0;
  (void)rocprim::radix_sort_pairs(nullptr, a, (uint64_t*)nullptr, (uint64_t*)nullptr, (uint32_t*)nullptr,
                                  (uint32_t*)nullptr, (size_t)std::max<uint64_t>(m, 1), 0, key_bits(m + n));
  (void)rocprim::inclusive_scan(nullptr, b, (uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)std::max<uint64_t>(m, 1),
                                rocprim::plus<uint32_t>());
  return std::max<uint64_t>(a, b) + 256;
}

uint64_t group_bytes(uint64_t m, uint64_t n, uint32_t kq) {
  const uint64_t e = m + kEdgePad;
  // keys in/out, indices in/out, heads/gid, starts, ghi, glo, rows, count, sort temp
  return 8 * e * 2 + 4 * e * 2 + 4 * e * 2 + 4 * (e + 1) + 4 * e * 2 + 8 * e * kq + 256 + group_temp_bytes(m, n);
}

GroupView group_view(uint8_t* buf, uint64_t m, uint32_t kq) {
  const uint64_t e = m + kEdgePad;
  GroupView v;
  uint8_t* p = buf;
  auto take = [&](uint64_t bytes) {
    uint8_t* r = p;
    p += (bytes + 255) & ~255ull;
    return r;
  };
  v.key_in = (uint64_t*)take(8 * e);
  v.key_out = (uint64_t*)take(8 * e);
  v.idx_in = (uint32_t*)take(4 * e);
  v.idx_out = (uint32_t*)take(4 * e);
  v.head = (uint32_t*)take(4 * e);
  v.gid = (uint32_t*)take(4 * e);
  v.gstart = (uint32_t*)take(4 * (e + 1));
  v.ghi = (uint32_t*)take(4 * e);
  v.glo = (uint32_t*)take(4 * e);
  v.gq = (uint64_t*)take(8 * e * kq);
  v.gcount = (uint32_t*)take(256);
  v.temp = p;
  return v;
}

hipError_t launch_group(const LevelList& Lk, const uint32_t* count, uint32_t n_entries, uint64_t slots, uint32_t kq,
                        const GroupView& v, uint64_t temp_bytes, hipStream_t st) {
  if (!n_entries) return launch_fill32(v.gcount, 0, 1, st);
  const uint32_t g = gblocks(n_entries, 256);
  hipLaunchKernelGGL(k_group_keys, dim3(g), dim3(256), 0, st, Lk.chi, Lk.clo, count, v.key_in, v.idx_in);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t tb = temp_bytes;
  e = rocprim::radix_sort_pairs(v.temp, tb, v.key_in, v.key_out, v.idx_in, v.idx_out, (size_t)n_entries, 0,
                                key_bits(slots), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_heads, dim3(g), dim3(256), 0, st, v.key_out, count, v.head);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  tb = temp_bytes;
  e = rocprim::inclusive_scan(v.temp, tb, v.head, v.gid, (size_t)n_entries, rocprim::plus<uint32_t>(), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_starts, dim3(g), dim3(256), 0, st, v.key_out, v.gid, count, v.gstart, v.ghi, v.glo,
                     v.gcount);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_group_rows, dim3(gblocks((uint64_t)n_entries * kq, 256)), dim3(256), 0, st, v.gstart,
                     v.gcount, v.idx_out, Lk.cq, kq, v.gq);
  return hipGetLastError();
}

}  // namespace rs
