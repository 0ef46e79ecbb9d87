// Random-row bandwidth probe: what MI355X delivers for the prefix state's
// access pattern (whole 512-byte rows at random rows of a large array), the
// practical ceiling against which the level kernels' HBM traffic is read.
// Not part of the sieve.
#include "rs_level.h"

namespace rs {

constexpr int kProbeRows = 16;  // rows each wave has in flight per step

// Row g of step s of wave w: a hash, masked to the power-of-two row count.
__device__ __forceinline__ uint64_t probe_row(uint64_t w, uint32_t s, uint32_t g, uint64_t mask) {
  return mix64((w << 32) ^ ((uint64_t)s << 8) ^ g ^ 0x9E3779B97F4A7C15ull) & mask;
}

// MODE 0: kProbeRows random row reads per step, XORed into the wave's row of
// `out`; MODE 1: as many random row writes; MODE 2: kProbeRows reads and
// kProbeRows / 2 writes per step. Rows are read and written with the
// non-temporal hint, as the prefix levels do.
template <int MODE>
__global__ __launch_bounds__(256) void k_probe_rows(uint64_t* __restrict__ rows, uint64_t mask,
                                                    uint64_t* __restrict__ out, uint32_t steps) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint64_t acc = 0;
  for (uint32_t s = 0; s < steps; ++s) {
    if constexpr (MODE != 1) {
      uint64_t v[kProbeRows];
#pragma unroll
      for (int g = 0; g < kProbeRows; ++g) v[g] = p_load(rows + probe_row(w, s, g, mask) * kLanes + lane);
#pragma unroll
      for (int g = 0; g < kProbeRows; ++g) acc ^= v[g];
    }
    if constexpr (MODE != 0) {
      constexpr int kW = MODE == 1 ? kProbeRows : kProbeRows / 2;
#pragma unroll
      for (int g = 0; g < kW; ++g) p_store(rows + probe_row(w, s, 64 + g, mask) * kLanes + lane, acc ^ (uint64_t)g);
    }
  }
  out[w * kLanes + lane] = acc;
}

}  // namespace rs

extern "C" rs_status rs_probe_rows(uint64_t* rows, uint64_t n_rows, uint64_t* out, uint32_t waves, uint32_t steps,
                                   uint32_t mode, void* hip_stream) {
  using namespace rs;
  if (!rows || !out || waves == 0 || waves % 4 || n_rows == 0 || (n_rows & (n_rows - 1)) || mode > 2)
    return RS_EINVAL;
  if (steps == 0) return RS_OK;
  const hipStream_t st = (hipStream_t)hip_stream;
  const dim3 g(waves / 4), b(256);
  const uint64_t mask = n_rows - 1;
  switch (mode) {
    case 0: hipLaunchKernelGGL(k_probe_rows<0>, g, b, 0, st, rows, mask, out, steps); break;
    case 1: hipLaunchKernelGGL(k_probe_rows<1>, g, b, 0, st, rows, mask, out, steps); break;
    default: hipLaunchKernelGGL(k_probe_rows<2>, g, b, 0, st, rows, mask, out, steps); break;
  }
  return hipGetLastError() == hipSuccess ? RS_OK : RS_EDEVICE;
}
