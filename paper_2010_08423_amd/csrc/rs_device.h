// Device-side building blocks of the sieve: GF(2^64) multiply on the VALU with
// a per-lane nibble table in LDS, the seed-keyed hash, and wave helpers.
//
// Field: GF(2^64) = GF(2)[x] / (x^64 + x^4 + x^3 + x + 1); bit i of a uint64 is
// the coefficient of x^i, addition is XOR (Sec. 4.2; b = 64 as in Sec. 5.1).
//
// gfx950 has no carry-less multiply instruction. A product a*w is formed as
//   1. table:  T[v] = v(x) * w mod p for the 16 polynomials v of degree < 4
//              (three doublings w*x, w*x^2, w*x^3 plus XOR combinations),
//              written to this lane's column of a [16][64] uint64 LDS array;
//   2. comb:   for nibble position j = 7..0 of both 32-bit halves a_0, a_1 of
//              a, XOR T[nibble_j(a_h)] into the 128-bit accumulator at dword h,
//              then shift the accumulator left by 4; the result is the
//              unreduced sum of T entries times x^(32h+4j), of degree <= 123;
//   3. reduce: with r = L + H x^64 (deg H <= 59), r = L + H (x^4+x^3+x+1),
//              which no longer overflows 64 bits.
// Step 3 is linear, so sums of unreduced products may be reduced once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kLanes = 64;

struct Acc128 {
  uint32_t d0, d1, d2, d3;
};

__device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }
__device__ __forceinline__ uint64_t mk64(uint32_t lo, uint32_t hi) {
  return ((uint64_t)hi << 32) | lo;
}

// 3-input XOR in one VALU op (gfx950 v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// (a & m) ^ c in one VALU op (truth table 0x6A).
__device__ __forceinline__ uint32_t and_xor(uint32_t a, uint32_t m, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, m, c, 0x6A);
}

typedef __attribute__((address_space(3))) uint64_t lds_u64;

// LDS byte address of a __shared__ location.
__device__ __forceinline__ uint32_t lds_addr(const uint64_t* p) {
  return (uint32_t)(uintptr_t)(const lds_u64*)p;
}
__device__ __forceinline__ uint64_t lds_load(uint32_t addr) {
  return *(const lds_u64*)(uintptr_t)addr;
}

// (hi:lo) >> s, low 32 bits.
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s) {
  return __builtin_amdgcn_alignbit(hi, lo, s);
}

// w * x mod p.
__device__ __forceinline__ void gf_times_x(uint32_t& lo, uint32_t& hi) {
  const uint32_t carry = (uint32_t)((int32_t)hi >> 31);
  hi = funnel(hi, lo, 31);
  lo = (lo << 1) ^ (carry & 0x1Bu);
}

// Writes T[1..15] of w into this lane's table column (tab = &lds[0][lane],
// row stride 64 entries). T[0] must hold 0.
__device__ __forceinline__ void gf_table(uint64_t* tab, uint64_t w) {
  uint32_t l1 = lo32(w), h1 = hi32(w);
  uint32_t l2 = l1, h2 = h1;
  gf_times_x(l2, h2);
  uint32_t l4 = l2, h4 = h2;
  gf_times_x(l4, h4);
  uint32_t l8 = l4, h8 = h4;
  gf_times_x(l8, h8);
  const uint64_t t1 = w, t2 = mk64(l2, h2), t4 = mk64(l4, h4), t8 = mk64(l8, h8);
  const uint64_t t3 = t1 ^ t2, t5 = t4 ^ t1, t6 = t4 ^ t2, t7 = t4 ^ t3;
  tab[1 * kLanes] = t1;
  tab[2 * kLanes] = t2;
  tab[3 * kLanes] = t3;
  tab[4 * kLanes] = t4;
  tab[5 * kLanes] = t5;
  tab[6 * kLanes] = t6;
  tab[7 * kLanes] = t7;
  tab[8 * kLanes] = t8;
  tab[9 * kLanes] = t8 ^ t1;  // entries combine at most two earlier ones
  tab[10 * kLanes] = t8 ^ t2;
  tab[11 * kLanes] = t8 ^ t3;
  tab[12 * kLanes] = t8 ^ t4;
  tab[13 * kLanes] = t8 ^ t5;
  tab[14 * kLanes] = t8 ^ t6;
  tab[15 * kLanes] = t8 ^ t7;
}

// Unreduced product of a with the tabled operand, XORed into r. The table
// column of this lane starts at LDS byte address `base`, entry v at
// base + v*512; bits 9..12 of base are zero, so the entry address is
// base | (v << 9).
__device__ __forceinline__ void gf_comb_acc(uint32_t base, uint64_t a, Acc128& r) {
  const uint32_t a0 = lo32(a), a1 = hi32(a);
  uint32_t d0 = 0, d1 = 0, d2 = 0, d3 = 0;
#pragma unroll
  for (int j = 7; j >= 0; --j) {
    const uint32_t s0 = (4 * j >= 9) ? (a0 >> (4 * j - 9)) : (a0 << (9 - 4 * j));
    const uint32_t s1 = (4 * j >= 9) ? (a1 >> (4 * j - 9)) : (a1 << (9 - 4 * j));
    // base has bits 9..12 clear, so OR equals XOR and the address takes one
    // three-input op after the shift
    const uint64_t x = lds_load(and_xor(s0, 0x1E00u, base));
    const uint64_t y = lds_load(and_xor(s1, 0x1E00u, base));
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

// r mod p for r of degree <= 123.
__device__ __forceinline__ uint64_t gf_reduce(const Acc128& r) {
  const uint32_t h0 = r.d2, h1 = r.d3;
  const uint32_t lo = xor3(xor3(r.d0, h0, h0 << 1), h0 << 3, h0 << 4);
  const uint32_t hi = xor3(xor3(r.d1, h1, funnel(h1, h0, 31)), funnel(h1, h0, 29), funnel(h1, h0, 28));
  return mk64(lo, hi);
}

// Full product a*w through this lane's table (overwrites the table).
__device__ __forceinline__ uint64_t gf_mul(uint64_t* tab, uint64_t a, uint64_t w) {
  gf_table(tab, w);
  Acc128 r = {0, 0, 0, 0};
  gf_comb_acc(lds_addr(tab), a, r);
  return gf_reduce(r);
}

// SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

// Keyed hash H(seed, tag, w0[, w1]): h = mix64(seed + tag*G), then
// h = mix64(h ^ (w + G)) per word.
__device__ __forceinline__ uint64_t hash1(uint64_t seed, uint64_t tag, uint64_t w0) {
  uint64_t h = mix64(seed + tag * kGolden);
  return mix64(h ^ (w0 + kGolden));
}
__device__ __forceinline__ uint64_t hash2(uint64_t seed, uint64_t tag, uint64_t w0, uint64_t w1) {
  uint64_t h = mix64(seed + tag * kGolden);
  h = mix64(h ^ (w0 + kGolden));
  return mix64(h ^ (w1 + kGolden));
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return mk64(__builtin_amdgcn_readfirstlane(lo32(v)), __builtin_amdgcn_readfirstlane(hi32(v)));
}

}  // namespace rs
