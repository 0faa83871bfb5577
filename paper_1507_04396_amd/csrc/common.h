// Shared device helpers for the pMMF kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PMMF_WAVE 64

// SplitMix64 output finalizer (Steele, Lea & Flood, OOPSLA 2014).  The seed row of each greedy
// step and the cluster sizes are drawn from chains of it, so host and device agree bit for bit.
__host__ __device__ inline uint64_t pmmf_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// x <- mix64((x xor v) + golden ratio constant), for v = a, b, c, d in turn, from x = seed.
__host__ __device__ inline uint64_t pmmf_hash4(uint64_t seed, uint64_t a, uint64_t b, uint64_t c,
                                               uint64_t d) {
  const uint64_t g = 0x9E3779B97F4A7C15ull;
  uint64_t x = seed;
  x = pmmf_mix64((x ^ a) + g);
  x = pmmf_mix64((x ^ b) + g);
  x = pmmf_mix64((x ^ c) + g);
  x = pmmf_mix64((x ^ d) + g);
  return x;
}

// floor(x * n / 2^64): uniform index in [0, n) from a 64-bit hash (multiply-shift).
__host__ __device__ inline uint64_t pmmf_mulhi(uint64_t x, uint64_t n) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(x, n);
#else
  return (uint64_t)(((unsigned __int128)x * (unsigned __int128)n) >> 64);
#endif
}

constexpr uint64_t PMMF_TAG_SEED_ROW = 1;
constexpr uint64_t PMMF_TAG_CLUSTER_SIZE = 2;

__device__ inline int pmmf_lane() { return threadIdx.x & (PMMF_WAVE - 1); }
__device__ inline int pmmf_wave() { return threadIdx.x / PMMF_WAVE; }

// Workgroups of a launch are dispatched round robin over the eight XCDs, each with its own L2:
// workgroup b runs on XCD b % 8.  This renumbering gives each XCD one contiguous range of the
// n workgroups' work, taken in dispatch order, so that neighbouring work items share an L2.
__device__ inline int pmmf_xcd_block(int b, int n) {
  const int x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + i;
}

__device__ inline int pmmf_wave_sum_int(int v) {
  for (int o = PMMF_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline int pmmf_wave_min_int(int v) {
  for (int o = PMMF_WAVE / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ inline int pmmf_wave_max_int(int v) {
  for (int o = PMMF_WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double pmmf_wave_sum_double(double v) {
  for (int o = PMMF_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline float pmmf_wave_sum_float(float v) {
  for (int o = PMMF_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
// Sum over the 64 lanes through DPP row shifts (inclusive sums inside each row of 16 lanes) and
// the four row totals read back with readlane: no LDS traffic.  Every lane must be active; all
// lanes receive the same result.
template <int CTRL>
__device__ inline float pmmf_dpp_row_shr(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                               0xf, 0xf, false));
}
__device__ inline float pmmf_wave_sum_dpp(float v) {
  v += pmmf_dpp_row_shr<0x111>(v);
  v += pmmf_dpp_row_shr<0x112>(v);
  v += pmmf_dpp_row_shr<0x114>(v);
  v += pmmf_dpp_row_shr<0x118>(v);
  const int b = __builtin_bit_cast(int, v);
  return (__builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 15)) +
          __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 31))) +
         (__builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 47)) +
          __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 63)));
}
__device__ inline float pmmf_readlane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// inclusive prefix sum over the lanes of a wave
__device__ inline int pmmf_wave_incl_scan(int v) {
  const int lane = pmmf_lane();
  for (int o = 1; o < PMMF_WAVE; o <<= 1) {
    int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// inclusive prefix sum over the lanes of a wave through DPP (row shifts inside rows of 16, then
// the row totals broadcast into the following rows): no LDS traffic.  Every lane must be active.
__device__ inline int pmmf_wave_incl_scan_dpp(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
  return v;
}

// inclusive maximum over the lanes of a wave through DPP, for values >= -1 (-1 is the identity);
// same shifts and broadcasts as the prefix sum above.  Every lane must be active.
__device__ inline int pmmf_wave_incl_max_dpp(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return v;
}

// position of the n-th (0-based) set bit of m, n < popcount(m): binary search on popcounts
__device__ inline int pmmf_nth_bit(uint32_t m, int n) {
  int pos = 0;
#pragma unroll
  for (int w = 16; w > 0; w >>= 1) {
    const uint32_t lo = m & ((1u << w) - 1u);
    const int pc = __popc(lo);
    const bool up = n >= pc;
    n -= up ? pc : 0;
    m = up ? (m >> w) : lo;
    pos += up ? w : 0;
  }
  return pos;
}

// Number of set bits of a 64-bit ballot below this lane.
__device__ inline int pmmf_lanes_below(uint64_t mask) {
  const int lane = pmmf_lane();
  uint64_t below = lane == 0 ? 0ull : (mask & ((~0ull) >> (64 - lane)));
  return __popcll(below);
}
