// Counter-based random numbers for MoCHy-A+ sampling on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): per round, the two
// multiplier constants multiply counter words 0 and 2; the new state is
// (hi(w2*M1) ^ w1 ^ k0, lo(w2*M1), hi(w0*M0) ^ w3 ^ k1, lo(w0*M0)); the key
// advances by the two Weyl constants between rounds.
__device__ __forceinline__ uint4 philox_4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
  constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t h0 = __umulhi(kMul0, c.x), l0 = kMul0 * c.x;
    const uint32_t h1 = __umulhi(kMul1, c.z), l1 = kMul1 * c.z;
    c = make_uint4(h1 ^ c.y ^ k0, l1, h0 ^ c.w ^ k1, l0);
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return c;
}

// Hyperwedge index of sample n: floor(u * W / 2^64) with u = (x1 << 32) | x0
// of Philox4x32-10(counter (lo32 n, hi32 n, 0, 0), key (lo32 seed, hi32 seed)).
__device__ __forceinline__ uint64_t sample_wedge(uint64_t n, uint64_t seed, uint64_t W) {
  const uint4 x = philox_4x32_10(make_uint4(uint32_t(n), uint32_t(n >> 32), 0u, 0u),
                                 uint32_t(seed), uint32_t(seed >> 32));
  const uint64_t u = (uint64_t(x.y) << 32) | x.x;
  return __umul64hi(u, W);
}

// Row i of a hyperwedge index: the last i with up_ptr[i] <= idx (rows with no
// upper neighbour share their successor's prefix and are never chosen).
__device__ __forceinline__ int64_t wedge_row(const int64_t* __restrict__ up_ptr, int64_t E,
                                             int64_t idx) {
  int64_t lo = 0, hi = E;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (up_ptr[mid] <= idx) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
