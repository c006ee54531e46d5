// Device helpers shared by the on-the-fly samplers: wave reductions, the
// per-slot node lists (padded to 4 nodes), the per-sample hash of
// u = e_i ∪ e_j and the packed per-visit sums of a walk, and the heavy-node
// superset counts.
#pragma once

#include "common.h"

namespace {

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int lo = __shfl_xor(int(uint32_t(v)), off);
    const int hi = __shfl_xor(int(uint32_t(uint64_t(v) >> 32)), off);
    v += int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned lo = unsigned(__shfl_xor(int(uint32_t(v)), off));
    const unsigned hi = unsigned(__shfl_xor(int(uint32_t(v >> 32)), off));
    const uint64_t o = (uint64_t(hi) << 32) | lo;
    v = o > v ? o : v;
  }
  return v;
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const int lo = __shfl_up(int(uint32_t(v)), off);
    const int hi = __shfl_up(int(uint32_t(uint64_t(v) >> 32)), off);
    const int64_t o = int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
    if (lane >= off) v += o;
  }
  return v;
}

// Expanded lists are padded with -1 to a multiple of 4 nodes, so each is read
// as independent 16-byte loads.
constexpr int kXPad = 4;

// The first 8 entries of a padded list (entries past its end read as -1).
__device__ __forceinline__ void load8(const int32_t* __restrict__ xnodes, uint32_t xs, uint32_t xe,
                                      int4& q0, int4& q1) {
  const int4* src = reinterpret_cast<const int4*>(xnodes + xs);
  q0 = src[0];
  q1 = xe - xs > uint32_t(kXPad) ? src[1] : make_int4(-1, -1, -1, -1);
}

// position of the heavy-index triple x0 < x1 < x2 among all such triples
__device__ __forceinline__ int triple_index(int x0, int x1, int x2) {
  return x2 * (x2 - 1) * (x2 - 2) / 6 + x1 * (x1 - 1) / 2 + x0;
}
constexpr int kHeavyTriples = kHeavyBits * (kHeavyBits - 1) * (kHeavyBits - 2) / 6;

// Per-sample enumeration state (one wave per sampled pair (i, j)).
//
// u = e_i ∪ e_j lives in a per-wave hash table of 64 buckets of 4 slots;
// slot = ((node + 1) << 4) | flags, 0 = free, flags = in e_i (bit 0), in e_j
// (bit 1), and the rank 1..3 of a skipped node (bits 2-3, 0 if walked).  A
// lookup reads one bucket (16 bytes) and compares its four slots without
// branching; a member whose bucket is full goes to a short overflow list.
constexpr int kEnumWaves = 4;
constexpr int kBuckets = 64;
constexpr int kSkip = 3;                   // heavy lists counted in bulk
constexpr int kPatterns = (1 << kSkip) - 1;
constexpr uint32_t kFI = 1, kFJ = 2;
constexpr int kBatch = 4;                  // samples taken from the queue at a time
constexpr int kMaxChunks = kWave * (MOCHY_MAX_EDGE / kXPad);  // chunks of one window

// Per-wave LDS of one sample's walk.
struct WalkLds {
  uint4 tab[kBuckets];
  uint32_t ovf[2 * MOCHY_MAX_EDGE];
  int32_t ei[MOCHY_MAX_EDGE], ej[MOCHY_MAX_EDGE];
  int32_t wn[2 * MOCHY_MAX_EDGE];          // walked nodes
  int64_t wb[2 * MOCHY_MAX_EDGE];          // node_ptr of each walked node
  int64_t pre[2 * MOCHY_MAX_EDGE + 1];     // prefix of walked list lengths
  // one window of 64 visits, split into 4-node chunks
  uint32_t vx[kWave];                      // start of the visit's node list in xnodes
  uint32_t vc[kWave];                      // its first chunk in the window
  int32_t vv[kWave];                       // the walked node it was reached through
  unsigned long long acc[kWave];           // packed sums of its chunks
  uint8_t cmap[kMaxChunks];                // chunk -> visit (lane)
  uint32_t novf;
};

// The plain enumeration's per-wave LDS: the walk's, and the walked e_k by
// skipped nodes held and size (a memoized key's samples need no tally, so
// their kernel keeps the smaller struct and more waves resident).
struct EnumLds : WalkLds {
  uint32_t tally[kPatterns * kSizeSlots];
};

__device__ __forceinline__ uint32_t bucket_of(int32_t z) {
  return (uint32_t(z) * 2654435761u) >> 26;  // 6 bits
}

// flags of node z (0 if z is not in u, or z = -1 padding); the overflow list
// is scanned only for the (rare) samples that have one
template <bool kOvf, class Tab>
__device__ __forceinline__ uint32_t lookup(const Tab& L, int32_t z, uint32_t novf) {
  const uint32_t key = uint32_t(z + 1) << 4;
  const uint4 q = L.tab[bucket_of(z)];
  uint32_t f = (q.x & ~15u) == key ? q.x : 0u;
  f |= (q.y & ~15u) == key ? q.y : 0u;
  f |= (q.z & ~15u) == key ? q.z : 0u;
  f |= (q.w & ~15u) == key ? q.w : 0u;
  if (kOvf)
    for (uint32_t t = 0; t < novf; ++t) f |= (L.ovf[t] & ~15u) == key ? L.ovf[t] : 0u;
  return f & 15u;
}

// Packed per-visit sums (6 bits each): |e_k|, |e_k ∩ e_i|, |e_k ∩ e_j|,
// |e_k ∩ e_i ∩ e_j|, walked members in e_k below the visit's node, and (2
// bits each) the three skipped nodes held.  The walked members are those of u
// that are not skipped, or with kJOnly those of e_j only (when e_i's lists
// are not walked).
constexpr int kSc = 0, kSi = 6, kSj = 12, kSt = 18, kSb = 24, kSp = 30;

template <bool kOvf, bool kJOnly = false, class Tab>
__device__ __forceinline__ unsigned long long chunk_sums(const Tab& L, int4 z4, int32_t v,
                                                         uint32_t novf) {
  unsigned long long s = 0;
  auto one = [&](int32_t z) {
    const uint32_t ff = lookup<kOvf>(L, z, novf);
    const uint32_t rk = ff >> 2;
    uint32_t w = z >= 0 ? 1u : 0u;
    w += (ff & 1u) << kSi;
    w += ((ff >> 1) & 1u) << kSj;
    w += ((ff & 3u) == 3u ? 1u : 0u) << kSt;
    const bool walked = kJOnly ? (ff & 2u) != 0u : ff != 0u;
    w += (walked && !rk && z < v) ? 1u << kSb : 0u;
    s += w;
    s += rk ? 1ull << (kSp + 2 * (rk - 1u)) : 0ull;
  };
  one(z4.x); one(z4.y); one(z4.z); one(z4.w);
  return s;
}

__device__ __forceinline__ uint32_t big_slot(uint64_t mask, int log2cap) {
  return uint32_t((mask * 0x9E3779B97F4A7C15ull) >> (64 - log2cap));
}

// hyperedges of size c holding every heavy node of the set `xmask` (bits =
// heavy indices, 1 to 6 of them)
__device__ __forceinline__ int64_t heavy_set_count(uint64_t xmask, int c,
                                                   const uint32_t* __restrict__ hsize,
                                                   const uint32_t* __restrict__ hpair,
                                                   const uint32_t* __restrict__ htriple,
                                                   const unsigned long long* __restrict__ big_key,
                                                   const uint32_t* __restrict__ big_val,
                                                   int big_log2) {
  const int n = __popcll(xmask);
  const int x0 = __ffsll((long long)xmask) - 1;
  if (n == 1) return hsize[x0 * kSizeSlots + c];
  const uint64_t r1 = xmask & (xmask - 1);
  const int x1 = __ffsll((long long)r1) - 1;
  if (n == 2) return hpair[(x0 * kHeavyBits + x1) * kSizeSlots + c];
  if (n == 3) {
    const int x2 = __ffsll((long long)(r1 & (r1 - 1))) - 1;
    return htriple[int64_t(triple_index(x0, x1, x2)) * kSizeSlots + c];
  }
  const uint32_t cap_mask = (1u << big_log2) - 1u;
  for (uint32_t s = big_slot(xmask, big_log2);; s = (s + 1u) & cap_mask) {
    const unsigned long long k = big_key[s];
    if (k == xmask) return big_val[uint64_t(s) * kSizeSlots + c];
    if (k == 0ull) return 0;
  }
}

// hyperedges of size c holding every heavy node of `mask` (bits index hb[])
__device__ __forceinline__ int64_t superset_count(uint32_t mask, const int* hb, int c,
                                                  const uint32_t* __restrict__ hsize,
                                                  const uint32_t* __restrict__ hpair,
                                                  const uint32_t* __restrict__ htriple) {
  int h[kSkip], n = 0;
  for (int x = 0; x < kSkip; ++x)
    if (mask & (1u << x)) h[n++] = hb[x];
  if (n == 1) return hsize[h[0] * kSizeSlots + c];
  if (n == 2) return hpair[(h[0] * kHeavyBits + h[1]) * kSizeSlots + c];
  int x0 = h[0], x1 = h[1], x2 = h[2];  // sort the three heavy indices
  if (x0 > x1) { const int t = x0; x0 = x1; x1 = t; }
  if (x1 > x2) { const int t = x1; x1 = x2; x2 = t; }
  if (x0 > x1) { const int t = x0; x0 = x1; x1 = t; }
  return htriple[int64_t(triple_index(x0, x1, x2)) * kSizeSlots + c];
}

}  // namespace
