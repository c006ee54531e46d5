// Exact h-motif / 3h-motif counts on the device (MoCHy-E, Algorithm 2).
//
// Algorithm 2 takes every centre e_i and every unordered pair {e_j, e_k} of
// its line-graph neighbours and counts the triple iff e_j and e_k are
// disjoint or i < min(j, k); the class comes from the seven region sizes of
// Lemma 2.  Here the neighbours of e_i are the row's positions 0..d-1 in
// ascending id order, and u = number of neighbours with id < i, so
//   * a pair with a position < u (a neighbour below i) is counted iff the two
//     neighbours are disjoint (an open instance whose middle is e_i);
//   * a pair with both positions >= u is always counted.
//
// Region sizes of a pair from the per-neighbour records of the centre:
//   t  = |e_i ∩ e_j ∩ e_k|     = popcount(m_j & m_k)
//   R4 = p_j - t, R6 = s_k - t, R1 = |e_i| - p_j - s_k + t, R7 = t
//   R5 = |e_j ∩ e_k - e_i|,  R2 = o_j - R5,  R3 = o_k - R5
// R5 is the only quantity that needs nodes outside e_i.  The records carry
// an exact bit for each of the 64 highest-degree nodes, so the main kernel
// uses R5 = popcount(h_j & h_k).  That is exact unless e_j and e_k also share
// a lower-degree ("light") node outside e_i; the correction kernel finds every
// such pair (from the node->hyperedge lists of the light nodes), undoes what
// the main kernel recorded for it and records the exact class.
//
// Main kernel work decomposition: an item is (row, block of 64 positions);
// lane l of a wave holds the record of position 64*block + l ("k") and the
// wave walks j over the positions below it; the j record is uniform and read
// through the scalar cache.  Items are ordered by block index descending, so
// the largest items start first, and pulled from a global counter by
// persistent waves.  Counts go to a per-workgroup LDS histogram (several
// copies, picked by lane, to thin same-bin conflicts), flushed once per
// workgroup with 64-bit global atomics.
//
// Grouped path (the default, k_group + k_exact_grouped): neighbours of e_i
// with equal records (m, outside count clamped to popcount(h) + 2, h) form a
// group with N members and A members above the centre; a pair of groups
// stands for N_j N_k candidates if they look disjoint, A_j A_k otherwise,
// and a group with itself for C(A, 2).  Each row's region holds the groups
// with A > 0 first.  A pair involving a group with A = 0 counts only if open,
// and an open class depends on j only through (popcount(m_j), min(o_j, 2)):
// such pairs are summed per lane over runs of one such class (the groups are
// class-ordered within each hash part) and added once per run.
#include <vector>

#include "classify.h"
#include "common.h"

namespace {

constexpr int kCopies = 2;                 // histogram copies per wave (picked by lane)
constexpr int kStride = kHistSlots + 1;    // odd stride spreads the copies over banks
constexpr int kWavesPerGroup = 4;
constexpr int64_t kFlushVisits = int64_t(1) << 26;  // 32 lanes share a copy: counters < 2^32

// ---------------------------------------------------------------------------
// Scheduling, graph-major: the rows of graph 0 come first, then graph 1, ...;
// inside a graph, rows are sorted by number of 64-blocks (descending) and a
// row's items (its blocks, largest block index first) are consecutive, so
// big work starts first and the waves working on one row share its records
// in L2.  Per graph g, with NB = maxnb + 1 slots:
//   cnt[g][b]   rows of g with more than b blocks (cnt[g][maxnb] = 0), i.e.
//               the first slot of g's rows with b+... blocks in `order`
//   seg[g]      first slot of graph g's rows in `order`
// `order` lists rows (-1 in unused slots); rstart = prefix sums of the rows'
// block counts, so item q is block (nb - 1 - (q - rstart[k])) of row order[k].

__global__ void k_sched_count(int64_t c0, int64_t c1, int32_t NB, const int64_t* __restrict__ row_ptr,
                              int64_t min_len, const int32_t* __restrict__ row_graph,
                              unsigned long long* nbhist) {
  const int64_t i = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= c1) return;
  const int64_t d = row_ptr[i + 1] - row_ptr[i];
  if (d < min_len) return;
  atomicAdd(&nbhist[int64_t(row_graph[i]) * NB + (d + kWave - 1) / kWave], 1ull);
}

// One block per graph.
__global__ __launch_bounds__(1024) void k_sched_scan(int32_t maxnb,
                                                     const unsigned long long* __restrict__ nbhist_all,
                                                     int64_t* cnt_all, int64_t* item_start_all,
                                                     int64_t* total) {
  __shared__ int64_t part[1024];
  const int64_t NB = maxnb + 1;
  const unsigned long long* nbhist = nbhist_all + blockIdx.x * NB;
  int64_t* cnt = cnt_all + blockIdx.x * NB;
  int64_t* item_start = item_start_all + blockIdx.x * NB;
  const int n = maxnb;  // entries b = 0..maxnb-1; cnt[maxnb] = 0
  const int chunk = (n + 1023) / 1024;
  // suffix sums computed as prefix sums over the reversed index r = n-1-b
  // pass 1: cnt[b] = sum_{m > b} hist[m]  (m in 1..maxnb)
  {
    const int r0 = min(n, int(threadIdx.x) * chunk), r1 = min(n, r0 + chunk);
    int64_t s = 0;
    for (int r = r0; r < r1; ++r) s += int64_t(nbhist[n - r]);  // hist[b+1] for b = n-1-r
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int r = r0; r < r1; ++r) {
      run += int64_t(nbhist[n - r]);
      cnt[n - 1 - r] = run;
    }
    if (threadIdx.x == 0) cnt[n] = 0;
    __syncthreads();
  }
  // pass 2: item_start[b] = sum_{b' > b} cnt[b']
  {
    const int r0 = min(n, int(threadIdx.x) * chunk), r1 = min(n, r0 + chunk);
    int64_t s = 0;
    for (int r = r0; r < r1; ++r) s += cnt[n - 1 - r];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int r = r0; r < r1; ++r) {
      item_start[n - 1 - r] = run;
      run += cnt[n - 1 - r];
    }
    if (threadIdx.x == 1023) total[blockIdx.x] = part[1023];
  }
}

// Single block: gq = exclusive prefix of the per-graph item totals (gq[ng] =
// all items), seg[g] = first slot of graph g's rows in `order`.
__global__ __launch_bounds__(1024) void k_sched_graphs(int32_t ng, int64_t c0, int64_t c1,
                                                       const int64_t* __restrict__ geoff,
                                                       const int64_t* __restrict__ total,
                                                       int64_t* gq, int64_t* seg) {
  __shared__ int64_t part[1024];
  const int chunk = (ng + 1023) / 1024;
  const int g0 = min(ng, int(threadIdx.x) * chunk), g1 = min(ng, g0 + chunk);
  int64_t s = 0;
  for (int g = g0; g < g1; ++g) s += total[g];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - s;
  for (int g = g0; g < g1; ++g) {
    gq[g] = run;
    run += total[g];
    const int64_t lo = geoff[g] < c0 ? c0 : (geoff[g] > c1 ? c1 : geoff[g]);
    seg[g] = lo - c0;
  }
  if (threadIdx.x == 1023) gq[ng] = part[1023];
}

// Blocks per slot of `order` (0 for unused slots), the input of rstart.
__global__ void k_item_counts(int64_t n, const int32_t* __restrict__ order,
                              const int64_t* __restrict__ row_ptr, int64_t* nbk) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k > n) return;
  int64_t v = 0;
  if (k < n && order[k] >= 0) {
    const int32_t i = order[k];
    v = (row_ptr[i + 1] - row_ptr[i] + kWave - 1) / kWave;
  }
  nbk[k] = v;
}

__global__ void k_sched_scatter(int64_t c0, int64_t c1, int32_t NB, const int64_t* __restrict__ row_ptr,
                                int64_t min_len, const int32_t* __restrict__ row_graph,
                                const int64_t* __restrict__ cnt, const int64_t* __restrict__ seg,
                                unsigned long long* fill, int32_t* order) {
  const int64_t i = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= c1) return;
  const int64_t d = row_ptr[i + 1] - row_ptr[i];
  if (d < min_len) return;
  const int64_t g = row_graph[i];
  const int64_t nb = (d + kWave - 1) / kWave;
  const unsigned long long slot = atomicAdd(&fill[g * NB + nb], 1ull);
  order[seg[g] + cnt[g * NB + nb] + int64_t(slot)] = int32_t(i);
}

// Walk j over [j0, j1) against the lane's k.  kCountAll: both j and k are
// above the centre (count every pair); otherwise count only disjoint pairs.
// kDiag: the j range overlaps the lane block, so require j < kp.
template <bool kCountAll, bool kDiag>
__device__ __forceinline__ void pair_step(const uint4& rj, int j, uint32_t a, const Side& k,
                                          uint32_t khl, uint32_t khh, int kp, bool valid,
                                          const uint16_t* __restrict__ lut, uint32_t* hist) {
  const uint32_t mj = rj.x;
  bool act = valid;
  if (kDiag) act = act && (j < kp);
  if (!kCountAll) {
    // below the centre only disjoint pairs count: test with ANDs, no popcounts
    act = act && (((mj & k.m) | (rj.z & khl) | (rj.w & khh)) == 0u);
  }
  if (act) {
    const uint32_t t = kCountAll ? uint32_t(__popc(mj & k.m)) : 0u;
    const uint32_t r5 = kCountAll ? uint32_t(__popc(rj.z & khl) + __popc(rj.w & khh)) : 0u;
    const uint32_t code = pair_code(a, __popc(mj), rj.y & 0xffu, k, t, r5);
    atomicAdd(&hist[lut[code]], 1u);
  }
}

// Walk j over [j0, j1) against the lane's k, four records per step (the
// four uniform loads are issued together).  kCountAll: both j and k are
// above the centre (count every pair); otherwise count only disjoint pairs.
// kDiag: the j range overlaps the lane block, so require j < kp.
template <bool kCountAll, bool kDiag>
__device__ __forceinline__ void walk(const uint4* __restrict__ row, int j0, int j1, uint32_t a,
                                     const Side& k, int kp, bool valid,
                                     const uint16_t* __restrict__ lut, uint32_t* hist) {
  const uint32_t khl = uint32_t(k.h), khh = uint32_t(k.h >> 32);
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
    const uint4 r0 = row[j], r1 = row[j + 1], r2 = row[j + 2], r3 = row[j + 3];
    pair_step<kCountAll, kDiag>(r0, j, a, k, khl, khh, kp, valid, lut, hist);
    pair_step<kCountAll, kDiag>(r1, j + 1, a, k, khl, khh, kp, valid, lut, hist);
    pair_step<kCountAll, kDiag>(r2, j + 2, a, k, khl, khh, kp, valid, lut, hist);
    pair_step<kCountAll, kDiag>(r3, j + 3, a, k, khl, khh, kp, valid, lut, hist);
  }
  for (; j < j1; ++j) pair_step<kCountAll, kDiag>(row[j], j, a, k, khl, khh, kp, valid, lut, hist);
}

// Adds a wave's histogram copies into graph g's global counts and clears them.
__device__ __forceinline__ void flush_wave(uint32_t* whist, int lane, int64_t g,
                                           unsigned long long* hist_out) {
  __builtin_amdgcn_wave_barrier();
  for (int t = lane; t < kHistSlots; t += kWave) {
    unsigned long long s = 0;
    for (int c = 0; c < kCopies; ++c) {
      s += whist[c * kStride + t];
      whist[c * kStride + t] = 0u;
    }
    if (s) atomicAdd(&hist_out[g * kHistSlots + t], s);
  }
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(256) void k_exact_main(
    const int64_t* __restrict__ edge_ptr, const int64_t* __restrict__ lg_ptr,
    const int32_t* __restrict__ up_first, const uint4* __restrict__ rec,
    const int32_t* __restrict__ order, const int64_t* __restrict__ rstart, int64_t nslots,
    const int32_t* __restrict__ row_graph, unsigned long long* queue,
    const uint16_t* __restrict__ code_to_id3, unsigned long long* hist_out) {
  __shared__ uint16_t lut[kNumCodes];
  __shared__ uint32_t hist[kWavesPerGroup * kCopies * kStride];
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  for (int t = threadIdx.x; t < kWavesPerGroup * kCopies * kStride; t += blockDim.x) hist[t] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  uint32_t* whist = hist + wave * (kCopies * kStride);
  uint32_t* myhist = whist + (lane & (kCopies - 1)) * kStride;
  const int64_t total = rstart[nslots];
  int dirty_g = -1;
  int64_t visits = 0;
  for (;;) {
    unsigned long long qq = 0;
    if (lane == 0) qq = atomicAdd(queue, 1ull);
    const int64_t q = (int64_t)(((unsigned long long)__builtin_amdgcn_readfirstlane(int(qq >> 32)) << 32) |
                                (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(int(qq)));
    if (q >= total) break;
    // slot k of `order` with rstart[k] <= q < rstart[k + 1]
    int64_t lo = 0, hi = nslots;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (rstart[mid] <= q) lo = mid; else hi = mid;
    }
    const int32_t i = order[lo];
    const int g = row_graph[i];
    if (dirty_g >= 0 && (dirty_g != g || visits > kFlushVisits)) {
      flush_wave(whist, lane, dirty_g, hist_out);
      visits = 0;
    }
    dirty_g = g;
    const int nbi = int(rstart[lo + 1] - rstart[lo]);
    const int b = nbi - 1 - int(q - rstart[lo]);
    const int64_t base = lg_ptr[i];
    const int d = int(lg_ptr[i + 1] - base);
    const int u = up_first[i];
    const uint32_t a = uint32_t(edge_ptr[i + 1] - edge_ptr[i]);
    const uint4* __restrict__ row = rec + base;
    const int kp = b * kWave + lane;
    const bool valid = kp < d;
    Side k;
    {
      const uint4 rk = valid ? row[kp] : make_uint4(0, 0, 0, 0);
      k.m = rk.x;
      k.o = rk.y & 0xffu;
      k.s = __popc(rk.x);
      k.h = (unsigned long long)rk.z | ((unsigned long long)rk.w << 32);
    }
    const int blo = b * kWave;
    const int kmax = min(blo + kWave, d);
    visits += int64_t(kmax);
    // j below the centre: count disjoint pairs only
    const int ua = min(u, blo);
    walk<false, false>(row, 0, ua, a, k, kp, valid, lut, myhist);
    walk<false, true>(row, max(ua, blo), min(u, kmax), a, k, kp, valid, lut, myhist);
    // j (and so k) above the centre: count every pair
    walk<true, false>(row, u, blo, a, k, kp, valid, lut, myhist);
    walk<true, true>(row, max(u, blo), kmax, a, k, kp, valid, lut, myhist);
  }
  if (dirty_g >= 0) flush_wave(whist, lane, dirty_g, hist_out);
}

// ---------------------------------------------------------------------------
// Neighbour groups.  The main kernel's class of a pair (j, k) of a centre,
// and whether Algorithm 2 counts it, depend only on the two records: the
// masks m (nodes of e_i held) and h (heavy nodes outside e_i) and the outside
// counts o, where only min(o - R5, 2) is ever used and R5 <= popcount(h), so o
// may be clamped to popcount(h) + 2.  Neighbours with equal (m, clamped o, h)
// form a group; a group keeps N (members) and A (members above the centre).
// Between two groups x != y the main kernel's count is N_x N_y if they are
// disjoint (every pair counts) and A_x A_y otherwise (only pairs above the
// centre count); inside a group it is C(A, 2) (members share their nodes of
// e_i, so never disjoint).  Pairs sharing a light node are corrected from the
// ungrouped records afterwards, as before.
//
// One block per row groups the row's records in an LDS hash table
// keyed by a 64-bit hash of the signature.  A row longer than the table is
// cut into parts by the hash (records of one part per pass); a pass whose
// table fills is redone with twice the parts.  After each pass every record
// checks its signature against its slot's first member: two signatures with
// one hash restart the row with another hash seed, so groups are exact.
// Two table sizes.  Rows of at most kShortRow records: 512-thread blocks,
// 2048 slots (41 KB of LDS, three blocks per CU), one block per row over all
// rows (a longer row's block returns at once).  Longer rows: 1024-thread
// blocks with 8000 slots (160 KB, one block per CU) over a list of those
// rows: a larger table means fewer hash parts, and every part re-reads the
// row twice.  On medium the long-row table took the grouping from 62 ms (all
// rows at 2048 slots: up to 18 parts, 12,805 rows regrouped) to 37 ms (up to
// 4 parts); 4032 slots in 512-thread blocks took 48 ms.  Small graphs keep
// the short-row table, whose blocks clear only 2048 slots and share the CU.
constexpr int kShortThreads = 512, kShortSlots = 2048;
constexpr int kLongThreads = 1024, kLongSlots = 8000;
constexpr int64_t kShortRow = 2 * kShortSlots;

// Home slot of a 64-bit signature hash (multiply-shift range reduction of
// its low 32 bits, any table size) and the next slot of a linear probe.
template <int kSlots>
__device__ __forceinline__ uint32_t home_slot(uint64_t kk) {
  return uint32_t((uint64_t(uint32_t(kk)) * uint32_t(kSlots)) >> 32);
}
template <int kSlots>
__device__ __forceinline__ uint32_t next_slot(uint32_t s) { return s + 1u == uint32_t(kSlots) ? 0u : s + 1u; }

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  // SplitMix64 finalizer (Steele, Lea, Flood, OOPSLA'14)
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

__device__ __forceinline__ uint32_t clamp_outside(const uint4& r) {
  const uint32_t o = r.y & 0xffu;
  const uint32_t cap = uint32_t(__popc(r.z) + __popc(r.w)) + 2u;
  return o < cap ? o : cap;
}

__device__ __forceinline__ uint64_t sig_hash(const uint4& r, uint32_t o, uint64_t seed) {
  uint64_t x = mix64(seed ^ (uint64_t(r.x) | (uint64_t(o) << 32)));
  x = mix64(x ^ (uint64_t(r.z) | (uint64_t(r.w) << 32)));
  return x | 1ull;  // 0 marks a free slot
}

constexpr int kGroupTries = 40;  // restarts before a row gives up (flags bit 0)

// Open class of a group: (|its overlap with e_i|, min(outside, 2)); the code
// of an open pair depends on j only through it.  Below kOpenClasses.
constexpr int kOpenClasses = 128;
__device__ __forceinline__ uint32_t open_class(uint32_t m, uint32_t o) {
  return uint32_t(__popc(m)) * 3u + st3(o);
}

template <int kSlots>
struct GroupTable {
  unsigned long long key[kSlots];
  uint32_t nall[kSlots], nabove[kSlots], first[kSlots];
  uint32_t s_out, s_outb, s_bad, s_cnt;
  uint32_t cfill[2 * kOpenClasses];  // per (above, open class): count, then next slot
};

// Groups of row i with the block's table.  kWrite: row i's groups go to its
// region [base[i] - cap0, base[i + 1] - cap0) of grec / gcnt: base = lg_ptr
// with the row-capacity layout (a row has at most as many groups as
// records), or the prefix of the counts with cap0 = 0 (compact layout,
// counted by a first pass).  Groups with members above the centre fill the
// region from its start (their count goes to gna[i]), the others from its
// end, so that the pair kernel can take the pairs that can only be open
// apart; within each hash part of the row, both kinds are ordered by open
// class.  The count goes to gcount[i].  Hash parts: a first guess of
// 2 * kSlots records per part, doubled whenever a part has more than
// 3/4 * kSlots groups (rows have 0.38 groups per record on medium).
template <bool kWrite, int kThreads, int kSlots>
__device__ __forceinline__ int64_t group_row(
    GroupTable<kSlots>& T, int64_t i, const int64_t* __restrict__ lg_ptr,
    const int32_t* __restrict__ up_first, const uint4* __restrict__ rec, int64_t* gcount,
    const int64_t* __restrict__ obase_of, int64_t cap0, uint4* grec, uint2* gcnt, int32_t* gna,
    int32_t* flags, bool pack16) {
  constexpr int64_t kPartRecords = 2 * kSlots;
  constexpr uint32_t kPartGroups = kSlots * 3 / 4;
  const int tid = threadIdx.x;
  const int64_t base = lg_ptr[i];
  const int64_t d = lg_ptr[i + 1] - base;
  const int64_t u = up_first[i];
  const uint4* row = rec + base;
  int64_t parts = (d + kPartRecords - 1) / kPartRecords;
  if (parts < 1) parts = 1;
  const int64_t parts0 = parts;
  uint64_t seed = 0;
  const int64_t obase = kWrite ? obase_of[i] - cap0 : 0;
  const int64_t oend = kWrite ? obase_of[i + 1] - cap0 : 0;  // one past the row's region
  for (int tries = 0;; ++tries) {  // until a grouping without overflow or hash collision
    if (tries == kGroupTries) {  // cannot happen with a sound hash; the host pairs records
      if (tid == 0) {
        atomicOr(flags, 1);
        if (gcount) gcount[i] = 0;
      }
      __syncthreads();
      return 0;
    }
    __syncthreads();
    if (tid == 0) {
      T.s_out = 0u;
      T.s_outb = 0u;
    }
    bool redo = false;
    for (int64_t part = 0; part < parts && !redo; ++part) {
      for (int t = tid; t < kSlots; t += kThreads) {
        T.key[t] = 0ull;
        T.nall[t] = 0u;
        T.nabove[t] = 0u;
      }
      if (tid == 0) {
        T.s_bad = 0u;
        T.s_cnt = 0u;
      }
      __syncthreads();
      for (int64_t r = tid; r < d; r += kThreads) {
        if (*(volatile uint32_t*)&T.s_bad) break;  // this part overflowed: the row is redone
        const uint4 rr = row[r];
        const uint64_t kk = sig_hash(rr, clamp_outside(rr), seed);
        if (int64_t((kk >> 40) % uint64_t(parts)) != part) continue;
        uint32_t slot = home_slot<kSlots>(kk);
        int n = 0;
        for (; n < kSlots; ++n) {
          const unsigned long long old = atomicCAS(&T.key[slot], 0ull, kk);
          if (old == 0ull) {
            T.first[slot] = uint32_t(r);
            if (atomicAdd(&T.s_cnt, 1u) >= kPartGroups) atomicOr(&T.s_bad, 4u);
            break;
          }
          if (old == kk) break;
          slot = next_slot<kSlots>(slot);
        }
        if (n == kSlots) { atomicOr(&T.s_bad, 1u); continue; }
        atomicAdd(&T.nall[slot], 1u);
        if (r >= u) atomicAdd(&T.nabove[slot], 1u);
      }
      __syncthreads();
      const uint32_t full = T.s_bad;
      __syncthreads();  // every thread has read the flag before it is written again
      if (full) {  // too many groups in the part: twice the parts
        parts *= 2;
        redo = true;
        break;
      }
      // every record against its slot's first member
      for (int64_t r = tid; r < d; r += kThreads) {
        const uint4 rr = row[r];
        const uint32_t o = clamp_outside(rr);
        const uint64_t kk = sig_hash(rr, o, seed);
        if (int64_t((kk >> 40) % uint64_t(parts)) != part) continue;
        uint32_t slot = home_slot<kSlots>(kk);
        while (T.key[slot] != kk) slot = next_slot<kSlots>(slot);
        const uint4 f = row[T.first[slot]];
        if (f.x != rr.x || f.z != rr.z || f.w != rr.w || clamp_outside(f) != o) atomicOr(&T.s_bad, 2u);
      }
      __syncthreads();
      const uint32_t clash = T.s_bad;
      __syncthreads();
      if (clash) {  // two signatures with one hash: another seed
        seed += 0x9E3779B97F4A7C15ull;
        redo = true;
        break;
      }
      if (!kWrite) {
        for (int t = tid; t < kSlots; t += kThreads)
          if (T.key[t] != 0ull) atomicAdd(&T.s_out, 1u);
        __syncthreads();
        continue;
      }
      // counting sort of the part's groups by (above, open class)
      for (int t = tid; t < 2 * kOpenClasses; t += kThreads) T.cfill[t] = 0u;
      __syncthreads();
      for (int t = tid; t < kSlots; t += kThreads) {
        if (T.key[t] == 0ull) continue;
        const uint4 f = row[T.first[t]];
        atomicAdd(&T.cfill[(T.nabove[t] != 0u ? 0 : kOpenClasses) + open_class(f.x, clamp_outside(f))], 1u);
      }
      __syncthreads();
      if (tid < 2 * kWave) {  // exclusive prefix per kind (one wave each), from where its output stands
        static_assert(kOpenClasses == 2 * kWave, "two classes per lane");
        const int kind = tid / kWave, ln = tid % kWave;
        uint32_t* cf = T.cfill + kind * kOpenClasses + 2 * ln;
        const uint32_t n0 = cf[0], n1 = cf[1];
        uint32_t inc = n0 + n1;
        for (int off = 1; off < kWave; off <<= 1) {
          const uint32_t up = __shfl_up(inc, off, kWave);
          if (ln >= off) inc += up;
        }
        const uint32_t start = (kind == 0 ? T.s_out : T.s_outb) + inc - (n0 + n1);
        cf[0] = start;
        cf[1] = start + n0;
      }
      __syncthreads();
      for (int t = tid; t < kSlots; t += kThreads) {
        if (T.key[t] == 0ull) continue;
        const bool above = T.nabove[t] != 0u;
        const uint4 f = row[T.first[t]];
        const uint32_t oc = clamp_outside(f);
        const uint32_t pos = atomicAdd(&T.cfill[(above ? 0 : kOpenClasses) + open_class(f.x, oc)], 1u);
        const int64_t o = above ? obase + pos : oend - 1 - pos;
        // y: |m| (bits 0-7), 2 |m| + 4 (8-15), the clamped outside count
        // (16-23) and the open class (24-30), which the pair kernel then
        // reads instead of recomputing them per pair: (|m|, outside) is y
        // with bits 8-15 and 24-31 cleared, one scalar AND
        const uint32_t pm = uint32_t(__popc(f.x));
        grec[o] = make_uint4(f.x, pm | ((2u * pm + 4u) << 8) | (oc << 16) | (open_class(f.x, oc) << 24), f.z, f.w);
        // pack16 (every row shorter than 2^16 neighbours): the second word
        // holds nabove and nall as 16-bit halves, for the pair kernel's
        // two-term dot product of the weight
        gcnt[o] = make_uint2(T.nall[t], pack16 ? T.nabove[t] | (T.nall[t] << 16) : T.nabove[t]);
      }
      __syncthreads();
      if (tid == 0) {  // both kinds' ends: the last class's next slot
        T.s_out = T.cfill[kOpenClasses - 1];
        T.s_outb = T.cfill[2 * kOpenClasses - 1];
      }
      __syncthreads();
    }
    if (!redo) break;
  }
  if (tid == 0) {
    if (gcount) gcount[i] = int64_t(T.s_out) + T.s_outb;
    if (kWrite) gna[i] = int32_t(T.s_out);
  }
  __syncthreads();  // the table is free for the block's next row
  return parts > parts0 ? -parts : parts;  // the parts used, negative if the row was regrouped
}

// Short rows: one block per row of [c0, c0 + gridDim.x); longer rows are
// the long-row kernel's.
template <bool kWrite>
__global__ __launch_bounds__(kShortThreads) void k_group_short(
    int64_t c0, const int64_t* __restrict__ lg_ptr, const int32_t* __restrict__ up_first,
    const uint4* __restrict__ rec, int64_t* gcount, const int64_t* __restrict__ obase_of,
    int64_t cap0, uint4* grec, uint2* gcnt, int32_t* gna, int32_t* flags, unsigned long long* stats,
    bool pack16) {
  __shared__ GroupTable<kShortSlots> T;
  const int64_t i = c0 + blockIdx.x;
  if (lg_ptr[i + 1] - lg_ptr[i] > kShortRow) return;  // uniform
  const int64_t p = group_row<kWrite, kShortThreads, kShortSlots>(T, i, lg_ptr, up_first, rec, gcount, obase_of,
                                                                  cap0, grec, gcnt, gna, flags, pack16);
  // one pass of the grouping reports the parts; a row of one part is the
  // common case and needs no report (the host's maximum starts at 1)
  if (stats && threadIdx.x == 0 && (p < 0 || p > 1)) {
    if (p < 0) atomicAdd(&stats[kStRegrouped], 1ull);
    atomicMax(&stats[kStMaxParts], (unsigned long long)(p < 0 ? -p : p));
  }
}

// Long rows: rows[0 .. *nrows), each block pulling the next from `queue`.
template <bool kWrite>
__global__ __launch_bounds__(kLongThreads) void k_group_long(
    const int32_t* __restrict__ rows, const unsigned long long* __restrict__ nrows,
    unsigned long long* queue,
    const int64_t* __restrict__ lg_ptr, const int32_t* __restrict__ up_first,
    const uint4* __restrict__ rec, int64_t* gcount, const int64_t* __restrict__ obase_of,
    int64_t cap0, uint4* grec, uint2* gcnt, int32_t* gna, int32_t* flags, unsigned long long* stats,
    bool pack16) {
  __shared__ GroupTable<kLongSlots> T;
  __shared__ int64_t s_q;
  const int64_t n = int64_t(*nrows);
  unsigned long long regrouped = 0, most = 0;  // this block's rows (thread 0's copy is used)
  for (;;) {  // rows pulled from a counter; every block leaves once the list is taken
    if (threadIdx.x == 0) s_q = int64_t(atomicAdd(queue, 1ull));
    __syncthreads();
    const int64_t q = s_q;
    __syncthreads();
    if (q >= n) break;
    const int64_t p = group_row<kWrite, kLongThreads, kLongSlots>(T, rows[q], lg_ptr, up_first, rec, gcount,
                                                                  obase_of, cap0, grec, gcnt, gna, flags, pack16);
    regrouped += p < 0 ? 1ull : 0ull;
    most = max(most, (unsigned long long)(p < 0 ? -p : p));
  }
  if (stats && threadIdx.x == 0 && most > 0) {
    if (regrouped) atomicAdd(&stats[kStRegrouped], regrouped);
    atomicMax(&stats[kStMaxParts], most);
  }
}

// The rows of [c0, c1) longer than kShortRow, appended to rows[] (any order).
__global__ void k_long_rows(int64_t c0, int64_t c1, const int64_t* __restrict__ lg_ptr,
                            int32_t* rows, unsigned long long* nrows) {
  const int64_t i = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < c1 && lg_ptr[i + 1] - lg_ptr[i] > kShortRow) rows[atomicAdd(nrows, 1ull)] = int32_t(i);
}

// Per-row group statistics of rows [c0, c1): groups, groups with members
// above the centre, pairs of such groups (classified in full by the pair
// kernel) and the other pairs of groups (counted only when open).
__global__ __launch_bounds__(256) void k_group_stats(int64_t c0, int64_t c1, const int64_t* __restrict__ goff,
                                                     const int32_t* __restrict__ gna,
                                                     unsigned long long* stats) {
  const int64_t i = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  unsigned long long ng = 0, na = 0;
  if (i < c1) {
    ng = (unsigned long long)(goff[i + 1] - goff[i]);
    na = (unsigned long long)gna[i];
  }
  unsigned long long v[4] = {ng, na, na * (na - (na ? 1 : 0)) / 2,
                             ng * (ng - (ng ? 1 : 0)) / 2 - na * (na - (na ? 1 : 0)) / 2};
  __shared__ unsigned long long red[4][256 / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int x = 0; x < 4; ++x) {
    for (int off = kWave / 2; off > 0; off >>= 1) v[x] += __shfl_xor(v[x], off, kWave);
    if (lane == 0) red[x][wave] = v[x];
  }
  __syncthreads();
  if (threadIdx.x < 4) {  // one atomic per block and counter
    unsigned long long t = 0;
    for (int w = 0; w < 256 / kWave; ++w) t += red[threadIdx.x][w];
    const int slot = kStGroups + int(threadIdx.x);  // groups, above, full pairs, open pairs
    if (t) atomicAdd(&stats[slot], t);
  }
}

// Pairs of groups (x < y) and each group with itself, weighted as above.
constexpr int kGCopies = 2;
constexpr int kGStride = kHistSlots + 1;

// max(a - b, 0) in one saturating subtract.
__device__ __forceinline__ uint32_t usat(uint32_t a, uint32_t b) { return a > b ? a - b : 0u; }

// max(a - b, 0) on both 16-bit halves at once (a packed saturating subtract).
__device__ __forceinline__ uint32_t pk_usat_sv(uint32_t a, uint32_t b) {  // a uniform
  uint32_t r;
  asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(r) : "s"(a), "v"(b));
  return r;
}
__device__ __forceinline__ uint32_t pk_usat_vv(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ uint32_t pk_usat_vs(uint32_t a, uint32_t b) {  // b uniform
  uint32_t r;
  asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(r) : "v"(a), "s"(b));
  return r;
}

// lo(d) * lo(w) + hi(d) * hi(w) + c, 16-bit halves (w uniform): two
// multiply-adds of a Horner chain in one instruction.
__device__ __forceinline__ uint32_t dot2(uint32_t d, uint32_t w, uint32_t c) {
  uint32_t r;
  asm("v_dot2_u32_u16 %0, %1, %2, %3" : "=v"(r) : "v"(d), "s"(w), "v"(c));
  return r;
}

// lo(a) * lo(b) + hi(a) * hi(b), 16-bit halves, both per lane.
__device__ __forceinline__ uint32_t dot2_vv(uint32_t a, uint32_t b) {
  uint32_t r;
  asm("v_dot2_u32_u16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Twice the reversed ternary code 2186 - code of a pair (code as
// pair_code gives it, same digit order): the byte offset of its entry in
// the pair kernel's class table (stored reversed, 2-byte entries).  Digit r
// enters as 2 - min(R_r, 2) = max(2 - R_r, 0).  With tr holding t + 2 =
// |e_i ∩ e_j ∩ e_k| + 2 and r5 + 2 = |e_j ∩ e_k - e_i| + 2 (its heavy part)
// as 16-bit halves, three packed saturating subtracts give two digits each:
// (4, 4) - tr is (R7, R5), tr - (|e_i ∩ e_k|, k's outside count) is
// (R6, R3), tr - (pj, oj) is (R4, R2).  R1 = aks - pj + t (aks = |e_i| -
// |e_i ∩ e_k|) enters doubled, from 2 (t + 2) + aks2 with aks2 = 2 aks - 4,
// as the start of three two-term dot products that add 2 (3^6 R7 + ...)
// pair by pair.
// jy is j's record word: pj in bits 0-7, 2 pj + 4 in bits 8-15, oj in bits
// 16-23; kso = k.s | k.o << 16.
__device__ __forceinline__ uint32_t pair_rcode2(uint32_t t2, uint32_t tr, uint32_t aks2, uint32_t jy,
                                                uint32_t kso) {
  const uint32_t pjo = jy & 0x00ff00ffu, pj24 = (jy >> 8) & 0xffu;
  uint32_t v2;  // 2 (aks + t) = 2 t2 + aks2, one shift-add
  asm("v_lshl_add_u32 %0, %1, 1, %2" : "=v"(v2) : "v"(t2), "v"(aks2));
  const uint32_t d75 = pk_usat_sv(0x00040004u, tr);     // (R7, R5)
  const uint32_t d63 = pk_usat_vv(tr, kso);             // (R6, R3)
  const uint32_t d42 = pk_usat_vs(tr, pjo);             // (R4, R2)
  uint32_t c = usat(pj24, v2);                          // 2 R1
  c = dot2(d42, 54u | (6u << 16), c);
  c = dot2(d63, 486u | (18u << 16), c);
  return dot2(d75, 1458u | (162u << 16), c);
}

// t + 2 and r5 + 2 of a pair from its mask intersections (population counts
// with the constant added in the same instruction; r5 over two words).
// tr = (t + 2) | (r5 + 2) << 16.
__device__ __forceinline__ void pair_counts(uint32_t xm, uint32_t xl, uint32_t xh, uint32_t& t2, uint32_t& tr) {
  t2 = uint32_t(__popc(xm)) + 2u;
  uint32_t r2;
  asm("v_bcnt_u32_b32 %0, %1, 2\n\tv_bcnt_u32_b32 %0, %2, %0" : "=&v"(r2) : "v"(xl), "v"(xh));
  asm("v_lshl_or_b32 %0, %1, 16, %2" : "=v"(tr) : "v"(r2), "v"(t2));
}

// The histogram word at a byte offset the class table gives.
__device__ __forceinline__ unsigned long long* hist_at(unsigned long long* hist, uint32_t off) {
  return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(hist) + off);
}

// The class table entry at a byte offset.
__device__ __forceinline__ uint32_t lut_at(const uint16_t* __restrict__ lut, uint32_t off2) {
  return *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(lut) + off2);
}

// Every row is shorter than 2^24 (a graph has at most 200000 hyperedges), so
// a weight is a product of two 24-bit counts (two full-rate multiplies
// instead of a 64-bit one).  A disjoint pair (open at the centre) weighs nall_j * nall_k, an
// overlapping one nabove_j * nabove_k.  gwalk walks only groups j with
// members above the centre (they come first in a row), so the selected lane
// count is zero exactly when the pair weighs nothing (every group holds at
// least one neighbour, and kn = 0 on lanes past the row).
// kAllA: every lane's group and j have members above the centre, so every
// pair weighs at least 1 (N_j N_k or A_j A_k): no test and no branch (a lane
// past the row's end has N = A = 0 and adds 0 at a valid class).
// kNarrow: every row is shorter than 2^16 neighbours, so the group counts
// fit 16 bits and the weight of a pair of distinct groups, at most (row
// length / 2)^2, fits 32 bits: one 24-bit multiply (its high half is zero),
// or, in the full-class loop, a two-term dot product of the packed counts.
template <bool kNarrow>
__device__ __forceinline__ uint64_t pair_weight(uint32_t x, uint32_t y) {
  return kNarrow ? uint64_t(x * y) : uint64_t(x) * y;
}

template <bool kDiag, bool kAllA, bool kNarrow>
__device__ __forceinline__ void gpair_step(const uint4& rj, const uint2& cj, int j, uint32_t aks2,
                                           const Side& k, uint32_t khl, uint32_t khh, uint32_t kso,
                                           uint32_t kn, uint32_t ka, int kp, const uint16_t* __restrict__ lut,
                                           unsigned long long* hist) {
  const uint32_t mj = rj.x;
  const uint32_t xm = mj & k.m, xl = rj.z & khl, xh = rj.w & khh;
  uint32_t t2, tr;
  pair_counts(xm, xl, xh, t2, tr);
  const bool disjoint = tr == 0x00020002u;  // t = r5 = 0
  // j's counts arrive in vector registers (gwalk loads them per lane), so
  // the selects below need no copies of scalar values
  const uint32_t y = disjoint ? kn : ka;
  const uint32_t nab = kNarrow ? (cj.y & 0xffffu) : cj.y;  // nabove_j
  if (kAllA && !kDiag) {
    const uint32_t x = (disjoint ? cj.x : nab) & 0xffffffu;
    const uint32_t rc2 = pair_rcode2(t2, tr, aks2, rj.y, kso);
    atomicAdd(hist_at(hist, lut_at(lut, rc2)), pair_weight<kNarrow>(x, y));
    return;
  }
  bool act = y != 0u;
  if (kDiag) act = act && (j < kp);
  if (act) {
    const uint32_t x = (disjoint ? cj.x : nab) & 0xffffffu;
    const uint64_t w = pair_weight<kNarrow>(x, y);
    const uint32_t rc2 = pair_rcode2(t2, tr, aks2, rj.y, kso);
    atomicAdd(hist_at(hist, lut_at(lut, rc2)), w);
  }
}

// A full-class pair's class table offset and weight (every lane's group and
// j with members above the centre).
// kNarrow: j's second count word holds (nabove_j, nall_j) as 16-bit halves,
// so the weight is one dot product with the lane's (0, N_k) or (A_k, 0).
template <bool kNarrow>
__device__ __forceinline__ void pair_full(const uint4& rj, const uint2& cj, uint32_t aks2, const Side& k,
                                          uint32_t khl, uint32_t khh, uint32_t kso, uint32_t kn,
                                          uint32_t ka, uint32_t kn16, uint32_t& rc2, uint64_t& w) {
  const uint32_t xm = rj.x & k.m, xl = rj.z & khl, xh = rj.w & khh;
  uint32_t t2, tr;
  pair_counts(xm, xl, xh, t2, tr);
  const bool disjoint = tr == 0x00020002u;  // t = r5 = 0
  rc2 = pair_rcode2(t2, tr, aks2, rj.y, kso);
  if (kNarrow) {
    w = dot2_vv(cj.y, disjoint ? kn16 : ka);
  } else {
    const uint32_t y = disjoint ? kn : ka;
    const uint32_t x = (disjoint ? cj.x : cj.y) & 0xffffffu;
    w = pair_weight<kNarrow>(x, y);
  }
}

template <bool kDiag, bool kAllA, bool kNarrow>
__device__ __forceinline__ void gwalk(const uint4* __restrict__ grow, const uint2* __restrict__ gc0,
                                      int j0, int j1, uint32_t aks, const Side& k, uint32_t kn,
                                      uint32_t ka, int kp, const uint16_t* __restrict__ lut,
                                      unsigned long long* hist) {
  const uint32_t khl = uint32_t(k.h), khh = uint32_t(k.h >> 32);
  // a lane-held zero makes the count loads vector loads (one 8-byte word
  // broadcast to every lane) instead of scalar loads
  int z = 0;
  asm volatile("" : "+v"(z));
  const uint2* gc = gc0 + z;
  const uint32_t aks2 = 2u * aks - 4u;
  const uint32_t kso = k.s | (k.o << 16);
  const uint32_t kn16 = kn << 16;
  int j = j0;
  if (kAllA && !kDiag) {
    // four pairs at a time: the four class table reads are issued together
    // and waited for once, then the four histogram adds
    for (; j + 4 <= j1; j += 4) {
      const uint4 r0 = grow[j], r1 = grow[j + 1], r2 = grow[j + 2], r3 = grow[j + 3];
      const uint2 c0 = gc[j], c1 = gc[j + 1], c2 = gc[j + 2], c3 = gc[j + 3];
      uint32_t o0, o1, o2, o3;
      uint64_t w0, w1, w2, w3;
      pair_full<kNarrow>(r0, c0, aks2, k, khl, khh, kso, kn, ka, kn16, o0, w0);
      pair_full<kNarrow>(r1, c1, aks2, k, khl, khh, kso, kn, ka, kn16, o1, w1);
      pair_full<kNarrow>(r2, c2, aks2, k, khl, khh, kso, kn, ka, kn16, o2, w2);
      pair_full<kNarrow>(r3, c3, aks2, k, khl, khh, kso, kn, ka, kn16, o3, w3);
      o0 = lut_at(lut, o0);
      o1 = lut_at(lut, o1);
      o2 = lut_at(lut, o2);
      o3 = lut_at(lut, o3);
      atomicAdd(hist_at(hist, o0), w0);
      atomicAdd(hist_at(hist, o1), w1);
      atomicAdd(hist_at(hist, o2), w2);
      atomicAdd(hist_at(hist, o3), w3);
    }
  } else {
    for (; j + 4 <= j1; j += 4) {
      const uint4 r0 = grow[j], r1 = grow[j + 1], r2 = grow[j + 2], r3 = grow[j + 3];
      const uint2 c0 = gc[j], c1 = gc[j + 1], c2 = gc[j + 2], c3 = gc[j + 3];
      gpair_step<kDiag, kAllA, kNarrow>(r0, c0, j, aks2, k, khl, khh, kso, kn, ka, kp, lut, hist);
      gpair_step<kDiag, kAllA, kNarrow>(r1, c1, j + 1, aks2, k, khl, khh, kso, kn, ka, kp, lut, hist);
      gpair_step<kDiag, kAllA, kNarrow>(r2, c2, j + 2, aks2, k, khl, khh, kso, kn, ka, kp, lut, hist);
      gpair_step<kDiag, kAllA, kNarrow>(r3, c3, j + 3, aks2, k, khl, khh, kso, kn, ka, kp, lut, hist);
    }
  }
  for (; j < j1; ++j)
    gpair_step<kDiag, kAllA, kNarrow>(grow[j], gc[j], j, aks2, k, khl, khh, kso, kn, ka, kp, lut, hist);
}

// A pair in which one group has no member above the centre counts only when
// open at the centre (disjoint), with weight nall_j * nall_k and t = r5 = 0:
// its code is k0 (the lane's digits R6, R3) + j's digits R4, R2 + st3(|e_i|
// - k.s - pj) (R1), so j enters only through its open class (pj, st3(oj)).
// The groups are ordered by open class within each hash part, so each lane
// sums nall_j over a run of one class and adds sum * nall_k to the
// histogram when the class changes.
__device__ __forceinline__ void open_flush(uint32_t cls, uint32_t acc, uint32_t aks, uint32_t k0,
                                           uint32_t kn, const uint16_t* __restrict__ lut,
                                           unsigned long long* hist) {
  if (acc != 0u && kn != 0u) {
    const uint32_t pj = cls / 3u, oc = cls - 3u * pj;
    const uint32_t code = k0 + 27u * st3(pj) + 3u * oc + st3(aks - pj);
    atomicAdd(hist_at(hist, lut[kNumCodes - 1 - code]), uint64_t(acc) * kn);
  }
}

// (a & b) | c in one instruction, a taken from a scalar register.
__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "s"(a), "v"(b), "v"(c));
  return r;
}

// acc += n if x = 0 (n < 2^24, from a scalar register): max(1 - x, 0), a
// saturating subtract (a full-rate instruction, unlike a minimum), and a
// 24-bit multiply-add, written as instructions so that they are not turned
// into a compare and a select.
__device__ __forceinline__ void acc_disjoint(uint32_t& acc, uint32_t x, uint32_t n) {
  uint32_t z;
  asm("v_sub_u32_e64 %1, 1, %2 clamp\n\tv_mad_u32_u24 %0, %1, %3, %0" : "+v"(acc), "=&v"(z) : "v"(x), "s"(n));
}

// Lanes past the diagonal block sum nall_j over the j of a run that are
// disjoint from the lane's group, as max(1 - overlap bits, 0) * nall_j (a
// saturating subtract and a multiply-add).  The diagonal block (j < k
// only) adds per lane.
template <bool kDiag>
__device__ __forceinline__ void open_step(const uint4& rj, const uint2& cj, int j, const Side& k,
                                          uint32_t khl, uint32_t khh, uint32_t kn, int kp,
                                          uint32_t aks, uint32_t k0, uint32_t& cur, uint32_t& acc,
                                          const uint16_t* __restrict__ lut,
                                          unsigned long long* hist) {
  const uint32_t cls = rj.y >> 24;  // uniform: the open class the grouping stored
  if (cls != cur) {
    open_flush(cur, acc, aks, k0, kn, lut, hist);
    cur = cls;
    acc = 0u;
  }
  if (kDiag) {
    bool act = ((rj.x & k.m) | (rj.z & khl) | (rj.w & khh)) == 0u && kn != 0u;
    act = act && (j < kp);
    if (act) acc += cj.x;
  } else {
    const uint32_t x = and_or(rj.w, khh, and_or(rj.z, khl, rj.x & k.m));
    acc_disjoint(acc, x, cj.x);
  }
}

template <bool kDiag>
__device__ __forceinline__ void owalk(const uint4* __restrict__ grow, const uint2* __restrict__ gc,
                                      int j0, int j1, uint32_t aks, uint32_t k0, const Side& k,
                                      uint32_t kn, int kp, const uint16_t* __restrict__ lut,
                                      unsigned long long* hist) {
  const uint32_t khl = uint32_t(k.h), khh = uint32_t(k.h >> 32);
  uint32_t cur = 0u, acc = 0u;
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
    const uint4 r0 = grow[j], r1 = grow[j + 1], r2 = grow[j + 2], r3 = grow[j + 3];
    const uint2 c0 = gc[j], c1 = gc[j + 1], c2 = gc[j + 2], c3 = gc[j + 3];
    open_step<kDiag>(r0, c0, j, k, khl, khh, kn, kp, aks, k0, cur, acc, lut, hist);
    open_step<kDiag>(r1, c1, j + 1, k, khl, khh, kn, kp, aks, k0, cur, acc, lut, hist);
    open_step<kDiag>(r2, c2, j + 2, k, khl, khh, kn, kp, aks, k0, cur, acc, lut, hist);
    open_step<kDiag>(r3, c3, j + 3, k, khl, khh, kn, kp, aks, k0, cur, acc, lut, hist);
  }
  for (; j < j1; ++j)
    open_step<kDiag>(grow[j], gc[j], j, k, khl, khh, kn, kp, aks, k0, cur, acc, lut, hist);
  open_flush(cur, acc, aks, k0, kn, lut, hist);
}

__device__ __forceinline__ void gflush_wave(unsigned long long* whist, int lane, int64_t g,
                                            unsigned long long* hist_out) {
  __builtin_amdgcn_wave_barrier();
  for (int t = lane; t < kHistSlots; t += kWave) {
    unsigned long long s = 0;
    for (int c = 0; c < kGCopies; ++c) {
      s += whist[c * kGStride + t];
      whist[c * kGStride + t] = 0ull;
    }
    if (s) atomicAdd(&hist_out[g * kHistSlots + t], s);
  }
  __builtin_amdgcn_wave_barrier();
}

// kShared (one graph per launch: a single graph, or one graph of a batch of
// large graphs): 512-thread blocks whose 8 histogram copies are shared by
// their waves, lane l adding to copy l % 8, flushed once at the end: 32 KB of
// LDS per block, so 4 blocks (32 waves, as many as the registers allow) fit
// on a CU.  Lanes of one add that hit the same word are serialized, so the
// copies count: on the medium workload the pair kernel took 556 ms with 2
// copies and 448 ms with 4 (256-thread blocks), 434 ms with 8 (512-thread
// blocks), 538 ms with 16 (1024-thread blocks, 2 per CU), and 853 ms with a
// single histogram over the 2187 codes (no class table read).  Otherwise
// (kShared false) each wave has 2 copies of its own, flushed whenever its
// rows change graph.
constexpr int kGSharedCopies = 8;
constexpr int kGSharedThreads = 512;
// batches of up to this many graphs whose graphs average a full grid of
// work items count each graph with its own launch of the shared-histogram
// kernel; others use per-wave histograms in one launch
constexpr int kPerGraphLaunches = 256;
// At most 100 scalar registers for the shared-histogram kernel, so that a
// SIMD holds 8 of its waves (4 blocks of 512 threads per compute unit, the
// default launch); its loops left to themselves take 106 registers, which
// allow 7 waves per SIMD and so only 3 blocks per compute unit (measured on
// medium: 403 ms at 3 blocks, 360 ms at 4).  The per-wave-histogram kernel
// is held to 5 waves per SIMD by its shared memory anyway.
template <bool kShared, bool kNarrow>
__global__ __launch_bounds__(kShared ? kGSharedThreads : 256)
__attribute__((amdgpu_waves_per_eu(kShared ? 8 : 5, 8))) void k_exact_grouped(
    const int64_t* __restrict__ edge_ptr, const int64_t* __restrict__ goff,
    const int64_t* __restrict__ gbase, int64_t cap0,
    const uint4* __restrict__ grec, const uint2* __restrict__ gcnt, const int32_t* __restrict__ gna,
    const int32_t* __restrict__ order, const int64_t* __restrict__ rstart, int64_t nslots,
    int64_t item0, int64_t item1, const int32_t* __restrict__ row_graph, unsigned long long* queue,
    const uint16_t* __restrict__ code_to_id3, unsigned long long* hist_out) {
  __shared__ uint16_t lut[kNumCodes];
  constexpr int kAll = kShared ? kGSharedCopies : kWavesPerGroup * kGCopies;
  __shared__ unsigned long long hist[kAll * kGStride];
  // indexed by the reversed code; entries are byte offsets of the ids
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = uint16_t(code_to_id3[kNumCodes - 1 - t] * 8u);
  for (int t = threadIdx.x; t < kAll * kGStride; t += blockDim.x) hist[t] = 0ull;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  unsigned long long* whist = kShared ? hist : hist + wave * (kGCopies * kGStride);  // per-wave copies only
  unsigned long long* myhist = kShared ? hist + (lane & (kAll - 1)) * kGStride
                                       : whist + (lane & (kGCopies - 1)) * kGStride;
  const int64_t total = item1 >= 0 ? item1 : rstart[nslots];  // items [item0, total)
  int dirty_g = -1;
  for (;;) {
    unsigned long long qq = 0;
    if (lane == 0) qq = atomicAdd(queue, 1ull);
    const int64_t q = item0 + (int64_t)(((unsigned long long)__builtin_amdgcn_readfirstlane(int(qq >> 32)) << 32) |
                                        (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(int(qq)));
    if (q >= total) break;
    int64_t lo = 0, hi = nslots;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (rstart[mid] <= q) lo = mid; else hi = mid;
    }
    const int32_t i = order[lo];
    const int g = kShared ? 0 : row_graph[i];
    if (!kShared && dirty_g >= 0 && dirty_g != g) gflush_wave(whist, lane, dirty_g, hist_out);
    dirty_g = g;
    const int nbi = int(rstart[lo + 1] - rstart[lo]);
    const int b = nbi - 1 - int(q - rstart[lo]);
    const int64_t gb = gbase[i] - cap0;
    const int ng = int(goff[i + 1] - goff[i]);
    // groups with members above the centre at [0, na), the others at
    // [na, ng) + gap (gap = the row region's unused middle)
    const int na = gna[i];
    const int64_t gap = (gbase[i + 1] - gbase[i]) - ng;
    const uint32_t a = uint32_t(edge_ptr[i + 1] - edge_ptr[i]);
    const uint4* __restrict__ grow = grec + gb;
    const uint2* __restrict__ gc = gcnt + gb;
    const uint4* __restrict__ growb = grow + gap;
    const uint2* __restrict__ gcb = gc + gap;
    const int kp = b * kWave + lane;
    const bool valid = kp < ng;
    Side k;
    uint32_t kn = 0, ka = 0;
    {
      const int64_t kpos = kp < na ? int64_t(kp) : kp + gap;
      const uint4 rk = valid ? grow[kpos] : make_uint4(0, 0, 0, 0);
      const uint2 ck = valid ? gc[kpos] : make_uint2(0, 0);
      k.m = rk.x;
      k.o = (rk.y >> 16) & 0xffu;
      k.s = __popc(rk.x);
      k.h = (unsigned long long)rk.z | ((unsigned long long)rk.w << 32);
      kn = ck.x;
      ka = ck.y;
    }
    kn &= 0xffffffu;
    ka &= kNarrow ? 0xffffu : 0xffffffu;  // packed: (nabove, nall) halves
    const int blo = b * kWave;
    const int kmax = min(blo + kWave, ng);
    const uint32_t aks = a - k.s;
    const uint32_t k0 = 243u * st3(k.s) + 9u * st3(k.o);
    if (blo >= na) {  // no lane has members above the centre: open pairs only
      owalk<false>(grow, gc, 0, na, aks, k0, k, kn, kp, lut, myhist);
      owalk<false>(growb, gcb, na, blo, aks, k0, k, kn, kp, lut, myhist);
      owalk<true>(growb, gcb, blo, kmax, aks, k0, k, kn, kp, lut, myhist);
    } else if (blo + kWave <= na) {  // every lane has members above the centre
      gwalk<false, true, kNarrow>(grow, gc, 0, blo, aks, k, kn, ka, kp, lut, myhist);
      gwalk<true, false, kNarrow>(grow, gc, blo, kmax, aks, k, kn, ka, kp, lut, myhist);
    } else {  // j with members above the centre: every pair; the others: open only
      const int ka1 = min(kmax, na);
      gwalk<false, false, kNarrow>(grow, gc, 0, blo, aks, k, kn, ka, kp, lut, myhist);
      gwalk<true, false, kNarrow>(grow, gc, blo, ka1, aks, k, kn, ka, kp, lut, myhist);
      owalk<true>(growb, gcb, ka1, kmax, aks, k0, k, kn, kp, lut, myhist);
    }
    if (valid && ka >= 2u) {  // pairs inside the group: above the centre only
      const uint32_t r5 = uint32_t(__popcll(k.h));
      const uint32_t code = pair_code(a, k.s, k.o, k, k.s, r5);
      atomicAdd(hist_at(myhist, lut[kNumCodes - 1 - code]), uint64_t(ka) * (ka - 1u) / 2u);
    }
  }
  if (kShared) {
    __syncthreads();
    for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x) {
      unsigned long long v = 0;
      for (int c = 0; c < kAll; ++c) v += hist[c * kGStride + t];
      if (v) atomicAdd(&hist_out[t], v);
    }
  } else if (dirty_g >= 0) {
    gflush_wave(whist, lane, dirty_g, hist_out);
  }
}

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

}  // namespace

namespace {

// Work list of (row, 64-block) items over rows [c0, c1) of row_ptr (rows
// shorter than min_len have no pairs); see the scheduling kernels above.
struct Schedule {
  char* scratch = nullptr;
  int32_t* order = nullptr;
  int64_t* rstart = nullptr;
  unsigned long long* queue = nullptr;
  int64_t* gq = nullptr;  // [ng + 1] first item of each graph
  int64_t rows = 0;
};

mochy_status build_schedule(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                            const int64_t* row_ptr, int64_t min_len, Schedule& S) {
  hipStream_t st = ctx->stream;
  const int ng = g->ng;
  const int32_t maxnb = (g->max_deg + kWave - 1) / kWave;
  const int64_t NB = maxnb + 1;
  const int64_t rows = c1 - c0;
  // scratch (8-byte slots): nbhist, cnt, item_start, fill [ng*NB each], total [ng],
  // gq [ng+1], seg [ng], queue [1], nbk [rows+1], rstart [rows+1], tmp; then order [rows] int32
  const size_t tmpn = scan_tmp_elems(rows + 1);
  const size_t n8 = size_t(ng) * NB * 4 + size_t(ng) * 3 + 2 + size_t(rows + 1) * 2 + tmpn;
  mochy_status rc = device_alloc(ctx, (void**)&S.scratch, n8 * 8 + size_t(rows) * 4);
  if (rc != MOCHY_OK) return rc;
  unsigned long long* nbhist = (unsigned long long*)S.scratch;
  int64_t* cnt = (int64_t*)(nbhist + ng * NB);
  int64_t* item_start = cnt + ng * NB;
  unsigned long long* fill = (unsigned long long*)(item_start + ng * NB);
  int64_t* total = (int64_t*)(fill + ng * NB);
  int64_t* gq = total + ng;
  S.gq = gq;
  int64_t* seg = gq + (ng + 1);
  S.queue = (unsigned long long*)(seg + ng);
  int64_t* nbk = (int64_t*)(S.queue + 1);
  S.rstart = nbk + (rows + 1);
  int64_t* tmp = S.rstart + (rows + 1);
  S.order = (int32_t*)(S.scratch + n8 * 8);
  S.rows = rows;
  launch_fill_u32(S.scratch, 0u, (size_t(ng) * NB * 4 + size_t(ng) * 3 + 2) * 8, st);
  launch_fill_u32(S.order, 0xffffffffu, size_t(rows) * 4, st);
  k_sched_count<<<blocks(rows, 256), 256, 0, st>>>(c0, c1, int32_t(NB), row_ptr, min_len, g->row_graph,
                                                   nbhist);
  k_sched_scan<<<unsigned(ng), 1024, 0, st>>>(maxnb, nbhist, cnt, item_start, total);
  k_sched_graphs<<<1, 1024, 0, st>>>(ng, c0, c1, g->geoff, total, gq, seg);
  k_sched_scatter<<<blocks(rows, 256), 256, 0, st>>>(c0, c1, int32_t(NB), row_ptr, min_len,
                                                     g->row_graph, cnt, seg, fill, S.order);
  k_item_counts<<<blocks(rows + 1, 256), 256, 0, st>>>(rows, S.order, row_ptr, nbk);
  launch_exclusive_scan_i64(nbk, S.rstart, rows + 1, tmp, st);
  return MOCHY_OK;
}

// Groups of rows [c0, c1): goff[E+1] the prefix of the rows' group counts,
// row i's groups in grec / gcnt [gbase[i] - cap0, gbase[i + 1] - cap0): the
// gna[i] with members above the centre first, the others at the region's
// end (the region holds exactly the groups in the compact layout).  With up
// to ctx->group_cap_bytes of row capacity (a graph or a whole batch), one
// pass writes each row's groups at its line-graph offset (gbase = lg_ptr);
// otherwise, or if that capacity cannot be allocated, the groups are counted
// first and allocated exactly (gbase = goff, cap0 = 0).  Returns MOCHY_ENOMEM (nothing held) if
// the group arrays do not fit or a row could not be grouped; the caller then
// pairs every record.
mochy_status build_groups(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                          int64_t** goff, uint4** grec, uint2** gcnt, int32_t** gna,
                          const int64_t** gbase, int64_t* cap0, unsigned long long* stats, bool pack16) {
  hipStream_t st = ctx->stream;
  const int64_t E = g->E;
  int64_t* cntarr = nullptr;
  int64_t* tmp = nullptr;
  int32_t* longrows = nullptr;
  *goff = nullptr;
  *grec = nullptr;
  *gcnt = nullptr;
  *gna = nullptr;
  auto fail = [&](mochy_status rc) {
    device_free(ctx, cntarr);
    device_free(ctx, tmp);
    device_free(ctx, longrows);
    device_free(ctx, *goff);
    device_free(ctx, *grec);
    device_free(ctx, *gcnt);
    device_free(ctx, *gna);
    *goff = nullptr;
    *grec = nullptr;
    *gcnt = nullptr;
    *gna = nullptr;
    return rc;
  };
  MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small, g->lg_ptr + c0, 8, hipMemcpyDeviceToHost, st), fail);
  MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small + 1, g->lg_ptr + c1, 8, hipMemcpyDeviceToHost, st), fail);
  MOCHY_HIP_OR(hipStreamSynchronize(st), fail);
  const int64_t row0 = ctx->h_small[0];
  const int64_t cap = ctx->h_small[1] - row0;
  // one pass into row capacity (a graph or a batch) when that fits the limit
  bool by_rows = cap * 24 <= ctx->group_cap_bytes;
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&cntarr, size_t(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&tmp, scan_tmp_elems(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)goff, size_t(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)gna, size_t(std::max<int64_t>(E, 1)) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&longrows, size_t(std::max<int64_t>(c1 - c0, 1)) * 4)) != MOCHY_OK)
    return fail(rc);
  launch_fill_u32(cntarr, 0u, size_t(E + 1) * 8, st);
  launch_fill_u32(ctx->d_flags + 3, 0u, 4, st);
  // the rows too long for the short-row table, listed once; two queue
  // counters (one per grouping pass), all in the context's small scratch
  unsigned long long* nlong = (unsigned long long*)(ctx->d_small + 508);
  unsigned long long* lqueue = nlong + 1;  // [2]
  launch_fill_u32(nlong, 0u, 3 * 8, st);
  if (c1 > c0) k_long_rows<<<blocks(c1 - c0, 256), 256, 0, st>>>(c0, c1, g->lg_ptr, longrows, nlong);
  const unsigned lgrid = unsigned(ctx->num_cus);  // one 160 KB block per CU
  if (by_rows && ((ctx->test_faults & 1) ||
                  device_alloc(ctx, (void**)grec, size_t(std::max<int64_t>(cap, 1)) * 16) != MOCHY_OK ||
                  device_alloc(ctx, (void**)gcnt, size_t(std::max<int64_t>(cap, 1)) * 8) != MOCHY_OK)) {
    // no room for the row capacity: count the groups first and allocate them exactly
    device_free(ctx, *grec);
    device_free(ctx, *gcnt);
    *grec = nullptr;
    *gcnt = nullptr;
    ctx->err.clear();
    by_rows = false;
  }
  if (by_rows) {
    *gbase = g->lg_ptr;
    *cap0 = row0;
    if (c1 > c0) {
      k_group_short<true><<<unsigned(c1 - c0), kShortThreads, 0, st>>>(
          c0, g->lg_ptr, g->up_first, g->rec, cntarr, g->lg_ptr, row0, *grec, *gcnt, *gna, ctx->d_flags + 3, stats,
          pack16);
      k_group_long<true><<<lgrid, kLongThreads, 0, st>>>(longrows, nlong, lqueue, g->lg_ptr, g->up_first, g->rec,
                                                         cntarr, g->lg_ptr, row0, *grec, *gcnt, *gna,
                                                         ctx->d_flags + 3, stats, pack16);
    }
    launch_exclusive_scan_i64(cntarr, *goff, E + 1, tmp, st);
  } else {
    *gbase = *goff;
    *cap0 = 0;
    if (c1 > c0) {
      k_group_short<false><<<unsigned(c1 - c0), kShortThreads, 0, st>>>(
          c0, g->lg_ptr, g->up_first, g->rec, cntarr, nullptr, 0, nullptr, nullptr, nullptr, ctx->d_flags + 3,
          stats, pack16);
      k_group_long<false><<<lgrid, kLongThreads, 0, st>>>(longrows, nlong, lqueue, g->lg_ptr, g->up_first,
                                                          g->rec, cntarr, nullptr, 0, nullptr, nullptr, nullptr,
                                                          ctx->d_flags + 3, stats, pack16);
    }
    launch_exclusive_scan_i64(cntarr, *goff, E + 1, tmp, st);
    MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small, *goff + E, 8, hipMemcpyDeviceToHost, st), fail);
    MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small + 1, ctx->d_flags + 3, 4, hipMemcpyDeviceToHost, st), fail);
    MOCHY_HIP_OR(hipStreamSynchronize(st), fail);
    if (*reinterpret_cast<int32_t*>(ctx->h_small + 1) != 0) return fail(MOCHY_ENOMEM);
    const int64_t ngroups = ctx->h_small[0];
    if ((rc = device_alloc(ctx, (void**)grec, size_t(std::max<int64_t>(ngroups, 1)) * 16)) != MOCHY_OK ||
        (rc = device_alloc(ctx, (void**)gcnt, size_t(std::max<int64_t>(ngroups, 1)) * 8)) != MOCHY_OK)
      return fail(rc);
    // the same grouping again, written this time (its parts were reported above)
    if (c1 > c0) {
      k_group_short<true><<<unsigned(c1 - c0), kShortThreads, 0, st>>>(
          c0, g->lg_ptr, g->up_first, g->rec, nullptr, *goff, 0, *grec, *gcnt, *gna, ctx->d_flags + 3, nullptr,
          pack16);
      k_group_long<true><<<lgrid, kLongThreads, 0, st>>>(longrows, nlong, lqueue + 1, g->lg_ptr, g->up_first,
                                                         g->rec, nullptr, *goff, 0, *grec, *gcnt, *gna,
                                                         ctx->d_flags + 3, nullptr, pack16);
    }
  }
  if (c1 > c0)
    k_group_stats<<<blocks(c1 - c0, 256), 256, 0, st>>>(c0, c1, *goff, *gna, stats);
  MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small + 1, ctx->d_flags + 3, 4, hipMemcpyDeviceToHost, st), fail);
  MOCHY_HIP_OR(hipStreamSynchronize(st), fail);
  if (*reinterpret_cast<int32_t*>(ctx->h_small + 1) != 0) return fail(MOCHY_ENOMEM);
  device_free(ctx, cntarr);
  device_free(ctx, tmp);
  device_free(ctx, longrows);
  cntarr = nullptr;
  tmp = nullptr;
  longrows = nullptr;
  MOCHY_HIP_OR(hipGetLastError(), fail);
  return MOCHY_OK;
}

}  // namespace

mochy_status exact_device(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                          int64_t* d_hist) {
  hipStream_t st = ctx->stream;
  const int ng = g->ng;
  unsigned long long* stats = (unsigned long long*)(ctx->d_small + kExactStatsSlot);
  launch_fill_u32(d_hist, 0u, size_t(ng) * kHistSlots * 8, st);
  launch_fill_u32(stats, 0u, kStBatches * 8, st);
  if (c1 <= c0 || g->max_deg < 2) return MOCHY_OK;
  if (g->max_deg >= (1 << 24)) {  // group sizes are multiplied as 24-bit numbers
    ctx->err = "a line-graph row of 2^24 or more neighbours";
    return MOCHY_EUNSUPPORTED;
  }
  const unsigned grid = unsigned(ctx->num_cus) * unsigned(ctx->pair_blocks);
  // the shared-histogram kernel's blocks are kGSharedThreads wide: as many
  // waves in flight as `grid` blocks of 256
  constexpr int kSharedWaves = kGSharedThreads / kWave;
  const unsigned sgrid = std::max(1u, grid * 256u / unsigned(kGSharedThreads));
  int64_t* goff = nullptr;
  const int64_t* gbase = nullptr;
  int64_t cap0 = 0;
  uint4* grec = nullptr;
  uint2* gcnt = nullptr;
  int32_t* gna = nullptr;
  unsigned long long* gqueue = nullptr;
  mochy_status rc;
  phase_begin(ctx, kPhSched);
  // rows shorter than 2^16 neighbours: the group counts fit 16 bits and a
  // pair's weight (below 2^32) is a two-term dot product of packed counts
  // (test bit 4 takes the 48-bit form regardless)
  const bool narrow = g->max_deg < (1 << 16) && !(ctx->test_faults & 16);
  bool grouped = ctx->group_neighbours;
  if (grouped) {
    rc = (ctx->test_faults & 4) && ng > 2
             ? MOCHY_ENOMEM  // forced for tests of the batch split
             : build_groups(ctx, g, c0, c1, &goff, &grec, &gcnt, &gna, &gbase, &cap0, stats, narrow);
    if (rc == MOCHY_ENOMEM && ng > 1) {
      return rc;  // a batch: the caller splits it and counts the parts with groups
    } else if (rc == MOCHY_ENOMEM) {  // not enough memory for one graph's groups: pair every record
      grouped = false;
      ctx->err.clear();
      launch_fill_u32(stats, 0u, kStBatches * 8, st);
    } else if (rc != MOCHY_OK) {
      return rc;
    }
  }
  Schedule S;
  auto release = [&](mochy_status s) {
    device_free(ctx, S.scratch);
    device_free(ctx, goff);
    device_free(ctx, grec);
    device_free(ctx, gcnt);
    device_free(ctx, gna);
    device_free(ctx, gqueue);
    S.scratch = nullptr;
    goff = nullptr;
    grec = nullptr;
    gcnt = nullptr;
    gna = nullptr;
    gqueue = nullptr;
    return s;
  };
  rc = build_schedule(ctx, g, c0, c1, grouped ? goff : g->lg_ptr, grouped ? 1 : 2, S);
  if (rc != MOCHY_OK) return release(rc);
  phase_end(ctx, kPhSched);
  phase_begin(ctx, kPhPairs);
  // a batch of graphs large enough to fill the device each: the
  // shared-histogram kernel once per graph (a graph's items are contiguous in
  // the schedule), each launch with its own queue counter; smaller graphs are
  // counted together in one launch, which keeps their tails overlapped
  // (MOCHY_OPT_BATCH_LAUNCH can force either form)
  std::vector<int64_t> hgq;
  if (grouped && ng > 1 && ng <= kPerGraphLaunches && ctx->batch_launch != 1) {
    hgq.resize(size_t(ng) + 1);
    MOCHY_HIP_OR(hipMemcpyAsync(hgq.data(), S.gq, hgq.size() * 8, hipMemcpyDeviceToHost, st), release);
    MOCHY_HIP_OR(hipStreamSynchronize(st), release);
    if (ctx->batch_launch == 0 && hgq[ng] < int64_t(ng) * grid * kWavesPerGroup) hgq.clear();
  }
  const auto kshared = narrow ? k_exact_grouped<true, true> : k_exact_grouped<true, false>;
  if (!hgq.empty()) {
    if ((rc = device_alloc(ctx, (void**)&gqueue, size_t(ng) * 8)) != MOCHY_OK) return release(rc);
    launch_fill_u32(gqueue, 0u, size_t(ng) * 8, st);
    for (int gi = 0; gi < ng; ++gi) {
      const int64_t items = hgq[gi + 1] - hgq[gi];
      if (items <= 0) continue;
      // at most one wave per item
      const unsigned ggrid = unsigned(std::min<int64_t>(sgrid, (items + kSharedWaves - 1) / kSharedWaves));
      kshared<<<ggrid, kGSharedThreads, 0, st>>>(
          g->edge_ptr, goff, gbase, cap0, grec, gcnt, gna, S.order, S.rstart, S.rows, hgq[gi], hgq[gi + 1],
          g->row_graph, gqueue + gi, ctx->d_code_to_id3, (unsigned long long*)d_hist + size_t(gi) * kHistSlots);
    }
  } else if (grouped) {
    if (ng == 1)
      kshared<<<sgrid, kGSharedThreads, 0, st>>>(
          g->edge_ptr, goff, gbase, cap0, grec, gcnt, gna, S.order, S.rstart, S.rows, 0, -1, g->row_graph,
          S.queue, ctx->d_code_to_id3, (unsigned long long*)d_hist);
    else
      (narrow ? k_exact_grouped<false, true> : k_exact_grouped<false, false>)<<<grid, 256, 0, st>>>(
          g->edge_ptr, goff, gbase, cap0, grec, gcnt, gna, S.order, S.rstart, S.rows, 0, -1, g->row_graph,
          S.queue, ctx->d_code_to_id3, (unsigned long long*)d_hist);
  } else {
    k_exact_main<<<grid, 256, 0, st>>>(g->edge_ptr, g->lg_ptr, g->up_first, g->rec, S.order, S.rstart,
                                       S.rows, g->row_graph, S.queue, ctx->d_code_to_id3,
                                       (unsigned long long*)d_hist);
  }
  phase_end(ctx, kPhPairs);
  MOCHY_HIP_OR(hipGetLastError(), release);
  release(MOCHY_OK);  // stream-ordered; the correction reads rows and records only
  phase_begin(ctx, kPhCorrect);
  rc = correct_device(ctx, g, c0, c1, d_hist, stats);
  if (rc != MOCHY_OK) return rc;
  phase_end(ctx, kPhCorrect);
  MOCHY_HIP(hipGetLastError());
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small + kExactStatsSlot, stats, kStBatches * 8,
                           hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  phases_collect(ctx);
  const int64_t* hs = ctx->h_small + kExactStatsSlot;
  for (int x = 0; x < kStBatches; ++x)  // the device counters (the batch count is the host's)
    ctx->exact_stats[x] = x == kStMaxParts ? std::max(ctx->exact_stats[x], hs[x]) : ctx->exact_stats[x] + hs[x];
  if (grouped) {
    ctx->exact_stats[kStRows] += c1 - c0;
    // rows of one hash part are not reported by the kernels
    ctx->exact_stats[kStMaxParts] = std::max<int64_t>(ctx->exact_stats[kStMaxParts], 1);
  }
  return MOCHY_OK;
}
