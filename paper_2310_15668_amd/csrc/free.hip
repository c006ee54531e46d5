// Line-graph-free mode: MoCHy-A+ (Algorithm 5) on hypergraphs whose line
// graph does not fit in device memory.  Neighbourhoods are formed on demand
// from the incidence and its transpose (the on-the-fly neighbourhoods of
// section 4.4), never stored.
//
// Projection keeps, besides the incidence and E_v:
//   * expanded lists: for every slot (v, e_k) of E_v a copy of e_k's node
//     list (xoff / xnodes), so walking E_v streams the neighbours' node sets
//     instead of gathering them;
//   * line-graph degrees and upper degrees (neighbours above the row), counted
//     with an ownership rule: e_k in N_i is counted at the smallest node of
//     e_i ∩ e_k, so each neighbour is seen once with no per-row set;
//   * for the 64 heavy nodes, how many hyperedges of each size hold a heavy
//     node, and hold a pair of heavy nodes.
//
// Sampling runs in chunks of samples: draw the hyperwedge index of each
// sample and its row i; group samples by row; pick j, the m-th neighbour of
// e_i above i, from a bitmap of N_i built in LDS; enumerate N_i ∪ N_j.  The
// enumeration visits the lists E_v of u = e_i ∪ e_j except for the (at most
// two) heavy nodes with the longest lists; hyperedges reached through the
// skipped lists only are counted in bulk per size from the heavy-node tables
// (their class depends only on which skipped nodes they hold and on |e_k|),
// by inclusion-exclusion against the walked ones.
#include <algorithm>

#include "classify.h"
#include "common.h"
#include "rng.h"

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

// ---------------------------------------------------------------- projection

// size of the hyperedge at every slot of E_v (slot nnz holds 0)
__global__ void k_xsize(int64_t nnz, const int64_t* __restrict__ edge_ptr,
                        const int32_t* __restrict__ node_edges, int64_t* out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < nnz) {
    const int32_t k = node_edges[p];
    out[p] = edge_ptr[k + 1] - edge_ptr[k];
  }
  if (p == 0) out[nnz] = 0;
}

__global__ void k_xfill(int64_t nnz, const int64_t* __restrict__ edge_ptr,
                        const int32_t* __restrict__ edge_nodes,
                        const int32_t* __restrict__ node_edges, const int64_t* __restrict__ x64,
                        uint32_t* xoff, int32_t* xnodes) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p == 0) xoff[nnz] = uint32_t(x64[nnz]);
  if (p >= nnz) return;
  const int32_t k = node_edges[p];
  const int64_t s = edge_ptr[k], c = edge_ptr[k + 1] - s;
  const int64_t o = x64[p];
  xoff[p] = uint32_t(o);
  for (int64_t t = 0; t < c; ++t) xnodes[o + t] = edge_nodes[s + t];
}

// per hyperedge: +1 to hsize[b][|e|] for each heavy node b it holds and to
// hpair[b1][b2][|e|] (both orders) for each pair of them
__global__ void k_heavy_tables(int64_t E, const int64_t* __restrict__ edge_ptr,
                               const int32_t* __restrict__ edge_nodes,
                               const int8_t* __restrict__ heavy_bit, uint32_t* hsize,
                               uint32_t* hpair) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int64_t s = edge_ptr[e];
  const int c = int(edge_ptr[e + 1] - s);
  unsigned long long seen = 0;
  for (int q = 0; q < c; ++q) {
    const int hb = heavy_bit[edge_nodes[s + q]];
    if (hb < 0) continue;
    atomicAdd(&hsize[hb * kSizeSlots + c], 1u);
    for (unsigned long long m = seen; m; m &= m - 1) {
      const int h2 = __ffsll((long long)m) - 1;
      atomicAdd(&hpair[(hb * kHeavyBits + h2) * kSizeSlots + c], 1u);
      atomicAdd(&hpair[(h2 * kHeavyBits + hb) * kSizeSlots + c], 1u);
    }
    seen |= 1ull << hb;
  }
}

// One wave per row i: d_i = |N_i| and the upper degree |{j > i in N_i}|.
// The row's visits are the slots of E_v for v in e_i, flattened over the
// lanes; e_k is counted at the visit through v = min(e_i ∩ e_k).  A visit of
// a hyperedge of e_i's size lying inside e_i is a repeat of e_i.
constexpr int kDegWaves = 4;

__global__ __launch_bounds__(256) void k_free_degree(
    int64_t E, const int64_t* __restrict__ edge_ptr, const int32_t* __restrict__ edge_nodes,
    const int64_t* __restrict__ node_ptr, const int32_t* __restrict__ node_edges,
    const uint32_t* __restrict__ xoff, const int32_t* __restrict__ xnodes, int64_t* deg,
    int64_t* up_len, int32_t* max_deg, int32_t* flags) {
  __shared__ int32_t s_e[kDegWaves][MOCHY_MAX_EDGE];
  __shared__ int64_t s_pre[kDegWaves][MOCHY_MAX_EDGE + 1];
  __shared__ int64_t s_base[kDegWaves][MOCHY_MAX_EDGE];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = int64_t(blockIdx.x) * kDegWaves + wave;
  if (i >= E) return;  // whole wave; no block-wide barrier below
  int32_t* ei = s_e[wave];
  int64_t* pre = s_pre[wave];
  int64_t* base = s_base[wave];
  const int64_t es = edge_ptr[i];
  const int a = int(edge_ptr[i + 1] - es);
  int64_t dv = 0;
  if (lane < a) {
    const int32_t v = edge_nodes[es + lane];
    ei[lane] = v;
    base[lane] = node_ptr[v];
    dv = node_ptr[v + 1] - base[lane];
  }
  const int64_t incl = wave_incl_scan_i64(dv, lane);
  if (lane < a) pre[lane + 1] = incl;
  if (lane == 0) pre[0] = 0;
  wave_sync();
  const int64_t L = pre[a];
  int64_t cnt = 0, ucnt = 0;
  bool dup = false;
  int x = 0;
  for (int64_t q = lane; q < L; q += kWave) {
    while (pre[x + 1] <= q) ++x;
    const int32_t v = ei[x];
    const int64_t p = base[x] + (q - pre[x]);
    const int32_t k = node_edges[p];
    if (k == int32_t(i)) continue;
    const uint32_t xs = xoff[p], c = xoff[p + 1] - xs;
    bool owned = true;
    for (uint32_t t = 0; t < c; ++t) {
      const int32_t u = xnodes[xs + t];
      if (u >= v) break;
      if (in_sorted(ei, a, u)) { owned = false; break; }
    }
    if (!owned) continue;
    ++cnt;
    if (k > int32_t(i)) ++ucnt;
    if (c == uint32_t(a)) {
      uint32_t hit = 0;
      for (uint32_t t = 0; t < c; ++t) hit += in_sorted(ei, a, xnodes[xs + t]) ? 1u : 0u;
      if (hit == c) dup = true;
    }
  }
  if (dup) atomicOr(flags, kFlagDup);
  cnt = wave_sum_i64(cnt);
  ucnt = wave_sum_i64(ucnt);
  if (lane == 0) {
    deg[i] = cnt;
    up_len[i] = ucnt;
    atomicMax(max_deg, int32_t(cnt));
  }
}

__global__ void k_deg_stats(int64_t E, const int64_t* __restrict__ deg, unsigned long long* out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= E) return;
  const unsigned long long d = (unsigned long long)deg[i];
  atomicAdd(&out[0], d * (d - (d ? 1 : 0)) / 2);
  atomicAdd(&out[2], d * d);
}

// ------------------------------------------------------------------ sampling

constexpr int64_t kChunk = int64_t(1) << 25;  // samples per chunk

// Hyperwedge index of each sample -> (row i, rank m of j among i's upper
// neighbours); counts samples per row and lists each row drawn once.
__global__ void k_draw(int64_t n_start, int64_t cnt, uint64_t seed, uint64_t W, int64_t E,
                       const int64_t* __restrict__ up_ptr, int32_t* key_i, int32_t* key_m,
                       unsigned long long* bcnt, int32_t* keys, unsigned int* nkeys) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  const int64_t idx = int64_t(sample_wedge(uint64_t(n_start) + uint64_t(s), seed, W));
  const int64_t i = wedge_row(up_ptr, E, idx);
  key_i[s] = int32_t(i);
  key_m[s] = int32_t(idx - up_ptr[i]);
  if (atomicAdd(&bcnt[i], 1ull) == 0ull) keys[atomicAdd(nkeys, 1u)] = int32_t(i);
}

__global__ void k_bucket(int64_t cnt, const int32_t* __restrict__ key_i,
                         const int32_t* __restrict__ key_m, const int64_t* __restrict__ boff,
                         unsigned int* cursor, int32_t* sm) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  const int32_t i = key_i[s];
  sm[boff[i] + atomicAdd(&cursor[i], 1u)] = key_m[s];
}

// One 1024-thread block per drawn row i: N_i above i as a bitmap over a tile
// of 2^20 hyperedge ids in LDS, with a popcount per 1024-bit block; the m-th
// set bit of the row is j.  Bits are set by walking E_v for v in e_i, so the
// row comes out sorted and de-duplicated.
constexpr int kSelThreads = 1024;
constexpr int kTileBits = 1 << 20;
constexpr int kTileWords = kTileBits / 32;
constexpr int kBlkBits = 1024;
constexpr int kTileBlks = kTileBits / kBlkBits;
static_assert(kTileBlks == kSelThreads, "one counter per thread");

__global__ __launch_bounds__(kSelThreads) void k_select(
    int64_t E, const int64_t* __restrict__ edge_ptr, const int32_t* __restrict__ edge_nodes,
    const int64_t* __restrict__ node_ptr, const int32_t* __restrict__ node_edges,
    const int32_t* __restrict__ keys, const unsigned int* __restrict__ nkeys, unsigned int* queue,
    const int64_t* __restrict__ boff, const int32_t* __restrict__ sm, int2* pairs, int32_t* flags) {
  __shared__ uint32_t bm[kTileWords];
  __shared__ uint32_t blk[kTileBlks];
  __shared__ int64_t s_lo[MOCHY_MAX_EDGE], s_hi[MOCHY_MAX_EDGE];
  __shared__ uint32_t s_wsum[kSelThreads / kWave];
  __shared__ int64_t s_red[kSelThreads / kWave];
  __shared__ unsigned int s_key;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int w = tid; w < kTileWords; w += kSelThreads) bm[w] = 0u;
  blk[tid] = 0u;
  const unsigned nk = *nkeys;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_key = atomicAdd(queue, 1u);
    __syncthreads();
    const unsigned kq = s_key;
    if (kq >= nk) break;
    const int64_t i = keys[kq];
    const int64_t b0 = boff[i], b1 = boff[i + 1];
    const int64_t es = edge_ptr[i];
    const int a = int(edge_ptr[i + 1] - es);
    if (tid < a) {
      const int32_t v = edge_nodes[es + tid];
      s_lo[tid] = node_ptr[v];
      s_hi[tid] = node_ptr[v + 1];
    }
    int64_t mm = -1;
    for (int64_t s = b0 + tid; s < b1; s += kSelThreads) mm = max(mm, int64_t(sm[s]));
    for (int off = 32; off > 0; off >>= 1) {
      const int lo = __shfl_xor(int(uint32_t(mm)), off);
      const int hi = __shfl_xor(int(uint32_t(uint64_t(mm) >> 32)), off);
      const int64_t o = int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo));
      mm = o > mm ? o : mm;
    }
    if (lane == 0) s_red[wave] = mm;
    __syncthreads();
    int64_t maxm = s_red[0];
    for (int w = 1; w < kSelThreads / kWave; ++w) maxm = s_red[w] > maxm ? s_red[w] : maxm;
    int64_t base = 0;  // upper neighbours of i below the current tile
    for (int64_t t0 = i + 1; t0 < E && base <= maxm; t0 += kTileBits) {
      const int64_t t1 = t0 + kTileBits < E ? t0 + kTileBits : E;
      for (int x = 0; x < a; ++x)
        for (int64_t r = s_lo[x] + tid; r < s_hi[x]; r += kSelThreads) {
          const int64_t k = node_edges[r];
          if (k < t0 || k >= t1) continue;
          const uint32_t off = uint32_t(k - t0), bit = 1u << (off & 31);
          const uint32_t old = atomicOr(&bm[off >> 5], bit);
          if (!(old & bit)) atomicAdd(&blk[off / kBlkBits], 1u);
        }
      __syncthreads();
      // exclusive prefix of the block counters, in place
      const uint32_t mine = blk[tid];
      uint32_t incl = mine;
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = uint32_t(__shfl_up(int(incl), off));
        if (lane >= off) incl += o;
      }
      if (lane == 63) s_wsum[wave] = incl;
      __syncthreads();
      uint32_t before = 0, total = 0;
      for (int w = 0; w < kSelThreads / kWave; ++w) {
        if (w < wave) before += s_wsum[w];
        total += s_wsum[w];
      }
      blk[tid] = before + incl - mine;
      __syncthreads();
      for (int64_t s = b0 + tid; s < b1; s += kSelThreads) {
        const int64_t m = int64_t(sm[s]) - base;
        if (m < 0 || m >= int64_t(total)) continue;
        int lo = 0, hi = kTileBlks;  // last block whose prefix is <= m
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (int64_t(blk[mid]) <= m) lo = mid; else hi = mid;
        }
        uint32_t rem = uint32_t(m - int64_t(blk[lo]));
        int w = lo * (kBlkBits / 32);
        const int wend = w + kBlkBits / 32;
        for (; w < wend; ++w) {
          const uint32_t pc = __popc(bm[w]);
          if (rem < pc) break;
          rem -= pc;
        }
        if (w == wend) {  // cannot happen for a consistent bitmap
          atomicOr(flags, 1);
          pairs[s] = make_int2(int32_t(i), -1);
          continue;
        }
        uint32_t bits = bm[w];
        for (uint32_t c = 0; c < rem; ++c) bits &= bits - 1;
        pairs[s] = make_int2(int32_t(i), int32_t(t0 + int64_t(w) * 32 + (__ffs(bits) - 1)));
      }
      __syncthreads();
      for (int x = 0; x < a; ++x)
        for (int64_t r = s_lo[x] + tid; r < s_hi[x]; r += kSelThreads) {
          const int64_t k = node_edges[r];
          if (k >= t0 && k < t1) bm[uint32_t(k - t0) >> 5] = 0u;
        }
      blk[tid] = 0u;
      base += total;
      __syncthreads();
    }
  }
}

// Enumeration: one wave per sampled pair (i, j).
constexpr int kEnumWaves = 4;
constexpr int kHash = 128;                 // open-addressing table of u = e_i ∪ e_j
constexpr uint32_t kFI = 1, kFJ = 2, kFSkip = 4, kFW2 = 8;
constexpr int kBatch = 4;                  // samples taken from the queue at a time

struct EnumLds {
  int32_t hk[kHash];                       // node id, -1 = free
  uint8_t hf[kHash];                       // kFI | kFJ | kFSkip | kFW2
  int32_t ei[MOCHY_MAX_EDGE], ej[MOCHY_MAX_EDGE];
  int32_t wn[2 * MOCHY_MAX_EDGE];          // walked nodes
  int64_t wb[2 * MOCHY_MAX_EDGE];          // node_ptr of each walked node
  int64_t pre[2 * MOCHY_MAX_EDGE + 1];     // prefix of walked list lengths
  uint32_t tally[3 * kSizeSlots];          // walked e_k holding skipped nodes, by pattern and size
  unsigned long long hist[kHistSlots];
};

__device__ __forceinline__ uint32_t node_hash(int32_t z) {
  return (uint32_t(z) * 2654435761u) >> 25;  // 7 bits
}

__device__ __forceinline__ uint32_t lookup(const EnumLds& L, int32_t z) {
  uint32_t h = node_hash(z);
  for (;;) {
    const int32_t kk = L.hk[h];
    if (kk == z) return L.hf[h];
    if (kk < 0) return 0u;
    h = (h + 1) & (kHash - 1);
  }
}

__global__ __launch_bounds__(256) void k_enum(
    int64_t cnt, int64_t E, const int2* __restrict__ pairs, const int64_t* __restrict__ edge_ptr,
    const int32_t* __restrict__ edge_nodes, const int64_t* __restrict__ node_ptr,
    const int8_t* __restrict__ heavy_bit, const uint32_t* __restrict__ xoff,
    const int32_t* __restrict__ xnodes, const uint32_t* __restrict__ hsize,
    const uint32_t* __restrict__ hpair, const uint16_t* __restrict__ code_to_id3,
    unsigned long long* queue, unsigned long long* hist_out, int32_t* flags) {
  __shared__ uint16_t lut[kNumCodes];
  __shared__ EnumLds lds[kEnumWaves];
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  EnumLds& L = lds[wave];
  for (int t = lane; t < kHash; t += kWave) L.hk[t] = -1;
  for (int t = lane; t < 3 * kSizeSlots; t += kWave) L.tally[t] = 0u;
  for (int t = lane; t < kHistSlots; t += kWave) L.hist[t] = 0ull;
  __syncthreads();
  bool bad = false;
  for (;;) {
    unsigned long long sq = 0;
    if (lane == 0) sq = atomicAdd(queue, (unsigned long long)kBatch);
    const int64_t sb = int64_t(uniform64(sq));
    if (sb >= cnt) break;
    const int64_t se = sb + kBatch < cnt ? sb + kBatch : cnt;
    for (int64_t s = sb; s < se; ++s) {
      const int2 pr = pairs[s];
      const int64_t i = pr.x, j = pr.y;
      if (i < 0 || i >= E || j < 0 || j >= E || j == i) { bad = true; continue; }
      const int64_t si = edge_ptr[i], sj = edge_ptr[j];
      const int a = int(edge_ptr[i + 1] - si), b = int(edge_ptr[j + 1] - sj);
      if (lane < a) L.ei[lane] = edge_nodes[si + lane];
      if (lane < b) L.ej[lane] = edge_nodes[sj + lane];
      wave_sync();
      // members of u: lanes 0..31 carry e_i's nodes, lanes 32..63 the nodes
      // of e_j outside e_i
      int32_t u = -1;
      uint32_t f = 0;
      if (lane < a) {
        u = L.ei[lane];
        f = kFI | (in_sorted(L.ej, b, u) ? kFJ : 0u);
      } else if (lane >= 32 && lane - 32 < b) {
        const int32_t z = L.ej[lane - 32];
        if (!in_sorted(L.ei, a, z)) { u = z; f = kFJ; }
      }
      const bool mem = u >= 0;
      const uint32_t wij = uint32_t(__popcll(__ballot(lane < a && (f & kFJ))));
      int64_t nb = 0, du = 0;
      int hb = -1;
      if (mem) {
        nb = node_ptr[u];
        du = node_ptr[u + 1] - nb;
        hb = heavy_bit[u];
      }
      // the two heavy members with the longest lists are not walked
      const uint64_t key = (mem && hb >= 0) ? ((uint64_t(du) << 6) | uint64_t(lane)) : 0ull;
      const uint64_t k1 = wave_max_u64(key);
      const int l1 = k1 ? int(k1 & 63) : -1;
      const uint64_t k2 = wave_max_u64(lane == l1 ? 0ull : key);
      const int l2 = k2 ? int(k2 & 63) : -1;
      if (lane == l1) f |= kFSkip;
      if (lane == l2) f |= kFSkip | kFW2;
      const int hb1 = l1 >= 0 ? __shfl(hb, l1) : -1;
      const int hb2 = l2 >= 0 ? __shfl(hb, l2) : -1;
      const uint32_t f1 = l1 >= 0 ? uint32_t(__shfl(int(f), l1)) : 0u;
      const uint32_t f2 = l2 >= 0 ? uint32_t(__shfl(int(f), l2)) : 0u;
      int slot = -1;
      if (mem) {
        uint32_t h = node_hash(u);
        for (;;) {
          if (atomicCAS(&L.hk[h], -1, u) == -1) { slot = int(h); break; }
          h = (h + 1) & (kHash - 1);
        }
        L.hf[slot] = uint8_t(f);
      }
      const bool walk = mem && !(f & kFSkip);
      const uint64_t wm = __ballot(walk);
      const int nw = __popcll(wm);
      const int wpos = __popcll(wm & ((1ull << lane) - 1ull));
      const int64_t incl = wave_incl_scan_i64(walk ? du : 0, lane);
      if (walk) {
        L.wn[wpos] = u;
        L.wb[wpos] = nb;
        L.pre[wpos + 1] = incl;
      }
      if (lane == 0) L.pre[0] = 0;
      wave_sync();
      const int64_t T = L.pre[nw];
      int x = 0;
      for (int64_t q = lane; q < T; q += kWave) {
        while (L.pre[x + 1] <= q) ++x;
        const int32_t v = L.wn[x];
        const int64_t p = L.wb[x] + (q - L.pre[x]);
        const uint32_t xs = xoff[p], c = xoff[p + 1] - xs;
        uint32_t wi = 0, wj = 0, t3 = 0, pat = 0;
        int32_t first = -1;
        for (uint32_t t = 0; t < c; ++t) {
          const int32_t z = xnodes[xs + t];
          const uint32_t ff = lookup(L, z);
          if (!ff) continue;
          wi += ff & kFI;
          wj += (ff >> 1) & 1u;
          t3 += (ff & 3u) == 3u ? 1u : 0u;
          if (ff & kFSkip) pat |= (ff & kFW2) ? 2u : 1u;
          else if (first < 0) first = z;
        }
        // e_k = e_i or e_j: a hyperedge of that size inside it (no repeats)
        const bool self = (c == uint32_t(a) && wi == c) || (c == uint32_t(b) && wj == c);
        if (first != v || self) continue;  // counted at the smallest walked node of e_k
        atomicAdd(&L.hist[lut[triple_code(a, b, c, wij, wj, wi, t3)]], 1ull);
        if (pat) atomicAdd(&L.tally[(pat - 1) * kSizeSlots + c], 1u);
      }
      wave_sync();
      // bulk: e_k whose only members of u are skipped nodes, by size c = lane
      if (l1 >= 0 && lane >= 1 && lane <= MOCHY_MAX_EDGE) {
        const int c = lane;
        const int64_t h1 = hsize[hb1 * kSizeSlots + c];
        const int64_t h2 = l2 >= 0 ? int64_t(hsize[hb2 * kSizeSlots + c]) : 0;
        const int64_t pc = l2 >= 0 ? int64_t(hpair[(hb1 * kHeavyBits + hb2) * kSizeSlots + c]) : 0;
        int64_t n[3] = {h1 - pc - L.tally[c], h2 - pc - L.tally[kSizeSlots + c],
                        pc - L.tally[2 * kSizeSlots + c]};
        // e_i and e_j themselves are in the tables but not in N_i ∪ N_j
        const uint32_t pi = ((f1 & kFI) ? 1u : 0u) | ((f2 & kFI) ? 2u : 0u);
        const uint32_t pj = ((f1 & kFJ) ? 1u : 0u) | ((f2 & kFJ) ? 2u : 0u);
        if (pi && a == c) n[pi - 1] -= 1;
        if (pj && b == c) n[pj - 1] -= 1;
        for (uint32_t pat = 1; pat <= 3; ++pat) {
          const int64_t m = n[pat - 1];
          if (m == 0) continue;
          if (m < 0) { bad = true; continue; }
          const uint32_t g1 = (pat & 1u) ? f1 : 0u, g2 = (pat & 2u) ? f2 : 0u;
          const uint32_t sik = (g1 & kFI ? 1u : 0u) + (g2 & kFI ? 1u : 0u);
          const uint32_t sjk = (g1 & kFJ ? 1u : 0u) + (g2 & kFJ ? 1u : 0u);
          const uint32_t tt = ((g1 & 3u) == 3u ? 1u : 0u) + ((g2 & 3u) == 3u ? 1u : 0u);
          atomicAdd(&L.hist[lut[triple_code(a, b, uint32_t(c), wij, sjk, sik, tt)]],
                    (unsigned long long)m);
        }
      }
      wave_sync();
      if (slot >= 0) L.hk[slot] = -1;
      for (int t = lane; t < 3 * kSizeSlots; t += kWave) L.tally[t] = 0u;
      wave_sync();
    }
  }
  if (bad) atomicOr(flags, 2);
  wave_sync();
  for (int t = lane; t < kHistSlots; t += kWave)
    if (L.hist[t]) atomicAdd(&hist_out[t], L.hist[t]);
}

}  // namespace

mochy_status project_free_device(mochy_ctx* ctx, mochy_graph* g) {
  hipStream_t st = ctx->stream;
  if (g->ng != 1) {
    ctx->err = "the line-graph-free mode takes single graphs";
    return MOCHY_EUNSUPPORTED;
  }
  mochy_status rc = project_incidence(ctx, g);
  if (rc != MOCHY_OK) return rc;
  const int64_t E = g->E, nnz = g->nnz;
  g->lg_free = true;
  int64_t* tmp = nullptr;
  int64_t* x64 = nullptr;
  int64_t* up_len = nullptr;
  auto cleanup = [&]() { (void)hipFree(tmp); (void)hipFree(x64); (void)hipFree(up_len); };
  if ((rc = device_alloc(ctx, (void**)&tmp, scan_tmp_elems(std::max(nnz, E) + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&x64, size_t(nnz + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&up_len, size_t(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->xoff, size_t(nnz + 1) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->deg, size_t(std::max<int64_t>(E, 1)) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->hsize, size_t(kHeavyBits) * kSizeSlots * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->hpair,
                         size_t(kHeavyBits) * kHeavyBits * kSizeSlots * 4)) != MOCHY_OK) {
    cleanup();
    return rc;
  }
  g->bytes += size_t(nnz + 1) * 4 + size_t(E) * 8 + size_t(kHeavyBits) * (kHeavyBits + 1) * kSizeSlots * 4;

  // expanded lists
  phase_begin(ctx, kPhRows);
  k_xsize<<<blocks(nnz + 1, 256), 256, 0, st>>>(nnz, g->edge_ptr, g->node_edges, x64);
  launch_exclusive_scan_i64(x64, x64, nnz + 1, tmp, st);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, x64 + nnz, 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  const int64_t xtotal = ctx->h_small[0];
  if (xtotal >= (int64_t(1) << 32)) {
    cleanup();
    ctx->err = "line-graph-free mode: sum of squared hyperedge sizes reaches 2^32";
    return MOCHY_ERANGE;
  }
  if ((rc = device_alloc(ctx, (void**)&g->xnodes, size_t(std::max<int64_t>(xtotal, 1)) * 4)) != MOCHY_OK) {
    cleanup();
    return rc;
  }
  g->bytes += size_t(xtotal) * 4;
  k_xfill<<<blocks(std::max<int64_t>(nnz, 1), 256), 256, 0, st>>>(nnz, g->edge_ptr, g->edge_nodes,
                                                                  g->node_edges, x64, g->xoff,
                                                                  g->xnodes);
  MOCHY_HIP(hipMemsetAsync(g->hsize, 0, size_t(kHeavyBits) * kSizeSlots * 4, st));
  MOCHY_HIP(hipMemsetAsync(g->hpair, 0, size_t(kHeavyBits) * kHeavyBits * kSizeSlots * 4, st));
  if (E > 0)
    k_heavy_tables<<<blocks(E, 256), 256, 0, st>>>(E, g->edge_ptr, g->edge_nodes, g->heavy_bit,
                                                   g->hsize, g->hpair);
  phase_end(ctx, kPhRows);

  // degrees and the hyperwedge order
  phase_begin(ctx, kPhDegree);
  MOCHY_HIP(hipMemsetAsync(ctx->d_flags, 0, 2 * sizeof(int32_t), st));
  MOCHY_HIP(hipMemsetAsync(up_len, 0, size_t(E + 1) * 8, st));
  if (E > 0)
    k_free_degree<<<blocks(E, kDegWaves), kDegWaves * kWave, 0, st>>>(
        E, g->edge_ptr, g->edge_nodes, g->node_ptr, g->node_edges, g->xoff, g->xnodes, g->deg,
        up_len, ctx->d_flags + 1, ctx->d_flags);
  launch_exclusive_scan_i64(up_len, g->up_ptr, E + 1, tmp, st);
  phase_end(ctx, kPhDegree);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, g->up_ptr + E, 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small + 1, ctx->d_flags, 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  phases_collect(ctx);
  cleanup();
  g->W = ctx->h_small[0];
  const int32_t* fl = reinterpret_cast<const int32_t*>(ctx->h_small + 1);
  g->max_deg = fl[1];
  if (fl[0] & kFlagDup) { ctx->err = "duplicate hyperedges (pass MOCHY_DEDUP for host input)"; return MOCHY_EDUP; }
  return MOCHY_OK;
}

mochy_status free_graph_stats(mochy_ctx* ctx, const mochy_graph* g, unsigned long long* d_out) {
  if (g->E > 0)
    k_deg_stats<<<blocks(g->E, 256), 256, 0, ctx->stream>>>(g->E, g->deg, d_out);
  MOCHY_HIP(hipGetLastError());
  return MOCHY_OK;
}

mochy_status sampled_free_device(mochy_ctx* ctx, const mochy_graph* g, int64_t r, uint64_t seed,
                                 int64_t n0, int64_t* d_hist) {
  hipStream_t st = ctx->stream;
  MOCHY_HIP(hipMemsetAsync(d_hist, 0, kHistSlots * 8, st));
  if (g->W == 0 || r == 0) return MOCHY_OK;
  const int64_t E = g->E;
  const int64_t C = std::min(r, kChunk);
  int32_t *key_i = nullptr, *key_m = nullptr, *sm = nullptr, *keys = nullptr;
  int2* pairs = nullptr;
  unsigned long long* bcnt = nullptr;
  int64_t *boff = nullptr, *tmp = nullptr;
  unsigned int* cursor = nullptr;
  unsigned long long* ctr = nullptr;  // [0] nkeys | select queue, [1] enum queue
  auto cleanup = [&]() {
    void* bufs[] = {key_i, key_m, sm, keys, pairs, bcnt, boff, tmp, cursor, ctr};
    for (void* p : bufs) (void)hipFree(p);
  };
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&key_i, size_t(C) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&key_m, size_t(C) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&sm, size_t(C) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&pairs, size_t(C) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&keys, size_t(E) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&bcnt, size_t(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&boff, size_t(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&tmp, scan_tmp_elems(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&cursor, size_t(E) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&ctr, 4 * 8)) != MOCHY_OK) {
    cleanup();
    return rc;
  }
  unsigned int* nkeys = reinterpret_cast<unsigned int*>(ctr);
  unsigned int* sel_queue = nkeys + 1;
  unsigned long long* enum_queue = ctr + 1;
  int32_t* flags = ctx->d_flags + 2;
  MOCHY_HIP(hipMemsetAsync(flags, 0, 4, st));
  for (int64_t off = 0; off < r; off += C) {
    const int64_t cnt = std::min(C, r - off);
    if (hipMemsetAsync(bcnt, 0, size_t(E + 1) * 8, st) != hipSuccess ||
        hipMemsetAsync(cursor, 0, size_t(E) * 4, st) != hipSuccess ||
        hipMemsetAsync(ctr, 0, 4 * 8, st) != hipSuccess) {
      cleanup();
      ctx->err = "hipMemsetAsync failed";
      return MOCHY_EDEVICE;
    }
    phase_begin(ctx, kPhDraw);
    k_draw<<<blocks(cnt, 256), 256, 0, st>>>(n0 + off, cnt, seed, uint64_t(g->W), E, g->up_ptr,
                                              key_i, key_m, bcnt, keys, nkeys);
    launch_exclusive_scan_i64(reinterpret_cast<int64_t*>(bcnt), boff, E + 1, tmp, st);
    k_bucket<<<blocks(cnt, 256), 256, 0, st>>>(cnt, key_i, key_m, boff, cursor, sm);
    k_select<<<unsigned(ctx->num_cus), kSelThreads, 0, st>>>(E, g->edge_ptr, g->edge_nodes,
                                                             g->node_ptr, g->node_edges, keys,
                                                             nkeys, sel_queue, boff, sm, pairs,
                                                             flags);
    phase_end(ctx, kPhDraw);
    phase_begin(ctx, kPhSample);
    k_enum<<<unsigned(ctx->num_cus) * 8u, kEnumWaves * kWave, 0, st>>>(
        cnt, E, pairs, g->edge_ptr, g->edge_nodes, g->node_ptr, g->heavy_bit, g->xoff, g->xnodes,
        g->hsize, g->hpair, ctx->d_code_to_id3, enum_queue, (unsigned long long*)d_hist, flags);
    phase_end(ctx, kPhSample);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      cleanup();
      ctx->err = std::string("sampling kernels failed: ") + hipGetErrorString(e);
      return MOCHY_EDEVICE;
    }
    phases_collect(ctx);
  }
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, flags, 4, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  cleanup();
  if (*reinterpret_cast<int32_t*>(ctx->h_small) != 0) {
    ctx->err = "internal error in line-graph-free sampling (flags " +
               std::to_string(*reinterpret_cast<int32_t*>(ctx->h_small)) + ")";
    return MOCHY_EDEVICE;
  }
  return MOCHY_OK;
}
