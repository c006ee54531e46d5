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
//     node, a pair and a triple of heavy nodes.
//
// Sampling runs in chunks of samples: draw the hyperwedge index of each
// sample and its row i; group samples by row; pick j, the m-th neighbour of
// e_i above i, from a bitmap of N_i built in LDS; enumerate N_i ∪ N_j.  The
// enumeration visits the lists E_v of u = e_i ∪ e_j except for the (at most
// three) heavy nodes with the longest lists; hyperedges reached through the
// skipped lists only are counted in bulk per size from the heavy-node tables
// (their class depends only on which skipped nodes they hold and on |e_k|),
// by inclusion-exclusion against the walked ones.
#include <algorithm>

#include "classify.h"
#include "common.h"
#include "rng.h"
#include "walk.h"

namespace {

// ---------------------------------------------------------------- projection

// padded size of the hyperedge at every slot of E_v (slot nnz holds 0)
__global__ void k_xsize(int64_t nnz, const int64_t* __restrict__ edge_ptr,
                        const int32_t* __restrict__ node_edges, int64_t* out) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < nnz) {
    const int32_t k = node_edges[p];
    out[p] = (edge_ptr[k + 1] - edge_ptr[k] + kXPad - 1) / kXPad * kXPad;
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
  const int64_t o = x64[p], o1 = x64[p + 1];
  xoff[p] = uint32_t(o);
  for (int64_t t = 0; t < o1 - o; ++t) xnodes[o + t] = t < c ? edge_nodes[s + t] : -1;
}

// per hyperedge of size c: +1 to hsize[b][c] for each heavy node b it holds,
// to hpair[b1][b2][c] (both orders) for each pair and to htriple[{b1,b2,b3}][c]
// for each triple of them
__global__ void k_heavy_tables(int64_t E, const int64_t* __restrict__ edge_ptr,
                               const int32_t* __restrict__ edge_nodes,
                               const int8_t* __restrict__ heavy_bit, uint32_t* hsize,
                               uint32_t* hpair, uint32_t* htriple) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int64_t s = edge_ptr[e];
  const int c = int(edge_ptr[e + 1] - s);
  unsigned long long held = 0;
  for (int q = 0; q < c; ++q) {
    const int hb = heavy_bit[edge_nodes[s + q]];
    if (hb >= 0) held |= 1ull << hb;
  }
  for (unsigned long long m0 = held; m0; m0 &= m0 - 1) {
    const int x0 = __ffsll((long long)m0) - 1;
    atomicAdd(&hsize[x0 * kSizeSlots + c], 1u);
    if (c > kSizeTail) atomicAdd(&hsize[x0 * kSizeSlots], 1u);
    for (unsigned long long m1 = m0 & (m0 - 1); m1; m1 &= m1 - 1) {
      const int x1 = __ffsll((long long)m1) - 1;
      atomicAdd(&hpair[(x0 * kHeavyBits + x1) * kSizeSlots + c], 1u);
      atomicAdd(&hpair[(x1 * kHeavyBits + x0) * kSizeSlots + c], 1u);
      if (c > kSizeTail) {
        atomicAdd(&hpair[(x0 * kHeavyBits + x1) * kSizeSlots], 1u);
        atomicAdd(&hpair[(x1 * kHeavyBits + x0) * kSizeSlots], 1u);
      }
      for (unsigned long long m2 = m1 & (m1 - 1); m2; m2 &= m2 - 1) {
        const int x2 = __ffsll((long long)m2) - 1;
        atomicAdd(&htriple[int64_t(triple_index(x0, x1, x2)) * kSizeSlots + c], 1u);
        if (c > kSizeTail) atomicAdd(&htriple[int64_t(triple_index(x0, x1, x2)) * kSizeSlots], 1u);
      }
    }
  }
}

// heavy nodes held by each hyperedge, as a 64-bit mask of heavy indices
__global__ void k_hmask(int64_t E, const int64_t* __restrict__ edge_ptr,
                        const int32_t* __restrict__ edge_nodes, const int8_t* __restrict__ heavy_bit,
                        uint64_t* hmask) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E) return;
  uint64_t m = 0;
  for (int64_t q = edge_ptr[e]; q < edge_ptr[e + 1]; ++q) {
    const int hb = heavy_bit[edge_nodes[q]];
    if (hb >= 0) m |= 1ull << hb;
  }
  hmask[e] = m;
}

// Sets of 4 to 6 heavy nodes held together by some hyperedge: their number
// (upper bound of the table's entries); a hyperedge with more than
// kBigHeavy heavy nodes makes the table too large (flag).
constexpr int kBigHeavy = 16;

__host__ __device__ constexpr int64_t choose(int n, int k) {
  return k < 0 || k > n ? 0 : (k == 0 ? 1 : choose(n - 1, k - 1) * n / k);
}

__global__ void k_bigcount(int64_t E, const uint64_t* __restrict__ hmask, unsigned long long* total,
                           int32_t* too_many) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int m = __popcll(hmask[e]);
  if (m > kBigHeavy) { atomicOr(too_many, 1); return; }
  const int64_t n = choose(m, 4) + choose(m, 5) + choose(m, 6);
  if (n) atomicAdd(total, (unsigned long long)n);
}

__global__ void k_bigfill(int64_t E, const int64_t* __restrict__ edge_ptr,
                          const uint64_t* __restrict__ hmask, unsigned long long* key, uint32_t* val,
                          int log2cap) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const uint64_t hm = hmask[e];
  const int m = __popcll(hm);
  if (m < 4 || m > kBigHeavy) return;
  const int c = int(edge_ptr[e + 1] - edge_ptr[e]);
  int h[kBigHeavy];
  int n = 0;
  for (uint64_t r = hm; r; r &= r - 1) h[n++] = __ffsll((long long)r) - 1;
  const uint32_t cap_mask = (1u << log2cap) - 1u;
  for (uint32_t sub = 0; sub < (1u << m); ++sub) {
    const int k = __popc(sub);
    if (k < 4 || k > 6) continue;
    uint64_t xm = 0;
    for (int t = 0; t < m; ++t)
      if (sub & (1u << t)) xm |= 1ull << h[t];
    for (uint32_t s = big_slot(xm, log2cap);; s = (s + 1u) & cap_mask) {
      const unsigned long long prev = atomicCAS(&key[s], 0ull, (unsigned long long)xm);
      if (prev == 0ull || prev == xm) {
        atomicAdd(&val[uint64_t(s) * kSizeSlots + c], 1u);
        if (c > kSizeTail) atomicAdd(&val[uint64_t(s) * kSizeSlots], 1u);
        break;
      }
    }
  }
}

// line-graph degrees from stored rows
__global__ void k_row_deg(int64_t E, const int64_t* __restrict__ lg_ptr, int64_t* deg) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < E) deg[i] = lg_ptr[i + 1] - lg_ptr[i];
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
    const uint32_t xs = xoff[p], xe = xoff[p + 1];
    int4 q0, q1;
    load8(xnodes, xs, xe, q0, q1);
    // e_k is owned here iff no node of e_k below v lies in e_i (nodes are
    // ascending, so only the ones before v are tested)
    bool owned = true;
    auto below = [&](int32_t u) {
      if (u >= 0 && u < v && owned && in_sorted(ei, a, u)) owned = false;
    };
    below(q0.x); below(q0.y); below(q0.z); below(q0.w);
    below(q1.x); below(q1.y); below(q1.z); below(q1.w);
    for (uint32_t t = xs + 2 * kXPad; t < xe && owned; t += kXPad) {
      const int4 q = *reinterpret_cast<const int4*>(xnodes + t);
      if (q.x >= v) break;
      below(q.x); below(q.y); below(q.z); below(q.w);
    }
    if (!owned) continue;
    ++cnt;
    if (k > int32_t(i)) ++ucnt;
    if (xe - xs >= uint32_t(a) && xe - xs < uint32_t(a) + kXPad) {
      // same padded length as e_i: a repeat iff e_k has a nodes, all in e_i
      int c = 0, hit = 0;
      for (uint32_t t = xs; t < xe; ++t) {
        const int32_t u = xnodes[t];
        if (u < 0) break;
        ++c;
        hit += in_sorted(ei, a, u) ? 1 : 0;
      }
      if (c == a && hit == a) dup = true;
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

constexpr int64_t kChunk = int64_t(1) << 25;      // samples per chunk
constexpr int64_t kChunkMemo = int64_t(1) << 27;  // with key memos: more samples per key and build

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

// Walks the lists of the non-skipped members of u for one sample, 64 visits
// (flattened over the lists) at a time.  The node lists of a window's visits
// are consecutive in xnodes within a list, so the window is cut into 4-node
// chunks that the lanes take one each (coalesced 16-byte loads); a chunk's
// sums go to its visit by an LDS add.  Then each lane classifies its own
// visit: e_k is counted at its smallest walked member (no walked member of u
// below the visit's node) and is neither e_i nor e_j; equal motif ids in a row
// are summed in a register before the LDS add.
template <bool kOvf>
__device__ __forceinline__ void walk_lists(EnumLds& L, int lane, int64_t T, uint32_t a, uint32_t b,
                                           uint32_t wij, uint32_t novf,
                                           const uint32_t* __restrict__ xoff,
                                           const int32_t* __restrict__ xnodes,
                                           const uint16_t* lut, unsigned long long* hist) {
  if (T <= 0) return;
  int x = 0;
  int64_t lend = L.pre[1];
  int64_t base = L.wb[0];
  int32_t v = L.wn[0];
  uint32_t run_id = 0, run_n = 0;
  for (int64_t q0 = 0; q0 < T; q0 += kWave) {
    const int64_t q = q0 + lane;
    uint32_t nch = 0, xs = 0;
    if (q < T) {
      while (lend <= q) {  // cursor to the list holding visit q
        ++x;
        lend = L.pre[x + 1];
        base = L.wb[x] - L.pre[x];
        v = L.wn[x];
      }
      xs = xoff[base + q];
      nch = (xoff[base + q + 1] - xs) / kXPad;
    }
    uint32_t incl = nch;
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t o = uint32_t(__shfl_up(int(incl), off));
      if (lane >= off) incl += o;
    }
    const uint32_t first_chunk = incl - nch;
    const uint32_t nchunks = uint32_t(__shfl(int(incl), kWave - 1));
    L.vx[lane] = xs;
    L.vc[lane] = first_chunk;
    L.vv[lane] = v;
    L.acc[lane] = 0ull;
    for (uint32_t t = 0; t < nch; ++t) L.cmap[first_chunk + t] = uint8_t(lane);
    wave_sync();
    for (uint32_t k = lane; k < nchunks; k += kWave) {
      const int owner = L.cmap[k];
      const int4 z4 = *reinterpret_cast<const int4*>(xnodes + L.vx[owner] + (k - L.vc[owner]) * kXPad);
      atomicAdd(&L.acc[owner], chunk_sums<kOvf>(L, z4, L.vv[owner], novf));
    }
    wave_sync();
    if (q < T) {
      const unsigned long long s = L.acc[lane];
      const uint32_t c = uint32_t(s >> kSc) & 63u, wi = uint32_t(s >> kSi) & 63u;
      const uint32_t wj = uint32_t(s >> kSj) & 63u, t3 = uint32_t(s >> kSt) & 63u;
      const uint32_t below = uint32_t(s >> kSb) & 63u;
      uint32_t pat = 0;
      for (int y = 0; y < kSkip; ++y) pat |= ((s >> (kSp + 2 * y)) & 3ull) ? 1u << y : 0u;
      // e_k = e_i or e_j: a hyperedge of that size inside it (no repeats)
      const bool self = (c == a && wi == c) || (c == b && wj == c);
      if (below == 0 && !self) {
        const uint32_t id = lut[triple_code(a, b, c, wij, wj, wi, t3)];
        if (id != run_id) {
          if (run_n) atomicAdd(&hist[run_id], (unsigned long long)run_n);
          run_id = id;
          run_n = 0;
        }
        ++run_n;
        if (pat) atomicAdd(&L.tally[(pat - 1) * kSizeSlots + c], 1u);
      }
    }
    wave_sync();
  }
  if (run_n) atomicAdd(&hist[run_id], (unsigned long long)run_n);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_enum(
    int64_t cnt, int64_t E, const int2* __restrict__ pairs, const int64_t* __restrict__ edge_ptr,
    const int32_t* __restrict__ edge_nodes, const int64_t* __restrict__ node_ptr,
    const int8_t* __restrict__ heavy_bit, const uint32_t* __restrict__ xoff,
    const int32_t* __restrict__ xnodes, const uint32_t* __restrict__ hsize,
    const uint32_t* __restrict__ hpair, const uint32_t* __restrict__ htriple,
    const uint16_t* __restrict__ code_to_id3, unsigned long long* queue,
    unsigned long long* hist_out, int32_t* flags) {
  __shared__ uint16_t lut[kNumCodes];
  __shared__ unsigned long long hist[kHistSlots];  // shared by the block's waves
  __shared__ EnumLds lds[kEnumWaves];
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x) hist[t] = 0ull;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  EnumLds& L = lds[wave];
  for (int t = lane; t < kBuckets; t += kWave) L.tab[t] = make_uint4(0u, 0u, 0u, 0u);
  for (int t = lane; t < kPatterns * kSizeSlots; t += kWave) L.tally[t] = 0u;
  if (lane == 0) L.novf = 0u;
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
      int hbit = -1;
      if (mem) {
        nb = node_ptr[u];
        du = node_ptr[u + 1] - nb;
        hbit = heavy_bit[u];
      }
      // the kSkip heavy members with the longest lists are not walked
      uint64_t key = (mem && hbit >= 0) ? ((uint64_t(du) << 6) | uint64_t(lane)) : 0ull;
      int nskip = 0;
      int hb[kSkip] = {-1, -1, -1};
      uint32_t sf[kSkip] = {0u, 0u, 0u};  // in-e_i / in-e_j flags of the skipped nodes
      for (int x = 0; x < kSkip; ++x) {
        const uint64_t top = wave_max_u64(key);
        if (!top) break;
        const int l = int(top & 63);
        if (lane == l) { f |= uint32_t(x + 1) << 2; key = 0ull; }
        hb[x] = __shfl(hbit, l);
        sf[x] = uint32_t(__shfl(int(f), l)) & 3u;
        ++nskip;
      }
      int slot = -1;
      if (mem) {
        const uint32_t packed = (uint32_t(u + 1) << 4) | f;
        uint32_t* bk = reinterpret_cast<uint32_t*>(&L.tab[bucket_of(u)]);
        for (int t = 0; t < 4 && slot < 0; ++t)
          if (atomicCAS(&bk[t], 0u, packed) == 0u) slot = t;
        if (slot < 0) L.ovf[atomicAdd(&L.novf, 1u)] = packed;
      }
      const bool walk = mem && (f >> 2) == 0u;
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
      const uint32_t novf = L.novf;
      const int64_t T = L.pre[nw];
      if (novf == 0)
        walk_lists<false>(L, lane, T, a, b, wij, 0u, xoff, xnodes, lut, hist);
      else
        walk_lists<true>(L, lane, T, a, b, wij, novf, xoff, xnodes, lut, hist);
      wave_sync();
      // bulk: e_k whose members of u are all skipped nodes (pattern T of them),
      // by size c = lane; inclusion-exclusion over the supersets of T
      if (nskip > 0 && lane >= 1 && lane <= MOCHY_MAX_EDGE) {
        const int c = lane;
        const uint32_t all = (1u << nskip) - 1u;
        int64_t F[kPatterns + 1];
        for (uint32_t m = 1; m <= all; ++m) F[m] = superset_count(m, hb, c, hsize, hpair, htriple);
        uint32_t pi = 0, pj = 0;  // skipped nodes held by e_i, e_j
        for (int y = 0; y < nskip; ++y) {
          pi |= (sf[y] & kFI) ? 1u << y : 0u;
          pj |= (sf[y] & kFJ) ? 1u << y : 0u;
        }
        for (uint32_t m = 1; m <= all; ++m) {
          int64_t n = 0;
          for (uint32_t sup = m; sup <= all; sup = (sup + 1) | m)  // supersets of m within all
            n += (__popc(sup ^ m) & 1) ? -F[sup] : F[sup];
          n -= L.tally[(m - 1) * kSizeSlots + c];
          // e_i and e_j themselves are in the tables but not in N_i ∪ N_j
          if (pi == m && a == c) n -= 1;
          if (pj == m && b == c) n -= 1;
          if (n == 0) continue;
          if (n < 0) { bad = true; continue; }
          uint32_t sik = 0, sjk = 0, tt = 0;
          for (int y = 0; y < nskip; ++y) {
            if (!(m & (1u << y))) continue;
            sik += sf[y] & kFI;
            sjk += (sf[y] >> 1) & 1u;
            tt += sf[y] == 3u ? 1u : 0u;
          }
          atomicAdd(&hist[lut[triple_code(a, b, uint32_t(c), wij, sjk, sik, tt)]],
                    (unsigned long long)n);
        }
      }
      wave_sync();
      if (mem && slot >= 0) reinterpret_cast<uint32_t*>(&L.tab[bucket_of(u)])[slot] = 0u;
      for (int t = lane; t < kPatterns * kSizeSlots; t += kWave) L.tally[t] = 0u;
      if (lane == 0) L.novf = 0u;
      wave_sync();
    }
  }
  if (bad) atomicOr(flags, 2);
  __syncthreads();
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x)
    if (hist[t]) atomicAdd(&hist_out[t], hist[t]);
}

}  // namespace

// Per-slot node lists and heavy-node tables (what the sampler walks), for a
// single graph whose incidence and transpose are built.
mochy_status build_walk_tables(mochy_ctx* ctx, mochy_graph* g) {
  hipStream_t st = ctx->stream;
  if (g->ng != 1 || g->V >= (int64_t(1) << 28)) {
    ctx->err = "on-the-fly sampling takes single graphs of fewer than 2^28 nodes";
    return MOCHY_EUNSUPPORTED;
  }
  const int64_t E = g->E, nnz = g->nnz;
  int64_t* tmp = nullptr;
  int64_t* x64 = nullptr;
  auto cleanup = [&]() { device_free(ctx, tmp); device_free(ctx, x64); };
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&tmp, scan_tmp_elems(nnz + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&x64, size_t(nnz + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->xoff, size_t(nnz + 1) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->hsize, size_t(kHeavyBits) * kSizeSlots * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->hpair,
                         size_t(kHeavyBits) * kHeavyBits * kSizeSlots * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->htriple, size_t(kHeavyTriples) * kSizeSlots * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->hmask, size_t(std::max<int64_t>(E, 1)) * 8)) != MOCHY_OK) {
    cleanup();
    return rc;
  }
  g->bytes += size_t(nnz + 1) * 4 + size_t(kHeavyBits * (kHeavyBits + 1) + kHeavyTriples) * kSizeSlots * 4 +
              size_t(E) * 8;
  if (g->lg_ptr && !g->deg) {  // stored rows: degrees for the key order of the memoized sampler
    if ((rc = device_alloc(ctx, (void**)&g->deg, size_t(std::max<int64_t>(E, 1)) * 8)) != MOCHY_OK) {
      cleanup();
      return rc;
    }
    g->bytes += size_t(E) * 8;
    if (E > 0) k_row_deg<<<blocks(E, 256), 256, 0, st>>>(E, g->lg_ptr, g->deg);
  }
  phase_begin(ctx, kPhRows);
  k_xsize<<<blocks(nnz + 1, 256), 256, 0, st>>>(nnz, g->edge_ptr, g->node_edges, x64);
  launch_exclusive_scan_i64(x64, x64, nnz + 1, tmp, st);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, x64 + nnz, 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  const int64_t xtotal = ctx->h_small[0];
  if (xtotal >= (int64_t(1) << 32)) {
    cleanup();
    ctx->err = "on-the-fly sampling: the per-slot node lists would exceed 2^32 entries";
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
  MOCHY_HIP(hipMemsetAsync(g->htriple, 0, size_t(kHeavyTriples) * kSizeSlots * 4, st));
  if (E > 0) {
    k_heavy_tables<<<blocks(E, 256), 256, 0, st>>>(E, g->edge_ptr, g->edge_nodes, g->heavy_bit,
                                                   g->hsize, g->hpair, g->htriple);
    k_hmask<<<blocks(E, 256), 256, 0, st>>>(E, g->edge_ptr, g->edge_nodes, g->heavy_bit, g->hmask);
  }
  // table of the sets of 4 to 6 heavy nodes (for the key memos)
  MOCHY_HIP(hipMemsetAsync(ctx->d_small, 0, 16, st));
  if (E > 0)
    k_bigcount<<<blocks(E, 256), 256, 0, st>>>(E, g->hmask, (unsigned long long*)ctx->d_small,
                                                reinterpret_cast<int32_t*>(ctx->d_small + 1));
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, ctx->d_small, 16, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  const int64_t big_sets = ctx->h_small[0];
  const bool too_many = (*reinterpret_cast<const int32_t*>(ctx->h_small + 1)) != 0;
  g->memo_ok = !too_many && big_sets <= (int64_t(1) << 22);
  if (g->memo_ok) {
    int lg = 6;
    while ((int64_t(1) << lg) < 2 * big_sets) ++lg;
    const size_t cap = size_t(1) << lg;
    if ((rc = device_alloc(ctx, (void**)&g->hbig_key, cap * 8)) != MOCHY_OK ||
        (rc = device_alloc(ctx, (void**)&g->hbig_val, cap * kSizeSlots * 4)) != MOCHY_OK) {
      cleanup();
      return rc;
    }
    g->hbig_log2 = lg;
    g->bytes += cap * (8 + kSizeSlots * 4);
    MOCHY_HIP(hipMemsetAsync(g->hbig_key, 0, cap * 8, st));
    MOCHY_HIP(hipMemsetAsync(g->hbig_val, 0, cap * kSizeSlots * 4, st));
    if (big_sets > 0)
      k_bigfill<<<blocks(E, 256), 256, 0, st>>>(E, g->edge_ptr, g->hmask, g->hbig_key, g->hbig_val, lg);
  }
  phase_end(ctx, kPhRows);
  MOCHY_HIP(hipStreamSynchronize(st));
  cleanup();
  return MOCHY_OK;
}

mochy_status project_free_device(mochy_ctx* ctx, mochy_graph* g) {
  hipStream_t st = ctx->stream;
  if (g->ng != 1) {
    ctx->err = "the line-graph-free mode takes single graphs";
    return MOCHY_EUNSUPPORTED;
  }
  if (g->V >= (int64_t(1) << 28)) {
    ctx->err = "the line-graph-free mode takes fewer than 2^28 nodes";
    return MOCHY_ERANGE;
  }
  mochy_status rc = project_incidence(ctx, g);
  if (rc != MOCHY_OK) return rc;
  const int64_t E = g->E;
  g->lg_free = true;
  if ((rc = build_walk_tables(ctx, g)) != MOCHY_OK) return rc;
  int64_t* tmp = nullptr;
  int64_t* up_len = nullptr;
  auto cleanup = [&]() { device_free(ctx, tmp); device_free(ctx, up_len); };
  if ((rc = device_alloc(ctx, (void**)&tmp, scan_tmp_elems(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&up_len, size_t(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&g->deg, size_t(std::max<int64_t>(E, 1)) * 8)) != MOCHY_OK) {
    cleanup();
    return rc;
  }
  g->bytes += size_t(E) * 8;

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
  const bool use_memo = ctx->memo_budget > 0 && g->deg && g->memo_ok;
  const int64_t C = std::min(r, use_memo ? kChunkMemo : kChunk);
  int32_t *key_i = nullptr, *key_m = nullptr, *sm = nullptr, *keys = nullptr;
  int2* pairs = nullptr;
  unsigned long long* bcnt = nullptr;
  int64_t *boff = nullptr, *tmp = nullptr;
  unsigned int* cursor = nullptr;
  unsigned long long* ctr = nullptr;  // [0] nkeys | select queue, [1] enum queue
  memo_bufs* memo = nullptr;
  auto cleanup = [&]() {
    void* bufs[] = {key_i, key_m, sm, keys, pairs, bcnt, boff, tmp, cursor, ctr};
    for (void* p : bufs) device_free(ctx, p);
    memo_end(ctx, memo);
    memo = nullptr;
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
  if (use_memo) {
    if ((rc = memo_begin(ctx, g, C, &memo)) != MOCHY_OK) {
      cleanup();
      return rc;
    }
  }
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
    const int2* enum_pairs = pairs;
    int64_t n_enum = cnt;
    ctx->memo_stats[0] += cnt;
    if (memo && (rc = memo_chunk(ctx, g, memo, cnt, pairs, g->deg, d_hist, flags, &enum_pairs,
                                 &n_enum)) != MOCHY_OK) {
      cleanup();
      return rc;
    }
    if (n_enum > 0)
      k_enum<<<unsigned(ctx->num_cus) * 8u, kEnumWaves * kWave, 0, st>>>(
          n_enum, E, enum_pairs, g->edge_ptr, g->edge_nodes, g->node_ptr, g->heavy_bit, g->xoff,
          g->xnodes, g->hsize, g->hpair, g->htriple, ctx->d_code_to_id3, enum_queue,
          (unsigned long long*)d_hist, flags);
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
