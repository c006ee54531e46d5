// Exact fix-up of the pairs the pair kernel classified with an incomplete R5.
//
// The pair kernel takes R5 = |e_j ∩ e_k - e_i| from exact bits for the 64
// highest-degree ("heavy") nodes only.  It is exact for every pair of
// neighbours of e_i unless e_j and e_k also share a lower-degree ("light")
// node outside e_i.  Whether two hyperedges share a light node does not
// depend on the centre, and few pairs do (sum over light nodes w of
// C(|E_w|, 2)), so the fix-up works pair by pair:
//
//  1. light pairs: for every light node w, every pair {e_j, e_k} of E_w whose
//     smallest shared light node is w (each pair once).  The pair is owned by
//     the endpoint with the longer line-graph row.
//  2. for every light pair, the centres are N_j ∩ N_k: one workgroup per
//     owner j holds row j as an LDS bitmap (with per-word ranks, so a hit gives
//     the position of e_i in row j) and scans the partner's row.  With masks
//     over the nodes of e_k (m_kj: e_k ∩ e_j, and its heavy and light parts
//     H, L, formed once per pair from the two node lists) and, for a centre
//     e_i, m_ki (e_k ∩ e_i) from the record of row k at the scanned position:
//        t   = popcount(m_ki & m_kj)                 = |e_i ∩ e_j ∩ e_k|
//        r5h = popcount(H & ~m_ki)                   heavy part of R5
//        ls  = popcount(L & ~m_ki)                   light part of R5
//     and |e_j ∩ e_i|, |e_i| from the size word of row j at e_i's position
//     (the only read outside the scanned row).
//     If ls = 0 the pair kernel was exact at this centre.  Otherwise the pair
//     kernel recorded the class with R5 = r5h, counted iff both neighbours
//     are above e_i or the two looked disjoint; the exact class has
//     R5 = r5h + ls and, since e_j and e_k meet, is counted iff both are
//     above e_i (Algorithm 2's condition).  The first is removed, the second
//     added.
#include "classify.h"
#include "common.h"

namespace {

// Is w the smallest light node shared by e_x and e_y?  (Both contain w.)
__device__ __forceinline__ bool smallest_shared_light(int32_t x, int32_t y, int32_t w,
                                                      const int64_t* __restrict__ edge_ptr,
                                                      const int32_t* __restrict__ edge_nodes,
                                                      const int8_t* __restrict__ heavy_bit) {
  int64_t p = edge_ptr[x], q = edge_ptr[y];
  const int64_t pe = edge_ptr[x + 1], qe = edge_ptr[y + 1];
  while (p < pe && q < qe) {
    const int32_t u = edge_nodes[p], v = edge_nodes[q];
    if (u >= w || v >= w) {
      if (u < v) ++p;
      else if (u > v) ++q;
      else return true;  // reached w (u == v >= w means u == w: first shared light is w)
      continue;
    }
    if (u < v) ++p;
    else if (u > v) ++q;
    else {
      if (heavy_bit[u] < 0) return false;
      ++p; ++q;
    }
  }
  return true;
}

// One wave per light node w: every pair of E_w whose smallest shared light
// node is w.  kCount counts pairs per owner; kFill also writes the partners
// (a second pass, after the owners' offsets are known).  Where the flat list
// of candidate slots fits, k_light_slots runs the merges once instead.
enum LightMode { kCount = 0, kFill = 1 };
template <int kMode>
__global__ __launch_bounds__(256) void k_light_pairs(
    int64_t V, const int64_t* __restrict__ node_ptr, const int32_t* __restrict__ node_edges,
    const int8_t* __restrict__ heavy_bit, const int64_t* __restrict__ edge_ptr,
    const int32_t* __restrict__ edge_nodes, const int64_t* __restrict__ lg_ptr,
    unsigned long long* pcount, const int64_t* __restrict__ poff, int32_t* partners) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  if (w >= V || heavy_bit[w] >= 0) return;  // uniform per wave
  const int64_t lo = node_ptr[w];
  const int D = int(node_ptr[w + 1] - lo);
  for (int kc = 0; kc < D; kc += 64) {
    const int b = kc + lane;
    const int32_t yb = b < D ? node_edges[lo + b] : 0;
    const int64_t db = b < D ? lg_ptr[yb + 1] - lg_ptr[yb] : 0;
    const int aend = min(kc + 64, D) - 1;
    for (int a = 0; a < aend; ++a) {
      const int32_t ya = node_edges[lo + a];
      if (!(b < D && a < b)) continue;
      if (!smallest_shared_light(ya, yb, int32_t(w), edge_ptr, edge_nodes, heavy_bit)) continue;
      const int64_t da = lg_ptr[ya + 1] - lg_ptr[ya];
      const bool a_owns = da > db || (da == db && ya < yb);
      const int32_t owner = a_owns ? ya : yb, partner = a_owns ? yb : ya;
      const unsigned long long slot = atomicAdd(&pcount[owner], 1ull);
      if (kMode == kFill) partners[poff[owner] + int64_t(slot)] = partner;
    }
  }
}

// The flat list of candidate slots (slot noff[w] + b (b - 1) / 2 + a for
// members a < b of E_w): (owner, partner), or (-1, -1) where w is not the
// pair's smallest shared light node, so that the merges run once and a
// scatter pass replaces the filling pass.  One thread per slot t: the light node w with
// noff[w] <= t < noff[w + 1] (a binary search), then the members a < b of
// E_w with t - noff[w] = b (b - 1) / 2 + a, merged as in k_light_pairs.  A
// node's C(|E_w|, 2) merges are spread over as many threads, where the
// one-wave-per-node kernel leaves the largest light node's wave running
// long after the others.
__global__ __launch_bounds__(256) void k_light_slots(
    int64_t V, int64_t ncand, const int64_t* __restrict__ node_ptr, const int32_t* __restrict__ node_edges,
    const int8_t* __restrict__ heavy_bit, const int64_t* __restrict__ edge_ptr,
    const int32_t* __restrict__ edge_nodes, const int64_t* __restrict__ lg_ptr,
    unsigned long long* pcount, const int64_t* __restrict__ noff, int2* flat) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ncand) return;
  int64_t lo = 0, hi = V;  // largest w with noff[w] <= t (noff is nondecreasing, noff[V] = ncand > t)
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (noff[mid] <= t) lo = mid; else hi = mid;
  }
  const int64_t w = lo;
  const int64_t r = t - noff[w];
  // b (b - 1) / 2 <= r < b (b + 1) / 2
  int64_t b = int64_t((1.0 + sqrt(1.0 + 8.0 * double(r))) * 0.5);
  while (b * (b - 1) / 2 > r) --b;
  while ((b + 1) * b / 2 <= r) ++b;
  const int64_t a = r - b * (b - 1) / 2;
  const int64_t base = node_ptr[w];
  const int32_t ya = node_edges[base + a], yb = node_edges[base + b];
  if (!smallest_shared_light(ya, yb, int32_t(w), edge_ptr, edge_nodes, heavy_bit)) {
    flat[t] = make_int2(-1, -1);
    return;
  }
  const int64_t da = lg_ptr[ya + 1] - lg_ptr[ya], db = lg_ptr[yb + 1] - lg_ptr[yb];
  const bool a_owns = da > db || (da == db && ya < yb);
  const int32_t owner = a_owns ? ya : yb, partner = a_owns ? yb : ya;
  atomicAdd(&pcount[owner], 1ull);
  flat[t] = make_int2(owner, partner);
}

// Candidate pairs C(|E_w|, 2) of every light node (0 for heavy ones), the
// input of the flat list's offsets; cnt[V] = 0.
__global__ void k_pair_slots(int64_t V, const int64_t* __restrict__ node_ptr,
                             const int8_t* __restrict__ heavy_bit, int64_t* cnt) {
  const int64_t w = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w > V) return;
  int64_t c = 0;
  if (w < V && heavy_bit[w] < 0) {
    const int64_t d = node_ptr[w + 1] - node_ptr[w];
    c = d * (d - 1) / 2;
  }
  cnt[w] = c;
}

// The flat list's pairs into each owner's partner range (cursor[] from zero).
__global__ void k_scatter_pairs(int64_t n, const int2* __restrict__ flat, const int64_t* __restrict__ eoff,
                                unsigned long long* cursor, int32_t* partners) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int2 v = flat[t];
    if (v.x < 0) continue;
    const unsigned long long s = atomicAdd(&cursor[v.x], 1ull);
    partners[eoff[v.x] + int64_t(s)] = v.y;
  }
}

// Workgroups are dealt to the 8 XCDs in turn; block b takes the owner that
// gives each XCD a contiguous range of the owner list (a bijection onto
// [0, nb)), so that owners listed together share one XCD's L2.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b % kXcds, k = b / kXcds, per = nb / kXcds, extra = nb % kXcds;
  return int64_t(x) * per + (x < extra ? x : extra) + k;
}

// One block per work item, an item being up to kFixChunk partners of one
// owner (an owner's items are consecutive, so they run at the same time on
// one XCD and share the owner's row in its L2); 512 threads, so that the LDS
// the row bitmap takes still leaves room for 24 resident waves per CU (the
// scan waits on loads).  128 partners per item build an owner's bitmap half
// as often as 64 (on medium 121 ms against 125; 256 no better).
constexpr int kFixThreads = 512;
constexpr size_t kFlatBytes = size_t(4) << 30;  // largest flat list of candidate light pairs
constexpr int kFixCopies = 2;
constexpr int kFixChunk = 128;

// At most 64 registers (8 waves per SIMD, room for 4 blocks, 32 waves per CU,
// when the LDS allows; the scan waits on loads, so resident waves count more
// than entries per lane).
__global__ __launch_bounds__(kFixThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_light_fix(
    int64_t c0, int64_t c1, const int32_t* __restrict__ row_graph, const int64_t* __restrict__ geoff,
    const int32_t* __restrict__ owners, const int32_t* __restrict__ item_owner,
    const int64_t* __restrict__ ioff, const int64_t* __restrict__ poff,
    const int32_t* __restrict__ partners,
    const int64_t* __restrict__ edge_ptr, const int32_t* __restrict__ edge_nodes,
    const int8_t* __restrict__ heavy_bit, const int64_t* __restrict__ lg_ptr,
    const int32_t* __restrict__ lg_col, const uint32_t* __restrict__ recm,
    const uint16_t* __restrict__ rsz, const uint16_t* __restrict__ code_to_id3,
    unsigned long long* hist_out, uint2* tally) {
  extern __shared__ uint32_t sm[];
  __shared__ uint16_t lut[kNumCodes];
  // kFixCopies histogram copies, lane l adding to copy l % kFixCopies (fewer
  // same-word adds in one instruction); 2 keep a block within 40 KB of LDS on
  // graphs of up to 85k hyperedges, so that 4 blocks reside per CU
  __shared__ unsigned long long hist[kFixCopies * kHistSlots];
  __shared__ int32_t part[kFixThreads];
  __shared__ int32_t ej[MOCHY_MAX_EDGE];  // e_j's nodes (ascending)
  __shared__ uint32_t s_tally[2];  // centres examined, centres reclassified
  const int64_t it = xcd_block(blockIdx.x, gridDim.x);
  const int64_t ob = item_owner[it];
  const int32_t j = owners[ob];
  const int64_t p0 = poff[ob] + (it - ioff[ob]) * kFixChunk;  // this item's partners
  const int64_t p1 = min(poff[ob + 1], p0 + kFixChunk);
  const int gj = row_graph[j];
  const int64_t e0 = geoff[gj];  // row j's graph owns hyperedges [e0, geoff[gj + 1])
  const int nwE = int((geoff[gj + 1] - e0 + 31) / 32);
  uint32_t* bm = sm;          // row j over the graph's hyperedge ids
  uint32_t* rank = sm + nwE;  // set bits before each word
  const int64_t jb = lg_ptr[j];
  const int dj = int(lg_ptr[j + 1] - jb);
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  for (int t = threadIdx.x; t < kFixCopies * kHistSlots; t += blockDim.x) hist[t] = 0;
  for (int w = threadIdx.x; w < nwE; w += blockDim.x) bm[w] = 0;
  const uint32_t sizej = uint32_t(edge_ptr[j + 1] - edge_ptr[j]);
  if (threadIdx.x < sizej) ej[threadIdx.x] = edge_nodes[edge_ptr[j] + threadIdx.x];
  if (threadIdx.x == 0) {
    s_tally[0] = 0u;
    s_tally[1] = 0u;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < dj; p += blockDim.x) {
    const int64_t x = lg_col[jb + p] - e0;
    atomicOr(&bm[x >> 5], 1u << (x & 31));
  }
  __syncthreads();
  {
    const int chunk = (nwE + kFixThreads - 1) / kFixThreads;
    const int w0 = min(nwE, int(threadIdx.x) * chunk), w1 = min(nwE, w0 + chunk);
    int32_t c = 0;
    for (int w = w0; w < w1; ++w) c += __popc(bm[w]);
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kFixThreads; off <<= 1) {
      const int32_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    int32_t run = part[threadIdx.x] - c;
    for (int w = w0; w < w1; ++w) {
      rank[w] = uint32_t(run);
      run += __popc(bm[w]);
    }
  }
  __syncthreads();
  // one partner per wave at a time (rows shorter than a block's sweep leave
  // no lanes idle)
  const int lane = int(threadIdx.x) & (kWave - 1), wave = int(threadIdx.x) / kWave;
  unsigned long long* myhist = hist + (lane & (kFixCopies - 1)) * kHistSlots;
  uint32_t n_centres = 0, n_changed = 0;  // this wave's, for mochy_exact_stats
  for (int64_t pp = p0 + wave; pp < p1; pp += kFixThreads / kWave) {
    const int32_t k = partners[pp];
    // masks over e_k's nodes: e_j ∩ e_k (mkj), its heavy and light nodes
    const int64_t kn0 = edge_ptr[k];
    const uint32_t sizek = uint32_t(edge_ptr[k + 1] - kn0);
    bool in_j = false, heavy = false;
    if (uint32_t(lane) < sizek) {
      const int32_t v = edge_nodes[kn0 + lane];
      in_j = in_sorted(ej, int(sizej), v);
      heavy = heavy_bit[v] >= 0;
    }
    const uint32_t mkj = uint32_t(__ballot(in_j));
    const uint32_t Hk = mkj & uint32_t(__ballot(heavy)), Lk = mkj & ~Hk;
    const int64_t kb = lg_ptr[k];
    const int dk = int(lg_ptr[k + 1] - kb);
    // row k scanned kUnroll entries per thread at a time; the loads of one
    // stage are issued together, with no branch between them (an entry that
    // is not a centre reads a valid dummy slot), since the work is bound by
    // load latency: 3 of 4 scanned entries are centres on hub-heavy graphs
    // (7 entries per lane fit the 64 registers; 8 spill and were slower)
    constexpr int kUnroll = 7;
    constexpr int step = kWave;
    for (int r0 = lane; r0 < dk; r0 += kUnroll * step) {
      int32_t iv[kUnroll];
      uint32_t mki[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int r = r0 + u * step;
        iv[u] = r < dk ? lg_col[kb + r] : -1;
        mki[u] = recm[kb + min(r, dk - 1)];  // e_k ∩ e_i over e_k's nodes
      }
      int qj[kUnroll];
      bool hit[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int32_t i = iv[u];
        const bool in = i >= c0 && i < c1;  // also excludes the -1 past the row's end
        const int64_t il = in ? i - e0 : 0;
        const uint32_t iw = bm[il >> 5];
        const uint32_t ibit = 1u << (il & 31);
        hit[u] = in && (iw & ibit) != 0u;  // a neighbour of e_j (i == j never is)
        qj[u] = hit[u] ? int(rank[il >> 5] + __popc(iw & (ibit - 1u))) : 0;
      }
      uint32_t szj[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) szj[u] = rsz[jb + qj[u]];  // |e_j ∩ e_i| | |e_i| << 8
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        // wave-uniform tallies (a ballot counts the lanes still scanning)
        n_centres += uint32_t(__popcll(__ballot(hit[u])));
        if (!hit[u]) continue;
        const uint32_t ls = __popc(Lk & ~mki[u]);
        n_changed += uint32_t(__popcll(__ballot(ls != 0u)));
        if (ls == 0u) continue;  // the pair kernel was exact at this centre
        const int32_t i = iv[u];
        const uint32_t wik = __popc(mki[u]);
        const uint32_t t = __popc(mki[u] & mkj);
        const uint32_t r5h = __popc(Hk & ~mki[u]);
        const uint32_t pj = szj[u] & 0xffu;
        const uint32_t a = szj[u] >> 8;
        Side K;
        K.m = 0u; K.s = wik; K.o = sizek - wik; K.h = 0ull;
        const uint32_t oj = sizej - pj;
        const bool above = (j > i) && (k > i);
        if (above || (t | r5h) == 0u) atomicAdd(&myhist[lut[pair_code(a, pj, oj, K, t, r5h)]], ~0ull);
        if (above) atomicAdd(&myhist[lut[pair_code(a, pj, oj, K, t, r5h + ls)]], 1ull);
      }
    }
  }
  if (lane == 0 && (n_centres | n_changed) != 0u) {
    atomicAdd(&s_tally[0], n_centres);
    atomicAdd(&s_tally[1], n_changed);
  }
  __syncthreads();
  if (threadIdx.x == 0) tally[it] = make_uint2(s_tally[0], s_tally[1]);  // summed by k_fix_tally
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x) {
    unsigned long long v = 0;
    for (int c = 0; c < kFixCopies; ++c) v += hist[c * kHistSlots + t];
    if (v) atomicAdd(&hist_out[int64_t(gj) * kHistSlots + t], v);
  }
}

// The correction's work counters for mochy_exact_stats: row entries scanned
// (the partner row of every light pair) and the per-item tallies of the fix
// kernel, summed over a fixed grid with one atomic per block and counter
// (atomics on one address from every wave or item would serialize).
constexpr int kTallyBlocks = 256;
__global__ __launch_bounds__(256) void k_fix_tally(int64_t npairs, const int32_t* __restrict__ partners,
                                                   const int64_t* __restrict__ lg_ptr, int64_t nitems,
                                                   const uint2* __restrict__ tally, unsigned long long* stats) {
  __shared__ unsigned long long red[3][256 / kWave];
  unsigned long long v[3] = {0, 0, 0};
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < npairs; p += stride) {
    const int32_t k = partners[p];
    v[0] += (unsigned long long)(lg_ptr[k + 1] - lg_ptr[k]);
  }
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < nitems; q += stride) {
    v[1] += tally[q].x;
    v[2] += tally[q].y;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int x = 0; x < 3; ++x) {
    for (int off = kWave / 2; off > 0; off >>= 1) v[x] += __shfl_xor(v[x], off, kWave);
    if (lane == 0) red[x][wave] = v[x];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    unsigned long long t = 0;
    for (int w = 0; w < 256 / kWave; ++w) t += red[threadIdx.x][w];
    const int slot = threadIdx.x == 0 ? kStFixScanned : threadIdx.x == 1 ? kStFixCentres : kStFixChanged;
    if (t) atomicAdd(&stats[slot], t);
  }
}

// owners: hyperedges with at least one light partner, compacted.
__global__ void k_owner_list(int64_t E, const unsigned long long* __restrict__ pcount,
                             unsigned long long* nown, int32_t* owners, int64_t* ocount) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= E || pcount[x] == 0) return;
  const unsigned long long s = atomicAdd(nown, 1ull);
  owners[s] = int32_t(x);
  ocount[s] = int64_t(pcount[x]);
}

__global__ void k_owner_offsets(int64_t n, const int32_t* __restrict__ owners,
                                const int64_t* __restrict__ poff, int64_t* eoff, int64_t* icount) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < n) {
    eoff[owners[s]] = poff[s];
    icount[s] = (poff[s + 1] - poff[s] + kFixChunk - 1) / kFixChunk;
  }
  if (s == n) icount[n] = 0;
}

// item_owner[q] = the owner of work item q (items of owner s: [ioff[s], ioff[s + 1])).
__global__ void k_item_owners(int64_t n, const int64_t* __restrict__ ioff, int32_t* item_owner) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) return;
  for (int64_t q = ioff[s]; q < ioff[s + 1]; ++q) item_owner[q] = int32_t(s);
}

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

}  // namespace

mochy_status correct_device(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                            int64_t* d_hist, unsigned long long* stats) {
  hipStream_t st = ctx->stream;
  const int64_t E = g->E, V = g->V;
  if (c1 <= c0 || E == 0 || V == 0) return MOCHY_OK;
  const int nwE = int((g->max_graph_edges + 31) / 32);
  const size_t dyn = size_t(nwE) * 8;
  if (dyn > 60 * 1024)
    MOCHY_HIP(hipFuncSetAttribute((const void*)k_light_fix, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  int(dyn)));
  // pcount[E] | nown | owners[E] | ocount[E+1] | poff[E+1] | tmp
  const size_t tmpn = scan_tmp_elems(std::max(E, V) + 1);  // scans of E + 1 and V + 1 entries
  const size_t n64 = size_t(E) + 1 + size_t(E + 1) * 2 + tmpn;
  char* buf = nullptr;
  int64_t* eoff = nullptr;
  int32_t* partners = nullptr;
  int64_t* ioff = nullptr;
  int32_t* item_owner = nullptr;
  uint2* tally = nullptr;
  int64_t* noff = nullptr;
  int2* flat = nullptr;
  auto done = [&](mochy_status s) {
    device_free(ctx, noff);
    device_free(ctx, flat);
    device_free(ctx, buf);
    device_free(ctx, eoff);
    device_free(ctx, partners);
    device_free(ctx, ioff);
    device_free(ctx, item_owner);
    device_free(ctx, tally);
    return s;
  };
  mochy_status rc = device_alloc(ctx, (void**)&buf, n64 * 8 + size_t(E) * 4);
  if (rc != MOCHY_OK) return rc;
  unsigned long long* pcount = (unsigned long long*)buf;
  unsigned long long* nown = pcount + E;
  int64_t* ocount = (int64_t*)(nown + 1);
  int64_t* poff = ocount + (E + 1);
  int64_t* tmp = poff + (E + 1);
  int32_t* owners = (int32_t*)(buf + n64 * 8);
  launch_fill_u32(buf, 0u, (size_t(E) + 1 + size_t(E + 1)) * 8, st);
  const unsigned wblocks = blocks(V * 64, 256);
  // one pass over the candidate pairs into a flat list when it is small
  // (8 bytes per pair of a light node's hyperedges, at most kFlatBytes, not
  // carved from a caller's arena); otherwise a counting pass now and a
  // filling pass once the owners' offsets are known
  int64_t ncand = 0;
  if (!ctx->arena && !(ctx->test_faults & 8)) {
    if ((rc = device_alloc(ctx, (void**)&noff, size_t(V + 1) * 8)) != MOCHY_OK) return done(rc);
    k_pair_slots<<<blocks(V + 1, 256), 256, 0, st>>>(V, g->node_ptr, g->heavy_bit, noff);
    launch_exclusive_scan_i64(noff, noff, V + 1, tmp, st);
    MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small + 503, noff + V, 8, hipMemcpyDeviceToHost, st), done);
    MOCHY_HIP_OR(hipStreamSynchronize(st), done);
    ncand = ctx->h_small[503];
    if (ncand > 0 && size_t(ncand) * 8 <= kFlatBytes &&
        device_alloc(ctx, (void**)&flat, size_t(ncand) * 8) != MOCHY_OK) {
      (void)hipGetLastError();  // no room for the list: the two passes instead
      flat = nullptr;
    }
  }
  if (flat)
    k_light_slots<<<unsigned(blocks(ncand, 256)), 256, 0, st>>>(V, ncand, g->node_ptr, g->node_edges,
                                                              g->heavy_bit, g->edge_ptr, g->edge_nodes,
                                                              g->lg_ptr, pcount, noff, flat);
  else
    k_light_pairs<kCount><<<wblocks, 256, 0, st>>>(V, g->node_ptr, g->node_edges, g->heavy_bit,
                                                   g->edge_ptr, g->edge_nodes, g->lg_ptr, pcount,
                                                   nullptr, nullptr);
  k_owner_list<<<blocks(E, 256), 256, 0, st>>>(E, pcount, nown, owners, ocount);
  MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small + 504, nown, 8, hipMemcpyDeviceToHost, st), done);
  MOCHY_HIP_OR(hipStreamSynchronize(st), done);
  const int64_t nowners = ctx->h_small[504];
  if (nowners == 0) return done(MOCHY_OK);
  launch_exclusive_scan_i64(ocount, poff, nowners + 1, tmp, st);  // ocount[nowners] is 0
  MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small + 505, poff + nowners, 8, hipMemcpyDeviceToHost, st), done);
  MOCHY_HIP_OR(hipStreamSynchronize(st), done);
  const int64_t npairs = ctx->h_small[505];
  ctx->exact_stats[kStLightPairs] += npairs;
  // per-owner offsets indexed by hyperedge id for the fill pass
  if ((rc = device_alloc(ctx, (void**)&eoff, size_t(E) * 8)) != MOCHY_OK) return done(rc);
  if ((rc = device_alloc(ctx, (void**)&partners, size_t(npairs) * 4)) != MOCHY_OK) return done(rc);
  if ((rc = device_alloc(ctx, (void**)&ioff, size_t(nowners + 1) * 8)) != MOCHY_OK) return done(rc);
  // scatter owner offsets to hyperedge ids and count each owner's work items
  // (ioff holds the counts, then their prefix, in place), reset counters, fill
  k_owner_offsets<<<blocks(nowners + 1, 256), 256, 0, st>>>(nowners, owners, poff, eoff, ioff);
  launch_exclusive_scan_i64(ioff, ioff, nowners + 1, tmp, st);
  MOCHY_HIP_OR(hipMemcpyAsync(ctx->h_small + 506, ioff + nowners, 8, hipMemcpyDeviceToHost, st), done);
  launch_fill_u32(pcount, 0u, size_t(E) * 8, st);
  if (flat)
    k_scatter_pairs<<<unsigned(std::min<int64_t>(blocks(ncand, 256), int64_t(ctx->num_cus) * 16)), 256, 0, st>>>(
        ncand, flat, eoff, pcount, partners);
  else
    k_light_pairs<kFill><<<wblocks, 256, 0, st>>>(V, g->node_ptr, g->node_edges, g->heavy_bit,
                                                  g->edge_ptr, g->edge_nodes, g->lg_ptr, pcount, eoff,
                                                  partners);
  MOCHY_HIP_OR(hipStreamSynchronize(st), done);
  const int64_t nitems = ctx->h_small[506];
  if ((rc = device_alloc(ctx, (void**)&item_owner, size_t(nitems) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&tally, size_t(nitems) * 8)) != MOCHY_OK)
    return done(rc);
  k_item_owners<<<blocks(nowners, 256), 256, 0, st>>>(nowners, ioff, item_owner);
  phase_begin(ctx, kPhFix);
  k_light_fix<<<unsigned(nitems), kFixThreads, dyn, st>>>(c0, c1, g->row_graph, g->geoff, owners, item_owner,
                                                          ioff, poff, partners,
                                                           g->edge_ptr, g->edge_nodes, g->heavy_bit, g->lg_ptr,
                                                           g->lg_col, g->recm, g->rsz, ctx->d_code_to_id3,
                                                           (unsigned long long*)d_hist, tally);
  phase_end(ctx, kPhFix);
  k_fix_tally<<<kTallyBlocks, 256, 0, st>>>(npairs, partners, g->lg_ptr, nitems, tally, stats);
  MOCHY_HIP_OR(hipGetLastError(), done);
  MOCHY_HIP_OR(hipStreamSynchronize(st), done);
  return done(MOCHY_OK);
}
