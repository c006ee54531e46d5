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
#include "common.h"

namespace {

constexpr int kCopies = 4;
constexpr int kStride = kHistSlots + 1;  // odd stride spreads the copies over banks

// ---------------------------------------------------------------------------
// Scheduling: rows sorted by number of 64-blocks, descending.

__global__ void k_sched_count(int64_t c0, int64_t c1, const int64_t* __restrict__ lg_ptr,
                              unsigned long long* nbhist) {
  const int64_t i = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= c1) return;
  const int64_t d = lg_ptr[i + 1] - lg_ptr[i];
  if (d < 2) return;
  atomicAdd(&nbhist[(d + kWave - 1) / kWave], 1ull);
}

// Single block: cnt[b] = #rows with more than b blocks; item_start[b] =
// number of items with a larger block index; total = sum_b cnt[b].
__global__ __launch_bounds__(1024) void k_sched_scan(int32_t maxnb,
                                                     const unsigned long long* __restrict__ nbhist,
                                                     int64_t* cnt, int64_t* item_start,
                                                     int64_t* total) {
  __shared__ int64_t part[1024];
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
    if (threadIdx.x == 1023) *total = part[1023];
  }
}

__global__ void k_sched_scatter(int64_t c0, int64_t c1, const int64_t* __restrict__ lg_ptr,
                                const int64_t* __restrict__ cnt, unsigned long long* fill,
                                int32_t* order) {
  const int64_t i = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= c1) return;
  const int64_t d = lg_ptr[i + 1] - lg_ptr[i];
  if (d < 2) return;
  const int64_t nb = (d + kWave - 1) / kWave;
  const unsigned long long slot = atomicAdd(&fill[nb], 1ull);
  order[cnt[nb] + int64_t(slot)] = int32_t(i);
}

// ---------------------------------------------------------------------------
// Classification of one pair, shared by the main and the correction kernels.

struct Side {          // neighbour k held by a lane
  uint32_t m, o, s;    // mask in e_i, outside count, popcount(m)
  unsigned long long h;
};

__device__ __forceinline__ uint32_t st3(uint32_t c) { return c < 2u ? c : 2u; }

// code = sum_r min(R_r, 2) * 3^r with R1 least significant
__device__ __forceinline__ uint32_t pair_code(uint32_t a, uint32_t mj, uint32_t pj, uint32_t oj,
                                              const Side& k, uint32_t t, uint32_t r5) {
  const uint32_t R1 = a + t - pj - k.s;
  const uint32_t R2 = oj - r5;
  const uint32_t R3 = k.o - r5;
  const uint32_t R4 = pj - t;
  const uint32_t R6 = k.s - t;
  uint32_t code = st3(t);                 // R7
  code = code * 3u + st3(R6);
  code = code * 3u + st3(r5);             // R5
  code = code * 3u + st3(R4);
  code = code * 3u + st3(R3);
  code = code * 3u + st3(R2);
  code = code * 3u + st3(R1);
  return code;
}

// Walk j over [j0, j1) against the lane's k.  kCountAll: both j and k are
// above the centre (count every pair); otherwise count only disjoint pairs.
// kDiag: the j range overlaps the lane block, so require j < kp.
template <bool kCountAll, bool kDiag>
__device__ __forceinline__ void walk(const uint4* __restrict__ row, int j0, int j1, uint32_t a,
                                     const Side& k, int kp, bool valid,
                                     const uint16_t* __restrict__ lut, unsigned long long* hist) {
  for (int j = j0; j < j1; ++j) {
    const uint4 rj = row[j];
    const uint32_t mj = rj.x;
    const uint32_t oj = rj.y & 0xffu;
    const unsigned long long hj = (unsigned long long)rj.z | ((unsigned long long)rj.w << 32);
    const uint32_t t = __popc(mj & k.m);
    const uint32_t r5 = __popcll(hj & k.h);
    bool act = valid;
    if (kDiag) act = act && (j < kp);
    if (!kCountAll) act = act && ((t | r5) == 0u);
    if (act) {
      const uint32_t pj = __popc(mj);
      const uint32_t code = pair_code(a, mj, pj, oj, k, t, r5);
      atomicAdd(&hist[lut[code]], 1ull);
    }
  }
}

__global__ __launch_bounds__(256) void k_exact_main(
    const int64_t* __restrict__ edge_ptr, const int64_t* __restrict__ lg_ptr,
    const int32_t* __restrict__ up_first, const uint4* __restrict__ rec,
    const int32_t* __restrict__ order, const int64_t* __restrict__ item_start,
    const int64_t* __restrict__ cnt, int32_t maxnb, const int64_t* __restrict__ total_items,
    unsigned long long* queue, const uint16_t* __restrict__ code_to_id3,
    unsigned long long* hist_out) {
  __shared__ uint16_t lut[kNumCodes];
  __shared__ unsigned long long hist[kCopies * kStride];
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  for (int t = threadIdx.x; t < kCopies * kStride; t += blockDim.x) hist[t] = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long* myhist = hist + (lane & (kCopies - 1)) * kStride;
  const int64_t total = total_items[0];
  int b = maxnb - 1;
  for (;;) {
    unsigned long long qq = 0;
    if (lane == 0) qq = atomicAdd(queue, 1ull);
    const int64_t q = (int64_t)(((unsigned long long)__builtin_amdgcn_readfirstlane(int(qq >> 32)) << 32) |
                                (unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(int(qq)));
    if (q >= total) break;
    // items are ordered by block index descending; q only grows per wave
    while (b > 0 && q >= item_start[b] + cnt[b]) --b;
    const int32_t i = order[q - item_start[b]];
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
    // j below the centre: count disjoint pairs only
    const int ua = min(u, blo);
    walk<false, false>(row, 0, ua, a, k, kp, valid, lut, myhist);
    walk<false, true>(row, max(ua, blo), min(u, kmax), a, k, kp, valid, lut, myhist);
    // j (and so k) above the centre: count every pair
    walk<true, false>(row, u, blo, a, k, kp, valid, lut, myhist);
    walk<true, true>(row, max(u, blo), kmax, a, k, kp, valid, lut, myhist);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x) {
    unsigned long long s = 0;
    for (int c = 0; c < kCopies; ++c) s += hist[c * kStride + t];
    if (s) atomicAdd(&hist_out[t], s);
  }
}

// ---------------------------------------------------------------------------
// Correction for pairs of neighbours that share a light node outside e_i.
// One workgroup per centre.  LDS: the row as a bitmap over hyperedge ids plus
// per-word ranks (position of a neighbour = rank of its bit).

__device__ __forceinline__ bool in_sorted(const int32_t* s, int n, int32_t v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo < n && s[lo] == v;
}

__global__ __launch_bounds__(256) void k_exact_correct(
    int64_t c0, int nwords, const int64_t* __restrict__ edge_ptr,
    const int32_t* __restrict__ edge_nodes, const int64_t* __restrict__ node_ptr,
    const int32_t* __restrict__ node_edges, const int8_t* __restrict__ heavy_bit,
    const int64_t* __restrict__ lg_ptr, const int32_t* __restrict__ lg_col,
    const int32_t* __restrict__ up_first, const uint4* __restrict__ rec,
    const uint16_t* __restrict__ code_to_id3, unsigned long long* hist_out) {
  extern __shared__ uint32_t sm[];
  uint32_t* bm = sm;
  uint32_t* rank = sm + nwords;
  __shared__ uint16_t lut[kNumCodes];
  __shared__ unsigned long long hist[kHistSlots];
  __shared__ int32_t ei[MOCHY_MAX_EDGE];
  __shared__ int32_t part[256];
  const int64_t i = c0 + blockIdx.x;
  const int64_t base = lg_ptr[i];
  const int d = int(lg_ptr[i + 1] - base);
  if (d < 2) return;  // uniform for the block, before any barrier
  const int a = int(edge_ptr[i + 1] - edge_ptr[i]);
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x) hist[t] = 0;
  for (int w = threadIdx.x; w < nwords; w += blockDim.x) bm[w] = 0;
  if (threadIdx.x < unsigned(a)) ei[threadIdx.x] = edge_nodes[edge_ptr[i] + threadIdx.x];
  __syncthreads();
  for (int p = threadIdx.x; p < d; p += blockDim.x) {
    const int32_t x = lg_col[base + p];
    atomicOr(&bm[x >> 5], 1u << (x & 31));
  }
  __syncthreads();
  {
    const int chunk = (nwords + 255) / 256;
    const int w0 = min(nwords, int(threadIdx.x) * chunk), w1 = min(nwords, w0 + chunk);
    int32_t c = 0;
    for (int w = w0; w < w1; ++w) c += __popc(bm[w]);
    part[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
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
  const int u = up_first[i];
  const uint32_t ua = uint32_t(a);
  for (int p = threadIdx.x; p < d; p += blockDim.x) {
    const uint4 rp = rec[base + p];
    if (!(rp.y & kRecLight)) continue;
    const int32_t x = lg_col[base + p];
    const int64_t xs = edge_ptr[x], xe = edge_ptr[x + 1];
    for (int64_t qx = xs; qx < xe; ++qx) {
      const int32_t w = edge_nodes[qx];
      if (heavy_bit[w] >= 0 || in_sorted(ei, a, w)) continue;
      for (int64_t r = node_ptr[w]; r < node_ptr[w + 1]; ++r) {
        const int32_t y = node_edges[r];
        if (y == i || y == x) continue;
        const uint32_t word = bm[y >> 5];
        const uint32_t bit = 1u << (y & 31);
        if (!(word & bit)) continue;
        const int q = int(rank[y >> 5] + __popc(word & (bit - 1u)));
        if (q <= p) continue;
        // light nodes outside e_i shared by e_x and e_y: count and smallest
        int64_t pa = xs, pb = edge_ptr[y];
        const int64_t pe = edge_ptr[y + 1];
        uint32_t shared = 0;
        int32_t smallest = 0x7fffffff;
        while (pa < xe && pb < pe) {
          const int32_t va = edge_nodes[pa], vb = edge_nodes[pb];
          if (va < vb) ++pa;
          else if (va > vb) ++pb;
          else {
            if (heavy_bit[va] < 0 && !in_sorted(ei, a, va)) {
              ++shared;
              smallest = min(smallest, va);
            }
            ++pa; ++pb;
          }
        }
        if (smallest != w) continue;  // handled at the smallest shared light node
        const uint4 rq = rec[base + q];
        Side k;
        k.m = rq.x; k.o = rq.y & 0xffu; k.s = __popc(rq.x);
        k.h = (unsigned long long)rq.z | ((unsigned long long)rq.w << 32);
        const uint32_t mj = rp.x, oj = rp.y & 0xffu, pj = __popc(rp.x);
        const unsigned long long hj = (unsigned long long)rp.z | ((unsigned long long)rp.w << 32);
        const uint32_t t = __popc(mj & k.m);
        const uint32_t r5h = __popcll(hj & k.h);
        const bool above = (p >= u) && (q >= u);
        // what the main kernel recorded
        if (above || (t | r5h) == 0u)
          atomicAdd(&hist[lut[pair_code(ua, mj, pj, oj, k, t, r5h)]], ~0ull);  // -1
        // the exact class: e_j and e_k meet, so counted iff both are above e_i
        if (above)
          atomicAdd(&hist[lut[pair_code(ua, mj, pj, oj, k, t, r5h + shared)]], 1ull);
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x)
    if (hist[t]) atomicAdd(&hist_out[t], hist[t]);
}

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

}  // namespace

mochy_status exact_device(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                          int64_t* d_hist) {
  hipStream_t st = ctx->stream;
  MOCHY_HIP(hipMemsetAsync(d_hist, 0, kHistSlots * 8, st));
  if (c1 <= c0 || g->max_deg < 2) return MOCHY_OK;
  const int32_t maxnb = (g->max_deg + kWave - 1) / kWave;
  // scratch: nbhist[maxnb+1], cnt[maxnb+1], item_start[maxnb], fill[maxnb+1], total, queue, order[E]
  const size_t n8 = size_t(maxnb + 1) * 4 + 4;
  const size_t bytes = n8 * 8 + size_t(c1 - c0) * 4;
  char* scratch = nullptr;
  mochy_status rc = device_alloc(ctx, (void**)&scratch, bytes);
  if (rc != MOCHY_OK) return rc;
  unsigned long long* nbhist = (unsigned long long*)scratch;
  int64_t* cnt = (int64_t*)(nbhist + (maxnb + 1));
  int64_t* item_start = cnt + (maxnb + 1);
  unsigned long long* fill = (unsigned long long*)(item_start + (maxnb + 1));
  int64_t* total = (int64_t*)(fill + (maxnb + 1));
  unsigned long long* queue = (unsigned long long*)(total + 1);
  int32_t* order = (int32_t*)(scratch + n8 * 8);
  MOCHY_HIP(hipMemsetAsync(scratch, 0, n8 * 8, st));
  const int64_t rows = c1 - c0;
  k_sched_count<<<blocks(rows, 256), 256, 0, st>>>(c0, c1, g->lg_ptr, nbhist);
  k_sched_scan<<<1, 1024, 0, st>>>(maxnb, nbhist, cnt, item_start, total);
  k_sched_scatter<<<blocks(rows, 256), 256, 0, st>>>(c0, c1, g->lg_ptr, cnt, fill, order);
  const unsigned grid = unsigned(ctx->num_cus) * 8u;
  k_exact_main<<<grid, 256, 0, st>>>(g->edge_ptr, g->lg_ptr, g->up_first, g->rec, order, item_start,
                                     cnt, maxnb, total, queue, ctx->d_code_to_id3,
                                     (unsigned long long*)d_hist);
  const int nwords = int((g->E + 31) / 32);
  k_exact_correct<<<unsigned(rows), 256, size_t(nwords) * 8, st>>>(
      c0, nwords, g->edge_ptr, g->edge_nodes, g->node_ptr, g->node_edges, g->heavy_bit, g->lg_ptr,
      g->lg_col, g->up_first, g->rec, ctx->d_code_to_id3, (unsigned long long*)d_hist);
  MOCHY_HIP(hipGetLastError());
  MOCHY_HIP(hipStreamSynchronize(st));
  (void)hipFree(scratch);
  return MOCHY_OK;
}
