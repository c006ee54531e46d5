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

__global__ void k_sched_count(int64_t c0, int64_t c1, int32_t NB, const int64_t* __restrict__ lg_ptr,
                              const int32_t* __restrict__ row_graph, unsigned long long* nbhist) {
  const int64_t i = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= c1) return;
  const int64_t d = lg_ptr[i + 1] - lg_ptr[i];
  if (d < 2) return;
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
                              const int64_t* __restrict__ lg_ptr, int64_t* nbk) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k > n) return;
  int64_t v = 0;
  if (k < n && order[k] >= 0) {
    const int32_t i = order[k];
    v = (lg_ptr[i + 1] - lg_ptr[i] + kWave - 1) / kWave;
  }
  nbk[k] = v;
}

__global__ void k_sched_scatter(int64_t c0, int64_t c1, int32_t NB, const int64_t* __restrict__ lg_ptr,
                                const int32_t* __restrict__ row_graph,
                                const int64_t* __restrict__ cnt, const int64_t* __restrict__ seg,
                                unsigned long long* fill, int32_t* order) {
  const int64_t i = c0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= c1) return;
  const int64_t d = lg_ptr[i + 1] - lg_ptr[i];
  if (d < 2) return;
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

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

}  // namespace

mochy_status exact_device(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                          int64_t* d_hist) {
  hipStream_t st = ctx->stream;
  const int ng = g->ng;
  MOCHY_HIP(hipMemsetAsync(d_hist, 0, size_t(ng) * kHistSlots * 8, st));
  if (c1 <= c0 || g->max_deg < 2) return MOCHY_OK;
  const int32_t maxnb = (g->max_deg + kWave - 1) / kWave;
  const int64_t NB = maxnb + 1;
  const int64_t rows = c1 - c0;
  // scratch (8-byte slots): nbhist, cnt, item_start, fill [ng*NB each], total [ng],
  // gq [ng+1], seg [ng], queue [1], rstart [rows+1], tmp; then order [rows] int32
  const size_t tmpn = scan_tmp_elems(rows + 1);
  const size_t n8 = size_t(ng) * NB * 4 + size_t(ng) * 3 + 2 + size_t(rows + 1) * 2 + tmpn;
  char* scratch = nullptr;
  mochy_status rc = device_alloc(ctx, (void**)&scratch, n8 * 8 + size_t(rows) * 4);
  if (rc != MOCHY_OK) return rc;
  unsigned long long* nbhist = (unsigned long long*)scratch;
  int64_t* cnt = (int64_t*)(nbhist + ng * NB);
  int64_t* item_start = cnt + ng * NB;
  unsigned long long* fill = (unsigned long long*)(item_start + ng * NB);
  int64_t* total = (int64_t*)(fill + ng * NB);
  int64_t* gq = total + ng;
  int64_t* seg = gq + (ng + 1);
  unsigned long long* queue = (unsigned long long*)(seg + ng);
  int64_t* nbk = (int64_t*)(queue + 1);
  int64_t* rstart = nbk + (rows + 1);
  int64_t* tmp = rstart + (rows + 1);
  int32_t* order = (int32_t*)(scratch + n8 * 8);
  phase_begin(ctx, kPhSched);
  MOCHY_HIP(hipMemsetAsync(scratch, 0, (size_t(ng) * NB * 4 + size_t(ng) * 3 + 2) * 8, st));
  MOCHY_HIP(hipMemsetAsync(order, 0xff, size_t(rows) * 4, st));
  k_sched_count<<<blocks(rows, 256), 256, 0, st>>>(c0, c1, int32_t(NB), g->lg_ptr, g->row_graph, nbhist);
  k_sched_scan<<<unsigned(ng), 1024, 0, st>>>(maxnb, nbhist, cnt, item_start, total);
  k_sched_graphs<<<1, 1024, 0, st>>>(ng, c0, c1, g->geoff, total, gq, seg);
  k_sched_scatter<<<blocks(rows, 256), 256, 0, st>>>(c0, c1, int32_t(NB), g->lg_ptr, g->row_graph, cnt,
                                                     seg, fill, order);
  k_item_counts<<<blocks(rows + 1, 256), 256, 0, st>>>(rows, order, g->lg_ptr, nbk);
  launch_exclusive_scan_i64(nbk, rstart, rows + 1, tmp, st);
  phase_end(ctx, kPhSched);
  const unsigned grid = unsigned(ctx->num_cus) * 8u;
  phase_begin(ctx, kPhPairs);
  k_exact_main<<<grid, 256, 0, st>>>(g->edge_ptr, g->lg_ptr, g->up_first, g->rec, order, rstart, rows,
                                     g->row_graph, queue, ctx->d_code_to_id3,
                                     (unsigned long long*)d_hist);
  phase_end(ctx, kPhPairs);
  phase_begin(ctx, kPhCorrect);
  rc = correct_device(ctx, g, c0, c1, d_hist);
  if (rc != MOCHY_OK) { device_free(ctx, scratch); return rc; }
  phase_end(ctx, kPhCorrect);
  MOCHY_HIP(hipGetLastError());
  MOCHY_HIP(hipStreamSynchronize(st));
  phases_collect(ctx);
  device_free(ctx, scratch);
  return MOCHY_OK;
}
