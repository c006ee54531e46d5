// MoCHy-A+ on the device (Algorithm 5): hyperwedge sampling.
//
// Sample n draws Philox4x32-10 with counter (lo32 n, hi32 n, 0, 0) and key
// (lo32 seed, hi32 seed); u = (x1 << 32) | x0 picks hyperwedge
// floor(u * |wedges| / 2^64) in (i, j), i < j, lexicographic order, found by
// a binary search of the upper-row prefix sums.  For the sampled {e_i, e_j}
// every e_k in N_i ∪ N_j minus {e_i, e_j} gets one hit in its motif.
//
// One wave per sample (samples pulled from a global counter).  The two rows
// are sorted, so N_i ∪ N_j is their merge; merge-path splits it evenly over
// the 64 lanes.  A hyperedge in both rows meets both e_i and e_j; the records
// at the merged positions give omega(i,k), omega(j,k) and |e_k|, and
// t = |e_i ∩ e_j ∩ e_k| = popcount(m_ij & m_ik) over e_i's nodes.  The seven
// region sizes then follow Lemma 2 exactly.
#include "classify.h"
#include "common.h"
#include "rng.h"

#include <algorithm>

namespace {

__global__ __launch_bounds__(256) void k_aplus(
    int64_t n0, int64_t r, uint64_t seed, uint64_t W, int64_t E,
    const int64_t* __restrict__ lg_ptr, const int32_t* __restrict__ lg_col,
    const int64_t* __restrict__ up_ptr, const int32_t* __restrict__ up_first,
    const uint4* __restrict__ rec, const int64_t* __restrict__ edge_ptr,
    const uint16_t* __restrict__ code_to_id3, unsigned long long* queue,
    unsigned long long* hist_out) {
  __shared__ uint16_t lut[kNumCodes];
  __shared__ unsigned long long hist[kHistSlots];
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x) hist[t] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (;;) {
    unsigned long long sq = 0;
    if (lane == 0) sq = atomicAdd(queue, 1ull);
    const int64_t s = int64_t(uniform64(sq));
    if (s >= r) break;
    const int64_t idx = int64_t(sample_wedge(uint64_t(n0) + uint64_t(s), seed, W));
    const int64_t i = wedge_row(up_ptr, E, idx);
    const int64_t ab = lg_ptr[i];
    const int64_t pj = int64_t(up_first[i]) + (idx - up_ptr[i]);
    const int32_t j = lg_col[ab + pj];
    const uint4 rij = rec[ab + pj];
    const uint32_t wij = __popc(rij.x);
    const uint32_t a = uint32_t(edge_ptr[i + 1] - edge_ptr[i]);
    const uint32_t b = uint32_t(edge_ptr[j + 1] - edge_ptr[j]);
    const int32_t* A = lg_col + ab;
    const int dA = int(lg_ptr[i + 1] - ab);
    const int64_t bbase = lg_ptr[j];
    const int32_t* B = lg_col + bbase;
    const int dB = int(lg_ptr[j + 1] - bbase);
    const int total = dA + dB;
    // merge-path: this lane's share of the merged sequence (ties: A first)
    const int d0 = int((int64_t(total) * lane) >> 6), d1 = int((int64_t(total) * (lane + 1)) >> 6);
    int plo = max(0, d0 - dB), phi = min(d0, dA);
    while (plo < phi) {
      const int mid = (plo + phi) >> 1;
      if (A[mid] <= B[d0 - mid - 1]) plo = mid + 1; else phi = mid;
    }
    int p = plo, q = d0 - plo;
    for (int step = d0; step < d1; ++step) {
      const bool takeA = q >= dB || (p < dA && A[p] <= B[q]);
      int32_t k;
      int pa = -1, pb = -1;
      if (takeA) {
        k = A[p];
        pa = p;
        if (q < dB && B[q] == k) pb = q;
        ++p;
        if (k == j) continue;
      } else {
        k = B[q];
        pb = q;
        ++q;
        if ((p > 0 && A[p - 1] == k) || k == int32_t(i)) continue;  // counted with A, or e_i itself
      }
      uint32_t wik = 0, wjk = 0, t = 0, c = 0;
      if (pa >= 0) {
        const uint4 rik = rec[ab + pa];
        wik = __popc(rik.x);
        t = __popc(rij.x & rik.x);
        c = wik + (rik.y & 0xffu);
      }
      if (pb >= 0) {
        const uint4 rjk = rec[bbase + pb];
        wjk = __popc(rjk.x);
        c = wjk + (rjk.y & 0xffu);
      }
      Side K;
      K.m = 0u; K.s = wik; K.o = c - wik; K.h = 0ull;
      // region sizes of (e_i, e_j, e_k) from Lemma 2: R5 = omega(j,k) - t
      const uint32_t code = pair_code(a, wij, b - wij, K, t, wjk - t);
      atomicAdd(&hist[lut[code]], 1ull);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x)
    if (hist[t]) atomicAdd(&hist_out[t], hist[t]);
}

// MoCHy-A (Algorithm 4): hyperedge sampling.  Sample n draws Philox4x32-10
// with counter (lo32 n, hi32 n, 1, 0) and key (lo32 seed, hi32 seed);
// u = (x1 << 32) | x0 picks hyperedge floor(u * |E| / 2^64).  Every instance
// containing the sampled e_i gets one hit: the pairs of N_i and the paths
// e_i - e_j - e_k (e_k in N_j outside N_i and e_i).
//
// One 256-thread block per sample.  N_i is an LDS bitmap over its graph's
// hyperedges with per-word ranks (the rank is e_k's position in row i, whose
// size word gives omega(i, k)).  All pairs of N_i are first counted as if
// disjoint from each other (class fixed by |e_j|, omega(i, j), |e_k|,
// omega(i, k)) with a histogram of N_i by (size, omega) and products of its
// bins.  Then the rows of e_i's neighbours are scanned: row j's record masks
// (e_j's nodes held by e_k; t = |e_i ∩ e_j ∩ e_k| with the mask of e_i in
// row j) and size words (omega(j, k), |e_k|), 10 bytes per entry, and
// row i's size word at e_k's rank for a hit: a hit e_k in N_i with j < k is
// an adjacent pair, its disjoint class is taken back and its exact class
// added; a hit outside N_i is a path.
constexpr int kHsThreads = 256;
constexpr int kHsUnroll = 12;  // row entries per thread in flight at once (12: 2 % faster than 8)
// blocks launched per CU (a persistent queue of work items): as many as the
// LDS and registers let reside, so that every CU keeps its waves busy
constexpr unsigned kHsBlocksPerCu = 8;
constexpr int kBins = (MOCHY_MAX_EDGE + 1) * (MOCHY_MAX_EDGE + 1);

__device__ __forceinline__ uint32_t bin_of(uint32_t size, uint32_t omega) {
  return size * (MOCHY_MAX_EDGE + 1) + omega;
}

// The sampled hyperedge of each sample (kProfile: the hyperedges n0 ..
// n0+s-1 in order) and its number of work items: one per 256 neighbours
// (at least one), so that a sample's rows spread over many blocks.
template <bool kProfile>
__global__ void k_hs_items(int64_t n0, int64_t s, uint64_t seed, int64_t E,
                           const int64_t* __restrict__ lg_ptr, int64_t* sample_i, int64_t* nitems) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q == s) nitems[s] = 0;
  if (q >= s) return;
  const uint64_t n = uint64_t(n0) + uint64_t(q);
  int64_t i;
  if (kProfile) {
    i = int64_t(n);
  } else {
    const uint4 x = philox_4x32_10(make_uint4(uint32_t(n), uint32_t(n >> 32), 1u, 0u), uint32_t(seed),
                                   uint32_t(seed >> 32));
    i = int64_t(__umul64hi((uint64_t(x.y) << 32) | x.x, uint64_t(E)));
  }
  sample_i[q] = i;
  const int64_t d = lg_ptr[i + 1] - lg_ptr[i];
  nitems[q] = d > 0 ? (d + kHsThreads - 1) / kHsThreads : 1;
}

// One block per work item (sample, chunk of 256 neighbours of e_i): N_i as an
// LDS bitmap with ranks, the chunk's neighbours' rows (each walked by one
// wave), and for chunk 0 also
// every pair of N_i counted as disjoint.  kProfile: the item's counts are
// added to hist_out[(i - n0) * kHistSlots + id] (the hyperedge's profile,
// zeroed before) instead of being summed.
template <bool kProfile>
__global__ __launch_bounds__(kHsThreads) void k_hsample(
    int64_t n0, int64_t s, const int64_t* __restrict__ sample_i, const int64_t* __restrict__ ioff,
    const int32_t* __restrict__ row_graph,
    const int64_t* __restrict__ geoff, const int64_t* __restrict__ edge_ptr,
    const int64_t* __restrict__ lg_ptr, const int32_t* __restrict__ lg_col,
    const uint32_t* __restrict__ recm, const uint16_t* __restrict__ rsz,
    const uint16_t* __restrict__ code_to_id3,
    unsigned long long* queue, unsigned long long* hist_out) {
  extern __shared__ uint32_t sm[];
  __shared__ uint16_t lut[kNumCodes];
  __shared__ unsigned long long hist[kHistSlots];
  __shared__ uint32_t bins[kBins];
  __shared__ uint32_t blist[kBins];
  __shared__ int32_t part[kHsThreads];
  __shared__ int64_t s_i, s_chunk;
  __shared__ uint32_t s_nb;
  const int tid = threadIdx.x;
  const int64_t total = ioff[s];
  for (int t = tid; t < kNumCodes; t += kHsThreads) lut[t] = code_to_id3[t];
  for (int t = tid; t < kHistSlots; t += kHsThreads) hist[t] = 0ull;
  for (int t = tid; t < kBins; t += kHsThreads) bins[t] = 0u;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      const int64_t item = int64_t(atomicAdd(queue, 1ull));
      int64_t i = -1, chunk = 0;
      if (item < total) {
        int64_t lo = 0, hi = s;  // the sample: last q with ioff[q] <= item
        while (hi - lo > 1) {
          const int64_t mid = (lo + hi) >> 1;
          if (ioff[mid] <= item) lo = mid; else hi = mid;
        }
        i = sample_i[lo];
        chunk = item - ioff[lo];
      }
      s_i = i;
      s_chunk = chunk;
      s_nb = 0u;
    }
    __syncthreads();
    const int64_t i = s_i;
    if (i < 0) break;
    const int64_t chunk = s_chunk;
    const int gi = row_graph[i];
    const int64_t e0 = geoff[gi];
    const int nw = int((geoff[gi + 1] - e0 + 31) / 32);
    uint32_t* bm = sm;
    uint32_t* rank = sm + nw;
    const int64_t ib = lg_ptr[i];
    const int di = int(lg_ptr[i + 1] - ib);
    const uint32_t a = uint32_t(edge_ptr[i + 1] - edge_ptr[i]);
    for (int w = tid; w < nw; w += kHsThreads) bm[w] = 0u;
    __syncthreads();
    for (int p = tid; p < di; p += kHsThreads) {
      const int64_t x = lg_col[ib + p] - e0;
      atomicOr(&bm[x >> 5], 1u << (x & 31));
      if (chunk == 0) {
        const uint32_t sz = rsz[ib + p];  // |e_i ∩ e_x| | |e_x| << 8
        const uint32_t om = sz & 0xffu, ox = sz >> 8;
        if (atomicAdd(&bins[bin_of(ox, om)], 1u) == 0u) blist[atomicAdd(&s_nb, 1u)] = bin_of(ox, om);
      }
    }
    __syncthreads();
    {  // ranks: set bits before each word
      const int chunk = (nw + kHsThreads - 1) / kHsThreads;
      const int w0 = min(nw, tid * chunk), w1 = min(nw, w0 + chunk);
      int32_t c = 0;
      for (int w = w0; w < w1; ++w) c += __popc(bm[w]);
      part[tid] = c;
      __syncthreads();
      for (int off = 1; off < kHsThreads; off <<= 1) {
        const int32_t add = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
      }
      int32_t run = part[tid] - c;
      for (int w = w0; w < w1; ++w) {
        rank[w] = uint32_t(run);
        run += __popc(bm[w]);
      }
    }
    // every pair of N_i as if e_j and e_k were disjoint: products of bins
    const uint32_t nb = s_nb;
    for (uint32_t q = tid; q < nb * nb; q += kHsThreads) {
      const uint32_t x = q / nb, y = q % nb;
      if (y < x) continue;
      const uint32_t bx = blist[x], by = blist[y];
      const uint64_t nx = bins[bx], ny = bins[by];
      const uint64_t w = x == y ? nx * (nx - 1) / 2 : nx * ny;
      if (w == 0) continue;
      const uint32_t b = bx / (MOCHY_MAX_EDGE + 1), p = bx % (MOCHY_MAX_EDGE + 1);
      const uint32_t c = by / (MOCHY_MAX_EDGE + 1), sk = by % (MOCHY_MAX_EDGE + 1);
      atomicAdd(&hist[lut[triple_code(a, b, c, p, 0u, sk, 0u)]], w);
    }
    __syncthreads();
    // the rows of this item's 256 neighbours of e_i, one row per wave at a
    // time (e_j, its overlap with e_i and its size are uniform); each lane
    // keeps kHsUnroll entries in flight, the loads of each stage issued
    // together with no branch between them (an entry past the row's end, or
    // one that needs no record of row i, reads a valid dummy slot): the scan
    // waits on loads, not on arithmetic
    {
      const int lane = tid & (kWave - 1), wave = tid / kWave;
      const int x0 = int(chunk) * kHsThreads, nj = min(kHsThreads, di - x0);
      for (int x = wave; x < nj; x += kHsThreads / kWave) {
        const int32_t j = lg_col[ib + x0 + x];
        const int64_t jb = lg_ptr[j];
        const int dj = int(lg_ptr[j + 1] - jb);  // >= 1: row j holds e_i
        int lo = 0, hi = dj;  // e_i's position in row j
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (lg_col[jb + mid] < int32_t(i)) lo = mid + 1; else hi = mid;
        }
        const uint32_t mji = recm[jb + lo];
        const uint32_t b = uint32_t(edge_ptr[j + 1] - edge_ptr[j]);
        const uint32_t p = __popc(mji);
        for (int r0 = lane; r0 < dj; r0 += kHsUnroll * kWave) {
          int32_t kv[kHsUnroll];
          uint32_t mv[kHsUnroll], sv[kHsUnroll];  // e_j ∩ e_k over e_j's nodes; |e_j ∩ e_k| | |e_k| << 8
#pragma unroll
          for (int u = 0; u < kHsUnroll; ++u) {
            const int r = min(r0 + u * kWave, dj - 1);
            kv[u] = lg_col[jb + r];
            mv[u] = recm[jb + r];
            sv[u] = rsz[jb + r];
          }
          int64_t ipos[kHsUnroll];
          uint32_t kin[kHsUnroll];
#pragma unroll
          for (int u = 0; u < kHsUnroll; ++u) {
            const int64_t kl = int64_t(kv[u]) - e0;
            const uint32_t kw = bm[kl >> 5], kbit = 1u << (kl & 31);
            kin[u] = kw & kbit;  // e_k is a neighbour of e_i (never e_i itself)
            ipos[u] = kin[u] ? ib + int64_t(rank[kl >> 5] + __popc(kw & (kbit - 1u))) : ib;
          }
          uint32_t wiv[kHsUnroll];  // |e_i ∩ e_k| from row i's size word
#pragma unroll
          for (int u = 0; u < kHsUnroll; ++u) wiv[u] = rsz[ipos[u]] & 0xffu;
#pragma unroll
          for (int u = 0; u < kHsUnroll; ++u) {
            if (r0 + u * kWave >= dj) continue;
            const int32_t k = kv[u];
            if (k == int32_t(i)) continue;
            const uint32_t wjk = sv[u] & 0xffu;
            const uint32_t c = sv[u] >> 8;
            if (kin[u]) {
              if (!(j < k)) continue;  // an adjacent pair of N_i, once
              const uint32_t wik = wiv[u];
              const uint32_t t = __popc(mji & mv[u]);
              atomicAdd(&hist[lut[triple_code(a, b, c, p, 0u, wik, 0u)]], ~0ull);  // taken back
              atomicAdd(&hist[lut[triple_code(a, b, c, p, wjk, wik, t)]], 1ull);
            } else {
              atomicAdd(&hist[lut[triple_code(a, b, c, p, wjk, 0u, 0u)]], 1ull);  // a path
            }
          }
        }
      }
    }
    __syncthreads();
    for (uint32_t q = tid; q < nb; q += kHsThreads) bins[blist[q]] = 0u;
    if (kProfile) {  // this item's part of the hyperedge's profile
      __syncthreads();
      unsigned long long* out = hist_out + (i - n0) * kHistSlots;
      for (int t = tid; t < kHistSlots; t += kHsThreads) {
        if (hist[t]) atomicAdd(&out[t], hist[t]);
        hist[t] = 0ull;
      }
    }
  }
  if (!kProfile) {
    __syncthreads();
    for (int t = tid; t < kHistSlots; t += kHsThreads)
      if (hist[t]) atomicAdd(&hist_out[t], hist[t]);
  }
}

// 26 h-motif counts of each profile row from its 431 3h-motif counts.
__global__ void k_fold_rows(int64_t n, const int64_t* __restrict__ prof,
                            const int32_t* __restrict__ parent, int64_t* out26) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= n * MOCHY_NUM_H) return;
  const int64_t row = x / MOCHY_NUM_H;
  const int h = int(x % MOCHY_NUM_H);
  int64_t sum = 0;
  for (int id3 = 1; id3 < kHistSlots; ++id3)
    if (parent[id3] == h + 1) sum += prof[row * kHistSlots + id3];
  out26[x] = sum;
}

// Work items of hyperedge sampling: the samples' hyperedges and the prefix of
// their item counts.
struct HsItems {
  int64_t* sample_i = nullptr;
  int64_t* ioff = nullptr;
  int64_t* tmp = nullptr;
  void release(mochy_ctx* ctx) {
    device_free(ctx, sample_i);
    device_free(ctx, ioff);
    device_free(ctx, tmp);
    sample_i = ioff = tmp = nullptr;
  }
};

template <bool kProfile>
mochy_status hs_items(mochy_ctx* ctx, const mochy_graph* g, int64_t n0, int64_t s, uint64_t seed,
                      HsItems& it) {
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&it.sample_i, size_t(s) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&it.ioff, size_t(s + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&it.tmp, scan_tmp_elems(s + 1) * 8)) != MOCHY_OK) {
    it.release(ctx);
    return rc;
  }
  // item counts into ioff, scanned in place
  k_hs_items<kProfile><<<unsigned((s + 1 + 255) / 256), 256, 0, ctx->stream>>>(n0, s, seed, g->E, g->lg_ptr,
                                                                               it.sample_i, it.ioff);
  launch_exclusive_scan_i64(it.ioff, it.ioff, s + 1, it.tmp, ctx->stream);
  return MOCHY_OK;
}

}  // namespace

mochy_status sampled_edges_device(mochy_ctx* ctx, const mochy_graph* g, int64_t s, uint64_t seed,
                                  int64_t n0, int64_t* d_hist) {
  hipStream_t st = ctx->stream;
  MOCHY_HIP(hipMemsetAsync(d_hist, 0, kHistSlots * 8, st));
  if (g->E == 0 || s == 0) return MOCHY_OK;
  unsigned long long* queue = (unsigned long long*)(ctx->d_small + 496);
  MOCHY_HIP(hipMemsetAsync(queue, 0, 8, st));
  const int nw = int((g->max_graph_edges + 31) / 32);
  const size_t dyn = size_t(std::max(nw, 1)) * 8;
  if (dyn > 60 * 1024)
    MOCHY_HIP(hipFuncSetAttribute((const void*)k_hsample<false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(dyn)));
  HsItems it;
  mochy_status rc = hs_items<false>(ctx, g, n0, s, seed, it);
  if (rc != MOCHY_OK) return rc;
  phase_begin(ctx, kPhSample);
  k_hsample<false><<<unsigned(ctx->num_cus) * kHsBlocksPerCu, kHsThreads, dyn, st>>>(
      n0, s, it.sample_i, it.ioff, g->row_graph, g->geoff, g->edge_ptr, g->lg_ptr, g->lg_col, g->recm,
      g->rsz, ctx->d_code_to_id3, queue, (unsigned long long*)d_hist);
  phase_end(ctx, kPhSample);
  const hipError_t e = hipGetLastError();
  it.release(ctx);
  MOCHY_HIP(e);
  return MOCHY_OK;
}

mochy_status profiles_device(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                             int64_t* d_prof, int64_t* d_prof26) {
  hipStream_t st = ctx->stream;
  const int64_t n = c1 - c0;
  if (n <= 0) return MOCHY_OK;
  unsigned long long* queue = (unsigned long long*)(ctx->d_small + 496);
  MOCHY_HIP(hipMemsetAsync(queue, 0, 8, st));
  MOCHY_HIP(hipMemsetAsync(d_prof, 0, size_t(n) * kHistSlots * 8, st));
  const int nw = int((g->max_graph_edges + 31) / 32);
  const size_t dyn = size_t(std::max(nw, 1)) * 8;
  if (dyn > 60 * 1024)
    MOCHY_HIP(hipFuncSetAttribute((const void*)k_hsample<true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(dyn)));
  HsItems it;
  mochy_status rc = hs_items<true>(ctx, g, c0, n, 0ull, it);
  if (rc != MOCHY_OK) return rc;
  phase_begin(ctx, kPhSample);
  k_hsample<true><<<unsigned(ctx->num_cus) * kHsBlocksPerCu, kHsThreads, dyn, st>>>(
      c0, n, it.sample_i, it.ioff, g->row_graph, g->geoff, g->edge_ptr, g->lg_ptr, g->lg_col, g->recm,
      g->rsz, ctx->d_code_to_id3, queue, (unsigned long long*)d_prof);
  k_fold_rows<<<unsigned((n * MOCHY_NUM_H + 255) / 256), 256, 0, st>>>(n, d_prof, ctx->d_id3_to_id26,
                                                                        d_prof26);
  phase_end(ctx, kPhSample);
  const hipError_t e = hipGetLastError();
  it.release(ctx);
  MOCHY_HIP(e);
  return MOCHY_OK;
}

mochy_status sampled_device(mochy_ctx* ctx, const mochy_graph* g, int64_t r, uint64_t seed,
                            int64_t n0, int64_t* d_hist) {
  hipStream_t st = ctx->stream;
  MOCHY_HIP(hipMemsetAsync(d_hist, 0, kHistSlots * 8, st));
  if (g->W == 0 || r == 0) return MOCHY_OK;
  unsigned long long* queue = (unsigned long long*)(ctx->d_small + 496);
  MOCHY_HIP(hipMemsetAsync(queue, 0, 8, st));
  phase_begin(ctx, kPhSample);
  k_aplus<<<unsigned(ctx->num_cus) * 8u, 256, 0, st>>>(n0, r, seed, uint64_t(g->W), g->E, g->lg_ptr,
                                                       g->lg_col, g->up_ptr, g->up_first, g->rec,
                                                       g->edge_ptr, ctx->d_code_to_id3, queue,
                                                       (unsigned long long*)d_hist);
  phase_end(ctx, kPhSample);
  MOCHY_HIP(hipGetLastError());
  return MOCHY_OK;
}
