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

}  // namespace

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
