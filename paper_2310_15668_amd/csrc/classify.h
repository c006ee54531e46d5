// Region classification of a triple of hyperedges, shared by the exact and
// sampled kernels (Lemma 2: region sizes from |e_i|, the two overlaps with
// e_i, the triple overlap and the overlap of e_j and e_k outside e_i).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct Side {          // a neighbour of the centre
  uint32_t m, o, s;    // mask of e_i's nodes it holds, nodes outside e_i, popcount(m)
  unsigned long long h;
};

__device__ __forceinline__ uint32_t st3(uint32_t c) { return c < 2u ? c : 2u; }

// Ternary code sum_r min(R_r, 2) * 3^r (R1 least significant) of the triple
// (e_i, e_j, e_k): a = |e_i|, j given by (pj = popcount(mj), oj), k by `k`,
// t = |e_i ∩ e_j ∩ e_k|, r5 = |e_j ∩ e_k - e_i|.
__device__ __forceinline__ uint32_t pair_code(uint32_t a, uint32_t pj, uint32_t oj, const Side& k,
                                              uint32_t t, uint32_t r5) {
  const uint32_t R1 = a + t - pj - k.s;
  const uint32_t R2 = oj - r5;
  const uint32_t R3 = k.o - r5;
  const uint32_t R4 = pj - t;
  const uint32_t R6 = k.s - t;
  // Horner steps as 24-bit multiply-adds (full-rate on CDNA)
  uint32_t code = st3(t);                                   // R7
  code = __umul24(code, 3u) + st3(R6);
  code = __umul24(code, 3u) + st3(r5);                      // R5
  code = __umul24(code, 3u) + st3(R4);
  code = __umul24(code, 3u) + st3(R3);
  code = __umul24(code, 3u) + st3(R2);
  code = __umul24(code, 3u) + st3(R1);
  return code;
}

// The same code from the three sizes and the four overlaps of Lemma 2:
// a = |e_i|, b = |e_j|, c = |e_k|, p = |e_i ∩ e_j|, q = |e_j ∩ e_k|,
// s = |e_k ∩ e_i|, t = |e_i ∩ e_j ∩ e_k|.
__device__ __forceinline__ uint32_t triple_code(uint32_t a, uint32_t b, uint32_t c, uint32_t p,
                                                uint32_t q, uint32_t s, uint32_t t) {
  uint32_t code = st3(t);                                   // R7
  code = __umul24(code, 3u) + st3(s - t);                   // R6
  code = __umul24(code, 3u) + st3(q - t);                   // R5
  code = __umul24(code, 3u) + st3(p - t);                   // R4
  code = __umul24(code, 3u) + st3(c + t - s - q);           // R3
  code = __umul24(code, 3u) + st3(b + t - p - q);           // R2
  code = __umul24(code, 3u) + st3(a + t - p - s);           // R1
  return code;
}

__device__ __forceinline__ bool in_sorted(const int32_t* s, int n, int32_t v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo < n && s[lo] == v;
}
