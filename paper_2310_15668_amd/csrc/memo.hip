// Key-grouped MoCHy-A+ on the fly with memoized neighbourhoods: the advanced
// on-the-fly variant of the appendix on counting without the line graph
// (Algorithm 9), shaped for the device.
//
// Each sampled hyperwedge {e_i, e_j} is filed under its key hyperedge, the
// one with the larger (line-graph degree, index); the other is e_o.  Keys are
// taken in descending (degree, index) order and a key's neighbourhood is
// memoized into a device arena of a fixed byte budget, the memo's priority
// being its degree as in the paper.  What is memoized is not the list of
// (e_k, ω) pairs but what the samples of the key need from it:
//   * B[c][s]: neighbours e_k of the key with |e_k| = c and |e_k ∩ e_key| = s;
//   * G_Q[c][s]: the same restricted to the e_k holding every node of Q, for
//     each set Q of heavy nodes that the samples of the key skip (below).
// A sample then walks the lists E_v of e_o's nodes only, skipping e_o's (at
// most three) heavy nodes with the longest lists, and assembles
// N_key ∪ N_o \ {e_key, e_o}:
//   * e_k reached through a walked node: classified exactly from its nodes;
//   * e_k meeting e_o only in skipped nodes P: counted per (c, s) from G_Q by
//     inclusion-exclusion over Q ⊇ P, and for s = 0 (not adjacent to the key)
//     from the heavy-node tables minus G_Q, less the walked ones;
//   * e_k adjacent to the key only: B less everything above.
// Counts of the last two kinds are first added under the class they would
// have if e_k met e_o nowhere and then moved by the walked and skipped
// corrections; these provisional classes cancel exactly in the integer
// histogram (additions are modulo 2^64, every final count is exact).
//
// A key is memoized only if its group is large enough to repay the walk of
// its whole neighbourhood, or the arena has room; other samples go through
// the plain on-the-fly enumeration.  Either way each sample's hits are the
// same as Algorithm 5's for that hyperwedge.
#include <algorithm>
#include <hipcub/hipcub.hpp>

#include "classify.h"
#include "common.h"
#include "rng.h"
#include "walk.h"

namespace {

constexpr int kMemoThreads = 256;
constexpr int kMemoCtr = 16384;  // LDS counters of one pass over a neighbourhood
constexpr int kMaxQ = 256;       // heavy-node sets memoized per key
constexpr int kQHash = 1024;     // LDS hash slots for collecting them
constexpr uint32_t kQNone = 127u;
constexpr int kCellsC = MOCHY_MAX_EDGE;  // c = 1..32 by s = 1..|e_key|

__device__ __forceinline__ bool first_is_key(int64_t di, int64_t i, int64_t dj, int64_t j) {
  return di > dj || (di == dj && i > j);
}

// Heavy-node set code: heavy indices ascending, 7 bits each, 127 = absent.
__device__ __forceinline__ uint32_t qcode(int n, int h0, int h1, int h2) {
  int x[3] = {n > 0 ? h0 : int(kQNone), n > 1 ? h1 : int(kQNone), n > 2 ? h2 : int(kQNone)};
  if (x[0] > x[1]) { const int t = x[0]; x[0] = x[1]; x[1] = t; }
  if (x[1] > x[2]) { const int t = x[1]; x[1] = x[2]; x[2] = t; }
  if (x[0] > x[1]) { const int t = x[0]; x[0] = x[1]; x[1] = t; }
  return uint32_t(x[0]) | (uint32_t(x[1]) << 7) | (uint32_t(x[2]) << 14);
}

__device__ __forceinline__ int find_code(const uint32_t* qs, int n, uint32_t code) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (qs[mid] < code) lo = mid + 1; else hi = mid;
  }
  return lo < n && qs[lo] == code ? lo : -1;
}

// The skipped nodes of e_o: its (at most three) heavy nodes with the longest
// lists E_v, ties to the later position; packed as their heavy indices in
// rank order, 7 bits each (127 = none).
__device__ uint32_t skip_set(const int32_t* __restrict__ nodes, int b,
                             const int8_t* __restrict__ heavy_bit,
                             const int64_t* __restrict__ node_ptr) {
  uint32_t packed = kQNone | (kQNone << 7) | (kQNone << 14);
  uint64_t taken = 0;
  for (int r = 0; r < kSkip; ++r) {
    uint64_t best = 0;
    int bp = -1, bh = -1;
    for (int x = 0; x < b; ++x) {
      if ((taken >> x) & 1ull) continue;
      const int32_t v = nodes[x];
      const int hb = heavy_bit[v];
      if (hb < 0) continue;
      const uint64_t key = (uint64_t(node_ptr[v + 1] - node_ptr[v]) << 6) | uint64_t(x);
      if (key > best) { best = key; bp = x; bh = hb; }
    }
    if (bp < 0) break;
    taken |= 1ull << bp;
    packed = (packed & ~(127u << (7 * r))) | (uint32_t(bh) << (7 * r));
  }
  return packed;
}

__global__ void k_keycount(int64_t cnt, const int2* __restrict__ pairs, const int64_t* __restrict__ deg,
                           unsigned long long* kcnt, int32_t* klist, unsigned int* nk) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  const int2 pr = pairs[s];
  const int32_t key = (pr.y < 0 || first_is_key(deg[pr.x], pr.x, deg[pr.y], pr.y)) ? pr.x : pr.y;
  if (atomicAdd(&kcnt[key], 1ull) == 0ull) klist[atomicAdd(nk, 1u)] = key;
}

__global__ void k_keyscatter(int64_t cnt, const int2* __restrict__ pairs, const int64_t* __restrict__ deg,
                             const int64_t* __restrict__ koff, unsigned int* kcur, int2* gp) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  const int2 pr = pairs[s];
  const bool ik = pr.y < 0 || first_is_key(deg[pr.x], pr.x, deg[pr.y], pr.y);
  const int32_t key = ik ? pr.x : pr.y, other = ik ? pr.y : pr.x;
  gp[koff[key] + atomicAdd(&kcur[key], 1u)] = make_int2(key, other);
}

__global__ void k_sortkey(const unsigned int* __restrict__ nk, const int32_t* __restrict__ klist,
                          const int64_t* __restrict__ deg, uint64_t* skey) {
  const unsigned x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= *nk) return;
  const int32_t k = klist[x];
  skey[x] = (uint64_t(deg[k]) << 32) | uint32_t(k);
}

// One block per key, in descending (degree, index) order: the skipped set of
// each of the key's samples, the heavy-node sets they need, then the counters
// B and G_Q over one walk of N_key per pass (e_k counted at the smallest node
// of e_key ∩ e_k), accumulated in LDS and copied to the key's arena space.
// Arena layout of a key: |e_key|, number of sets, the set codes ascending, then
// (1 + sets) x 32 x |e_key| counters, [slot][c - 1][s - 1], slot 0 = B.
__global__ __launch_bounds__(kMemoThreads) void k_memo(
    const int64_t* __restrict__ edge_ptr, const int32_t* __restrict__ edge_nodes,
    const int64_t* __restrict__ node_ptr, const int32_t* __restrict__ node_edges,
    const int8_t* __restrict__ heavy_bit, const uint64_t* __restrict__ hmask,
    const uint32_t* __restrict__ xoff, const int32_t* __restrict__ xnodes,
    const uint64_t* __restrict__ skey, const unsigned int* __restrict__ nk, unsigned int* queue,
    const int64_t* __restrict__ koff, const int2* __restrict__ gp, uint32_t* sS, uint32_t* arena,
    uint64_t arena_words, unsigned long long* arena_top, int64_t* memo_off, int memo_all) {
  __shared__ uint32_t ctr[kMemoCtr];
  __shared__ uint32_t qh[kQHash];  // code + 1, 0 = free
  __shared__ uint32_t qtmp[kMaxQ], qs[kMaxQ];
  __shared__ int32_t se[MOCHY_MAX_EDGE];
  __shared__ int64_t slo[MOCHY_MAX_EDGE], spre[MOCHY_MAX_EDGE + 1];
  __shared__ unsigned int s_kq, s_nq, s_ovf;
  __shared__ int s_go;
  __shared__ unsigned long long s_umask, s_off;
  const int tid = threadIdx.x, lane = tid & 63;
  const unsigned nkeys = *nk;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_kq = atomicAdd(queue, 1u);
    for (int t = tid; t < kQHash; t += kMemoThreads) qh[t] = 0u;
    __syncthreads();
    const unsigned kq = s_kq;
    if (kq >= nkeys) break;
    const int64_t key = int64_t(uint32_t(skey[kq]));
    const int64_t s0 = koff[key], s1 = koff[key + 1];
    const int64_t es = edge_ptr[key];
    const int a = int(edge_ptr[key + 1] - es);
    if (tid < 64) {
      int64_t len = 0;
      if (lane < a) {
        const int32_t v = edge_nodes[es + lane];
        se[lane] = v;
        slo[lane] = node_ptr[v];
        len = node_ptr[v + 1] - slo[lane];
      }
      const int64_t incl = wave_incl_scan_i64(len, lane);
      if (lane < a) spre[lane + 1] = incl;
      if (lane == 0) spre[0] = 0;
    }
    __syncthreads();
    if (tid == 0) {
      // memoize if the group's walks of the key's side (its heavy lists are
      // skipped per sample) outweigh twice one walk of the whole neighbourhood
      const int64_t build = spre[a];
      const uint32_t sk = skip_set(se, a, heavy_bit, node_ptr);
      int64_t skipped = 0;
      for (int x = 0; x < a; ++x) {
        const int hb = heavy_bit[se[x]];
        if (hb >= 0 && (uint32_t(hb) == (sk & 127u) || uint32_t(hb) == ((sk >> 7) & 127u) ||
                        uint32_t(hb) == ((sk >> 14) & 127u)))
          skipped += spre[x + 1] - spre[x];
      }
      const double gain = double(s1 - s0) * double(build - skipped);
      s_go = (memo_all || gain > 2.0 * double(build)) ? 1 : 0;
      s_nq = 0u;
      s_ovf = 0u;
      s_umask = 0ull;
    }
    __syncthreads();
    if (!s_go) {
      if (tid == 0) memo_off[key] = -1;
      continue;
    }
    for (int64_t x = s0 + tid; x < s1; x += kMemoThreads) {
      const int64_t o = gp[x].y;
      uint32_t packed = kQNone | (kQNone << 7) | (kQNone << 14);
      if (o >= 0) {
        const int64_t os = edge_ptr[o];
        packed = skip_set(edge_nodes + os, int(edge_ptr[o + 1] - os), heavy_bit, node_ptr);
      }
      sS[x] = packed;
      int h[kSkip], n = 0;
      for (int r = 0; r < kSkip; ++r) {
        const uint32_t hb = (packed >> (7 * r)) & 127u;
        if (hb != kQNone) h[n++] = int(hb);
      }
      unsigned long long um = 0ull;
      for (int m = 1; m < (1 << n); ++m) {
        int y[3], ny = 0;
        for (int r = 0; r < n; ++r)
          if (m & (1 << r)) { y[ny++] = h[r]; um |= 1ull << h[r]; }
        const uint32_t code = qcode(ny, y[0], ny > 1 ? y[1] : 0, ny > 2 ? y[2] : 0);
        uint32_t slot = (code * 2654435761u) >> 22;  // 10 bits
        for (int probe = 0;; ++probe) {
          if (probe == kQHash) { s_ovf = 1u; break; }
          const uint32_t old = atomicCAS(&qh[slot], 0u, code + 1u);
          if (old == 0u) {
            const unsigned at = atomicAdd(&s_nq, 1u);
            if (at < unsigned(kMaxQ)) qtmp[at] = code; else s_ovf = 1u;
            break;
          }
          if (old == code + 1u) break;
          slot = (slot + 1u) & (kQHash - 1);
        }
      }
      if (um) atomicOr(&s_umask, um);
    }
    __syncthreads();
    const int nq = int(s_nq);
    const uint32_t cells = uint32_t(kCellsC) * uint32_t(a);
    const uint64_t words = 2ull + uint64_t(nq) + (1ull + uint64_t(nq)) * cells;
    if (tid == 0) {
      unsigned long long off = ~0ull;
      if (!s_ovf) {
        unsigned long long top = *arena_top;
        while (top + words <= arena_words) {
          const unsigned long long prev = atomicCAS(arena_top, top, top + words);
          if (prev == top) { off = top; break; }
          top = prev;
        }
      }
      s_off = off;
      memo_off[key] = off == ~0ull ? -1 : int64_t(off);
    }
    if (!s_ovf)  // then nq <= kMaxQ: rank sort of the set codes
      for (int t = tid; t < nq; t += kMemoThreads) {
        const uint32_t c = qtmp[t];
        int r = 0;
        for (int y = 0; y < nq; ++y) r += qtmp[y] < c ? 1 : 0;
        qs[r] = c;
      }
    __syncthreads();
    if (s_off == ~0ull) continue;
    uint32_t* mem = arena + s_off;
    if (tid == 0) {
      mem[0] = uint32_t(a);
      mem[1] = uint32_t(nq);
    }
    for (int t = tid; t < nq; t += kMemoThreads) mem[2 + t] = qs[t];
    uint32_t* gctr = mem + 2 + nq;
    const unsigned long long umask = s_umask;
    const int per_pass = int(kMemoCtr / cells);  // >= 16
    const int64_t L = spre[a];
    for (int sl0 = 0; sl0 < 1 + nq; sl0 += per_pass) {
      const int sl1 = min(1 + nq, sl0 + per_pass);
      const uint32_t n_ctr = uint32_t(sl1 - sl0) * cells;
      for (uint32_t t = tid; t < n_ctr; t += kMemoThreads) ctr[t] = 0u;
      __syncthreads();
      int x = 0;
      for (int64_t q = tid; q < L; q += kMemoThreads) {
        while (spre[x + 1] <= q) ++x;
        const int32_t v = se[x];
        const int64_t p = slo[x] + (q - spre[x]);
        const int32_t k = node_edges[p];
        if (k == int32_t(key)) continue;
        const uint32_t xs = xoff[p], xe = xoff[p + 1];
        int c = 0, s = 0;
        bool owned = true;
        for (uint32_t t = xs; t < xe; t += kXPad) {
          const int4 z4 = *reinterpret_cast<const int4*>(xnodes + t);
          const int32_t zz[4] = {z4.x, z4.y, z4.z, z4.w};
          for (int y = 0; y < 4; ++y) {
            const int32_t z = zz[y];
            if (z < 0) continue;
            ++c;
            if (in_sorted(se, a, z)) {
              ++s;
              if (z < v) owned = false;
            }
          }
        }
        if (!owned) continue;
        const uint32_t cell = uint32_t(c - 1) * uint32_t(a) + uint32_t(s - 1);
        if (sl0 == 0) atomicAdd(&ctr[cell], 1u);
        // every set of at most three heavy nodes of e_k that some sample needs
        auto count_set = [&](int n, int h0, int h1, int h2) {
          const int idx = find_code(qs, nq, qcode(n, h0, h1, h2));
          const int slot = 1 + idx;
          if (idx >= 0 && slot >= sl0 && slot < sl1)
            atomicAdd(&ctr[uint32_t(slot - sl0) * cells + cell], 1u);
        };
        const uint64_t hm = hmask[k] & umask;
        for (uint64_t m0 = hm; m0; m0 &= m0 - 1) {
          const int h0 = __ffsll((long long)m0) - 1;
          count_set(1, h0, 0, 0);
          for (uint64_t m1 = m0 & (m0 - 1); m1; m1 &= m1 - 1) {
            const int h1 = __ffsll((long long)m1) - 1;
            count_set(2, h0, h1, 0);
            for (uint64_t m2 = m1 & (m1 - 1); m2; m2 &= m2 - 1)
              count_set(3, h0, h1, __ffsll((long long)m2) - 1);
          }
        }
      }
      __syncthreads();
      for (uint32_t t = tid; t < n_ctr; t += kMemoThreads) gctr[uint64_t(sl0) * cells + t] = ctr[t];
      __syncthreads();
    }
  }
}

// samples whose key was not memoized, for the plain on-the-fly enumeration
__global__ void k_leftover(int64_t cnt, const int2* __restrict__ gp, const int64_t* __restrict__ memo_off,
                           int2* out, unsigned long long* nout) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  const int2 pr = gp[s];
  if (memo_off[pr.x] < 0) out[atomicAdd(nout, 1ull)] = pr;
}

__device__ __forceinline__ void hadd(unsigned long long* hist, const uint16_t* lut, uint32_t code,
                                     int64_t n) {
  atomicAdd(&hist[lut[code]], (unsigned long long)n);
}

// The walk of e_o's non-skipped lists for one sample (i = key, j = o in the
// per-visit sums).  An e_k is taken at its smallest walked node; it adds its
// exact class, and moves what the memo counts would otherwise give it: the
// key-only class if it is adjacent to the key, or the class of an e_k meeting
// e_o only in its skipped nodes P if it holds some.
template <bool kOvf>
__device__ __forceinline__ void walk_other(EnumLds& L, int lane, int64_t T, uint32_t a, uint32_t b,
                                           uint32_t p, uint32_t kin, uint32_t novf,
                                           const uint32_t* __restrict__ xoff,
                                           const int32_t* __restrict__ xnodes, const uint16_t* lut,
                                           unsigned long long* hist) {
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
      while (lend <= q) {
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
      atomicAdd(&L.acc[owner], chunk_sums<kOvf, true>(L, z4, L.vv[owner], novf));
    }
    wave_sync();
    if (q < T) {
      const unsigned long long s = L.acc[lane];
      const uint32_t c = uint32_t(s >> kSc) & 63u, wi = uint32_t(s >> kSi) & 63u;
      const uint32_t wj = uint32_t(s >> kSj) & 63u, t3 = uint32_t(s >> kSt) & 63u;
      const uint32_t below = uint32_t(s >> kSb) & 63u;
      uint32_t pat = 0;
      for (int y = 0; y < kSkip; ++y) pat |= ((s >> (kSp + 2 * y)) & 3ull) ? 1u << y : 0u;
      const bool self = (c == a && wi == c) || (c == b && wj == c);
      if (below == 0 && !self) {
        const uint32_t id = lut[triple_code(a, b, c, p, wj, wi, t3)];
        if (id != run_id) {
          if (run_n) atomicAdd(&hist[run_id], (unsigned long long)run_n);
          run_id = id;
          run_n = 0;
        }
        ++run_n;
        if (pat)
          hadd(hist, lut, triple_code(a, b, c, p, __popc(pat), wi, __popc(pat & kin)), -1);
        else if (wi)
          hadd(hist, lut, triple_code(a, b, c, p, 0u, wi, 0u), -1);
      }
    }
    wave_sync();
  }
  if (run_n) atomicAdd(&hist[run_id], (unsigned long long)run_n);
}

// One wave per sample of a memoized key (samples of other keys are skipped).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_msample(
    int64_t cnt, int64_t E, const int2* __restrict__ gp, const uint32_t* __restrict__ sS,
    const int64_t* __restrict__ memo_off, const uint32_t* __restrict__ arena,
    const int64_t* __restrict__ edge_ptr, const int32_t* __restrict__ edge_nodes,
    const int64_t* __restrict__ node_ptr, const int8_t* __restrict__ heavy_bit,
    const uint32_t* __restrict__ xoff, const int32_t* __restrict__ xnodes,
    const uint32_t* __restrict__ hsize, const uint32_t* __restrict__ hpair,
    const uint32_t* __restrict__ htriple, const uint16_t* __restrict__ code_to_id3,
    unsigned long long* queue, unsigned long long* hist_out, int32_t* flags) {
  __shared__ uint16_t lut[kNumCodes];
  __shared__ unsigned long long hist[kHistSlots];
  __shared__ EnumLds lds[kEnumWaves];
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x) hist[t] = 0ull;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  EnumLds& L = lds[wave];
  for (int t = lane; t < kBuckets; t += kWave) L.tab[t] = make_uint4(0u, 0u, 0u, 0u);
  if (lane == 0) L.novf = 0u;
  __syncthreads();
  bool bad = false;
  for (;;) {
    unsigned long long sq = 0;
    if (lane == 0) sq = atomicAdd(queue, (unsigned long long)kBatch);
    const int64_t sb = int64_t(uniform64(sq));
    if (sb >= cnt) break;
    const int64_t se_ = sb + kBatch < cnt ? sb + kBatch : cnt;
    for (int64_t smp = sb; smp < se_; ++smp) {
      const int2 pr = gp[smp];
      const int64_t key = pr.x, o = pr.y;
      if (key < 0 || key >= E || o < 0 || o >= E || key == o) { bad = true; continue; }
      const int64_t mo = memo_off[key];
      if (mo < 0) continue;
      const int64_t sk = edge_ptr[key], so = edge_ptr[o];
      const int a = int(edge_ptr[key + 1] - sk), b = int(edge_ptr[o + 1] - so);
      if (lane < a) L.ei[lane] = edge_nodes[sk + lane];
      if (lane < b) L.ej[lane] = edge_nodes[so + lane];
      wave_sync();
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
      const uint32_t p = uint32_t(__popcll(__ballot(lane < a && (f & kFJ))));
      const uint32_t packed = sS[smp];
      int hb[kSkip];
      int nskip = 0;
      for (int r = 0; r < kSkip; ++r) {
        hb[r] = int((packed >> (7 * r)) & 127u);
        if (uint32_t(hb[r]) != kQNone) ++nskip;
      }
      uint32_t rank = 0;
      if (mem && (f & kFJ)) {
        const int hbit = heavy_bit[u];
        for (int r = 0; r < nskip; ++r)
          if (hbit >= 0 && hbit == hb[r]) rank = uint32_t(r + 1);
      }
      f |= rank << 2;
      uint32_t kin = 0;
      for (int r = 0; r < nskip; ++r) {
        const uint64_t held = __ballot(rank == uint32_t(r + 1));
        if (__popcll(held) != 1) bad = true;
        if (__ballot(rank == uint32_t(r + 1) && (f & kFI))) kin |= 1u << r;
      }
      int slot = -1;
      if (mem) {
        const uint32_t pk = (uint32_t(u + 1) << 4) | f;
        uint32_t* bk = reinterpret_cast<uint32_t*>(&L.tab[bucket_of(u)]);
        for (int t = 0; t < 4 && slot < 0; ++t)
          if (atomicCAS(&bk[t], 0u, pk) == 0u) slot = t;
        if (slot < 0) L.ovf[atomicAdd(&L.novf, 1u)] = pk;
      }
      int64_t du = 0, nb = 0;
      const bool walk = mem && (f & kFJ) && rank == 0;
      if (walk) {
        nb = node_ptr[u];
        du = node_ptr[u + 1] - nb;
      }
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
        walk_other<false>(L, lane, T, a, b, p, kin, 0u, xoff, xnodes, lut, hist);
      else
        walk_other<true>(L, lane, T, a, b, p, kin, novf, xoff, xnodes, lut, hist);
      // memoized counts of the key
      const uint32_t* mk = arena + mo;
      const int nq = int(mk[1]);
      if (int(mk[0]) != a) bad = true;
      const uint32_t* qs = mk + 2;
      const uint32_t* g0 = mk + 2 + nq;
      const uint32_t cells = uint32_t(kCellsC) * uint32_t(a);
      for (uint32_t x = lane; x < cells; x += kWave) {
        const uint32_t m = g0[x];
        if (m) {
          const uint32_t c = x / uint32_t(a) + 1u, s = x % uint32_t(a) + 1u;
          hadd(hist, lut, triple_code(a, b, c, p, 0u, s, 0u), int64_t(m));
        }
      }
      if (lane == 0) hadd(hist, lut, triple_code(a, b, b, p, 0u, p, 0u), -1);  // e_o itself
      for (uint32_t qm = 1; qm < (1u << nskip); ++qm) {
        int y[3], ny = 0;
        for (int r = 0; r < nskip; ++r)
          if (qm & (1u << r)) y[ny++] = hb[r];
        const int idx = find_code(qs, nq, qcode(ny, y[0], ny > 1 ? y[1] : 0, ny > 2 ? y[2] : 0));
        if (idx < 0) { bad = true; continue; }
        const uint32_t* gq = g0 + uint64_t(1 + idx) * cells;
        const int nqm = __popc(qm);
        for (uint32_t x = lane; x < cells; x += kWave) {
          const uint32_t c = x / uint32_t(a) + 1u, s = x % uint32_t(a) + 1u;
          const int64_t m = int64_t(gq[x]) - ((c == uint32_t(b) && s == p) ? 1 : 0);
          if (!m) continue;
          for (uint32_t pm = qm; pm; pm = (pm - 1u) & qm) {
            const int np = __popc(pm);
            hadd(hist, lut, triple_code(a, b, c, p, uint32_t(np), s, uint32_t(__popc(pm & kin))),
                 ((nqm - np) & 1) ? -m : m);
          }
          hadd(hist, lut, triple_code(a, b, c, p, 0u, s, 0u), (nqm & 1) ? -m : m);
        }
        if ((qm & kin) == 0u && lane < kCellsC) {
          // e_k holding Q and not adjacent to the key: the heavy tables less G_Q
          const int c = lane + 1;
          int64_t in_key = 0;
          for (int s = 0; s < a; ++s) in_key += gq[uint32_t(c - 1) * uint32_t(a) + uint32_t(s)];
          const int64_t m0 = superset_count(qm, hb, c, hsize, hpair, htriple) - in_key;
          if (m0 < 0) bad = true;
          if (m0 > 0)
            for (uint32_t pm = qm; pm; pm = (pm - 1u) & qm) {
              const int np = __popc(pm);
              hadd(hist, lut, triple_code(a, b, uint32_t(c), p, uint32_t(np), 0u, 0u),
                   ((nqm - np) & 1) ? -m0 : m0);
            }
        }
      }
      wave_sync();
      if (mem && slot >= 0) reinterpret_cast<uint32_t*>(&L.tab[bucket_of(u)])[slot] = 0u;
      if (lane == 0) L.novf = 0u;
      wave_sync();
    }
  }
  if (bad) atomicOr(flags, 4);
  __syncthreads();
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x)
    if (hist[t]) atomicAdd(&hist_out[t], hist[t]);
}

}  // namespace

struct memo_bufs {
  int64_t chunk = 0;
  unsigned long long* kcnt = nullptr;  // [E + 1] samples per key
  int64_t* koff = nullptr;             // [E + 1]
  unsigned int* kcur = nullptr;        // [E]
  int32_t* klist = nullptr;            // [E] keys drawn in the chunk
  uint64_t *skey = nullptr, *skey2 = nullptr;  // [E] (degree, key) before and after the sort
  int64_t* memo_off = nullptr;         // [E] arena offset of each drawn key, -1 if not memoized
  int64_t* tmp = nullptr;              // scan scratch
  int2* gp = nullptr;                  // [chunk] samples grouped by key, (key, other)
  int2* left = nullptr;                // [chunk] samples of keys not memoized
  uint32_t* sS = nullptr;              // [chunk] skipped heavy nodes of each sample's e_o
  uint32_t* arena = nullptr;
  uint64_t arena_words = 0;
  void* cub = nullptr;
  size_t cub_bytes = 0;
  unsigned long long* ctr = nullptr;   // [0] nk | queue, [1] arena top, [2] leftovers, [3] sample queue
  int64_t* deg_tmp = nullptr;          // [E] line-graph degrees when the graph keeps none
};

void memo_end(mochy_ctx* ctx, memo_bufs* m) {
  if (!m) return;
  void* bufs[] = {m->kcnt, m->koff, m->kcur, m->klist, m->skey, m->skey2, m->memo_off, m->tmp,
                  m->gp,   m->left, m->sS,   m->arena, m->cub,  m->ctr,   m->deg_tmp};
  for (void* p : bufs) device_free(ctx, p);
  delete m;
}

mochy_status memo_begin(mochy_ctx* ctx, const mochy_graph* g, int64_t chunk, memo_bufs** out) {
  *out = nullptr;
  const int64_t E = g->E;
  memo_bufs* m = new memo_bufs();
  m->chunk = chunk;
  // at most about 1 MiB per drawn key (a key of 32 nodes with 256 sets)
  m->arena_words = std::min<uint64_t>(uint64_t(ctx->memo_budget), uint64_t(E) << 20) / 4;
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&m->kcnt, size_t(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->koff, size_t(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->kcur, size_t(E) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->klist, size_t(E) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->skey, size_t(E) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->skey2, size_t(E) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->memo_off, size_t(E) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->tmp, scan_tmp_elems(E + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->gp, size_t(chunk) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->left, size_t(chunk) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->sS, size_t(chunk) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->arena, size_t(std::max<uint64_t>(m->arena_words, 1)) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->ctr, 4 * 8)) != MOCHY_OK) {
    memo_end(ctx, m);
    return rc;
  }
  if (hipcub::DeviceRadixSort::SortKeysDescending(nullptr, m->cub_bytes, m->skey, m->skey2, int(E), 0, 64,
                                                  ctx->stream) != hipSuccess ||
      (rc = device_alloc(ctx, &m->cub, std::max<size_t>(m->cub_bytes, 1))) != MOCHY_OK) {
    memo_end(ctx, m);
    if (rc == MOCHY_OK) {
      ctx->err = "radix sort workspace query failed";
      rc = MOCHY_EDEVICE;
    }
    return rc;
  }
  *out = m;
  return MOCHY_OK;
}

// One chunk of sampled pairs (pairs[0..cnt), each (i, j)): grouped by key,
// memoized keys counted by k_msample, the rest returned in m->left with their
// number, for the plain enumeration.
mochy_status memo_chunk(mochy_ctx* ctx, const mochy_graph* g, memo_bufs* m, int64_t cnt,
                        const int2* pairs, const int64_t* deg, int64_t* d_hist, int32_t* flags,
                        const int2** left, int64_t* n_left) {
  hipStream_t st = ctx->stream;
  const int64_t E = g->E;
  unsigned int* nk = reinterpret_cast<unsigned int*>(m->ctr);
  unsigned int* kqueue = nk + 1;
  unsigned long long* top = m->ctr + 1;
  unsigned long long* nleft = m->ctr + 2;
  unsigned long long* squeue = m->ctr + 3;
  MOCHY_HIP(hipMemsetAsync(m->kcnt, 0, size_t(E + 1) * 8, st));
  MOCHY_HIP(hipMemsetAsync(m->kcur, 0, size_t(E) * 4, st));
  MOCHY_HIP(hipMemsetAsync(m->ctr, 0, 4 * 8, st));
  k_keycount<<<blocks(cnt, 256), 256, 0, st>>>(cnt, pairs, deg, m->kcnt, m->klist, nk);
  launch_exclusive_scan_i64(reinterpret_cast<int64_t*>(m->kcnt), m->koff, E + 1, m->tmp, st);
  k_keyscatter<<<blocks(cnt, 256), 256, 0, st>>>(cnt, pairs, deg, m->koff, m->kcur, m->gp);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, m->ctr, 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  const unsigned nkeys = *reinterpret_cast<const unsigned*>(ctx->h_small);
  if (nkeys > 0) {
    k_sortkey<<<blocks(nkeys, 256), 256, 0, st>>>(nk, m->klist, deg, m->skey);
    size_t cb = m->cub_bytes;
    MOCHY_HIP(hipcub::DeviceRadixSort::SortKeysDescending(m->cub, cb, m->skey, m->skey2, int(nkeys), 0, 64,
                                                          st));
  }
  k_memo<<<unsigned(ctx->num_cus) * 2u, kMemoThreads, 0, st>>>(
      g->edge_ptr, g->edge_nodes, g->node_ptr, g->node_edges, g->heavy_bit, g->hmask, g->xoff,
      g->xnodes, m->skey2, nk, kqueue, m->koff, m->gp, m->sS, m->arena, m->arena_words, top,
      m->memo_off, ctx->memo_all ? 1 : 0);
  k_leftover<<<blocks(cnt, 256), 256, 0, st>>>(cnt, m->gp, m->memo_off, m->left, nleft);
  k_msample<<<unsigned(ctx->num_cus) * 8u, kEnumWaves * kWave, 0, st>>>(
      cnt, E, m->gp, m->sS, m->memo_off, m->arena, g->edge_ptr, g->edge_nodes, g->node_ptr,
      g->heavy_bit, g->xoff, g->xnodes, g->hsize, g->hpair, g->htriple, ctx->d_code_to_id3, squeue,
      (unsigned long long*)d_hist, flags);
  MOCHY_HIP(hipGetLastError());
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, nleft, 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  *n_left = ctx->h_small[0];
  *left = m->left;
  return MOCHY_OK;
}
