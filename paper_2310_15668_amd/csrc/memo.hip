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
// A key is memoized if it has at least kMinGroup samples in the chunk and the
// arena has room; other samples go through the plain on-the-fly enumeration.  Either way each sample's hits are the
// same as Algorithm 5's for that hyperwedge.
#include <algorithm>
#include <hipcub/hipcub.hpp>

#include "classify.h"
#include "common.h"
#include "rng.h"
#include "walk.h"

namespace {

constexpr int kMemoThreads = 512;
constexpr int kMemoCtr = 8192;   // LDS counters of one pass over a neighbourhood
constexpr int kMaxQ = 1024;      // heavy-node sets memoized per key
constexpr int kQHash = 2048;     // LDS hash slots for collecting them
constexpr uint32_t kQNone = 127u;
// A memo slot (a heavy-node set Q, or none) counts the neighbours e_k of the
// key holding Q by (s = |e_k ∩ e_key|, d = min(|e_k| - s, 5)): every region
// of the triple but the key's outside region depends on c only through s, and
// that region's state only through c - s shifted by at most 3, so d = 5
// stands for every larger difference.  Then come the hyperedges holding Q and
// not adjacent to the key by size min(c, 5) (a region of c minus at most 3
// nodes).  Words per slot: 6 |e_key| + 5.
constexpr int kDiff = 6;
constexpr int kFarBins = 5;
__device__ __forceinline__ uint32_t slot_words(int a) { return uint32_t(kDiff * a + kFarBins); }

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

// The skipped nodes of a hyperedge: its (at most three) heavy nodes among
// `allowed` (heavy indices) with the longest lists E_v, ties to the later
// position; packed as their heavy indices in rank order, 7 bits each (127 =
// none).
__device__ uint32_t skip_set(const int32_t* __restrict__ nodes, int b,
                             const int8_t* __restrict__ heavy_bit,
                             const int64_t* __restrict__ node_ptr, uint64_t allowed = ~0ull) {
  uint32_t packed = kQNone | (kQNone << 7) | (kQNone << 14);
  uint64_t taken = 0;
  for (int r = 0; r < kSkip; ++r) {
    uint64_t best = 0;
    int bp = -1, bh = -1;
    for (int x = 0; x < b; ++x) {
      if ((taken >> x) & 1ull) continue;
      const int32_t v = nodes[x];
      const int hb = heavy_bit[v];
      if (hb < 0 || !((allowed >> hb) & 1ull)) continue;
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
// each of the key's samples and the heavy-node sets Q they need, then the
// counters B (= G of the empty set) and G_Q per pass over the slots.  The key
// skips its own (at most three) heavy nodes with the longest lists: one walk
// of the other lists of e_key counts every neighbour e_k holding a walked node
// (taken at its smallest walked node of e_key), with its size c, overlap s and
// heavy nodes, and tallies those that also hold skipped nodes of the key; the
// neighbours meeting e_key only in a set P of skipped nodes (so s = |P|) come
// from the heavy-set tables by inclusion-exclusion over the skipped sets
// above P, less the tally and e_key itself.
// Arena layout of a key: |e_key|, number of sets, the set codes ascending, then
// (1 + sets) slots of slot_words(|e_key|) counters, slot 0 = no set (B).
constexpr int kMinGroup = 4;                  // samples a key needs to be memoized
// heavy nodes a key's samples may skip on their other side when its sets Q
// would overflow: the kSkipPool with the most list entries over the key's
// samples (bounds the sets to 16 + 120 + 560 < kMaxQ); the other heavy nodes
// of e_o are then walked
constexpr int kSkipPool = 16;
constexpr int kSigHash = 2048;                // distinct sample signatures of a key (LDS hash)
static_assert(4 * kSigHash <= kMemoCtr, "signatures live in the counters' LDS");

// e_key's nodes for a memo build, hashed as in the per-sample table (flags:
// bit 0 = in e_key, bits 2-3 = rank of a skipped node of e_key)
struct KeyTab {
  uint4 tab[kBuckets];
  uint32_t ovf[MOCHY_MAX_EDGE];
};
// one window of 64 visits of a wave, cut into 4-node chunks
struct MemoWin {
  uint32_t vx[kWave], vc[kWave];
  int32_t vv[kWave];
  unsigned long long acc[kWave];
  uint8_t cmap[kMaxChunks];
};
// Sizes in the tallies and the table part: c = 1..8 exactly, then all larger
// sizes in one bin (table slot 0), which no class below tells apart.
constexpr int kCBins = kSizeTail + 1;
__device__ __forceinline__ uint32_t cbin(int c) { return uint32_t(c > kSizeTail ? kSizeTail : c - 1); }
__device__ __forceinline__ int tcol(int bin) { return bin < kSizeTail ? bin + 1 : 0; }
constexpr int kTally = kPatterns * kCBins;    // walked e_k by skipped key nodes held, by size bin

// One memo build's walk of the key's non-skipped lists, the block's waves
// taking windows of 64 visits in turn; each window's node lists are cut into
// 4-node chunks over the lanes (as in the per-sample walk) and summed per
// visit: |e_k|, |e_k ∩ e_key|, walked key nodes below the visit's node, and
// the skipped key nodes held.  A visit owns e_k if no walked key node lies
// below it; it counts e_k in slot 0 (first pass) and in each memoized set Q
// of heavy nodes e_k holds, in slots [sl0, sl1) of this pass.
template <bool kOvf>
__device__ __forceinline__ void memo_walk(
    const KeyTab& kt, MemoWin& Wn, int lane, int wave, int64_t L, const int32_t* wn,
    const int64_t* wlo, const int64_t* wpre, int32_t key, uint32_t novf,
    const int32_t* __restrict__ node_edges, const uint32_t* __restrict__ xoff,
    const int32_t* __restrict__ xnodes, const uint64_t* __restrict__ hmask, uint64_t umask,
    const uint32_t* qs, int nq, int sl0, int sl1, int a, uint32_t cells, uint32_t stride,
    uint32_t tot0, uint32_t* ctr) {
  int x = 0;
  for (int64_t q0 = int64_t(wave) * kWave; q0 < L; q0 += kMemoThreads) {
    const int64_t q = q0 + lane;
    uint32_t nch = 0, xs = 0;
    int32_t k = key, v = 0;
    if (q < L) {
      while (wpre[x + 1] <= q) ++x;
      const int64_t p = wlo[x] + (q - wpre[x]);
      v = wn[x];
      k = node_edges[p];
      xs = xoff[p];
      nch = (xoff[p + 1] - xs) / kXPad;
    }
    uint32_t incl = nch;
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t o = uint32_t(__shfl_up(int(incl), off));
      if (lane >= off) incl += o;
    }
    const uint32_t first_chunk = incl - nch;
    const uint32_t nchunks = uint32_t(__shfl(int(incl), kWave - 1));
    Wn.vx[lane] = xs;
    Wn.vc[lane] = first_chunk;
    Wn.vv[lane] = v;
    Wn.acc[lane] = 0ull;
    for (uint32_t t = 0; t < nch; ++t) Wn.cmap[first_chunk + t] = uint8_t(lane);
    wave_sync();
    for (uint32_t ch = lane; ch < nchunks; ch += kWave) {
      const int owner = Wn.cmap[ch];
      const int4 z4 = *reinterpret_cast<const int4*>(xnodes + Wn.vx[owner] + (ch - Wn.vc[owner]) * kXPad);
      atomicAdd(&Wn.acc[owner], chunk_sums<kOvf>(kt, z4, Wn.vv[owner], novf));
    }
    wave_sync();
    if (q < L && k != key) {
      const unsigned long long sm = Wn.acc[lane];
      const int c = int(sm >> kSc) & 63, s = int(sm >> kSi) & 63;
      const uint32_t below = uint32_t(sm >> kSb) & 63u;
      uint32_t pk = 0;  // skipped key nodes held
      for (int y = 0; y < kSkip; ++y) pk |= ((sm >> (kSp + 2 * y)) & 3ull) ? 1u << y : 0u;
      if (below == 0u) {
        const uint32_t cell = uint32_t(s - 1) * kDiff + uint32_t(min(c - s, kDiff - 1));
        const uint32_t tcell = cells + (pk ? (pk - 1u) * kCBins + cbin(c) : 0u);
        const uint32_t ccell = tot0 + cbin(c);
        if (sl0 == 0) {
          atomicAdd(&ctr[cell], 1u);
          atomicAdd(&ctr[ccell], 1u);
          if (pk) atomicAdd(&ctr[tcell], 1u);
        }
        auto count_set = [&](int n, int h0, int h1, int h2) {
          const int idx = find_code(qs, nq, qcode(n, h0, h1, h2));
          const int slot = 1 + idx;
          if (idx >= 0 && slot >= sl0 && slot < sl1) {
            const uint32_t base = uint32_t(slot - sl0) * stride;
            atomicAdd(&ctr[base + cell], 1u);
            atomicAdd(&ctr[base + ccell], 1u);
            if (pk) atomicAdd(&ctr[base + tcell], 1u);
          }
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
    }
    wave_sync();
  }
}

__global__ __launch_bounds__(kMemoThreads) void k_memo(
    const int64_t* __restrict__ edge_ptr, const int32_t* __restrict__ edge_nodes,
    const int64_t* __restrict__ node_ptr, const int32_t* __restrict__ node_edges,
    const int8_t* __restrict__ heavy_bit, const uint64_t* __restrict__ hmask,
    const uint32_t* __restrict__ xoff, const int32_t* __restrict__ xnodes,
    const uint32_t* __restrict__ hsize, const uint32_t* __restrict__ hpair,
    const uint32_t* __restrict__ htriple, const unsigned long long* __restrict__ big_key,
    const uint32_t* __restrict__ big_val, int big_log2,
    const uint64_t* __restrict__ skey, const unsigned int* __restrict__ nk, unsigned int* queue,
    const int64_t* __restrict__ koff, const int2* __restrict__ gp, uint32_t* sS, uint32_t* smul,
    uint32_t* arena, uint64_t arena_words, unsigned long long* arena_top, int64_t* memo_off,
    int memo_all, int memo_pool, unsigned long long* n_memo, int32_t* flags) {
  __shared__ __align__(16) uint32_t ctr[kMemoCtr];
  __shared__ uint32_t qh[kQHash];  // code + 1, 0 = free
  __shared__ uint32_t qtmp[kMaxQ], qs[kMaxQ];
  __shared__ int32_t se[MOCHY_MAX_EDGE];
  __shared__ int32_t s_wn[MOCHY_MAX_EDGE];                    // walked nodes of e_key
  __shared__ int64_t s_wlo[MOCHY_MAX_EDGE], s_wpre[MOCHY_MAX_EDGE + 1];
  __shared__ int32_t s_skn[kSkip];                            // skipped nodes of e_key
  __shared__ int s_skh[kSkip];                                // and their heavy indices
  __shared__ KeyTab ktab;
  __shared__ MemoWin win[kMemoThreads / kWave];
  __shared__ unsigned int s_kq, s_nq, s_ovf, s_novf;
  __shared__ int s_go, s_nw, s_nsk;
  __shared__ unsigned long long s_umask, s_off, s_allowed;
  __shared__ unsigned long long hscore[kHeavyBits];
  const int tid = threadIdx.x;
  const unsigned nkeys = *nk;
  bool bad = false;
  // distinct sample signatures of the key (before the counting passes, in the
  // counters' LDS): key + 1, samples with it, the representative sample
  unsigned long long* sig_key = reinterpret_cast<unsigned long long*>(ctr);
  uint32_t* sig_cnt = ctr + 2 * kSigHash;
  uint32_t* sig_rep = ctr + 3 * kSigHash;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_kq = atomicAdd(queue, 1u);
    for (int t = tid; t < kQHash; t += kMemoThreads) qh[t] = 0u;
    for (int t = tid; t < kBuckets; t += kMemoThreads) ktab.tab[t] = make_uint4(0u, 0u, 0u, 0u);
    for (int t = tid; t < kHeavyBits; t += kMemoThreads) hscore[t] = 0ull;
    if (tid == 0) s_novf = 0u;
    for (int t = tid; t < kSigHash; t += kMemoThreads) {
      sig_key[t] = 0ull;
      sig_cnt[t] = 0u;
      sig_rep[t] = ~0u;
    }
    __syncthreads();
    const unsigned kq = s_kq;
    if (kq >= nkeys) break;
    const int64_t key = int64_t(uint32_t(skey[kq]));
    const int64_t s0 = koff[key], s1 = koff[key + 1];
    const int64_t es = edge_ptr[key];
    const int a = int(edge_ptr[key + 1] - es);
    if (tid < a) se[tid] = edge_nodes[es + tid];
    __syncthreads();
    if (tid == 0) {
      const uint32_t sk = skip_set(se, a, heavy_bit, node_ptr);
      int nsk = 0;
      for (int r = 0; r < kSkip; ++r) {
        const uint32_t hb = (sk >> (7 * r)) & 127u;
        if (hb == kQNone) break;
        s_skh[r] = int(hb);
        ++nsk;
      }
      int nw = 0;
      int64_t acc = 0;
      s_wpre[0] = 0;
      for (int x = 0; x < a; ++x) {
        const int32_t v = se[x];
        const int hb = heavy_bit[v];
        int r = -1;
        for (int y = 0; y < nsk; ++y)
          if (hb >= 0 && hb == s_skh[y]) r = y;
        if (r >= 0) {
          s_skn[r] = v;
          continue;
        }
        s_wn[nw] = v;
        s_wlo[nw] = node_ptr[v];
        acc += node_ptr[v + 1] - node_ptr[v];
        s_wpre[++nw] = acc;
      }
      s_nw = nw;
      s_nsk = nsk;
      s_go = (memo_all || s1 - s0 >= kMinGroup) ? 1 : 0;
      s_nq = 0u;
      s_ovf = 0u;
      s_umask = 0ull;
    }
    __syncthreads();
    if (!s_go) {
      if (tid == 0) memo_off[key] = -1;
      continue;
    }
    if (tid < a) {
      const int32_t v = se[tid];
      uint32_t f = 1u;
      for (int r = 0; r < s_nsk; ++r)
        if (v == s_skn[r]) f |= uint32_t(r + 1) << 2;
      const uint32_t pk = (uint32_t(v + 1) << 4) | f;
      uint32_t* bk = reinterpret_cast<uint32_t*>(&ktab.tab[bucket_of(v)]);
      bool put = false;
      for (int t = 0; t < 4 && !put; ++t) put = atomicCAS(&bk[t], 0u, pk) == 0u;
      if (!put) ktab.ovf[atomicAdd(&s_novf, 1u)] = pk;
    }
    // First every heavy node of a sample's other side may be skipped; if the
    // key's sets Q overflow, its samples are redone with the skip pool: the
    // kSkipPool heavy nodes with the most list entries over the key's samples.
    for (int attempt = memo_pool ? 1 : 0; attempt < 2; ++attempt) {
      if (attempt == 1) {
        for (int64_t x = s0 + tid; x < s1; x += kMemoThreads) {
          const int64_t o = gp[x].y;
          if (o < 0) continue;
          for (int64_t q = edge_ptr[o]; q < edge_ptr[o + 1]; ++q) {
            const int32_t v = edge_nodes[q];
            const int hb = heavy_bit[v];
            if (hb >= 0) atomicAdd(&hscore[hb], (unsigned long long)(node_ptr[v + 1] - node_ptr[v]));
          }
        }
        for (int t = tid; t < kQHash; t += kMemoThreads) qh[t] = 0u;
        for (int t = tid; t < kSigHash; t += kMemoThreads) {
          sig_key[t] = 0ull;
          sig_cnt[t] = 0u;
          sig_rep[t] = ~0u;
        }
        __syncthreads();
        if (tid == 0) {
          uint64_t pool = 0;
          for (int r = 0; r < kSkipPool; ++r) {
            unsigned long long best = 0;
            int bh = -1;
            for (int h = 0; h < kHeavyBits; ++h)
              if (!((pool >> h) & 1ull) && hscore[h] > best) { best = hscore[h]; bh = h; }
            if (bh < 0) break;
            pool |= 1ull << bh;
          }
          s_allowed = pool;
          s_nq = 0u;
          s_ovf = 0u;
          s_umask = 0ull;
        }
      } else if (tid == 0) {
        s_allowed = ~0ull;
      }
      __syncthreads();
      const uint64_t allowed = s_allowed;
      for (int64_t x = s0 + tid; x < s1; x += kMemoThreads) {
        const int64_t o = gp[x].y;
        uint32_t packed = kQNone | (kQNone << 7) | (kQNone << 14);
        if (o >= 0) {
          const int64_t os = edge_ptr[o];
          packed = skip_set(edge_nodes + os, int(edge_ptr[o + 1] - os), heavy_bit, node_ptr, allowed);
        }
        sS[x] = packed;
        {
          // signature: |e_o|, |e_o ∩ e_key|, the skipped set, which of it lies in e_key
          uint64_t sig = ~0ull;
          if (o >= 0) {
            const int64_t os = edge_ptr[o];
            const int b = int(edge_ptr[o + 1] - os);
            int pp = 0;
            for (int y = 0; y < b; ++y) pp += in_sorted(se, a, edge_nodes[os + y]) ? 1 : 0;
            uint32_t kin = 0;
            for (int r = 0; r < kSkip; ++r) {
              const uint32_t hb = (packed >> (7 * r)) & 127u;
              if (hb != kQNone && ((hmask[key] >> hb) & 1ull)) kin |= 1u << r;
            }
            sig = (uint64_t(b) | (uint64_t(pp) << 6) | (uint64_t(packed) << 12) | (uint64_t(kin) << 33)) + 1ull;
          }
          uint32_t slot = uint32_t((sig * 0x9E3779B97F4A7C15ull) >> 53) & (kSigHash - 1);  // 11 bits
          uint32_t found = ~0u;
          for (int probe = 0; probe < 64; ++probe, slot = (slot + 1u) & (kSigHash - 1)) {
            const unsigned long long old = atomicCAS(&sig_key[slot], 0ull, sig);
            if (old == 0ull || old == sig) {
              atomicAdd(&sig_cnt[slot], 1u);
              found = slot;
              break;
            }
          }
          smul[x] = found;  // the signature's slot for now (~0: table full)
        }
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
          uint32_t slot = (code * 2654435761u) >> 21;  // 11 bits
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
      if (!s_ovf) break;
    }
    // one representative per signature does the memo part for all of them
    for (int64_t x = s0 + tid; x < s1; x += kMemoThreads) {
      const uint32_t slot = smul[x];
      uint32_t mult = 1u;
      if (slot != ~0u) mult = atomicCAS(&sig_rep[slot], ~0u, uint32_t(x - s0)) == ~0u ? sig_cnt[slot] : 0u;
      smul[x] = mult;
    }
    __syncthreads();
    const int nq = int(s_nq);
    const uint32_t cells = uint32_t(kDiff) * uint32_t(a);  // binned cells of a slot
    const uint32_t sw = slot_words(a);
    const uint64_t words = 2ull + uint64_t(nq) + (1ull + uint64_t(nq)) * sw;
    if (tid == 0) {
      // one fetch-and-add per key (no retries); once a key overruns the
      // arena, every later one does too and is left to plain enumeration
      unsigned long long off = ~0ull;
      if (!s_ovf) {
        const unsigned long long at = atomicAdd(arena_top, (unsigned long long)words);
        if (at + words <= arena_words) off = at;
      }
      s_off = off;
      memo_off[key] = off == ~0ull ? -1 : int64_t(off);
      if (off != ~0ull) {
        atomicAdd(n_memo, 1ull);
        // list entries the memo build walks (one walk per pass of slots)
        const int per = int(kMemoCtr / (uint32_t(kDiff) * uint32_t(a) + uint32_t(kTally) + uint32_t(kCBins)));
        atomicAdd(n_memo + 1, (unsigned long long)(s_wpre[s_nw]) * (unsigned long long)((nq + per) / per));
      }
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
    uint32_t* gctr = mem + 2 + nq;  // (1 + nq) slots of sw words
    const unsigned long long umask = s_umask;
    const uint64_t key_hm = hmask[key];
    const int nw = s_nw, nsk = s_nsk;
    const uint32_t full = (1u << nsk) - 1u;
    // LDS per slot: binned cells, the tally of walked e_k holding skipped key
    // nodes (by pattern and size), and the neighbours holding Q by size
    const uint32_t stride = cells + uint32_t(kTally) + uint32_t(kCBins);
    const uint32_t tot0 = cells + uint32_t(kTally);
    const int per_pass = int(kMemoCtr / stride);  // >= 36
    const int64_t L = s_wpre[nw];
    for (int sl0 = 0; sl0 < 1 + nq; sl0 += per_pass) {
      const int sl1 = min(1 + nq, sl0 + per_pass);
      const uint32_t n_ctr = uint32_t(sl1 - sl0) * stride;
      for (uint32_t t = tid; t < n_ctr; t += kMemoThreads) ctr[t] = 0u;
      __syncthreads();
      if (s_novf == 0u)
        memo_walk<false>(ktab, win[tid >> 6], tid & 63, tid >> 6, L, s_wn, s_wlo, s_wpre, int32_t(key),
                         0u, node_edges, xoff, xnodes, hmask, umask, qs, nq, sl0, sl1, a, cells,
                         stride, tot0, ctr);
      else
        memo_walk<true>(ktab, win[tid >> 6], tid & 63, tid >> 6, L, s_wn, s_wlo, s_wpre, int32_t(key),
                        s_novf, node_edges, xoff, xnodes, hmask, umask, qs, nq, sl0, sl1, a, cells,
                        stride, tot0, ctr);
      __syncthreads();
      // neighbours meeting e_key only in skipped nodes P: s = |P|
      for (uint32_t t = tid; t < uint32_t(sl1 - sl0) * kTally; t += kMemoThreads) {
        const int slot = sl0 + int(t / kTally);
        const uint32_t rem = t % kTally;
        const uint32_t pat = rem / kCBins + 1u;
        const int bin = int(rem % kCBins);
        if (pat & ~full) continue;
        uint64_t qmask = 0;
        if (slot > 0) {
          const uint32_t code = qs[slot - 1];
          for (int r = 0; r < 3; ++r) {
            const uint32_t hb = (code >> (7 * r)) & 127u;
            if (hb != kQNone) qmask |= 1ull << hb;
          }
        }
        int64_t n = 0;
        for (uint32_t sup = pat; sup <= full; sup = (sup + 1u) | pat) {  // supersets of pat
          uint64_t xm = qmask;
          for (int r = 0; r < nsk; ++r)
            if (sup & (1u << r)) xm |= 1ull << s_skh[r];
          const int64_t f = heavy_set_count(xm, tcol(bin), hsize, hpair, htriple, big_key, big_val, big_log2);
          n += (__popc(sup ^ pat) & 1) ? -f : f;
        }
        const uint32_t base = uint32_t(slot - sl0) * stride;
        n -= ctr[base + cells + (pat - 1u) * kCBins + uint32_t(bin)];
        if (pat == full && (qmask & ~key_hm) == 0ull && cbin(a) == uint32_t(bin)) n -= 1;  // e_key itself
        if (n < 0) bad = true;
        if (n > 0) {
          const int np = __popc(pat);
          const int d = bin == kSizeTail ? kDiff - 1 : min(bin + 1 - np, kDiff - 1);
          atomicAdd(&ctr[base + uint32_t(np - 1) * kDiff + uint32_t(d)], uint32_t(n));
          atomicAdd(&ctr[base + tot0 + uint32_t(bin)], uint32_t(n));
        }
      }
      __syncthreads();
      for (uint32_t t = tid; t < uint32_t(sl1 - sl0) * sw; t += kMemoThreads) {
        const uint32_t sl = t / sw, w = t % sw;
        const int slot = sl0 + int(sl);
        uint32_t out = 0;
        if (w < cells) {
          out = ctr[sl * stride + w];
        } else if (slot > 0) {
          // hyperedges holding Q and not adjacent to the key (Q has no node of
          // e_key, else there are none), by size bin
          const uint32_t code = qs[slot - 1];
          uint64_t qmask = 0;
          for (int r = 0; r < 3; ++r) {
            const uint32_t hb = (code >> (7 * r)) & 127u;
            if (hb != kQNone) qmask |= 1ull << hb;
          }
          if ((qmask & key_hm) == 0ull) {
            const int fb = int(w - cells);  // sizes fb + 1, the last bin every size from 5
            const int b_lo = fb, b_hi = fb == kFarBins - 1 ? kSizeTail : fb;
            int64_t n = 0;
            for (int bin = b_lo; bin <= b_hi; ++bin)
              n += heavy_set_count(qmask, tcol(bin), hsize, hpair, htriple, big_key, big_val, big_log2) -
                   int64_t(ctr[sl * stride + tot0 + uint32_t(bin)]);
            if (n < 0) bad = true;
            out = uint32_t(n);
          }
        }
        gctr[uint64_t(slot) * sw + w] = out;
      }
      __syncthreads();
    }
  }
  if (bad) atomicOr(flags, 8);
}

// samples whose key was not memoized, for the plain on-the-fly enumeration
__global__ void k_leftover(int64_t cnt, const int2* __restrict__ gp, const int64_t* __restrict__ memo_off,
                           int2* out, unsigned long long* nout) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  const int2 pr = gp[s];
  if (memo_off[pr.x] < 0) out[atomicAdd(nout, 1ull)] = pr;
}

// hist[id] += v over the lanes of the wave (all lanes call it), one LDS atomic
// per distinct id; additions are modulo 2^64
__device__ __forceinline__ void wave_hadd(unsigned long long* hist, uint32_t id, int64_t v, int lane) {
  uint64_t pend = __ballot(v != 0);
  while (pend) {
    const int leader = __ffsll((long long)pend) - 1;
    const uint32_t lid = uint32_t(__shfl(int(id), leader));
    const bool mine = v != 0 && id == lid;
    pend &= ~__ballot(mine);
    const int64_t sum = wave_sum_i64(mine ? v : 0);
    if (lane == leader) atomicAdd(&hist[lid], (unsigned long long)sum);
  }
}

// The walk of e_o's non-skipped lists for one sample (i = key, j = o in the
// per-visit sums).  An e_k is taken at its smallest walked node; it adds its
// exact class, and moves what the memo counts would otherwise give it: the
// key-only class if it is adjacent to the key, or the class of an e_k meeting
// e_o only in its skipped nodes P if it holds some.
template <bool kOvf>
__device__ __forceinline__ void walk_other(WalkLds& L, int lane, int64_t T, uint32_t a, uint32_t b,
                                           uint32_t p, uint32_t kin, uint32_t novf,
                                           const uint32_t* __restrict__ xoff,
                                           const int32_t* __restrict__ xnodes, const uint16_t* lut,
                                           unsigned long long* hist) {
  if (T <= 0) return;
  int x = 0;
  int64_t lend = L.pre[1];
  int64_t base = L.wb[0];
  int32_t v = L.wn[0];
  uint32_t run_id = 0, run_n = 0, off_id = 0, off_n = 0;
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
        if (pat || wi) {
          const uint32_t oid = pat ? lut[triple_code(a, b, c, p, __popc(pat), wi, __popc(pat & kin))]
                                   : lut[triple_code(a, b, c, p, 0u, wi, 0u)];
          if (oid != off_id) {
            if (off_n) atomicAdd(&hist[off_id], (unsigned long long)(-int64_t(off_n)));
            off_id = oid;
            off_n = 0;
          }
          ++off_n;
        }
      }
    }
    wave_sync();
  }
  if (run_n) atomicAdd(&hist[run_id], (unsigned long long)run_n);
  if (off_n) atomicAdd(&hist[off_id], (unsigned long long)(-int64_t(off_n)));
}

// One wave per sample of a memoized key (samples of other keys are skipped).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_msample(
    int64_t cnt, int64_t E, const int2* __restrict__ gp, const uint32_t* __restrict__ sS,
    const uint32_t* __restrict__ smul, const int64_t* __restrict__ memo_off,
    const uint32_t* __restrict__ arena,
    const int64_t* __restrict__ edge_ptr, const int32_t* __restrict__ edge_nodes,
    const int64_t* __restrict__ node_ptr, const int8_t* __restrict__ heavy_bit,
    const uint32_t* __restrict__ xoff, const int32_t* __restrict__ xnodes,
    const uint32_t* __restrict__ hsize, const uint32_t* __restrict__ hpair,
    const uint32_t* __restrict__ htriple, const uint16_t* __restrict__ code_to_id3,
    unsigned long long* queue, unsigned long long* hist_out, int32_t* flags) {
  __shared__ uint16_t lut[kNumCodes];
  __shared__ unsigned long long hist[kHistSlots];
  __shared__ WalkLds lds[kEnumWaves];
  for (int t = threadIdx.x; t < kNumCodes; t += blockDim.x) lut[t] = code_to_id3[t];
  for (int t = threadIdx.x; t < kHistSlots; t += blockDim.x) hist[t] = 0ull;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  WalkLds& L = lds[wave];
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
      // memoized counts of the key, once per signature (times its samples)
      const int64_t mult = int64_t(smul[smp]);
      const uint32_t* mk = arena + mo;
      const int nq = int(mk[1]);
      if (int(mk[0]) != a) bad = true;
      const uint32_t* qs = mk + 2;
      const uint32_t sw = slot_words(a);
      const uint32_t cells = uint32_t(kDiff) * uint32_t(a);
      const uint32_t* g0 = mk + 2 + nq;
      // e_o's own cell (it is a neighbour of the key holding every set Q)
      const uint32_t ob = (p - 1u) * kDiff + uint32_t(min(b - int(p), kDiff - 1));
      // the key's neighbours, each first counted as if it met e_o nowhere
      for (uint32_t x0 = 0; mult && x0 < cells; x0 += kWave) {
        const uint32_t x = x0 + uint32_t(lane);
        const bool act = x < cells;
        const uint32_t s = x / kDiff + 1u, c = s + x % kDiff;
        int64_t m = act ? int64_t(g0[x]) : 0;
        if (x == ob) m -= 1;
        wave_hadd(hist, lut[triple_code(a, b, c, p, 0u, s, 0u)], m * mult, lane);
      }
      for (uint32_t qm = 1; mult && qm < (1u << nskip); ++qm) {
        int y[3], ny = 0;
        for (int r = 0; r < nskip; ++r)
          if (qm & (1u << r)) y[ny++] = hb[r];
        const int idx = find_code(qs, nq, qcode(ny, y[0], ny > 1 ? y[1] : 0, ny > 2 ? y[2] : 0));
        if (idx < 0) { bad = true; continue; }
        const uint32_t* gq = g0 + uint64_t(1 + idx) * sw;
        const int nqm = __popc(qm);
        // neighbours of the key meeting e_o in exactly P ⊆ Q: inclusion-exclusion
        for (uint32_t x0 = 0; x0 < cells; x0 += kWave) {
          const uint32_t x = x0 + uint32_t(lane);
          const bool act = x < cells;
          const uint32_t s = x / kDiff + 1u, c = s + x % kDiff;
          int64_t m = act ? int64_t(gq[x]) : 0;
          if (x == ob) m -= 1;
          m *= mult;
          for (uint32_t pm = qm; pm; pm = (pm - 1u) & qm) {
            const int np = __popc(pm);
            wave_hadd(hist, lut[triple_code(a, b, c, p, uint32_t(np), s, uint32_t(__popc(pm & kin)))],
                      ((nqm - np) & 1) ? -m : m, lane);
          }
          wave_hadd(hist, lut[triple_code(a, b, c, p, 0u, s, 0u)], (nqm & 1) ? -m : m, lane);
        }
        if ((qm & kin) == 0u) {
          // hyperedges holding Q and not adjacent to the key, by size bin
          const int64_t m0 = lane < kFarBins ? int64_t(gq[cells + uint32_t(lane)]) * mult : 0;
          const uint32_t c = uint32_t(lane) + 1u;
          for (uint32_t pm = qm; pm; pm = (pm - 1u) & qm) {
            const int np = __popc(pm);
            wave_hadd(hist, lut[triple_code(a, b, c, p, uint32_t(np), 0u, 0u)],
                      ((nqm - np) & 1) ? -m0 : m0, lane);
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
  uint32_t* smul = nullptr;            // [chunk] samples sharing the sample's memo part (0: another does it)
  uint32_t* arena = nullptr;
  uint64_t arena_words = 0;
  void* cub = nullptr;
  size_t cub_bytes = 0;
  unsigned long long* ctr = nullptr;   // [0] nk | queue, [1] arena top, [2] leftovers, [3] sample
                                       // queue, [4] keys memoized, [5] entries the builds walk
  int64_t* deg_tmp = nullptr;          // [E] line-graph degrees when the graph keeps none
};

void memo_end(mochy_ctx* ctx, memo_bufs* m) {
  if (!m) return;
  void* bufs[] = {m->kcnt, m->koff, m->kcur, m->klist, m->skey,  m->skey2, m->memo_off, m->tmp,
                  m->gp,   m->left, m->sS,   m->smul,  m->arena, m->cub,   m->ctr,      m->deg_tmp};
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
      (rc = device_alloc(ctx, (void**)&m->smul, size_t(chunk) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->arena, size_t(std::max<uint64_t>(m->arena_words, 1)) * 4)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&m->ctr, 6 * 8)) != MOCHY_OK) {
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
  MOCHY_HIP(hipMemsetAsync(m->ctr, 0, 6 * 8, st));
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
      g->xnodes, g->hsize, g->hpair, g->htriple, g->hbig_key, g->hbig_val, g->hbig_log2, m->skey2,
      nk, kqueue, m->koff, m->gp, m->sS, m->smul, m->arena, m->arena_words, top, m->memo_off,
      ctx->memo_all ? 1 : 0, ctx->memo_pool ? 1 : 0, m->ctr + 4, flags);
  k_leftover<<<blocks(cnt, 256), 256, 0, st>>>(cnt, m->gp, m->memo_off, m->left, nleft);
  k_msample<<<unsigned(ctx->num_cus) * 8u, kEnumWaves * kWave, 0, st>>>(
      cnt, E, m->gp, m->sS, m->smul, m->memo_off, m->arena, g->edge_ptr, g->edge_nodes, g->node_ptr,
      g->heavy_bit, g->xoff, g->xnodes, g->hsize, g->hpair, g->htriple, ctx->d_code_to_id3, squeue,
      (unsigned long long*)d_hist, flags);
  MOCHY_HIP(hipGetLastError());
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, m->ctr, 6 * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  *n_left = ctx->h_small[2];
  ctx->memo_stats[1] += cnt - ctx->h_small[2];
  ctx->memo_stats[2] += ctx->h_small[4];
  ctx->memo_stats[3] = std::max<int64_t>(
      ctx->memo_stats[3], std::min<int64_t>(ctx->h_small[1], int64_t(m->arena_words)) * 4);
  ctx->memo_stats[4] += ctx->h_small[5];
  *left = m->left;
  return MOCHY_OK;
}
