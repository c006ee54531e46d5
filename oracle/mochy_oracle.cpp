// CPU oracle for hypergraph-motif counting (MoCHy, arXiv 2310.15668).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code with the HIP library.
//
// Plain, slow, obviously correct.  Every count is an int64.  Each function
// cites the passage it follows.
//
// Classification of a triple (shared by all counters here): the seven region
// cardinalities (section 2.2; Lemma 2 gives them from |e_i|,|e_j|,|e_k|, the
// three pairwise overlaps and the triple overlap) are mapped to ternary
// states (section 5.1: 0 if empty, 1 if at most theta, 2 otherwise), the
// tuple is relabelled by all six permutations of (i, j, k), the
// lexicographically smallest tuple is looked up in a table of canonical codes
// handed in by the Python side of the oracle (oracle/patterns.py), which
// gives the 3h-motif id; the caller folds 3h ids into h ids.

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>
#include <omp.h>

namespace {

// Regions as subsets of {i=bit0, j=bit1, k=bit2}, in the paper's order R1..R7.
const int kRegionMask[7] = {1, 2, 4, 3, 6, 5, 7};

struct Perms {
  int map[6][7];  // map[p][r] = region index of the image of region r under permutation p
  Perms() {
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int p = 0; p < 6; ++p)
      for (int r = 0; r < 7; ++r) {
        int img = 0;
        for (int x = 0; x < 3; ++x)
          if (kRegionMask[r] & (1 << x)) img |= 1 << perm[p][x];
        for (int q = 0; q < 7; ++q)
          if (kRegionMask[q] == img) map[p][r] = q;
      }
  }
};
const Perms kPerms;

inline int state_of(int64_t c, int theta) { return c == 0 ? 0 : (c <= theta ? 1 : 2); }

// 3h id (1..431) of a triple with region cardinalities card[0..6]; 0 if the
// pattern is not a valid motif (duplicate or disconnected hyperedges).
inline int classify(const int64_t card[7], int theta, const int32_t* canon_to_id3) {
  int st[7];
  for (int r = 0; r < 7; ++r) st[r] = state_of(card[r], theta);
  int best = 1 << 30;
  for (int p = 0; p < 6; ++p) {
    // region r of the relabelled triple is region map[p][r] of this one
    int code = 0;
    for (int r = 0; r < 7; ++r) code = code * 3 + st[kPerms.map[p][r]];
    best = std::min(best, code);
  }
  return canon_to_id3[best];
}

// Region cardinalities from the quantities of Lemma 2.
inline void regions_from_overlaps(int64_t a, int64_t b, int64_t c, int64_t wij, int64_t wjk,
                                  int64_t wki, int64_t t, int64_t card[7]) {
  card[0] = a - wij - wki + t;
  card[1] = b - wij - wjk + t;
  card[2] = c - wki - wjk + t;
  card[3] = wij - t;
  card[4] = wjk - t;
  card[5] = wki - t;
  card[6] = t;
}

struct Graph {
  int64_t E, V;
  const int64_t* ptr;
  const int32_t* nodes;
  std::vector<int64_t> vptr;   // E_v, transposed incidence
  std::vector<int32_t> vedges;
  Graph(int64_t E_, int64_t V_, const int64_t* p, const int32_t* n) : E(E_), V(V_), ptr(p), nodes(n) {
    vptr.assign(V + 1, 0);
    for (int64_t q = 0; q < ptr[E]; ++q) vptr[nodes[q] + 1]++;
    for (int64_t v = 0; v < V; ++v) vptr[v + 1] += vptr[v];
    vedges.resize(ptr[E]);
    std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
    for (int64_t e = 0; e < E; ++e)
      for (int64_t q = ptr[e]; q < ptr[e + 1]; ++q) vedges[fill[nodes[q]]++] = (int32_t)e;
  }
  int64_t size(int64_t e) const { return ptr[e + 1] - ptr[e]; }
  // |e_x ∩ e_y| by merging the two sorted node lists.
  int64_t overlap(int64_t x, int64_t y) const {
    int64_t p = ptr[x], q = ptr[y], n = 0;
    while (p < ptr[x + 1] && q < ptr[y + 1]) {
      if (nodes[p] < nodes[q]) ++p;
      else if (nodes[p] > nodes[q]) ++q;
      else { ++n; ++p; ++q; }
    }
    return n;
  }
  bool contains(int64_t e, int32_t v) const {
    return std::binary_search(nodes + ptr[e], nodes + ptr[e + 1], v);
  }
  // |e_x ∩ e_y ∩ e_z|: check each node of the smallest for membership in the
  // other two (Lemma 2).
  int64_t triple(int64_t x, int64_t y, int64_t z) const {
    int64_t s[3] = {x, y, z};
    std::sort(s, s + 3, [&](int64_t a, int64_t b) { return size(a) < size(b); });
    int64_t n = 0;
    for (int64_t q = ptr[s[0]]; q < ptr[s[0] + 1]; ++q)
      if (contains(s[1], nodes[q]) && contains(s[2], nodes[q])) ++n;
    return n;
  }
  // N_{e_i} with omega: Algorithm 1's inner loops for one hyperedge, both
  // directions (every e_j in E_v for v in e_i, j != i, adds one to omega).
  void neighbors(int64_t i, std::vector<std::pair<int32_t, int32_t>>& out) const {
    std::unordered_map<int32_t, int32_t> omega;
    for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) {
      int32_t v = nodes[q];
      for (int64_t r = vptr[v]; r < vptr[v + 1]; ++r)
        if (vedges[r] != i) omega[vedges[r]] += 1;
    }
    out.assign(omega.begin(), omega.end());
    std::sort(out.begin(), out.end());
  }
};

inline void add_hist(std::vector<int64_t>& local, int id3) { local[id3] += 1; }

}  // namespace

extern "C" {

int orc_abi_version() { return 6; }

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
// as 1, 2, 3", SC'11): ten rounds of the 4x32 S-box; each round multiplies
// words 0 and 2 by the two round multipliers, swaps and xors the high halves
// with the key, and the key is advanced by the two Weyl constants between
// rounds.
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c[0];
    uint64_t p1 = (uint64_t)M1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  memcpy(out, c, sizeof(c));
}

// Region cardinalities of one triple, straight from the definition: every node
// of the union is placed in the region given by which of the three contain it.
void orc_region_cards(const int64_t* ptr, const int32_t* nodes, int64_t i, int64_t j, int64_t k,
                      int64_t card[7]) {
  auto in = [&](int64_t e, int32_t v) { return std::binary_search(nodes + ptr[e], nodes + ptr[e + 1], v); };
  int64_t by_mask[8] = {0};
  for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) {
    const int32_t v = nodes[q];
    by_mask[1 | (in(j, v) ? 2 : 0) | (in(k, v) ? 4 : 0)] += 1;
  }
  for (int64_t q = ptr[j]; q < ptr[j + 1]; ++q) {
    const int32_t v = nodes[q];
    if (!in(i, v)) by_mask[2 | (in(k, v) ? 4 : 0)] += 1;
  }
  for (int64_t q = ptr[k]; q < ptr[k + 1]; ++q) {
    const int32_t v = nodes[q];
    if (!in(i, v) && !in(j, v)) by_mask[4] += 1;
  }
  for (int r = 0; r < 7; ++r) card[r] = by_mask[kRegionMask[r]];
}

int orc_classify(const int64_t card[7], int theta, const int32_t* canon_to_id3) {
  return classify(card, theta, canon_to_id3);
}

// Tier 1: brute force over all C(|E|,3) triples (definition, section 2.2):
// a triple is counted iff it is connected (one hyperedge meets the other two);
// out3[id] += 1 for its 3h id; out3[0] collects connected triples whose
// pattern is invalid (possible only if hyperedges repeat).
void orc_bruteforce(int64_t E, const int64_t* ptr, const int32_t* nodes, int theta,
                    const int32_t* canon_to_id3, int64_t* out3 /*432*/, int nthreads) {
  std::vector<int64_t> total(432, 0);
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int64_t> local(432, 0);
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < E; ++i)
      for (int64_t j = i + 1; j < E; ++j)
        for (int64_t k = j + 1; k < E; ++k) {
          int64_t card[7];
          orc_region_cards(ptr, nodes, i, j, k, card);
          bool ij = card[3] + card[6] > 0, jk = card[4] + card[6] > 0, ki = card[5] + card[6] > 0;
          bool connected = (ij && ki) || (ij && jk) || (jk && ki);
          if (!connected) continue;
          add_hist(local, classify(card, theta, canon_to_id3));
        }
#pragma omp critical
    for (int t = 0; t < 432; ++t) total[t] += local[t];
  }
  memcpy(out3, total.data(), 432 * sizeof(int64_t));
}

// Line-graph degrees d_i = |N_{e_i}| (section 2.1) and |wedges| (Algorithm 1).
int64_t orc_line_graph_degrees(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes,
                               int64_t* deg, int nthreads) {
  Graph g(E, V, ptr, nodes);
  int64_t total = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : total)
  {
    std::vector<int64_t> mark(E, -1);
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < E; ++i) {
      int64_t d = 0;
      for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) {
        int32_t v = nodes[q];
        for (int64_t r = g.vptr[v]; r < g.vptr[v + 1]; ++r) {
          int64_t x = g.vedges[r];
          if (x != i && mark[x] != i) { mark[x] = i; ++d; }
        }
      }
      deg[i] = d;
      total += d;
    }
  }
  return total / 2;
}

// Tier 2: plain MoCHy-E (Algorithm 1 for the neighbourhood of each centre,
// Algorithm 2 for the pairs), restricted to centres in [c0, c1).  For each
// centre e_i and each unordered pair {e_j, e_k} of its neighbours, the
// instance is counted iff e_j and e_k are disjoint or i < min(j, k)
// (Algorithm 2's condition), which attributes every instance to exactly one
// centre: the middle hyperedge of an open instance, the smallest index of a
// closed one.  omega(e_j, e_k) is |e_j ∩ e_k|, the value the line graph
// stores, obtained here by merging the node lists.
static void mochy_e_over(const Graph& g, const int64_t* centers, int64_t n, int theta,
                         const int32_t* canon_to_id3, int64_t* out3, int nthreads) {
  std::vector<int64_t> total(432, 0);
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int64_t> local(432, 0);
    std::vector<std::pair<int32_t, int32_t>> nb;
#pragma omp for schedule(dynamic, 1)
    for (int64_t c = 0; c < n; ++c) {
      const int64_t i = centers[c];
      g.neighbors(i, nb);
      const int64_t a = g.size(i);
      for (size_t x = 0; x < nb.size(); ++x)
        for (size_t y = x + 1; y < nb.size(); ++y) {
          const int64_t j = nb[x].first, k = nb[y].first;
          const int64_t wjk = g.overlap(j, k);
          if (!(wjk == 0 || i < std::min(j, k))) continue;
          const int64_t t = g.triple(i, j, k);
          int64_t card[7];
          regions_from_overlaps(a, g.size(j), g.size(k), nb[x].second, wjk, nb[y].second, t, card);
          add_hist(local, classify(card, theta, canon_to_id3));
        }
    }
#pragma omp critical
    for (int t = 0; t < 432; ++t) total[t] += local[t];
  }
  memcpy(out3, total.data(), 432 * sizeof(int64_t));
}

void orc_mochy_e(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes, int64_t c0,
                 int64_t c1, int theta, const int32_t* canon_to_id3, int64_t* out3 /*432*/,
                 int nthreads) {
  Graph g(E, V, ptr, nodes);
  std::vector<int64_t> centers;
  for (int64_t i = c0; i < c1; ++i) centers.push_back(i);
  mochy_e_over(g, centers.data(), int64_t(centers.size()), theta, canon_to_id3, out3, nthreads);
}

// The same for an explicit list of centres (each instance is attributed to
// one centre by Algorithm 2's condition, so any subset is well defined).
void orc_mochy_e_centers(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes,
                         const int64_t* centers, int64_t n, int theta,
                         const int32_t* canon_to_id3, int64_t* out3 /*432*/, int nthreads) {
  Graph g(E, V, ptr, nodes);
  mochy_e_over(g, centers, n, theta, canon_to_id3, out3, nthreads);
}

// MoCHy-E candidates of centres [c0, c1): sum of C(d_i, 2).
int64_t orc_candidates(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes, int64_t c0,
                       int64_t c1) {
  std::vector<int64_t> deg(E);
  orc_line_graph_degrees(E, V, ptr, nodes, deg.data(), 1);
  int64_t s = 0;
  for (int64_t i = c0; i < c1; ++i) s += deg[i] * (deg[i] - 1) / 2;
  return s;
}

// Number of triangles of the line graph (textbook edge-iterator with sorted
// forward adjacency): a check on closed-motif totals that shares nothing with
// the motif counters above.
int64_t orc_line_graph_triangles(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes,
                                 int nthreads) {
  Graph g(E, V, ptr, nodes);
  std::vector<std::vector<int32_t>> fwd(E);
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int64_t> mark(E, -1);
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < E; ++i) {
      for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q)
        for (int64_t r = g.vptr[nodes[q]]; r < g.vptr[nodes[q] + 1]; ++r) {
          int64_t x = g.vedges[r];
          if (x > i && mark[x] != i) { mark[x] = i; fwd[i].push_back((int32_t)x); }
        }
      std::sort(fwd[i].begin(), fwd[i].end());
    }
  }
  int64_t tri = 0;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64) reduction(+ : tri)
  for (int64_t i = 0; i < E; ++i)
    for (int32_t j : fwd[i]) {
      const auto& a = fwd[i];
      const auto& b = fwd[j];
      size_t p = 0, q = 0;
      while (p < a.size() && q < b.size()) {
        if (a[p] < b[q]) ++p;
        else if (a[p] > b[q]) ++q;
        else { ++tri; ++p; ++q; }
      }
    }
  return tri;
}

// Sorted N_{e_i} built on demand from E_v (section 4.4's on-the-fly
// neighbourhood: the union of E_v over v in e_i, minus e_i itself), so that
// no line graph has to be stored.  `mark` is a per-thread scratch of size |E|
// holding, for each hyperedge, the stamp of the last build that listed it;
// every build takes a fresh stamp.
static void neighbor_list(const Graph& g, int64_t i, std::vector<int64_t>& mark, int64_t& stamp,
                          std::vector<int32_t>& out) {
  out.clear();
  const int64_t st = ++stamp;
  for (int64_t q = g.ptr[i]; q < g.ptr[i + 1]; ++q) {
    const int32_t v = g.nodes[q];
    for (int64_t r = g.vptr[v]; r < g.vptr[v + 1]; ++r) {
      const int64_t x = g.vedges[r];
      if (x != i && mark[x] != st) { mark[x] = st; out.push_back((int32_t)x); }
    }
  }
  std::sort(out.begin(), out.end());
}

// Hyperwedge order for sampling: hyperwedges {e_i, e_j}, i < j, listed by
// (i, j) lexicographically; up_ptr[i] = number of hyperwedges whose smaller
// hyperedge is below i (exclusive prefix of the upper degrees
// |{j > i : e_i ∩ e_j non-empty}|).  Returns |wedges|.
int64_t orc_wedge_prefix(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes,
                         int64_t* up_ptr /*E+1*/, int nthreads) {
  Graph g(E, V, ptr, nodes);
  std::vector<int64_t> up(E, 0);
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int64_t> mark(E, -1);
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < E; ++i) {
      int64_t d = 0;
      for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q)
        for (int64_t r = g.vptr[nodes[q]]; r < g.vptr[nodes[q] + 1]; ++r) {
          const int64_t x = g.vedges[r];
          if (x > i && mark[x] != i) { mark[x] = i; ++d; }
        }
      up[i] = d;
    }
  }
  up_ptr[0] = 0;
  for (int64_t i = 0; i < E; ++i) up_ptr[i + 1] = up_ptr[i] + up[i];
  return up_ptr[E];
}

// MoCHy-A+ (Algorithm 5), hit counts before rescaling, for sample numbers
// n in [n0, n1).  Hyperwedges are ordered as in orc_wedge_prefix.  Sample n
// draws Philox4x32-10 with counter (lo32 n, hi32 n, 0, 0) and key
// (lo32 seed, hi32 seed); u = (x1 << 32) | x0; the hyperwedge index is
// floor(u * |wedges| / 2^64).  For the sampled wedge {e_i, e_j}, every
// e_k in N_i ∪ N_j minus {e_i, e_j} adds one to raw[h(i, j, k)].
// Both neighbourhoods are built on demand for each sample, so the line graph
// is never stored.  If `indices` is non-null, sample n uses hyperwedge
// indices[n] instead of Philox (used to visit every hyperwedge exactly once).
// `up_ptr_in` (E+1 entries, from orc_wedge_prefix) may be passed to skip
// recomputing the hyperwedge order; NULL computes it.
int64_t orc_aplus_raw(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes, int64_t n0,
                      int64_t n1, uint64_t seed, const int64_t* indices, const int64_t* up_ptr_in,
                      int theta, const int32_t* canon_to_id3, int64_t* raw3 /*432*/,
                      int nthreads) {
  Graph g(E, V, ptr, nodes);
  std::vector<int64_t> up_own;
  const int64_t* up_ptr = up_ptr_in;
  if (!up_ptr) {
    up_own.assign(E + 1, 0);
    orc_wedge_prefix(E, V, ptr, nodes, up_own.data(), nthreads);
    up_ptr = up_own.data();
  }
  const uint64_t W = (uint64_t)up_ptr[E];
  std::vector<int64_t> total(432, 0);
  if (W == 0) { memcpy(raw3, total.data(), 432 * sizeof(int64_t)); return 0; }
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int64_t> local(432, 0);
    std::vector<int64_t> mark(E, -1);
    std::vector<int32_t> ni, nj, uni;
    int64_t stamp = -1;
#pragma omp for schedule(dynamic, 1)
    for (int64_t n = n0; n < n1; ++n) {
      uint64_t idx;
      if (indices) {
        idx = (uint64_t)indices[n];
      } else {
        uint32_t ctr[4] = {(uint32_t)n, (uint32_t)((uint64_t)n >> 32), 0u, 0u};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t x[4];
        orc_philox4x32_10(ctr, key, x);
        uint64_t u = ((uint64_t)x[1] << 32) | x[0];
        idx = (uint64_t)(((unsigned __int128)u * W) >> 64);
      }
      const int64_t i = std::upper_bound(up_ptr, up_ptr + E + 1, (int64_t)idx) - up_ptr - 1;
      neighbor_list(g, i, mark, stamp, ni);
      const int64_t first_up = std::upper_bound(ni.begin(), ni.end(), (int32_t)i) - ni.begin();
      const int64_t j = ni[first_up + ((int64_t)idx - up_ptr[i])];
      neighbor_list(g, j, mark, stamp, nj);
      uni.clear();
      std::set_union(ni.begin(), ni.end(), nj.begin(), nj.end(), std::back_inserter(uni));
      const int64_t wij = g.overlap(i, j);
      for (int32_t k : uni) {
        if (k == i || k == j) continue;
        int64_t card[7];
        regions_from_overlaps(g.size(i), g.size(j), g.size(k), wij, g.overlap(j, k), g.overlap(k, i),
                              g.triple(i, j, k), card);
        add_hist(local, classify(card, theta, canon_to_id3));
      }
    }
#pragma omp critical
    for (int t = 0; t < 432; ++t) total[t] += local[t];
  }
  memcpy(raw3, total.data(), 432 * sizeof(int64_t));
  return (int64_t)W;
}

// Every instance (connected triple) that contains e_i, counted into local:
// each pair {e_j, e_k} of N_i (adjacent to each other or not), and each path
// e_i - e_j - e_k with e_j in N_i and e_k in N_j outside N_i and e_i (the
// 1-hop and 2-hop neighbourhoods explored by Algorithm 4).
static void instances_of(const Graph& g, int64_t i, int theta, const int32_t* canon_to_id3,
                         std::vector<int64_t>& mark, int64_t& stamp, std::vector<int32_t>& ni,
                         std::vector<int32_t>& nj, std::vector<int64_t>& local) {
  neighbor_list(g, i, mark, stamp, ni);
  int64_t card[7];
  for (size_t a = 0; a < ni.size(); ++a)
    for (size_t b = a + 1; b < ni.size(); ++b) {
      orc_region_cards(g.ptr, g.nodes, i, ni[a], ni[b], card);
      add_hist(local, classify(card, theta, canon_to_id3));
    }
  for (int32_t j : ni) {
    neighbor_list(g, j, mark, stamp, nj);
    for (int32_t k : nj) {
      if (k == i || std::binary_search(ni.begin(), ni.end(), k)) continue;
      orc_region_cards(g.ptr, g.nodes, i, j, k, card);
      add_hist(local, classify(card, theta, canon_to_id3));
    }
  }
}

// MoCHy-A (Algorithm 4), hit counts before rescaling, for sample numbers
// n in [n0, n1): sample n draws Philox4x32-10 with counter (lo32 n, hi32 n,
// 1, 0) and key (lo32 seed, hi32 seed); u = (x1 << 32) | x0; the sampled
// hyperedge is floor(u * |E| / 2^64), and every instance that contains it
// adds one to raw[h(instance)] (instances_of).  With `indices`, sample n is
// hyperedge indices[n].  Returns |E|.
int64_t orc_mochy_a_raw(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes, int64_t n0,
                        int64_t n1, uint64_t seed, const int64_t* indices, int theta,
                        const int32_t* canon_to_id3, int64_t* raw3 /*432*/, int nthreads) {
  Graph g(E, V, ptr, nodes);
  std::vector<int64_t> total(432, 0);
  if (E == 0) { memcpy(raw3, total.data(), 432 * sizeof(int64_t)); return 0; }
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int64_t> local(432, 0);
    std::vector<int64_t> mark(E, -1);
    std::vector<int32_t> ni, nj;
    int64_t stamp = -1;
#pragma omp for schedule(dynamic, 1)
    for (int64_t n = n0; n < n1; ++n) {
      int64_t i;
      if (indices) {
        i = indices[n];
      } else {
        uint32_t ctr[4] = {(uint32_t)n, (uint32_t)((uint64_t)n >> 32), 1u, 0u};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        uint32_t x[4];
        orc_philox4x32_10(ctr, key, x);
        const uint64_t u = ((uint64_t)x[1] << 32) | x[0];
        i = (int64_t)(((unsigned __int128)u * (uint64_t)E) >> 64);
      }
      instances_of(g, i, theta, canon_to_id3, mark, stamp, ni, nj, local);
    }
#pragma omp critical
    for (int t = 0; t < 432; ++t) total[t] += local[t];
  }
  memcpy(raw3, total.data(), 432 * sizeof(int64_t));
  return E;
}

// Hyperedge profiles (section 3.2): for each e_i with c0 <= i < c1, the
// number of instances of each motif that contain e_i; out[(i - c0) * 432 + id3].
void orc_hyperedge_profiles(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes,
                            int64_t c0, int64_t c1, int theta, const int32_t* canon_to_id3,
                            int64_t* out, int nthreads) {
  Graph g(E, V, ptr, nodes);
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int64_t> local(432, 0);
    std::vector<int64_t> mark(E, -1);
    std::vector<int32_t> ni, nj;
    int64_t stamp = -1;
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = c0; i < c1; ++i) {
      std::fill(local.begin(), local.end(), 0);
      instances_of(g, i, theta, canon_to_id3, mark, stamp, ni, nj, local);
      memcpy(out + (i - c0) * 432, local.data(), 432 * sizeof(int64_t));
    }
  }
}

}  // extern "C"
