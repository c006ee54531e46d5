// Host-sanitizer driver of the CPU oracle (oracle/mochy_oracle.cpp), built by
// tests/test_sanitizers_cpu.py with AddressSanitizer and
// UndefinedBehaviorSanitizer.  Runs every oracle counter on seeded random
// small hypergraphs (sizes 1..6, repeated hyperedges removed) and checks
// the identities that hold between them: brute force equals plain MoCHy-E,
// hyperedge profiles sum to three times the counts, and an exhaustive
// MoCHy-A+ pass (every hyperwedge once) gives w times the counts.
// argv[1]: the canonical-code table (2187 int32, from oracle/patterns.py).
#include <cstdint>
#include <cstdio>
#include <set>
#include <vector>

extern "C" {
void orc_bruteforce(int64_t E, const int64_t* ptr, const int32_t* nodes, int theta,
                    const int32_t* canon_to_id3, int64_t* out3, int nthreads);
void orc_mochy_e(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes, int64_t c0,
                 int64_t c1, int theta, const int32_t* canon_to_id3, int64_t* out3, int nthreads);
int64_t orc_wedge_prefix(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes,
                         int64_t* up_ptr, int nthreads);
int64_t orc_aplus_raw(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes, int64_t n0,
                      int64_t n1, uint64_t seed, const int64_t* indices, const int64_t* up_ptr_in,
                      int theta, const int32_t* canon_to_id3, int64_t* raw3, int nthreads);
int64_t orc_mochy_a_raw(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes, int64_t n0,
                        int64_t n1, uint64_t seed, const int64_t* indices, int theta,
                        const int32_t* canon_to_id3, int64_t* raw3, int nthreads);
void orc_hyperedge_profiles(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes,
                            int64_t c0, int64_t c1, int theta, const int32_t* canon_to_id3,
                            int64_t* out, int nthreads);
int64_t orc_line_graph_triangles(int64_t E, int64_t V, const int64_t* ptr, const int32_t* nodes,
                                 int nthreads);
}

static uint64_t lcg(uint64_t& s) {
  s = s * 6364136223846793005ull + 1442695040888963407ull;
  return s >> 33;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  std::vector<int32_t> canon(2187);
  FILE* f = std::fopen(argv[1], "rb");
  if (!f || std::fread(canon.data(), 4, canon.size(), f) != canon.size()) return 2;
  std::fclose(f);
  std::vector<int32_t> parent(432);  // argv[2]: 3h id -> h id (432 int32)
  f = std::fopen(argv[2], "rb");
  if (!f || std::fread(parent.data(), 4, parent.size(), f) != parent.size()) return 2;
  std::fclose(f);
  std::vector<int> open26(27, 0);
  for (int t = 17; t <= 22; ++t) open26[t] = 1;
  uint64_t s = 12345;
  for (int trial = 0; trial < 25; ++trial) {
    const int V = 6 + int(lcg(s) % 10), Edraw = 4 + int(lcg(s) % 24);
    std::set<std::vector<int32_t>> seen;
    std::vector<int64_t> ptr{0};
    std::vector<int32_t> nodes;
    for (int e = 0; e < Edraw; ++e) {
      const int size = 1 + int(lcg(s) % 6);
      std::set<int32_t> m;
      while (int(m.size()) < std::min(size, V)) m.insert(int32_t(lcg(s) % V));
      std::vector<int32_t> row(m.begin(), m.end());
      if (!seen.insert(row).second) continue;
      nodes.insert(nodes.end(), row.begin(), row.end());
      ptr.push_back(int64_t(nodes.size()));
    }
    const int64_t E = int64_t(ptr.size()) - 1;
    std::vector<int64_t> bf(432), me(432), ap(432), ma(432), prof(size_t(E) * 432);
    orc_bruteforce(E, ptr.data(), nodes.data(), 1, canon.data(), bf.data(), 2);
    orc_mochy_e(E, V, ptr.data(), nodes.data(), 0, E, 1, canon.data(), me.data(), 2);
    for (int t = 0; t < 432; ++t)
      if (bf[t] != me[t]) { std::printf("trial %d: brute force and MoCHy-E differ at %d\n", trial, t); return 1; }
    std::vector<int64_t> up(E + 1);
    const int64_t W = orc_wedge_prefix(E, V, ptr.data(), nodes.data(), up.data(), 2);
    std::vector<int64_t> idx(W);
    for (int64_t w = 0; w < W; ++w) idx[w] = w;
    orc_aplus_raw(E, V, ptr.data(), nodes.data(), 0, W, 7, W ? idx.data() : nullptr, up.data(), 1,
                  canon.data(), ap.data(), 2);
    for (int t = 1; t < 432; ++t) {
      const int64_t w = open26[parent[t]] ? 2 : 3;
      if (ap[t] != w * bf[t]) { std::printf("trial %d: exhaustive A+ differs at %d\n", trial, t); return 1; }
    }
    std::vector<int64_t> all(E);
    for (int64_t e = 0; e < E; ++e) all[e] = e;
    orc_mochy_a_raw(E, V, ptr.data(), nodes.data(), 0, E, 3, E ? all.data() : nullptr, 1, canon.data(),
                    ma.data(), 2);
    orc_hyperedge_profiles(E, V, ptr.data(), nodes.data(), 0, E, 1, canon.data(), prof.data(), 2);
    for (int t = 0; t < 432; ++t) {
      int64_t col = 0;
      for (int64_t e = 0; e < E; ++e) col += prof[size_t(e) * 432 + t];
      if (col != 3 * bf[t] || ma[t] != 3 * bf[t]) {
        std::printf("trial %d: profiles or exhaustive MoCHy-A differ at %d\n", trial, t);
        return 1;
      }
    }
    (void)orc_line_graph_triangles(E, V, ptr.data(), nodes.data(), 2);
  }
  std::printf("oracle ok\n");
  return 0;
}
