// Pattern tables of the library: which ternary region code is which motif.
//
// Section 2.2: an h-motif is the emptiness pattern of the seven Venn regions
// of three hyperedges, up to relabelling the hyperedges, restricted to
// patterns three distinct, connected hyperedges can produce (26 of them).
// Section 5.1: a 3h-motif refines each region to empty / one node / more
// (theta = 1); 431 of them.
//
// Id rule (the paper's figure with the numbering is not available; the rule
// keeps every fact the text states: 17..22 open, 16 = all regions, 3h 1..6
// refine h 1): canonical tuple = lexicographically smallest (R1..R7) tuple over
// the six relabellings; h ids in three groups (closed with R7 non-empty, open,
// closed with R7 empty), each ordered by number of non-empty regions then
// canonical tuple; 3h ids ordered by parent h id then canonical ternary tuple.
#include <algorithm>
#include <array>
#include <map>
#include <set>

#include "common.h"

namespace {

using Tuple = std::array<uint8_t, 7>;

// Hyperedges i, j, k are bits 0, 1, 2; region r (R1..R7) is the set below.
constexpr uint8_t kRegion[7] = {0b001, 0b010, 0b100, 0b011, 0b110, 0b101, 0b111};

int region_index(uint8_t set) {
  for (int r = 0; r < 7; ++r)
    if (kRegion[r] == set) return r;
  return -1;
}

Tuple canonical(const Tuple& t) {
  std::array<int, 3> perm = {0, 1, 2};
  Tuple best;
  bool first = true;
  do {
    Tuple u;
    for (int r = 0; r < 7; ++r) {
      uint8_t img = 0;
      for (int b = 0; b < 3; ++b)
        if (kRegion[r] & (1u << b)) img |= uint8_t(1u << perm[b]);
      u[r] = t[region_index(img)];
    }
    if (first || u < best) best = u;
    first = false;
  } while (std::next_permutation(perm.begin(), perm.end()));
  return best;
}

bool meets(const Tuple& t, int x, int y) {
  for (int r = 0; r < 7; ++r)
    if (t[r] && (kRegion[r] >> x & 1) && (kRegion[r] >> y & 1)) return true;
  return false;
}

bool differ(const Tuple& t, int x, int y) {
  for (int r = 0; r < 7; ++r)
    if (t[r] && ((kRegion[r] >> x & 1) != (kRegion[r] >> y & 1))) return true;
  return false;
}

bool valid(const Tuple& t) {
  const bool ij = meets(t, 0, 1), jk = meets(t, 1, 2), ik = meets(t, 0, 2);
  const bool connected = (ij && ik) || (ij && jk) || (ik && jk);
  return connected && differ(t, 0, 1) && differ(t, 1, 2) && differ(t, 0, 2);
}

bool open_pattern(const Tuple& t) { return !(meets(t, 0, 1) && meets(t, 1, 2) && meets(t, 0, 2)); }

Tuple emptiness(const Tuple& t) {
  Tuple b;
  for (int r = 0; r < 7; ++r) b[r] = t[r] ? 1 : 0;
  return b;
}

PatternTables build() {
  PatternTables pt{};
  // h-motifs
  std::set<Tuple> bin;
  for (int m = 0; m < 128; ++m) {
    Tuple t;
    for (int r = 0; r < 7; ++r) t[r] = (m >> r) & 1;
    if (valid(t)) bin.insert(canonical(t));
  }
  std::vector<Tuple> hs(bin.begin(), bin.end());
  auto group = [](const Tuple& t) { return open_pattern(t) ? 1 : (t[6] ? 0 : 2); };
  auto nonempty = [](const Tuple& t) { int n = 0; for (auto s : t) n += s != 0; return n; };
  std::sort(hs.begin(), hs.end(), [&](const Tuple& a, const Tuple& b) {
    if (group(a) != group(b)) return group(a) < group(b);
    if (nonempty(a) != nonempty(b)) return nonempty(a) < nonempty(b);
    return a < b;
  });
  std::map<Tuple, int> hid;
  for (size_t n = 0; n < hs.size(); ++n) {
    hid[hs[n]] = int(n) + 1;
    std::copy(hs[n].begin(), hs[n].end(), pt.id26_state[n + 1]);
    pt.id26_open[n + 1] = open_pattern(hs[n]) ? 1 : 0;
  }
  // 3h-motifs
  std::set<std::pair<int, Tuple>> ter;
  for (int c = 0; c < kNumCodes; ++c) {
    Tuple t;
    int x = c;
    for (int r = 0; r < 7; ++r) { t[r] = uint8_t(x % 3); x /= 3; }
    if (!valid(emptiness(t))) continue;
    ter.insert({hid[canonical(emptiness(t))], canonical(t)});
  }
  std::map<Tuple, int> tid;
  int n = 0;
  for (const auto& e : ter) {
    ++n;
    tid[e.second] = n;
    pt.id3_to_id26[n] = int16_t(e.first);
    std::copy(e.second.begin(), e.second.end(), pt.id3_state[n]);
  }
  for (int c = 0; c < kNumCodes; ++c) {
    Tuple t;
    int x = c;
    for (int r = 0; r < 7; ++r) { t[r] = uint8_t(x % 3); x /= 3; }
    pt.code_to_id3[c] = valid(emptiness(t)) ? uint16_t(tid[canonical(t)]) : 0;
  }
  return pt;
}

}  // namespace

const PatternTables& pattern_tables() {
  static const PatternTables pt = build();
  return pt;
}

extern "C" mochy_status mochy_motif_pattern(int32_t id, uint32_t kind, uint8_t states[7]) {
  const PatternTables& pt = pattern_tables();
  if (!states) return MOCHY_EINVAL;
  if (kind == 2 && id >= 1 && id <= MOCHY_NUM_H) {
    std::copy(pt.id26_state[id], pt.id26_state[id] + 7, states);
    return MOCHY_OK;
  }
  if (kind == 3 && id >= 1 && id <= MOCHY_NUM_3H) {
    std::copy(pt.id3_state[id], pt.id3_state[id] + 7, states);
    return MOCHY_OK;
  }
  return MOCHY_EINVAL;
}

extern "C" int32_t mochy_parent_motif(int32_t id3) {
  if (id3 < 1 || id3 > MOCHY_NUM_3H) return 0;
  return pattern_tables().id3_to_id26[id3];
}
