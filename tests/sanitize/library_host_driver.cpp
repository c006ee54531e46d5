// Host-sanitizer driver of the library's host-only pattern code
// (paper_2310_15668_amd/csrc/patterns.cpp), built by
// tests/test_sanitizers_cpu.py with AddressSanitizer and
// UndefinedBehaviorSanitizer: every ternary code and every motif id,
// including the invalid ones, through the tables and the two pattern calls.
#include <cstdio>

#include "common.h"

int main() {
  const PatternTables& t = pattern_tables();
  int ids3 = 0, ids26 = 0;
  bool seen3[kHistSlots] = {}, seen26[27] = {};
  for (int c = 0; c < kNumCodes; ++c) {
    const int id = t.code_to_id3[c];
    if (id < 0 || id >= kHistSlots) return 1;
    if (id && !seen3[id]) { seen3[id] = true; ++ids3; }
  }
  for (int id = 1; id < kHistSlots; ++id) {
    const int h = t.id3_to_id26[id];
    if (h < 1 || h > 26) return 1;
    if (!seen26[h]) { seen26[h] = true; ++ids26; }
    if (mochy_parent_motif(id) != h) return 1;
  }
  uint8_t st[7];
  for (int id = -2; id <= 440; ++id)
    for (uint32_t kind = 1; kind <= 4; ++kind) (void)mochy_motif_pattern(id, kind, st);
  if (mochy_parent_motif(0) != 0 || mochy_parent_motif(432) != 0) return 1;
  std::printf("library tables ok: %d 3h ids, %d h ids\n", ids3, ids26);
  return ids3 == 431 && ids26 == 26 ? 0 : 1;
}
