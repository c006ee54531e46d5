// Internal declarations of the MI355X MoCHy library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "mochy.h"

// Ternary region code used on the device: code = sum_r state(R_r) * 3^r with
// R1 in the least significant digit, state(c) = min(c, 2) (theta = 1).
constexpr int kNumCodes = 2187;
constexpr int kHistSlots = 432;       // slot 0 = invalid pattern, 1..431 = 3h ids
constexpr int kHeavyBits = 64;        // nodes with an exact outside-overlap bit
constexpr int kWave = 64;

// Host-side pattern tables (patterns.cpp).
struct PatternTables {
  uint16_t code_to_id3[kNumCodes];    // any ternary code -> 3h id (0 if invalid)
  int16_t id3_to_id26[kHistSlots];    // 3h id -> h id (slot 0 -> 0)
  uint8_t id26_state[27][7];          // canonical binary tuple of each h id
  uint8_t id3_state[kHistSlots][7];   // canonical ternary tuple of each 3h id
  uint8_t id26_open[27];
};
const PatternTables& pattern_tables();

struct mochy_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool async_alloc = false;           // stream-ordered allocation of graph / scratch buffers
  bool group_neighbours = true;       // exact counting over neighbour groups (MOCHY_OPT_GROUPS)
  bool aplus_rows = false;            // A+ by merging stored rows (MOCHY_OPT_APLUS_ROWS)
  int64_t group_cap_bytes = 0;        // one-pass grouping limit (MOCHY_OPT_GROUP_CAPACITY; half the
                                      // device memory from creation)
  int64_t memo_budget = int64_t(16) << 30;  // key memo arena bytes (MOCHY_OPT_MEMO_BUDGET)
  bool memo_all = false;              // memoize every key that fits (MOCHY_OPT_MEMO_ALL)
  bool memo_pool = false;             // always restrict other-side skips (MOCHY_OPT_MEMO_POOL)
  int batch_launch = 0;               // pair kernel over a batch: 0 size rule, 1 one launch, 2 per graph
  int pair_blocks = 8;                // pair kernel waves per CU / 4 (MOCHY_OPT_PAIR_BLOCKS)
  int test_faults = 0;                // MOCHY_OPT_TEST_FAULTS bits (forced fallbacks)
  // allocation-free calls: device_alloc carves from this device's static
  // scratch array (bump allocation, reset per call; device_free does nothing)
  char* arena = nullptr;              // nullptr: ordinary allocation
  size_t arena_cap = 0, arena_used = 0;
  void* noalloc_scratch = nullptr;    // this device's scratch array (from hipGetSymbolAddress)
  // freed transient buffers of at least kCacheMinBytes kept for reuse on this
  // context's stream (MOCHY_OPT_CACHE_BYTES): size -> block, and the size of
  // every block handed out from or destined for the cache
  int64_t cache_limit = 0;            // bytes (half the device memory from creation)
  int64_t cache_bytes = 0;
  std::multimap<size_t, void*> cache_free;
  std::unordered_map<void*, size_t> cache_live;
  int num_cus = 0;
  std::string err;
  uint16_t* d_code_to_id3 = nullptr;  // [kNumCodes]
  int32_t* d_id3_to_id26 = nullptr;   // [kHistSlots]
  int32_t* d_flags = nullptr;         // device error flags (bit set by validation kernels)
  int64_t* d_small = nullptr;         // [kSmallSlots] small scratch for readbacks
  int64_t* h_small = nullptr;         // [kSmallSlots] pinned host mirror
  int32_t* d_open26 = nullptr;        // [27]: 1 if the h-motif is open
  double* d_dbl = nullptr;            // [512] double outputs
  double* h_dbl = nullptr;            // pinned host mirror
  hipEvent_t ev[2 * MOCHY_NUM_PHASES] = {};
  uint32_t phases_begun = 0;          // phases whose start event was recorded
  uint32_t phases_run = 0;            // phases recorded since the last reset
  double phase_ms[MOCHY_NUM_PHASES] = {};
  // last on-the-fly sampling call: samples, samples counted through key
  // memos, keys memoized, most arena bytes one chunk used, list entries the
  // memo builds walked
  int64_t memo_stats[5] = {};
  // last exact counting call (mochy_exact_stats), summed over its passes
  int64_t exact_stats[MOCHY_NUM_EXACT_STATS] = {};
};

// Layout of ctx->d_small / h_small (int64 slots): 0..63 small outputs,
// 64..495 a histogram of kHistSlots, 500..511 readbacks of single values,
// kExactStatsSlot.. the device counters of mochy_exact_stats.
constexpr int kSmallSlots = 1024;
constexpr int kExactStatsSlot = 512;
enum ExactStat { kStRows = 0, kStGroups, kStGroupsAbove, kStPairsFull, kStPairsOpen, kStRegrouped,
                 kStMaxParts, kStLightPairs, kStFixScanned, kStFixCentres, kStFixChanged, kStBatches };

// Phase timing: bracket device work on the context stream.
enum Phase { kPhUpload = 0, kPhTranspose, kPhDegree, kPhRows, kPhRecords, kPhSched, kPhPairs,
             kPhCorrect, kPhDraw, kPhSample, kPhProfile, kPhFix };
inline void phase_begin(mochy_ctx* c, int p) {
  if (hipEventRecord(c->ev[2 * p], c->stream) == hipSuccess) c->phases_begun |= 1u << p;
}
inline void phase_end(mochy_ctx* c, int p) {
  if (!(c->phases_begun & (1u << p))) return;
  if (hipEventRecord(c->ev[2 * p + 1], c->stream) == hipSuccess) c->phases_run |= 1u << p;
}
// after the stream is synchronized: fold recorded phases into phase_ms
void phases_collect(mochy_ctx* c);

// A graph set: one hypergraph or a batch of them stored as a disjoint union
// (graph g owns hyperedges [geoff[g], geoff[g+1]) and nodes [gvoff[g],
// gvoff[g+1])); every line-graph row stays inside its graph.
struct mochy_graph {
  mochy_ctx* ctx = nullptr;
  int64_t E = 0, V = 0, nnz = 0, W = 0;  // hyperedges, nodes, incidences, hyperwedges (all graphs)
  int32_t max_deg = 0;                   // max line-graph degree
  int32_t ng = 1;                        // graphs in the set
  std::vector<int64_t> h_geoff, h_gvoff, h_gnoff;  // host copies of the offsets
  int64_t max_graph_edges = 0;           // largest graph (sizes the LDS row bitmaps)
  int64_t* geoff = nullptr;              // [ng+1] device
  int64_t* gvoff = nullptr;              // [ng+1] device
  int64_t* gnoff = nullptr;              // [ng+1] device: incidence offsets
  int32_t* row_graph = nullptr;          // [E] graph of each hyperedge
  int64_t* edge_ptr = nullptr;           // [E+1]
  int32_t* edge_nodes = nullptr;         // [nnz]
  int64_t* node_ptr = nullptr;           // [V+1]
  int32_t* node_edges = nullptr;         // [nnz]
  int8_t* heavy_bit = nullptr;           // [V]: bit index for the 64 highest-degree nodes, -1 otherwise
  int64_t* lg_ptr = nullptr;             // [E+1] full line-graph rows
  int32_t* lg_col = nullptr;             // [2W] ascending neighbour ids
  int32_t* up_first = nullptr;           // [E]: position in row i of the first neighbour > i
  int64_t* up_ptr = nullptr;             // [E+1]: prefix sums of upper-row lengths (wedge order)
  uint4* rec = nullptr;                  // [2W]: per (centre, neighbour) region record
  uint32_t* recm = nullptr;              // [2W]: rec[].x alone (the light-pair correction's reads)
  uint16_t* rsz = nullptr;               // [2W]: |e_i ∩ e_x| | |e_x| << 8 of each (centre i, neighbour x)
  // line-graph-free mode (no lg_ptr / lg_col / up_first / rec)
  bool lg_free = false;
  uint32_t* xoff = nullptr;              // [nnz+1]: slot p of E_v -> start of e_k's nodes in xnodes
  int32_t* xnodes = nullptr;             // [xoff[nnz]]: node list of the hyperedge at each slot
  int64_t* deg = nullptr;                // [E]: line-graph degrees
  uint64_t* hmask = nullptr;             // [E]: heavy nodes held by each hyperedge (bit = heavy index)
  // sets of 4 to 6 heavy nodes: open-addressed table (key = set as a mask of
  // heavy indices, 0 = free) of the hyperedges holding the set, by size
  unsigned long long* hbig_key = nullptr;  // [1 << hbig_log2]
  uint32_t* hbig_val = nullptr;            // [1 << hbig_log2][kSizeSlots]
  int hbig_log2 = 0;
  bool memo_ok = false;                  // heavy-set tables complete: key memos allowed
  bool walk_tried = false;               // walk tables built (or found too large) for a graph with rows
  uint32_t* hsize = nullptr;             // [64][kSizeSlots]: hyperedges holding heavy node b, by size
                                         // (slot 0: sizes above kSizeTail)
  uint32_t* hpair = nullptr;             // [64][64][kSizeSlots]: holding heavy nodes b1 and b2, by size
  uint32_t* htriple = nullptr;           // [C(64,3)][kSizeSlots]: holding three heavy nodes, by size
  size_t bytes = 0;                      // device bytes held
};
// Heavy-node tables count hyperedges by size c = 1..32 in slot c; slot 0
// (no hyperedge is empty) holds those of size above kSizeTail, whose classes
// never depend on the exact size where the tables are read with at most three
// nodes taken off (the region keeps at least 6 nodes).
constexpr int kSizeSlots = MOCHY_MAX_EDGE + 1;
constexpr int kSizeTail = 8;

// Per (centre i, neighbour x) record, 16 bytes:
//   x: bit p set iff the p-th node of e_i (ascending) is in e_x
//   y: bits 0..7  = |e_x \ e_i|;  bit 8 = e_x \ e_i holds a node without a heavy bit
//   z,w: 64-bit mask of heavy nodes in e_x \ e_i
constexpr uint32_t kRecLight = 1u << 8;

// Error flag bits (d_flags[0]).
constexpr int kFlagInval = 1, kFlagRange = 2, kFlagDup = 4;

#define MOCHY_HIP(call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
      return MOCHY_EDEVICE;                                                    \
    }                                                                          \
  } while (0)

// The same for code that holds buffers: `handler` (a callable taking and
// returning a mochy_status) releases them and gives the status back.
#define MOCHY_HIP_OR(call, handler)                                            \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
      return handler(MOCHY_EDEVICE);                                           \
    }                                                                          \
  } while (0)

// scan.hip
void launch_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp,
                               hipStream_t s);
size_t scan_tmp_elems(int64_t n);
// Fills `bytes` (a multiple of 4) with a 32-bit pattern by a kernel on the
// stream.  Used instead of hipMemsetAsync on the exact counting path, which
// callers of the allocation-free entry point may record into a HIP graph.
void launch_fill_u32(void* p, uint32_t value, size_t bytes, hipStream_t s);

// project.hip: validation, transpose and heavy nodes (project_incidence),
// then the line graph
mochy_status project_incidence(mochy_ctx* ctx, mochy_graph* g);
mochy_status project_device(mochy_ctx* ctx, mochy_graph* g);

// free.hip: line-graph-free projection and MoCHy-A+ (single graphs)
mochy_status project_free_device(mochy_ctx* ctx, mochy_graph* g);
// per-slot node lists and heavy tables for the on-the-fly sampler (single graphs)
mochy_status build_walk_tables(mochy_ctx* ctx, mochy_graph* g);
mochy_status sampled_free_device(mochy_ctx* ctx, const mochy_graph* g, int64_t r, uint64_t seed,
                                 int64_t n0, int64_t* d_hist);
// memo.hip: key-grouped, memoized enumeration of sampled pairs (per call:
// begin, one chunk at a time, end); a chunk's samples of keys left without a
// memo are returned for the plain enumeration
struct memo_bufs;
mochy_status memo_begin(mochy_ctx* ctx, const mochy_graph* g, int64_t chunk, memo_bufs** out);
mochy_status memo_chunk(mochy_ctx* ctx, const mochy_graph* g, memo_bufs* m, int64_t cnt,
                        const int2* pairs, const int64_t* deg, int64_t* d_hist, int32_t* flags,
                        const int2** left, int64_t* n_left);
void memo_end(mochy_ctx* ctx, memo_bufs* m);
// adds sum_i C(d_i, 2) to d_out[0] and sum_i d_i^2 to d_out[2]
mochy_status free_graph_stats(mochy_ctx* ctx, const mochy_graph* g, unsigned long long* d_out);

// exact.hip: per-graph histograms d_hist[ng][kHistSlots], zeroed inside
mochy_status exact_device(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                          int64_t* d_hist);

// correct.hip: exact fix-up of pairs that share a light node outside the centre
mochy_status correct_device(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                            int64_t* d_hist, unsigned long long* stats);

// sampled.hip: MoCHy-A+ (hyperwedges) and MoCHy-A (hyperedges)
mochy_status sampled_device(mochy_ctx* ctx, const mochy_graph* g, int64_t r, uint64_t seed,
                            int64_t n0, int64_t* d_hist);
mochy_status sampled_edges_device(mochy_ctx* ctx, const mochy_graph* g, int64_t s, uint64_t seed,
                                  int64_t n0, int64_t* d_hist);
// hyperedge profiles of [c0, c1): d_prof[(c1-c0) x kHistSlots], d_prof26[(c1-c0) x 26]
mochy_status profiles_device(mochy_ctx* ctx, const mochy_graph* g, int64_t c0, int64_t c1,
                             int64_t* d_prof, int64_t* d_prof26);

// noalloc.hip: the static scratch array of this device (looked up once per
// device at context creation) and its size
mochy_status noalloc_setup(mochy_ctx* ctx);
extern const size_t kNoallocBytes;

// api.hip helpers: allocation and release ordered on the context stream
mochy_status device_alloc(mochy_ctx* ctx, void** p, size_t bytes);
void device_free(mochy_ctx* ctx, void* p);
void cache_release(mochy_ctx* ctx);  // frees every cached block
constexpr size_t kCacheMinBytes = size_t(64) << 20;

// Largest graph (hyperedges) whose row bitmap and rank table fit in LDS.
constexpr int64_t kMaxGraphEdges = 200000;
