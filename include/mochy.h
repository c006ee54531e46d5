/*
 * mochy.h - C ABI of the MI355X hypergraph-motif counter.
 *
 * Method: MoCHy (Lee, Yoon, Ko, Kim, Shin, "Hypergraph motifs and their
 * extensions beyond binary", arXiv 2310.15668).  A hypergraph goes in; counts
 * of the 26 h-motifs (section 2.2) and 431 3h-motifs (section 5.1, theta = 1),
 * unbiased sampled estimates (MoCHy-A+, Algorithm 5), significance (Eq. 1)
 * and the characteristic profile (Eq. 2) come out.
 *
 * Conventions for every call:
 *  - Return value is a mochy_status; outputs are written only on MOCHY_OK.
 *  - Array arguments marked "host" are ordinary host memory owned by the
 *    caller and never retained past the call.
 *  - All device work is enqueued on the context's HIP stream; every call is
 *    synchronous on return (results are on the host, device work finished).
 *  - A context is not thread-safe: one host thread at a time per context.
 *  - Motif ids: h-motifs 1..26, 3h-motifs 1..431; count arrays are indexed
 *    id-1.  mochy_motif_pattern() gives the region pattern behind every id.
 *    Ids 17..22 are the open h-motifs, the others closed.
 *  - Hyperedge ids are positions in the input CSR.
 */
#ifndef MOCHY_H
#define MOCHY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MOCHY_OK = 0,
  MOCHY_EINVAL = -1,      /* malformed input: a node list not strictly ascending,
                             a node id outside [0, num_nodes), an empty hyperedge,
                             decreasing edge_ptr, or a bad argument */
  MOCHY_EDUP = -2,        /* two hyperedges hold the same node set (hyperedges form a
                             set, section 2.1); pass MOCHY_DEDUP to drop repeats */
  MOCHY_ERANGE = -3,      /* a hyperedge holds more than MOCHY_MAX_EDGE nodes, or a
                             size exceeds what the library can address */
  MOCHY_ENOMEM = -4,      /* device or host allocation failed */
  MOCHY_EDEVICE = -5,     /* a HIP runtime call failed */
  MOCHY_EUNSUPPORTED = -6 /* valid request the library does not handle (message says why) */
} mochy_status;

/* Nodes per hyperedge.  Section 2.1 allows any non-empty node set; this
 * library keeps one 32-bit mask of a centre's nodes per line-graph neighbour
 * (16-byte region records), so it accepts hyperedges of at most 32 nodes and
 * answers MOCHY_ERANGE above that.  A stated deviation: the paper's datasets
 * have at most 25 nodes per hyperedge (Table 2), and a 64-bit mask would
 * widen every record and every per-pair mask operation of the hot kernels. */
#define MOCHY_MAX_EDGE 32
#define MOCHY_NUM_H 26
#define MOCHY_NUM_3H 431

/* `which` selector of the counting calls: the h-motif outputs (26 classes,
 * section 2.2), the 3h-motif outputs (431 classes, section 5.1), or both.
 * The device always classifies a triple into its 3h-motif (its h-motif is
 * that 3h-motif's parent), so `which` selects outputs, not work.  Outputs of
 * a kind not selected are never written; an output of a selected kind may be
 * NULL if it is not wanted.  MOCHY_EINVAL if `which` is 0 or has other bits. */
#define MOCHY_H26 1u
#define MOCHY_H431 2u
#define MOCHY_WHICH_ALL (MOCHY_H26 | MOCHY_H431)

typedef struct mochy_ctx mochy_ctx;      /* device, stream, pattern tables, error text */
typedef struct mochy_graph mochy_graph;  /* device-resident incidence, its transpose and
                                            the line graph; owned by the library */

/* CSR incidence of a hypergraph: hyperedge e holds the node ids
 * edge_nodes[edge_ptr[e] .. edge_ptr[e+1]-1], strictly ascending.
 * edge_ptr has num_edges+1 int64 entries starting at 0.
 * on_device = 0: host pointers; 1: device pointers (memory already in HBM of
 * the context's device; read during mochy_project only, never retained). */
typedef struct {
  int64_t num_nodes;
  int64_t num_edges;
  const int64_t* edge_ptr;
  const int32_t* edge_nodes;
  int32_t on_device;
} mochy_csr;

/* mochy_project flags */
#define MOCHY_DEDUP 1u    /* host input only: drop repeated hyperedges, keeping the first;
                             later ids shift down */
#define MOCHY_CANONICALIZE 2u  /* host input only: sort each hyperedge's node list and
                                  drop repeated nodes (a hyperedge is a node set,
                                  section 2.1) before validation; a list that still
                                  holds more than MOCHY_MAX_EDGE nodes is MOCHY_ERANGE */
#define MOCHY_LG_FREE 4u  /* do not store the line graph (section 4.4's on-the-fly
                             neighbourhoods); implied above 200000 hyperedges */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to use,
 * or NULL to create a private one (default priority).  Builds the pattern
 * tables on the device. */
mochy_status mochy_ctx_create(int device, void* hip_stream, mochy_ctx** out);
void mochy_ctx_destroy(mochy_ctx* ctx);
/* Text of the last error on this context ("" if none); owned by the context. */
const char* mochy_last_error(const mochy_ctx* ctx);

/* Options of a context; they change how results are computed, never the
 * results.  MOCHY_EINVAL for an unknown option or value. */
#define MOCHY_OPT_GROUPS 1  /* exact counting pairs groups of neighbours with equal region
                               records, weighted by their sizes (1, default), or every
                               pair of neighbours (0); with too little device memory
                               for the groups it pairs every neighbour */
#define MOCHY_OPT_APLUS_ROWS 2  /* MoCHy-A+ on a graph with a stored line graph: enumerate
                                   N_i ∪ N_j on the fly from the node lists (0, default) or
                                   by merging the two stored rows (1); same hits */
#define MOCHY_OPT_GROUP_CAPACITY 6  /* exact counting (of a graph, or of a whole batch in
                                       mochy_profile) groups each row's neighbours in one
                                       pass into space for all of its records when that
                                       takes at most this many bytes (24 per record; default
                                       half the device memory) and can be allocated, else
                                       counts the groups first and allocates them exactly;
                                       0 = always count first; same counts */
#define MOCHY_OPT_MEMO_BUDGET 3  /* on-the-fly MoCHy-A+ groups its samples by key hyperedge
                                    (the endpoint of larger line-graph degree, Algorithm 9)
                                    and memoizes the neighbourhood counts of keys, in
                                    descending degree order, in a device arena of this many
                                    bytes per call (default 16 GiB; 0 = no memoization, every
                                    sample enumerated on its own); same hits */
#define MOCHY_OPT_MEMO_ALL 4  /* 1: memoize every key that fits the budget; 0 (default):
                                 only keys with at least 4 samples in a chunk; same hits */
#define MOCHY_OPT_MEMO_POOL 5  /* heavy nodes a key's samples skip on their other side:
                                  any (0, default; the 16 with the most list entries
                                  if the key would need too many node sets) or always
                                  those 16 (1); same hits */
#define MOCHY_OPT_BATCH_LAUNCH 7  /* exact counting of a batch (mochy_profile) launches the
                                     group-pair kernel once for the whole batch (1), once
                                     per graph (2; batches of at most 256 graphs, larger
                                     ones take one launch), or per graph when the graphs
                                     average a full grid of work items each (0, default);
                                     same counts */
#define MOCHY_OPT_PAIR_BLOCKS 8  /* waves of the exact pair kernel launched per compute
                                    unit, in fours, 1..16 (default 8: 32 waves, as blocks
                                    of 256 threads, or half as many blocks of 512 where
                                    one histogram serves a whole graph; a launch per graph
                                    takes at most one wave per work item); same counts */
#define MOCHY_OPT_CACHE_BYTES 9  /* device buffers of 64 MiB or more that a call frees are
                                    kept by the context, up to this many bytes in all, and
                                    reused by later calls on it (default half of the
                                    device memory; 0 = free at once, releasing what is
                                    kept); an allocation that fails first releases them
                                    (this context's only: several contexts on one device
                                    should share the memory by their limits);
                                    mochy_ctx_destroy frees them; same results */
#define MOCHY_OPT_TEST_FAULTS 10  /* for tests of the fallbacks: bit 0 makes the one-pass
                                     grouping's row-capacity allocation report
                                     MOCHY_ENOMEM, so exact counting takes the
                                     counted-first layout; bit 1 caps the scratch of
                                     mochy_count_exact_range_noalloc at 64 KiB; bit 2
                                     makes the grouping of a batch of more than two
                                     graphs report MOCHY_ENOMEM, so mochy_profile splits
                                     it; bit 3 leaves out the light-pair correction's
                                     flat candidate list, so its pairs are listed in a
                                     counting and a filling pass; bit 4 makes the pair
                                     kernel form 48-bit pair weights from unpacked group
                                     counts, as for graphs whose line-graph degree
                                     reaches 2^16 (default 0);
                                     same counts */
mochy_status mochy_ctx_set_option(mochy_ctx* ctx, int32_t option, int64_t value);

/* Line-graph construction (Algorithm 1, section 4.1).  Validates the CSR,
 * builds on the device the transposed incidence E_v (node -> hyperedges),
 * the full line graph rows N_{e_i} (ascending hyperedge ids) with
 * omega(e_i, e_j) = |e_i ∩ e_j| folded into per-neighbour region masks, and
 * returns it.  *num_hyperwedges = |wedges| = number of adjacent unordered
 * pairs.
 * Line-graph-free mode (flag MOCHY_LG_FREE, and always for more than 200000
 * hyperedges): no rows are stored; the graph keeps E_v, a copy of each
 * neighbour's node list per slot of E_v (sum of |e|^2 node ids, which must
 * stay below 2^32, else MOCHY_ERANGE), the line-graph degrees and the
 * hyperwedge order, and serves mochy_count_sampled (neighbourhoods formed on
 * demand, section 4.4); mochy_count_exact then returns MOCHY_EUNSUPPORTED.
 * Errors: MOCHY_EINVAL, MOCHY_EDUP, MOCHY_ERANGE, MOCHY_ENOMEM,
 * MOCHY_EDEVICE.  Free the result with mochy_graph_free. */
mochy_status mochy_project(mochy_ctx* ctx, const mochy_csr* g, uint32_t flags,
                           mochy_graph** out, int64_t* num_hyperwedges);
void mochy_graph_free(mochy_graph* g);

/* Exact counts (MoCHy-E, Algorithm 2): every connected triple of distinct
 * hyperedges counted once in its h-motif and its 3h-motif.  which: MOCHY_H26,
 * MOCHY_H431 or both; counts26 (host, 26 int64) and counts431 (host, 431
 * int64) receive the selected kinds (each may be NULL if not wanted).
 * Errors: MOCHY_EINVAL (bad graph or which), MOCHY_EUNSUPPORTED (graph
 * projected without its line graph), MOCHY_ENOMEM, MOCHY_EDEVICE. */
mochy_status mochy_count_exact(mochy_ctx* ctx, const mochy_graph* g, uint32_t which,
                               int64_t* counts26, int64_t* counts431);

/* The same, restricted to the instances Algorithm 2 attributes to centres
 * e_i with center_begin <= i < center_end (an open instance belongs to its
 * middle hyperedge, a closed one to its smallest index).  Summing disjoint
 * ranges that cover [0, num_edges) gives mochy_count_exact. */
mochy_status mochy_count_exact_range(mochy_ctx* ctx, const mochy_graph* g,
                                     int64_t center_begin, int64_t center_end, uint32_t which,
                                     int64_t* counts26, int64_t* counts431);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * counts as mochy_count_exact_range (same arguments, same results), computed
 * without any device or host allocation.  Every neighbour pair of a centre
 * is classified (no neighbour groups, which would need memory in proportion
 * to the line graph), and the work-item schedule and the correction's
 * light-pair lists live in a static device array of MOCHY_NOALLOC_SCRATCH
 * bytes that each device the library runs on holds from the first context
 * created on it until the process ends.  The graph, the context and the
 * outputs are the caller's, as in mochy_count_exact_range.
 * MOCHY_ERANGE (with the sizes in the message) if a call would need more
 * scratch than that; the work it needs grows with |E|, the largest
 * line-graph degree and the pairs of hyperedges that share a light node
 * (about 40 MiB for the medium workload of 85,476 hyperedges).
 * All calls on one device share its scratch array, whose contents persist
 * from call to call (each call initializes what it reads); calls that
 * overlap in time on one device, from any contexts or threads, race on it
 * and must not be issued.  Slower than mochy_count_exact_range on large
 * rows (every pair instead of pairs of groups). */
#define MOCHY_NOALLOC_SCRATCH (64u << 20)
mochy_status mochy_count_exact_range_noalloc(mochy_ctx* ctx, const mochy_graph* g,
                                             int64_t center_begin, int64_t center_end,
                                             uint32_t which, int64_t* counts26,
                                             int64_t* counts431);

/* MoCHy-A+ (Algorithm 5): samples n = sample_begin .. sample_begin+r-1 each
 * draw one hyperwedge uniformly with replacement, using Philox4x32-10 with
 * counter (lo32 n, hi32 n, 0, 0), key (lo32 seed, hi32 seed),
 * u = (x1 << 32) | x0 and hyperwedge index floor(u * |wedges| / 2^64) in the
 * order of (i, j), i < j, lexicographic.  For the sampled {e_i, e_j}, each
 * e_k in N_i ∪ N_j minus {e_i, e_j} adds one hit to its motif.  raw26/raw431
 * (host int64) receive the hits; est26/est431 (host double) the unbiased
 * estimates raw * |wedges| / (w * r), w = 2 for open and 3 for closed motifs
 * (w of a 3h-motif is its h-motif's).  which selects the kinds written
 * (raw26/est26 are MOCHY_H26, raw431/est431 MOCHY_H431); any output pointer
 * of a selected kind may be NULL.  r must be > 0; a graph with no hyperwedge
 * gives zeros. */
mochy_status mochy_count_sampled(mochy_ctx* ctx, const mochy_graph* g, int64_t r,
                                 uint64_t seed, int64_t sample_begin, uint32_t which,
                                 int64_t* raw26, double* est26,
                                 int64_t* raw431, double* est431);

/* MoCHy-A (Algorithm 4): samples n = sample_begin .. sample_begin+s-1 each
 * draw one hyperedge uniformly with replacement, using Philox4x32-10 with
 * counter (lo32 n, hi32 n, 1, 0), key (lo32 seed, hi32 seed),
 * u = (x1 << 32) | x0 and hyperedge index floor(u * |E| / 2^64).  Every
 * instance that contains the sampled hyperedge adds one hit to its motif
 * (found from its 1-hop and 2-hop neighbourhoods).  raw26/raw431 (host int64)
 * receive the hits; est26/est431 (host double) the unbiased estimates
 * raw * |E| / (3 s).  Any output pointer may be NULL; s must be > 0.
 * Needs the stored line graph: MOCHY_EUNSUPPORTED for a graph projected
 * line-graph-free. */
mochy_status mochy_count_sampled_edges(mochy_ctx* ctx, const mochy_graph* g, int64_t s,
                                       uint64_t seed, int64_t sample_begin,
                                       int64_t* raw26, double* est26,
                                       int64_t* raw431, double* est431);

/* Hyperedge profiles (section 3.2): for each hyperedge e with
 * e_begin <= e < e_end, the number of instances of every h-motif (hp26, host,
 * (e_end-e_begin) x 26 int64, row-major) and 3h-motif (hp431, host,
 * (e_end-e_begin) x 431 int64) that contain e; either may be NULL.  Summed
 * over all hyperedges, each motif's profile column is 3 times its count.
 * Work per hyperedge: its 1-hop and 2-hop neighbourhoods (sum over its
 * neighbours e_j of |N_j|), as one MoCHy-A sample.  Needs the stored line
 * graph (MOCHY_EUNSUPPORTED otherwise). */
mochy_status mochy_hyperedge_profiles(mochy_ctx* ctx, const mochy_graph* g, int64_t e_begin,
                                      int64_t e_end, int64_t* hp26, int64_t* hp431);

/* Significance and characteristic profile against randomized copies
 * (section 3.1).  graphs[0] is the hypergraph, graphs[1..num_graphs-1] its
 * randomized copies (host or device CSRs, each of at most 200000
 * hyperedges).  All graphs are projected and counted exactly on the device,
 * as one batch.  Outputs (host): counts (num_graphs x 457 int64: per graph
 * 26 h-motif then 431 3h-motif counts; the columns of a kind not selected by
 * `which` are left untouched), sig26/cp26 (26 doubles, MOCHY_H26) and
 * sig431/cp431 (431 doubles, MOCHY_H431), each may be NULL.
 *   Delta_t = (M[t] - Mr[t]) / (M[t] + Mr[t] + eps),  Mr = mean over copies;
 *   CP_t    = Delta_t / sqrt(sum_t Delta_t^2)    (0 for all t if every Delta is 0).
 * num_graphs >= 2.
 * Deviation from a (num_random, seeds) signature: the caller draws the
 * copies and passes them in, so the null model (stub matching with exact
 * degrees and sizes, or the paper's Chung-Lu randomizer of Algorithms 6-7)
 * stays the caller's choice and its random numbers stay outside the library. */
mochy_status mochy_profile(mochy_ctx* ctx, int32_t num_graphs, const mochy_csr* graphs,
                           double eps, uint32_t which, int64_t* counts,
                           double* sig26, double* cp26, double* sig431, double* cp431);

/* Region pattern of a motif id: states[r] for regions R1..R7 of section 2.2
 * (R1 = e_i - e_j - e_k, ..., R4 = e_i ∩ e_j - e_k, ..., R7 = all three), in
 * the canonical labelling.  kind = 2: h-motif (0 empty / 1 non-empty);
 * kind = 3: 3h-motif (0 empty, 1 one node, 2 more).  MOCHY_EINVAL for an id
 * out of range.  Host only, needs no context. */
mochy_status mochy_motif_pattern(int32_t id, uint32_t kind, uint8_t states[7]);

/* Parent h-motif id of a 3h-motif id (1..431), or 0 if out of range. */
int32_t mochy_parent_motif(int32_t id3);

/* Workload statistics of a projected graph, computed on the device:
 * out[0] |E|, out[1] |V|, out[2] sum |e|, out[3] |wedges|, out[4] max
 * line-graph degree, out[5] MoCHy-E candidates sum_i C(d_i, 2) (pairs
 * Algorithm 2 considers), out[6] sum over those candidates of
 * min(|e_i|, |e_j|, |e_k|) (the size factor of Lemma 2's triple
 * intersection; -1 for a line-graph-free graph), out[7] sum_i d_i^2.
 * out: host, 8 int64. */
mochy_status mochy_graph_stats(mochy_ctx* ctx, const mochy_graph* g, int64_t* out);

/* Milliseconds spent in each device phase by the most recent call on this
 * context, from HIP events recorded on the context stream (0 for phases the
 * call did not run).  Phases: 0 upload+validate, 1 transpose + heavy-node
 * pick, 2 line-graph degrees, 3 line-graph rows (line-graph-free mode, and
 * a stored-row graph's first on-the-fly sampling call: the per-slot node
 * lists and heavy-node tables), 4 region records,
 * 5 exact scheduling, 6 exact pair kernel, 7 exact light-node correction,
 * 8 sampling draws (line-graph-free mode: with grouping by row and the pick
 * of e_j), 9 sampled enumeration, 10 profile significance + CP, 11 the
 * light-pair fix kernel alone (part of phase 7).
 * ms: host, MOCHY_NUM_PHASES doubles. */
#define MOCHY_NUM_PHASES 12
mochy_status mochy_phase_ms(const mochy_ctx* ctx, double* ms);

/* What the most recent exact counting call (mochy_count_exact, _range, or
 * the exact counts of mochy_profile) did, summed over its graphs:
 * out[0] rows grouped, out[1] neighbour groups, out[2] groups with a member
 * above the centre, out[3] pairs of groups that both have a member above the
 * centre (classified in full), out[4] other pairs of groups (counted only
 * when open), out[5] rows regrouped with more hash parts than first
 * guessed, out[6] most hash parts of one row, out[7] hyperedge pairs sharing
 * a light node (the correction's pairs), out[8] row entries the correction
 * scanned, out[9] common neighbours it examined (centres of a light pair),
 * out[10] of those, the centres whose class it changed, out[11] the
 * sub-batches a mochy_profile call counted its graphs in (a batch that does
 * not fit in device memory is split).  Zeros for parts a call did not run
 * (out[0..6] when every neighbour was paired).
 * out: host, MOCHY_NUM_EXACT_STATS int64. */
#define MOCHY_NUM_EXACT_STATS 12
mochy_status mochy_exact_stats(const mochy_ctx* ctx, int64_t* out);

/* Measurement helper (not part of the method): the integer vector-ALU rate
 * the device sustains.  One timed launch of 32 waves per compute unit, every
 * lane running `iters` rounds of 32 integer vector instructions in the
 * proportions the exact pair kernel issues them (AND, add, saturating and
 * packed 16-bit saturating subtract, population count, two-term 16-bit dot
 * product, select, AND-OR, shift-or, shift-add, 24-bit multiply-add) over
 * independent chains.  *ms (host) receives the launch's duration from HIP
 * events on the context stream, *lane_ops (host) the lane instructions it
 * executed (threads x iters x 32).
 * iters in [1, 2^32], else MOCHY_EINVAL. */
mochy_status mochy_calibrate_valu(mochy_ctx* ctx, int64_t iters, double* ms, int64_t* lane_ops);

/* What the key memos of the most recent on-the-fly MoCHy-A+ call did
 * (Algorithm 9 with a memo budget, MOCHY_OPT_MEMO_BUDGET): out[0] samples,
 * out[1] samples counted through a key memo (the rest were enumerated on
 * their own), out[2] keys memoized (summed over chunks), out[3] most arena
 * bytes used by one chunk, out[4] list entries E_v walked to build the memos.
 * Zeros after calls that sampled nothing on the fly.  out: host, 5 int64. */
mochy_status mochy_memo_stats(const mochy_ctx* ctx, int64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* MOCHY_H */
