// C ABI of the library (declared in include/mochy.h).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "common.h"

namespace {

// 26 h-motif counts folded from the 431 3h-motif counts (every 3h-motif
// refines exactly one h-motif, section 5.1).
__global__ void k_fold(const int64_t* __restrict__ hist, const int32_t* __restrict__ parent,
                       int64_t* out26) {
  const int h = threadIdx.x;
  if (h >= MOCHY_NUM_H) return;
  int64_t s = 0;
  for (int id3 = 1; id3 < kHistSlots; ++id3)
    if (parent[id3] == h + 1) s += hist[id3];
  out26[h] = s;
}

// Algorithm 5's rescaling in float64: est = raw * |wedges| / (w * r), w = 2
// for open and 3 for closed motifs (a 3h-motif takes its h-motif's w).
__global__ void k_aplus_est(const int64_t* __restrict__ hist, const int32_t* __restrict__ parent,
                            const int32_t* __restrict__ open26, int64_t W, int64_t r,
                            int64_t* raw26, double* est26, double* est431) {
  const int t = threadIdx.x;
  if (t >= 1 && t < kHistSlots) {
    const double w = open26[parent[t]] ? 2.0 : 3.0;
    est431[t - 1] = (double(hist[t]) * double(W)) / (w * double(r));
  }
  if (t < MOCHY_NUM_H) {
    int64_t s = 0;
    for (int id3 = 1; id3 < kHistSlots; ++id3)
      if (parent[id3] == t + 1) s += hist[id3];
    raw26[t] = s;
    const double w = open26[t + 1] ? 2.0 : 3.0;
    est26[t] = (double(s) * double(W)) / (w * double(r));
  }
}

// Algorithm 4's rescaling in float64: est = raw * |E| / (3 s).
__global__ void k_hsample_est(const int64_t* __restrict__ hist, const int32_t* __restrict__ parent,
                              int64_t E, int64_t s, int64_t* raw26, double* est26, double* est431) {
  const int t = threadIdx.x;
  if (t >= 1 && t < kHistSlots) est431[t - 1] = (double(hist[t]) * double(E)) / (3.0 * double(s));
  if (t < MOCHY_NUM_H) {
    int64_t sum = 0;
    for (int id3 = 1; id3 < kHistSlots; ++id3)
      if (parent[id3] == t + 1) sum += hist[id3];
    raw26[t] = sum;
    est26[t] = (double(sum) * double(E)) / (3.0 * double(s));
  }
}

// Significance and characteristic profile (Eq. 1, Eq. 2) of graph 0 against
// graphs 1..ng-1, in float64.  counts[g][t] for the 26 h-motifs (folded from
// the 3h-motifs) and the 431 3h-motifs; Mr = (sum over copies, exact in
// int64) / R; Delta = (M - Mr) / (M + Mr + eps); CP = Delta / sqrt(sum of
// Delta^2 in order t = 1, 2, ...), all zeros if every Delta is 0.  The sum of
// squares is formed with separately rounded multiplies and adds.
__global__ void k_profile(const int64_t* __restrict__ hist, const int32_t* __restrict__ parent,
                          int32_t ng, double eps, int64_t* counts, double* sig26, double* cp26,
                          double* sig431, double* cp431) {
  __shared__ double d26[MOCHY_NUM_H];
  __shared__ double d431[MOCHY_NUM_3H];
  const int t = threadIdx.x;
  for (int g = 0; g < ng; ++g) {
    const int64_t* hg = hist + int64_t(g) * kHistSlots;
    int64_t* cg = counts + int64_t(g) * (MOCHY_NUM_H + MOCHY_NUM_3H);
    if (t < MOCHY_NUM_H) {
      int64_t s = 0;
      for (int id3 = 1; id3 < kHistSlots; ++id3)
        if (parent[id3] == t + 1) s += hg[id3];
      cg[t] = s;
    }
    if (t < MOCHY_NUM_3H) cg[MOCHY_NUM_H + t] = hg[t + 1];
  }
  __syncthreads();
  const int R = ng - 1;
  for (int x = t; x < MOCHY_NUM_H + MOCHY_NUM_3H; x += blockDim.x) {
    int64_t sum = 0;
    for (int g = 1; g < ng; ++g) sum += counts[int64_t(g) * (MOCHY_NUM_H + MOCHY_NUM_3H) + x];
    const double mr = double(sum) / double(R);
    const double m = double(counts[x]);
    const double d = __ddiv_rn(__dsub_rn(m, mr), __dadd_rn(__dadd_rn(m, mr), eps));
    if (x < MOCHY_NUM_H) d26[x] = d; else d431[x - MOCHY_NUM_H] = d;
  }
  __syncthreads();
  if (t == 0 || t == 1) {
    const int n = t == 0 ? MOCHY_NUM_H : MOCHY_NUM_3H;
    double* d = t == 0 ? d26 : d431;
    double* sig = t == 0 ? sig26 : sig431;
    double* cp = t == 0 ? cp26 : cp431;
    double s = 0.0;
    for (int x = 0; x < n; ++x) s = __dadd_rn(s, __dmul_rn(d[x], d[x]));
    const double norm = __dsqrt_rn(s);
    for (int x = 0; x < n; ++x) {
      sig[x] = d[x];
      cp[x] = s == 0.0 ? 0.0 : __ddiv_rn(d[x], norm);
    }
  }
}

// Adds the per-graph edge and node offsets to one graph's slice of the union.
__global__ void k_union_offsets(int64_t e_begin, int64_t e_count, int64_t nnz_off, int64_t* edge_ptr,
                                int64_t n_begin, int64_t n_count, int32_t node_off,
                                int32_t* edge_nodes) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x < e_count) edge_ptr[e_begin + x] += nnz_off;
  if (x < n_count) edge_nodes[n_begin + x] += node_off;
}

struct RowHash {
  const int64_t* ptr;
  const int32_t* nodes;
  size_t operator()(int64_t e) const {
    size_t h = 1469598103934665603ull;
    for (int64_t q = ptr[e]; q < ptr[e + 1]; ++q) h = (h ^ size_t(uint32_t(nodes[q]))) * 1099511628211ull;
    return h;
  }
};
struct RowEq {
  const int64_t* ptr;
  const int32_t* nodes;
  bool operator()(int64_t a, int64_t b) const {
    const int64_t la = ptr[a + 1] - ptr[a], lb = ptr[b + 1] - ptr[b];
    return la == lb && std::equal(nodes + ptr[a], nodes + ptr[a + 1], nodes + ptr[b]);
  }
};

mochy_status check_host_csr(mochy_ctx* ctx, const mochy_csr* c) {
  if (c->num_edges > 0 && (!c->edge_ptr || (c->edge_ptr[c->num_edges] > 0 && !c->edge_nodes))) {
    ctx->err = "null CSR pointer";
    return MOCHY_EINVAL;
  }
  if (c->edge_ptr && c->edge_ptr[0] != 0) { ctx->err = "edge_ptr[0] must be 0"; return MOCHY_EINVAL; }
  for (int64_t e = 0; e < c->num_edges; ++e) {
    const int64_t s = c->edge_ptr[e], t = c->edge_ptr[e + 1];
    if (t <= s) { ctx->err = "empty hyperedge or decreasing edge_ptr at edge " + std::to_string(e); return MOCHY_EINVAL; }
    if (t - s > MOCHY_MAX_EDGE) { ctx->err = "hyperedge " + std::to_string(e) + " exceeds MOCHY_MAX_EDGE"; return MOCHY_ERANGE; }
    for (int64_t q = s; q < t; ++q) {
      const int32_t v = c->edge_nodes[q];
      if (v < 0 || v >= c->num_nodes || (q > s && c->edge_nodes[q - 1] >= v)) {
        ctx->err = "node list of hyperedge " + std::to_string(e) + " not strictly ascending in [0, num_nodes)";
        return MOCHY_EINVAL;
      }
    }
  }
  return MOCHY_OK;
}

// Per-row workload statistics from the region records: candidates C(d,2),
// the sum over candidate pairs of min(|e_i|, |e_j|, |e_k|), and d^2.
__global__ __launch_bounds__(256) void k_stats(const int64_t* __restrict__ edge_ptr,
                                               const int64_t* __restrict__ lg_ptr,
                                               const uint4* __restrict__ rec,
                                               unsigned long long* out) {
  __shared__ unsigned int cnt[MOCHY_MAX_EDGE + 2];
  const int64_t i = blockIdx.x;
  if (threadIdx.x < MOCHY_MAX_EDGE + 2) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = lg_ptr[i], d = lg_ptr[i + 1] - base;
  for (int64_t p = threadIdx.x; p < d; p += blockDim.x) {
    const uint4 r = rec[base + p];
    atomicAdd(&cnt[__popc(r.x) + (r.y & 0xffu)], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long a = (unsigned long long)(edge_ptr[i + 1] - edge_ptr[i]);
    unsigned long long ge = 0, sum = 0;  // ge = neighbours of size >= s
    for (int s = MOCHY_MAX_EDGE; s >= 1; --s) {
      const unsigned long long gt = ge;
      ge += cnt[s];
      const unsigned long long pairs_min_s = ge * (ge - (ge ? 1 : 0)) / 2 - gt * (gt - (gt ? 1 : 0)) / 2;
      sum += pairs_min_s * (a < (unsigned long long)s ? a : (unsigned long long)s);
    }
    const unsigned long long dd = (unsigned long long)d;
    atomicAdd(&out[0], dd * (dd - (dd ? 1 : 0)) / 2);
    atomicAdd(&out[1], sum);
    atomicAdd(&out[2], dd * dd);
  }
}

}  // namespace

void phases_collect(mochy_ctx* c) {
  for (int p = 0; p < MOCHY_NUM_PHASES; ++p) {
    if (!(c->phases_run & (1u << p))) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[2 * p], c->ev[2 * p + 1]) == hipSuccess) c->phase_ms[p] += ms;
    else (void)hipGetLastError();  // a timing query never fails the computation
  }
  c->phases_run = 0;
  c->phases_begun = 0;
}

static void phases_reset(mochy_ctx* c) {
  c->phases_run = 0;
  c->phases_begun = 0;
  for (double& m : c->phase_ms) m = 0.0;
  for (int64_t& m : c->memo_stats) m = 0;
}

extern "C" mochy_status mochy_phase_ms(const mochy_ctx* ctx, double* ms) {
  if (!ctx || !ms) return MOCHY_EINVAL;
  std::memcpy(ms, ctx->phase_ms, sizeof(ctx->phase_ms));
  return MOCHY_OK;
}

extern "C" mochy_status mochy_exact_stats(const mochy_ctx* ctx, int64_t* out) {
  if (!ctx || !out) return MOCHY_EINVAL;
  std::memcpy(out, ctx->exact_stats, sizeof(ctx->exact_stats));
  return MOCHY_OK;
}

extern "C" mochy_status mochy_memo_stats(const mochy_ctx* ctx, int64_t* out) {
  if (!ctx || !out) return MOCHY_EINVAL;
  std::memcpy(out, ctx->memo_stats, sizeof(ctx->memo_stats));
  return MOCHY_OK;
}

// Graph and scratch buffers are stream-ordered allocations on the context's
// stream when the device has memory pools, so that a free never waits for
// work queued by other contexts on other streams.
static hipError_t raw_alloc(mochy_ctx* ctx, void** p, size_t n) {
  return ctx->async_alloc ? hipMallocAsync(p, n, ctx->stream) : hipMalloc(p, n);
}

static void raw_free(mochy_ctx* ctx, void* p) {
  if (ctx->async_alloc) (void)hipFreeAsync(p, ctx->stream);
  else (void)hipFree(p);
}

void cache_release(mochy_ctx* ctx) {
  for (auto& kv : ctx->cache_free) {
    ctx->cache_live.erase(kv.second);
    raw_free(ctx, kv.second);
  }
  ctx->cache_free.clear();
  ctx->cache_bytes = 0;
}

// Buffers of at least kCacheMinBytes go through a per-context cache: a freed
// block is kept (up to cache_limit bytes in all) and handed to a later
// request that it fits with at most half of it unused.  Freeing and mapping
// again the hundred-odd GB that a batch of 65 graphs holds costs up to
// seconds per call; reusing the blocks costs nothing.  A context works on one
// stream, so a reused block's earlier readers are ordered before its new
// writers.
mochy_status device_alloc(mochy_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  size_t n = std::max<size_t>(bytes, 8);
  if (ctx->arena) {  // allocation-free call: carve from the static scratch array
    const size_t at = (ctx->arena_used + 255) & ~size_t(255);
    if (at + n > ctx->arena_cap) {
      ctx->err = "the allocation-free call needs more than its " + std::to_string(ctx->arena_cap) +
                 "-byte scratch array (" + std::to_string(at + n) + " bytes so far)";
      return MOCHY_ERANGE;
    }
    *p = ctx->arena + at;
    ctx->arena_used = at + n;
    return MOCHY_OK;
  }
  const bool cached = ctx->cache_limit > 0 && n >= kCacheMinBytes;
  if (cached) {
    auto it = ctx->cache_free.lower_bound(n);
    if (it != ctx->cache_free.end() && it->first / 2 <= n) {
      *p = it->second;
      ctx->cache_bytes -= int64_t(it->first);
      ctx->cache_free.erase(it);
      return MOCHY_OK;
    }
    n = (n + (size_t(2) << 20) - 1) & ~((size_t(2) << 20) - 1);  // whole 2 MiB pages
  }
  hipError_t e = raw_alloc(ctx, p, n);
  if (e != hipSuccess && !ctx->cache_free.empty()) {  // give the cached blocks back and retry
    (void)hipGetLastError();
    cache_release(ctx);
    (void)hipStreamSynchronize(ctx->stream);
    e = raw_alloc(ctx, p, n);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    ctx->err = "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
    return MOCHY_ENOMEM;
  }
  if (cached) ctx->cache_live[*p] = n;
  return MOCHY_OK;
}

void device_free(mochy_ctx* ctx, void* p) {
  if (!p || ctx->arena) return;  // arena blocks are released with the call
  auto it = ctx->cache_live.find(p);
  if (it != ctx->cache_live.end() && ctx->cache_bytes + int64_t(it->second) <= ctx->cache_limit) {
    ctx->cache_free.emplace(it->second, p);  // stays in cache_live until released
    ctx->cache_bytes += int64_t(it->second);
    return;
  }
  if (it != ctx->cache_live.end()) ctx->cache_live.erase(it);
  raw_free(ctx, p);
}

// Buffers that live as long as the context.
static mochy_status ctx_alloc(mochy_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  if (hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    ctx->err = "device allocation failed";
    return MOCHY_ENOMEM;
  }
  return MOCHY_OK;
}

extern "C" mochy_status mochy_ctx_create(int device, void* hip_stream, mochy_ctx** out) {
  if (!out) return MOCHY_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return MOCHY_EDEVICE;
  if (device < 0 || device >= n) return MOCHY_EINVAL;
  mochy_ctx* ctx = new (std::nothrow) mochy_ctx();
  if (!ctx) return MOCHY_ENOMEM;
  ctx->device = device;
  auto fail = [&](mochy_status s) { mochy_ctx_destroy(ctx); return s; };
  if (hipSetDevice(device) != hipSuccess) return fail(MOCHY_EDEVICE);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(MOCHY_EDEVICE);
  ctx->num_cus = prop.multiProcessorCount;
  ctx->cache_limit = int64_t(prop.totalGlobalMem / 2);
  ctx->group_cap_bytes = int64_t(prop.totalGlobalMem / 2);
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) return fail(MOCHY_EDEVICE);
    ctx->own_stream = true;
  }
  const PatternTables& pt = pattern_tables();
  int32_t parent[kHistSlots];
  for (int t = 0; t < kHistSlots; ++t) parent[t] = pt.id3_to_id26[t];
  if (ctx_alloc(ctx, (void**)&ctx->d_code_to_id3, sizeof(pt.code_to_id3)) != MOCHY_OK ||
      ctx_alloc(ctx, (void**)&ctx->d_id3_to_id26, sizeof(parent)) != MOCHY_OK ||
      ctx_alloc(ctx, (void**)&ctx->d_flags, 16 * sizeof(int32_t)) != MOCHY_OK ||
      ctx_alloc(ctx, (void**)&ctx->d_small, kSmallSlots * sizeof(int64_t)) != MOCHY_OK ||
      ctx_alloc(ctx, (void**)&ctx->d_open26, 27 * sizeof(int32_t)) != MOCHY_OK ||
      ctx_alloc(ctx, (void**)&ctx->d_dbl, 512 * sizeof(double)) != MOCHY_OK)
    return fail(MOCHY_ENOMEM);
  int pools = 0;
  ctx->async_alloc = hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, device) ==
                         hipSuccess && pools != 0;
  (void)hipGetLastError();
  if (hipHostMalloc((void**)&ctx->h_dbl, 512 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(MOCHY_ENOMEM);
  if (hipHostMalloc((void**)&ctx->h_small, kSmallSlots * sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
    return fail(MOCHY_ENOMEM);
  for (auto& e : ctx->ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(MOCHY_EDEVICE);
  // the allocation-free call's scratch address on this device; a failure
  // here is reported by that call (it retries the lookup), not by this one
  if (noalloc_setup(ctx) != MOCHY_OK) ctx->err.clear();
  int32_t open26[27];
  for (int t = 0; t < 27; ++t) open26[t] = pt.id26_open[t];
  if (hipMemcpy(ctx->d_open26, open26, sizeof(open26), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ctx->d_code_to_id3, pt.code_to_id3, sizeof(pt.code_to_id3), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ctx->d_id3_to_id26, parent, sizeof(parent), hipMemcpyHostToDevice) != hipSuccess)
    return fail(MOCHY_EDEVICE);
  *out = ctx;
  return MOCHY_OK;
}

extern "C" void mochy_ctx_destroy(mochy_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  cache_release(ctx);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(ctx->d_code_to_id3);
  (void)hipFree(ctx->d_id3_to_id26);
  (void)hipFree(ctx->d_flags);
  (void)hipFree(ctx->d_small);
  (void)hipFree(ctx->d_open26);
  (void)hipFree(ctx->d_dbl);
  if (ctx->h_small) (void)hipHostFree(ctx->h_small);
  if (ctx->h_dbl) (void)hipHostFree(ctx->h_dbl);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

extern "C" const char* mochy_last_error(const mochy_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

extern "C" mochy_status mochy_ctx_set_option(mochy_ctx* ctx, int32_t option, int64_t value) {
  if (!ctx) return MOCHY_EINVAL;
  if (option == MOCHY_OPT_GROUPS && (value == 0 || value == 1)) {
    ctx->group_neighbours = value != 0;
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_APLUS_ROWS && (value == 0 || value == 1)) {
    ctx->aplus_rows = value != 0;
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_GROUP_CAPACITY && value >= 0) {
    ctx->group_cap_bytes = value;
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_MEMO_BUDGET && value >= 0) {
    ctx->memo_budget = value;
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_MEMO_ALL && (value == 0 || value == 1)) {
    ctx->memo_all = value != 0;
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_MEMO_POOL && (value == 0 || value == 1)) {
    ctx->memo_pool = value != 0;
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_BATCH_LAUNCH && value >= 0 && value <= 2) {
    ctx->batch_launch = int(value);
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_PAIR_BLOCKS && value >= 1 && value <= 16) {
    ctx->pair_blocks = int(value);
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_CACHE_BYTES && value >= 0) {
    ctx->cache_limit = value;
    if (ctx->cache_bytes > value) cache_release(ctx);
    return MOCHY_OK;
  }
  if (option == MOCHY_OPT_TEST_FAULTS && value >= 0 && value <= 31) {
    ctx->test_faults = int(value);
    return MOCHY_OK;
  }
  ctx->err = "unknown option or value";
  return MOCHY_EINVAL;
}

extern "C" void mochy_graph_free(mochy_graph* g) {
  if (!g) return;
  if (g->ctx) (void)hipSetDevice(g->ctx->device);  // frees are ordered on the context stream
  void* bufs[] = {g->edge_ptr, g->edge_nodes, g->node_ptr, g->node_edges, g->heavy_bit, g->lg_ptr,
                  g->lg_col,   g->up_first,   g->up_ptr,   g->rec,        g->geoff,     g->gvoff,
                  g->gnoff,    g->row_graph,  g->xoff,     g->xnodes,     g->deg,       g->hsize,
                  g->hpair,    g->htriple,    g->hmask,      g->hbig_key,   g->hbig_val,
                  g->recm,     g->rsz};
  for (void* b : bufs) {
    if (g->ctx) device_free(g->ctx, b);
    else (void)hipFree(b);
  }
  delete g;
}

static mochy_status set_graph_offsets(mochy_ctx* ctx, mochy_graph* g) {
  g->ng = int32_t(g->h_geoff.size()) - 1;
  g->max_graph_edges = 0;
  for (int x = 0; x < g->ng; ++x)
    g->max_graph_edges = std::max(g->max_graph_edges, g->h_geoff[x + 1] - g->h_geoff[x]);
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&g->geoff, g->h_geoff.size() * 8)) != MOCHY_OK) return rc;
  if ((rc = device_alloc(ctx, (void**)&g->gvoff, g->h_gvoff.size() * 8)) != MOCHY_OK) return rc;
  if ((rc = device_alloc(ctx, (void**)&g->gnoff, g->h_gnoff.size() * 8)) != MOCHY_OK) return rc;
  MOCHY_HIP(hipMemcpyAsync(g->gnoff, g->h_gnoff.data(), g->h_gnoff.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  MOCHY_HIP(hipMemcpyAsync(g->geoff, g->h_geoff.data(), g->h_geoff.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  MOCHY_HIP(hipMemcpyAsync(g->gvoff, g->h_gvoff.data(), g->h_gvoff.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  MOCHY_HIP(hipStreamSynchronize(ctx->stream));
  return MOCHY_OK;
}

static mochy_status set_single_graph(mochy_ctx* ctx, mochy_graph* g) {
  g->h_geoff = {0, g->E};
  g->h_gvoff = {0, g->V};
  g->h_gnoff = {0, g->nnz};
  return set_graph_offsets(ctx, g);
}

extern "C" mochy_status mochy_project(mochy_ctx* ctx, const mochy_csr* c, uint32_t flags,
                                      mochy_graph** out, int64_t* num_hyperwedges) {
  if (!ctx) return MOCHY_EINVAL;
  if (!c || !out) { ctx->err = "null argument"; return MOCHY_EINVAL; }
  *out = nullptr;
  ctx->err.clear();
  phases_reset(ctx);
  if (c->num_edges < 0 || c->num_nodes < 0 || c->num_nodes > INT32_MAX || c->num_edges > INT32_MAX - 1) {
    ctx->err = "num_nodes / num_edges out of range";
    return MOCHY_EINVAL;
  }
  if (flags & ~(MOCHY_DEDUP | MOCHY_CANONICALIZE | MOCHY_LG_FREE)) {
    ctx->err = "unknown mochy_project flag";
    return MOCHY_EINVAL;
  }
  MOCHY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  mochy_graph* g = new (std::nothrow) mochy_graph();
  if (!g) return MOCHY_ENOMEM;
  g->ctx = ctx;
  g->E = c->num_edges;
  g->V = c->num_nodes;
  auto fail = [&](mochy_status s) { mochy_graph_free(g); return s; };
  mochy_status rc;
  phase_begin(ctx, kPhUpload);
  if (!c->on_device) {
    const int64_t* ptr = c->edge_ptr;
    const int32_t* nodes = c->edge_nodes;
    std::vector<int64_t> cptr;
    std::vector<int32_t> cnodes;
    if (flags & MOCHY_CANONICALIZE) {
      // each hyperedge as a node set: its list sorted, repeated nodes dropped
      if (g->E > 0 && (!ptr || ptr[0] != 0 || (ptr[g->E] > 0 && !nodes))) {
        ctx->err = "edge_ptr must start at 0 and the CSR pointers be non-null";
        return fail(MOCHY_EINVAL);
      }
      cptr.assign(1, 0);
      std::vector<int32_t> row;
      for (int64_t e = 0; e < g->E; ++e) {
        if (ptr[e + 1] < ptr[e]) {
          ctx->err = "decreasing edge_ptr at edge " + std::to_string(e);
          return fail(MOCHY_EINVAL);
        }
        row.assign(nodes + ptr[e], nodes + ptr[e + 1]);
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
        cnodes.insert(cnodes.end(), row.begin(), row.end());
        cptr.push_back(int64_t(cnodes.size()));
      }
      ptr = cptr.data();
      nodes = cnodes.data();
    }
    mochy_csr chk = *c;
    chk.edge_ptr = ptr;
    chk.edge_nodes = nodes;
    if ((rc = check_host_csr(ctx, &chk)) != MOCHY_OK) return fail(rc);
    std::vector<int64_t> dptr;
    std::vector<int32_t> dnodes;
    if (flags & MOCHY_DEDUP) {
      std::unordered_set<int64_t, RowHash, RowEq> seen(size_t(g->E) * 2 + 1, RowHash{ptr, nodes},
                                                      RowEq{ptr, nodes});
      dptr.push_back(0);
      for (int64_t e = 0; e < g->E; ++e) {
        if (!seen.insert(e).second) continue;
        dnodes.insert(dnodes.end(), nodes + ptr[e], nodes + ptr[e + 1]);
        dptr.push_back(int64_t(dnodes.size()));
      }
      g->E = int64_t(dptr.size()) - 1;
      ptr = dptr.data();
      nodes = dnodes.data();
    }
    g->nnz = g->E ? ptr[g->E] : 0;
    if ((rc = device_alloc(ctx, (void**)&g->edge_ptr, size_t(g->E + 1) * 8)) != MOCHY_OK) return fail(rc);
    if ((rc = device_alloc(ctx, (void**)&g->edge_nodes, size_t(g->nnz) * 4)) != MOCHY_OK) return fail(rc);
    if (g->E) {
      MOCHY_HIP(hipMemcpyAsync(g->edge_ptr, ptr, size_t(g->E + 1) * 8, hipMemcpyHostToDevice, st));
      if (g->nnz)
        MOCHY_HIP(hipMemcpyAsync(g->edge_nodes, nodes, size_t(g->nnz) * 4, hipMemcpyHostToDevice, st));
    } else {
      MOCHY_HIP(hipMemsetAsync(g->edge_ptr, 0, 8, st));
    }
    MOCHY_HIP(hipStreamSynchronize(st));  // host vectors above go out of scope
  } else {
    if (flags & (MOCHY_DEDUP | MOCHY_CANONICALIZE)) {
      ctx->err = "MOCHY_DEDUP and MOCHY_CANONICALIZE need host input";
      return fail(MOCHY_EINVAL);
    }
    int64_t ends[2] = {0, 0};
    if (g->E) {
      MOCHY_HIP(hipMemcpyAsync(&ends[0], c->edge_ptr, 8, hipMemcpyDeviceToHost, st));
      MOCHY_HIP(hipMemcpyAsync(&ends[1], c->edge_ptr + g->E, 8, hipMemcpyDeviceToHost, st));
      MOCHY_HIP(hipStreamSynchronize(st));
    }
    if (ends[0] != 0 || ends[1] < 0) { ctx->err = "edge_ptr must start at 0 and end >= 0"; return fail(MOCHY_EINVAL); }
    g->nnz = ends[1];
    if ((rc = device_alloc(ctx, (void**)&g->edge_ptr, size_t(g->E + 1) * 8)) != MOCHY_OK) return fail(rc);
    if ((rc = device_alloc(ctx, (void**)&g->edge_nodes, size_t(g->nnz) * 4)) != MOCHY_OK) return fail(rc);
    if (g->E) {
      MOCHY_HIP(hipMemcpyAsync(g->edge_ptr, c->edge_ptr, size_t(g->E + 1) * 8, hipMemcpyDeviceToDevice, st));
      if (g->nnz)
        MOCHY_HIP(hipMemcpyAsync(g->edge_nodes, c->edge_nodes, size_t(g->nnz) * 4, hipMemcpyDeviceToDevice, st));
    } else {
      MOCHY_HIP(hipMemsetAsync(g->edge_ptr, 0, 8, st));
    }
  }
  g->bytes = size_t(g->E + 1) * 8 + size_t(g->nnz) * 4;
  if ((rc = set_single_graph(ctx, g)) != MOCHY_OK) return fail(rc);
  const bool lg_free = (flags & MOCHY_LG_FREE) || g->E > kMaxGraphEdges;
  rc = lg_free ? project_free_device(ctx, g) : project_device(ctx, g);
  if (rc != MOCHY_OK) return fail(rc);
  *out = g;
  if (num_hyperwedges) *num_hyperwedges = g->W;
  return MOCHY_OK;
}

static bool which_ok(mochy_ctx* ctx, uint32_t which) {
  if (which == 0u || (which & ~MOCHY_WHICH_ALL) != 0u) {
    ctx->err = "which must select MOCHY_H26, MOCHY_H431 or both";
    return false;
  }
  return true;
}

static mochy_status finish_counts(mochy_ctx* ctx, int64_t* d_hist, uint32_t which, int64_t* counts26,
                                  int64_t* counts431) {
  hipStream_t st = ctx->stream;
  int64_t* d_out26 = ctx->d_small;  // [26]
  k_fold<<<1, 32, 0, st>>>(d_hist, ctx->d_id3_to_id26, d_out26);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, d_hist, kHistSlots * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small + kHistSlots, d_out26, MOCHY_NUM_H * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  if (ctx->h_small[0] != 0) {
    ctx->err = "internal error: " + std::to_string(ctx->h_small[0]) + " triples with an invalid pattern";
    return MOCHY_EDEVICE;
  }
  if (counts431 && (which & MOCHY_H431)) std::memcpy(counts431, ctx->h_small + 1, MOCHY_NUM_3H * 8);
  if (counts26 && (which & MOCHY_H26)) std::memcpy(counts26, ctx->h_small + kHistSlots, MOCHY_NUM_H * 8);
  return MOCHY_OK;
}

extern "C" mochy_status mochy_count_exact_range(mochy_ctx* ctx, const mochy_graph* g,
                                                int64_t c0, int64_t c1, uint32_t which,
                                                int64_t* counts26, int64_t* counts431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err.clear();
  phases_reset(ctx);
  for (int64_t& v : ctx->exact_stats) v = 0;
  if (!g || g->ctx != ctx || c0 < 0 || c1 < c0 || c1 > g->E) {
    ctx->err = "bad graph or centre range";
    return MOCHY_EINVAL;
  }
  if (!which_ok(ctx, which)) return MOCHY_EINVAL;
  if (g->lg_free) {
    ctx->err = "exact counting walks stored line-graph rows; this graph was projected without "
               "them (MOCHY_LG_FREE or more than 200000 hyperedges): use mochy_count_sampled";
    return MOCHY_EUNSUPPORTED;
  }
  MOCHY_HIP(hipSetDevice(ctx->device));
  int64_t* d_hist = ctx->d_small + 64;  // [432]
  mochy_status rc = exact_device(ctx, g, c0, c1, d_hist);
  if (rc != MOCHY_OK) return rc;
  return finish_counts(ctx, d_hist, which, counts26, counts431);
}

extern "C" mochy_status mochy_count_exact_range_noalloc(mochy_ctx* ctx, const mochy_graph* g,
                                                        int64_t c0, int64_t c1, uint32_t which,
                                                        int64_t* counts26, int64_t* counts431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err.clear();
  phases_reset(ctx);
  for (int64_t& v : ctx->exact_stats) v = 0;
  if (!g || g->ctx != ctx || c0 < 0 || c1 < c0 || c1 > g->E) {
    ctx->err = "bad graph or centre range";
    return MOCHY_EINVAL;
  }
  if (!which_ok(ctx, which)) return MOCHY_EINVAL;
  if (g->lg_free) {
    ctx->err = "exact counting walks stored line-graph rows; this graph was projected without them";
    return MOCHY_EUNSUPPORTED;
  }
  MOCHY_HIP(hipSetDevice(ctx->device));
  if (!ctx->noalloc_scratch && noalloc_setup(ctx) != MOCHY_OK) return MOCHY_EDEVICE;
  // every neighbour pair (the groups would need memory in proportion to the
  // line graph), schedule and light-pair lists carved from the scratch array
  const bool grouped = ctx->group_neighbours;
  ctx->group_neighbours = false;
  ctx->arena = static_cast<char*>(ctx->noalloc_scratch);
  ctx->arena_cap = (ctx->test_faults & 2) ? (size_t(64) << 10) : kNoallocBytes;
  ctx->arena_used = 0;
  int64_t* d_hist = ctx->d_small + 64;  // [432]
  mochy_status rc = exact_device(ctx, g, c0, c1, d_hist);
  ctx->group_neighbours = grouped;
  ctx->arena = nullptr;
  ctx->arena_cap = ctx->arena_used = 0;
  if (rc != MOCHY_OK) {
    (void)hipStreamSynchronize(ctx->stream);  // nothing may still use the scratch array
    return rc;
  }
  return finish_counts(ctx, d_hist, which, counts26, counts431);
}

extern "C" mochy_status mochy_count_exact(mochy_ctx* ctx, const mochy_graph* g, uint32_t which,
                                          int64_t* counts26, int64_t* counts431) {
  if (!g) {
    if (ctx) ctx->err = "null graph";
    return MOCHY_EINVAL;
  }
  return mochy_count_exact_range(ctx, g, 0, g->E, which, counts26, counts431);
}

extern "C" mochy_status mochy_graph_stats(mochy_ctx* ctx, const mochy_graph* g, int64_t* out) {
  if (!ctx) return MOCHY_EINVAL;
  if (!g || g->ctx != ctx || !out) { ctx->err = "bad argument"; return MOCHY_EINVAL; }
  MOCHY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  unsigned long long* d = (unsigned long long*)(ctx->d_small + 500);
  MOCHY_HIP(hipMemsetAsync(d, 0, 3 * 8, st));
  if (g->lg_free) {
    const mochy_status rc = free_graph_stats(ctx, g, d);
    if (rc != MOCHY_OK) return rc;
  } else if (g->E > 0) {
    k_stats<<<unsigned(g->E), 256, 0, st>>>(g->edge_ptr, g->lg_ptr, g->rec, d);
  }
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small + 500, d, 3 * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  out[0] = g->E; out[1] = g->V; out[2] = g->nnz; out[3] = g->W; out[4] = g->max_deg;
  out[5] = ctx->h_small[500];
  out[6] = g->lg_free ? -1 : ctx->h_small[501];
  out[7] = ctx->h_small[502];
  return MOCHY_OK;
}

extern "C" mochy_status mochy_count_sampled_edges(mochy_ctx* ctx, const mochy_graph* g, int64_t s,
                                                  uint64_t seed, int64_t sample_begin, int64_t* raw26,
                                                  double* est26, int64_t* raw431, double* est431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err.clear();
  phases_reset(ctx);
  if (!g || g->ctx != ctx || s <= 0 || sample_begin < 0 || s > INT64_MAX - sample_begin) {
    ctx->err = "bad graph, sample count or sample range";
    return MOCHY_EINVAL;
  }
  if (g->lg_free) {
    ctx->err = "hyperedge sampling walks stored line-graph rows; this graph was projected without "
               "them: use mochy_count_sampled";
    return MOCHY_EUNSUPPORTED;
  }
  MOCHY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  int64_t* d_hist = ctx->d_small + 64;
  mochy_status rc = sampled_edges_device(ctx, g, s, seed, sample_begin, d_hist);
  if (rc != MOCHY_OK) return rc;
  int64_t* d_raw26 = ctx->d_small;
  k_hsample_est<<<1, 512, 0, st>>>(d_hist, ctx->d_id3_to_id26, g->E, s, d_raw26, ctx->d_dbl,
                                   ctx->d_dbl + 32);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, d_hist, kHistSlots * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small + kHistSlots, d_raw26, MOCHY_NUM_H * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipMemcpyAsync(ctx->h_dbl, ctx->d_dbl, (32 + MOCHY_NUM_3H) * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  phases_collect(ctx);
  if (ctx->h_small[0] != 0) {
    ctx->err = "internal error: sampled triples with an invalid pattern";
    return MOCHY_EDEVICE;
  }
  if (raw431) std::memcpy(raw431, ctx->h_small + 1, MOCHY_NUM_3H * 8);
  if (raw26) std::memcpy(raw26, ctx->h_small + kHistSlots, MOCHY_NUM_H * 8);
  if (est26) std::memcpy(est26, ctx->h_dbl, MOCHY_NUM_H * 8);
  if (est431) std::memcpy(est431, ctx->h_dbl + 32, MOCHY_NUM_3H * 8);
  return MOCHY_OK;
}

extern "C" mochy_status mochy_hyperedge_profiles(mochy_ctx* ctx, const mochy_graph* g, int64_t e_begin,
                                                 int64_t e_end, int64_t* hp26, int64_t* hp431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err.clear();
  phases_reset(ctx);
  if (!g || g->ctx != ctx || e_begin < 0 || e_end < e_begin || e_end > g->E) {
    ctx->err = "bad graph or hyperedge range";
    return MOCHY_EINVAL;
  }
  if (g->lg_free) {
    ctx->err = "hyperedge profiles walk stored line-graph rows; this graph was projected without them";
    return MOCHY_EUNSUPPORTED;
  }
  MOCHY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  constexpr int64_t kChunkRows = int64_t(1) << 16;
  const int64_t rows = std::min(kChunkRows, std::max<int64_t>(e_end - e_begin, 1));
  int64_t* d_prof = nullptr;
  int64_t* d_prof26 = nullptr;
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&d_prof, size_t(rows) * kHistSlots * 8)) != MOCHY_OK) return rc;
  if ((rc = device_alloc(ctx, (void**)&d_prof26, size_t(rows) * MOCHY_NUM_H * 8)) != MOCHY_OK) {
    device_free(ctx, d_prof);
    return rc;
  }
  std::vector<int64_t> h_prof(size_t(rows) * kHistSlots);
  for (int64_t c0 = e_begin; c0 < e_end && rc == MOCHY_OK; c0 += rows) {
    const int64_t c1 = std::min(e_end, c0 + rows), n = c1 - c0;
    rc = profiles_device(ctx, g, c0, c1, d_prof, d_prof26);
    if (rc != MOCHY_OK) break;
    if (hipMemcpyAsync(h_prof.data(), d_prof, size_t(n) * kHistSlots * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        (hp26 && hipMemcpyAsync(hp26 + (c0 - e_begin) * MOCHY_NUM_H, d_prof26, size_t(n) * MOCHY_NUM_H * 8,
                                hipMemcpyDeviceToHost, st) != hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess) {
      ctx->err = "copying the profiles back failed";
      rc = MOCHY_EDEVICE;
      break;
    }
    for (int64_t x = 0; x < n; ++x) {
      const int64_t* row = h_prof.data() + x * kHistSlots;
      if (row[0] != 0) {
        ctx->err = "internal error: instances with an invalid pattern";
        rc = MOCHY_EDEVICE;
        break;
      }
      if (hp431) std::memcpy(hp431 + (c0 - e_begin + x) * MOCHY_NUM_3H, row + 1, MOCHY_NUM_3H * 8);
    }
  }
  phases_collect(ctx);
  device_free(ctx, d_prof);
  device_free(ctx, d_prof26);
  return rc;
}

extern "C" mochy_status mochy_count_sampled(mochy_ctx* ctx, const mochy_graph* g, int64_t r,
                                            uint64_t seed, int64_t sample_begin, uint32_t which,
                                            int64_t* raw26, double* est26, int64_t* raw431,
                                            double* est431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err.clear();
  phases_reset(ctx);
  if (!g || g->ctx != ctx || r <= 0 || sample_begin < 0 || r > INT64_MAX - sample_begin) {
    ctx->err = "bad graph, sample count or sample range";
    return MOCHY_EINVAL;
  }
  if (!which_ok(ctx, which)) return MOCHY_EINVAL;
  if (!(which & MOCHY_H26)) raw26 = nullptr, est26 = nullptr;
  if (!(which & MOCHY_H431)) raw431 = nullptr, est431 = nullptr;
  MOCHY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  int64_t* d_hist = ctx->d_small + 64;
  if (!g->lg_free && !ctx->aplus_rows && !g->walk_tried && g->ng == 1 && g->V < (int64_t(1) << 28)) {
    // first on-the-fly sampling of a single graph with stored rows: the
    // per-slot node lists and heavy tables (a few MB; without them, when the
    // lists would exceed 2^32 entries, sampling merges the stored rows)
    mochy_graph* gm = const_cast<mochy_graph*>(g);
    gm->walk_tried = true;
    const mochy_status wr = build_walk_tables(ctx, gm);
    if (wr == MOCHY_ERANGE) ctx->err.clear();
    else if (wr != MOCHY_OK) return wr;
  }
  const bool walk = g->xnodes != nullptr && (g->lg_free || !ctx->aplus_rows);
  mochy_status rc = walk ? sampled_free_device(ctx, g, r, seed, sample_begin, d_hist)
                         : sampled_device(ctx, g, r, seed, sample_begin, d_hist);
  if (rc != MOCHY_OK) return rc;
  int64_t* d_raw26 = ctx->d_small;
  k_aplus_est<<<1, 512, 0, st>>>(d_hist, ctx->d_id3_to_id26, ctx->d_open26, g->W, r, d_raw26,
                                 ctx->d_dbl, ctx->d_dbl + 32);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, d_hist, kHistSlots * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small + kHistSlots, d_raw26, MOCHY_NUM_H * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipMemcpyAsync(ctx->h_dbl, ctx->d_dbl, (32 + MOCHY_NUM_3H) * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  phases_collect(ctx);
  if (ctx->h_small[0] != 0) {
    ctx->err = "internal error: sampled triples with an invalid pattern";
    return MOCHY_EDEVICE;
  }
  if (raw431) std::memcpy(raw431, ctx->h_small + 1, MOCHY_NUM_3H * 8);
  if (raw26) std::memcpy(raw26, ctx->h_small + kHistSlots, MOCHY_NUM_H * 8);
  if (est26) std::memcpy(est26, ctx->h_dbl, MOCHY_NUM_H * 8);
  if (est431) std::memcpy(est431, ctx->h_dbl + 32, MOCHY_NUM_3H * 8);
  return MOCHY_OK;
}

// Builds graphs [g0, g1) of the input as one graph set (disjoint union) on the
// device and projects it.
static mochy_status build_set(mochy_ctx* ctx, const mochy_csr* graphs, int32_t g0, int32_t g1,
                              mochy_graph** out) {
  hipStream_t st = ctx->stream;
  *out = nullptr;
  mochy_graph* g = new (std::nothrow) mochy_graph();
  if (!g) return MOCHY_ENOMEM;
  g->ctx = ctx;
  auto fail = [&](mochy_status s) { mochy_graph_free(g); return s; };
  phase_begin(ctx, kPhUpload);
  std::vector<int64_t> nnz(g1 - g0);
  g->h_geoff.assign(1, 0);
  g->h_gvoff.assign(1, 0);
  for (int32_t x = g0; x < g1; ++x) {
    const mochy_csr& c = graphs[x];
    if (c.num_edges < 0 || c.num_nodes < 0 || c.num_nodes > INT32_MAX) {
      ctx->err = "graph " + std::to_string(x) + ": sizes out of range";
      return fail(MOCHY_EINVAL);
    }
    int64_t n = 0;
    if (!c.on_device) {
      const mochy_status rc = check_host_csr(ctx, &c);
      if (rc != MOCHY_OK) { ctx->err = "graph " + std::to_string(x) + ": " + ctx->err; return fail(rc); }
      n = c.num_edges ? c.edge_ptr[c.num_edges] : 0;
    } else if (c.num_edges) {
      int64_t ends[2] = {0, 0};
      MOCHY_HIP(hipMemcpyAsync(&ends[0], c.edge_ptr, 8, hipMemcpyDeviceToHost, st));
      MOCHY_HIP(hipMemcpyAsync(&ends[1], c.edge_ptr + c.num_edges, 8, hipMemcpyDeviceToHost, st));
      MOCHY_HIP(hipStreamSynchronize(st));
      if (ends[0] != 0 || ends[1] < 0) { ctx->err = "graph " + std::to_string(x) + ": bad edge_ptr"; return fail(MOCHY_EINVAL); }
      n = ends[1];
    }
    nnz[x - g0] = n;
    g->h_geoff.push_back(g->h_geoff.back() + c.num_edges);
    g->h_gvoff.push_back(g->h_gvoff.back() + c.num_nodes);
  }
  g->E = g->h_geoff.back();
  g->V = g->h_gvoff.back();
  if (g->E > INT32_MAX - 1 || g->V > INT32_MAX) { ctx->err = "batch too large"; return fail(MOCHY_ERANGE); }
  g->nnz = 0;
  g->h_gnoff.assign(1, 0);
  for (int64_t n : nnz) {
    g->nnz += n;
    g->h_gnoff.push_back(g->nnz);
  }
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&g->edge_ptr, size_t(g->E + 1) * 8)) != MOCHY_OK) return fail(rc);
  if ((rc = device_alloc(ctx, (void**)&g->edge_nodes, size_t(g->nnz) * 4)) != MOCHY_OK) return fail(rc);
  int64_t noff = 0;
  for (int32_t x = g0; x < g1; ++x) {
    const mochy_csr& c = graphs[x];
    const int64_t eb = g->h_geoff[x - g0], ne = c.num_edges, nn = nnz[x - g0];
    const hipMemcpyKind kind = c.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (ne) MOCHY_HIP(hipMemcpyAsync(g->edge_ptr + eb, c.edge_ptr, size_t(ne) * 8, kind, st));
    if (nn) MOCHY_HIP(hipMemcpyAsync(g->edge_nodes + noff, c.edge_nodes, size_t(nn) * 4, kind, st));
    const int64_t mx = std::max(ne, nn);
    if (mx > 0)
      k_union_offsets<<<unsigned((mx + 255) / 256), 256, 0, st>>>(eb, ne, noff, g->edge_ptr, noff, nn,
                                                                  int32_t(g->h_gvoff[x - g0]), g->edge_nodes);
    noff += nn;
  }
  MOCHY_HIP(hipMemcpyAsync(g->edge_ptr + g->E, &g->nnz, 8, hipMemcpyHostToDevice, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  if ((rc = set_graph_offsets(ctx, g)) != MOCHY_OK) return fail(rc);
  if ((rc = project_device(ctx, g)) != MOCHY_OK) return fail(rc);
  *out = g;
  return MOCHY_OK;
}

// Exact counts of graphs [g0, g1) into d_all[g][kHistSlots], in consecutive
// sub-batches.  The first takes graphs up to kFirstBatchEdges hyperedges;
// the hyperwedges and device bytes per hyperedge that each one needed (its
// graph set, and row capacity for one-pass grouping: 24 B per row entry)
// size the next: at most three quarters of the memory then free (including
// this context's cached buffers), row capacity within the one-pass limit,
// and at most kBatchWedges hyperwedges, about what fills the device (a
// hypergraph of that size already keeps every kernel's grid full, and a
// sub-batch of such graphs would only need more memory than counting them
// one by one).  A sub-batch that still runs out of memory is halved.  A
// single graph whose groups do not fit pairs every neighbour instead.
constexpr int64_t kFirstBatchEdges = 200000;
constexpr double kBatchWedges = 1e9;
static mochy_status profile_counts(mochy_ctx* ctx, const mochy_csr* graphs, int32_t g0, int32_t g1,
                                   int64_t* d_all) {
  // MOCHY_LOG_BATCHES=1: one line on stderr per sub-batch counted (progress of long calls)
  const char* lb = std::getenv("MOCHY_LOG_BATCHES");
  const bool log_batches = lb && lb[0] == '1';
  int64_t budget_edges = kFirstBatchEdges;  // hyperedges the next sub-batch may hold
  int32_t cap = g1 - g0;                    // graphs it may hold (halved on running out)
  for (int32_t a = g0; a < g1;) {
    int32_t b = a + 1;
    int64_t edges = std::max<int64_t>(graphs[a].num_edges, 0);
    while (b < g1 && b - a < cap && edges + std::max<int64_t>(graphs[b].num_edges, 0) <= budget_edges)
      edges += std::max<int64_t>(graphs[b++].num_edges, 0);
    mochy_graph* set = nullptr;
    mochy_status rc = build_set(ctx, graphs, a, b, &set);
    double per_edge = 0.0, wedges_per_edge = 0.0;
    if (rc == MOCHY_OK) {
      rc = exact_device(ctx, set, 0, set->E, d_all + int64_t(a) * kHistSlots);
      if (set->E > 0) {
        per_edge = (double(set->bytes) + 48.0 * double(set->W)) / double(set->E);
        wedges_per_edge = double(set->W) / double(set->E);
      }
      mochy_graph_free(set);
    }
    if (rc == MOCHY_ENOMEM && b - a > 1) {
      ctx->err.clear();
      cap = (b - a + 1) / 2;  // halved, rounded up (still smaller: b - a >= 2)
      continue;
    }
    if (rc != MOCHY_OK) return rc;
    ctx->exact_stats[kStBatches] += 1;
    if (log_batches) std::fprintf(stderr, "[mochy] profile: graphs [%d, %d) of %d counted\n", a, b, g1);
    size_t free_b = 0, total_b = 0;
    if (per_edge > 0.0 && hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
      const double avail = 0.75 * (double(free_b) + double(ctx->cache_bytes));
      double e = avail / per_edge;
      if (wedges_per_edge > 0.0) {
        e = std::min(e, double(ctx->group_cap_bytes) / (48.0 * wedges_per_edge));
        e = std::min(e, kBatchWedges / wedges_per_edge);
      }
      budget_edges = std::max<int64_t>(1, int64_t(e));
    } else {
      (void)hipGetLastError();
    }
    a = b;
  }
  return MOCHY_OK;
}

extern "C" mochy_status mochy_profile(mochy_ctx* ctx, int32_t num_graphs, const mochy_csr* graphs,
                                      double eps, uint32_t which, int64_t* counts, double* sig26,
                                      double* cp26, double* sig431, double* cp431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err.clear();
  phases_reset(ctx);
  for (int64_t& v : ctx->exact_stats) v = 0;
  if (num_graphs < 2 || !graphs || !(eps >= 0.0)) {
    ctx->err = "need the hypergraph and at least one randomized copy, and eps >= 0";
    return MOCHY_EINVAL;
  }
  if (!which_ok(ctx, which)) return MOCHY_EINVAL;
  if (!(which & MOCHY_H26)) sig26 = nullptr, cp26 = nullptr;
  if (!(which & MOCHY_H431)) sig431 = nullptr, cp431 = nullptr;
  MOCHY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const size_t per = MOCHY_NUM_H + MOCHY_NUM_3H;
  int64_t* d_all = nullptr;     // [ng][kHistSlots]
  int64_t* d_counts = nullptr;  // [ng][per]
  double* d_out = nullptr;      // sig26, cp26, sig431, cp431
  mochy_status rc;
  if ((rc = device_alloc(ctx, (void**)&d_all, size_t(num_graphs) * kHistSlots * 8)) != MOCHY_OK) return rc;
  auto cleanup = [&]() { device_free(ctx, d_all); device_free(ctx, d_counts); device_free(ctx, d_out); };
  if ((rc = device_alloc(ctx, (void**)&d_counts, size_t(num_graphs) * per * 8)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&d_out, 2 * per * 8)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = profile_counts(ctx, graphs, 0, num_graphs, d_all)) != MOCHY_OK) { cleanup(); return rc; }
  phase_begin(ctx, kPhProfile);
  k_profile<<<1, 512, 0, st>>>(d_all, ctx->d_id3_to_id26, num_graphs, eps, d_counts, d_out,
                               d_out + MOCHY_NUM_H, d_out + 2 * MOCHY_NUM_H,
                               d_out + 2 * MOCHY_NUM_H + MOCHY_NUM_3H);
  phase_end(ctx, kPhProfile);
  std::vector<int64_t> hc(size_t(num_graphs) * per);
  std::vector<double> ho(2 * per);
  std::vector<int64_t> hall(size_t(num_graphs) * kHistSlots);
  if (hipMemcpyAsync(hc.data(), d_counts, hc.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(ho.data(), d_out, ho.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(hall.data(), d_all, hall.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    cleanup();
    ctx->err = "device-to-host copy failed";
    return MOCHY_EDEVICE;
  }
  phases_collect(ctx);
  cleanup();
  for (int32_t x = 0; x < num_graphs; ++x)
    if (hall[size_t(x) * kHistSlots] != 0) {
      ctx->err = "internal error: invalid pattern counted in graph " + std::to_string(x);
      return MOCHY_EDEVICE;
    }
  if (counts) {
    for (int32_t x = 0; x < num_graphs; ++x) {
      const int64_t* src = hc.data() + size_t(x) * per;
      int64_t* dst = counts + size_t(x) * per;
      if (which & MOCHY_H26) std::memcpy(dst, src, MOCHY_NUM_H * 8);
      if (which & MOCHY_H431) std::memcpy(dst + MOCHY_NUM_H, src + MOCHY_NUM_H, MOCHY_NUM_3H * 8);
    }
  }
  if (sig26) std::memcpy(sig26, ho.data(), MOCHY_NUM_H * 8);
  if (cp26) std::memcpy(cp26, ho.data() + MOCHY_NUM_H, MOCHY_NUM_H * 8);
  if (sig431) std::memcpy(sig431, ho.data() + 2 * MOCHY_NUM_H, MOCHY_NUM_3H * 8);
  if (cp431) std::memcpy(cp431, ho.data() + 2 * MOCHY_NUM_H + MOCHY_NUM_3H, MOCHY_NUM_3H * 8);
  return MOCHY_OK;
}
