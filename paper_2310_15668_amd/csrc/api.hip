// C ABI of the library (declared in include/mochy.h).
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <unordered_set>

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
  }
  c->phases_run = 0;
}

static void phases_reset(mochy_ctx* c) {
  c->phases_run = 0;
  for (double& m : c->phase_ms) m = 0.0;
}

extern "C" mochy_status mochy_phase_ms(const mochy_ctx* ctx, double* ms) {
  if (!ctx || !ms) return MOCHY_EINVAL;
  std::memcpy(ms, ctx->phase_ms, sizeof(ctx->phase_ms));
  return MOCHY_OK;
}

mochy_status device_alloc(mochy_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  const hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 8));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    ctx->err = "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
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
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) return fail(MOCHY_EDEVICE);
    ctx->own_stream = true;
  }
  const PatternTables& pt = pattern_tables();
  int32_t parent[kHistSlots];
  for (int t = 0; t < kHistSlots; ++t) parent[t] = pt.id3_to_id26[t];
  if (device_alloc(ctx, (void**)&ctx->d_code_to_id3, sizeof(pt.code_to_id3)) != MOCHY_OK ||
      device_alloc(ctx, (void**)&ctx->d_id3_to_id26, sizeof(parent)) != MOCHY_OK ||
      device_alloc(ctx, (void**)&ctx->d_flags, 16 * sizeof(int32_t)) != MOCHY_OK ||
      device_alloc(ctx, (void**)&ctx->d_small, 512 * sizeof(int64_t)) != MOCHY_OK ||
      device_alloc(ctx, (void**)&ctx->d_open26, 27 * sizeof(int32_t)) != MOCHY_OK ||
      device_alloc(ctx, (void**)&ctx->d_dbl, 512 * sizeof(double)) != MOCHY_OK)
    return fail(MOCHY_ENOMEM);
  if (hipHostMalloc((void**)&ctx->h_dbl, 512 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return fail(MOCHY_ENOMEM);
  if (hipHostMalloc((void**)&ctx->h_small, 512 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
    return fail(MOCHY_ENOMEM);
  for (auto& e : ctx->ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(MOCHY_EDEVICE);
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

extern "C" void mochy_graph_free(mochy_graph* g) {
  if (!g) return;
  if (g->ctx) {
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
  }
  void* bufs[] = {g->edge_ptr, g->edge_nodes, g->node_ptr, g->node_edges, g->heavy_bit, g->lg_ptr,
                  g->lg_col,   g->up_first,   g->up_ptr,   g->rec};
  for (void* b : bufs) (void)hipFree(b);
  delete g;
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
    if ((rc = check_host_csr(ctx, c)) != MOCHY_OK) return fail(rc);
    const int64_t* ptr = c->edge_ptr;
    const int32_t* nodes = c->edge_nodes;
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
    if (flags & MOCHY_DEDUP) { ctx->err = "MOCHY_DEDUP needs host input"; return fail(MOCHY_EINVAL); }
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
  if ((rc = project_device(ctx, g)) != MOCHY_OK) return fail(rc);
  *out = g;
  if (num_hyperwedges) *num_hyperwedges = g->W;
  return MOCHY_OK;
}

// Largest hyperedge count the exact path's LDS row bitmap (plus ranks) handles.
constexpr int64_t kMaxEdgesExact = 200000;

static mochy_status finish_counts(mochy_ctx* ctx, int64_t* d_hist, int64_t* counts26,
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
  if (counts431) std::memcpy(counts431, ctx->h_small + 1, MOCHY_NUM_3H * 8);
  if (counts26) std::memcpy(counts26, ctx->h_small + kHistSlots, MOCHY_NUM_H * 8);
  return MOCHY_OK;
}

extern "C" mochy_status mochy_count_exact_range(mochy_ctx* ctx, const mochy_graph* g,
                                                int64_t c0, int64_t c1, int64_t* counts26,
                                                int64_t* counts431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err.clear();
  phases_reset(ctx);
  if (!g || g->ctx != ctx || c0 < 0 || c1 < c0 || c1 > g->E) {
    ctx->err = "bad graph or centre range";
    return MOCHY_EINVAL;
  }
  if (g->E > kMaxEdgesExact) {
    ctx->err = "exact counting handles at most 200000 hyperedges in this build";
    return MOCHY_EUNSUPPORTED;
  }
  MOCHY_HIP(hipSetDevice(ctx->device));
  int64_t* d_hist = ctx->d_small + 64;  // [432]
  mochy_status rc = exact_device(ctx, g, c0, c1, d_hist);
  if (rc != MOCHY_OK) return rc;
  return finish_counts(ctx, d_hist, counts26, counts431);
}

extern "C" mochy_status mochy_count_exact(mochy_ctx* ctx, const mochy_graph* g, int64_t* counts26,
                                          int64_t* counts431) {
  if (!g) {
    if (ctx) ctx->err = "null graph";
    return MOCHY_EINVAL;
  }
  return mochy_count_exact_range(ctx, g, 0, g->E, counts26, counts431);
}

extern "C" mochy_status mochy_graph_stats(mochy_ctx* ctx, const mochy_graph* g, int64_t* out) {
  if (!ctx) return MOCHY_EINVAL;
  if (!g || g->ctx != ctx || !out) { ctx->err = "bad argument"; return MOCHY_EINVAL; }
  MOCHY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  unsigned long long* d = (unsigned long long*)(ctx->d_small + 500);
  MOCHY_HIP(hipMemsetAsync(d, 0, 3 * 8, st));
  if (g->E > 0) k_stats<<<unsigned(g->E), 256, 0, st>>>(g->edge_ptr, g->lg_ptr, g->rec, d);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small + 500, d, 3 * 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  out[0] = g->E; out[1] = g->V; out[2] = g->nnz; out[3] = g->W; out[4] = g->max_deg;
  out[5] = ctx->h_small[500]; out[6] = ctx->h_small[501]; out[7] = ctx->h_small[502];
  return MOCHY_OK;
}

extern "C" mochy_status mochy_count_sampled(mochy_ctx* ctx, const mochy_graph* g, int64_t r,
                                            uint64_t seed, int64_t sample_begin, int64_t* raw26,
                                            double* est26, int64_t* raw431, double* est431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err.clear();
  phases_reset(ctx);
  if (!g || g->ctx != ctx || r <= 0 || sample_begin < 0 || r > INT64_MAX - sample_begin) {
    ctx->err = "bad graph, sample count or sample range";
    return MOCHY_EINVAL;
  }
  MOCHY_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  int64_t* d_hist = ctx->d_small + 64;
  mochy_status rc = sampled_device(ctx, g, r, seed, sample_begin, d_hist);
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

extern "C" mochy_status mochy_profile(mochy_ctx* ctx, int32_t num_graphs, const mochy_csr* graphs,
                                      double eps, int64_t* counts, double* sig26, double* cp26,
                                      double* sig431, double* cp431) {
  if (!ctx) return MOCHY_EINVAL;
  ctx->err = "not built yet";
  (void)num_graphs; (void)graphs; (void)eps; (void)counts; (void)sig26; (void)cp26; (void)sig431; (void)cp431;
  return MOCHY_EUNSUPPORTED;
}
