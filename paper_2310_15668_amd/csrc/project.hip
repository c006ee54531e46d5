// Line-graph construction on the device (Algorithm 1, section 4.1).
//
// project_incidence (steps 1-3) is shared with the line-graph-free mode.
// Steps, all on the context stream:
//   1. validate the CSR (sorted, in range, non-empty, size <= MOCHY_MAX_EDGE);
//   2. transpose it into E_v (node -> hyperedges): count, scan, scatter;
//   3. pick the 64 highest-degree nodes ("heavy"; ties to the smaller id);
//   4. line-graph degree of every hyperedge: the row of e_i is the union of
//      E_v over v in e_i minus e_i itself, formed as a bitmap over hyperedge
//      ids in LDS (so the row comes out sorted and de-duplicated);
//   5. scan the degrees into row pointers; |wedges| = sum / 2;
//   6. fill the rows (ascending neighbour ids) from the same bitmap;
//   7. one 16-byte record per (centre, neighbour): which nodes of e_i the
//      neighbour holds (a 32-bit mask; omega = its popcount), how many of its
//      nodes lie outside e_i, which heavy nodes lie outside e_i, and whether a
//      non-heavy node does.  Identical hyperedges show up here (no outside
//      node, every node of e_i) and are reported.
#include "common.h"

namespace {

// Each hyperedge is checked against its own graph: incidences inside the
// graph's slice, node ids inside the graph's node range, strictly ascending.
__global__ void k_validate(int64_t E, int32_t ng, const int64_t* __restrict__ geoff,
                           const int64_t* __restrict__ gvoff, const int64_t* __restrict__ gnoff,
                           const int64_t* __restrict__ ptr, const int32_t* __restrict__ nodes,
                           int32_t* flags) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int lo = 0, hi = ng;  // last graph with geoff[g] <= e
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (geoff[mid] <= e) lo = mid; else hi = mid;
  }
  const int64_t s = ptr[e], t = ptr[e + 1];
  if (s < gnoff[lo] || t > gnoff[lo + 1] || t <= s) { atomicOr(flags, kFlagInval); return; }
  if (t - s > MOCHY_MAX_EDGE) { atomicOr(flags, kFlagRange); return; }
  const int64_t v0 = gvoff[lo], v1 = gvoff[lo + 1];
  int64_t prev = v0 - 1;
  for (int64_t q = s; q < t; ++q) {
    const int64_t v = nodes[q];
    if (v < v0 || v >= v1 || v <= prev) { atomicOr(flags, kFlagInval); return; }
    prev = v;
  }
}

__global__ void k_node_count(int64_t nnz, const int32_t* __restrict__ nodes,
                             unsigned long long* cnt) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < nnz) atomicAdd(&cnt[nodes[q]], 1ull);
}

__global__ void k_node_fill(int64_t E, const int64_t* __restrict__ ptr,
                            const int32_t* __restrict__ nodes, const int64_t* __restrict__ node_ptr,
                            unsigned int* fill, int32_t* node_edges) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= E) return;
  for (int64_t q = ptr[e]; q < ptr[e + 1]; ++q) {
    const int32_t v = nodes[q];
    const unsigned slot = atomicAdd(&fill[v], 1u);
    node_edges[node_ptr[v] + slot] = int32_t(e);
  }
}

// One block of 1024 threads per graph: 64 rounds of "largest degree not yet
// taken" over the graph's nodes.
__global__ __launch_bounds__(1024) void k_heavy(const int64_t* __restrict__ gvoff,
                                                const int64_t* __restrict__ node_ptr,
                                                int8_t* heavy_bit) {
  __shared__ unsigned long long best[1024];
  const int64_t v0 = gvoff[blockIdx.x], v1 = gvoff[blockIdx.x + 1];
  for (int64_t v = v0 + threadIdx.x; v < v1; v += 1024) heavy_bit[v] = -1;
  __syncthreads();
  for (int round = 0; round < kHeavyBits; ++round) {
    unsigned long long mine = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 1024) {
      if (heavy_bit[v] >= 0) continue;
      const unsigned long long deg = (unsigned long long)(node_ptr[v + 1] - node_ptr[v]);
      const unsigned long long key = (deg << 32) | (0xffffffffull - (unsigned long long)v);
      mine = key > mine ? key : mine;
    }
    best[threadIdx.x] = mine;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
      if (threadIdx.x < unsigned(off) && best[threadIdx.x + off] > best[threadIdx.x])
        best[threadIdx.x] = best[threadIdx.x + off];
      __syncthreads();
    }
    const unsigned long long top = best[0];
    __syncthreads();
    if ((top >> 32) < 2) break;  // a node in fewer than two hyperedges is never shared
    if (threadIdx.x == 0) heavy_bit[0xffffffffull - (top & 0xffffffffull)] = int8_t(round);
    __syncthreads();
  }
}

// Builds the neighbour bitmap of row i in LDS: bit x - e0 for neighbour x,
// where the row's graph owns hyperedges [e0, e0 + 32 * nwords).
__device__ void build_row_bitmap(int64_t i, int64_t e0, const int64_t* __restrict__ ptr,
                                 const int32_t* __restrict__ nodes,
                                 const int64_t* __restrict__ node_ptr,
                                 const int32_t* __restrict__ node_edges, uint32_t* bm, int nwords) {
  for (int w = threadIdx.x; w < nwords; w += blockDim.x) bm[w] = 0;
  __syncthreads();
  for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) {
    const int32_t v = nodes[q];
    const int64_t lo = node_ptr[v], hi = node_ptr[v + 1];
    for (int64_t r = lo + threadIdx.x; r < hi; r += blockDim.x) {
      const int64_t x = node_edges[r];
      if (x != i) atomicOr(&bm[(x - e0) >> 5], 1u << ((x - e0) & 31));
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void graph_range(int64_t i, const int32_t* __restrict__ row_graph,
                                            const int64_t* __restrict__ geoff, int64_t& e0,
                                            int& nwords) {
  const int gi = row_graph[i];
  e0 = geoff[gi];
  nwords = int((geoff[gi + 1] - e0 + 31) / 32);
}

__global__ __launch_bounds__(256) void k_proj_degree(int64_t E, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ nodes,
                                                     const int64_t* __restrict__ node_ptr,
                                                     const int32_t* __restrict__ node_edges,
                                                     const int32_t* __restrict__ row_graph,
                                                     const int64_t* __restrict__ geoff,
                                                     int64_t* deg, int32_t* max_deg) {
  extern __shared__ uint32_t bm[];
  __shared__ int32_t red[256];
  const int64_t i = blockIdx.x;
  int64_t e0;
  int nwords;
  graph_range(i, row_graph, geoff, e0, nwords);
  build_row_bitmap(i, e0, ptr, nodes, node_ptr, node_edges, bm, nwords);
  int32_t c = 0;
  for (int w = threadIdx.x; w < nwords; w += blockDim.x) c += __popc(bm[w]);
  red[threadIdx.x] = c;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < unsigned(off)) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    deg[i] = red[0];
    atomicMax(max_deg, red[0]);
  }
}

__global__ __launch_bounds__(256) void k_proj_fill(int64_t E, const int64_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ nodes,
                                                   const int64_t* __restrict__ node_ptr,
                                                   const int32_t* __restrict__ node_edges,
                                                   const int32_t* __restrict__ row_graph,
                                                   const int64_t* __restrict__ geoff,
                                                   const int64_t* __restrict__ lg_ptr,
                                                   int32_t* lg_col, int32_t* up_first) {
  extern __shared__ uint32_t bm[];
  __shared__ int32_t part[256];
  const int64_t i = blockIdx.x;
  int64_t e0;
  int nwords;
  graph_range(i, row_graph, geoff, e0, nwords);
  build_row_bitmap(i, e0, ptr, nodes, node_ptr, node_edges, bm, nwords);
  // each thread owns a contiguous chunk of words
  const int chunk = (nwords + 255) / 256;
  const int w0 = min(nwords, int(threadIdx.x) * chunk), w1 = min(nwords, w0 + chunk);
  int32_t c = 0;
  for (int w = w0; w < w1; ++w) c += __popc(bm[w]);
  part[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int32_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t pos = part[threadIdx.x] - c;  // exclusive
  int32_t* out = lg_col + lg_ptr[i];
  const int64_t il = i - e0;
  const int wi = int(il >> 5);
  for (int w = w0; w < w1; ++w) {
    uint32_t bits = bm[w];
    if (w == wi) up_first[i] = pos + __popc(bits & ((1u << (il & 31)) - 1u));
    while (bits) {
      const int b = __ffs(bits) - 1;
      bits &= bits - 1;
      out[pos++] = int32_t(e0 + ((w << 5) | b));
    }
  }
}

// Each hyperedge's heavy nodes as a 64-bit mask (bit heavy_bit[v]).
__global__ void k_edge_heavy(int64_t E, const int64_t* __restrict__ ptr, const int32_t* __restrict__ nodes,
                             const int8_t* __restrict__ heavy_bit, unsigned long long* hmask) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x >= E) return;
  unsigned long long h = 0;
  for (int64_t q = ptr[x]; q < ptr[x + 1]; ++q) {
    const int b = heavy_bit[nodes[q]];
    if (b >= 0) h |= 1ull << b;
  }
  hmask[x] = h;
}

// Row i's records: for each neighbour e_x, the mask of e_i's nodes it holds
// (found by scanning e_x's nodes against e_i), its outside count, and its
// heavy outside nodes, hmask[x] less e_i's own heavy nodes.
__global__ __launch_bounds__(256) void k_records(int64_t E, const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ nodes,
                                                 const unsigned long long* __restrict__ hmask,
                                                 const int64_t* __restrict__ lg_ptr,
                                                 const int32_t* __restrict__ lg_col, uint4* rec,
                                                 uint32_t* recm, uint16_t* rsz, int32_t* flags) {
  __shared__ int32_t ei[MOCHY_MAX_EDGE];
  // membership filter of e_i's nodes by their low 10 bits: most nodes of a
  // neighbour are outside e_i and leave after one read
  __shared__ uint32_t filt[32];
  const int64_t i = blockIdx.x;
  const int64_t s = ptr[i];
  const int a = int(ptr[i + 1] - s);
  if (threadIdx.x < 32u) filt[threadIdx.x] = 0u;
  __syncthreads();
  if (threadIdx.x < unsigned(a)) {
    const int32_t v = nodes[s + threadIdx.x];
    ei[threadIdx.x] = v;
    atomicOr(&filt[(v >> 5) & 31], 1u << (v & 31));
  }
  __syncthreads();
  const int64_t base = lg_ptr[i];
  const int64_t d = lg_ptr[i + 1] - base;
  const unsigned long long hi = hmask[i];
  for (int64_t p = threadIdx.x; p < d; p += blockDim.x) {
    const int32_t x = lg_col[base + p];
    uint32_t m = 0;
    const int64_t q0 = ptr[x], q1 = ptr[x + 1];
    const unsigned long long hv = hmask[x] & ~hi;  // heavy nodes of e_x outside e_i
    // four of e_x's nodes at a time, their loads issued together before any
    // is used; -1 pads past the list's end
    for (int64_t q = q0; q < q1; q += 4) {
      int32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = q + u < q1 ? nodes[q + u] : -1;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        int lo = 0, hb = a;  // binary search of v in e_i, past the filter
        if (v[u] < 0 || !((filt[(v[u] >> 5) & 31] >> (v[u] & 31)) & 1u)) hb = 0;
        while (lo < hb) {
          const int mid = (lo + hb) >> 1;
          if (ei[mid] < v[u]) lo = mid + 1; else hb = mid;
        }
        if (lo < a && ei[lo] == v[u]) m |= 1u << lo;
      }
    }
    const uint32_t o = uint32_t(q1 - q0) - uint32_t(__popc(m));
    const uint32_t light = o > uint32_t(__popcll(hv)) ? 1u : 0u;  // an outside node that is not heavy
    if (o == 0 && __popc(m) == a) atomicOr(flags, kFlagDup);
    rec[base + p] = make_uint4(m, o | (light ? kRecLight : 0u), uint32_t(hv), uint32_t(hv >> 32));
    recm[base + p] = m;
    rsz[base + p] = uint16_t(uint32_t(__popc(m)) | ((uint32_t(__popc(m)) + o) << 8));
  }
}

__global__ void k_upper_len(int64_t E, const int64_t* __restrict__ lg_ptr,
                            const int32_t* __restrict__ up_first, int64_t* up_len) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < E) up_len[i] = (lg_ptr[i + 1] - lg_ptr[i]) - up_first[i];
  if (i == E) up_len[E] = 0;
}

__global__ void k_row_graph(int64_t E, int32_t ng, const int64_t* __restrict__ geoff,
                            int32_t* row_graph) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= E) return;
  int lo = 0, hi = ng;  // last g with geoff[g] <= i
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (geoff[mid] <= i) lo = mid; else hi = mid;
  }
  row_graph[i] = lo;
}

inline unsigned blocks(int64_t n, int t) { return unsigned((n + t - 1) / t); }

}  // namespace

mochy_status project_incidence(mochy_ctx* ctx, mochy_graph* g) {
  hipStream_t st = ctx->stream;
  const int64_t E = g->E, V = g->V, nnz = g->nnz;
  MOCHY_HIP(hipMemsetAsync(ctx->d_flags, 0, 4 * sizeof(int32_t), st));
  if (E > 0)
    k_validate<<<blocks(E, 256), 256, 0, st>>>(E, g->ng, g->geoff, g->gvoff, g->gnoff, g->edge_ptr,
                                               g->edge_nodes, ctx->d_flags);
  phase_end(ctx, kPhUpload);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, ctx->d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  phases_collect(ctx);
  const int32_t f0 = *reinterpret_cast<int32_t*>(ctx->h_small);
  if (f0 & kFlagInval) { ctx->err = "malformed CSR (unsorted, out-of-range or empty hyperedge)"; return MOCHY_EINVAL; }
  if (f0 & kFlagRange) { ctx->err = "a hyperedge exceeds MOCHY_MAX_EDGE nodes"; return MOCHY_ERANGE; }

  // 2. transpose
  const size_t tmpn = scan_tmp_elems(std::max<int64_t>(V, E) + 1);
  int64_t* tmp = nullptr;
  int64_t* cnt = nullptr;
  unsigned int* fill = nullptr;
  mochy_status rc;
  auto cleanup = [&]() { device_free(ctx, tmp); device_free(ctx, cnt); device_free(ctx, fill); };
  if ((rc = device_alloc(ctx, (void**)&tmp, tmpn * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&cnt, size_t(std::max(V, E) + 1) * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&fill, size_t(V + 1) * 4)) != MOCHY_OK) {
    cleanup();
    return rc;
  }
  if ((rc = device_alloc(ctx, (void**)&g->node_ptr, size_t(V + 1) * 8)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&g->node_edges, size_t(std::max<int64_t>(nnz, 1)) * 4)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&g->heavy_bit, size_t(std::max<int64_t>(V, 1)))) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&g->up_ptr, size_t(E + 1) * 8)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&g->row_graph, size_t(std::max<int64_t>(E, 1)) * 4)) != MOCHY_OK) { cleanup(); return rc; }
  if (E > 0) k_row_graph<<<blocks(E, 256), 256, 0, st>>>(E, g->ng, g->geoff, g->row_graph);
  g->bytes += size_t(V + 1) * 8 + size_t(nnz) * 4 + size_t(V) + size_t(E + 1) * 8 + size_t(E) * 4;

  phase_begin(ctx, kPhTranspose);
  MOCHY_HIP(hipMemsetAsync(cnt, 0, size_t(V + 1) * 8, st));
  MOCHY_HIP(hipMemsetAsync(fill, 0, size_t(V + 1) * 4, st));
  if (nnz > 0)
    k_node_count<<<blocks(nnz, 256), 256, 0, st>>>(nnz, g->edge_nodes, (unsigned long long*)cnt);
  launch_exclusive_scan_i64(cnt, g->node_ptr, V + 1, tmp, st);
  if (E > 0)
    k_node_fill<<<blocks(E, 256), 256, 0, st>>>(E, g->edge_ptr, g->edge_nodes, g->node_ptr, fill,
                                                g->node_edges);
  // 3. heavy nodes
  if (V > 0) k_heavy<<<unsigned(g->ng), 1024, 0, st>>>(g->gvoff, g->node_ptr, g->heavy_bit);
  phase_end(ctx, kPhTranspose);
  MOCHY_HIP(hipStreamSynchronize(st));
  cleanup();
  return MOCHY_OK;
}

mochy_status project_device(mochy_ctx* ctx, mochy_graph* g) {
  hipStream_t st = ctx->stream;
  const int64_t E = g->E;
  if (g->max_graph_edges > kMaxGraphEdges) {
    ctx->err = "a graph of a batch exceeds 200000 hyperedges (the line-graph-free mode takes single graphs)";
    return MOCHY_EUNSUPPORTED;
  }
  mochy_status rc = project_incidence(ctx, g);
  if (rc != MOCHY_OK) return rc;
  const size_t tmpn = scan_tmp_elems(E + 1);
  int64_t* tmp = nullptr;
  int64_t* cnt = nullptr;
  auto cleanup = [&]() { device_free(ctx, tmp); device_free(ctx, cnt); };
  if ((rc = device_alloc(ctx, (void**)&tmp, tmpn * 8)) != MOCHY_OK ||
      (rc = device_alloc(ctx, (void**)&cnt, size_t(E + 1) * 8)) != MOCHY_OK) {
    cleanup();
    return rc;
  }
  if ((rc = device_alloc(ctx, (void**)&g->lg_ptr, size_t(E + 1) * 8)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&g->up_first, size_t(std::max<int64_t>(E, 1)) * 4)) != MOCHY_OK) { cleanup(); return rc; }
  g->bytes += size_t(E + 1) * 8 + size_t(E) * 4;

  // 4-5. degrees and row pointers
  const int nwords = int((g->max_graph_edges + 31) / 32);
  const size_t bm_bytes = size_t(std::max(nwords, 1)) * 4;
  phase_begin(ctx, kPhDegree);
  MOCHY_HIP(hipMemsetAsync(cnt, 0, size_t(E + 1) * 8, st));
  MOCHY_HIP(hipMemsetAsync(ctx->d_flags + 1, 0, sizeof(int32_t), st));
  if (E > 0)
    k_proj_degree<<<unsigned(E), 256, bm_bytes, st>>>(E, g->edge_ptr, g->edge_nodes, g->node_ptr,
                                                      g->node_edges, g->row_graph, g->geoff, cnt,
                                                      ctx->d_flags + 1);
  launch_exclusive_scan_i64(cnt, g->lg_ptr, E + 1, tmp, st);
  phase_end(ctx, kPhDegree);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, g->lg_ptr + E, 8, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small + 1, ctx->d_flags + 1, 4, hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  phases_collect(ctx);
  const int64_t twoW = ctx->h_small[0];
  g->W = twoW / 2;
  g->max_deg = *reinterpret_cast<int32_t*>(ctx->h_small + 1);

  // 6. rows
  if ((rc = device_alloc(ctx, (void**)&g->lg_col, size_t(std::max<int64_t>(twoW, 1)) * 4)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&g->rec, size_t(std::max<int64_t>(twoW, 1)) * 16)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&g->recm, size_t(std::max<int64_t>(twoW, 1)) * 4)) != MOCHY_OK) { cleanup(); return rc; }
  if ((rc = device_alloc(ctx, (void**)&g->rsz, size_t(std::max<int64_t>(twoW, 1)) * 2)) != MOCHY_OK) { cleanup(); return rc; }
  g->bytes += size_t(twoW) * 26;
  phase_begin(ctx, kPhRows);
  if (E > 0)
    k_proj_fill<<<unsigned(E), 256, bm_bytes, st>>>(E, g->edge_ptr, g->edge_nodes, g->node_ptr,
                                                    g->node_edges, g->row_graph, g->geoff, g->lg_ptr,
                                                    g->lg_col, g->up_first);
  phase_end(ctx, kPhRows);
  // 7. records (cnt, free until the upper-row prefix, holds the heavy masks)
  phase_begin(ctx, kPhRecords);
  if (E > 0) {
    unsigned long long* hmask = reinterpret_cast<unsigned long long*>(cnt);
    k_edge_heavy<<<blocks(E, 256), 256, 0, st>>>(E, g->edge_ptr, g->edge_nodes, g->heavy_bit, hmask);
    k_records<<<unsigned(E), 256, 0, st>>>(E, g->edge_ptr, g->edge_nodes, hmask, g->lg_ptr, g->lg_col,
                                           g->rec, g->recm, g->rsz, ctx->d_flags);
  }
  // upper-row prefix (hyperwedge order for sampling)
  k_upper_len<<<blocks(E + 1, 256), 256, 0, st>>>(E, g->lg_ptr, g->up_first, cnt);
  launch_exclusive_scan_i64(cnt, g->up_ptr, E + 1, tmp, st);
  phase_end(ctx, kPhRecords);
  MOCHY_HIP(hipMemcpyAsync(ctx->h_small, ctx->d_flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  MOCHY_HIP(hipStreamSynchronize(st));
  phases_collect(ctx);
  cleanup();
  const int32_t f1 = *reinterpret_cast<int32_t*>(ctx->h_small);
  if (f1 & kFlagDup) { ctx->err = "duplicate hyperedges (pass MOCHY_DEDUP for host input)"; return MOCHY_EDUP; }
  // what the on-the-fly sampler walks is built on a single graph's first
  // sampling call (mochy_count_sampled)
  return MOCHY_OK;
}
