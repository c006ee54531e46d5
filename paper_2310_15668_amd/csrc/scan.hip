// Exclusive prefix sum of int64 arrays (row pointers of the CSR structures).
// Tile of 1024 elements per 256-thread block, tile sums scanned recursively,
// then added back.
#include <algorithm>

#include "common.h"

namespace {

constexpr int kTile = 1024;

__global__ __launch_bounds__(256) void k_scan_tile(const int64_t* in, int64_t* out,
                                                   int64_t n, int64_t* sums) {
  __shared__ int64_t part[256];
  const int64_t base = int64_t(blockIdx.x) * kTile + threadIdx.x * 4;
  int64_t v[4];
  int64_t run = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t x = (base + q < n) ? in[base + q] : 0;
    v[q] = run;
    run += x;
  }
  part[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan of the 256 thread totals
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t add = threadIdx.x >= unsigned(off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  const int64_t before = threadIdx.x ? part[threadIdx.x - 1] : 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (base + q < n) out[base + q] = before + v[q];
  if (threadIdx.x == 255) sums[blockIdx.x] = part[255];
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < n; x += int64_t(gridDim.x) * blockDim.x)
    p[x] = v;
}

__global__ void k_add_tile_offsets(int64_t* out, int64_t n, const int64_t* __restrict__ offs) {
  const int64_t x = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (x < n) out[x] += offs[x / kTile];
}

}  // namespace

size_t scan_tmp_elems(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  do {
    m = (m + kTile - 1) / kTile;
    total += size_t(m) + 1;
  } while (m > 1);
  return total + 8;
}

void launch_exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp,
                               hipStream_t s) {
  if (n <= 0) return;
  const int64_t tiles = (n + kTile - 1) / kTile;
  k_scan_tile<<<dim3(unsigned(tiles)), 256, 0, s>>>(in, out, n, tmp);
  if (tiles > 1) {
    launch_exclusive_scan_i64(tmp, tmp, tiles, tmp + tiles + 1, s);
    k_add_tile_offsets<<<dim3(unsigned((n + 255) / 256)), 256, 0, s>>>(out, n, tmp);
  }
}

void launch_fill_u32(void* p, uint32_t value, size_t bytes, hipStream_t s) {
  const int64_t n = int64_t(bytes / 4);
  if (n <= 0) return;
  const int64_t nb = std::min<int64_t>((n + 255) / 256, 4096);
  k_fill_u32<<<dim3(unsigned(nb)), 256, 0, s>>>(static_cast<uint32_t*>(p), value, n);
}
