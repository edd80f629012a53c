// Exclusive prefix sum of int32 counts (tile and bin offsets of the counting sorts).
//
// Three launches: per-block sums, a single-block scan of the block sums,
// then a per-block scan that adds its block offset. Each block covers
// SCAN_BLOCK * SCAN_ITEMS consecutive entries. out[n] receives the total.
#include "ftcg_internal.h"

namespace ftcg {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;   // 2048 entries per block
constexpr int SCAN_MAX_BLOCKS = SCAN_BLOCK * 64;     // second level: one block, 64 items/thread

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* lds, int32_t* total) {
  // Hillis-Steele over the block in LDS (256 entries)
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
    int32_t add = (t >= off) ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  int32_t incl = lds[t];
  *total = lds[SCAN_BLOCK - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_block_sums(const int32_t* __restrict__ in, int64_t n,
                                                                int32_t* __restrict__ sums) {
  __shared__ int32_t lds[SCAN_BLOCK];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int32_t s = 0;
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  int32_t tot;
  (void)block_exclusive_scan(s, lds, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_sums(int32_t* __restrict__ sums, int nblocks) {
  // in-place exclusive scan of nblocks <= SCAN_MAX_BLOCKS block sums
  __shared__ int32_t lds[SCAN_BLOCK];
  constexpr int PER = SCAN_MAX_BLOCKS / SCAN_BLOCK;
  int32_t v[PER];
  int32_t s = 0;
  const int base = threadIdx.x * PER;
  for (int i = 0; i < PER; ++i) {
    int idx = base + i;
    v[i] = (idx < nblocks) ? sums[idx] : 0;
    s += v[i];
  }
  int32_t tot;
  int32_t run = block_exclusive_scan(s, lds, &tot);
  for (int i = 0; i < PER; ++i) {
    int idx = base + i;
    if (idx < nblocks) sums[idx] = run;
    run += v[i];
  }
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_final(const int32_t* __restrict__ in, int64_t n,
                                                           const int32_t* __restrict__ sums,
                                                           int32_t* __restrict__ out) {
  __shared__ int32_t lds[SCAN_BLOCK];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t s = 0;
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    v[i] = (idx < n) ? in[idx] : 0;
    s += v[i];
  }
  int32_t tot;
  int32_t run = block_exclusive_scan(s, lds, &tot) + sums[blockIdx.x];
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t idx = base + i;
    if (idx < n) out[idx] = run;
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) out[n] = run;
}

size_t scan_tmp_bytes(int64_t n) {
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  return (size_t)(nb + 1) * sizeof(int32_t);
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s) {
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb < 1) nb = 1;
  if (nb > SCAN_MAX_BLOCKS) throw StatusError{FTCG_EUNSUPPORTED};
  hipLaunchKernelGGL(k_scan_block_sums, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BLOCK), 0, s, tmp, (int)nb);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, tmp, out);
  FTCG_HIP(hipGetLastError());
}

}  // namespace ftcg
