// Exclusive prefix sum of int32 counts (tile and bin offsets of the counting sorts).
//
// Up to 16384 entries: one launch of one 1024-thread workgroup (the pair
// scan walks up to SCAN_SINGLE_MAX entries in chunks of 16384, carrying the
// running total). Beyond that, three launches: per-block sums, a single-block scan of the block
// sums, then a per-block scan that adds its block offset, each block covering
// SCAN_BLOCK * SCAN_ITEMS consecutive entries. out[n] receives the total.
// When `cursor` is given, out[0..n) is written there too (it may be `in`
// itself: every entry is read by the thread that later overwrites it), which
// gives the counting sorts their scatter cursors without another copy.
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

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_final(const int32_t* in, int64_t n,
                                                           const int32_t* __restrict__ sums,
                                                           int32_t* __restrict__ out, int32_t* cursor) {
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
    if (idx < n) {
      out[idx] = run;
      if (cursor) cursor[idx] = run;
    }
    run += v[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) out[n] = run;
}

constexpr int SS_BLOCK = 1024;
constexpr int SS_ITEMS = 16;
constexpr int64_t SCAN_SINGLE_MAX = 8 * SS_BLOCK * SS_ITEMS;

__device__ inline int32_t wave_inclusive_scan(int32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  return v;
}

// one chunk of SS_BLOCK * SS_ITEMS entries passes through LDS so that global
// loads and stores are coalesced while each thread scans SS_ITEMS consecutive
// entries; entry e sits at LDS word e + e / 16 (conflict-free at stride 16)
__device__ inline int ss_pad(int e) { return e + (e >> 4); }

// ITEMS entries per thread and chunk (ITEMS, or fewer for short arrays,
// which then pass through less LDS)
template <int ITEMS>
__device__ void scan_single_block(const int32_t* in, int64_t n, int32_t* __restrict__ out, int32_t* cursor) {
  constexpr int CH = SS_BLOCK * ITEMS;
  __shared__ int32_t buf[CH + CH / 16];
  __shared__ int32_t wsum[SS_BLOCK / 64];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < n; c0 += CH) {
    const int64_t len = n - c0 < CH ? n - c0 : CH;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = i * SS_BLOCK + t;
      buf[ss_pad(e)] = e < len ? in[c0 + e] : 0;
    }
    __syncthreads();
    int32_t v[ITEMS];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      v[i] = buf[ss_pad(t * ITEMS + i)];
      s += v[i];
    }
    const int32_t incl = wave_inclusive_scan(s);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t wpre = 0, tot = 0;
#pragma unroll
    for (int j = 0; j < SS_BLOCK / 64; ++j) {
      const int32_t x = wsum[j];
      wpre += j < w ? x : 0;
      tot += x;
    }
    int32_t run = carry + wpre + incl - s;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      buf[ss_pad(t * ITEMS + i)] = run;
      run += v[i];
    }
    carry += tot;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int e = i * SS_BLOCK + t;
      if (e < len) {
        const int32_t x = buf[ss_pad(e)];
        out[c0 + e] = x;
        if (cursor) cursor[c0 + e] = x;
      }
    }
    __syncthreads();  // buf and wsum are rewritten by the next chunk
  }
  if (t == 0) out[n] = carry;
}

template <int ITEMS>
__global__ __launch_bounds__(SS_BLOCK) void k_scan_single(const int32_t* in, int64_t n, int32_t* __restrict__ out,
                                                          int32_t* cursor) {
  scan_single_block<ITEMS>(in, n, out, cursor);
}

// two independent single-workgroup scans in one launch (workgroup b scans
// array b)
template <int ITEMS>
__global__ __launch_bounds__(SS_BLOCK) void k_scan_pair(const int32_t* in0, int64_t n0, int32_t* __restrict__ out0,
                                                        int32_t* cursor0, const int32_t* in1, int64_t n1,
                                                        int32_t* __restrict__ out1, int32_t* cursor1) {
  if (blockIdx.x == 0)
    scan_single_block<ITEMS>(in0, n0, out0, cursor0);
  else
    scan_single_block<ITEMS>(in1, n1, out1, cursor1);
}

void exclusive_scan_pair_i32(const int32_t* in0, int32_t* out0, int64_t n0, int32_t* cursor0, const int32_t* in1,
                             int32_t* out1, int64_t n1, int32_t* cursor1, hipStream_t s) {
  if (n0 > SCAN_SINGLE_MAX || n1 > SCAN_SINGLE_MAX) throw StatusError{FTCG_EUNSUPPORTED};
  // arrays of at most 4 entries per thread (the 512^2 raster's tiles and
  // bin rows) take one pass through 16 KiB of LDS instead of 64 KiB
  if (n0 <= 4 * SS_BLOCK && n1 <= 4 * SS_BLOCK)
    hipLaunchKernelGGL(k_scan_pair<4>, dim3(2), dim3(SS_BLOCK), 0, s, in0, n0, out0, cursor0, in1, n1, out1,
                       cursor1);
  else
    hipLaunchKernelGGL(k_scan_pair<SS_ITEMS>, dim3(2), dim3(SS_BLOCK), 0, s, in0, n0, out0, cursor0, in1, n1, out1,
                       cursor1);
  FTCG_HIP(hipGetLastError());
}

size_t scan_tmp_bytes(int64_t n) {
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  return (size_t)(nb + 1) * sizeof(int32_t);
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s, int32_t* cursor) {
  if (n <= 4 * SS_BLOCK) {   // one pass through 16 KiB of LDS
    hipLaunchKernelGGL(k_scan_single<4>, dim3(1), dim3(SS_BLOCK), 0, s, in, n, out, cursor);
    FTCG_HIP(hipGetLastError());
    return;
  }
  // one workgroup walks at most one chunk: beyond that, its chunks' loads
  // wait one after another (65 536 entries: 29 us in one workgroup)
  if (n <= SS_BLOCK * SS_ITEMS) {
    hipLaunchKernelGGL(k_scan_single<SS_ITEMS>, dim3(1), dim3(SS_BLOCK), 0, s, in, n, out, cursor);
    FTCG_HIP(hipGetLastError());
    return;
  }
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb < 1) nb = 1;
  if (nb > SCAN_MAX_BLOCKS) throw StatusError{FTCG_EUNSUPPORTED};
  hipLaunchKernelGGL(k_scan_block_sums, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BLOCK), 0, s, tmp, (int)nb);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, tmp, out, cursor);
  FTCG_HIP(hipGetLastError());
}

}  // namespace ftcg
