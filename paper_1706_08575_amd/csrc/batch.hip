// Batched execution: many independent pings (items) with uneven sample counts
// and image sizes in one persistent spreading launch, followed by batched
// inverse-FFT passes; the whole sequence is replayed from a captured hipGraph.
//
// Work decomposition: every tile of every item becomes one or more tasks of at
// most `chunk` records. A fixed grid of workgroups pulls tasks from a global
// counter in the order of the task table (built heaviest first), so a few
// dense tiles cannot stall the launch. All tasks of a tile share the tile's
// bound (computed first, from order-independent reductions) and therefore the
// same fixed-point scale: a tile with one task writes its floats directly; the
// tasks of a split tile add their exact packed integers into a 64-bit scratch
// tile with global integer atomics (order-independent), and a last pass
// converts those tiles to floats.
//
// Kernels read the value and image pointers of the current call from a small
// device argument block, so the captured graph is replayed unchanged; the
// caller's pointers are written into that block before each replay.
#include "batch_internal.h"

using ftcg_batch = ftcg_batch_s*;

namespace ftcg {

constexpr int BATCH_BLOCK = 256;

__device__ inline float2 z2() {
  float2 z;
  z.x = 0.f;
  z.y = 0.f;
  return z;
}

// bound of every tile (the same order-independent formula as the single-plan
// spreading kernel) -> bounds[tile id]; 0 for empty tiles
__global__ __launch_bounds__(BATCH_BLOCK) void k_batch_bounds(const BatchTile* __restrict__ tiles, int ntiles,
                                                             const BatchItem* __restrict__ items,
                                                             const BatchArgs* __restrict__ args,
                                                             float* __restrict__ bounds) {
  __shared__ float red[BATCH_BLOCK / 64];
  __shared__ long long red2[BATCH_BLOCK / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BatchTile tl = tiles[t];
    const BatchItem it = items[tl.item];
    const float2* fhat = args->fhat + it.fhat_off;
    float mx = 0.f;
    for (int r = tl.beg + tid; r < tl.end; r += BATCH_BLOCK) {
      const float a = it.alpha_s[r];
      const float2 v = fhat[it.recs[r].src];
      const float cr = v.x * a, ci = v.y * a;
    // fmaxf drops NaN operands: flag non-finite values explicitly
    mx = (isfinite(cr) && isfinite(ci)) ? fmaxf(mx, fmaxf(fabsf(cr), fabsf(ci))) : __builtin_inff();
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    mx = 0.f;
    for (int w = 0; w < BATCH_BLOCK / 64; ++w) mx = fmaxf(mx, red[w]);
    long long qsum = 0;
    if (mx > 0.f && isfinite(mx)) {
      const float qs = 1048576.f / mx;
      for (int r = tl.beg + tid; r < tl.end; r += BATCH_BLOCK) {
        const float a = it.alpha_s[r];
        const float2 v = fhat[it.recs[r].src];
        qsum += (long long)ceilf(fmaxf(fabsf(v.x * a), fabsf(v.y * a)) * qs) + 1;
      }
    }
    for (int off = 32; off > 0; off >>= 1) qsum += __shfl_xor(qsum, off);
    if (lane == 0) red2[wave] = qsum;
    __syncthreads();
    if (tid == 0) {
      long long q = 0;
      for (int w = 0; w < BATCH_BLOCK / 64; ++w) q += red2[w];
      float b;
      if (!(mx >= 0.f) || !isfinite(mx)) b = __builtin_nanf("");
      else if (mx == 0.f) b = 0.f;
      else b = (float)((double)q * (double)mx * (1.0 / 1048576.0) * (1.0 + 1e-6));
      bounds[t] = b;
    }
    __syncthreads();
  }
}

// graph-safe clearing: task counter and the 64-bit scratch of split tiles
__global__ void k_batch_clear(unsigned long long* __restrict__ scratch, int64_t nwords, int* __restrict__ counter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *counter = 0;
  for (int64_t w = i; w < nwords; w += (int64_t)gridDim.x * blockDim.x) scratch[w] = 0ull;
}

template <int W, int T>
__global__ __launch_bounds__(BATCH_BLOCK) void k_spread_persistent(const BatchTask* __restrict__ tasks, int ntasks,
                                                                  const BatchTile* __restrict__ tiles,
                                                                  const BatchItem* __restrict__ items,
                                                                  const BatchArgs* __restrict__ args,
                                                                  const float* __restrict__ bounds,
                                                                  unsigned long long* __restrict__ scratch,
                                                                  int* __restrict__ counter) {
  constexpr int L = 2 * W;
  constexpr int PAD = 2 * W - 1;
  constexpr int TP = T + 1;
  constexpr int ROWS = T + 2 * PAD;
  constexpr int RPW = 64 / L;
  constexpr int NWAVES = BATCH_BLOCK / 64;
  __shared__ unsigned long long acc[ROWS * TP];
  __shared__ int task_sh;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int s = lane / L, i = lane - (lane / L) * L;
  const float scale_num = 2147483648.f - 16777216.f;
  for (;;) {
    if (tid == 0) task_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int t = task_sh;
    __syncthreads();
    if (t >= ntasks) break;
    const BatchTask tk = tasks[t];
    const BatchTile tl = tiles[tk.tile];
    const BatchItem it = items[tl.item];
    float2* out = args->grid + it.grid_off + (int64_t)tl.t0 * T * it.G + (int64_t)tl.t1 * T;
    const float bound = bounds[tk.tile];
    if (!(bound > 0.f) || !isfinite(bound)) {
      // empty (or all-zero) tile, or non-finite values: only the first task writes
      if (tk.part == 0) {
        const float fill = bound == 0.f ? 0.f : __builtin_nanf("");
        float2 z;
        z.x = fill;
        z.y = fill;
        for (int idx = tid; idx < T * T; idx += BATCH_BLOCK) out[(int64_t)(idx / T) * it.G + (idx % T)] = z;
      }
      continue;
    }
    const float scale = scale_num / bound;
    const float beta = it.beta;
    const float e2b = __expf(-2.f * beta);
    const float2* fhat = args->fhat + it.fhat_off;
    for (int idx = tid; idx < ROWS * TP; idx += BATCH_BLOCK) acc[idx] = 0ull;
    __syncthreads();
    for (int base = tk.beg + wave * RPW; base < tk.end; base += NWAVES * RPW) {
      const int r = base + s;
      if (s < RPW && r < tk.end) {
        const Rec<float> rec = it.recs[r];
        const int c1 = rec.c01 >> 16;
        const int col = c1 - W + 1 + i;
        if (col >= 0 && col < T) {
          const float a = it.alpha_s[r] * scale;
          const float2 v = fhat[rec.src];
          const int c0 = (int)(int16_t)(rec.c01 & 0xffff);
          const float d1 = (float)(i - W + 1) - rec.f1;
          const float d0 = (float)(1 - W) - rec.f0;
          const float w10 = __expf(-beta * (d1 * d1 + d0 * d0)) * a;
          float q = __expf(-beta * (2.f * d0 + 1.f));
          float pr = v.x * w10, pi = v.y * w10;
          unsigned long long* dst = acc + (c0 - W + 1 + PAD) * TP + col;
#pragma unroll
          for (int j = 0; j < L; ++j) {
            __hip_atomic_fetch_add(dst + j * TP, fx_pack(pr, pi), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            pr *= q;
            pi *= q;
            q *= e2b;
          }
        }
      }
    }
    __syncthreads();
    if (tl.split < 0) {
      const float inv = bound / scale_num;
      for (int idx = tid; idx < T * T; idx += BATCH_BLOCK) {
        const int row = idx / T, col = idx - (idx / T) * T;
        const unsigned long long vv = acc[(row + PAD) * TP + col];
        const int re = (int)(unsigned)(vv & 0xffffffffull);
        const int im = (int)((long long)(vv - (unsigned long long)(long long)re) >> 32);
        float2 o;
        o.x = (float)re * inv;
        o.y = (float)im * inv;
        out[(int64_t)row * it.G + col] = o;
      }
    } else {
      unsigned long long* sc = scratch + (int64_t)tl.split * T * T;
      for (int idx = tid; idx < T * T; idx += BATCH_BLOCK) {
        const int row = idx / T, col = idx - (idx / T) * T;
        const unsigned long long vv = acc[(row + PAD) * TP + col];
        if (vv) atomicAdd(&sc[idx], vv);
      }
    }
    __syncthreads();
  }
}

// split tiles: packed integer sums -> floats
template <int T>
__global__ __launch_bounds__(BATCH_BLOCK) void k_batch_finalize(const int* __restrict__ split_tiles, int nsplit,
                                                               const BatchTile* __restrict__ tiles,
                                                               const BatchItem* __restrict__ items,
                                                               const BatchArgs* __restrict__ args,
                                                               const float* __restrict__ bounds,
                                                               const unsigned long long* __restrict__ scratch) {
  const float scale_num = 2147483648.f - 16777216.f;
  for (int sidx = blockIdx.x; sidx < nsplit; sidx += gridDim.x) {
    const int tile = split_tiles[sidx];
    const BatchTile tl = tiles[tile];
    const BatchItem it = items[tl.item];
    const float bound = bounds[tile];
    if (!(bound > 0.f) || !isfinite(bound)) continue;   // written by the spreading kernel
    const float inv = bound / scale_num;
    float2* out = args->grid + it.grid_off + (int64_t)tl.t0 * T * it.G + (int64_t)tl.t1 * T;
    const unsigned long long* sc = scratch + (int64_t)tl.split * T * T;
    for (int idx = threadIdx.x; idx < T * T; idx += BATCH_BLOCK) {
      const unsigned long long vv = sc[idx];
      const int re = (int)(unsigned)(vv & 0xffffffffull);
      const int im = (int)((long long)(vv - (unsigned long long)(long long)re) >> 32);
      float2 o;
      o.x = (float)re * inv;
      o.y = (float)im * inv;
      out[(int64_t)(idx / T) * it.G + (idx % T)] = o;
    }
  }
}

template <int W, int T>
static void launch_spread_wt(ftcg_batch b) {
  hipLaunchKernelGGL((k_spread_persistent<W, T>), dim3(b->persistent_blocks), dim3(BATCH_BLOCK), 0, b->stream,
                     b->tasks.as<BatchTask>(), (int)b->ntasks, b->tiles.as<BatchTile>(), b->items_dev.as<BatchItem>(),
                     b->args_dev.as<BatchArgs>(), b->bounds.as<float>(), b->scratch.as<unsigned long long>(),
                     b->counter.as<int>());
  if (b->nsplit > 0) {
    const unsigned nb = (unsigned)(b->nsplit < 4096 ? b->nsplit : 4096);
    hipLaunchKernelGGL((k_batch_finalize<T>), dim3(nb), dim3(BATCH_BLOCK), 0, b->stream,
                       b->split_tiles.as<int>(), (int)b->nsplit, b->tiles.as<BatchTile>(),
                       b->items_dev.as<BatchItem>(), b->args_dev.as<BatchArgs>(), b->bounds.as<float>(),
                       b->scratch.as<unsigned long long>());
  }
}

template <int W>
static void launch_spread_w(ftcg_batch b) {
  switch (b->tile) {
    case 16: launch_spread_wt<W, 16>(b); break;
    case 32: launch_spread_wt<W, 32>(b); break;
    case 64: launch_spread_wt<W, 64>(b); break;
    case 128: launch_spread_wt<W, 128>(b); break;
    default: throw StatusError{FTCG_EUNSUPPORTED};
  }
}

void batch_spread(ftcg_batch b) {
  const int64_t nw = b->nsplit * (int64_t)b->tile * b->tile;
  hipLaunchKernelGGL(k_batch_clear, dim3(nw > 0 ? (unsigned)((nw + 255) / 256 < 8192 ? (nw + 255) / 256 : 8192) : 1),
                     dim3(256), 0, b->stream, b->scratch.as<unsigned long long>(), nw, b->counter.as<int>());
  const unsigned nbb = (unsigned)(b->ntiles < 8192 ? b->ntiles : 8192);
  hipLaunchKernelGGL(k_batch_bounds, dim3(nbb), dim3(BATCH_BLOCK), 0, b->stream, b->tiles.as<BatchTile>(),
                     (int)b->ntiles, b->items_dev.as<BatchItem>(), b->args_dev.as<BatchArgs>(), b->bounds.as<float>());
  switch (b->W) {
    case 2: launch_spread_w<2>(b); break;
    case 3: launch_spread_w<3>(b); break;
    case 4: launch_spread_w<4>(b); break;
    case 5: launch_spread_w<5>(b); break;
    case 6: launch_spread_w<6>(b); break;
    case 7: launch_spread_w<7>(b); break;
    case 8: launch_spread_w<8>(b); break;
    default: throw StatusError{FTCG_EUNSUPPORTED};
  }
  FTCG_HIP(hipGetLastError());
}

}  // namespace ftcg
