// Weighting + spreading (the products D fhat and Omega (D fhat) of eq:cgmatrix /
// eq:twodcgmatrix): H[g] = sum_j alpha_j fhat_j prod_a exp(-beta (g_a - u_ja)^2).
//
// One workgroup owns one T x T tile of the oversampled grid. It reads the
// records binned to its tile (samples whose footprint reaches the tile),
// accumulates their taps into the tile held in LDS, and writes the tile to
// HBM once with plain, coalesced stores; tiles with no records are written as
// zeros, so the grid needs no separate clearing pass and no global atomics.
//
// Lane layout (2D): a wavefront takes 64 / (2W) records at a time (5 for
// W = 6); within a record, lane i owns footprint column i and walks the 2W
// rows. The row kernel values follow the recursion
//   e^{-beta (d+1)^2} = e^{-beta d^2} * q,  q_{next} = q * e^{-2 beta},
// so each tap costs three multiplies and two LDS float atomics.
//
// The tile accumulates in float64 LDS words with ds_add_f64 for both value
// precisions: on gfx950 the float32 LDS atomic add retires about 0.33 lanes
// per clock per CU, the float64 one about 7.6 (measured), so float64
// accumulation is both the faster and the more accurate choice. Tap values
// are formed in the plan's precision and widened before the add.
//
// With lds_copies > 1, wave w accumulates into partial tile w % copies and the
// partial tiles are combined at the flush with compensated (TwoSum) addition.
#include "ftcg_internal.h"

namespace ftcg {

constexpr int SPREAD_BLOCK = 256;

template <class real>
struct Cx;
template <>
struct Cx<float> { using t = float2; };
template <>
struct Cx<double> { using t = double2; };

__device__ inline float kexp(float x) { return __expf(x); }
__device__ inline double kexp(double x) { return exp(x); }

__device__ inline void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// compensated sum of the partial tiles at one LDS offset
template <class real>
__device__ inline real sum_copies(const real* base, int copy_stride, int copies) {
  real s = base[0];
  if (copies == 1) return s;
  real comp = (real)0;
  for (int c = 1; c < copies; ++c) {
    const real x = base[c * copy_stride];
    const real t = s + x;
    // TwoSum: exact error of s + x
    const real bp = t - s;
    const real e = (s - (t - bp)) + (x - bp);
    comp += e;
    s = t;
  }
  return s + comp;
}

template <class real, int W>
__global__ __launch_bounds__(SPREAD_BLOCK) void k_spread2d(const Rec<real>* __restrict__ recs,
                                                           const real* __restrict__ alpha_s,
                                                           const int32_t* __restrict__ tile_off,
                                                           const typename Cx<real>::t* __restrict__ fhat,
                                                           typename Cx<real>::t* __restrict__ grid, int64_t G,
                                                           int nt, int T, int copies, real beta) {
  using cx = typename Cx<real>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  const int tile = blockIdx.x;
  const int t0 = tile / nt, t1 = tile - (tile / nt) * nt;
  const int beg = tile_off[tile], end = tile_off[tile + 1];
  cx* out = grid + (int64_t)t0 * T * G + (int64_t)t1 * T;
  const int tid = threadIdx.x;
  if (beg == end) {
    const cx z = {(real)0, (real)0};
    for (int idx = tid; idx < T * T; idx += SPREAD_BLOCK) out[(int64_t)(idx / T) * G + (idx % T)] = z;
    return;
  }
  const int TP = T + 1;                 // padded row pitch
  const int plane = T * TP;             // one real plane
  const int copy_stride = 2 * plane;    // re plane + im plane
  for (int idx = tid; idx < copies * copy_stride; idx += SPREAD_BLOCK) lds[idx] = 0.0;
  __syncthreads();

  constexpr int L = 2 * W;              // lanes per record
  constexpr int RPW = 64 / L;           // records per wavefront pass
  const int wave = tid >> 6, lane = tid & 63;
  const int s = lane / L, i = lane - (lane / L) * L;
  double* mine = lds + (wave % copies) * copy_stride;
  const real e2b = kexp(-2 * beta);
  constexpr int NWAVES = SPREAD_BLOCK / 64;
  for (int base = beg + wave * RPW; base < end; base += NWAVES * RPW) {
    const int r = base + s;
    if (s < RPW && r < end) {
      const Rec<real> rec = recs[r];
      const real a = alpha_s[r];
      const cx v = fhat[rec.src];
      const int c0 = (int)(int16_t)(rec.c01 & 0xffff);
      const int c1 = rec.c01 >> 16;
      const int col = c1 - W + 1 + i;
      if (col >= 0 && col < T) {
        const real d1 = (real)(i - W + 1) - rec.f1;
        const real w1 = kexp(-beta * d1 * d1) * a;
        const real d0 = (real)(1 - W) - rec.f0;
        const real w0 = kexp(-beta * d0 * d0);
        real q = kexp(-beta * (2 * d0 + 1));
        real pr = v.x * w1 * w0, pi = v.y * w1 * w0;
        const int row0 = c0 - W + 1;
        double* pre = mine + col;
#pragma unroll
        for (int j = 0; j < L; ++j) {
          const int row = row0 + j;
          if (row >= 0 && row < T) {
            lds_add(pre + row * TP, (double)pr);
            lds_add(pre + plane + row * TP, (double)pi);
          }
          pr *= q;
          pi *= q;
          q *= e2b;
        }
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < T * T; idx += SPREAD_BLOCK) {
    const int row = idx / T, col = idx - (idx / T) * T;
    const int o = row * TP + col;
    cx val;
    val.x = (real)sum_copies(lds + o, copy_stride, copies);
    val.y = (real)sum_copies(lds + plane + o, copy_stride, copies);
    out[(int64_t)row * G + col] = val;
  }
}

// 1D: one thread per record walks its 2W taps
template <class real, int W>
__global__ __launch_bounds__(SPREAD_BLOCK) void k_spread1d(const Rec<real>* __restrict__ recs,
                                                           const real* __restrict__ alpha_s,
                                                           const int32_t* __restrict__ tile_off,
                                                           const typename Cx<real>::t* __restrict__ fhat,
                                                           typename Cx<real>::t* __restrict__ grid, int T, int copies,
                                                           real beta) {
  using cx = typename Cx<real>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* lds = reinterpret_cast<double*>(smem_raw);
  const int tile = blockIdx.x;
  const int beg = tile_off[tile], end = tile_off[tile + 1];
  cx* out = grid + (int64_t)tile * T;
  const int tid = threadIdx.x;
  const int copy_stride = 2 * T;
  for (int idx = tid; idx < copies * copy_stride; idx += SPREAD_BLOCK) lds[idx] = 0.0;
  __syncthreads();
  double* mine = lds + ((tid >> 6) % copies) * copy_stride;
  const real e2b = kexp(-2 * beta);
  for (int r = beg + tid; r < end; r += SPREAD_BLOCK) {
    const Rec<real> rec = recs[r];
    const real a = alpha_s[r];
    const cx v = fhat[rec.src];
    const int c0 = (int)(int16_t)(rec.c01 & 0xffff);
    const real d0 = (real)(1 - W) - rec.f0;
    real q = kexp(-beta * (2 * d0 + 1));
    const real w0 = kexp(-beta * d0 * d0) * a;
    real pr = v.x * w0, pi = v.y * w0;
    const int cell0 = c0 - W + 1;
#pragma unroll
    for (int j = 0; j < 2 * W; ++j) {
      const int cell = cell0 + j;
      if (cell >= 0 && cell < T) {
        lds_add(mine + cell, (double)pr);
        lds_add(mine + T + cell, (double)pi);
      }
      pr *= q;
      pi *= q;
      q *= e2b;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < T; idx += SPREAD_BLOCK) {
    cx val;
    val.x = (real)sum_copies(lds + idx, copy_stride, copies);
    val.y = (real)sum_copies(lds + T + idx, copy_stride, copies);
    out[idx] = val;
  }
}

template <class real, int W>
static void launch_spread_w(ftcg_plan p, const void* fhat, void* grid) {
  using cx = typename Cx<real>::t;
  const int T = p->tile;
  const real beta = (real)p->beta;
  const int copies = p->lds_copies;
  if (p->dim == 2) {
    const size_t lds = (size_t)copies * 2 * T * (T + 1) * sizeof(double);
    static bool attr_done = false;
    if (!attr_done) {
      FTCG_HIP(hipFuncSetAttribute((const void*)k_spread2d<real, W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024));
      attr_done = true;
    }
    hipLaunchKernelGGL((k_spread2d<real, W>), dim3((unsigned)p->ntiles), dim3(SPREAD_BLOCK), lds, p->stream,
                       p->recs.as<Rec<real>>(), p->alpha_s.as<real>(), p->tile_off.as<int32_t>(),
                       static_cast<const cx*>(fhat), static_cast<cx*>(grid), p->G, (int)p->nt, T, copies, beta);
  } else {
    const size_t lds = (size_t)copies * 2 * T * sizeof(double);
    hipLaunchKernelGGL((k_spread1d<real, W>), dim3((unsigned)p->ntiles), dim3(SPREAD_BLOCK), lds, p->stream,
                       p->recs.as<Rec<real>>(), p->alpha_s.as<real>(), p->tile_off.as<int32_t>(),
                       static_cast<const cx*>(fhat), static_cast<cx*>(grid), T, copies, beta);
  }
  FTCG_HIP(hipGetLastError());
}

template <class real>
static void launch_spread_t(ftcg_plan p, const void* fhat, void* grid) {
  switch (p->W) {
    case 2: launch_spread_w<real, 2>(p, fhat, grid); break;
    case 3: launch_spread_w<real, 3>(p, fhat, grid); break;
    case 4: launch_spread_w<real, 4>(p, fhat, grid); break;
    case 5: launch_spread_w<real, 5>(p, fhat, grid); break;
    case 6: launch_spread_w<real, 6>(p, fhat, grid); break;
    case 7: launch_spread_w<real, 7>(p, fhat, grid); break;
    case 8: launch_spread_w<real, 8>(p, fhat, grid); break;
    default: throw StatusError{FTCG_EUNSUPPORTED};
  }
}

void spread(ftcg_plan p, const void* fhat, void* grid) {
  if (p->dtype == FTCG_F64)
    launch_spread_t<double>(p, fhat, grid);
  else
    launch_spread_t<float>(p, fhat, grid);
}

}  // namespace ftcg
