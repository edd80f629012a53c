// Forward (type-2) transform: image on the n^d pixel grid -> values at the
// raster, fhat_j ~ sum_p I[p] exp(-2 pi i k_j . x_p). It is the adjoint of
// the reconstruction of eq:cgmatrix (Omega^T after the forward DFT of the
// deapodized, zero-padded image), the operator that the frame approximation's
// Psi and the iterative weights of the cited density compensation apply.
//
// Steps:
//   1. forward FFT passes (fft.hip): columns of the image times the
//      deapodization factors, zero-padded to G, transformed, each written as
//      a contiguous row; in 2D the second pass transforms the G columns of
//      that intermediate into H (G x G, the grid's own layout);
//   2. interpolation: fhat_j = sum over the 2W x 2W taps of H[g]
//      prod_a exp(-beta (g_a - u_ja)^2), the taps of the spread. One
//      workgroup per square of ST x ST cells (S x S tiles of the spread's
//      binning, ST = 32, or 64 for tiles of 64 in float32) stages that square's
//      window of H (its ST + 2W - 1 rows and columns, indices modulo G) in
//      LDS with coalesced loads, and walks the records of its tiles one per
//      lane, keeping each sample's home record only (the record in the tile
//      that holds its cell floor(u), so every sample is computed once): the
//      lane forms the 2W column factors once, and for each row adds
//      the row's taps against them (two fused multiply-adds and one LDS read
//      per tap) before scaling the row sum by the row factor (rows by the
//      centre of each axis outward). Squares wider than LDS allows (tile 128, or
//      tile 64 in float64) use one workgroup per tile and 16 lanes per
//      record instead (lane i = footprint column i < 2W, the lanes' partial
//      sums added by shuffles), walking the tile's records and skipping the
//      ones that are not home.
#include "ftcg_internal.h"

namespace ftcg {

constexpr int FWD_BLOCK = 256;

template <class real>
struct CxI;
template <>
struct CxI<float> { using t = float2; };
template <>
struct CxI<double> { using t = double2; };

__device__ inline float iexp(float x) { return __expf(x); }
__device__ inline double iexp(double x) { return exp(x); }

template <class real, int W>
__global__ __launch_bounds__(FWD_BLOCK) void k_interp2d(const Rec<real>* __restrict__ recs,
                                                       const int32_t* __restrict__ tile_off,
                                                       const typename CxI<real>::t* __restrict__ grid, int64_t G,
                                                       int nt, int T, real beta,
                                                       typename CxI<real>::t* __restrict__ fhat) {
  using cx = typename CxI<real>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx* win = reinterpret_cast<cx*>(smem_raw);
  const int tile = blockIdx.x;
  const int beg = tile_off[tile], end = tile_off[tile + 1];
  if (beg == end) return;
  const int t0 = tile / nt, t1 = tile - (tile / nt) * nt;
  const int WS = T + 2 * W - 1;                 // window edge
  const int64_t g0 = (int64_t)t0 * T - (W - 1), g1 = (int64_t)t1 * T - (W - 1);
  for (int idx = threadIdx.x; idx < WS * WS; idx += FWD_BLOCK) {
    const int r = idx / WS, c = idx - (idx / WS) * WS;
    int64_t gr = g0 + r, gc = g1 + c;
    gr = gr < 0 ? gr + G : (gr >= G ? gr - G : gr);
    gc = gc < 0 ? gc + G : (gc >= G ? gc - G : gc);
    win[idx] = grid[gr * G + gc];
  }
  __syncthreads();
  constexpr int L = 2 * W;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = lane >> 4, i = lane & 15;
  const real e2b = iexp((real)-2 * beta);
  for (int base = beg + wave * 4; base < end; base += (FWD_BLOCK / 64) * 4) {
    const int r = base + s;
    real ar = 0, ai = 0;
    bool home = false;
    Rec<real> rec;
    if (r < end) {
      rec = recs[r];
      const int c0 = (int)(int16_t)(rec.c01 & 0xffff), c1 = rec.c01 >> 16;
      home = c0 >= 0 && c0 < T && c1 >= 0 && c1 < T;
      if (home && i < L) {
        const real d1 = (real)(i - W + 1) - rec.f1;
        const real d0 = (real)(1 - W) - rec.f0;
        real w = iexp(-beta * (d0 * d0 + d1 * d1));
        real q = iexp(-beta * ((real)2 * d0 + (real)1));
        const cx* p = win + c0 * WS + c1 + i;
#pragma unroll
        for (int j = 0; j < L; ++j) {
          const cx v = p[j * WS];
          ar += w * v.x;
          ai += w * v.y;
          w *= q;
          q *= e2b;
        }
      }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      ar += __shfl_xor(ar, off, 64);
      ai += __shfl_xor(ai, off, 64);
    }
    if (home && i == 0) {
      cx o;
      o.x = ar;
      o.y = ai;
      fhat[rec.src] = o;
    }
  }
}


// the 2W kernel values exp(-beta (c - W + 1 - f)^2), c < 2W, of one axis
// (f the fractional position): the largest, at c = W - 1, from an exponent
// of at most beta in size, then outward by the ratio recursion in both
// directions, so the large taps carry the exponential's error at a small
// argument (an exponential at the footprint's edge, argument near -W^2 beta,
// would put |argument| x 2^-24 of relative error on every tap of the sample)
template <class real, int W>
__device__ inline void gauss_taps(real f, real beta, real e2b, real (&out)[2 * W]) {
  out[W - 1] = iexp(-beta * f * f);
  real qu = iexp(-beta * ((real)1 - (real)2 * f)), qd = iexp(-beta * ((real)1 + (real)2 * f));
#pragma unroll
  for (int c = W; c < 2 * W; ++c) {
    out[c] = out[c - 1] * qu;
    qu *= e2b;
  }
#pragma unroll
  for (int c = W - 2; c >= 0; --c) {
    out[c] = out[c + 1] * qd;
    qd *= e2b;
  }
}


template <class real, int W, int T, int ST>
__global__ __launch_bounds__(FWD_BLOCK) void k_interp2d_sq(const Rec<real>* __restrict__ recs,
                                                           const int32_t* __restrict__ tile_off,
                                                           const typename CxI<real>::t* __restrict__ grid,
                                                           int64_t G, int nt, real beta,
                                                           typename CxI<real>::t* __restrict__ fhat) {
  using cx = typename CxI<real>::t;
  constexpr int S = ST / T;             // tiles per edge of the square
  constexpr int L = 2 * W;
  constexpr int WS = ST + L - 1;        // window edge
  __shared__ cx win[WS * WS];
  const int tid = threadIdx.x;
  const int nsq = nt / S;
  const int sq = (int)xcd_block(blockIdx.x, gridDim.x);
  const int sr = sq / nsq, sc = sq - (sq / nsq) * nsq;
  const int64_t g0 = (int64_t)sr * ST - (W - 1), g1 = (int64_t)sc * ST - (W - 1);
  for (int idx = tid; idx < WS * WS; idx += FWD_BLOCK) {
    const int r = idx / WS, c = idx - (idx / WS) * WS;
    int64_t gr = g0 + r, gc = g1 + c;
    gr = gr < 0 ? gr + G : (gr >= G ? gr - G : gr);
    gc = gc < 0 ? gc + G : (gc >= G ? gc - G : gc);
    win[idx] = grid[gr * G + gc];
  }
  __syncthreads();
  const real e2b = iexp((real)-2 * beta);
  for (int k = 0; k < S; ++k) {
    // the S tiles of this row of the square hold one contiguous record range
    const int id0 = (sr * S + k) * nt + sc * S;
    const int rbeg = tile_off[id0], rend = tile_off[id0 + S];
    int bnd[S > 1 ? S - 1 : 1];
#pragma unroll
    for (int q = 1; q < S; ++q) bnd[q - 1] = tile_off[id0 + q];
    for (int r = rbeg + tid; r < rend; r += FWD_BLOCK) {
      const Rec<real> rec = recs[r];
      const int c0 = (int)(int16_t)(rec.c01 & 0xffff), c1 = rec.c01 >> 16;
      if (c0 < 0 || c0 >= T || c1 < 0 || c1 >= T) continue;   // not the sample's home record
      int q = 0;
#pragma unroll
      for (int m = 1; m < S; ++m) q += r >= bnd[m - 1];
      real a[L], b[L];
      gauss_taps<real, W>(rec.f0, beta, e2b, a);
      gauss_taps<real, W>(rec.f1, beta, e2b, b);
      const cx* p = win + (c0 + k * T) * WS + c1 + q * T;
      real ar = 0, ai = 0;
#pragma unroll 2   // two rows of reads in flight (all 2W rows would hold them all in registers)
      for (int j = 0; j < L; ++j) {
        real sr_ = 0, si_ = 0;
#pragma unroll
        for (int c = 0; c < L; ++c) {
          const cx v = p[j * WS + c];
          sr_ += b[c] * v.x;
          si_ += b[c] * v.y;
        }
        ar += a[j] * sr_;
        ai += a[j] * si_;
      }
      cx o;
      o.x = ar;
      o.y = ai;
      fhat[rec.src] = o;
    }
  }
}

// 1D: one workgroup per tile, one thread per home record, 2W taps from global memory
template <class real, int W>
__global__ __launch_bounds__(FWD_BLOCK) void k_interp1d_tiles(const Rec<real>* __restrict__ recs,
                                                             const int32_t* __restrict__ tile_off,
                                                             const typename CxI<real>::t* __restrict__ grid,
                                                             int64_t G, int T, real beta,
                                                             typename CxI<real>::t* __restrict__ fhat) {
  using cx = typename CxI<real>::t;
  const int tile = blockIdx.x;
  const int beg = tile_off[tile], end = tile_off[tile + 1];
  const real e2b = iexp((real)-2 * beta);
  for (int r = beg + (int)threadIdx.x; r < end; r += FWD_BLOCK) {
    const Rec<real> rec = recs[r];
    const int c0 = (int)(int16_t)(rec.c01 & 0xffff);
    if (c0 < 0 || c0 >= T) continue;   // not the home record
    const real d0 = (real)(1 - W) - rec.f0;
    real w = iexp(-beta * d0 * d0);
    real q = iexp(-beta * ((real)2 * d0 + (real)1));
    real ar = 0, ai = 0;
    int64_t g = (int64_t)tile * T + c0 - W + 1;
    g = g < 0 ? g + G : g;
#pragma unroll
    for (int j = 0; j < 2 * W; ++j) {
      const cx v = grid[g];
      ar += w * v.x;
      ai += w * v.y;
      w *= q;
      q *= e2b;
      g = g + 1 == G ? 0 : g + 1;
    }
    cx o;
    o.x = ar;
    o.y = ai;
    fhat[rec.src] = o;
  }
}

template <class real, int W, int ST>
static void launch_interp_sq(ftcg_plan p, void* fhat) {
  using cx = typename CxI<real>::t;
  const unsigned nsq = (unsigned)((p->G / ST) * (p->G / ST));
  const auto* k = p->recs.as<Rec<real>>();
  const auto* off = p->tile_off.as<int32_t>();
  const auto* gr = p->grid.as<cx>();
  auto* out = static_cast<cx*>(fhat);
  const real beta = (real)p->beta;
  switch (p->tile) {
    case 16:
      hipLaunchKernelGGL((k_interp2d_sq<real, W, 16, ST>), dim3(nsq), dim3(FWD_BLOCK), 0, p->stream, k, off, gr, p->G,
                         (int)p->nt, beta, out);
      break;
    case 32:
      hipLaunchKernelGGL((k_interp2d_sq<real, W, 32, ST>), dim3(nsq), dim3(FWD_BLOCK), 0, p->stream, k, off, gr, p->G,
                         (int)p->nt, beta, out);
      break;
    default:
      if constexpr (ST == 64) {
        hipLaunchKernelGGL((k_interp2d_sq<real, W, 64, ST>), dim3(nsq), dim3(FWD_BLOCK), 0, p->stream, k, off, gr,
                           p->G, (int)p->nt, beta, out);
        break;
      }
      throw StatusError{FTCG_EUNSUPPORTED};
  }
  FTCG_HIP(hipGetLastError());
}

template <class real, int W>
static void launch_interp(ftcg_plan p, void* fhat) {
  using cx = typename CxI<real>::t;
  const real beta = (real)p->beta;
  if (p->dim == 1) {
    hipLaunchKernelGGL((k_interp1d_tiles<real, W>), dim3((unsigned)p->ntiles), dim3(FWD_BLOCK), 0, p->stream,
                       p->recs.as<Rec<real>>(), p->tile_off.as<int32_t>(), p->grid.as<cx>(), p->G, p->tile, beta,
                       static_cast<cx*>(fhat));
  } else {
    // squares of 32 x 32 cells (64 for tile 64 in float32): squares of 64
    // re-read fewer window cells (1.37 instead of 1.81 per cell) but their
    // 45 KiB windows leave three workgroups per compute unit, and measured
    // slower (4096^2 raster: 0.645 against 0.576 ms)
    constexpr int STMAX = sizeof(real) == 4 ? 64 : 32;
    const int T = p->tile;
    if constexpr (STMAX == 64) {
      if (T == 64 && p->G % 64 == 0) {
        launch_interp_sq<real, W, 64>(p, fhat);
        return;
      }
    }
    if (T <= 32 && p->G % 32 == 0) {
      launch_interp_sq<real, W, 32>(p, fhat);
      return;
    }
    // tiles of 128, or of 64 in float64: one workgroup per tile
    const int WS = p->tile + 2 * W - 1;
    const size_t lds = (size_t)WS * WS * sizeof(cx);
    if (lds > 160 * 1024) throw StatusError{FTCG_EUNSUPPORTED};   // tile 128 in float64
    static bool attr_done = false;
    if (!attr_done) {
      FTCG_HIP(hipFuncSetAttribute((const void*)k_interp2d<real, W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   160 * 1024));
      attr_done = true;
    }
    hipLaunchKernelGGL((k_interp2d<real, W>), dim3((unsigned)p->ntiles), dim3(FWD_BLOCK), lds, p->stream,
                       p->recs.as<Rec<real>>(), p->tile_off.as<int32_t>(), p->grid.as<cx>(), p->G, (int)p->nt,
                       p->tile, beta, static_cast<cx*>(fhat));
  }
  FTCG_HIP(hipGetLastError());
}

template <class real>
static void launch_interp_w(ftcg_plan p, void* fhat) {
  switch (p->W) {
    case 2: launch_interp<real, 2>(p, fhat); break;
    case 3: launch_interp<real, 3>(p, fhat); break;
    case 4: launch_interp<real, 4>(p, fhat); break;
    case 5: launch_interp<real, 5>(p, fhat); break;
    case 6: launch_interp<real, 6>(p, fhat); break;
    case 7: launch_interp<real, 7>(p, fhat); break;
    case 8: launch_interp<real, 8>(p, fhat); break;
    default: throw StatusError{FTCG_EUNSUPPORTED};
  }
}

void interpolate_grid(ftcg_plan p, void* out) {
  if (p->dtype == FTCG_F64)
    launch_interp_w<double>(p, out);
  else
    launch_interp_w<float>(p, out);
}

void forward_transform(ftcg_plan p, const void* image, void* fhat) {
  const bool f64 = p->dtype == FTCG_F64;
  const int64_t n = p->n, G = p->G;
  const double* d = p->deapod.as<double>();
  timing_begin(p, STEP_FWD_FFT);
  if (p->dim == 1) {
    fft_cols_forward(f64, image, 1, p->grid.p, G, G, n, 1, d, nullptr, p->twiddle.p, p->stream);
  } else {
    // columns p1 of the image (positions p0) -> T[p1][g0] (n x G);
    // columns g0 of T (positions p1) -> H[g0][g1]
    fft_cols_forward(f64, image, n, p->fft_tmp.p, G, G, n, (int)n, d, d, p->twiddle.p, p->stream);
    fft_cols_forward(f64, p->fft_tmp.p, G, p->grid.p, G, G, n, (int)G, nullptr, nullptr, p->twiddle.p, p->stream);
  }
  timing_end(p, STEP_FWD_FFT);
  timing_begin(p, STEP_FWD_INTERP);
  if (f64)
    launch_interp_w<double>(p, fhat);
  else
    launch_interp_w<float>(p, fhat);
  timing_end(p, STEP_FWD_INTERP);
}

}  // namespace ftcg
