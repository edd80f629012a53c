// Frame-optimal diagonal quadrature weights in float64 (Sec. III-C, eq:difopt).
//
// min over diagonal D of ||T D - I||_F separates into one least-squares
// problem per column n: alpha_n = conj(T_nn) / sum_i |T_in|^2. With T the
// Gram matrix of the data frame on the unit field of view,
// T_in = prod_a sinc(k_ia - k_na) (sinc t = sin(pi t) / (pi t)), T_nn = 1 and
// alpha_n = 1 / sum_i T_in^2. The sum is truncated to the infinity-norm box
// ||k_i - k_n||_inf <= R (a tensor box keeps the weights of tensor rasters
// exactly separable).
//
// GPU layout: samples are counting-sorted into square neighbour bins of edge
// h = R / s (k units; s in [2, 16] for about 6 samples per bin), so the box
// of every sample lies in the (2s+1)^d bins around its own; the bins of one
// row are contiguous in bin order, so each row is one candidate range. Sorted
// arrays hold k and the
// per-sample sin(pi k), cos(pi k), so each pair needs
// sin(pi (k_i - k_n)) = sin(pi k_i) cos(pi k_n) - cos(pi k_i) sin(pi k_n)
// instead of a transcendental, and one float64 reciprocal.
#include "ftcg_internal.h"

namespace ftcg {

constexpr int WB_BLOCK = 256;

template <int DIM>
__device__ inline int wbin_of(const double* x, const WBinGeom& g, int* b) {
  int id = 0;
  for (int a = 0; a < DIM; ++a) {
    int v = (int)floor((x[a] - g.kmin[a]) / g.h);
    v = v < 0 ? 0 : (v >= g.nb[a] ? g.nb[a] - 1 : v);
    b[a] = v;
    id = id * g.nb[a] + v;
  }
  return id;
}

template <int DIM>
__global__ __launch_bounds__(WB_BLOCK) void k_wbin_count(const double* __restrict__ k, int64_t m, WBinGeom g,
                                                         int32_t* __restrict__ cnt, int32_t* __restrict__ bin_of) {
  const int64_t j = (int64_t)blockIdx.x * WB_BLOCK + threadIdx.x;
  int id = 0;
  if (j < m) {
    double x[DIM];
    int b[DIM];
    for (int a = 0; a < DIM; ++a) x[a] = k[j * DIM + a];
    id = wbin_of<DIM>(x, g, b);
    bin_of[j] = id;
  }
  agg_atomic_add(cnt, id, j < m);
}

template <int DIM>
__global__ __launch_bounds__(WB_BLOCK) void k_wbin_scatter(const double* __restrict__ k, int64_t m,
                                                           const int32_t* __restrict__ bin_of,
                                                           int32_t* __restrict__ cursor,
                                                           WSample<DIM>* __restrict__ ss, int32_t* __restrict__ sidx,
                                                           double* __restrict__ sc_orig) {
  const int64_t j = (int64_t)blockIdx.x * WB_BLOCK + threadIdx.x;
  const int pos = agg_atomic_add(cursor, j < m ? bin_of[j] : 0, j < m);
  if (j >= m) return;
  WSample<DIM> w;
  for (int a = 0; a < DIM; ++a) {
    w.k[a] = k[j * DIM + a];
    sincospi(w.k[a], &w.sc[a][0], &w.sc[a][1]);
    sc_orig[j * 2 * DIM + 2 * a] = w.sc[a][0];
    sc_orig[j * 2 * DIM + 2 * a + 1] = w.sc[a][1];
  }
  ss[pos] = w;
  sidx[pos] = (int32_t)j;
}

// 1/x to full float64 precision: hardware reciprocal estimate + two Newton steps
__device__ inline double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// T_in^2 of one candidate i for sample n = (x, sn, cs), 0 outside the box.
// Branch free: a coordinate difference of exactly 0 gives the factor
// sinc(0) = 1 through selects, so every operand of the candidate is loaded
// up front and the loop body has no data-dependent control flow.
template <int DIM>
__device__ inline double pair_term(const WSample<DIM>& o, const double* x, const double* sn, const double* cs,
                                   double R) {
  const double pi = 3.141592653589793238462643383279502884;
  double num = 1.0, den = 1.0;
  bool inside = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double d = o.k[a] - x[a];
    inside = inside && (fabs(d) <= R);
    // sin(pi (k_i - k_n)) from the per-sample sin/cos
    const double sd = o.sc[a][0] * cs[a] - o.sc[a][1] * sn[a];
    const bool z = d == 0.0;
    num *= z ? 1.0 : sd;
    den *= z ? 1.0 : pi * d;
  }
  const double q = num * rcp64(den);
  return inside ? q * q : 0.0;
}

// Adds to acc[u] the T_in^2 of every candidate i in [beg, end) for the NT
// samples u (all of them when !MASKED, else those with bit u of `mask`).
// Candidates alternate between two register sets, each loaded while the
// other one's pair terms are formed.
template <int DIM, int NT, bool MASKED>
__device__ inline void range_sum(const WSample<DIM>* __restrict__ ss, int beg, int end, const double (&x)[NT][DIM],
                                 const double (&sn)[NT][DIM], const double (&cs)[NT][DIM], double R,
                                 double (&acc)[NT], unsigned mask) {
  if (beg >= end) return;
  WSample<DIM> a = ss[beg];
  for (int i = beg; i < end; i += 2) {
    const bool has_b = i + 1 < end;
    const WSample<DIM> b = ss[has_b ? i + 1 : i];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const double t = pair_term<DIM>(a, x[u], sn[u], cs[u], R);
      acc[u] += (!MASKED || ((mask >> u) & 1u)) ? t : 0.0;
    }
    a = ss[i + 2 < end ? i + 2 : i];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const double t = pair_term<DIM>(b, x[u], sn[u], cs[u], R);
      acc[u] += (has_b && (!MASKED || ((mask >> u) & 1u))) ? t : 0.0;
    }
  }
}

// WT consecutive sorted samples per group of S lanes. Sorted samples are
// bin-major, so the WT samples nearly always share a bin row; then one pass
// over the union of their candidate ranges (rows b0 - s .. b0 + s, bins
// min b1 - s .. max b1 + s, which the box test trims back to each sample's own
// box) feeds every loaded candidate to all WT pair terms. Samples in
// different bin rows (the ends of rows) take their own ranges one after
// another. The S lanes of a group split the rows round-robin and add their
// partial sums by shuffles; S > 1 is for small rasters, where one lane per
// group would leave most of the GPU idle.
template <int DIM, int WT, int S>
__global__ __launch_bounds__(WB_BLOCK) void k_frame_weights(const WSample<DIM>* __restrict__ ss,
                                                            const int32_t* __restrict__ sidx,
                                                            const int32_t* __restrict__ boff, int64_t m, WBinGeom g,
                                                            double* __restrict__ alpha) {
  const int64_t gt = xcd_block(blockIdx.x, gridDim.x) * WB_BLOCK + threadIdx.x;
  const int ls = (int)(gt % S);
  const int64_t t0 = (gt / S) * WT;
  if (t0 >= m) return;   // whole groups leave together (S divides the block)
  double x[WT][DIM], sn[WT][DIM], cs[WT][DIM], acc[WT];
  int b[WT][DIM];
#pragma unroll
  for (int u = 0; u < WT; ++u) {
    const int64_t t = t0 + u < m ? t0 + u : m - 1;   // a last odd sample repeats (and is not stored twice)
    const WSample<DIM> me = ss[t];
    for (int a = 0; a < DIM; ++a) {
      x[u][a] = me.k[a];
      sn[u][a] = me.sc[a][0];
      cs[u][a] = me.sc[a][1];
    }
    wbin_of<DIM>(x[u], g, b[u]);
    acc[u] = 0.0;
  }
  bool same_row = true;
  int bmin = b[0][DIM - 1], bmax = b[0][DIM - 1];
#pragma unroll
  for (int u = 1; u < WT; ++u) {
    same_row = same_row && (DIM == 1 || b[u][0] == b[0][0]);
    bmin = min(bmin, b[u][DIM - 1]);
    bmax = max(bmax, b[u][DIM - 1]);
  }
  if (DIM == 1) {
    // one candidate range, split into S contiguous pieces
    const int lo = max(bmin - g.span, 0), hi = min(bmax + g.span, g.nb[0] - 1);
    const int beg = boff[lo], end = boff[hi + 1];
    const int len = (end - beg + S - 1) / S;
    const int pb = beg + ls * len, pe = min(pb + len, end);
    range_sum<DIM, WT, false>(ss, pb, pe, x, sn, cs, g.R, acc, 0u);
  } else if (same_row) {
    const int lo0 = max(b[0][0] - g.span, 0), hi0 = min(b[0][0] + g.span, g.nb[0] - 1);
    const int lo1 = max(bmin - g.span, 0), hi1 = min(bmax + g.span, g.nb[DIM - 1] - 1);
    for (int b0 = lo0 + ls; b0 <= hi0; b0 += S) {
      const int first = b0 * g.nb[DIM - 1];
      range_sum<DIM, WT, false>(ss, boff[first + lo1], boff[first + hi1 + 1], x, sn, cs, g.R, acc, 0u);
    }
  } else {
    for (int u = 0; u < WT; ++u) {
      const int lo0 = max(b[u][0] - g.span, 0), hi0 = min(b[u][0] + g.span, g.nb[0] - 1);
      const int lo1 = max(b[u][DIM - 1] - g.span, 0), hi1 = min(b[u][DIM - 1] + g.span, g.nb[DIM - 1] - 1);
      for (int b0 = lo0 + ls; b0 <= hi0; b0 += S) {
        const int first = b0 * g.nb[DIM - 1];
        range_sum<DIM, WT, true>(ss, boff[first + lo1], boff[first + hi1 + 1], x, sn, cs, g.R, acc, 1u << u);
      }
    }
  }
#pragma unroll
  for (int off = 1; off < S; off <<= 1)
#pragma unroll
    for (int u = 0; u < WT; ++u) acc[u] += __shfl_xor(acc[u], off, 64);
  if (ls == 0) {
#pragma unroll
    for (int u = 0; u < WT; ++u)
      if (t0 + u < m) alpha[sidx[t0 + u]] = 1.0 / acc[u];
  }
}

// the same sum for listed samples (caller indices), for audits and checks:
// one wavefront per sample, lanes splitting its candidate ranges (the lists
// are short, so one thread per sample would leave the GPU idle)
template <int DIM>
__global__ __launch_bounds__(WB_BLOCK) void k_frame_weights_at(const double* __restrict__ k,
                                                               const double* __restrict__ sc_orig,
                                                               const int32_t* __restrict__ idx, int64_t n,
                                                               const WSample<DIM>* __restrict__ ss,
                                                               const int32_t* __restrict__ boff, WBinGeom g,
                                                               double* __restrict__ out) {
  const int64_t w = ((int64_t)blockIdx.x * WB_BLOCK + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= n) return;   // whole wavefront
  const int64_t j = idx[w];
  double x[DIM], sn[DIM], cs[DIM];
  for (int a = 0; a < DIM; ++a) {
    x[a] = k[j * DIM + a];
    sn[a] = sc_orig[j * 2 * DIM + 2 * a];
    cs[a] = sc_orig[j * 2 * DIM + 2 * a + 1];
  }
  int b[DIM];
  wbin_of<DIM>(x, g, b);
  const int lo0 = max(b[0] - g.span, 0), hi0 = min(b[0] + g.span, g.nb[0] - 1);
  const int lo1 = DIM == 2 ? max(b[DIM - 1] - g.span, 0) : 0;
  const int hi1 = DIM == 2 ? min(b[DIM - 1] + g.span, g.nb[DIM - 1] - 1) : 0;
  double acc = 0.0;
  for (int b0 = lo0; b0 <= hi0; ++b0) {
    const int first = DIM == 2 ? b0 * g.nb[1] + lo1 : b0;
    const int last = DIM == 2 ? b0 * g.nb[1] + hi1 : b0;
    const int beg = boff[first], end = boff[last + 1];
    for (int i = beg + lane; i < end; i += 64) acc += pair_term<DIM>(ss[i], x, sn, cs, g.R);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) out[w] = 1.0 / acc;
}

// Bin edge h = R / span with span in [2, 16] chosen for about BIN_TARGET
// samples per bin at the raster's mean density over its bounding box, so the
// 2 span + 1 bins of a row range end at the box of radius R (finer bins waste
// fewer out-of-box candidates); at most 4096 bins per axis in 2D (4M in 1D).
constexpr double BIN_TARGET = 6.0;
static WBinGeom wbin_geom(ftcg_plan p, const double* kmin, const double* kmax) {
  WBinGeom g{};
  g.R = p->R;
  double vol = 1.0;
  for (int a = 0; a < p->dim; ++a) vol *= fmax(kmax[a] - kmin[a], 1e-9);
  const double rho = (double)p->m / vol;
  const double h_target = p->dim == 2 ? sqrt(BIN_TARGET / rho) : BIN_TARGET / rho;
  // h = R / span exactly, so the 2 span + 1 bins of a row range end on the box
  int span = (int)lround(p->R / h_target);
  span = span < 2 ? 2 : (span > 16 ? 16 : span);
  double h = p->R / span;
  const int max_bins = p->dim == 1 ? (1 << 22) : 4096;
  for (int a = 0; a < p->dim; ++a) {
    double ext = kmax[a] - kmin[a];
    if (ext / h + 1.0 > (double)max_bins) h = ext / (double)(max_bins - 1);
  }
  g.h = h;
  g.span = (int)ceil(p->R / h);
  for (int a = 0; a < 2; ++a) {
    g.kmin[a] = a < p->dim ? kmin[a] : 0.0;
    g.nb[a] = a < p->dim ? (int)floor((kmax[a] - kmin[a]) / h) + 1 : 1;
  }
  return g;
}

void build_weight_bins(ftcg_plan p, const double* k, const double* kmin, const double* kmax) {
  const WBinGeom g = wbin_geom(p, kmin, kmax);
  p->wgeom = g;
  const int64_t m = p->m;
  const int dim = p->dim;
  const int64_t nbins = (int64_t)g.nb[0] * g.nb[1];
  hipStream_t s = p->stream;
  p->wb_cnt.ensure(sizeof(int32_t) * (nbins + 1));
  p->wb_off.ensure(sizeof(int32_t) * (nbins + 1));
  p->wb_of.ensure(sizeof(int32_t) * m);
  p->ws_k.ensure(sizeof(double) * m * dim * 3);
  p->ws_idx.ensure(sizeof(int32_t) * m);
  p->sc_orig.ensure(sizeof(double) * m * dim * 2);
  p->scan_tmp.ensure(scan_tmp_bytes(nbins));
  int32_t* cnt = p->wb_cnt.as<int32_t>();
  int32_t* off = p->wb_off.as<int32_t>();
  const unsigned nb = (unsigned)((m + WB_BLOCK - 1) / WB_BLOCK);
  timing_begin(p, STEP_WBIN);
  FTCG_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (nbins + 1), s));
  if (dim == 1)
    hipLaunchKernelGGL(k_wbin_count<1>, dim3(nb), dim3(WB_BLOCK), 0, s, k, m, g, cnt, p->wb_of.as<int32_t>());
  else
    hipLaunchKernelGGL(k_wbin_count<2>, dim3(nb), dim3(WB_BLOCK), 0, s, k, m, g, cnt, p->wb_of.as<int32_t>());
  exclusive_scan_i32(cnt, off, nbins, p->scan_tmp.as<int32_t>(), s, cnt);  // cnt becomes the cursor
  if (dim == 1)
    hipLaunchKernelGGL(k_wbin_scatter<1>, dim3(nb), dim3(WB_BLOCK), 0, s, k, m, p->wb_of.as<int32_t>(), cnt,
                       p->ws_k.as<WSample<1>>(), p->ws_idx.as<int32_t>(), p->sc_orig.as<double>());
  else
    hipLaunchKernelGGL(k_wbin_scatter<2>, dim3(nb), dim3(WB_BLOCK), 0, s, k, m, p->wb_of.as<int32_t>(), cnt,
                       p->ws_k.as<WSample<2>>(), p->ws_idx.as<int32_t>(), p->sc_orig.as<double>());
  FTCG_HIP(hipGetLastError());
  timing_end(p, STEP_WBIN);
  p->have_wbins = true;
}

// Launch shape: WT samples per lane group and S lanes per group, from the
// plan's tuning when set, else S = 1 and WT = 2 from 2^19 samples up (where
// sharing candidate loads pays) and WT = 1 below (where the GPU is short of
// wavefronts and longer per-lane chains cost more than they save).
template <int DIM, int WT, int S>
static void launch_weights(ftcg_plan p) {
  const int64_t groups = (p->m + WT - 1) / WT;
  const unsigned nb = (unsigned)((groups * S + WB_BLOCK - 1) / WB_BLOCK);
  hipLaunchKernelGGL((k_frame_weights<DIM, WT, S>), dim3(nb), dim3(WB_BLOCK), 0, p->stream,
                     p->ws_k.as<WSample<DIM>>(), p->ws_idx.as<int32_t>(), p->wb_off.as<int32_t>(), p->m, p->wgeom,
                     p->alpha.as<double>());
}

template <int DIM, int WT>
static void launch_weights_s(ftcg_plan p, int S) {
  switch (S) {
    case 1: launch_weights<DIM, WT, 1>(p); break;
    case 2: launch_weights<DIM, WT, 2>(p); break;
    case 4: launch_weights<DIM, WT, 4>(p); break;
    default: launch_weights<DIM, WT, 8>(p); break;
  }
}

template <int DIM>
static void launch_weights_dim(ftcg_plan p) {
  const int wt = p->w_samples ? p->w_samples : (p->m >= (int64_t(1) << 19) ? 2 : 1);
  const int S = p->w_lanes ? p->w_lanes : 1;
  switch (wt) {
    case 1: launch_weights_s<DIM, 1>(p, S); break;
    case 2: launch_weights_s<DIM, 2>(p, S); break;
    default: launch_weights_s<DIM, 4>(p, S); break;
  }
}

void run_plain_weights(ftcg_plan p) {
  timing_begin(p, STEP_WEIGHTS);
  if (p->dim == 1)
    launch_weights_dim<1>(p);
  else
    launch_weights_dim<2>(p);
  FTCG_HIP(hipGetLastError());
  timing_end(p, STEP_WEIGHTS);
}

void plain_weights_at(ftcg_plan p, const double* k, const int32_t* idx, int64_t n, double* out) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)((n * 64 + WB_BLOCK - 1) / WB_BLOCK);
  const int32_t* off = p->wb_off.as<int32_t>();
  if (p->dim == 1)
    hipLaunchKernelGGL(k_frame_weights_at<1>, dim3(nb), dim3(WB_BLOCK), 0, p->stream, k, p->sc_orig.as<double>(),
                       idx, n, p->ws_k.as<WSample<1>>(), off, p->wgeom, out);
  else
    hipLaunchKernelGGL(k_frame_weights_at<2>, dim3(nb), dim3(WB_BLOCK), 0, p->stream, k, p->sc_orig.as<double>(),
                       idx, n, p->ws_k.as<WSample<2>>(), off, p->wgeom, out);
  FTCG_HIP(hipGetLastError());
}

}  // namespace ftcg
