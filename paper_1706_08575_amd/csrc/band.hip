// Banded FTCG coefficient matrix C (Sec. III-C eq:ftcg, eq:cr; Sec. IV
// eq:twodftcg) and its application c = C fhat ahead of the spreading
// (tau = Omega C fhat).
//
// C is the band-constrained minimiser of ||T C - I||_F, T the truncated Gram
// matrix of the data frame (T_in = prod_a sinc(k_ia - k_na) within
// ||k_i - k_n||_inf <= R) and the band J(n) = {n - r + 1 .. n + r - 1} in
// the caller's sample (raster) order. Column n solves the least-squares
// problem min ||T[:, J(n)] c - e_n||, i.e. the normal equations
//   (T_J^T T_J) c = T_J^T e_n = (T_{n,j})_{j in J(n)}.
// Every entry of T_J^T T_J is an entry of the band of T^2 of half-width
// 2r - 2: (T^2)_{a,b} for a, b in J(n). So:
//   1. k_band_gram: P[a][e] = pi^(2 DIM) (T^2)_{a, a+e}, e = 0 .. 2r-2, one
//      thread per sample a, walking a's neighbour bins once per pass of up
//      to BAND_NC offsets e (each candidate i: T_ia and T_{i,a+e}; T_ia = 0
//      outside a's box, so a's box is the whole sum);
//   2. k_band_solve: per column n, the (2r-1)^2 normal matrix gathered from
//      P, the right-hand side from the pair terms of n, a float64 Cholesky
//      factorisation in LDS (one thread per column, the matrix interleaved
//      across the workgroup so consecutive threads hit consecutive banks),
//      forward and back substitution; writes C by columns and by rows;
//   3. k_band_apply: c_i = sum_{|n - i| < r} C[i, n] fhat_n in float64, one
//      thread per sample, from the row form (contiguous per i).
// Like the diagonal weight sums, every product that enters a sum of step 1
// is rounded to a multiple of 2^-36 (wq_product), so the sums are exact and
// independent of the order of the samples within their bins.
#include <algorithm>

#include "ftcg_internal.h"
#include "wbins.h"

namespace ftcg {

constexpr int BAND_BLOCK = 256;
constexpr int BAND_NC = 8;   // band offsets per pass of the T^2 kernel

__device__ inline double rcp64b(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// pi^DIM T_in of candidate o for sample (x, sn, cs), exactly 0 outside the
// box ||k_i - k_n||_inf <= R. Per axis sin(pi d) comes from the per-sample
// sine and cosine by the difference formula, products rounded separately, so
// the value does not depend on which of the two samples is the candidate;
// num / den with eps = 2^-500 added gives pi at d = 0 (as for the diagonal
// weights).
template <int DIM>
__device__ inline double band_term(const WSample<DIM>& o, const double* x, const double* sn, const double* cs,
                                   double R) {
#pragma clang fp contract(off)
  double num = 1.0, den = 1.0, dmax = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double d = o.k[a] - x[a];
    dmax = a == 0 ? fabs(d) : fmax(dmax, fabs(d));
    const double p1 = o.sc[a][0] * cs[a];
    const double p2 = o.sc[a][1] * sn[a];
    num *= (p1 - p2) + 0x1p-500 * WPI;
    den *= d + 0x1p-500;
  }
  const double q = num * rcp64b(den);
  return dmax <= R ? q : 0.0;
}

// a * b rounded to a multiple of 2^-36 (|a b| <= pi^4 < 2^16)
__device__ inline double wq_product(double a, double b) { return fma(a, b, WQ_MAGIC) - WQ_MAGIC; }

template <int DIM>
__device__ inline void load_sample(const WSample<DIM>& w, double* x, double* sn, double* cs) {
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    x[a] = w.k[a];
    sn[a] = w.sc[a][0];
    cs[a] = w.sc[a][1];
  }
}

template <int DIM, int NC>
__global__ __launch_bounds__(BAND_BLOCK) void k_band_gram(const WSample<DIM>* __restrict__ ss,
                                                         const int32_t* __restrict__ inv,
                                                         const int32_t* __restrict__ boff, int64_t m, WBinGeom g,
                                                         int nband, int e0, double* __restrict__ P) {
  const int64_t a = (int64_t)blockIdx.x * BAND_BLOCK + threadIdx.x;
  if (a >= m) return;
  double x[DIM], sn[DIM], cs[DIM];
  load_sample<DIM>(ss[inv[a]], x, sn, cs);
  double cx[NC][DIM], csn[NC][DIM], ccs[NC][DIM], acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t j = std::min<int64_t>(a + e0 + c, m - 1);   // past the end: repeated, never stored
    load_sample<DIM>(ss[inv[j]], cx[c], csn[c], ccs[c]);
    acc[c] = 0.0;
  }
  int b[DIM];
  wbin_of<DIM>(x, g, b);
  const int lo0 = max(b[0] - g.span, 0), hi0 = min(b[0] + g.span, g.nb[0] - 1);
  const int lo1 = DIM == 2 ? max(b[DIM - 1] - g.span, 0) : 0;
  const int hi1 = DIM == 2 ? min(b[DIM - 1] + g.span, g.nb[DIM - 1] - 1) : 0;
  for (int b0 = lo0; b0 <= hi0; ++b0) {
    const int first = DIM == 2 ? b0 * g.nb[1] + lo1 : b0;
    const int last = DIM == 2 ? b0 * g.nb[1] + hi1 : b0;
    const int beg = boff[first], end = boff[last + 1];
    for (int i = beg; i < end; ++i) {
      const WSample<DIM> o = ss[i];
      const double qa = band_term<DIM>(o, x, sn, cs, g.R);
      if (qa == 0.0) continue;   // outside a's box: every product is 0
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += wq_product(qa, band_term<DIM>(o, cx[c], csn[c], ccs[c], g.R));
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int e = e0 + c;
    if (e < nband && a + e < m) P[a * nband + e] = acc[c];
  }
}

template <class T>
__global__ __launch_bounds__(BAND_BLOCK) void k_band_fill(T* __restrict__ p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * BAND_BLOCK + threadIdx.x;
  if (i < n) p[i] = v;
}

// One thread per column n. LDS: the packed lower triangle of the normal
// matrix (NE = nb (nb + 1) / 2 entries) and the right-hand side (nb
// entries), entry t of thread u at sm[t * blockDim + u].
template <int DIM>
__global__ void k_band_solve(const double* __restrict__ P, const WSample<DIM>* __restrict__ ss,
                             const int32_t* __restrict__ inv, int64_t m, int r, double R,
                             double* __restrict__ bcol, double* __restrict__ crow, int* __restrict__ bad) {
  extern __shared__ double sm[];
  const int nt = blockDim.x, u = threadIdx.x;
  const int64_t n = (int64_t)blockIdx.x * nt + u;
  if (n >= m) return;   // no barrier below: threads are independent
  const int nb = 2 * r - 1;
  const int NE = nb * (nb + 1) / 2;
  const int64_t lo = std::max<int64_t>(0, n - r + 1), hi = std::min<int64_t>(m - 1, n + r - 1);
  const int L = (int)(hi - lo + 1);
  const int off = (int)(lo - (n - r + 1));   // band position of J(n)'s first member
  auto A = [&](int p, int q) -> double& { return sm[(int64_t)(p * (p + 1) / 2 + q) * nt + u]; };   // p >= q
  auto Y = [&](int p) -> double& { return sm[(int64_t)(NE + p) * nt + u]; };
  for (int p = 0; p < L; ++p)
    for (int q = 0; q <= p; ++q) A(p, q) = P[(lo + q) * nb + (p - q)];
  double x[DIM], sn[DIM], cs[DIM];
  load_sample<DIM>(ss[inv[n]], x, sn, cs);
  for (int p = 0; p < L; ++p) Y(p) = band_term<DIM>(ss[inv[lo + p]], x, sn, cs, R);
  // Cholesky factorisation A = L L^T in place (lower triangle)
  bool ok = true;
  for (int p = 0; p < L && ok; ++p) {
    double s = A(p, p);
    for (int t = 0; t < p; ++t) s -= A(p, t) * A(p, t);
    if (!(s > 1e-13 * A(p, p))) {
      ok = false;
      break;
    }
    const double d = sqrt(s), id = 1.0 / d;
    A(p, p) = d;
    for (int q = p + 1; q < L; ++q) {
      double v = A(q, p);
      for (int t = 0; t < p; ++t) v -= A(q, t) * A(p, t);
      A(q, p) = v * id;
    }
  }
  if (!ok) {
    atomicAdd(bad, 1);
    for (int p = 0; p < nb; ++p) bcol[n * nb + p] = 0.0;
    return;
  }
  for (int p = 0; p < L; ++p) {   // L z = y
    double v = Y(p);
    for (int t = 0; t < p; ++t) v -= A(p, t) * Y(t);
    Y(p) = v / A(p, p);
  }
  for (int p = L - 1; p >= 0; --p) {   // L^T x = z
    double v = Y(p);
    for (int t = p + 1; t < L; ++t) v -= A(t, p) * Y(t);
    Y(p) = v / A(p, p);
  }
  // the sums carry pi^(2 DIM), the right-hand side pi^DIM: C = pi^DIM x
  constexpr double SC = DIM == 1 ? WPI : WPI * WPI;
  for (int p = 0; p < nb; ++p) {
    const int q = p - off;
    const double c = (q >= 0 && q < L) ? SC * Y(q) : 0.0;
    bcol[n * nb + p] = c;
    // row i = n - r + 1 + p holds C[i, n] at e = n - i + r - 1 = 2 (r - 1) - p
    if (q >= 0 && q < L) crow[(n - r + 1 + p) * nb + (2 * (r - 1) - p)] = c;
  }
}

template <class cx>
__global__ __launch_bounds__(BAND_BLOCK) void k_band_apply(const double* __restrict__ crow,
                                                          const cx* __restrict__ fhat, int64_t m, int r,
                                                          cx* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * BAND_BLOCK + threadIdx.x;
  if (i >= m) return;
  const int nb = 2 * r - 1;
  double re = 0.0, im = 0.0;
  for (int e = 0; e < nb; ++e) {
    const int64_t n = i + e - (r - 1);
    if (n < 0 || n >= m) continue;
    const double c = crow[i * nb + e];
    const cx v = fhat[n];
    re = fma(c, (double)v.x, re);
    im = fma(c, (double)v.y, im);
  }
  cx o;
  o.x = (decltype(o.x))re;
  o.y = (decltype(o.y))im;
  out[i] = o;
}

// threads per solve workgroup: the LDS of 64 columns when it fits 160 KiB
static int solve_threads(int r) {
  const int nb = 2 * r - 1;
  const size_t per = (size_t)(nb * (nb + 1) / 2 + nb) * sizeof(double);
  return per * 64 <= 160 * 1024 ? 64 : 32;
}

template <int DIM>
static void launch_band(ftcg_plan p) {
  const int64_t m = p->m;
  const int r = p->band_r, nb = 2 * r - 1;
  hipStream_t s = p->stream;
  const WSample<DIM>* ss = p->ws_k.as<WSample<DIM>>();
  const int32_t* inv = p->ws_inv.as<int32_t>();
  const unsigned gb = (unsigned)((m + BAND_BLOCK - 1) / BAND_BLOCK);
  timing_begin(p, STEP_BAND_GRAM);
  for (int e0 = 0; e0 < nb; e0 += BAND_NC)
    hipLaunchKernelGGL((k_band_gram<DIM, BAND_NC>), dim3(gb), dim3(BAND_BLOCK), 0, s, ss, inv,
                       p->wb_off.as<int32_t>(), m, p->wgeom, nb, e0, p->band_P.as<double>());
  FTCG_HIP(hipGetLastError());
  timing_end(p, STEP_BAND_GRAM);
  timing_begin(p, STEP_BAND_SOLVE);
  const int64_t ne = m * nb;
  hipLaunchKernelGGL(k_band_fill<double>, dim3((unsigned)((ne + BAND_BLOCK - 1) / BAND_BLOCK)), dim3(BAND_BLOCK), 0,
                     s, p->band_row.as<double>(), ne, 0.0);
  int* bad = reinterpret_cast<int*>(p->flags.as<double>() + 8);
  hipLaunchKernelGGL(k_band_fill<int>, dim3(1), dim3(BAND_BLOCK), 0, s, bad, (int64_t)1, 0);
  const int nt = solve_threads(r);
  const size_t lds = (size_t)(nb * (nb + 1) / 2 + nb) * sizeof(double) * nt;
  static bool attr_done[2] = {false, false};
  if (!attr_done[DIM - 1]) {
    FTCG_HIP(hipFuncSetAttribute((const void*)k_band_solve<DIM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 160 * 1024));
    attr_done[DIM - 1] = true;
  }
  hipLaunchKernelGGL(k_band_solve<DIM>, dim3((unsigned)((m + nt - 1) / nt)), dim3(nt), lds, s,
                     p->band_P.as<double>(), ss, inv, m, r, p->R, p->band_col.as<double>(),
                     p->band_row.as<double>(), bad);
  FTCG_HIP(hipGetLastError());
  timing_end(p, STEP_BAND_SOLVE);
  // columns whose normal matrix is not positive definite (T[:, J(n)] without
  // full column rank, e.g. two samples at the same location within r
  // positions): reported as an error of set_points
  int* hb = reinterpret_cast<int*>(p->host_flags + 8);
  FTCG_HIP(hipMemcpyAsync(hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  FTCG_HIP(hipStreamSynchronize(s));
  p->band_bad = *hb;
  if (p->band_bad) throw StatusError{FTCG_EINVAL};
}

void run_band_weights(ftcg_plan p) {
  const int64_t m = p->m;
  const int nb = 2 * p->band_r - 1;
  p->band_P.ensure(sizeof(double) * m * nb);
  p->band_col.ensure(sizeof(double) * m * nb);
  p->band_row.ensure(sizeof(double) * m * nb);
  p->band_c.ensure((p->dtype == FTCG_F64 ? 16 : 8) * (size_t)m);
  if (p->dim == 1)
    launch_band<1>(p);
  else
    launch_band<2>(p);
}

void band_apply(ftcg_plan p, const void* fhat) {
  const unsigned gb = (unsigned)((p->m + BAND_BLOCK - 1) / BAND_BLOCK);
  timing_begin(p, STEP_BAND_APPLY);
  if (p->dtype == FTCG_F64)
    hipLaunchKernelGGL(k_band_apply<double2>, dim3(gb), dim3(BAND_BLOCK), 0, p->stream, p->band_row.as<double>(),
                       static_cast<const double2*>(fhat), p->m, p->band_r, p->band_c.as<double2>());
  else
    hipLaunchKernelGGL(k_band_apply<float2>, dim3(gb), dim3(BAND_BLOCK), 0, p->stream, p->band_row.as<double>(),
                       static_cast<const float2*>(fhat), p->m, p->band_r, p->band_c.as<float2>());
  FTCG_HIP(hipGetLastError());
  timing_end(p, STEP_BAND_APPLY);
}

}  // namespace ftcg
