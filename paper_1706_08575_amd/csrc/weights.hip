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
// h = R / s (k units; s in [2, 16] for about 3 samples per bin at the mean
// density of the bounding box), so the box
// of every sample lies in the (2s+1)^d bins around its own; the bins of one
// row are contiguous in bin order, so each row is one candidate range. Sorted
// arrays hold k and the
// per-sample sin(pi k), cos(pi k), so each pair needs
// sin(pi (k_i - k_n)) = sin(pi k_i) cos(pi k_n) - cos(pi k_i) sin(pi k_n)
// instead of a transcendental, and one float64 reciprocal.
#include "ftcg_internal.h"
#include "wbins.h"

namespace ftcg {

constexpr int WB_BLOCK = 256;


// Counting sort into neighbour bins. Bins hold a few samples each, so the
// lanes of a wavefront mostly hit different bins: plain per-lane atomics (one
// instruction for the wavefront) beat aggregating equal keys first, which
// would serialise one atomic round trip per distinct key.
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
    atomicAdd(&cnt[id], 1);
  }
}

template <int DIM>
__global__ __launch_bounds__(WB_BLOCK) void k_wbin_scatter(const double* __restrict__ k, int64_t m,
                                                           const int32_t* __restrict__ bin_of,
                                                           int32_t* __restrict__ cursor,
                                                           WSample<DIM>* __restrict__ ss, int32_t* __restrict__ sidx,
                                                           int32_t* __restrict__ inv) {
  const int64_t j = (int64_t)blockIdx.x * WB_BLOCK + threadIdx.x;
  if (j >= m) return;
  const int pos = atomicAdd(&cursor[bin_of[j]], 1);
  WSample<DIM> w;
  for (int a = 0; a < DIM; ++a) {
    w.k[a] = k[j * DIM + a];
    sincospi(w.k[a], &w.sc[a][0], &w.sc[a][1]);
  }
  ss[pos] = w;
  sidx[pos] = (int32_t)j;
  inv[j] = pos;
}

// 1/x: hardware float64 reciprocal estimate refined by one Newton step, which
// leaves an error of a few units in the last place
__device__ inline double rcp64(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// pi^(2 DIM) T_in^2 of one candidate i for sample n = (x, sn, cs), 0 outside
// the box (the kernels divide pi^(2 DIM) by the sum). Per axis, T factors into
// sin(pi d) / (pi d) with d = k_i - k_n; here num = sin(pi d) + pi eps and
// den = d + eps with eps = 2^-500. For d = 0, sin(pi d) comes out exactly 0
// (the per-sample sin and cos are equal bit for bit, and the two products are
// rounded separately, never fused), so num / den = pi: the factor pi * sinc(0)
// with no compare or select. For |d| >= 2^-447, d + eps == d and
// sin(pi d) + pi eps == sin(pi d) exactly, so nothing changes; eps^2 and
// (pi eps)^2 stay normal numbers. This keeps the loop body to plain float64
// arithmetic.
constexpr double WEPS = 0x1p-500;
constexpr double WPI_EPS = WPI * WEPS;

// pi^DIM T_in by the select-free form, or a value whose square is 0 when
// ||k_i - k_n||_inf > R
template <int DIM>
__device__ inline double pair_term(const WSample<DIM>& o, const double* x, const double* sn, const double* cs,
                                   double R) {
#pragma clang fp contract(off)
  double num = 1.0, den = 1.0, dmax = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double d = o.k[a] - x[a];
    dmax = a == 0 ? fabs(d) : fmax(dmax, fabs(d));
    // sin(pi (k_i - k_n)) = sin(pi k_i) cos(pi k_n) - cos(pi k_i) sin(pi k_n)
    const double p1 = o.sc[a][0] * cs[a];
    const double p2 = o.sc[a][1] * sn[a];
    num *= (p1 - p2) + WPI_EPS;
    den *= d + WEPS;
  }
  const double q = num * rcp64(den);
  // outside the box: clear the high word, which leaves at most 2^-1042, whose
  // square is 0
  const int hi = dmax <= R ? __double2hiint(q) : 0;
  return __hiloint2double(hi, __double2loint(q));
}

// acc + (pi^DIM T_in)^2, the square rounded to the sums' quantum (wq_square)
template <int DIM>
__device__ inline double pair_add(double acc, const WSample<DIM>& o, const double* x, const double* sn,
                                  const double* cs, double R) {
  return acc + wq_square(pair_term<DIM>(o, x, sn, cs, R));
}

// staged candidate p of an LDS chunk: the byte offset 48 p by the full-rate
// 24-bit multiply (the 32-bit one is quarter rate, and the pair loop forms one
// address per candidate)
__device__ inline const WSample<2>* cand_at(const WSample<2>* base, int p) {
  return reinterpret_cast<const WSample<2>*>(reinterpret_cast<const char*>(base) +
                                             __umul24((unsigned)p, (unsigned)sizeof(WSample<2>)));
}

// Copy of a chunk of staged candidates (n4 16-byte words, at most 3 CH) to
// LDS: each thread issues all its loads before the first store, so a chunk
// costs one memory latency instead of one per word a thread copies.
template <int CH>
__device__ inline void stage_chunk(const float4* __restrict__ src, float4* dst, int n4) {
  constexpr int PER = (3 * CH + WB_BLOCK - 1) / WB_BLOCK;
  float4 v[PER];
  // (a chunk is never empty: the clamped index of a thread past its end
  // reads the last word, and the store below skips it)
#pragma unroll
  for (int u = 0; u < PER; ++u) v[u] = src[min((int)threadIdx.x + u * WB_BLOCK, n4 - 1)];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = (int)threadIdx.x + u * WB_BLOCK;
    if (i < n4) dst[i] = v[u];
  }
}

// a candidate record; 2D records (48 bytes) sit in 16-byte aligned arrays
// and are read as three 16-byte words
template <int DIM>
__device__ inline WSample<DIM> ld_wsample(const WSample<DIM>* p) {
  if constexpr (DIM == 2) {
    const double2* q = reinterpret_cast<const double2*>(p);
    const double2 v0 = q[0], v1 = q[1], v2 = q[2];
    WSample<2> w;
    w.k[0] = v0.x;
    w.k[1] = v0.y;
    w.sc[0][0] = v1.x;
    w.sc[0][1] = v1.y;
    w.sc[1][0] = v2.x;
    w.sc[1][1] = v2.y;
    return w;
  } else {
    return *p;
  }
}

// Adds to acc[u] the pi^(2 DIM) T_in^2 of every candidate i in [beg, end) for the NT
// samples u: two candidates per step (both loaded before either pair term
// is formed), then at most one more.
template <int DIM, int NT>
__device__ inline void range_sum(const WSample<DIM>* __restrict__ ss, int beg, int end, const double (&x)[NT][DIM],
                                 const double (&sn)[NT][DIM], const double (&cs)[NT][DIM], double R,
                                 double (&acc)[NT]) {
  const WSample<DIM>* p = ss + beg;
  const WSample<DIM>* const pe = ss + end;
  for (; p + 1 < pe; p += 2) {
    const WSample<DIM> a = ld_wsample(p);
    const WSample<DIM> b = ld_wsample(p + 1);
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      acc[u] = pair_add<DIM>(acc[u], a, x[u], sn[u], cs[u], R);
      acc[u] = pair_add<DIM>(acc[u], b, x[u], sn[u], cs[u], R);
    }
  }
  if (p < pe) {
    const WSample<DIM> a = ld_wsample(p);
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[u] = pair_add<DIM>(acc[u], a, x[u], sn[u], cs[u], R);
  }
}

// 1D: WT consecutive sorted samples per lane share one pass over the union
// of their candidate ranges (bins min b - s .. max b + s, which the box test
// trims back to each sample's own box).
template <int WT>
__global__ __launch_bounds__(WB_BLOCK) void k_frame_weights_1d(const WSample<1>* __restrict__ ss,
                                                               const int32_t* __restrict__ sidx,
                                                               const int32_t* __restrict__ boff, int64_t m,
                                                               WBinGeom g, double* __restrict__ alpha) {
  const int64_t t0 = ((int64_t)blockIdx.x * WB_BLOCK + threadIdx.x) * WT;
  if (t0 >= m) return;
  double x[WT][1], sn[WT][1], cs[WT][1], acc[WT];
  int bmin = 1 << 30, bmax = -1;
#pragma unroll
  for (int u = 0; u < WT; ++u) {
    const int64_t t = t0 + u < m ? t0 + u : m - 1;   // a last partial group repeats (and is not stored twice)
    const WSample<1> me = ss[t];
    x[u][0] = me.k[0];
    sn[u][0] = me.sc[0][0];
    cs[u][0] = me.sc[0][1];
    int b[1];
    wbin_of<1>(x[u], g, b);
    bmin = min(bmin, b[0]);
    bmax = max(bmax, b[0]);
    acc[u] = 0.0;
  }
  const int lo = max(bmin - g.span, 0), hi = min(bmax + g.span, g.nb[0] - 1);
  range_sum<1, WT>(ss, boff[lo], boff[hi + 1], x, sn, cs, g.R, acc);
#pragma unroll
  for (int u = 0; u < WT; ++u)
    if (t0 + u < m) alpha[sidx[t0 + u]] = wscale<1>() / acc[u];
}

// 2D: one workgroup per (bin row b0, run of WB_BLOCK * WT / S consecutive
// samples of that row), so a workgroup's samples share their row window and
// their column window is lo1 .. hi1 (first and last sample's bins, widened by
// s). Row by row, the window's candidates are staged in LDS in chunks of
// WCH (coalesced 16-byte copies); every lane then walks its part of its
// samples' range inside the chunk from LDS. Candidates are read from global
// memory once per workgroup instead of once per lane, which takes the
// vector-memory path off the critical path. S lanes share each group of WT
// samples, splitting every row range into S pieces and adding their partial
// sums by shuffles at the end (S > 1: more, shorter lanes for small
// rasters). Rows with more samples than the grid's x extent covers are
// walked in steps of gridDim.x runs.
constexpr int WCH = 512;
template <int WT, int S>
__global__ __launch_bounds__(WB_BLOCK) void k_frame_weights_rows(const WSample<2>* __restrict__ ss,
                                                                 const int32_t* __restrict__ sidx,
                                                                 const int32_t* __restrict__ boff, WBinGeom g,
                                                                 int cx, int chunk, double* __restrict__ alpha) {
  constexpr int RUN = WB_BLOCK * WT / S;   // samples per workgroup run
  __shared__ __align__(16) WSample<2> cand[WCH];
  const int64_t lid = xcd_block_chunk(blockIdx.x, gridDim.x, chunk);
  const int b0 = (int)(lid / cx), bx = (int)(lid % cx);
  const int nb1 = g.nb[1];
  const int rs = boff[b0 * nb1], re = boff[(b0 + 1) * nb1];
  const int rlo = max(b0 - g.span, 0), rhi = min(b0 + g.span, g.nb[0] - 1);
  const int sub = (int)threadIdx.x % S;
  for (int c0 = rs + bx * RUN; c0 < re; c0 += cx * RUN) {
    const int cend = min(c0 + RUN, re);
    const int t0 = c0 + ((int)threadIdx.x / S) * WT;
    double x[WT][2], sn[WT][2], cs[WT][2], acc[WT];
    int mylo = 1 << 30, myhi = -1;
#pragma unroll
    for (int u = 0; u < WT; ++u) {
      const int t = t0 + u < cend ? t0 + u : cend - 1;
      const WSample<2> me = ss[t];
      for (int a = 0; a < 2; ++a) {
        x[u][a] = me.k[a];
        sn[u][a] = me.sc[a][0];
        cs[u][a] = me.sc[a][1];
      }
      int b[2];
      wbin_of<2>(x[u], g, b);
      mylo = min(mylo, b[1]);
      myhi = max(myhi, b[1]);
      acc[u] = 0.0;
    }
    const bool active = t0 < cend;
    mylo = max(mylo - g.span, 0);
    myhi = min(myhi + g.span, nb1 - 1);
    // the run's column window: bins of its first and last sample (bin order)
    int lo1, hi1;
    {
      int b[2];
      double xf[2] = {ss[c0].k[0], ss[c0].k[1]};
      wbin_of<2>(xf, g, b);
      lo1 = max(b[1] - g.span, 0);
      double xl[2] = {ss[cend - 1].k[0], ss[cend - 1].k[1]};
      wbin_of<2>(xl, g, b);
      hi1 = min(b[1] + g.span, nb1 - 1);
    }
    for (int r = rlo; r <= rhi; ++r) {
      const int gs = boff[r * nb1 + lo1], ge = boff[r * nb1 + hi1 + 1];
      int ms = 0, me = 0;
      if (active) {
        const int fs = boff[r * nb1 + mylo], fe = boff[r * nb1 + myhi + 1];
        const int part = (fe - fs + S - 1) / S;
        ms = min(fs + sub * part, fe);
        me = min(ms + part, fe);
      }
      for (int q0 = gs; q0 < ge; q0 += WCH) {
        const int q1 = min(q0 + WCH, ge);
        __syncthreads();  // the previous chunk has been consumed
        {
          stage_chunk<WCH>(reinterpret_cast<const float4*>(ss + q0), reinterpret_cast<float4*>(cand), (q1 - q0) * 3);
        }
        __syncthreads();
        const int a0 = max(ms, q0), a1 = min(me, q1);
        if (a0 < a1) range_sum<2, WT>(cand, a0 - q0, a1 - q0, x, sn, cs, g.R, acc);
      }
    }
#pragma unroll
    for (int off = 1; off < S; off <<= 1)
#pragma unroll
      for (int u = 0; u < WT; ++u) acc[u] += __shfl_xor(acc[u], off, 64);
    if (sub == 0) {
#pragma unroll
      for (int u = 0; u < WT; ++u)
        if (t0 + u < cend) alpha[sidx[t0 + u]] = wscale<2>() / acc[u];
    }
  }
}

// Symmetric form of the 2D sum. T is symmetric, so each unordered pair
// {n, i} is formed once, by the sample that comes first: i later in bin order
// in n's own bin row, or anywhere in n's column window in the s bin rows
// after it. The square goes to both sums: to n's in a register, and to i's in
// an LDS slot of its staged candidate, flushed after every chunk with one
// float64 atomic per touched candidate into the bin-order sums, which start
// from the self terms pi^4 preset by the bin sort. Launch shape and staging
// as k_frame_weights_rows with one sample per lane group.
// pi^2 T_in of one staged candidate for each of the WT (<= 2) samples of a
// lane, 0 outside the box. As pair_term, with one float64 reciprocal for both
// samples: r = 1 / (den_0 den_1), q_0 = num_0 den_1 r, q_1 = num_1 den_0 r.
// With eps = 2^-250 a den lies in [2^-500, 2^64) for a live sample (|d| below
// 2^32 inside any window) and near 2^200 for an idle one (at 2^100), so the
// product of two stays a normal number; d + eps == d for |d| >= 2^-196,
// below which the factor is pi to rounding either way.
constexpr double WEPS_SYM = 0x1p-250;
constexpr double WPI_EPS_SYM = WPI * WEPS_SYM;
template <int WT>
__device__ inline void sym_terms(const WSample<2>& o, const double (&x)[WT][2], const double (&sn)[WT][2],
                                 const double (&cs)[WT][2], double R, double (&q)[WT]) {
#pragma clang fp contract(off)
  static_assert(WT == 1 || WT == 2, "one shared reciprocal for at most two samples");
  double num[WT], den[WT];
  bool in[WT];
#pragma unroll
  for (int u = 0; u < WT; ++u) {
    const double d0 = o.k[0] - x[u][0], d1 = o.k[1] - x[u][1];
    in[u] = fmax(fabs(d0), fabs(d1)) <= R;
    // sin(pi (k_i - k_n)) = sin(pi k_i) cos(pi k_n) - cos(pi k_i) sin(pi k_n),
    // both products rounded, so it is exactly 0 when k_i == k_n
    const double s0 = o.sc[0][0] * cs[u][0] - o.sc[0][1] * sn[u][0];
    const double s1 = o.sc[1][0] * cs[u][1] - o.sc[1][1] * sn[u][1];
    num[u] = (s0 + WPI_EPS_SYM) * (s1 + WPI_EPS_SYM);
    den[u] = (d0 + WEPS_SYM) * (d1 + WEPS_SYM);
  }
  if constexpr (WT == 1) {
    q[0] = num[0] * rcp64(den[0]);
  } else {
    const double r = rcp64(den[0] * den[1]);
    q[0] = num[0] * (den[1] * r);
    q[1] = num[1] * (den[0] * r);
  }
#pragma unroll
  for (int u = 0; u < WT; ++u) q[u] = __hiloint2double(in[u] ? __double2hiint(q[u]) : 0, __double2loint(q[u]));
}

// One staged candidate (chunk slot p) against the WT samples of a lane. A
// lane's own sums take the squares as they are: the bin sort orders every bin
// by caller index, so a lane's samples, its ranges and the order in which it
// walks them are the same on every run, and each of its sums is rounded to
// the quantum of the sums once, before it leaves the lane. The candidate's
// slot, which lanes add to in any order, takes the sum of its squares rounded
// to that quantum (two fused multiply-adds onto 1.5 * 2^16, then the exact
// subtraction). Every candidate of a lane's ranges pairs with all of its
// samples: in the own bin row the range starts after the lane's last live
// sample (the pair of the lane's two samples is added once, outside the
// loop), and a lane's idle sample sits far outside every box. SKIP0 skips
// the slot's add when its sum is 0 (a candidate outside the boxes of all of
// the lane's samples); adding the 0 instead keeps the loop one basic block,
// which pays where a wavefront's lanes walk long ranges (two lanes per
// group), and not with four.
template <int WT, bool SKIP0>
__device__ inline void sym_pair(double (&acc)[WT], double* cacc, int p, const WSample<2>& o,
                                const double (&x)[WT][2], const double (&sn)[WT][2], const double (&cs)[WT][2],
                                double R) {
  double q[WT];
  sym_terms<WT>(o, x, sn, cs, R, q);
  double c = WQ_MAGIC;
#pragma unroll
  for (int u = 0; u < WT; ++u) {
    acc[u] = fma(q[u], q[u], acc[u]);
    c = fma(q[u], q[u], c);
  }
  const double csum = c - WQ_MAGIC;
  if (!SKIP0 || csum != 0.0) __hip_atomic_fetch_add(cacc + p, csum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Work balance of the symmetric sum: a wavefront runs its pair loop as long
// as its longest lane range, and the candidate counts of the groups' windows
// vary along a bin row by tens of percent (lattice rasters against the bin
// grid), so taken in bin order a wavefront's lanes idle about a quarter of
// the loop. With two lanes per group, each run therefore orders its groups by
// candidate count, heaviest first (a counting sort in LDS), and lanes take
// groups in that order: the wavefronts then hold groups of about equal work.
// With four lanes per group the runs are short and the ordering costs more
// than it balances (2^17 samples: 0.043 -> 0.038 ms without it; 2^20: no
// change), so those take groups in bin order. Which lane takes which group
// does not change the sums: a group's order of addition depends on the group
// alone (its start below), and the candidate slots add exactly quantized sums.
constexpr int WKEYS = 512;   // work buckets of the ordering; counts of WKEYS - 1 and more share the last
static_assert(WKEYS % WB_BLOCK == 0, "whole buckets per thread in the scan");

// Five workgroups per compute unit (launch bound): 96 VGPRs with the pair
// loop taking one candidate per iteration, and 31 KiB of LDS each (4096^2:
// 1.49 -> 1.41 ms against four workgroups at 100 VGPRs with two candidates
// per iteration).
template <int WT, int S>
__global__ __launch_bounds__(WB_BLOCK, 5) void k_frame_weights_sym(const WSample<2>* __restrict__ ss,
                                                                const int32_t* __restrict__ boff, WBinGeom g,
                                                                int cx, int chunk, double* __restrict__ wsum) {
  constexpr int RUN = WB_BLOCK * WT / S;
  // candidates per LDS chunk: 256 with one sample per lane (14 KiB with the
  // slot sums: occupancy 7 instead of 5, 2^17 samples 0.040 -> 0.038 ms),
  // 512 with two (0.366 against 0.388 ms at 2^20, 1.59 against 2.18 ms at
  // 2^23, where the wider runs fill the chunk)
  constexpr int CH = WT == 1 ? 256 : WCH;
  constexpr int NG = WB_BLOCK / S;   // groups of WT samples per run
  constexpr bool ORDER = S <= 2;      // work order (four lanes per group: short runs, order costs more)
  __shared__ __align__(16) WSample<2> cand[CH];
  __shared__ double cacc[CH];
  __shared__ int whist[WKEYS];
  __shared__ int wpart[WB_BLOCK / 64];
  __shared__ int gorder[NG];
  for (int i = threadIdx.x; i < CH; i += WB_BLOCK) cacc[i] = 0.0;   // ordered by the first chunk's barriers
  const int64_t lid = xcd_block_chunk(blockIdx.x, gridDim.x, chunk);
  const int b0 = (int)(lid / cx), bx = (int)(lid % cx);
  const int nb1 = g.nb[1];
  const int rs = boff[b0 * nb1], re = boff[(b0 + 1) * nb1];
  const int rhi = min(b0 + g.span, g.nb[0] - 1);
  const int sub = (int)threadIdx.x % S;
  for (int c0 = rs + bx * RUN; c0 < re; c0 += cx * RUN) {
    const int cend = min(c0 + RUN, re);
    int gi = (int)threadIdx.x / S;   // this lane's group: in bin order, or by work
    if constexpr (ORDER) {
      // order the run's groups by candidate count (the ranges of the pair loop
      // below, summed over the rows), heaviest first
      for (int i = threadIdx.x; i < WKEYS; i += WB_BLOCK) whist[i] = 0;
      __syncthreads();   // (also: the previous run's order has been read)
      int key = 0, slot = 0;
      if (sub == 0) {
        const int gt0 = c0 + gi * WT;
        int work = 0;
        if (gt0 < cend) {
          int lo = 1 << 30, hi = -1, nl = 0;
#pragma unroll
          for (int u = 0; u < WT; ++u)
            if (gt0 + u < cend) {
              const double2 kk = *reinterpret_cast<const double2*>(ss[gt0 + u].k);
              double xk[2] = {kk.x, kk.y};
              int b[2];
              wbin_of<2>(xk, g, b);
              lo = min(lo, b[1]);
              hi = max(hi, b[1]);
              ++nl;
            }
          lo = max(lo - g.span, 0);
          hi = min(hi + g.span, nb1 - 1);
          for (int r = b0; r <= rhi; ++r) {
            int fs = boff[r * nb1 + lo];
            const int fe = boff[r * nb1 + hi + 1];
            if (r == b0) fs = max(fs, gt0 + nl);
            work += max(fe - fs, 0);
          }
        }
        key = WKEYS - 1 - min(work, WKEYS - 1);
        slot = atomicAdd(&whist[key], 1);
      }
      __syncthreads();
      {   // exclusive scan of the bucket counts, WKEYS / WB_BLOCK buckets per thread
        constexpr int PER = WKEYS / WB_BLOCK;
        int v[PER], tot = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          v[q] = whist[threadIdx.x * PER + q];
          tot += v[q];
        }
        int incl = tot;
        const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int y = __shfl_up(incl, off, 64);
          if (lane >= off) incl += y;
        }
        if (lane == 63) wpart[wv] = incl;
        __syncthreads();
        int pre = incl - tot;
        for (int q = 0; q < wv; ++q) pre += wpart[q];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          whist[threadIdx.x * PER + q] = pre;
          pre += v[q];
        }
      }
      __syncthreads();
      if (sub == 0) gorder[whist[key] + slot] = (int)threadIdx.x / S;
      __syncthreads();
      gi = gorder[gi];
    }
    const int t0 = c0 + gi * WT;   // this lane's samples t0 .. t0 + WT - 1
    const bool active = t0 < cend;
    double x[WT][2], sn[WT][2], cs[WT][2];
    int mylo = 1 << 30, myhi = -1;
    bool live[WT];
#pragma unroll
    for (int u = 0; u < WT; ++u) {
      live[u] = t0 + u < cend;
      const WSample<2> me = ss[live[u] ? t0 + u : cend - 1];
      for (int a = 0; a < 2; ++a) {
        x[u][a] = me.k[a];
        sn[u][a] = me.sc[a][0];
        cs[u][a] = me.sc[a][1];
      }
      int b[2];
      wbin_of<2>(x[u], g, b);
      mylo = min(mylo, b[1]);
      myhi = max(myhi, b[1]);
    }
    mylo = max(mylo - g.span, 0);
    myhi = min(myhi + g.span, nb1 - 1);
    // an idle sample (past the run's end: a copy of its last sample, whose
    // bins set the window above) moves far outside every box: its terms
    // are 0, and it needs no test in the pair loop
#pragma unroll
    for (int u = 1; u < WT; ++u)
      if (!live[u]) x[u][0] = x[u][1] = 0x1p100;
    int nlive = 0;
#pragma unroll
    for (int u = 0; u < WT; ++u) nlive += live[u] ? 1 : 0;
    int lo1, hi1;
    {
      int b[2];
      double xf[2] = {ss[c0].k[0], ss[c0].k[1]};
      wbin_of<2>(xf, g, b);
      lo1 = max(b[1] - g.span, 0);
      double xl[2] = {ss[cend - 1].k[0], ss[cend - 1].k[1]};
      wbin_of<2>(xl, g, b);
      hi1 = min(b[1] + g.span, nb1 - 1);
    }
    double acc[WT];
#pragma unroll
    for (int u = 0; u < WT; ++u) acc[u] = 0.0;
    for (int r = b0; r <= rhi; ++r) {
      const int gs = boff[r * nb1 + lo1], ge = boff[r * nb1 + hi1 + 1];
      int ms = 0, me = 0;
      if (active) {
        int fs = boff[r * nb1 + mylo];
        const int fe = boff[r * nb1 + myhi + 1];
        // own row: the samples after this lane's live ones
        if (r == b0) fs = max(fs, t0 + nlive);
        if (fs < fe) {
          const int part = (fe - fs + S - 1) / S;
          ms = min(fs + sub * part, fe);
          me = min(ms + part, fe);
        }
      }
      for (int q0 = gs; q0 < ge; q0 += CH) {
        const int q1 = min(q0 + CH, ge);
        __syncthreads();   // the previous chunk has been consumed and flushed
        {
          stage_chunk<CH>(reinterpret_cast<const float4*>(ss + q0), reinterpret_cast<float4*>(cand), (q1 - q0) * 3);
        }
        __syncthreads();
        const int a0 = max(ms, q0) - q0, a1 = min(me, q1) - q0;
        // Each lane starts at its own rotation of its range, on slot
        // (t0 / WT) S + sub modulo 16: groups of one bin walk the same range,
        // and the work order (or the bin order, without it) puts neighbouring
        // groups (the same bins, so the same work) in neighbouring lanes,
        // whose starts then fall on
        // different LDS banks (a 48-byte record covers 12 of the 64 four-byte
        // banks; records 16 apart share them), for the record reads and the
        // slot atomics alike. The start is a function of the group and the
        // range, not of the lane, so a lane's order of addition is the same
        // on every run.
        const int len = a1 - a0;
        if (len > 0) {
          const unsigned ph = ((unsigned)((t0 / WT) * S + sub) - (unsigned)a0) & 15u;
          int p = a0 + (int)(ph % (unsigned)len);
          for (int j = 0; j < len; ++j) {
            sym_pair<WT, (S > 2)>(acc, cacc, p, ld_wsample(cand_at(cand, p)), x, sn, cs, g.R);
            p = p + 1 == a1 ? a0 : p + 1;
          }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < q1 - q0; i += WB_BLOCK) {
          const double v = cacc[i];
          if (v != 0.0) {
            unsafeAtomicAdd(wsum + q0 + i, v);
            cacc[i] = 0.0;
          }
        }
      }
    }
    // the pairs among this lane's own samples (left out of its own-row
    // range), formed once: by the first of the S lanes of the group, and as
    // the pair loop would (the later sample as the candidate)
    if (sub == 0) {
#pragma unroll
      for (int u = 0; u < WT; ++u)
#pragma unroll
        for (int w = u + 1; w < WT; ++w)
          if (live[w]) {
            WSample<2> o;
            for (int a = 0; a < 2; ++a) {
              o.k[a] = x[w][a];
              o.sc[a][0] = sn[w][a];
              o.sc[a][1] = cs[w][a];
            }
            const double q2 = wq_square(pair_term<2>(o, x[u], sn[u], cs[u], g.R));
            acc[u] += q2;
            acc[w] += q2;
          }
    }
#pragma unroll
    for (int u = 0; u < WT; ++u) {
#pragma unroll
      for (int off = 1; off < S; off <<= 1) acc[u] += __shfl_xor(acc[u], off, 64);
      // rounded to the quantum of the sums (exact from here on)
      if (sub == 0 && live[u]) unsafeAtomicAdd(wsum + t0 + u, (acc[u] + WQ_MAGIC) - WQ_MAGIC);
    }
  }
}

// alpha (caller order) from the bin-order sums
__global__ __launch_bounds__(WB_BLOCK) void k_weights_from_sums(const double* __restrict__ wsum,
                                                                const int32_t* __restrict__ sidx, int64_t m,
                                                                double* __restrict__ alpha) {
  const int64_t t = (int64_t)blockIdx.x * WB_BLOCK + threadIdx.x;
  if (t < m) alpha[sidx[t]] = wscale<2>() / wsum[t];
}

// the same, and the weights of the tile records (record r of sample j gets
// alpha_j), the record count read on the device: one launch for both orders
template <class real>
__global__ __launch_bounds__(WB_BLOCK) void k_weights_from_sums_recs(const double* __restrict__ wsum,
                                                                     const int32_t* __restrict__ sidx,
                                                                     const int32_t* __restrict__ inv, int64_t m,
                                                                     double* __restrict__ alpha,
                                                                     const Rec<real>* __restrict__ recs,
                                                                     const int32_t* __restrict__ nrec_dev,
                                                                     real* __restrict__ alpha_s) {
  const int64_t t0 = (int64_t)blockIdx.x * WB_BLOCK + threadIdx.x, gs = (int64_t)gridDim.x * WB_BLOCK;
  for (int64_t t = t0; t < m; t += gs) alpha[sidx[t]] = wscale<2>() / wsum[t];
  const int64_t nrec = *nrec_dev;
  for (int64_t r = t0; r < nrec; r += gs) alpha_s[r] = (real)(wscale<2>() / wsum[inv[recs[r].src]]);
}

__global__ __launch_bounds__(WB_BLOCK) void k_fill_f64(double* __restrict__ a, int64_t n, double v) {
  const int64_t t = (int64_t)blockIdx.x * WB_BLOCK + threadIdx.x;
  if (t < n) a[t] = v;
}

// the same sum for listed samples (caller indices), for audits and checks:
// one wavefront per sample, lanes splitting its candidate ranges (the lists
// are short, so one thread per sample would leave the GPU idle)
template <int DIM>
__global__ __launch_bounds__(WB_BLOCK) void k_frame_weights_at(const int32_t* __restrict__ inv,
                                                               const int32_t* __restrict__ idx, int64_t n,
                                                               const WSample<DIM>* __restrict__ ss,
                                                               const int32_t* __restrict__ boff, WBinGeom g,
                                                               double* __restrict__ out) {
  const int64_t w = ((int64_t)blockIdx.x * WB_BLOCK + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= n) return;   // whole wavefront
  const WSample<DIM> me = ss[inv[idx[w]]];
  double x[DIM], sn[DIM], cs[DIM];
  for (int a = 0; a < DIM; ++a) {
    x[a] = me.k[a];
    sn[a] = me.sc[a][0];
    cs[a] = me.sc[a][1];
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
    for (int i = beg + lane; i < end; i += 64) acc = pair_add<DIM>(acc, ss[i], x, sn, cs, g.R);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) out[w] = wscale<DIM>() / acc;
}

// Bin edge h = R / span with span in [2, 16] chosen for about BIN_TARGET
// samples per bin at the raster's mean density over its bounding box, so the
// 2 span + 1 bins of a row range end at the box of radius R; at most 4096
// bins per axis in 2D (4M in 1D). Finer bins waste fewer out-of-box
// candidates but cut the candidates into more, shorter row ranges: measured
// on SAS rasters of 2^17, 2^20 and 2^23 samples (span 3 against span 4), the
// weight kernel took 0.053 / 0.507 / 2.23 ms against 0.058 / 0.528 / 2.21 ms.
constexpr double BIN_TARGET = 4.5;
// Second step of the input check: one workgroup reduces the partials of
// k_check_points, rejects the points when one is non-finite or farther than
// 2^40 from the origin on an axis, and derives the neighbour-bin geometry
// from the bounding box. The result goes to device memory, for the binning
// passes enqueued before the host has looked at it, and to pinned host
// memory, from which the host launches the rest with the same values. A
// rejected set still gets a valid one-bin geometry, so those passes stay in
// bounds.
constexpr double KMAX_ABS = 1099511627776.0;   // 2^40

__device__ inline double decode_ordered_dev(unsigned long long o) {
  const unsigned long long b = (o & 0x8000000000000000ull) ? (o & 0x7fffffffffffffffull) : ~o;
  return __longlong_as_double((long long)b);
}

constexpr int CR_BLOCK = 256;
__global__ __launch_bounds__(CR_BLOCK) void k_check_reduce(const unsigned long long* __restrict__ part, int nparts,
                                                           int dim, int64_t m, double R, int seq,
                                                           CheckOut* __restrict__ out_dev,
                                                           CheckOut* __restrict__ out_host) {
  __shared__ unsigned long long sred[5][CR_BLOCK / 64];
  unsigned long long v[5] = {0ull, ~0ull, ~0ull, 0ull, 0ull};   // flag, lo0, lo1, hi0, hi1
  for (int b = threadIdx.x; b < nparts; b += CR_BLOCK) {
    const unsigned long long* q = part + 5 * b;
    v[0] |= q[0];
    v[1] = q[1] < v[1] ? q[1] : v[1];
    v[2] = q[2] < v[2] ? q[2] : v[2];
    v[3] = q[3] > v[3] ? q[3] : v[3];
    v[4] = q[4] > v[4] ? q[4] : v[4];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long y[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) y[i] = __shfl_xor(v[i], off, 64);
    v[0] |= y[0];
    v[1] = y[1] < v[1] ? y[1] : v[1];
    v[2] = y[2] < v[2] ? y[2] : v[2];
    v[3] = y[3] > v[3] ? y[3] : v[3];
    v[4] = y[4] > v[4] ? y[4] : v[4];
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int i = 0; i < 5; ++i) sred[i][w] = v[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int q = 1; q < CR_BLOCK / 64; ++q) {
    v[0] |= sred[0][q];
    v[1] = sred[1][q] < v[1] ? sred[1][q] : v[1];
    v[2] = sred[2][q] < v[2] ? sred[2][q] : v[2];
    v[3] = sred[3][q] > v[3] ? sred[3][q] : v[3];
    v[4] = sred[4][q] > v[4] ? sred[4][q] : v[4];
  }
  CheckOut o;
  bool bad = v[0] != 0;
  for (int a = 0; a < 2; ++a) {
    o.kmin[a] = a < dim ? decode_ordered_dev(v[1 + a]) : 0.0;
    o.kmax[a] = a < dim ? decode_ordered_dev(v[3 + a]) : 0.0;
    bad = bad || !(o.kmin[a] >= -KMAX_ABS && o.kmax[a] <= KMAX_ABS);
  }
  WBinGeom g;
  g.R = R;
  if (bad) {
    g.kmin[0] = g.kmin[1] = 0.0;
    g.h = 1.0;
    g.nb[0] = g.nb[1] = 1;
    g.span = 1;
  } else {
    // bins of about BIN_TARGET samples at the mean density of the box, with
    // h = R / span exactly, so the 2 span + 1 bins of a row range end on the
    // box of radius R; at most max_bins bins per axis
    double vol = 1.0;
    for (int a = 0; a < dim; ++a) vol *= fmax(o.kmax[a] - o.kmin[a], 1e-9);
    const double rho = (double)m / vol;
    const double h_target = dim == 2 ? sqrt(BIN_TARGET / rho) : BIN_TARGET / rho;
    const double sp = fmin(fmax(floor(R / h_target + 0.5), 2.0), 16.0);
    double h = R / sp;
    const double max_bins = dim == 1 ? (double)(1 << 22) : (double)WROW_MAX;
    for (int a = 0; a < dim; ++a) {
      const double ext = o.kmax[a] - o.kmin[a];
      if (ext / h + 1.0 > max_bins) h = ext / (max_bins - 1.0);
    }
    g.h = h;
    g.span = (int)ceil(R / h);
    for (int a = 0; a < 2; ++a) {
      g.kmin[a] = a < dim ? o.kmin[a] : 0.0;
      g.nb[a] = a < dim ? (int)fmin(fmax(floor((o.kmax[a] - o.kmin[a]) / h) + 1.0, 1.0), max_bins) : 1;
    }
  }
  o.g = g;
  o.bad = bad ? 1 : 0;
  o.seq = seq;
  *out_dev = o;
  *out_host = o;
}

void launch_check_reduce(ftcg_plan p, const unsigned long long* part, int nparts, int seq) {
  hipLaunchKernelGGL(k_check_reduce, dim3(1), dim3(CR_BLOCK), 0, p->stream, part, nparts, p->dim, p->m, p->R, seq,
                     p->geo.as<CheckOut>(), p->host_geo);
  FTCG_HIP(hipGetLastError());
}

// 2D neighbour binning in two levels, so no pass spreads atomics over all
// nb0 x nb1 bins (they outgrow the L2 on large rasters) and no pass gathers
// at random:
//  1. k_wrow_count: counts per bin row b0 in LDS, one global atomic per row a
//     workgroup saw;
//  2. exclusive scan over the <= 4096 rows (row_off; the counters become
//     cursors);
//  3. k_wrow_scatter: each workgroup claims one range per row and places its
//     samples there as {k, caller index, bin column} (rowbuf, grouped by row);
//  4. k_wrow_sort: one workgroup per row reads its range in order, counts the
//     samples per bin column in LDS, scans them, writes the bin offsets boff
//     of the whole row, orders the row in LDS (rows of up to WROW_LMAX_*
//     samples) and writes the sorted samples (k, sin, cos) and their caller
//     index coalesced, and (when asked) the inverse map; longer rows place
//     their samples directly. Every write stays inside the row's own range.
// The row counters arrive zeroed (the input check clears them).
constexpr int WROW_IPT = 4;
// Rows up to this many samples are ordered in LDS (a position, a column and
// a key array of 2 bytes per sample): 10240 with 1024 threads per row (77 KiB
// of LDS, two workgroups per compute unit), 6144 with 256 (53 KiB, three).
// Longer rows are placed by global claims and ordered after the placement.
constexpr int WROW_LMAX_WIDE = 10240;
constexpr int WROW_LMAX_NARROW = 6144;


// Steps 1 and 3 take `rounds` groups of WROW_IPT * WB_BLOCK consecutive
// samples per workgroup. A pulse of a polar raster crosses the bin rows one
// after another, so a group of samples from one pulse meets each row a few
// times; several groups (several neighbouring pulses) per workgroup give each
// row's global atomic more samples. The count (no atomic results waited for)
// gains from it; the placement, whose rounds run one after another, is
// launched with one.
__global__ __launch_bounds__(WB_BLOCK) void k_wrow_count(const double* __restrict__ k, int64_t m,
                                                         const WBinGeom* __restrict__ gp,
                                                         int32_t* __restrict__ row_cnt, int rounds) {
  const WBinGeom g = *gp;
  __shared__ int32_t hist[WROW_MAX];
  const int nrow = g.nb[0];
  for (int i = threadIdx.x; i < nrow; i += WB_BLOCK) hist[i] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * rounds * WROW_IPT * WB_BLOCK;
  for (int rr = 0; rr < rounds; ++rr) {
#pragma unroll
    for (int u = 0; u < WROW_IPT; ++u) {
      const int64_t j = j0 + (int64_t)(rr * WROW_IPT + u) * WB_BLOCK + threadIdx.x;
      if (j < m) {
        int b1;
        double x[2];
        atomicAdd(&hist[wbin_row_col(k, j, g, &b1, x)], 1);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nrow; i += WB_BLOCK) {
    const int v = hist[i];
    if (v) atomicAdd(&row_cnt[i], v);
  }
}

__global__ __launch_bounds__(WB_BLOCK) void k_wrow_scatter(const double* __restrict__ k, int64_t m,
                                                           const WBinGeom* __restrict__ gp,
                                                           int32_t* __restrict__ row_cursor,
                                                           RowRec* __restrict__ rowbuf, int rounds) {
  const WBinGeom g = *gp;
  __shared__ int32_t base[WROW_MAX + 64];   // row counters, then one spare word per lane
  const int nrow = g.nb[0];
  for (int i = threadIdx.x; i < nrow; i += WB_BLOCK) base[i] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * rounds * WROW_IPT * WB_BLOCK;
  for (int rr = 0; rr < rounds; ++rr) {
#pragma unroll
    for (int u = 0; u < WROW_IPT; ++u) {
      const int64_t j = j0 + (int64_t)(rr * WROW_IPT + u) * WB_BLOCK + threadIdx.x;
      if (j < m) {
        int b1;
        double x[2];
        atomicAdd(&base[wbin_row_col(k, j, g, &b1, x)], 1);
      }
    }
  }
  __syncthreads();
  {
    // one range per row seen; a thread's claims are all in flight together
    constexpr int PER = WROW_MAX / WB_BLOCK;
    int v[PER], r[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = threadIdx.x + q * WB_BLOCK;
      v[q] = i < nrow ? base[i] : 0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) r[q] = v[q] ? atomicAdd(&row_cursor[threadIdx.x + q * WB_BLOCK], v[q]) : 0;
#pragma unroll
    for (int q = 0; q < PER; ++q)
      if (v[q]) base[threadIdx.x + q * WB_BLOCK] = r[q];
  }
  __syncthreads();
  for (int rr = 0; rr < rounds; ++rr) {
    int row[WROW_IPT], col[WROW_IPT];
    double x[WROW_IPT][2];
#pragma unroll
    for (int u = 0; u < WROW_IPT; ++u) {
      const int64_t j = j0 + (int64_t)(rr * WROW_IPT + u) * WB_BLOCK + threadIdx.x;
      row[u] = j < m ? wbin_row_col(k, j, g, &col[u], x[u]) : -1;
    }
    // slots claimed without branches (a lane past the end adds to its spare
    // word), so all claims are in flight before the first is used
    int pos[WROW_IPT];
#pragma unroll
    for (int u = 0; u < WROW_IPT; ++u)
      pos[u] = atomicAdd(&base[row[u] >= 0 ? row[u] : WROW_MAX + (int)__lane_id()], 1);
#pragma unroll
    for (int u = 0; u < WROW_IPT; ++u) {
      const int64_t j = j0 + (int64_t)(rr * WROW_IPT + u) * WB_BLOCK + threadIdx.x;
      if (row[u] >= 0) {
        RowRec rec;
        rec.k0 = x[u][0];
        rec.k1 = x[u][1];
        rec.j = (int32_t)j;
        rec.b1 = col[u];
        rowbuf[pos[u]] = rec;
      }
    }
  }
}

// BS threads per row: 1024 for rows of thousands of samples (the LDS of a
// row keeps at most three workgroups on a compute unit, so wider workgroups
// are what puts more wavefronts in flight), 256 below
template <int BS, int LMAX>
__global__ __launch_bounds__(BS) void k_wrow_sort(WBinGeom g, const int32_t* __restrict__ row_off,
                                                  const RowRec* __restrict__ rowbuf,
                                                  int32_t* __restrict__ boff, WSample<2>* __restrict__ ss,
                                                  int32_t* __restrict__ sidx, int32_t* __restrict__ inv,
                                                  double* __restrict__ sums) {
  constexpr int ITEMS = 4096 / BS;
  __shared__ int32_t cnt[4096 + 64];   // bin counters, then one spare word per lane
  __shared__ int32_t wsum[BS / 64];
  __shared__ uint16_t perm[LMAX];
  __shared__ uint16_t col[LMAX];       // bin column of each row entry (from the counting pass)
  __shared__ uint16_t key[LMAX];       // low 16 bits of each row entry's caller index
  const int b0 = blockIdx.x, nb1 = g.nb[1];
  const int rs = row_off[b0], re = row_off[b0 + 1];
  const bool fits = re - rs <= LMAX;
  const int t = threadIdx.x;
  for (int i = t; i < nb1; i += BS) cnt[i] = 0;
  __syncthreads();
  // (SU entries per thread per step: their loads are in flight together)
  constexpr int SU = 4;
  for (int i0 = rs + t; i0 < re; i0 += SU * BS) {
    int b[SU], jj[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const bool in = i0 + u * BS < re;
      b[u] = in ? rowbuf[i0 + u * BS].b1 : -1;
      jj[u] = in ? rowbuf[i0 + u * BS].j : 0;
    }
#pragma unroll
    for (int u = 0; u < SU; ++u)
      if (b[u] >= 0) {
        atomicAdd(&cnt[b[u]], 1);
        if (fits) {
          col[i0 + u * BS - rs] = (uint16_t)b[u];
          key[i0 + u * BS - rs] = (uint16_t)(jj[u] & 0xffff);
        }
      }
  }
  __syncthreads();
  // exclusive scan of cnt[0 .. nb1): thread t owns entries t*ITEMS .. +ITEMS-1
  int v[ITEMS];
  int sum = 0;
#pragma unroll
  for (int q = 0; q < ITEMS; ++q) {
    const int e = t * ITEMS + q;
    v[q] = e < nb1 ? cnt[e] : 0;
    sum += v[q];
  }
  int incl = sum;
  const int lane = t & 63, w = t >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int run = incl - sum;
  for (int q = 0; q < w; ++q) run += wsum[q];
  run += rs;
#pragma unroll
  for (int q = 0; q < ITEMS; ++q) {
    const int e = t * ITEMS + q;
    if (e < nb1) {
      cnt[e] = run;
      boff[b0 * nb1 + e] = run;
    }
    run += v[q];
  }
  if (b0 == g.nb[0] - 1 && t == 0) boff[g.nb[0] * nb1] = re;
  __syncthreads();
  if (fits) {
    // rows that fit: the order is built in LDS first (perm[pos] = the row
    // entry claimed at pos; columns and keys kept by the counting pass, so the
    // records are not read again for the claims), so the sorted arrays are
    // written coalesced
    for (int i0 = rs + t; i0 < re; i0 += SU * BS) {
      int b[SU], pos[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) b[u] = i0 + u * BS < re ? (int)col[i0 + u * BS - rs] : -1;
      // branch-free claims (entries past the end add to a spare word per lane)
#pragma unroll
      for (int u = 0; u < SU; ++u) pos[u] = atomicAdd(&cnt[b[u] >= 0 ? b[u] : 4096 + (int)__lane_id()], 1);
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (b[u] >= 0) perm[pos[u] - rs] = (uint16_t)(i0 + u * BS - rs);
    }
    __syncthreads();
    // The claims above come in whatever order the lanes' atomics meet; each
    // sample then goes to its rank within its bin by caller index (low 16
    // bits first, the full index on equal low bits), so the order within a
    // bin, and everything summed in bin order, is the same on every run. The
    // counters now hold the end of each bin (the start of the next).
    for (int q0 = t; q0 < re - rs; q0 += SU * BS) {
      RowRec r[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int q = q0 + u * BS;
        if (q < re - rs) r[u] = rowbuf[rs + perm[q]];
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int q = q0 + u * BS;
        if (q < re - rs) {
          const int b = r[u].b1;
          const int bs = (b > 0 ? cnt[b - 1] : rs) - rs, be = cnt[b] - rs;
          const int kq = key[perm[q]];
          int rank = 0;
          for (int q2 = bs; q2 < be; ++q2) {
            const int k2 = key[perm[q2]];
            if (k2 < kq) {
              ++rank;
            } else if (k2 == kq && q2 != q) {
              if (rowbuf[rs + perm[q2]].j < r[u].j) ++rank;
            }
          }
          const int d = bs + rank;
          WSample<2> smp;
          smp.k[0] = r[u].k0;
          smp.k[1] = r[u].k1;
          sincospi(r[u].k0, &smp.sc[0][0], &smp.sc[0][1]);
          sincospi(r[u].k1, &smp.sc[1][0], &smp.sc[1][1]);
          ss[rs + d] = smp;
          sidx[rs + d] = r[u].j;
          if (inv) inv[r[u].j] = rs + d;
          if (sums) sums[rs + d] = wself<2>();   // the self term
        }
      }
    }
    return;
  }
  for (int i = rs + t; i < re; i += BS) {
    const RowRec r = rowbuf[i];
    const int pos = atomicAdd(&cnt[r.b1], 1);
    WSample<2> smp;
    smp.k[0] = r.k0;
    smp.k[1] = r.k1;
    sincospi(r.k0, &smp.sc[0][0], &smp.sc[0][1]);
    sincospi(r.k1, &smp.sc[1][0], &smp.sc[1][1]);
    ss[pos] = smp;
    sidx[pos] = r.j;
    if (sums) sums[pos] = wself<2>();
  }
  // Rows too long for LDS were placed in claim order; each of their bins is
  // then put in caller-index order (an insertion sort by one thread per bin,
  // on the records the workgroup has just written: the barrier makes them
  // visible), and the inverse map written from that order.
  __syncthreads();
  for (int c = t; c < nb1; c += BS) {
    const int bs = boff[b0 * nb1 + c], be = c + 1 < nb1 ? boff[b0 * nb1 + c + 1] : re;
    for (int i = bs + 1; i < be; ++i) {
      const WSample<2> w = ss[i];
      const int32_t j = sidx[i];
      int p = i;
      while (p > bs && sidx[p - 1] > j) {
        ss[p] = ss[p - 1];
        sidx[p] = sidx[p - 1];
        --p;
      }
      ss[p] = w;
      sidx[p] = j;
    }
    if (inv)
      for (int i = bs; i < be; ++i) inv[sidx[i]] = i;
  }
}

// buffers of the neighbour binning for the geometry in p->wgeom
void setup_weight_bins(ftcg_plan p) {
  const WBinGeom& g = p->wgeom;
  const int64_t m = p->m;
  const int64_t nbins = (int64_t)g.nb[0] * g.nb[1];
  p->wb_off.ensure(sizeof(int32_t) * (nbins + 1));
  p->wb_of.ensure(sizeof(int32_t) * m);
  p->ws_k.ensure(sizeof(double) * m * p->dim * 3);
  p->ws_idx.ensure(sizeof(int32_t) * m);
  p->ws_inv.ensure(sizeof(int32_t) * m);
}

// steps 1-3 of the 2D binning, with the geometry the input check left in
// device memory: rows are counted, the first nrows row counters scanned
// (WROW_MAX when the host has not read the geometry yet: rows past the
// geometry's count stay empty) and the samples placed in their row's range
void wrow_bin(ftcg_plan p, const double* k, int nrows) {
  const int64_t m = p->m;
  hipStream_t s = p->stream;
  const WBinGeom* gd = &p->geo.as<CheckOut>()->g;
  int32_t* row_cnt = p->wb_cnt.as<int32_t>();   // zeroed by the input check
  int32_t* row_off = p->wb_rowoff.as<int32_t>();
  // count rounds per workgroup: about 1024 workgroups, 1 to 8 rounds (a
  // 4096^2 raster: 0.058 -> 0.037 ms)
  const int64_t per_round = (int64_t)WROW_IPT * WB_BLOCK;
  const int rounds = (int)std::min<int64_t>(8, std::max<int64_t>(1, m / (1024 * per_round)));
  const unsigned nb = (unsigned)((m + rounds * per_round - 1) / (rounds * per_round));
  hipLaunchKernelGGL(k_wrow_count, dim3(nb), dim3(WB_BLOCK), 0, s, k, m, gd, row_cnt, rounds);
  exclusive_scan_i32(row_cnt, row_off, nrows, p->scan_tmp.as<int32_t>(), s, row_cnt);
  // the placement takes one round per workgroup: its rounds run one after
  // another (a 4096^2 raster: 8 rounds 0.18 ms against 0.11 ms for one)
  const unsigned nb1 = (unsigned)((m + per_round - 1) / per_round);
  hipLaunchKernelGGL(k_wrow_scatter, dim3(nb1), dim3(WB_BLOCK), 0, s, k, m, gd, row_cnt, p->wb_rowbuf.as<RowRec>(), 1);
  FTCG_HIP(hipGetLastError());
}

// step 4 of the 2D binning (rows placed by steps 1-3, here or fused with the
// tile binning)
void sort_weight_rows(ftcg_plan p) {
  const WBinGeom& g = p->wgeom;
  // the inverse map serves the learned features, the audit and the
  // record-order weights written by the finish of the weight sum
  const bool need_inv = p->wmode == FTCG_W_LEARNED || p->wmode == FTCG_W_BAND || p->weights_only || p->finish_recs;
  // the symmetric weight sum starts from the self terms, preset here
  p->ws_sum.ensure(sizeof(double) * p->m);
  auto launch = [&](auto kern, int bs) {
    hipLaunchKernelGGL(kern, dim3((unsigned)g.nb[0]), dim3(bs), 0, p->stream, g, p->wb_rowoff.as<int32_t>(),
                       p->wb_rowbuf.as<RowRec>(), p->wb_off.as<int32_t>(), p->ws_k.as<WSample<2>>(),
                       p->ws_idx.as<int32_t>(), need_inv ? p->ws_inv.as<int32_t>() : nullptr, p->ws_sum.as<double>());
  };
  if (p->m >= (int64_t)4096 * g.nb[0])   // rows of 4096 samples or more on average
    launch(k_wrow_sort<1024, WROW_LMAX_WIDE>, 1024);
  else
    launch(k_wrow_sort<WB_BLOCK, WROW_LMAX_NARROW>, WB_BLOCK);
  FTCG_HIP(hipGetLastError());
  p->ws_sum_fresh = true;
}

// 1D neighbour binning (after the host has read the geometry)
void build_weight_bins_1d(ftcg_plan p, const double* k) {
  setup_weight_bins(p);
  const WBinGeom g = p->wgeom;
  const int64_t m = p->m;
  const int64_t nbins = (int64_t)g.nb[0] * g.nb[1];
  hipStream_t s = p->stream;
  int32_t* off = p->wb_off.as<int32_t>();
  timing_begin(p, STEP_WBIN);
  const size_t cnt_bytes = sizeof(int32_t) * ((nbins + 4) & ~int64_t(3));  // 16-byte multiple: one fill
  p->wb_cnt.ensure(cnt_bytes);
  p->scan_tmp.ensure(scan_tmp_bytes(nbins));
  int32_t* cnt = p->wb_cnt.as<int32_t>();
  const unsigned nb = (unsigned)((m + WB_BLOCK - 1) / WB_BLOCK);
  FTCG_HIP(hipMemsetAsync(cnt, 0, cnt_bytes, s));
  hipLaunchKernelGGL(k_wbin_count<1>, dim3(nb), dim3(WB_BLOCK), 0, s, k, m, g, cnt, p->wb_of.as<int32_t>());
  exclusive_scan_i32(cnt, off, nbins, p->scan_tmp.as<int32_t>(), s, cnt);  // cnt becomes the cursor
  hipLaunchKernelGGL(k_wbin_scatter<1>, dim3(nb), dim3(WB_BLOCK), 0, s, k, m, p->wb_of.as<int32_t>(), cnt,
                     p->ws_k.as<WSample<1>>(), p->ws_idx.as<int32_t>(), p->ws_inv.as<int32_t>());
  FTCG_HIP(hipGetLastError());
  timing_end(p, STEP_WBIN);
  p->have_wbins = true;
}

template <int WT, int S>
static void launch_weights_rows(ftcg_plan p) {
  const WBinGeom& g = p->wgeom;
  const int64_t runs = (p->m * S + WB_BLOCK * WT - 1) / (WB_BLOCK * WT);
  // x extent: twice the mean runs per bin row, so dense rows are covered in
  // about one step while empty rows cost only idle workgroups
  const int cx = (int)std::max<int64_t>(1, (2 * runs + g.nb[0] - 1) / g.nb[0]);
  const int64_t nb = (int64_t)cx * g.nb[0];
  // XCD chunks of whole bands of nb0 / 64 bin rows: the rows a band stages
  // (its own and s more on each side) stay in one XCD's L2, and every XCD
  // still gets 8 bands spread over the raster
  const int chunk = cx * std::max(1, g.nb[0] / 64);
  hipLaunchKernelGGL((k_frame_weights_rows<WT, S>), dim3((unsigned)nb), dim3(WB_BLOCK), 0, p->stream,
                     p->ws_k.as<WSample<2>>(), p->ws_idx.as<int32_t>(), p->wb_off.as<int32_t>(), g, cx, chunk,
                     p->alpha.as<double>());
}

template <int WT, int S>
static void launch_weights_sym(ftcg_plan p) {
  const WBinGeom& g = p->wgeom;
  const int64_t m = p->m;
  double* wsum = p->ws_sum.as<double>();
  if (!p->ws_sum_fresh) {   // sums already used: start again from the self terms
    timing_begin(p, STEP_WFINISH);
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((m + WB_BLOCK - 1) / WB_BLOCK)), dim3(WB_BLOCK), 0, p->stream,
                       wsum, m, wself<2>());
    timing_end(p, STEP_WFINISH);
  }
  p->ws_sum_fresh = false;
  const int64_t runs = (m * S + WB_BLOCK * WT - 1) / (WB_BLOCK * WT);
  const int cx = (int)std::max<int64_t>(1, (2 * runs + g.nb[0] - 1) / g.nb[0]);
  const int64_t nb = (int64_t)cx * g.nb[0];
  const int chunk = cx * std::max(1, g.nb[0] / 64);
  // the weight step times this kernel alone (its launch is what the
  // roofline of the weight sum is measured on)
  timing_begin(p, STEP_WEIGHTS);
  hipLaunchKernelGGL((k_frame_weights_sym<WT, S>), dim3((unsigned)nb), dim3(WB_BLOCK), 0, p->stream,
                     p->ws_k.as<WSample<2>>(), p->wb_off.as<int32_t>(), g, cx, chunk, wsum);
  timing_end(p, STEP_WEIGHTS);
  if (p->finish_recs) {   // finished on demand (finish_deferred_weights) or inside the spread
    p->weights_deferred = true;
    p->finish_recs = false;
    return;
  }
  timing_begin(p, STEP_WFINISH);
  hipLaunchKernelGGL(k_weights_from_sums, dim3((unsigned)((m + WB_BLOCK - 1) / WB_BLOCK)), dim3(WB_BLOCK), 0,
                     p->stream, wsum, p->ws_idx.as<int32_t>(), m, p->alpha.as<double>());
  timing_end(p, STEP_WFINISH);
}

template <int WT>
static void launch_weights_rows_s(ftcg_plan p, int S) {
  switch (S) {
    case 1: launch_weights_rows<WT, 1>(p); break;
    case 2: launch_weights_rows<WT, 2>(p); break;
    default: launch_weights_rows<WT, 4>(p); break;
  }
}

template <int WT>
static void launch_weights_1d(ftcg_plan p) {
  const int64_t groups = (p->m + WT - 1) / WT;
  const unsigned nb = (unsigned)((groups + WB_BLOCK - 1) / WB_BLOCK);
  hipLaunchKernelGGL((k_frame_weights_1d<WT>), dim3(nb), dim3(WB_BLOCK), 0, p->stream, p->ws_k.as<WSample<1>>(),
                     p->ws_idx.as<int32_t>(), p->wb_off.as<int32_t>(), p->m, p->wgeom, p->alpha.as<double>());
}

void finish_deferred_weights(ftcg_plan p) {
  if (!p->weights_deferred) return;
  timing_begin(p, STEP_WFINISH);
  const int64_t m = p->m;
  const double* wsum = p->ws_sum.as<double>();
  const unsigned fb = (unsigned)std::min<int64_t>(2048, (2 * m + WB_BLOCK - 1) / WB_BLOCK);
  const int32_t* nrec = p->tile_off.as<int32_t>() + p->ntiles;
  if (p->dtype == FTCG_F64)
    hipLaunchKernelGGL(k_weights_from_sums_recs<double>, dim3(fb), dim3(WB_BLOCK), 0, p->stream, wsum,
                       p->ws_idx.as<int32_t>(), p->ws_inv.as<int32_t>(), m, p->alpha.as<double>(),
                       p->recs.as<Rec<double>>(), nrec, p->alpha_s.as<double>());
  else
    hipLaunchKernelGGL(k_weights_from_sums_recs<float>, dim3(fb), dim3(WB_BLOCK), 0, p->stream, wsum,
                       p->ws_idx.as<int32_t>(), p->ws_inv.as<int32_t>(), m, p->alpha.as<double>(),
                       p->recs.as<Rec<float>>(), nrec, p->alpha_s.as<float>());
  FTCG_HIP(hipGetLastError());
  timing_end(p, STEP_WFINISH);
  p->weights_deferred = false;
}

// samples per lane: the plan's tuning, else in 2D 2 from 2^20 samples (each
// staged candidate then serves two pairs and one LDS atomic; measured on SAS
// rasters of 2^20 and 2^23 samples: 0.371 against 0.402 ms and 1.76 against
// 1.92 ms) and 1 below (2^17 samples: 0.042 against 0.068 ms, where the
// lanes are too few); 1 in 1D
constexpr bool WEIGHT_SYMMETRIC = true;
constexpr int SYM_MAX_WT = 2;   // samples per lane the symmetric kernel is built for

void run_plain_weights(ftcg_plan p) {
  // candidates per sample (2D): the mean bin population times the window
  const WBinGeom& g = p->wgeom;
  const double cand =
      p->dim == 2 ? (double)p->m / ((double)g.nb[0] * g.nb[1]) * (2 * g.span + 1) * (2 * g.span + 1) : 0.0;
  // samples per lane: 2 in 2D from 2^20 samples, but 1 when a sample has more
  // than about 10^4 candidates (3.5 M samples on a 256^2 image: 39 against
  // 41 ms)
  const int wt = p->w_samples ? p->w_samples
                              : (p->dim == 2 && p->m >= (int64_t(1) << 20) && cand <= 1e4 ? 2 : 1);
  if (p->dim == 2) {
    // lanes per sample group: the plan's tuning, else 4 below 2^21 samples
    // and 2 from there, but 1 when a sample has more than about 10^4
    // candidates (measured on SAS rasters of 2^16 .. 2^23 samples at
    // 0.002 .. 13 samples per grid cell: long lists already fill the lanes,
    // and more lanes per sample only multiply the LDS staging per sample)
    const int S = p->w_lanes ? p->w_lanes : (cand > 1e4 ? 1 : (p->m < (int64_t(1) << 21) ? 4 : 2));
    if (wt <= SYM_MAX_WT && WEIGHT_SYMMETRIC) {
      const int key = (wt == 2 ? 10 : 0) + S;
      switch (key) {
        case 1: launch_weights_sym<1, 1>(p); break;
        case 2: launch_weights_sym<1, 2>(p); break;
        case 4: launch_weights_sym<1, 4>(p); break;
        case 11: launch_weights_sym<2, 1>(p); break;
        case 12: launch_weights_sym<2, 2>(p); break;
        default: launch_weights_sym<2, 4>(p); break;
      }
      FTCG_HIP(hipGetLastError());
      return;
    }
    timing_begin(p, STEP_WEIGHTS);
    switch (wt) {
      case 1: launch_weights_rows_s<1>(p, S); break;
      case 2: launch_weights_rows_s<2>(p, S); break;
      default: launch_weights_rows_s<4>(p, S); break;
    }
  } else {
    timing_begin(p, STEP_WEIGHTS);
    switch (wt) {
      case 1: launch_weights_1d<1>(p); break;
      case 2: launch_weights_1d<2>(p); break;
      default: launch_weights_1d<4>(p); break;
    }
  }
  FTCG_HIP(hipGetLastError());
  timing_end(p, STEP_WEIGHTS);
}

void plain_weights_at(ftcg_plan p, const double* k, const int32_t* idx, int64_t n, double* out) {
  if (n <= 0) return;
  const unsigned nb = (unsigned)((n * 64 + WB_BLOCK - 1) / WB_BLOCK);
  const int32_t* off = p->wb_off.as<int32_t>();
  if (p->dim == 1)
    hipLaunchKernelGGL(k_frame_weights_at<1>, dim3(nb), dim3(WB_BLOCK), 0, p->stream, p->ws_inv.as<int32_t>(),
                       idx, n, p->ws_k.as<WSample<1>>(), off, p->wgeom, out);
  else
    hipLaunchKernelGGL(k_frame_weights_at<2>, dim3(nb), dim3(WB_BLOCK), 0, p->stream, p->ws_inv.as<int32_t>(),
                       idx, n, p->ws_k.as<WSample<2>>(), off, p->wgeom, out);
  FTCG_HIP(hipGetLastError());
}

}  // namespace ftcg
