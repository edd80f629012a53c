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
//   e^{-beta (d+1)^2} = e^{-beta d^2} * q,  q_{next} = q * e^{-2 beta}.
//
// Two accumulations:
//   * float32 plans (k_spread2d_fx, the default): exact fixed-point integers,
//     one 64-bit LDS integer add per complex tap (see the block comment of
//     that kernel); on gfx950 the float32 LDS atomic add retires about 0.33
//     lanes per clock per CU and the 64-bit integer one about 9.9 (measured);
//   * float64 plans, and float32 plans that ask for it (k_spread2d,
//     k_spread1d): float64 LDS words with ds_add_f64; with lds_copies > 1
//     wave w accumulates into partial tile w % copies and the partial tiles
//     are combined at the flush with compensated (TwoSum) addition.
#include <type_traits>

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

// ---------------------------------------------------------------------------
// float32 plans, fixed-point tile accumulation (the default for FTCG_F32)
//
// Each tap value x (complex) is scaled by s = (2^31 - 2^24) / B_t, where B_t >=
// sum over the tile's records of max(|Re c_r|, |Im c_r|) bounds every cell of
// the tile (kernel values never exceed 1; B_t is formed from order-independent
// reductions, so it is the same for any record order), rounded to the nearest
// int32 per component (fx_pack), and both components are added with ONE
// 64-bit LDS integer atomic: the pair (re, im) is packed as im * 2^32 + re in
// two's complement, and integer addition of packed pairs adds both components
// exactly as long as neither sum leaves int32, which the bound guarantees (its
// 2^24 quanta of headroom also cover the half quantum each rounding may add).
// The accumulation is therefore exact and independent of record order
// (bitwise reproducible), and its only error is the rounding of each tap to
// the quantum 2^-31 B_t: unbiased, at most half a quantum per tap.
//
// The LDS tile carries 2W - 1 halo rows above and below, so the 2W rows of a
// record's footprint never need a bounds check (halo rows are dropped at the
// flush); columns outside the tile are skipped per lane.
// ---------------------------------------------------------------------------

// Records are staged in LDS in chunks of FX_STAGE (the first chunk while the
// bound is formed): each record's geometry, weight and sample value are read
// from global memory by one thread, in parallel over the workgroup, and the
// tap loop then reads LDS only, so the dependent record -> sample loads are
// not paid once per record batch of each wavefront (4096^2 SAS raster, 8.4M
// samples: 0.73 -> 0.59 ms; on small grids the LDS atomics bound the loop).
constexpr int FX_STAGE = 256;   // 6 KiB: keeps 7 workgroups of tile 32, W = 6 per CU

// SUMS: the records carry no weights yet; record r of sample j takes
// alpha_j = pi^2 pi^2 / wsum[inv[j]] (bin-order sums of the symmetric weight
// kernel, the same float64 division its finish does), rounded to float32
template <int W, int T, bool SUMS>
__global__ __launch_bounds__(SPREAD_BLOCK) void k_spread2d_fx(const Rec<float>* __restrict__ recs,
                                                              const float* __restrict__ alpha_s,
                                                              const double* __restrict__ wsum,
                                                              const int32_t* __restrict__ inv,
                                                              const int32_t* __restrict__ tile_off,
                                                              const float2* __restrict__ fhat,
                                                              float2* __restrict__ grid, int64_t G, int nt,
                                                              float beta) {
  auto weight = [&](int r, int src) -> float {
    if constexpr (SUMS)
      return (float)(wscale<2>() / wsum[inv[src]]);
    else
      return alpha_s[r];
  };
  constexpr int L = 2 * W;              // lanes per record / taps per axis
  constexpr int PAD = 2 * W - 1;        // halo rows each side
  constexpr int TP = T + 1;             // row pitch (64-bit words)
  constexpr int ROWS = T + 2 * PAD;
  // stage only while the tile and the stage fit 64 KiB of LDS together
  constexpr bool STAGED = ROWS * TP * 8 + FX_STAGE * 24 <= 64 * 1024;
  constexpr int STG = STAGED ? FX_STAGE : 1;
  __shared__ unsigned long long acc[ROWS * TP];
  __shared__ float4 sgeo[STG];          // f0, f1, c01 (bits), alpha
  __shared__ float2 sval[STG];          // fhat[src]
  __shared__ float red[SPREAD_BLOCK / 64];
  __shared__ long long red2[SPREAD_BLOCK / 64];

  const int tile = blockIdx.x;
  const int t0 = tile / nt, t1 = tile - (tile / nt) * nt;
  const int beg = tile_off[tile], end = tile_off[tile + 1];
  float2* out = grid + (int64_t)t0 * T * G + (int64_t)t1 * T;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  if (beg == end) {
    const float2 z = {0.f, 0.f};
    for (int idx = tid; idx < T * T; idx += SPREAD_BLOCK) out[(int64_t)(idx / T) * G + (idx % T)] = z;
    return;
  }
  // Bound of every cell of the tile, computed so that it does not depend on
  // the order of the records: first the largest |component| of alpha * fhat,
  // then the integer sum of each record's component bound rounded up in
  // units of 2^-20 of that maximum. The first pass stages the first chunk.
  const int first = STAGED ? min(end - beg, STG) : 0;
  float mx = 0.f;
  for (int r = beg + tid; r < end; r += SPREAD_BLOCK) {
    const Rec<float> rec = recs[r];
    const float a = weight(r, rec.src);
    const float2 v = fhat[rec.src];
    if (r - beg < first) {
      sgeo[r - beg] = make_float4(rec.f0, rec.f1, __int_as_float(rec.c01), a);
      sval[r - beg] = v;
    }
    const float cr = v.x * a, ci = v.y * a;
    // fmaxf drops NaN operands: flag non-finite values explicitly
    mx = (isfinite(cr) && isfinite(ci)) ? fmaxf(mx, fmaxf(fabsf(cr), fabsf(ci))) : __builtin_inff();
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if (lane == 0) red[wave] = mx;
  for (int idx = tid; idx < ROWS * TP; idx += SPREAD_BLOCK) acc[idx] = 0ull;
  __syncthreads();
  mx = 0.f;
#pragma unroll
  for (int w = 0; w < SPREAD_BLOCK / 64; ++w) mx = fmaxf(mx, red[w]);
  if (!(mx > 0.f) || !isfinite(mx)) {
    // all-zero tile, or non-finite values: propagate as the float path would
    const float fill = mx == 0.f ? 0.f : __builtin_nanf("");
    const float2 z = {fill, fill};
    for (int idx = tid; idx < T * T; idx += SPREAD_BLOCK) out[(int64_t)(idx / T) * G + (idx % T)] = z;
    return;
  }
  const float qs = 1048576.f / mx;
  long long qsum = 0;
  for (int r = beg + tid; r < end; r += SPREAD_BLOCK) {
    float a;
    float2 v;
    if (r - beg < first) {   // staged by this thread in the first pass
      a = sgeo[r - beg].w;
      v = sval[r - beg];
    } else {
      const int src = recs[r].src;
      a = weight(r, src);
      v = fhat[src];
    }
    qsum += (long long)ceilf(fmaxf(fabsf(v.x * a), fabsf(v.y * a)) * qs) + 1;
  }
  for (int off = 32; off > 0; off >>= 1) qsum += __shfl_xor(qsum, off);
  __syncthreads();
  if (lane == 0) reinterpret_cast<long long*>(red2)[wave] = qsum;
  __syncthreads();
  qsum = 0;
#pragma unroll
  for (int w = 0; w < SPREAD_BLOCK / 64; ++w) qsum += reinterpret_cast<long long*>(red2)[w];
  const float bound = (float)((double)qsum * (double)mx * (1.0 / 1048576.0) * (1.0 + 1e-6));
  const float scale = (2147483648.f - 16777216.f) / bound;

  constexpr int RPW = 64 / L;
  const int s = lane / L, i = lane - (lane / L) * L;
  const float e2b = __expf(-2.f * beta);
  constexpr int NWAVES = SPREAD_BLOCK / 64;
  // one record's 2W x 2W taps: lane i takes footprint column i
  auto splat = [&](float f0, float f1, int c01, float araw, float2 v) {
    const int c1 = c01 >> 16;
    const int col = c1 - W + 1 + i;
    if (col < 0 || col >= T) return;
    const float a = araw * scale;
    const int c0 = (int)(int16_t)(c01 & 0xffff);
    const float d1 = (float)(i - W + 1) - f1;
    const float d0 = (float)(1 - W) - f0;
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
  };
  if constexpr (STAGED) {
    for (int cb = beg; cb < end; cb += FX_STAGE) {
      const int cn = min(end - cb, FX_STAGE);
      if (cb != beg) {   // later chunks: restage once every wavefront has left the previous one
        __syncthreads();
        for (int r = tid; r < cn; r += SPREAD_BLOCK) {
          const Rec<float> rec = recs[cb + r];
          sgeo[r] = make_float4(rec.f0, rec.f1, __int_as_float(rec.c01), weight(cb + r, rec.src));
          sval[r] = fhat[rec.src];
        }
        __syncthreads();
      }
      // the RPW records of one pass are cn / RPW apart in the chunk: records
      // next to each other come from neighbouring samples of one pulse, whose
      // footprints overlap, and in one pass they would meet on the same LDS banks
      const int np = (cn + RPW - 1) / RPW;
      for (int pass = wave; pass < np; pass += NWAVES) {
        const int r = s * np + pass;
        if (s < RPW && r < cn) {
          const float4 g4 = sgeo[r];
          splat(g4.x, g4.y, __float_as_int(g4.z), g4.w, sval[r]);
        }
      }
    }
  } else {
    for (int base = beg + wave * RPW; base < end; base += NWAVES * RPW) {
      const int r = base + s;
      if (s < RPW && r < end) {
        const Rec<float> rec = recs[r];
        splat(rec.f0, rec.f1, rec.c01, weight(r, rec.src), fhat[rec.src]);
      }
    }
  }
  __syncthreads();
  const float unscale = bound / (2147483648.f - 16777216.f);
  for (int idx = tid; idx < T * T; idx += SPREAD_BLOCK) {
    const int row = idx / T, col = idx - (idx / T) * T;
    const unsigned long long vv = acc[(row + PAD) * TP + col];
    const int re = (int)(unsigned)(vv & 0xffffffffull);
    const int im = (int)((long long)(vv - (unsigned long long)(long long)re) >> 32);
    float2 o;
    o.x = (float)re * unscale;
    o.y = (float)im * unscale;
    out[(int64_t)row * G + col] = o;
  }
}

// ---------------------------------------------------------------------------
// Segmented float32 spread for large grids (the same exact fixed-point taps).
//
// The tile binning gives every tile the records of all samples whose
// footprint reaches it, so a sample near a tile edge has records in up to
// four tiles, and each walks all (2W)^2 taps (1.81 records per sample on the
// 4096^2 SAS raster at tile 32). Here one workgroup owns a segment of
// SEG_CW = 2 tile columns (64 cells) by K tile rows and walks its tile rows
// top to bottom, one step per tile row, taking the records of that row's two
// tiles. A record is used only in the tile where its sample is at home along
// the directions the segment covers: along rows, a record from the tile
// above or below is skipped (its home copy is taken in its own step) except
// in the segment's first and last step, where the home copy belongs to the
// next segment; along columns, a record of the left tile whose sample is at
// home in the right tile is skipped, and the other way round. So every
// sample is used once per segment it reaches (1.22 records per sample at
// K = 8 on the same raster).
//
// The step's LDS tile spans tile rows -(W-1) .. 32+W-1 (32 + 2W - 1 rows),
// which holds every tap of the step's home records. After the step, rows
// -(W-1) .. 31-(W-1) receive nothing more and are written out; the 2W - 1
// rows below them still receive taps from the next step's records, so they
// are carried in float (their fixed-point value times the step's quantum)
// and added to the next step's first 2W - 1 rows. Each step has its own
// bound B (the fixed-point kernel's rule over the step's records), so the
// carry is the sum of two exactly accumulated terms in a fixed order:
// deterministic, with one float rounding more than the tile kernel. Records
// from the neighbouring segments above and below (first and last step) have
// rows outside the LDS tile: they take a loop clipped to it.
// ---------------------------------------------------------------------------
constexpr int SEG_BLOCK = 512;
constexpr int SEG_CW = 2;               // tile columns per segment
constexpr int SEG_T = 32;               // tile edge
constexpr int SEG_COLS = SEG_CW * SEG_T;

template <int W, bool SUMS>
__global__ __launch_bounds__(SEG_BLOCK) void k_spread2d_seg(const Rec<float>* __restrict__ recs,
                                                            const float* __restrict__ alpha_s,
                                                            const double* __restrict__ wsum,
                                                            const int32_t* __restrict__ inv,
                                                            const int32_t* __restrict__ tile_off,
                                                            const float2* __restrict__ fhat,
                                                            float2* __restrict__ grid, int64_t G, int nt, int K,
                                                            float beta) {
  constexpr int L = 2 * W;
  constexpr int CROWS = 2 * W - 1;      // carried rows
  constexpr int ROWS = SEG_T + CROWS;   // LDS tile rows: tile rows -(W-1) .. SEG_T + W - 1
  constexpr int TP = SEG_COLS + 1;      // row pitch (64-bit words)
  __shared__ unsigned long long acc[ROWS * TP];
  __shared__ float2 carry[CROWS * SEG_COLS];
  __shared__ float2 sf[SEG_BLOCK];      // f0, f1
  __shared__ int sc[SEG_BLOCK];         // LDS row | LDS column << 16 of the record's first tap
  __shared__ float2 sv[SEG_BLOCK];      // alpha * fhat
  __shared__ float red[SEG_BLOCK / 64];
  __shared__ long long red2[SEG_BLOCK / 64];
  __shared__ int ncount[2];             // staged home records (from the front), clipped ones (from the back)

  auto weight = [&](int r, int src) -> float {
    if constexpr (SUMS)
      return (float)(wscale<2>() / wsum[inv[src]]);
    else
      return alpha_s[r];
  };
  const int ncs = nt / SEG_CW;
  const int seg = blockIdx.x / ncs, cs = blockIdx.x - (blockIdx.x / ncs) * ncs;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col_cell0 = cs * SEG_COLS;

  for (int idx = tid; idx < ROWS * TP; idx += SEG_BLOCK) acc[idx] = 0ull;
  for (int idx = tid; idx < CROWS * SEG_COLS; idx += SEG_BLOCK) carry[idx] = make_float2(0.f, 0.f);

  // record r of the step's two tiles [rb, rm) [rm, re): kept?, clipped?, and
  // the LDS position of its first tap
  struct Kept {
    bool keep, clip;
    int packed;
  };
  auto classify = [&](int r, int rm, int t, int c01) -> Kept {
    const int cc = r >= rm ? 1 : 0;
    const int l0 = (int)(int16_t)(c01 & 0xffff);
    const int l1 = c01 >> 16;
    const bool home0 = l0 >= 0 && l0 < SEG_T;
    const bool vk = home0 || (t == 0 && l0 < 0) || (t == K - 1 && l0 >= SEG_T);
    const bool hk = cc ? (l1 >= 0) : (l1 < SEG_T);
    Kept k;
    k.keep = vk && hk;
    k.clip = !home0;
    // LDS row of the first tap: tile row l0 - W + 1, LDS row 0 = tile row -(W-1)
    const int row0 = l0;
    const int col0 = l1 + cc * SEG_T - W + 1;
    k.packed = (int)(((uint32_t)row0 & 0xffffu) | ((uint32_t)col0 << 16));
    return k;
  };
  // stage one record (compacted: home records from the front, clipped ones
  // from the back of the stage)
  auto stage = [&](bool keep, bool clip, float f0, float f1, int packed, float2 c) {
    const unsigned long long bh = __ballot(keep && !clip), bc = __ballot(keep && clip);
    int baseh = 0, basec = 0;
    if (lane == 0) {
      if (bh) baseh = atomicAdd(&ncount[0], __popcll(bh));
      if (bc) basec = atomicAdd(&ncount[1], __popcll(bc));
    }
    baseh = __shfl(baseh, 0);
    basec = __shfl(basec, 0);
    if (keep) {
      const unsigned long long mine = clip ? bc : bh;
      const int rank = __popcll(mine & ((1ull << lane) - 1ull));
      const int slot = clip ? SEG_BLOCK - 1 - (basec + rank) : baseh + rank;
      sf[slot] = make_float2(f0, f1);
      sc[slot] = packed;
      sv[slot] = c;
    }
  };

  const float e2b = __expf(-2.f * beta);
  constexpr int RPW = 64 / L;
  const int s = lane / L, i = lane - (lane / L) * L;
  constexpr int NWAVES = SEG_BLOCK / 64;

  for (int t = 0; t < K; ++t) {
    const int trow = seg * K + t;
    const int key = trow * nt + cs * SEG_CW;
    const int rb = tile_off[key], rm = tile_off[key + 1], re = tile_off[key + 2];
    if (tid < 2) ncount[tid] = 0;
    __syncthreads();
    // pass 1: largest |component| of alpha * fhat over the kept records; the
    // first chunk of SEG_BLOCK records is staged
    float mx = 0.f;
    for (int cb = rb; cb < re; cb += SEG_BLOCK) {
      const int r = cb + tid;
      bool keep = false, clip = false;
      float2 c = make_float2(0.f, 0.f);
      float f0 = 0.f, f1 = 0.f;
      int packed = 0;
      if (r < re) {
        const Rec<float> rec = recs[r];
        const Kept k = classify(r, rm, t, rec.c01);
        keep = k.keep;
        clip = k.clip;
        packed = k.packed;
        if (keep) {
          const float a = weight(r, rec.src);
          const float2 v = fhat[rec.src];
          c = make_float2(v.x * a, v.y * a);
          f0 = rec.f0;
          f1 = rec.f1;
          mx = (isfinite(c.x) && isfinite(c.y)) ? fmaxf(mx, fmaxf(fabsf(c.x), fabsf(c.y))) : __builtin_inff();
        }
      }
      if (cb == rb) stage(keep, clip, f0, f1, packed, c);
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    mx = 0.f;
#pragma unroll
    for (int w = 0; w < NWAVES; ++w) mx = fmaxf(mx, red[w]);
    const bool bad = !isfinite(mx);
    float scale = 0.f, unscale = 0.f;
    if (mx > 0.f && !bad) {
      // pass 2: integer sum of each kept record's bound in units of 2^-20 mx
      const float qs = 1048576.f / mx;
      const int nh = ncount[0], ncl = ncount[1];
      long long qsum = 0;
      for (int q = tid; q < nh; q += SEG_BLOCK) {
        const float2 c = sv[q];
        qsum += (long long)ceilf(fmaxf(fabsf(c.x), fabsf(c.y)) * qs) + 1;
      }
      for (int q = tid; q < ncl; q += SEG_BLOCK) {
        const float2 c = sv[SEG_BLOCK - 1 - q];
        qsum += (long long)ceilf(fmaxf(fabsf(c.x), fabsf(c.y)) * qs) + 1;
      }
      for (int cb = rb + SEG_BLOCK; cb < re; cb += SEG_BLOCK) {
        const int r = cb + tid;
        if (r < re) {
          const Rec<float> rec = recs[r];
          if (classify(r, rm, t, rec.c01).keep) {
            const float a = weight(r, rec.src);
            const float2 v = fhat[rec.src];
            qsum += (long long)ceilf(fmaxf(fabsf(v.x * a), fabsf(v.y * a)) * qs) + 1;
          }
        }
      }
      for (int off = 32; off > 0; off >>= 1) qsum += __shfl_xor(qsum, off);
      __syncthreads();
      if (lane == 0) red2[wave] = qsum;
      __syncthreads();
      qsum = 0;
#pragma unroll
      for (int w = 0; w < NWAVES; ++w) qsum += red2[w];
      const float bound = (float)((double)qsum * (double)mx * (1.0 / 1048576.0) * (1.0 + 1e-6));
      scale = (2147483648.f - 16777216.f) / bound;
      unscale = bound / (2147483648.f - 16777216.f);

      // one record's taps: lane i takes LDS column col0 + i, rows row0 .. row0
      // + 2W - 1 (clipped to the LDS tile when clip)
      auto splat = [&](float2 f, int packed, float2 c, bool clip) {
        const int col = (packed >> 16) + i;
        if (col < 0 || col >= SEG_COLS) return;
        const int row0 = (int)(int16_t)(packed & 0xffff);
        const float d1 = (float)(i - W + 1) - f.y;
        int j0 = 0, j1 = L;
        if (clip) {
          j0 = max(0, -row0);
          j1 = min(L, ROWS - row0);
        }
        const float d0 = (float)(1 - W + j0) - f.x;
        const float w10 = __expf(-beta * (d1 * d1 + d0 * d0)) * scale;
        float q = __expf(-beta * (2.f * d0 + 1.f));
        float pr = c.x * w10, pi = c.y * w10;
        unsigned long long* dst = acc + (row0 + j0) * TP + col;
        if (!clip) {
#pragma unroll
          for (int j = 0; j < L; ++j) {
            __hip_atomic_fetch_add(dst + j * TP, fx_pack(pr, pi), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            pr *= q;
            pi *= q;
            q *= e2b;
          }
        } else {
          for (int j = j0; j < j1; ++j) {
            __hip_atomic_fetch_add(dst, fx_pack(pr, pi), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            dst += TP;
            pr *= q;
            pi *= q;
            q *= e2b;
          }
        }
      };
      // taps of the staged records: home ones, then clipped ones; the RPW
      // records of one pass are n / RPW apart (neighbouring samples of a pulse
      // overlap and would meet on the same LDS banks)
      auto taps = [&]() {
        const int nh = ncount[0], ncl = ncount[1];
        const int nph = (nh + RPW - 1) / RPW;
        for (int pass = wave; pass < nph; pass += NWAVES) {
          const int r = s * nph + pass;
          if (s < RPW && r < nh) splat(sf[r], sc[r], sv[r], false);
        }
        const int npc = (ncl + RPW - 1) / RPW;
        for (int pass = wave; pass < npc; pass += NWAVES) {
          const int r = s * npc + pass;
          if (s < RPW && r < ncl) {
            const int q = SEG_BLOCK - 1 - r;
            splat(sf[q], sc[q], sv[q], true);
          }
        }
      };
      taps();
      for (int cb = rb + SEG_BLOCK; cb < re; cb += SEG_BLOCK) {
        __syncthreads();   // every wavefront has left the previous chunk
        if (tid < 2) ncount[tid] = 0;
        __syncthreads();
        const int r = cb + tid;
        bool keep = false, clip = false;
        float2 c = make_float2(0.f, 0.f);
        float f0 = 0.f, f1 = 0.f;
        int packed = 0;
        if (r < re) {
          const Rec<float> rec = recs[r];
          const Kept k = classify(r, rm, t, rec.c01);
          keep = k.keep;
          clip = k.clip;
          packed = k.packed;
          if (keep) {
            const float a = weight(r, rec.src);
            const float2 v = fhat[rec.src];
            c = make_float2(v.x * a, v.y * a);
            f0 = rec.f0;
            f1 = rec.f1;
          }
        }
        stage(keep, clip, f0, f1, packed, c);
        __syncthreads();
        taps();
      }
    }
    __syncthreads();
    // write the rows that are final, carry the 2W - 1 rows below them
    const int bmin = t == 0 ? W - 1 : 0;
    const int bmax = t == K - 1 ? SEG_T + W - 1 : SEG_T;
    const int64_t row_cell0 = (int64_t)trow * SEG_T - (W - 1);
    const float fill = bad ? __builtin_nanf("") : 0.f;
    for (int idx = tid; idx < bmax * SEG_COLS; idx += SEG_BLOCK) {
      const int b = idx / SEG_COLS, col = idx - (idx / SEG_COLS) * SEG_COLS;
      float2 o;
      {
        const unsigned long long vv = acc[b * TP + col];
        const int re_ = (int)(unsigned)(vv & 0xffffffffull);
        const int im_ = (int)((long long)(vv - (unsigned long long)(long long)re_) >> 32);
        o.x = bad ? fill : (float)re_ * unscale;
        o.y = bad ? fill : (float)im_ * unscale;
      }
      if (b < CROWS) {
        const float2 cy = carry[b * SEG_COLS + col];
        o.x += cy.x;
        o.y += cy.y;
        if (t < K - 1) {
          const unsigned long long vv = acc[(SEG_T + b) * TP + col];
          const int re_ = (int)(unsigned)(vv & 0xffffffffull);
          const int im_ = (int)((long long)(vv - (unsigned long long)(long long)re_) >> 32);
          float2 nc;
          nc.x = bad ? fill : (float)re_ * unscale;
          nc.y = bad ? fill : (float)im_ * unscale;
          carry[b * SEG_COLS + col] = nc;
        }
      }
      if (b >= bmin) grid[(row_cell0 + b) * G + col_cell0 + col] = o;
    }
    __syncthreads();
    if (t + 1 < K)
      for (int idx = tid; idx < ROWS * TP; idx += SEG_BLOCK) acc[idx] = 0ull;
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

template <int W, int T>
static void launch_fx(ftcg_plan p, const void* fhat, void* grid) {
  if (p->weights_deferred)
    hipLaunchKernelGGL((k_spread2d_fx<W, T, true>), dim3((unsigned)p->ntiles), dim3(SPREAD_BLOCK), 0, p->stream,
                       p->recs.as<Rec<float>>(), p->alpha_s.as<float>(), p->ws_sum.as<double>(),
                       p->ws_inv.as<int32_t>(), p->tile_off.as<int32_t>(), static_cast<const float2*>(fhat),
                       static_cast<float2*>(grid), p->G, (int)p->nt, (float)p->beta);
  else
    hipLaunchKernelGGL((k_spread2d_fx<W, T, false>), dim3((unsigned)p->ntiles), dim3(SPREAD_BLOCK), 0, p->stream,
                       p->recs.as<Rec<float>>(), p->alpha_s.as<float>(), nullptr, nullptr,
                       p->tile_off.as<int32_t>(), static_cast<const float2*>(fhat), static_cast<float2*>(grid),
                       p->G, (int)p->nt, (float)p->beta);
}

// segments of K tile rows for the segmented kernel on grids with enough of
// them to fill the chip (at least 2048 workgroups), else 0 (the tile kernel)
static int spread_segment_rows(const ftcg_plan_s* p) {
  if (p->dim != 2 || p->dtype != FTCG_F32 || p->accum != ACCUM_FIXED || p->tile != SEG_T) return 0;
  const int64_t nt = p->nt;
  if (nt % SEG_CW != 0) return 0;
  for (int K : {8, 4})
    if (nt % K == 0 && (nt / SEG_CW) * (nt / K) >= 2048) return K;
  return 0;
}

template <int W>
static void launch_seg(ftcg_plan p, const void* fhat, void* grid, int K) {
  const unsigned nb = (unsigned)((p->nt / SEG_CW) * (p->nt / K));
  if (p->weights_deferred)
    hipLaunchKernelGGL((k_spread2d_seg<W, true>), dim3(nb), dim3(SEG_BLOCK), 0, p->stream, p->recs.as<Rec<float>>(),
                       p->alpha_s.as<float>(), p->ws_sum.as<double>(), p->ws_inv.as<int32_t>(),
                       p->tile_off.as<int32_t>(), static_cast<const float2*>(fhat), static_cast<float2*>(grid), p->G,
                       (int)p->nt, K, (float)p->beta);
  else
    hipLaunchKernelGGL((k_spread2d_seg<W, false>), dim3(nb), dim3(SEG_BLOCK), 0, p->stream,
                       p->recs.as<Rec<float>>(), p->alpha_s.as<float>(), nullptr, nullptr, p->tile_off.as<int32_t>(),
                       static_cast<const float2*>(fhat), static_cast<float2*>(grid), p->G, (int)p->nt, K,
                       (float)p->beta);
}

template <int W>
static void launch_fx_t(ftcg_plan p, const void* fhat, void* grid) {
  if (p->spread_segments) {
    const int K = spread_segment_rows(p);
    if (K > 0) {
      launch_seg<W>(p, fhat, grid, K);
      FTCG_HIP(hipGetLastError());
      return;
    }
  }
  switch (p->tile) {
    case 16: launch_fx<W, 16>(p, fhat, grid); break;
    case 32: launch_fx<W, 32>(p, fhat, grid); break;
    case 64: launch_fx<W, 64>(p, fhat, grid); break;
    case 128: launch_fx<W, 128>(p, fhat, grid); break;
    default: throw StatusError{FTCG_EUNSUPPORTED};
  }
  FTCG_HIP(hipGetLastError());
}

template <class real, int W>
static void launch_spread_w(ftcg_plan p, const void* fhat, void* grid) {
  using cx = typename Cx<real>::t;
  const int T = p->tile;
  if (std::is_same<real, float>::value && p->dim == 2 && p->accum == ACCUM_FIXED) {
    launch_fx_t<W>(p, fhat, grid);   // forms deferred weights itself
    return;
  }
  finish_deferred_weights(p);          // the other kernels read the records' weights
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
