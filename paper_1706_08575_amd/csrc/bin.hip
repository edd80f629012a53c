// Geometry stage: input checks, tile binning of spread records, and the
// neighbour binning used by the frame-weight sum.
//
// Tile binning (counting sort by tile): every sample j has grid position
// u_j = sigma k_j + G/2 per axis, taken modulo G and evaluated in float64.
// Its footprint covers cells floor(u) - W + 1 .. floor(u) + W per axis, which
// touches one or two tiles per axis; the sample gets one record per touched
// tile, so each tile can later be accumulated and written by one workgroup
// without global atomics. Records keep the integer cell relative to the tile
// origin and the fractional position u - floor(u) (exact in float64, rounded
// once to the spread precision), so the float32 path never handles absolute
// grid coordinates.
#include "ftcg_internal.h"
#include "wbins.h"

namespace ftcg {

constexpr int BIN_BLOCK = 256;

// ---------------------------------------------------------------------------
// input check: finiteness and bounding box (order-preserving integer encoding)
// ---------------------------------------------------------------------------

__device__ inline unsigned long long ordered_bits(double x) {
  unsigned long long b = __double_as_longlong(x);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// One pass over the points in at most CHECK_PARTS workgroups. Workgroup b
// reduces its points with wavefront shuffles and LDS and writes five words to
// part[5 b ..]: a non-finite flag, then the per-axis minimum and maximum as
// order-preserving integers; one workgroup of k_check_reduce then reduces the
// partials (no atomics, no initialisation pass). The same launch zeroes zero_a[0 .. zero_na) and
// zero_b[0 .. zero_nb), the counters of the binnings that follow.
// VEC: 2D points read as one 16-byte word each (k 16-byte aligned), 8 in
// flight per thread
template <bool VEC>
__global__ __launch_bounds__(BIN_BLOCK) void k_check_points(const double* __restrict__ k, int64_t m, int dim,
                                                            unsigned long long* __restrict__ part,
                                                            int32_t* __restrict__ zero_a, int64_t zero_na,
                                                            int32_t* __restrict__ zero_b, int64_t zero_nb) {
  __shared__ unsigned long long sred[4][BIN_BLOCK / 64];
  __shared__ int sbad;
  const int64_t gt = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x, gs = (int64_t)gridDim.x * BIN_BLOCK;
  for (int64_t i = gt; i < zero_na; i += gs) zero_a[i] = 0;
  for (int64_t i = gt; i < zero_nb; i += gs) zero_b[i] = 0;
  if (threadIdx.x == 0) sbad = 0;
  unsigned long long lo[2] = {~0ull, ~0ull}, hi[2] = {0ull, 0ull};
  bool bad = false;
  // CHECK_UNROLL points per thread per step, all loaded before any is used
  constexpr int CHECK_UNROLL = VEC ? 8 : 4;
  for (int64_t j0 = gt; j0 < m; j0 += CHECK_UNROLL * gs) {
    double x[CHECK_UNROLL][2];
#pragma unroll
    for (int u = 0; u < CHECK_UNROLL; ++u) {
      const int64_t j = j0 + u * gs;
      if constexpr (VEC) {
        const double2 v = j < m ? reinterpret_cast<const double2*>(k)[j] : make_double2(0.0, 0.0);
        x[u][0] = v.x;
        x[u][1] = v.y;
      } else {
        x[u][0] = j < m ? k[j * dim] : 0.0;
        x[u][1] = (j < m && dim == 2) ? k[j * dim + 1] : 0.0;
      }
    }
    // (branch-free; the axis loop has a compile-time bound for 2D points)
    const int nd = VEC ? 2 : dim;
#pragma unroll
    for (int u = 0; u < CHECK_UNROLL; ++u) {
      const bool in = j0 + u * gs < m;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (a >= nd) break;
        const bool fin = isfinite(x[u][a]);
        bad = bad || (in && !fin);
        const bool use = in && fin;
        const unsigned long long o = ordered_bits(x[u][a]);
        lo[a] = (use && o < lo[a]) ? o : lo[a];
        hi[a] = (use && o > hi[a]) ? o : hi[a];
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const unsigned long long x = __shfl_xor(lo[a], off, 64);
      const unsigned long long y = __shfl_xor(hi[a], off, 64);
      lo[a] = x < lo[a] ? x : lo[a];
      hi[a] = y > hi[a] ? y : hi[a];
    }
  }
  __syncthreads();
  if (bad) sbad = 1;
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sred[0][w] = lo[0];
    sred[1][w] = lo[1];
    sred[2][w] = hi[0];
    sred[3][w] = hi[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long* o = part + 5 * blockIdx.x;
    o[0] = sbad ? 1ull : 0ull;
    for (int a = 0; a < 2; ++a) {
      unsigned long long l = sred[a][0], h = sred[2 + a][0];
      for (int v = 1; v < BIN_BLOCK / 64; ++v) {
        l = sred[a][v] < l ? sred[a][v] : l;
        h = sred[2 + a][v] > h ? sred[2 + a][v] : h;
      }
      o[1 + a] = l;
      o[3 + a] = h;
    }
  }
}

int launch_check_points(ftcg_plan p, const double* k, int64_t m, unsigned long long* part, int32_t* zero_a,
                        int64_t zero_na, int32_t* zero_b, int64_t zero_nb) {
  int64_t nb = (m + 2 * BIN_BLOCK - 1) / (2 * BIN_BLOCK);  // 2 points per thread at least
  if (nb > CHECK_PARTS) nb = CHECK_PARTS;
  if (nb < 1) nb = 1;
  if (p->dim == 2 && reinterpret_cast<uintptr_t>(k) % 16 == 0)
    hipLaunchKernelGGL(k_check_points<true>, dim3((unsigned)nb), dim3(BIN_BLOCK), 0, p->stream, k, m, p->dim, part,
                       zero_a, zero_na, zero_b, zero_nb);
  else
    hipLaunchKernelGGL(k_check_points<false>, dim3((unsigned)nb), dim3(BIN_BLOCK), 0, p->stream, k, m, p->dim, part,
                       zero_a, zero_na, zero_b, zero_nb);
  FTCG_HIP(hipGetLastError());
  return (int)nb;
}

// ---------------------------------------------------------------------------
// tile binning
// ---------------------------------------------------------------------------

struct TileGeom {
  double sigma, half_g;   // u = sigma k + G/2
  int64_t G;
  int T;                  // tile edge
  int nt;                 // tiles per axis
  int W;
  int tshift;             // log2 T when T is a power of two, else -1
  double inv_g;           // 1 / G, used (exactly) when G is a power of two, else 0
};

__device__ inline int floor_div(int a, int b) {  // b > 0
  int q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

__device__ inline int wrap_tile(int t, int nt) { return t < 0 ? t + nt : (t >= nt ? t - nt : t); }

// u modulo G in [0, G). Rounding can land exactly on G; anything still
// outside [0, G) (a non-finite u, or |u| so large that the reduction has no
// bits left) becomes 0, so every tile key stays in range for any input. The
// binning can run before the host has seen the input check, which then
// rejects non-finite samples. Where G is a power of two (the usual case),
// u / G is exactly u * (1 / G), and where the tile edge T is one,
// floor(a / T) is exactly a >> log2 T: the same results bit for bit without
// the divisions.
__device__ inline double wrap_u(double u, const TileGeom& g) {
  const double G = (double)g.G;
  double w = u - G * floor(g.inv_g != 0.0 ? u * g.inv_g : u / G);
  if (w >= G) w -= G;
  return (w >= 0.0 && w < G) ? w : 0.0;
}
__device__ inline int tile_floor(int a, const TileGeom& g) { return g.tshift >= 0 ? a >> g.tshift : floor_div(a, g.T); }

template <int DIM>
__device__ inline void sample_tiles(const double* __restrict__ k, int64_t j, const TileGeom& g, double* u,
                                    int* c, int* tlo, int* thi) {
  for (int a = 0; a < DIM; ++a) {
    u[a] = wrap_u(g.sigma * k[j * DIM + a] + g.half_g, g);
    c[a] = (int)floor(u[a]);
    tlo[a] = tile_floor(c[a] - g.W + 1, g);
    thi[a] = tile_floor(c[a] + g.W, g);
  }
}

// up to 2^DIM (tile, local cell) pairs of one sample, invalid slots have key -1
template <int DIM>
__device__ inline void sample_keys(const double* __restrict__ k, int64_t j, int64_t m, const TileGeom& g,
                                   double* u, int* c, int* key, int* l0, int* l1) {
  int tlo[DIM], thi[DIM];
  for (int q = 0; q < 4; ++q) key[q] = -1;
  if (j >= m) return;
  sample_tiles<DIM>(k, j, g, u, c, tlo, thi);
  int q = 0;
  for (int t0 = tlo[0]; t0 <= thi[0]; ++t0) {
    if (DIM == 1) {
      key[q] = wrap_tile(t0, g.nt);
      l0[q] = c[0] - t0 * g.T;
      l1[q] = 0;
      ++q;
    } else {
      for (int t1 = tlo[DIM - 1]; t1 <= thi[DIM - 1]; ++t1) {
        key[q] = wrap_tile(t0, g.nt) * g.nt + wrap_tile(t1, g.nt);
        l0[q] = c[0] - t0 * g.T;
        l1[q] = c[DIM - 1] - t1 * g.T;
        ++q;
      }
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(BIN_BLOCK) void k_tile_count(const double* __restrict__ k, int64_t m, TileGeom g,
                                                          int32_t* __restrict__ cnt) {
  const int64_t j = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x;
  double u[DIM];
  int c[DIM], key[4], l0[4], l1[4];
  sample_keys<DIM>(k, j, m, g, u, c, key, l0, l1);
  // counts need no result: the leaders' atomics are not waited for
#pragma unroll
  for (int q = 0; q < (1 << DIM); ++q) {
    const KeyGroup kg = key_group(key[q], key[q] >= 0);
    if (kg.leader == (int)__lane_id()) atomicAdd(&cnt[key[q]], kg.size);
  }
}

template <int DIM, class real>
__global__ __launch_bounds__(BIN_BLOCK) void k_tile_scatter(const double* __restrict__ k, int64_t m, TileGeom g,
                                                            const double* __restrict__ alpha,
                                                            int32_t* __restrict__ cursor,
                                                            Rec<real>* __restrict__ recs,
                                                            real* __restrict__ alpha_s) {
  const int64_t j = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x;
  double u[DIM] = {};
  int c[DIM] = {}, key[4], l0[4], l1[4];
  sample_keys<DIM>(k, j, m, g, u, c, key, l0, l1);
  const real a = (j < m && alpha) ? (real)alpha[j] : (real)1;
  Rec<real> r;
  r.f0 = (real)(u[0] - (double)c[0]);
  r.f1 = (DIM == 2) ? (real)(u[DIM - 1] - (double)c[DIM - 1]) : (real)0;
  r.src = (int32_t)j;
  // every slot's groups claim their ranges before any claim is waited for
  KeyGroup kg[1 << DIM];
  int base[1 << DIM];
#pragma unroll
  for (int q = 0; q < (1 << DIM); ++q) kg[q] = key_group(key[q], key[q] >= 0);
#pragma unroll
  for (int q = 0; q < (1 << DIM); ++q) base[q] = group_claim(cursor, key[q], kg[q]);
#pragma unroll
  for (int q = 0; q < (1 << DIM); ++q) {
    const int pos = group_slot(base[q], kg[q]);
    if (key[q] >= 0) {
      r.c01 = (int32_t)(((uint32_t)l0[q] & 0xffffu) | ((uint32_t)l1[q] << 16));
      recs[pos] = r;
      alpha_s[pos] = a;
    }
  }
}

// The same two steps with the counters privatised in LDS, for up to
// LDS_TILE_KEYS tiles: a workgroup takes BIN_IPT * BIN_BLOCK consecutive
// samples (coalesced, all loads issued before the first count), counts their
// records in LDS, and only then touches the global counters, once per tile
// it saw. The scatter claims one range per tile with that count and hands
// out positions inside it from LDS. The LDS counters take one atomic per
// lane: lanes of a wavefront that hit the same counter are serialised inside
// that one instruction, and the atomics of all of a thread's records are in
// flight together (a wavefront-aggregated increment would wait for each
// distinct key's result in turn).
constexpr int BIN_IPT = 2;
constexpr int LDS_TILE_KEYS = 4096;   // 16 KiB of int32 counters (larger tables cost more LDS
                                      // occupancy than the global counters they replace)

// Slot claims take no branch (so all of them are issued before the first
// result is used): a lane without a key adds to its own spare counter in the
// 64 words past the live ones, at index spare + lane.
constexpr int LDS_SPARE = 64;
__device__ inline int lds_claim(int32_t* cnt, int key, int spare) {
  return atomicAdd(&cnt[key >= 0 ? key : spare + (int)__lane_id()], 1);
}

// rounds of BIN_IPT * BIN_BLOCK samples per workgroup: about one sample per
// two LDS counters cleared and flushed, at most 8 rounds (two samples per
// thread and round: the 512^2 SAS raster, 2^17 samples, then fills 256
// workgroups instead of 128; binning 33 -> 30 us)
static int bin_rounds(int64_t ncounters) {
  return (int)std::min<int64_t>(8, std::max<int64_t>(1, ncounters / (4 * BIN_BLOCK)));
}

template <int DIM>
__device__ inline void block_keys(const double* __restrict__ k, int64_t m, const TileGeom& g, int64_t j0,
                                  double (&u)[BIN_IPT][DIM], int (&c)[BIN_IPT][DIM], int (&key)[BIN_IPT][4],
                                  int (&l0)[BIN_IPT][4], int (&l1)[BIN_IPT][4]) {
#pragma unroll
  for (int i = 0; i < BIN_IPT; ++i)
    sample_keys<DIM>(k, j0 + (int64_t)i * BIN_BLOCK + threadIdx.x, m, g, u[i], c[i], key[i], l0[i], l1[i]);
}

// A workgroup takes `rounds` consecutive groups of BIN_IPT * BIN_BLOCK
// samples, so the clearing and flushing of its LDS counters is spread over
// rounds * BIN_IPT * BIN_BLOCK samples (rounds > 1 for large key counts).
template <int DIM>
__global__ __launch_bounds__(BIN_BLOCK) void k_tile_count_lds(const double* __restrict__ k, int64_t m, TileGeom g,
                                                              int32_t* __restrict__ cnt, int nkeys, int rounds) {
  extern __shared__ int32_t hist[];
  for (int i = threadIdx.x; i < nkeys; i += BIN_BLOCK) hist[i] = 0;
  __syncthreads();
  for (int rd = 0; rd < rounds; ++rd) {
    double u[BIN_IPT][DIM];
    int c[BIN_IPT][DIM], key[BIN_IPT][4], l0[BIN_IPT][4], l1[BIN_IPT][4];
    block_keys<DIM>(k, m, g, ((int64_t)blockIdx.x * rounds + rd) * BIN_IPT * BIN_BLOCK, u, c, key, l0, l1);
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i)
#pragma unroll
      for (int q = 0; q < (1 << DIM); ++q)
        if (key[i][q] >= 0) atomicAdd(&hist[key[i][q]], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nkeys; i += BIN_BLOCK) {
    const int v = hist[i];
    if (v) atomicAdd(&cnt[i], v);
  }
}

template <int DIM, class real>
__global__ __launch_bounds__(BIN_BLOCK) void k_tile_scatter_lds(const double* __restrict__ k, int64_t m, TileGeom g,
                                                                const double* __restrict__ alpha,
                                                                int32_t* __restrict__ cursor, int nkeys, int rounds,
                                                                Rec<real>* __restrict__ recs,
                                                                real* __restrict__ alpha_s) {
  extern __shared__ int32_t base[];   // nkeys counters, then LDS_SPARE spare words
  for (int i = threadIdx.x; i < nkeys; i += BIN_BLOCK) base[i] = 0;
  __syncthreads();
  for (int rd = 0; rd < rounds; ++rd) {
    double u[BIN_IPT][DIM];
    int c[BIN_IPT][DIM], key[BIN_IPT][4], l0[BIN_IPT][4], l1[BIN_IPT][4];
    block_keys<DIM>(k, m, g, ((int64_t)blockIdx.x * rounds + rd) * BIN_IPT * BIN_BLOCK, u, c, key, l0, l1);
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i)
#pragma unroll
      for (int q = 0; q < (1 << DIM); ++q)
        if (key[i][q] >= 0) atomicAdd(&base[key[i][q]], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nkeys; i += BIN_BLOCK) {
    const int v = base[i];
    if (v) base[i] = atomicAdd(&cursor[i], v);
  }
  __syncthreads();
  for (int rd = 0; rd < rounds; ++rd) {
    const int64_t j0 = ((int64_t)blockIdx.x * rounds + rd) * BIN_IPT * BIN_BLOCK;
    double u[BIN_IPT][DIM];
    int c[BIN_IPT][DIM], key[BIN_IPT][4], l0[BIN_IPT][4], l1[BIN_IPT][4];
    block_keys<DIM>(k, m, g, j0, u, c, key, l0, l1);
    int pos[BIN_IPT][4];
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i)
#pragma unroll
      for (int q = 0; q < (1 << DIM); ++q) pos[i][q] = lds_claim(base, key[i][q], nkeys);
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i) {
      const int64_t j = j0 + (int64_t)i * BIN_BLOCK + threadIdx.x;
      const real a = (j < m && alpha) ? (real)alpha[j] : (real)1;
      Rec<real> r;
      r.f0 = (real)(u[i][0] - (double)c[i][0]);
      r.f1 = (DIM == 2) ? (real)(u[i][DIM - 1] - (double)c[i][DIM - 1]) : (real)0;
      r.src = (int32_t)j;
#pragma unroll
      for (int q = 0; q < (1 << DIM); ++q) {
        if (key[i][q] >= 0) {
          r.c01 = (int32_t)(((uint32_t)l0[i][q] & 0xffffu) | ((uint32_t)l1[i][q] << 16));
          recs[pos[i][q]] = r;
          alpha_s[pos[i][q]] = a;
        }
      }
    }
  }
}

// Tile binning fused with the first steps of the 2D neighbour binning (the
// bin-row counting sort of the weight sum): one pass counts each sample's
// tile records and its bin row in two LDS histograms (tiles first, then the
// <= 4096 rows), one launch scans both counter arrays, and one pass claims
// ranges for both and writes the tile records (without weights: the weights
// are computed after this pass) and the row-grouped samples. Samples are
// read once per pass instead of twice.
__device__ inline void bin2_keys(const double* __restrict__ k, int64_t m, const TileGeom& tg, const WBinGeom& wg,
                                 int64_t j0, double (&u)[BIN_IPT][2], int (&c)[BIN_IPT][2], int (&key)[BIN_IPT][4],
                                 int (&l0)[BIN_IPT][4], int (&l1)[BIN_IPT][4], int (&row)[BIN_IPT],
                                 int (&col)[BIN_IPT], double (&x)[BIN_IPT][2]) {
  block_keys<2>(k, m, tg, j0, u, c, key, l0, l1);
#pragma unroll
  for (int i = 0; i < BIN_IPT; ++i) {
    const int64_t j = j0 + (int64_t)i * BIN_BLOCK + threadIdx.x;
    row[i] = j < m ? wbin_row_col(k, j, wg, &col[i], x[i]) : -1;
  }
}

template <class real>
__global__ __launch_bounds__(BIN_BLOCK) void k_bin2_count(const double* __restrict__ k, int64_t m, TileGeom tg,
                                                          const WBinGeom* __restrict__ wgp,
                                                          int32_t* __restrict__ tile_cnt, int ntiles,
                                                          int32_t* __restrict__ row_cnt, int rounds) {
  const WBinGeom wg = *wgp;
  extern __shared__ int32_t sm[];
  int32_t* ht = sm;
  int32_t* hr = sm + ntiles;
  const int nrow = wg.nb[0];
  for (int i = threadIdx.x; i < ntiles + nrow; i += BIN_BLOCK) sm[i] = 0;
  __syncthreads();
  for (int rd = 0; rd < rounds; ++rd) {
    double u[BIN_IPT][2], x[BIN_IPT][2];
    int c[BIN_IPT][2], key[BIN_IPT][4], l0[BIN_IPT][4], l1[BIN_IPT][4], row[BIN_IPT], col[BIN_IPT];
    bin2_keys(k, m, tg, wg, ((int64_t)blockIdx.x * rounds + rd) * BIN_IPT * BIN_BLOCK, u, c, key, l0, l1, row, col,
              x);
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (key[i][q] >= 0) atomicAdd(&ht[key[i][q]], 1);
      if (row[i] >= 0) atomicAdd(&hr[row[i]], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ntiles; i += BIN_BLOCK) {
    const int v = ht[i];
    if (v) atomicAdd(&tile_cnt[i], v);
  }
  for (int i = threadIdx.x; i < nrow; i += BIN_BLOCK) {
    const int v = hr[i];
    if (v) atomicAdd(&row_cnt[i], v);
  }
}

// ONE: a single round per workgroup (rounds == 1), whose keys stay in
// registers from the count to the placement instead of being recomputed
template <class real, bool ONE>
__global__ __launch_bounds__(BIN_BLOCK) void k_bin2_scatter(const double* __restrict__ k, int64_t m, TileGeom tg,
                                                            const WBinGeom* __restrict__ wgp,
                                                            int32_t* __restrict__ tile_cursor,
                                                            int ntiles, int32_t* __restrict__ row_cursor,
                                                            int rounds, Rec<real>* __restrict__ recs,
                                                            RowRec* __restrict__ rowbuf) {
  const WBinGeom wg = *wgp;
  extern __shared__ int32_t sm[];   // ntiles + nrow counters, then LDS_SPARE spare words
  int32_t* bt = sm;
  int32_t* br = sm + ntiles;
  const int nrow = wg.nb[0];
  for (int i = threadIdx.x; i < ntiles + nrow; i += BIN_BLOCK) sm[i] = 0;
  __syncthreads();
  double u[BIN_IPT][2], x[BIN_IPT][2];
  int c[BIN_IPT][2], key[BIN_IPT][4], l0[BIN_IPT][4], l1[BIN_IPT][4], row[BIN_IPT], col[BIN_IPT];
  for (int rd = 0; rd < rounds; ++rd) {
    bin2_keys(k, m, tg, wg, ((int64_t)blockIdx.x * rounds + rd) * BIN_IPT * BIN_BLOCK, u, c, key, l0, l1, row, col,
              x);
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (key[i][q] >= 0) atomicAdd(&bt[key[i][q]], 1);
      if (row[i] >= 0) atomicAdd(&br[row[i]], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ntiles; i += BIN_BLOCK) {
    const int v = bt[i];
    if (v) bt[i] = atomicAdd(&tile_cursor[i], v);
  }
  for (int i = threadIdx.x; i < nrow; i += BIN_BLOCK) {
    const int v = br[i];
    if (v) br[i] = atomicAdd(&row_cursor[i], v);
  }
  __syncthreads();
  for (int rd = 0; rd < rounds; ++rd) {
    const int64_t j0 = ((int64_t)blockIdx.x * rounds + rd) * BIN_IPT * BIN_BLOCK;
    if constexpr (!ONE) bin2_keys(k, m, tg, wg, j0, u, c, key, l0, l1, row, col, x);
    int pos[BIN_IPT][4], rpos[BIN_IPT];
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) pos[i][q] = lds_claim(bt, key[i][q], ntiles + nrow);
      rpos[i] = lds_claim(br, row[i], nrow);
    }
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i) {
      const int64_t j = j0 + (int64_t)i * BIN_BLOCK + threadIdx.x;
      Rec<real> r;
      r.f0 = (real)(u[i][0] - (double)c[i][0]);
      r.f1 = (real)(u[i][1] - (double)c[i][1]);
      r.src = (int32_t)j;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (key[i][q] >= 0) {
          r.c01 = (int32_t)(((uint32_t)l0[i][q] & 0xffffu) | ((uint32_t)l1[i][q] << 16));
          recs[pos[i][q]] = r;
        }
      }
      if (row[i] >= 0) {
        RowRec rr;
        rr.k0 = x[i][0];
        rr.k1 = x[i][1];
        rr.j = (int32_t)j;
        rr.b1 = col[i];
        rowbuf[rpos[i]] = rr;
      }
    }
  }
}

// The same fusion beyond LDS_TILE_KEYS tiles (the 4096^2 raster: 65 536
// tiles): the tile counters stay in global memory and take one atomic per
// group of lanes with the same key (key_group / group_claim), the bin rows
// are counted in LDS as above. Both passes take one group of BIN_IPT *
// BIN_BLOCK samples per workgroup.
// The tile counts of a workgroup are gathered first in a small LDS table
// (open addressing, one insertion per group of lanes with the same key): the
// consecutive samples of a workgroup meet about a hundred tiles, so the table
// turns one global atomic per key group and wavefront into one per tile and
// workgroup. A key that finds no slot within CNT_PROBES probes goes to the
// global counter directly.
constexpr int CNT_SLOTS = 1024;
constexpr int CNT_PROBES = 8;

__global__ __launch_bounds__(BIN_BLOCK) void k_bin2g_count(const double* __restrict__ k, int64_t m, TileGeom tg,
                                                           const WBinGeom* __restrict__ wgp,
                                                           int32_t* __restrict__ tile_cnt,
                                                           int32_t* __restrict__ row_cnt, int rounds) {
  const WBinGeom wg = *wgp;
  __shared__ int32_t hr[WROW_MAX];
  __shared__ int32_t tkey[CNT_SLOTS], tcnt[CNT_SLOTS];
  const int nrow = wg.nb[0];
  for (int i = threadIdx.x; i < nrow; i += BIN_BLOCK) hr[i] = 0;
  for (int i = threadIdx.x; i < CNT_SLOTS; i += BIN_BLOCK) {
    tkey[i] = -1;
    tcnt[i] = 0;
  }
  __syncthreads();
  for (int rd = 0; rd < rounds; ++rd) {
    double u[BIN_IPT][2], x[BIN_IPT][2];
    int c[BIN_IPT][2], key[BIN_IPT][4], l0[BIN_IPT][4], l1[BIN_IPT][4], row[BIN_IPT], col[BIN_IPT];
    bin2_keys(k, m, tg, wg, ((int64_t)blockIdx.x * rounds + rd) * BIN_IPT * BIN_BLOCK, u, c, key, l0, l1, row, col,
              x);
#pragma unroll
    for (int i = 0; i < BIN_IPT; ++i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const KeyGroup kg = key_group(key[i][q], key[i][q] >= 0);
        if (kg.leader == (int)__lane_id()) {
          const int kk = key[i][q];
          int h = (int)(((unsigned)kk * 2654435761u) >> 22);   // 10 bits
          bool placed = false;
          for (int pr = 0; pr < CNT_PROBES && !placed; ++pr, h = (h + 1) & (CNT_SLOTS - 1)) {
            const int old = atomicCAS(&tkey[h], -1, kk);
            if (old == -1 || old == kk) {
              atomicAdd(&tcnt[h], kg.size);
              placed = true;
            }
          }
          if (!placed) atomicAdd(&tile_cnt[kk], kg.size);
        }
      }
      if (row[i] >= 0) atomicAdd(&hr[row[i]], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < CNT_SLOTS; i += BIN_BLOCK) {
    const int kk = tkey[i];
    if (kk >= 0) atomicAdd(&tile_cnt[kk], tcnt[i]);
  }
  for (int i = threadIdx.x; i < nrow; i += BIN_BLOCK) {
    const int v = hr[i];
    if (v) atomicAdd(&row_cnt[i], v);
  }
}

template <class real>
__global__ __launch_bounds__(BIN_BLOCK) void k_bin2g_scatter(const double* __restrict__ k, int64_t m, TileGeom tg,
                                                             const WBinGeom* __restrict__ wgp,
                                                             int32_t* __restrict__ tile_cursor,
                                                             int32_t* __restrict__ row_cursor,
                                                             Rec<real>* __restrict__ recs,
                                                             RowRec* __restrict__ rowbuf) {
  const WBinGeom wg = *wgp;
  __shared__ int32_t br[WROW_MAX + LDS_SPARE];   // row counters, then one spare word per lane
  const int nrow = wg.nb[0];
  for (int i = threadIdx.x; i < nrow; i += BIN_BLOCK) br[i] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * BIN_IPT * BIN_BLOCK;
  double u[BIN_IPT][2], x[BIN_IPT][2];
  int c[BIN_IPT][2], key[BIN_IPT][4], l0[BIN_IPT][4], l1[BIN_IPT][4], row[BIN_IPT], col[BIN_IPT];
  bin2_keys(k, m, tg, wg, j0, u, c, key, l0, l1, row, col, x);
  // tile ranges: every slot's groups claim before any claim is waited for
  KeyGroup kg[BIN_IPT][4];
  int base[BIN_IPT][4];
#pragma unroll
  for (int i = 0; i < BIN_IPT; ++i) {
#pragma unroll
    for (int q = 0; q < 4; ++q) kg[i][q] = key_group(key[i][q], key[i][q] >= 0);
    if (row[i] >= 0) atomicAdd(&br[row[i]], 1);
  }
#pragma unroll
  for (int i = 0; i < BIN_IPT; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) base[i][q] = group_claim(tile_cursor, key[i][q], kg[i][q]);
  __syncthreads();
  {
    // one row range per row seen; a thread's claims are in flight eight at a
    // time (all sixteen took 97 VGPRs, occupancy 4; eight take 85, occupancy
    // 5: 4096^2 binning 0.438 -> 0.425 ms)
    constexpr int PER = WROW_MAX / BIN_BLOCK, HALF = PER / 2;
#pragma unroll
    for (int h = 0; h < PER; h += HALF) {
      int v[HALF], r[HALF];
#pragma unroll
      for (int q = 0; q < HALF; ++q) {
        const int i = threadIdx.x + (h + q) * BIN_BLOCK;
        v[q] = i < nrow ? br[i] : 0;
      }
#pragma unroll
      for (int q = 0; q < HALF; ++q)
        r[q] = v[q] ? atomicAdd(&row_cursor[threadIdx.x + (h + q) * BIN_BLOCK], v[q]) : 0;
#pragma unroll
      for (int q = 0; q < HALF; ++q)
        if (v[q]) br[threadIdx.x + (h + q) * BIN_BLOCK] = r[q];
    }
  }
  __syncthreads();
  int rpos[BIN_IPT];
#pragma unroll
  for (int i = 0; i < BIN_IPT; ++i) rpos[i] = lds_claim(br, row[i], nrow);
#pragma unroll
  for (int i = 0; i < BIN_IPT; ++i) {
    const int64_t j = j0 + (int64_t)i * BIN_BLOCK + threadIdx.x;
    Rec<real> rc;
    rc.f0 = (real)(u[i][0] - (double)c[i][0]);
    rc.f1 = (real)(u[i][1] - (double)c[i][1]);
    rc.src = (int32_t)j;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int pos = group_slot(base[i][q], kg[i][q]);
      if (key[i][q] >= 0) {
        rc.c01 = (int32_t)(((uint32_t)l0[i][q] & 0xffffu) | ((uint32_t)l1[i][q] << 16));
        recs[pos] = rc;
      }
    }
    if (row[i] >= 0) {
      RowRec rr;
      rr.k0 = x[i][0];
      rr.k1 = x[i][1];
      rr.j = (int32_t)j;
      rr.b1 = col[i];
      rowbuf[rpos[i]] = rr;
    }
  }
}

// record-order weights, record count read on the device
template <class real>
__global__ __launch_bounds__(BIN_BLOCK) void k_refill_alpha_dev(const Rec<real>* __restrict__ recs,
                                                                const int32_t* __restrict__ nrec_dev,
                                                                const double* __restrict__ alpha,
                                                                real* __restrict__ alpha_s) {
  const int64_t nrec = *nrec_dev;
  for (int64_t r = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x; r < nrec; r += (int64_t)gridDim.x * BIN_BLOCK)
    alpha_s[r] = (real)alpha[recs[r].src];
}

template <class real>
__global__ __launch_bounds__(BIN_BLOCK) void k_refill_alpha(const Rec<real>* __restrict__ recs, int64_t nrec,
                                                            const double* __restrict__ alpha,
                                                            real* __restrict__ alpha_s) {
  int64_t r = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x;
  if (r < nrec) alpha_s[r] = (real)alpha[recs[r].src];
}

static TileGeom tile_geom(ftcg_plan p) {
  TileGeom g;
  g.sigma = p->sigma;
  g.half_g = (double)(p->G / 2);
  g.G = p->G;
  g.T = p->tile;
  g.nt = (int)p->nt;
  g.W = p->W;
  g.tshift = -1;
  for (int s = 0; s < 31; ++s)
    if ((1 << s) == g.T) g.tshift = s;
  g.inv_g = (g.G > 0 && (g.G & (g.G - 1)) == 0) ? 1.0 / (double)g.G : 0.0;
  return g;
}

// tile binning; the tile counters were zeroed by the input check
// counting and scan of the tile binning (cnt then holds the cursors)
static void bin_count_t(ftcg_plan p, const double* k) {
  const TileGeom g = tile_geom(p);
  hipStream_t s = p->stream;
  const int64_t m = p->m;
  int32_t* cnt = p->tile_cnt.as<int32_t>();
  int32_t* off = p->tile_off.as<int32_t>();
  const int nkeys = (int)p->ntiles;
  if (nkeys <= LDS_TILE_KEYS) {
    const int rounds = bin_rounds(nkeys);
    const int64_t per = (int64_t)rounds * BIN_IPT * BIN_BLOCK;
    const unsigned nb = (unsigned)((m + per - 1) / per);
    const size_t lds = sizeof(int32_t) * (nkeys + LDS_SPARE);
    if (p->dim == 1)
      hipLaunchKernelGGL(k_tile_count_lds<1>, dim3(nb), dim3(BIN_BLOCK), lds, s, k, m, g, cnt, nkeys, rounds);
    else
      hipLaunchKernelGGL(k_tile_count_lds<2>, dim3(nb), dim3(BIN_BLOCK), lds, s, k, m, g, cnt, nkeys, rounds);
  } else {
    const unsigned nb = (unsigned)((m + BIN_BLOCK - 1) / BIN_BLOCK);
    if (p->dim == 1)
      hipLaunchKernelGGL(k_tile_count<1>, dim3(nb), dim3(BIN_BLOCK), 0, s, k, m, g, cnt);
    else
      hipLaunchKernelGGL(k_tile_count<2>, dim3(nb), dim3(BIN_BLOCK), 0, s, k, m, g, cnt);
  }
  exclusive_scan_i32(cnt, off, p->ntiles, p->tile_scan_tmp.as<int32_t>(), s, cnt);  // cnt becomes the cursor
  FTCG_HIP(hipGetLastError());
}

// scatter of the tile records; with weights (p->have_weights) they go into
// record order as the records are written, else every record gets weight 1
template <class real>
static void bin_scatter_t(ftcg_plan p, const double* k) {
  const TileGeom g = tile_geom(p);
  hipStream_t s = p->stream;
  const int64_t m = p->m;
  int32_t* cnt = p->tile_cnt.as<int32_t>();
  const double* alpha = p->have_weights ? p->alpha.as<double>() : nullptr;
  const int nkeys = (int)p->ntiles;
  if (nkeys <= LDS_TILE_KEYS) {
    const int rounds = bin_rounds(nkeys);
    const int64_t per = (int64_t)rounds * BIN_IPT * BIN_BLOCK;
    const unsigned nb = (unsigned)((m + per - 1) / per);
    const size_t lds = sizeof(int32_t) * (nkeys + LDS_SPARE);
    if (p->dim == 1)
      hipLaunchKernelGGL((k_tile_scatter_lds<1, real>), dim3(nb), dim3(BIN_BLOCK), lds, s, k, m, g, alpha, cnt,
                         nkeys, rounds, p->recs.as<Rec<real>>(), p->alpha_s.as<real>());
    else
      hipLaunchKernelGGL((k_tile_scatter_lds<2, real>), dim3(nb), dim3(BIN_BLOCK), lds, s, k, m, g, alpha, cnt,
                         nkeys, rounds, p->recs.as<Rec<real>>(), p->alpha_s.as<real>());
  } else {
    const unsigned nb = (unsigned)((m + BIN_BLOCK - 1) / BIN_BLOCK);
    if (p->dim == 1)
      hipLaunchKernelGGL((k_tile_scatter<1, real>), dim3(nb), dim3(BIN_BLOCK), 0, s, k, m, g, alpha, cnt,
                         p->recs.as<Rec<real>>(), p->alpha_s.as<real>());
    else
      hipLaunchKernelGGL((k_tile_scatter<2, real>), dim3(nb), dim3(BIN_BLOCK), 0, s, k, m, g, alpha, cnt,
                         p->recs.as<Rec<real>>(), p->alpha_s.as<real>());
  }
  FTCG_HIP(hipGetLastError());
}

bool tile_keys_in_lds(ftcg_plan p) { return p->ntiles <= LDS_TILE_KEYS; }

void bin_count_k(ftcg_plan p, const double* k) { bin_count_t(p, k); }

void bin_scatter_k(ftcg_plan p, const double* k) {
  if (p->dtype == FTCG_F64)
    bin_scatter_t<double>(p, k);
  else
    bin_scatter_t<float>(p, k);
}


// the bin-row geometry comes from the input check in device memory (these
// passes are enqueued before the host has read it): LDS is sized for
// WROW_MAX rows, the kernels clear and flush the geometry's own row count,
// and the row scan covers all WROW_MAX counters (rows past the count stay
// empty)
template <class real>
static void bin_points_fused_t(ftcg_plan p, const double* k) {
  const TileGeom tg = tile_geom(p);
  const WBinGeom* wg = &p->geo.as<CheckOut>()->g;
  hipStream_t s = p->stream;
  const int64_t m = p->m;
  int32_t* tcnt = p->tile_cnt.as<int32_t>();   // zeroed by the input check
  int32_t* rcnt = p->wb_cnt.as<int32_t>();     // zeroed by the input check
  const int rounds = bin_rounds(p->ntiles);
  const int64_t per = (int64_t)rounds * BIN_IPT * BIN_BLOCK;
  const unsigned nb = (unsigned)((m + per - 1) / per);
  const size_t lds = sizeof(int32_t) * (size_t)(p->ntiles + WROW_MAX + LDS_SPARE);   // <= 32.25 KiB
  hipLaunchKernelGGL(k_bin2_count<real>, dim3(nb), dim3(BIN_BLOCK), lds, s, k, m, tg, wg, tcnt, (int)p->ntiles,
                     rcnt, rounds);
  exclusive_scan_pair_i32(tcnt, p->tile_off.as<int32_t>(), p->ntiles, tcnt, rcnt, p->wb_rowoff.as<int32_t>(),
                          WROW_MAX, rcnt, s);
  if (rounds == 1)
    hipLaunchKernelGGL((k_bin2_scatter<real, true>), dim3(nb), dim3(BIN_BLOCK), lds, s, k, m, tg, wg, tcnt,
                       (int)p->ntiles, rcnt, rounds, p->recs.as<Rec<real>>(), p->wb_rowbuf.as<RowRec>());
  else
    hipLaunchKernelGGL((k_bin2_scatter<real, false>), dim3(nb), dim3(BIN_BLOCK), lds, s, k, m, tg, wg, tcnt,
                       (int)p->ntiles, rcnt, rounds, p->recs.as<Rec<real>>(), p->wb_rowbuf.as<RowRec>());
  FTCG_HIP(hipGetLastError());
}

// more tiles than LDS holds: global tile counters, LDS bin rows
template <class real>
static void bin_points_fused_g_t(ftcg_plan p, const double* k) {
  const TileGeom tg = tile_geom(p);
  const WBinGeom* wg = &p->geo.as<CheckOut>()->g;
  hipStream_t s = p->stream;
  const int64_t m = p->m;
  int32_t* tcnt = p->tile_cnt.as<int32_t>();   // zeroed by the input check
  int32_t* rcnt = p->wb_cnt.as<int32_t>();     // zeroed by the input check
  const int64_t per = (int64_t)BIN_IPT * BIN_BLOCK;
  // one round per workgroup (4096^2 raster, binning step with 1 / 2 / 4 / 8
  // count rounds: 0.440 / 0.471 / 0.492 / 0.487 ms: the rounds' loads and
  // key votes run one after another)
  const unsigned nbc = (unsigned)((m + per - 1) / per);
  hipLaunchKernelGGL(k_bin2g_count, dim3(nbc), dim3(BIN_BLOCK), 0, s, k, m, tg, wg, tcnt, rcnt, 1);
  exclusive_scan_i32(tcnt, p->tile_off.as<int32_t>(), p->ntiles, p->tile_scan_tmp.as<int32_t>(), s, tcnt);
  exclusive_scan_i32(rcnt, p->wb_rowoff.as<int32_t>(), WROW_MAX, p->scan_tmp.as<int32_t>(), s, rcnt);
  const unsigned nbs = (unsigned)((m + per - 1) / per);
  hipLaunchKernelGGL(k_bin2g_scatter<real>, dim3(nbs), dim3(BIN_BLOCK), 0, s, k, m, tg, wg, tcnt, rcnt,
                     p->recs.as<Rec<real>>(), p->wb_rowbuf.as<RowRec>());
  FTCG_HIP(hipGetLastError());
}

void bin_points_fused(ftcg_plan p, const double* k) {
  const bool lds = tile_keys_in_lds(p);
  if (p->dtype == FTCG_F64) {
    if (lds)
      bin_points_fused_t<double>(p, k);
    else
      bin_points_fused_g_t<double>(p, k);
  } else {
    if (lds)
      bin_points_fused_t<float>(p, k);
    else
      bin_points_fused_g_t<float>(p, k);
  }
}

void refill_alpha_dev(ftcg_plan p) {
  int64_t nb = ((p->m << p->dim) + BIN_BLOCK - 1) / BIN_BLOCK;
  if (nb > 2048) nb = 2048;
  const int32_t* nrec = p->tile_off.as<int32_t>() + p->ntiles;
  if (p->dtype == FTCG_F64)
    hipLaunchKernelGGL(k_refill_alpha_dev<double>, dim3((unsigned)nb), dim3(BIN_BLOCK), 0, p->stream,
                       p->recs.as<Rec<double>>(), nrec, p->alpha.as<double>(), p->alpha_s.as<double>());
  else
    hipLaunchKernelGGL(k_refill_alpha_dev<float>, dim3((unsigned)nb), dim3(BIN_BLOCK), 0, p->stream,
                       p->recs.as<Rec<float>>(), nrec, p->alpha.as<double>(), p->alpha_s.as<float>());
  FTCG_HIP(hipGetLastError());
}

void bin_points_k(ftcg_plan p, const double* k) {
  bin_count_k(p, k);
  bin_scatter_k(p, k);
}

void refill_alpha(ftcg_plan p) {
  const int64_t nrec = plan_nrec(p);
  const unsigned nb = (unsigned)((nrec + BIN_BLOCK - 1) / BIN_BLOCK);
  if (nrec == 0) return;
  if (p->dtype == FTCG_F64)
    hipLaunchKernelGGL(k_refill_alpha<double>, dim3(nb), dim3(BIN_BLOCK), 0, p->stream,
                       p->recs.as<Rec<double>>(), nrec, p->alpha.as<double>(), p->alpha_s.as<double>());
  else
    hipLaunchKernelGGL(k_refill_alpha<float>, dim3(nb), dim3(BIN_BLOCK), 0, p->stream,
                       p->recs.as<Rec<float>>(), nrec, p->alpha.as<double>(), p->alpha_s.as<float>());
  FTCG_HIP(hipGetLastError());
}

__global__ void k_fill_ones(double* a, int64_t m) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) a[j] = 1.0;
}

void fill_ones(double* a, int64_t m, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_fill_ones, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, m);
  FTCG_HIP(hipGetLastError());
}

}  // namespace ftcg
