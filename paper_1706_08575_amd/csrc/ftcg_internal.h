// Internal declarations of libftcg: plan state, record layout, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ftcg.h"

namespace ftcg {

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------

struct HipError {
  hipError_t err;
  const char* what;
};

#define FTCG_HIP(call)                                 \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) throw ::ftcg::HipError{e_, #call}; \
  } while (0)

struct StatusError {
  ftcg_status status;
};

// ---------------------------------------------------------------------------
// device buffer owned by a plan (grow-only)
// ---------------------------------------------------------------------------

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void ensure(size_t need) {
    if (need <= bytes) return;
    // work still queued may use the old buffer (a plan enqueues some of
    // its passes before it waits for anything)
    if (p) (void)hipDeviceSynchronize();
    release();
    if (hipMalloc(&p, need) != hipSuccess) {
      p = nullptr;
      bytes = 0;
      (void)hipGetLastError();
      throw StatusError{FTCG_ENOMEM};
    }
    bytes = need;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// spread record: one (sample, tile) pair; a sample whose 2W x 2W footprint
// crosses tile edges gets one record per tile it touches.
//   c0, c1 : integer grid cell floor(u) relative to the tile origin (int16 each,
//            packed c0 | c1 << 16), can be negative or >= tile for halo records;
//   f0, f1 : u - floor(u) in [0, 1) per axis (the fractional position);
//   src    : index of the sample in caller order.
// The footprint of a record covers local cells c - W + 1 .. c + W per axis.
// ---------------------------------------------------------------------------

template <class real>
struct Rec {
  real f0, f1;
  int32_t c01;
  int32_t src;
};

// neighbour bins of the frame-weight sum (square bins of edge h in k units)
struct WBinGeom {
  double kmin[2];
  double h;          // bin edge (k units)
  int nb[2];         // bins per axis
  int span;          // neighbour bins each side covering the box of radius R
  double R;
};

// bin rows (2D) at most: the row counters and the row scan have this size
constexpr int WROW_MAX = 4096;

// pi, and the self term pi^DIM of the frame-weight sums (alpha = pi^DIM / sum)
constexpr double WPI = 3.141592653589793238462643383279502884;
template <int DIM>
constexpr double wscale() { return DIM == 1 ? WPI * WPI : WPI * WPI * WPI * WPI; }

// Determinism of the frame-weight sums. Every value that an atomic adds to a
// sum is rounded to a multiple of 2^-36 (one fused multiply-add against
// 1.5 * 2^16, whose neighbours are 2^-36 apart, then the exact subtraction of
// that constant): each term (pi^DIM T_in)^2 <= pi^4 in most kernels, a lane's
// partial sum (added in a fixed order: bins are ordered by caller index) in
// the symmetric 2D kernel, and the self term. Sums of such multiples are
// exact while they stay below 2^17 (sum T^2 below about 1300 in 2D and 13000
// in 1D, far above any raster's density), so the order in which lanes, LDS
// atomics and global atomics add them does not change a bit: the weights are
// bitwise reproducible although the kernels add with atomics. Each rounding
// moves a value by at most 2^-37 absolutely, about 1e-13 of the sum, which
// always holds the self term pi^DIM.
constexpr double WQ_MAGIC = 98304.0;   // 1.5 * 2^16
__device__ inline double wq_square(double q) { return fma(q, q, WQ_MAGIC) - WQ_MAGIC; }
template <int DIM>
constexpr double wself() { return (wscale<DIM>() + WQ_MAGIC) - WQ_MAGIC; }

// the input check reduced on the device: bounding box, the neighbour-bin
// geometry derived from it, and whether the points are rejected
struct CheckOut {
  WBinGeom g;
  double kmin[2], kmax[2];
  int bad;   // a coordinate is non-finite or beyond 2^40 in magnitude
  int seq;   // number of the set_points call it answers (checked by the host)
};

// a sample in bin order: coordinates, then sin(pi k_a), cos(pi k_a) per axis
template <int DIM>
struct WSample {
  double k[DIM];
  double sc[DIM][2];
};

// tile accumulation of float32 plans
enum Accum { ACCUM_FIXED = 0, ACCUM_F64 = 1 };

// One fixed-point tap of the float32 spreading kernels: the scaled
// components rounded to the nearest integer (v_cvt_rpi_i32_f32 computes
// floor(x + 1/2); truncation toward zero would bias every tap by half a
// quantum against its sign, which adds up over the thousands of taps a cell
// of a dense tile receives) and packed as im * 2^32 + re in two's
// complement, so that one 64-bit integer add accumulates both exactly.
__device__ inline unsigned long long fx_pack(float pr, float pi) {
  int ir, ii;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(ir) : "v"(pr));
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(ii) : "v"(pi));
  const unsigned hi = (unsigned)ii + (unsigned)(ir >> 31);
  return ((unsigned long long)hi << 32) | (unsigned)ir;
}

enum Step {
  STEP_BIN = 0,      // input check + tile binning of spread records
  STEP_WEIGHTS = 1,  // frame-weight sum kernel
  STEP_SPREAD = 2,
  STEP_FFT1 = 3,
  STEP_FFT2 = 4,     // second FFT pass + deapodize + crop (the only pass in 1D)
  STEP_WBIN = 5,     // neighbour binning for the weight sum
  STEP_LEARNED = 6,  // fused 16-NN + MLP inference
  STEP_AUDIT = 7,    // audit of learned weights against plain ones
  STEP_WFINISH = 8,  // weights from the sums of the symmetric kernel (and their preset)
  STEP_BAND_GRAM = 9,    // banded C: the band of T^2
  STEP_BAND_SOLVE = 10,  // banded C: per-column normal equations
  STEP_BAND_APPLY = 11,  // c = C fhat ahead of the spread
  STEP_FWD_FFT = 12,     // forward transform: deapodize, pad, forward FFT passes
  STEP_FWD_INTERP = 13,  // forward transform: interpolation at the raster
  STEP_DENSITY = 14,     // iterative density compensation (all iterations)
  STEP_FRAME = 15,       // dense frame approximation (matrix, QR, solve, image)
  N_STEPS = 16       // entries of the timing arrays
};

// per-step HIP event pairs recorded on the plan's stream; resolved (and
// returned to the pool) when the caller asks for the sums
struct Timing {
  bool enabled = false;
  struct Pair {
    int step;
    hipEvent_t a, b;
  };
  std::vector<Pair> pending;
  std::vector<hipEvent_t> pool;
  int open_step = -1;
  hipEvent_t open_ev = nullptr;
};

// ---------------------------------------------------------------------------
// Lanes of a wavefront grouped by equal key (rasters arrive in acquisition
// order, so neighbouring lanes usually bin to the same tile): for each lane
// the first lane holding its key (the leader) and its rank among the lanes
// holding it; a leader also gets the group's size. Register-only, one ballot
// per distinct key. Lanes with valid == false take part in the vote and form
// no group (leader -1).
// ---------------------------------------------------------------------------
struct KeyGroup {
  int leader, rank, size;
};

__device__ inline KeyGroup key_group(int key, bool valid) {
  unsigned long long todo = __ballot(valid);
  const int lane = __lane_id();
  KeyGroup g{-1, 0, 0};
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lkey = __builtin_amdgcn_readlane(key, leader);
    const unsigned long long match = __ballot(valid && key == lkey) & todo;
    if ((match >> lane) & 1ull) {
      g.leader = leader;
      g.rank = __popcll(match & ((1ull << lane) - 1ull));
      if (lane == leader) g.size = __popcll(match);
    }
    todo &= ~match;
  }
  return g;
}

// The group's leader adds the group's size to counters[key]; the atomics of
// all groups of the wavefront go out as one instruction, so a wavefront waits
// for one round trip however many distinct keys it holds.
__device__ inline int group_claim(int32_t* counters, int key, const KeyGroup& g) {
  int base = 0;
  if (g.leader == (int)__lane_id()) base = atomicAdd(&counters[key], g.size);
  return base;
}

// this lane's slot from its leader's claim (every lane of the wavefront
// executes it); -1 for lanes in no group
__device__ inline int group_slot(int base, const KeyGroup& g) {
  const int b = __shfl(base, g.leader < 0 ? 0 : g.leader);
  return g.leader < 0 ? -1 : b + g.rank;
}

// XCD-aware block order. Workgroups are dealt to the 8 XCDs round-robin
// (block b to XCD b % 8), and each XCD has its own L2. This returns the
// logical block for hardware block b so that XCD x works through chunks x,
// x + 8, x + 16, ... of C consecutive logical blocks, C = nblocks / 64 clamped
// to [1, 64]: blocks that share data run on one L2, and every XCD still sees
// every part of the range, which keeps the XCDs evenly loaded when the cost of
// a block varies along it. Blocks past the last whole group of 8 chunks keep
// the plain order.
// The same with a chunk length chosen by the caller (C >= 1).
__device__ inline int64_t xcd_block_chunk(int64_t b, int64_t nblocks, int64_t C) {
  const int64_t full = nblocks / (8 * C) * (8 * C);
  if (b >= full) return b;
  const int64_t x = b & 7, i = b >> 3;
  return ((i / C) * 8 + x) * C + (i % C);
}

__device__ inline int64_t xcd_block(int64_t b, int64_t nblocks) {
  int64_t C = nblocks >> 6;
  C = C < 1 ? 1 : (C > 64 ? 64 : C);
  return xcd_block_chunk(b, nblocks, C);
}

}  // namespace ftcg

struct ftcg_plan_s {
  int dim = 0;
  int64_t n = 0;      // image edge (same on every axis)
  int W = 6;
  double sigma = 2.0;
  ftcg_dtype dtype = FTCG_F32;
  ftcg_wmode wmode = FTCG_W_PLAIN;
  double R = 8.0;
  hipStream_t stream = nullptr;

  int64_t G = 0;       // grid edge
  double beta = 0.0;   // kernel exp(-beta s^2)
  int tile_req = 0;    // requested tile edge (0 = automatic)
  bool spread_segments = true;   // segmented float32 spread on large grids (ftcg_plan_set_spread_layout)
  int w_samples = 0;   // frame-weight kernel: samples per lane (0 = automatic)
  int w_lanes = 0;     // frame-weight kernel (2D): lanes per sample group (0 = automatic)
  int lds_copies = 1;
  int accum = 0;       // ftcg::Accum for float32 plans (float64 plans always use ACCUM_F64)

  // geometry state
  int tile = 64;
  int64_t nt = 0;       // tiles per axis
  int64_t ntiles = 0;
  int64_t m = 0;
  int64_t nrec = 0;
  bool have_points = false;
  bool have_weights = false;
  int used_fallback = 0;

  ftcg::DevBuf alpha;        // m float64, caller order
  ftcg::DevBuf recs;         // nrec records
  ftcg::DevBuf alpha_s;      // nrec weights in record order (dtype real)
  ftcg::DevBuf tile_cnt;     // ntiles + 1 int32 (count, then cursor)
  ftcg::DevBuf tile_off;     // ntiles + 1 int32
  ftcg::DevBuf scan_tmp;     // scan scratch
  ftcg::DevBuf tile_scan_tmp;  // scan scratch of the tile binning (in flight while the host reads the check)
  ftcg::DevBuf flags;        // small device scratch: [6] audit estimate

  // weight binning
  ftcg::DevBuf wb_cnt, wb_off;  // 2D: wb_cnt holds the bin-row counters (WROW_CNT_ZERO entries)
  ftcg::DevBuf wb_rowoff, wb_rowbuf;  // 2D: bin-row offsets, sample indices grouped by row
  ftcg::DevBuf ws_k;         // sorted samples: k, sin(pi k), cos(pi k) (3*dim doubles each)
  ftcg::DevBuf ws_idx;       // sorted original index
  ftcg::DevBuf wb_of;        // weight-bin id per sample (caller order)
  ftcg::DevBuf ws_inv;       // sorted position of every sample (caller order)
  ftcg::DevBuf ws_sum;       // 2D: per-sample weight sums in bin order (symmetric form)
  bool ws_sum_fresh = false; // ws_sum holds the self terms only (preset by the bin sort)
  // set by the fused binning: the finish of the symmetric weight sum also
  // writes the record-order weights (through ws_inv) and then clears it
  bool finish_recs = false;
  // the symmetric sum's finish is pending (fused-binning grids): the
  // fixed-point spread forms each record's weight from ws_sum itself, and
  // finish_deferred_weights writes alpha and the records' weights when
  // anything else needs them
  bool weights_deferred = false;
  ftcg::WBinGeom wgeom{};
  bool have_wbins = false;
  bool weights_only = false;  // internal plans that only compute weights (no tile binning)

  // banded coefficient matrix C (FTCG_W_BAND)
  int band_r = 1;             // band half-width r: 2r - 1 entries per column
  int band_bad = 0;           // columns whose normal equations broke down (last set_points)
  ftcg::DevBuf band_P;        // m x (2r-1): pi^(2 dim) (T^2)_{a, a+e}
  ftcg::DevBuf band_col;      // m x (2r-1): C[n - r + 1 + p, n] (column form)
  ftcg::DevBuf band_row;      // m x (2r-1): C[i, i + e - r + 1] (row form, for the apply)
  ftcg::DevBuf band_c;        // m complex: C fhat of the last execute

  // iterative density compensation (FTCG_W_DENSITY)
  int den_iters = 20;
  ftcg::DevBuf den_val;       // m complex: the weights as spread values
  ftcg::DevBuf den_d;         // m complex: Omega^T Omega w

  // dense frame approximation (ftcg_frame_approx)
  ftcg::DevBuf fa_gl, fa_G, fa_A, fa_diag, fa_beta, fa_tw, fa_tmp;

  // learned weights
  struct ftcg_mlp_s* mlp = nullptr;
  double audit_threshold = 1e-4;
  int64_t audit_samples = 4096;
  double audit_estimate = -1.0;
  ftcg::DevBuf audit_buf;    // audit indices / plain weights / scratch

  // execute workspace
  ftcg::DevBuf grid;         // G^dim complex
  ftcg::DevBuf twiddle;      // two-level tables of e^{2 pi i j / G} (plan precision)
  ftcg::DevBuf fft_tmp;      // n x G complex (2D)
  ftcg::DevBuf deapod;       // n float64
  ftcg::DevBuf tile_order;   // ntiles int32 (heavy tiles first)

  ftcg::Timing timing;
  double* host_flags = nullptr;  // pinned host mirror of flags (FLAGS_BYTES)
  // the input check: per-workgroup partials, the reduced result on the
  // device, its pinned coherent host copy (written by the same kernel), and
  // the event after it, which is all the host waits for
  ftcg::DevBuf check_part;
  ftcg::DevBuf geo;
  ftcg::CheckOut* host_geo = nullptr;
  hipEvent_t ev_check = nullptr;
  int check_seq = 0;
  // between the two parts of set_points: the call's check number and the
  // binning decisions taken before the host has read the check
  struct PendingPoints {
    int seq = 0;
    bool tiles = false, early_scatter = false, fused = false, band = false;
  } pending;
};

namespace ftcg {

// launchers (defined in the .hip files); all enqueue on plan->stream
constexpr size_t FLAGS_BYTES = 128;       // device flags / pinned host mirror
constexpr int64_t WROW_CNT_ZERO = 4100;   // bin-row counters cleared by the input check (>= WROW_MAX + 1)
constexpr int CHECK_PARTS = 1024;         // input-check workgroups at most
// returns the number of partial records (5 words each) written to part
int launch_check_points(ftcg_plan p, const double* k, int64_t m, unsigned long long* part, int32_t* zero_a,
                        int64_t zero_na, int32_t* zero_b, int64_t zero_nb);
// reduces the partials into p->geo and p->host_geo (one workgroup)
void launch_check_reduce(ftcg_plan p, const unsigned long long* part, int nparts, int seq);
void bin_points_k(ftcg_plan p, const double* k);   // fills recs, alpha_s, tile_off
void bin_count_k(ftcg_plan p, const double* k);    // its counting + scan (tile_off, cursors)
void bin_scatter_k(ftcg_plan p, const double* k);  // its scatter (recs, alpha_s)
bool tile_keys_in_lds(ftcg_plan p);                 // the tile counters fit one workgroup's LDS
void refill_alpha(ftcg_plan p);                     // alpha_s[r] = alpha[recs[r].src]
void refill_alpha_dev(ftcg_plan p);  // the same, record count read on the device (no host sync)
// 2D, <= LDS_TILE_KEYS tiles: tile records and weight-bin rows from one
// counting pass, one paired scan and one scatter pass (geometry read from
// p->geo on the device)
void bin_points_fused(ftcg_plan p, const double* k);
void wrow_bin(ftcg_plan p, const double* k, int nrows);   // 2D bin rows, geometry from p->geo
void setup_weight_bins(ftcg_plan p);                 // buffers for the geometry p->wgeom
void sort_weight_rows(ftcg_plan p);                  // 2D bins from the rows (+ sin/cos)
void build_weight_bins_1d(ftcg_plan p, const double* k);   // 1D sorted neighbour bins
void run_plain_weights(ftcg_plan p);                // alpha (caller order) from the bins
void finish_deferred_weights(ftcg_plan p);          // no-op unless p->weights_deferred
// ftcg_set_points in two parts (a batch enqueues every item's first part
// before the host waits for the first input check); throw on errors
void set_points_begin(ftcg_plan p, int64_t m, const double* k_dev);
void set_points_end(ftcg_plan p, const double* k_dev);
// plain weights of the samples idx[0..n) (caller indices) into out[0..n)
void plain_weights_at(ftcg_plan p, const double* k, const int32_t* idx, int64_t n, double* out);
void fill_ones(double* a, int64_t m, hipStream_t s);
void run_band_weights(ftcg_plan p);                 // banded C from the neighbour bins (FTCG_W_BAND)
void band_apply(ftcg_plan p, const void* fhat);     // p->band_c = C fhat
// columns of n positions (column r at in[p in_stride + r]) -> zero-padded
// forward DFTs of length G, centred signs, one contiguous output row each
void fft_cols_forward(bool f64, const void* in, int64_t in_stride, void* out, int64_t out_row_stride, int64_t G,
                      int64_t n, int cols, const double* dq, const double* drow, const void* tw, hipStream_t s);
void forward_transform(ftcg_plan p, const void* image, void* fhat);   // type-2 transform at the plan's raster
void interpolate_grid(ftcg_plan p, void* out);      // out_j = taps of sample j applied to p->grid
void run_density_weights(ftcg_plan p);              // iterative density compensation into p->alpha
// dense frame approximation of the raster k (m samples) into image (float64 plans)
void frame_approx(ftcg_plan p, int64_t m, const double* k, const void* fhat, void* image);
void spread(ftcg_plan p, const void* fhat, void* grid);
void grid_to_image(ftcg_plan p, const void* grid, void* image);
void compute_deapod(ftcg_plan p);
void compute_deapod_raw(double* d, int64_t n, double sigma, double beta, hipStream_t s);
// the transform of grid_to_image with explicit sizes, tables and intermediate
void grid_to_image_raw(int dim, int64_t n, int64_t G, bool f64, hipStream_t stream, const void* tw,
                       const double* deapod, void* tmp, const void* grid, void* image);
// two-level twiddle tables of the L-th roots of unity (float2, or double2 when f64)
int64_t twiddle_entries(int64_t L);
void compute_twiddles(void* tw, int64_t L, bool f64, hipStream_t s);
int64_t plan_nrec(ftcg_plan p);  // records of the last set_points (one host sync)
// two scans of up to 131072 entries each in one launch
void exclusive_scan_pair_i32(const int32_t* in0, int32_t* out0, int64_t n0, int32_t* cursor0, const int32_t* in1,
                             int32_t* out1, int64_t n1, int32_t* cursor1, hipStream_t s);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s,
                        int32_t* cursor = nullptr);
size_t scan_tmp_bytes(int64_t n);

void timing_begin(ftcg_plan p, int step);
void timing_end(ftcg_plan p, int step);

}  // namespace ftcg
