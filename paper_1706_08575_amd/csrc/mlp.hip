// Learned frame weights: 16-nearest-neighbour geometry features, a 3-layer MLP
// (32 -> 64 -> 64 -> 1, SiLU) predicting log(alpha / base), its training
// (forward, backward, Adam) and the audit against the plain float64 weights.
//
// Definitions (shared with the float64 reference used by the tests):
//   candidates of sample j: samples i != j with ||k_i - k_j||_inf <= R;
//   ranking: d = k_i - k_j in float64, rounded to float32 per axis,
//            d2 = dx*dx + dy*dy with float32 products and sum (no fma),
//            ties by the smaller caller index; the 16 smallest, nearest first;
//   feature: (dx_1, dy_1, ..., dx_16, dy_16) in float32, missing = (R, R);
//   base   : 1 / (1 + sum over the 16 of sinc^2(dx) sinc^2(dy)) in float64;
//   alpha_hat = base * exp(y), y the MLP output.
//
// Inference runs on the matrix cores: every wavefront transforms blocks of 16
// samples with v_mfma_f32_16x16x16_f16 (half inputs and weights, float32
// accumulation). The product is formed transposed, Z^T = W^T X^T, so that the
// accumulator layout of one layer (lane l holds neurons 4(l/16)+r of sample
// l%16) is exactly the B-operand layout the next layer needs: activations
// never leave registers between layers.
//
// Training runs on the vector ALUs in float32: one workgroup takes 64 samples,
// keeps activations in LDS, and writes its partial gradient; a second kernel
// sums the partials in a fixed order and applies Adam to the float32 master
// weights, refreshing their half copy.
#include "ftcg_internal.h"
#include "mlp_internal.h"

namespace ftcg {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int KNN = 16;
constexpr int NF = 2 * KNN;   // 32 features
constexpr int HW = 64;        // hidden width

__device__ inline float silu_f(float z) { return z / (1.f + __expf(-z)); }
__device__ inline float silu_grad_f(float z) {
  const float s = 1.f / (1.f + __expf(-z));
  return s * (1.f + z * (1.f - s));
}
__device__ inline float round_h(float x) { return (float)(_Float16)x; }

// ---------------------------------------------------------------------------
// 16-nearest-neighbour search over the neighbour bins
// ---------------------------------------------------------------------------

__device__ inline int wbin_clamp(double x, double kmin, double h, int nb) {
  int v = (int)floor((x - kmin) / h);
  return v < 0 ? 0 : (v >= nb ? nb - 1 : v);
}

__device__ inline void knn_visit(double kx0, double kx1, int oi, const double* x, int jself, double R,
                                 unsigned long long (&key)[KNN]);

__device__ inline void knn_visit_bin(const WSample<2>* __restrict__ ss, const int32_t* __restrict__ sidx, int beg,
                                     int end, const double* x, int jself, double R,
                                     unsigned long long (&key)[KNN]) {
  for (int i = beg; i < end; ++i) knn_visit(ss[i].k[0], ss[i].k[1], sidx[i], x, jself, R, key);
}

// visits one candidate (caller index oi, coordinates kx) for sample (x, jself)
__device__ inline void knn_visit(double kx0, double kx1, int oi, const double* x, int jself, double R,
                                 unsigned long long (&key)[KNN]) {
  const double dx = kx0 - x[0];
  const double dy = kx1 - x[1];
  if (oi == jself || fabs(dx) > R || fabs(dy) > R) return;
  const float fx = (float)dx, fy = (float)dy;
  const float d2 = __fadd_rn(__fmul_rn(fx, fx), __fmul_rn(fy, fy));
  const unsigned long long kc = ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)oi;
  if (kc < key[KNN - 1]) {
    // sorted insertion, branch free: walk down using the old neighbours
#pragma unroll
    for (int q = KNN - 1; q > 0; --q) {
      const unsigned long long lo = key[q - 1];
      key[q] = (kc < lo) ? lo : (kc < key[q] ? kc : key[q]);
    }
    key[0] = kc < key[0] ? kc : key[0];
  }
}

// after the rings 0 .. r around bin (b0, b1): true when every unvisited
// sample lies at least `reach` (the distance from x to the edge of the
// (2r+1)^2 block, sides clipped at the bin grid's edge excluded) away and the
// 16th key is strictly nearer than that (with a margin for float rounding)
__device__ inline bool knn_done(const unsigned long long (&key)[KNN], const WBinGeom& g, const double* x, int b0,
                                int b1, int r) {
  if (key[KNN - 1] == ~0ull) return false;
  const int lo0 = max(b0 - r, 0), hi0 = min(b0 + r, g.nb[0] - 1);
  const int lo1 = max(b1 - r, 0), hi1 = min(b1 + r, g.nb[1] - 1);
  double reach = 1e300;
  if (lo0 > 0) reach = fmin(reach, x[0] - (g.kmin[0] + lo0 * g.h));
  if (hi0 < g.nb[0] - 1) reach = fmin(reach, g.kmin[0] + (hi0 + 1) * g.h - x[0]);
  if (lo1 > 0) reach = fmin(reach, x[1] - (g.kmin[1] + lo1 * g.h));
  if (hi1 < g.nb[1] - 1) reach = fmin(reach, g.kmin[1] + (hi1 + 1) * g.h - x[1]);
  const float d16 = __uint_as_float((unsigned)(key[KNN - 1] >> 32));
  return (double)d16 < reach * reach * (1.0 - 1e-6);
}

// rings r0 .. span around the sample's bin (b0, b1) from global memory, ring
// by ring, until knn_done
__device__ inline void knn_rings(const WSample<2>* __restrict__ ss, const int32_t* __restrict__ sidx,
                                 const int32_t* __restrict__ boff, const WBinGeom& g, const double* x, int jself,
                                 int b0, int b1, int r0, unsigned long long (&key)[KNN]) {
  for (int r = r0; r <= g.span; ++r) {
    const int lo0 = max(b0 - r, 0), hi0 = min(b0 + r, g.nb[0] - 1);
    const int lo1 = max(b1 - r, 0), hi1 = min(b1 + r, g.nb[1] - 1);
    for (int c0 = lo0; c0 <= hi0; ++c0) {
      const bool edge_row = (c0 == b0 - r) || (c0 == b0 + r);
      if (edge_row) {
        // the whole row of the ring: one contiguous range of the bin order
        knn_visit_bin(ss, sidx, boff[c0 * g.nb[1] + lo1], boff[c0 * g.nb[1] + hi1 + 1], x, jself, g.R, key);
      } else {
        if (b1 - r >= 0) {
          const int bin = c0 * g.nb[1] + b1 - r;
          knn_visit_bin(ss, sidx, boff[bin], boff[bin + 1], x, jself, g.R, key);
        }
        if (r > 0 && b1 + r < g.nb[1]) {
          const int bin = c0 * g.nb[1] + b1 + r;
          knn_visit_bin(ss, sidx, boff[bin], boff[bin + 1], x, jself, g.R, key);
        }
      }
    }
    if (knn_done(key, g, x, b0, b1, r)) return;
  }
}

// keys (float32 d2 bits << 32 | caller index) of the 16 nearest box
// neighbours of sample (x, jself); empty slots stay ~0. Bins are visited in
// rings of growing Chebyshev distance around the sample's bin, until every
// unvisited sample is farther than the 16th (knn_done).
__device__ inline void knn_search(const WSample<2>* __restrict__ ss, const int32_t* __restrict__ sidx,
                                  const int32_t* __restrict__ boff, const WBinGeom& g, const double* x, int jself,
                                  unsigned long long (&key)[KNN]) {
#pragma unroll
  for (int q = 0; q < KNN; ++q) key[q] = ~0ull;
  const int b0 = wbin_clamp(x[0], g.kmin[0], g.h, g.nb[0]);
  const int b1 = wbin_clamp(x[1], g.kmin[1], g.h, g.nb[1]);
  knn_rings(ss, sidx, boff, g, x, jself, b0, b1, 0, key);
}

// features (float32) and the analytic estimate of one sample (sorted
// position t) from its keys (caller indices, found in ss through inv)
__device__ inline double knn_features_of(const unsigned long long (&key)[KNN], const WSample<2>* __restrict__ ss,
                                         const int32_t* __restrict__ inv, int64_t t, float R, float* f) {
  const double pi = 3.141592653589793238462643383279502884;
  const WSample<2> me = ss[t];
  const double x0 = me.k[0], x1 = me.k[1];
  const double s0 = me.sc[0][0], c0 = me.sc[0][1], s1 = me.sc[1][0], c1 = me.sc[1][1];
  double sum = 0.0;
#pragma unroll
  for (int q = 0; q < KNN; ++q) {
    if (key[q] == ~0ull) {
      f[2 * q] = R;
      f[2 * q + 1] = R;
      continue;
    }
    const WSample<2> o = ss[inv[(int64_t)(unsigned)(key[q] & 0xffffffffull)]];
    const double dx = o.k[0] - x0, dy = o.k[1] - x1;
    f[2 * q] = (float)dx;
    f[2 * q + 1] = (float)dy;
    double g = 1.0;
    if (dx != 0.0) g *= (o.sc[0][0] * c0 - o.sc[0][1] * s0) / (pi * dx);
    if (dy != 0.0) g *= (o.sc[1][0] * c1 - o.sc[1][1] * s1) / (pi * dy);
    sum += g * g;
  }
  return 1.0 / (1.0 + sum);
}

// features of every sample (caller order); with alpha != null also the
// training target log(alpha / base)
__global__ __launch_bounds__(256) void k_knn_features(const WSample<2>* __restrict__ ss,
                                                      const int32_t* __restrict__ sidx,
                                                      const int32_t* __restrict__ boff, WBinGeom g,
                                                      const int32_t* __restrict__ inv, int64_t m,
                                                      float* __restrict__ feat, double* __restrict__ base,
                                                      const double* __restrict__ alpha, float* __restrict__ target) {
  const int64_t t = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (t >= m) return;
  const int j = sidx[t];
  const double x[2] = {ss[t].k[0], ss[t].k[1]};
  unsigned long long key[KNN];
  knn_search(ss, sidx, boff, g, x, j, key);
  float f[NF];
  const double b = knn_features_of(key, ss, inv, t, (float)g.R, f);
#pragma unroll
  for (int q = 0; q < NF; ++q) feat[(int64_t)j * NF + q] = f[q];
  if (base) base[j] = b;
  if (alpha && target) target[j] = (float)log(alpha[j] / b);
}

// ---------------------------------------------------------------------------
// MFMA inference
// ---------------------------------------------------------------------------

struct MlpFrags {
  half4_t w1[4][2];   // [m-tile][k-step]
  half4_t w2[4][4];
  half4_t w3[4];
  float b1[4][4];     // [m-tile][r]
  float b2[4][4];
  float b3;
};

__device__ inline void load_frags(const _Float16* __restrict__ P16, const float* __restrict__ P32, MlpFrags& F) {
  const int l = threadIdx.x & 63;
  const int n = l & 15, kq = 4 * (l >> 4);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int r = 0; r < 4; ++r) F.w1[mt][ks][r] = P16[MLP_W1 + (16 * ks + kq + r) * HW + 16 * mt + n];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int r = 0; r < 4; ++r) F.w2[mt][ks][r] = P16[MLP_W2 + (16 * ks + kq + r) * HW + 16 * mt + n];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      F.b1[mt][r] = P32[MLP_B1 + 16 * mt + kq + r];
      F.b2[mt][r] = P32[MLP_B2 + 16 * mt + kq + r];
    }
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int r = 0; r < 4; ++r) F.w3[ks][r] = (n == 0) ? P16[MLP_W3 + 16 * ks + kq + r] : (_Float16)0.f;
  F.b3 = P32[MLP_B3];
}

// y of 16 samples whose half features are rows [0,16) of xs (row pitch NF);
// every lane must be active. Lane l < 16 returns y of sample l.
__device__ inline float mlp_block16(const _Float16* xs, const MlpFrags& F) {
  const int l = threadIdx.x & 63;
  const int s = l & 15, kq = 4 * (l >> 4);
  half4_t xb[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
#pragma unroll
    for (int r = 0; r < 4; ++r) xb[ks][r] = xs[s * NF + 16 * ks + kq + r];
  half4_t h1[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x16f16(F.w1[mt][ks], xb[ks], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) h1[mt][r] = (_Float16)silu_f(acc[r] + F.b1[mt][r]);
  }
  half4_t h2[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x16f16(F.w2[mt][ks], h1[ks], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) h2[mt][r] = (_Float16)silu_f(acc[r] + F.b2[mt][r]);
  }
  float4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x16f16(F.w3[ks], h2[ks], acc, 0, 0, 0);
  return acc[0] + F.b3;   // row 0 of the output tile: lanes 0..15
}

// y for n given feature rows (float32 in, rounded to half)
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ feat, int64_t n,
                                                     const _Float16* __restrict__ P16,
                                                     const float* __restrict__ P32, float* __restrict__ y) {
  __shared__ _Float16 xs[256 * NF];
  __shared__ float ys[256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t base = (int64_t)blockIdx.x * 256;
  for (int e = tid; e < 256 * NF; e += 256) {
    const int64_t row = base + e / NF;
    xs[e] = (_Float16)(row < n ? feat[row * NF + (e % NF)] : 0.f);
  }
  __syncthreads();
  MlpFrags F;
  load_frags(P16, P32, F);
#pragma unroll
  for (int gq = 0; gq < 4; ++gq) {
    const float v = mlp_block16(xs + (wave * 64 + gq * 16) * NF, F);
    if (lane < 16) ys[wave * 64 + gq * 16 + lane] = v;
  }
  __syncthreads();
  if (base + tid < n) y[base + tid] = ys[tid];
}

// Staged search of a workgroup's 256 consecutive bin-sorted samples: when
// they share one bin row, the candidates of the rings 0 .. KNN_RING around
// all of their bins (bin rows b0 - 2 .. b0 + 2, the workgroup's bin columns
// widened by 2 on each side) are copied to LDS once (coalesced), and each
// sample walks its rings 0 .. 2 there, in the order and with the early exit
// of the search from global memory; a sample whose 16th neighbour is not yet
// known to be the nearest continues with ring 3 from global memory. A workgroup spanning two bin rows, or too many candidates,
// searches from global memory as before. The candidates visited differ, the
// result (the 16 smallest keys of the box) does not.
constexpr int KNN_RING = 2;
constexpr int KNN_ROWS = 2 * KNN_RING + 1;
constexpr int KNN_STAGE = 2048;    // staged candidates at most (k and caller index: 40 KiB)
constexpr int KNN_COLS = 128;      // staged bin columns per row at most

// fused: 16-NN features, MLP, alpha_hat = base * exp(y), in caller order
__global__ __launch_bounds__(256) void k_learned_weights(const WSample<2>* __restrict__ ss,
                                                         const int32_t* __restrict__ sidx,
                                                         const int32_t* __restrict__ boff, WBinGeom g,
                                                         const int32_t* __restrict__ inv, int64_t m,
                                                         const _Float16* __restrict__ P16,
                                                         const float* __restrict__ P32,
                                                         double* __restrict__ alpha) {
  // the staged candidates, then (after the search) the half features
  constexpr size_t STAGE_BYTES = KNN_STAGE * (sizeof(double2) + sizeof(int));
  constexpr size_t XS_BYTES = 256 * NF * sizeof(_Float16);
  __shared__ __align__(16) unsigned char pool[STAGE_BYTES > XS_BYTES ? STAGE_BYTES : XS_BYTES];
  double2* sk = reinterpret_cast<double2*>(pool);
  int* sid = reinterpret_cast<int*>(pool + KNN_STAGE * sizeof(double2));
  _Float16* xs = reinterpret_cast<_Float16*>(pool);
  __shared__ int sbo[KNN_ROWS][KNN_COLS + 1];   // LDS offset of each staged bin, per row
  __shared__ int sinfo[8];                       // b0 min, b0 max, b1 min, b1 max, staged flag, c1
  __shared__ float ys[256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t t = xcd_block(blockIdx.x, gridDim.x) * 256 + tid;
  double x[2] = {0.0, 0.0};
  int j = -1, b0 = 0, b1 = 0;
  if (t < m) {
    j = sidx[t];
    x[0] = ss[t].k[0];
    x[1] = ss[t].k[1];
    b0 = wbin_clamp(x[0], g.kmin[0], g.h, g.nb[0]);
    b1 = wbin_clamp(x[1], g.kmin[1], g.h, g.nb[1]);
  }
  if (tid < 4) sinfo[tid] = (tid & 1) ? -1 : (1 << 30);
  __syncthreads();
  if (j >= 0) {
    atomicMin(&sinfo[0], b0);
    atomicMax(&sinfo[1], b0);
    atomicMin(&sinfo[2], b1);
    atomicMax(&sinfo[3], b1);
  }
  __syncthreads();
  const int r0 = sinfo[0], c1 = max(sinfo[2] - KNN_RING, 0), c2 = min(sinfo[3] + KNN_RING, g.nb[1] - 1);
  bool staged = sinfo[1] == r0 && r0 >= 0 && c2 - c1 + 1 <= KNN_COLS;
  if (staged) {
    // per staged row: its candidate range in the bin order and LDS base
    if (tid == 0) {
      int base = 0;
      for (int q = 0; q < KNN_ROWS; ++q) {
        const int r = r0 - KNN_RING + q;
        const int n = (r >= 0 && r < g.nb[0]) ? boff[r * g.nb[1] + c2 + 1] - boff[r * g.nb[1] + c1] : 0;
        sbo[q][KNN_COLS] = base;   // (the row's base, overwritten below)
        base += n;
      }
      sinfo[4] = base <= KNN_STAGE ? 1 : 0;
    }
    __syncthreads();
    staged = sinfo[4] != 0;
    if (staged) {
      const int ncol = c2 - c1 + 2;
      int rbase[KNN_ROWS];
#pragma unroll
      for (int q = 0; q < KNN_ROWS; ++q) rbase[q] = sbo[q][KNN_COLS];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < KNN_ROWS; ++q) {
        const int r = r0 - KNN_RING + q;
        if (r < 0 || r >= g.nb[0]) continue;
        const int gb = boff[r * g.nb[1] + c1];
        const int n = boff[r * g.nb[1] + c2 + 1] - gb;
        for (int i = tid; i < n; i += 256) {
          sk[rbase[q] + i] = make_double2(ss[gb + i].k[0], ss[gb + i].k[1]);
          sid[rbase[q] + i] = sidx[gb + i];
        }
        for (int c = tid; c < ncol; c += 256) sbo[q][c] = rbase[q] + boff[r * g.nb[1] + c1 + c] - gb;
      }
      __syncthreads();
    }
  }
  unsigned long long key[KNN];
#pragma unroll
  for (int q = 0; q < KNN; ++q) key[q] = ~0ull;
  if (j >= 0) {
    if (staged) {
      // rings 0 .. KNN_RING from LDS, in the order and with the early exit
      // of the search from global memory, then ring KNN_RING + 1 on from there
      auto visit = [&](int q, int cb, int ce) {   // staged row q, bin columns cb .. ce
        const int e = sbo[q][ce + 1 - c1];
        for (int i = sbo[q][cb - c1]; i < e; ++i) {
          const double2 kc = sk[i];
          knn_visit(kc.x, kc.y, sid[i], x, j, g.R, key);
        }
      };
      bool done = false;
      for (int r = 0; r <= KNN_RING && !done; ++r) {
        const int lo0 = max(b0 - r, 0), hi0 = min(b0 + r, g.nb[0] - 1);
        const int lo1 = max(b1 - r, 0), hi1 = min(b1 + r, g.nb[1] - 1);
        for (int c0 = lo0; c0 <= hi0; ++c0) {
          const int q = c0 - (r0 - KNN_RING);
          if (c0 == b0 - r || c0 == b0 + r) {
            visit(q, lo1, hi1);
          } else {
            if (b1 - r >= 0) visit(q, b1 - r, b1 - r);
            if (r > 0 && b1 + r < g.nb[1]) visit(q, b1 + r, b1 + r);
          }
        }
        done = knn_done(key, g, x, b0, b1, r);
      }
      if (!done) knn_rings(ss, sidx, boff, g, x, j, b0, b1, KNN_RING + 1, key);
    } else {
      knn_rings(ss, sidx, boff, g, x, j, b0, b1, 0, key);
    }
  }
  float f[NF];
  double b = 1.0;
  if (j >= 0) b = knn_features_of(key, ss, inv, t, (float)g.R, f);
  __syncthreads();   // the stage is no longer read: its LDS takes the features
  if (j >= 0) {
#pragma unroll
    for (int q = 0; q < NF; ++q) xs[tid * NF + q] = (_Float16)f[q];
  } else {
#pragma unroll
    for (int q = 0; q < NF; ++q) xs[tid * NF + q] = (_Float16)0.f;
  }
  __syncthreads();
  MlpFrags F;
  load_frags(P16, P32, F);
#pragma unroll
  for (int gq = 0; gq < 4; ++gq) {
    const float v = mlp_block16(xs + (wave * 64 + gq * 16) * NF, F);
    if (lane < 16) ys[wave * 64 + gq * 16 + lane] = v;
  }
  __syncthreads();
  if (j >= 0) alpha[j] = b * exp((double)ys[tid]);
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------

constexpr int TS = 64;   // samples per training workgroup

// partial gradient of the mean squared error over one workgroup's samples.
// Minibatch `mb` holds samples j = mb + nmb * s, s in [0, batch) (and j < m).
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ X, const float* __restrict__ T,
                                                  int64_t m, int64_t mb, int64_t nmb, int64_t batch,
                                                  const float* __restrict__ P, int fp16,
                                                  float* __restrict__ partial) {
  __shared__ float sW1[NF * HW], sW2[HW * HW], sW3[HW], sb1[HW], sb2[HW];
  __shared__ float sX[TS][NF + 1];
  __shared__ float sZ1[TS][HW + 1], sH1[TS][HW + 1], sZ2[TS][HW + 1];
  __shared__ float sdy[TS], sloss[TS];
  const int tid = threadIdx.x;
  const float b3 = P[MLP_B3];
  for (int e = tid; e < NF * HW; e += 256) sW1[e] = fp16 ? round_h(P[MLP_W1 + e]) : P[MLP_W1 + e];
  for (int e = tid; e < HW * HW; e += 256) sW2[e] = fp16 ? round_h(P[MLP_W2 + e]) : P[MLP_W2 + e];
  if (tid < HW) {
    sW3[tid] = fp16 ? round_h(P[MLP_W3 + tid]) : P[MLP_W3 + tid];
    sb1[tid] = P[MLP_B1 + tid];
    sb2[tid] = P[MLP_B2 + tid];
  }
  const int64_t s0 = (int64_t)blockIdx.x * TS;
  for (int e = tid; e < TS * NF; e += 256) {
    const int s = e / NF, q = e % NF;
    const int64_t sg = s0 + s, j = mb + nmb * sg;
    float v = (sg < batch && j < m) ? X[j * NF + q] : 0.f;
    sX[s][q] = fp16 ? round_h(v) : v;
  }
  __syncthreads();
  const int s = tid >> 2, n0 = (tid & 3) * 16;
  // layer 1
  for (int c = 0; c < 16; ++c) {
    const int n = n0 + c;
    float z = sb1[n];
    for (int q = 0; q < NF; ++q) z += sX[s][q] * sW1[q * HW + n];
    sZ1[s][n] = z;
    const float h = silu_f(z);
    sH1[s][n] = fp16 ? round_h(h) : h;
  }
  __syncthreads();
  // layer 2
  for (int c = 0; c < 16; ++c) {
    const int n = n0 + c;
    float z = sb2[n];
    for (int q = 0; q < HW; ++q) z += sH1[s][q] * sW2[q * HW + n];
    sZ2[s][n] = z;
  }
  __syncthreads();
  // output, residual
  if (tid < TS) {
    const int64_t sg = s0 + tid, j = mb + nmb * sg;
    const bool valid = sg < batch && j < m;
    float y = b3;
    for (int q = 0; q < HW; ++q) {
      const float h = silu_f(sZ2[tid][q]);
      y += (fp16 ? round_h(h) : h) * sW3[q];
    }
    const float r = valid ? y - T[j] : 0.f;
    sdy[tid] = 2.f * r / (float)batch;
    sloss[tid] = r * r;
  }
  __syncthreads();
  float* out = partial + (int64_t)blockIdx.x * MLP_NPARAM_PAD;
  // dW3, db3 (from h2 = silu(z2)) before z2 is overwritten by dz2
  if (tid < HW) {
    float g = 0.f;
    for (int q = 0; q < TS; ++q) {
      const float h = silu_f(sZ2[q][tid]);
      g += (fp16 ? round_h(h) : h) * sdy[q];
    }
    out[MLP_W3 + tid] = g;
  }
  if (tid == HW) {
    float g = 0.f, L = 0.f;
    for (int q = 0; q < TS; ++q) {
      g += sdy[q];
      L += sloss[q];
    }
    out[MLP_B3] = g;
    out[MLP_NPARAM] = L;   // sum of squared residuals of this group
  }
  __syncthreads();
  for (int c = 0; c < 16; ++c) {
    const int n = n0 + c;
    sZ2[s][n] = sdy[s] * sW3[n] * silu_grad_f(sZ2[s][n]);   // dz2
  }
  __syncthreads();
  // dW2[i][n] = sum_s h1[s][i] dz2[s][n]; dz1 = (dz2 W2^T) * silu'(z1)
  {
    const int i = tid >> 2;
    for (int c = 0; c < 16; ++c) {
      const int n = n0 + c;
      float g = 0.f;
      for (int q = 0; q < TS; ++q) g += sH1[q][i] * sZ2[q][n];
      out[MLP_W2 + i * HW + n] = g;
    }
  }
  if (tid < HW) {
    float g = 0.f;
    for (int q = 0; q < TS; ++q) g += sZ2[q][tid];
    out[MLP_B2 + tid] = g;
  }
  for (int c = 0; c < 16; ++c) {
    const int i = n0 + c;
    float d = 0.f;
    for (int q = 0; q < HW; ++q) d += sZ2[s][q] * sW2[i * HW + q];
    sZ1[s][i] = d * silu_grad_f(sZ1[s][i]);   // dz1 (own entries only)
  }
  __syncthreads();
  // dW1[q][i] = sum_s x[s][q] dz1[s][i]
  {
    const int q = tid >> 3, i0 = (tid & 7) * 8;
    for (int c = 0; c < 8; ++c) {
      const int i = i0 + c;
      float g = 0.f;
      for (int r = 0; r < TS; ++r) g += sX[r][q] * sZ1[r][i];
      out[MLP_W1 + q * HW + i] = g;
    }
  }
  if (tid < HW) {
    float g = 0.f;
    for (int q = 0; q < TS; ++q) g += sZ1[q][tid];
    out[MLP_B1 + tid] = g;
  }
}

// sum the partial gradients in block order; optionally apply Adam
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, int nblk,
                                                    float* __restrict__ grad, float* __restrict__ loss_sum,
                                                    float* __restrict__ P, _Float16* __restrict__ P16,
                                                    float* __restrict__ Mo, float* __restrict__ Vo, int adam,
                                                    float lr, float beta1, float beta2, float eps, float bc1,
                                                    float bc2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > MLP_NPARAM) return;
  float g = 0.f;
  for (int b = 0; b < nblk; ++b) g += partial[(int64_t)b * MLP_NPARAM_PAD + p];
  if (p == MLP_NPARAM) {
    *loss_sum = g;
    return;
  }
  grad[p] = g;
  if (adam) {
    const float mm = beta1 * Mo[p] + (1.f - beta1) * g;
    const float vv = beta2 * Vo[p] + (1.f - beta2) * g * g;
    Mo[p] = mm;
    Vo[p] = vv;
    const float w = P[p] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    P[p] = w;
    P16[p] = (_Float16)w;
  }
}

__global__ void k_params_to_half(const float* __restrict__ P, _Float16* __restrict__ P16) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < MLP_NPARAM) P16[p] = (_Float16)P[p];
}

// ---------------------------------------------------------------------------
// audit: relative RMS difference of learned and plain weights on a subset
// ---------------------------------------------------------------------------

__global__ void k_audit_indices(int32_t* idx, int64_t n, int64_t m) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n) idx[q] = (int32_t)((q * m) / n);
}

__global__ __launch_bounds__(256) void k_audit(const int32_t* __restrict__ idx, const double* __restrict__ plain,
                                               int64_t n, const double* __restrict__ learned,
                                               double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += 256) {
    const double e = (learned[idx[q]] - plain[q]) / plain[q];
    s += e * e;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0] / (double)n);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

void launch_knn_features(ftcg_plan p, const double* k, float* feat, double* base, const double* alpha,
                         float* target) {
  const unsigned nb = (unsigned)((p->m + 255) / 256);
  hipLaunchKernelGGL(k_knn_features, dim3(nb), dim3(256), 0, p->stream, p->ws_k.as<WSample<2>>(),
                     p->ws_idx.as<int32_t>(), p->wb_off.as<int32_t>(), p->wgeom, p->ws_inv.as<int32_t>(), p->m,
                     feat, base, alpha, target);
  FTCG_HIP(hipGetLastError());
}

void launch_learned_weights(ftcg_plan p, const double* k, const ftcg_mlp_s* mlp) {
  const unsigned nb = (unsigned)((p->m + 255) / 256);
  hipLaunchKernelGGL(k_learned_weights, dim3(nb), dim3(256), 0, p->stream, p->ws_k.as<WSample<2>>(),
                     p->ws_idx.as<int32_t>(), p->wb_off.as<int32_t>(), p->wgeom, p->ws_inv.as<int32_t>(), p->m,
                     mlp->params16.as<_Float16>(), mlp->params.as<float>(), p->alpha.as<double>());
  FTCG_HIP(hipGetLastError());
}

void launch_mlp_forward(const ftcg_mlp_s* mlp, const float* feat, int64_t n, float* y) {
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(256), 0, mlp->stream, feat, n, mlp->params16.as<_Float16>(),
                     mlp->params.as<float>(), y);
  FTCG_HIP(hipGetLastError());
}

void launch_mlp_grad(ftcg_mlp_s* mlp, const float* X, const float* T, int64_t m, int64_t mb, int64_t nmb,
                     int64_t batch, int fp16, int adam, float lr, float* grad_out) {
  const int nblk = (int)((batch + TS - 1) / TS);
  mlp->partial.ensure(sizeof(float) * (size_t)nblk * MLP_NPARAM_PAD);
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, mlp->stream, X, T, m, mb, nmb, batch,
                     mlp->params.as<float>(), fp16, mlp->partial.as<float>());
  float bc1 = 1.f, bc2 = 1.f;
  if (adam) {
    mlp->step += 1;
    bc1 = 1.f - powf(mlp->beta1, (float)mlp->step);
    bc2 = 1.f - powf(mlp->beta2, (float)mlp->step);
  }
  hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, mlp->stream,
                     mlp->partial.as<float>(), nblk, grad_out ? grad_out : mlp->grad.as<float>(),
                     mlp->loss_dev.as<float>() + mlp->loss_slot, mlp->params.as<float>(),
                     mlp->params16.as<_Float16>(), mlp->adam_m.as<float>(), mlp->adam_v.as<float>(), adam, lr,
                     mlp->beta1, mlp->beta2, mlp->eps, bc1, bc2);
  FTCG_HIP(hipGetLastError());
}

void launch_params_to_half(ftcg_mlp_s* mlp) {
  hipLaunchKernelGGL(k_params_to_half, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, mlp->stream,
                     mlp->params.as<float>(), mlp->params16.as<_Float16>());
  FTCG_HIP(hipGetLastError());
}

void launch_audit(ftcg_plan p, const double* k, double* est_dev) {
  const int64_t n = p->audit_samples < p->m ? p->audit_samples : p->m;
  p->audit_buf.ensure(sizeof(int32_t) * n + sizeof(double) * n + 64);
  int32_t* idx = p->audit_buf.as<int32_t>();
  double* plain = reinterpret_cast<double*>(reinterpret_cast<char*>(p->audit_buf.p) +
                                            ((sizeof(int32_t) * n + 15) & ~(size_t)15));
  hipLaunchKernelGGL(k_audit_indices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p->stream, idx, n, p->m);
  plain_weights_at(p, k, idx, n, plain);
  hipLaunchKernelGGL(k_audit, dim3(1), dim3(256), 0, p->stream, idx, plain, n, p->alpha.as<double>(), est_dev);
  FTCG_HIP(hipGetLastError());
}

}  // namespace ftcg
