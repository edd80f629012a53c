// Inverse FFT of the oversampled grid, crop, and deapodization
// (the sum over psi_m = e^{2 pi i m x} / w(x) of eq:cgmatrix and zeta_n = psi_n / w
// of eq:newadm).
//
// The transform wanted is J[q] = sum_g H[g] e^{+2 pi i (g - G/2)(q - G/2)/G}
// for the centred n outputs q = p + (G - n)/2. With G divisible by 4,
// (g - G/2)(q - G/2)/G = gq/G - g/2 - q/2 + G/4, so J[q] = (-1)^q sum_g
// (-1)^g H[g] e^{2 pi i g q / G}: a plain unnormalised inverse DFT with sign
// flips on load and store.
//
// One workgroup transforms one row of length G held in LDS (Stockham
// autosort, one radix-2 stage when log2 G is odd, then radix-4 stages; every
// stage reads its butterfly inputs into registers, synchronises, and writes
// in place). Only the n cropped outputs are stored, transposed, so the next
// pass again reads contiguous rows:
//   pass 1: rows g0 of H (G x G)  -> T1[q1'][g0]  (n x G)
//   pass 2: rows q1' of T1         -> image[p0][p1] (n x n), times
//           1/Phi(x_p0/sigma) / Phi(x_p1/sigma) formed in float64.
// Rows are assigned so that each of the 8 XCDs (workgroups are dealt to XCDs
// round-robin) works on a contiguous block of rows; the transposed 8-byte
// stores of neighbouring rows then meet in that XCD's L2 and leave it as whole
// lines.
#include "ftcg_internal.h"
#include "batch_internal.h"

namespace ftcg {

template <class real>
struct CxF;
template <>
struct CxF<float> {
  using t = float2;
  static __device__ inline void sincospi_(float x, float* s, float* c) { sincospif(x, s, c); }
};
template <>
struct CxF<double> {
  using t = double2;
  static __device__ inline void sincospi_(double x, double* s, double* c) { sincospi(x, s, c); }
};

template <class cx>
__device__ inline cx cmul(cx a, cx b) {
  cx r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <class cx>
__device__ inline cx cadd(cx a, cx b) {
  cx r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <class cx>
__device__ inline cx csub(cx a, cx b) {
  cx r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <class cx>
__device__ inline cx cmul_i(cx a) {  // a * (+i)
  cx r;
  r.x = -a.y;
  r.y = a.x;
  return r;
}

constexpr int FFT_MAXB = 8;  // butterflies per thread per stage (radix-2 stage worst case)

// in-place inverse (positive exponent) FFT of buf[0..L) in LDS, L = 2^log2L
template <class real>
__device__ void lds_ifft(typename CxF<real>::t* buf, int L, int log2L) {
  using cx = typename CxF<real>::t;
  const int tid = threadIdx.x, nth = blockDim.x;
  int Ns = 1;
  if (log2L & 1) {
    // radix 2, Ns = 1: no twiddles
    cx v0[FFT_MAXB], v1[FFT_MAXB];
    const int half = L >> 1;
#pragma unroll
    for (int u = 0; u < FFT_MAXB; ++u)
      if (tid + u * nth < half) {
        const int b = tid + u * nth;
        v0[u] = buf[b];
        v1[u] = buf[b + half];
      }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < FFT_MAXB; ++u)
      if (tid + u * nth < half) {
        const int b = tid + u * nth;
        buf[2 * b] = cadd(v0[u], v1[u]);
        buf[2 * b + 1] = csub(v0[u], v1[u]);
      }
    __syncthreads();
    Ns = 2;
  }
  const int quarter = L >> 2;
  for (; Ns < L; Ns <<= 2) {
    cx v[FFT_MAXB / 2][4];
#pragma unroll
    for (int u = 0; u < FFT_MAXB / 2; ++u)
      if (tid + u * nth < quarter) {
        const int b = tid + u * nth;
        const int k = b & (Ns - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[u][r] = buf[b + r * quarter];
        if (Ns > 1) {
          real s, c;
          CxF<real>::sincospi_((real)k / (real)(2 * Ns), &s, &c);  // e^{2 pi i k / (4 Ns)}
          cx w1;
          w1.x = c;
          w1.y = s;
          const cx w2 = cmul(w1, w1);
          const cx w3 = cmul(w2, w1);
          v[u][1] = cmul(v[u][1], w1);
          v[u][2] = cmul(v[u][2], w2);
          v[u][3] = cmul(v[u][3], w3);
        }
      }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < FFT_MAXB / 2; ++u)
      if (tid + u * nth < quarter) {
        const int b = tid + u * nth;
        const int k = b & (Ns - 1);
        const cx a0 = cadd(v[u][0], v[u][2]);
        const cx a1 = csub(v[u][0], v[u][2]);
        const cx a2 = cadd(v[u][1], v[u][3]);
        const cx a3 = cmul_i(csub(v[u][1], v[u][3]));
        const int d = (b - k) * 4 + k;  // (b / Ns) * 4 Ns + k
        buf[d] = cadd(a0, a2);
        buf[d + Ns] = cadd(a1, a3);
        buf[d + 2 * Ns] = csub(a0, a2);
        buf[d + 3 * Ns] = csub(a1, a3);
      }
    __syncthreads();
  }
}

__device__ inline int xcd_row(int b, int rows) {
  // rows % 8 == 0: XCD x (= b % 8) gets rows x*rows/8 .. (x+1)*rows/8 - 1 in order
  if (rows & 7) return b;
  return (b & 7) * (rows >> 3) + (b >> 3);
}

// one row: load (with the (-1)^(row+g) modulation when pre_sign), transform,
// store the cropped outputs at out[q' * out_stride_q] times (-1)^q * fr * dq[q']
template <class real>
__device__ inline void fft_row(const typename CxF<real>::t* __restrict__ src, typename CxF<real>::t* __restrict__ dst,
                               int64_t out_stride_q, int L, int log2L, int ncrop, int crop_off, int row,
                               int pre_sign, const double* __restrict__ dq, double fr,
                               typename CxF<real>::t* buf) {
  using cx = typename CxF<real>::t;
  for (int g = threadIdx.x; g < L; g += blockDim.x) {
    cx v = src[g];
    if (pre_sign && ((row + g) & 1)) {
      v.x = -v.x;
      v.y = -v.y;
    }
    buf[g] = v;
  }
  __syncthreads();
  lds_ifft<real>(buf, L, log2L);
  for (int qp = threadIdx.x; qp < ncrop; qp += blockDim.x) {
    const int q = qp + crop_off;
    double f = ((q & 1) ? -1.0 : 1.0) * fr;
    if (dq) f *= dq[qp];
    const real fs = (real)f;
    cx v = buf[q];
    v.x *= fs;
    v.y *= fs;
    dst[(int64_t)qp * out_stride_q] = v;
  }
}

template <class real>
__global__ void k_fft_rows(const typename CxF<real>::t* __restrict__ in, int64_t in_row_stride,
                           typename CxF<real>::t* __restrict__ out, int64_t out_stride_q, int64_t out_stride_row,
                           int L, int log2L, int ncrop, int crop_off, int rows, int pre_sign,
                           const double* __restrict__ dq, const double* __restrict__ drow) {
  using cx = typename CxF<real>::t;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx* buf = reinterpret_cast<cx*>(smem_raw);
  const int row = xcd_row(blockIdx.x, rows);
  fft_row<real>(in + (int64_t)row * in_row_stride, out + (int64_t)row * out_stride_row, out_stride_q, L, log2L,
                ncrop, crop_off, row, pre_sign, dq, drow ? drow[row] : 1.0, buf);
}

// batched passes over the items of one grid size G (all with n = G / sigma):
// pass 1 maps row r to item list[r / G], grid row r % G; pass 2 maps row r to
// item list[r / n], intermediate row r % n
__global__ void k_fft_rows_batched(const BatchItem* __restrict__ items, const int* __restrict__ list,
                                   const BatchArgs* __restrict__ args, int pass, int L, int log2L, int n,
                                   int rows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float2* buf = reinterpret_cast<float2*>(smem_raw);
  const int r = xcd_row(blockIdx.x, rows);
  const int per = pass == 1 ? L : n;
  const BatchItem it = items[list[r / per]];
  const int row = r % per;
  const int crop_off = (L - n) / 2;
  if (pass == 1) {
    fft_row<float>(args->grid + it.grid_off + (int64_t)row * L, args->tmp + it.tmp_off + row, L, L, log2L, n,
                   crop_off, row, 1, nullptr, 1.0, buf);
  } else {
    const double* d = args->deapod + it.deapod_off;
    fft_row<float>(args->tmp + it.tmp_off + (int64_t)row * L, args->images + it.img_off + row, n, L, log2L, n,
                   crop_off, row, 0, d, d[row], buf);
  }
}

void batch_fft_prepare() {
  static bool attr_done = false;
  if (!attr_done) {
    FTCG_HIP(hipFuncSetAttribute((const void*)k_fft_rows_batched, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 160 * 1024));
    attr_done = true;
  }
}

void batch_fft(ftcg_batch_s* b) {
  const int* lists = b->group_items.as<int>();
  int64_t list_off = 0;
  for (const auto& grp : b->fft_groups) {
    const int64_t G = b->items[grp[0]].G;
    const int n = b->items[grp[0]].n;
    int log2L = 0;
    while ((int64_t(1) << log2L) < G) ++log2L;
    int nth = (int)(G / 16);
    nth = nth < 64 ? 64 : (nth > 1024 ? 1024 : nth);
    const size_t lds = (size_t)G * sizeof(float2);
    for (int pass = 1; pass <= 2; ++pass) {
      const int rows = (int)grp.size() * (pass == 1 ? (int)G : n);
      hipLaunchKernelGGL(k_fft_rows_batched, dim3((unsigned)rows), dim3(nth), lds, b->stream,
                         b->items_dev.as<BatchItem>(), lists + list_off, b->args_dev.as<BatchArgs>(), pass, (int)G,
                         log2L, n, rows);
    }
    list_off += (int64_t)grp.size();
  }
  FTCG_HIP(hipGetLastError());
}

template <class real>
static void launch_rows(ftcg_plan p, const void* in, int64_t in_row_stride, void* out, int64_t out_stride_q,
                        int64_t out_stride_row, int rows, int pre_sign, const double* dq, const double* drow) {
  using cx = typename CxF<real>::t;
  const int L = (int)p->G;
  int log2L = 0;
  while ((1 << log2L) < L) ++log2L;
  int nth = L / 16;
  nth = nth < 64 ? 64 : (nth > 1024 ? 1024 : nth);
  const size_t lds = (size_t)L * sizeof(cx);
  static bool attr_done = false;
  if (!attr_done) {
    FTCG_HIP(hipFuncSetAttribute((const void*)k_fft_rows<real>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 160 * 1024));
    attr_done = true;
  }
  const int ncrop = (int)p->n;
  const int crop_off = (int)((p->G - p->n) / 2);
  hipLaunchKernelGGL(k_fft_rows<real>, dim3((unsigned)rows), dim3(nth), lds, p->stream,
                     static_cast<const cx*>(in), in_row_stride, static_cast<cx*>(out), out_stride_q, out_stride_row,
                     L, log2L, ncrop, crop_off, rows, pre_sign, dq, drow);
  FTCG_HIP(hipGetLastError());
}

template <class real>
static void grid_to_image_t(ftcg_plan p, const void* grid, void* image) {
  const double* d = p->deapod.as<double>();
  const int64_t G = p->G, n = p->n;
  if (p->dim == 1) {
    timing_begin(p, STEP_FFT2);
    launch_rows<real>(p, grid, G, image, 1, 0, 1, 1, d, nullptr);
    timing_end(p, STEP_FFT2);
    return;
  }
  timing_begin(p, STEP_FFT1);
  launch_rows<real>(p, grid, G, p->fft_tmp.p, G, 1, (int)G, 1, nullptr, nullptr);
  timing_end(p, STEP_FFT1);
  timing_begin(p, STEP_FFT2);
  launch_rows<real>(p, p->fft_tmp.p, G, image, n, 1, (int)n, 0, d, d);
  timing_end(p, STEP_FFT2);
}

void grid_to_image(ftcg_plan p, const void* grid, void* image) {
  if (p->dtype == FTCG_F64)
    grid_to_image_t<double>(p, grid, image);
  else
    grid_to_image_t<float>(p, grid, image);
}

// deapodization factors 1 / Phi(x_p / sigma), Phi(t) = sqrt(pi/beta) exp(-pi^2 t^2 / beta), float64
__global__ void k_deapod(double* d, int64_t n, double sigma, double beta) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double pi = 3.141592653589793238462643383279502884;
  const double t = ((double)p - (double)(n / 2)) / (double)n / sigma;
  d[p] = 1.0 / (sqrt(pi / beta) * exp(-pi * pi * t * t / beta));
}

void compute_deapod(ftcg_plan p) {
  hipLaunchKernelGGL(k_deapod, dim3((unsigned)((p->n + 255) / 256)), dim3(256), 0, p->stream,
                     p->deapod.as<double>(), p->n, p->sigma, p->beta);
  FTCG_HIP(hipGetLastError());
}

}  // namespace ftcg
