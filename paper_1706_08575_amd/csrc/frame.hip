// Dense frame approximation A_fr (Sec. III-B eq:binv, eq:afr, eq:afrm; 2D
// Sec. IV eq:twodframe, eq:twodframeB), the accuracy reference that the
// banded FTCG approximates, for small rasters.
//
//   zeta_n(x) = exp(2 pi i n . x) / w(x), modes n_a in -N/2 .. N/2 - 1 (the
//               admissible frame of eq:newadm on the pixel frequencies),
//               w(x) = Phi(x / sigma) per axis (the window the path divides by);
//   Psi_{j,n} = <phi_j, zeta_n> = prod_a g(k_ja - n_a),
//               g(t) = int_{-1/2}^{1/2} cos(2 pi t x) / w(x) dx;
//   beta      = Psi^dagger fhat (least squares when the samples are at
//               least as many as the modes, minimum norm otherwise);
//   A_fr(x_p) = sum_n beta_n exp(2 pi i n . x_p) / w(x_p).
//
// Steps, all float64:
//   1. k_gl_nodes: Gauss-Legendre nodes and weights of order Q = 4N + 64 on
//      [-1/2, 1/2] (Newton's method on P_Q from the three-term recurrence,
//      one thread per node), the weights divided by w at the nodes;
//   2. k_frame_axis: the per-axis tables g(k_ja - n_a) (one thread per entry);
//   3. k_frame_assemble: the tall matrix of the QR: Psi with the real and
//      imaginary parts of fhat as two extra columns (m >= N^d), or Psi^T
//      (m < N^d), column-major;
//   4. Householder QR, one column at a time: k_house forms the unit
//      reflector of column j in place (R_jj apart), k_reflect applies it to
//      every later column (one workgroup per column);
//   5. k_backsub (least squares: R beta = Q^T fhat) or k_minnorm (R^T y =
//      fhat, beta = Q [y; 0]), one workgroup;
//   6. the inverse DFT of beta on the N^d mode grid and the division by w:
//      the grid-to-image passes with G = N (no crop).
#include "ftcg_internal.h"

namespace ftcg {

constexpr int FR_BLOCK = 256;

// node i of Gauss-Legendre order Q (x in (-1, 1), weight), mapped to
// [-1/2, 1/2]; the weight is divided by w(x) = sqrt(pi / beta) e^{-pi^2 (x / sigma)^2 / beta}
__global__ void k_gl_nodes(int Q, double sigma, double beta, double* __restrict__ xq, double* __restrict__ cw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Q) return;
  double x = cos(WPI * (i + 0.75) / (Q + 0.5));   // initial guess near the i-th root
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = x;
    for (int j = 2; j <= Q; ++j) {
      const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = Q * (x * p1 - p0) / (x * x - 1.0);       // P_Q'(x)
    const double dx = p1 / dp;
    x -= dx;
    if (fabs(dx) < 1e-16) break;
  }
  {
    double p0 = 1.0, p1 = x;
    for (int j = 2; j <= Q; ++j) {
      const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = Q * (x * p1 - p0) / (x * x - 1.0);
  }
  const double wgt = 2.0 / ((1.0 - x * x) * dp * dp);
  const double xh = 0.5 * x;
  const double t = xh / sigma;
  const double w = sqrt(WPI / beta) * exp(-WPI * WPI * t * t / beta);
  xq[i] = xh;
  cw[i] = 0.5 * wgt / w;
}

// G[a][j][i] = g(k_ja - (i - N/2)), a < dim
__global__ void k_frame_axis(const double* __restrict__ k, int64_t m, int dim, int N, int Q,
                             const double* __restrict__ xq, const double* __restrict__ cw, double* __restrict__ G) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)dim * m * N) return;
  const int i = (int)(t % N);
  const int64_t j = (t / N) % m;
  const int a = (int)(t / ((int64_t)N * m));
  const double d = k[j * dim + a] - (double)(i - N / 2);
  double s = 0.0;
  for (int q = 0; q < Q; ++q) s += cw[q] * cospi(2.0 * d * xq[q]);
  G[t] = s;
}

// over (m >= NM): A (m x (NM + 2)) = [Psi | Re fhat | Im fhat]; else A (NM x m) = Psi^T
__global__ void k_frame_assemble(const double* __restrict__ G, const double2* __restrict__ fhat, int64_t m, int dim,
                                 int N, int64_t NM, int over, double* __restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * NM) return;
  const int64_t j = t / NM, col = t % NM;
  double v;
  if (dim == 1) {
    v = G[j * N + col];
  } else {
    const int n0 = (int)(col / N), n1 = (int)(col % N);
    v = G[j * N + n0] * G[(m + j) * N + n1];
  }
  if (over) {
    A[col * m + j] = v;
    if (col == 0) {
      A[NM * m + j] = fhat[j].x;
      A[(NM + 1) * m + j] = fhat[j].y;
    }
  } else {
    A[j * NM + col] = v;
  }
}

__global__ void k_set_int(int* __restrict__ p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)blockDim.x / 64; ++i) s += red[i];
  return s;
}

// unit Householder vector of column j (rows j..r-1) in place, R_jj to diag[j]
__global__ __launch_bounds__(FR_BLOCK) void k_house(double* __restrict__ A, int64_t r, int j,
                                                    double* __restrict__ diag) {
  __shared__ double red[FR_BLOCK / 64];
  double* col = A + (int64_t)j * r;
  double s2 = 0.0;
  for (int64_t i = j + 1 + threadIdx.x; i < r; i += FR_BLOCK) s2 += col[i] * col[i];
  s2 = block_sum(s2, red);
  const double alpha = col[j];
  const double nrm = sqrt(alpha * alpha + s2);
  if (nrm == 0.0) {
    if (threadIdx.x == 0) diag[j] = 0.0;
    return;   // a zero column: the reflector stays 0 (identity); the solve reports it
  }
  const double rjj = alpha >= 0.0 ? -nrm : nrm;
  const double v0 = alpha - rjj;                  // |v0| = |alpha| + nrm: no cancellation
  const double inv = 1.0 / sqrt(v0 * v0 + s2);
  __syncthreads();
  for (int64_t i = j + 1 + threadIdx.x; i < r; i += FR_BLOCK) col[i] *= inv;
  if (threadIdx.x == 0) {
    col[j] = v0 * inv;
    diag[j] = rjj;
  }
}

// columns jc = j + 1 + block: A[j:, jc] -= 2 (v . A[j:, jc]) v
__global__ __launch_bounds__(FR_BLOCK) void k_reflect(double* __restrict__ A, int64_t r, int j) {
  __shared__ double red[FR_BLOCK / 64];
  const double* v = A + (int64_t)j * r;
  double* c = A + (int64_t)(j + 1 + blockIdx.x) * r;
  double s = 0.0;
  for (int64_t i = j + threadIdx.x; i < r; i += FR_BLOCK) s += v[i] * c[i];
  s = 2.0 * block_sum(s, red);
  for (int64_t i = j + threadIdx.x; i < r; i += FR_BLOCK) c[i] -= s * v[i];
}

__device__ inline bool tiny_pivot(const double* diag, int c, int i, double* red) {
  // |R_ii| against the largest |R_kk| (the rank test of the solve)
  double mx = 0.0;
  for (int k = threadIdx.x; k < c; k += FR_BLOCK) mx = fmax(mx, fabs(diag[k]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = 0.0;
  for (int w = 0; w < FR_BLOCK / 64; ++w) mx = fmax(mx, red[w]);
  return !(fabs(diag[i]) > 1e-14 * mx);
}

// least squares: R beta = (Q^T fhat)[0:c] (the two right-hand-side columns)
__global__ __launch_bounds__(FR_BLOCK) void k_backsub(const double* __restrict__ A, int64_t r, int c,
                                                      const double* __restrict__ diag, double2* __restrict__ beta,
                                                      int* __restrict__ bad) {
  __shared__ double red[FR_BLOCK / 64];
  __shared__ double red2[FR_BLOCK / 64];
  const double* yr = A + (int64_t)c * r;
  const double* yi = A + (int64_t)(c + 1) * r;
  for (int i = c - 1; i >= 0; --i) {
    if (tiny_pivot(diag, c, i, red)) {
      if (threadIdx.x == 0) *bad = 1;
      return;
    }
    double sr = 0.0, si = 0.0;
    for (int k = i + 1 + threadIdx.x; k < c; k += FR_BLOCK) {
      const double rik = A[(int64_t)k * r + i];
      sr += rik * beta[k].x;
      si += rik * beta[k].y;
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red2);
    if (threadIdx.x == 0) {
      double2 b;
      b.x = (yr[i] - sr) / diag[i];
      b.y = (yi[i] - si) / diag[i];
      beta[i] = b;
    }
    __syncthreads();
  }
}

// minimum norm (A = Psi^T, r = modes, c = samples): R^T y = fhat, beta = Q [y; 0]
__global__ __launch_bounds__(FR_BLOCK) void k_minnorm(const double* __restrict__ A, int64_t r, int c,
                                                      const double* __restrict__ diag,
                                                      const double2* __restrict__ fhat, double2* __restrict__ beta,
                                                      int* __restrict__ bad) {
  __shared__ double red[FR_BLOCK / 64];
  __shared__ double red2[FR_BLOCK / 64];
  for (int64_t i = threadIdx.x; i < r; i += FR_BLOCK) beta[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int i = 0; i < c; ++i) {
    if (tiny_pivot(diag, c, i, red)) {
      if (threadIdx.x == 0) *bad = 1;
      return;
    }
    double sr = 0.0, si = 0.0;
    for (int k = threadIdx.x; k < i; k += FR_BLOCK) {
      const double rki = A[(int64_t)i * r + k];
      sr += rki * beta[k].x;
      si += rki * beta[k].y;
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red2);
    if (threadIdx.x == 0) beta[i] = make_double2((fhat[i].x - sr) / diag[i], (fhat[i].y - si) / diag[i]);
    __syncthreads();
  }
  for (int j = c - 1; j >= 0; --j) {   // beta <- H_j beta, H_j = I - 2 v v^T on rows j..r-1
    const double* v = A + (int64_t)j * r;
    double sr = 0.0, si = 0.0;
    for (int64_t i = j + threadIdx.x; i < r; i += FR_BLOCK) {
      sr += v[i] * beta[i].x;
      si += v[i] * beta[i].y;
    }
    sr = 2.0 * block_sum(sr, red);
    si = 2.0 * block_sum(si, red2);
    for (int64_t i = j + threadIdx.x; i < r; i += FR_BLOCK) {
      double2 b = beta[i];
      b.x -= sr * v[i];
      b.y -= si * v[i];
      beta[i] = b;
    }
    __syncthreads();
  }
}

void frame_approx(ftcg_plan p, int64_t m, const double* k, const void* fhat, void* image) {
  const int dim = p->dim;
  const int N = (int)p->n;
  int64_t NM = N;
  for (int a = 1; a < dim; ++a) NM *= N;
  const bool over = m >= NM;
  const int64_t r = over ? m : NM, c = over ? NM : m;
  const int64_t cols = over ? c + 2 : c;
  hipStream_t s = p->stream;
  const int Q = 4 * N + 64;
  p->fa_gl.ensure(sizeof(double) * 2 * Q);
  p->fa_G.ensure(sizeof(double) * (size_t)dim * m * N);
  p->fa_A.ensure(sizeof(double) * (size_t)(r * cols));
  p->fa_diag.ensure(sizeof(double) * (size_t)c);
  p->fa_beta.ensure(sizeof(double2) * (size_t)NM);
  p->fa_tw.ensure(sizeof(double2) * (size_t)twiddle_entries(N));
  p->fa_tmp.ensure(sizeof(double2) * (size_t)NM);
  double* xq = p->fa_gl.as<double>();
  double* cw = xq + Q;
  int* bad = reinterpret_cast<int*>(p->flags.as<double>() + 10);
  timing_begin(p, STEP_FRAME);
  hipLaunchKernelGGL(k_gl_nodes, dim3((Q + 63) / 64), dim3(64), 0, s, Q, p->sigma, p->beta, xq, cw);
  const int64_t ng = (int64_t)dim * m * N;
  hipLaunchKernelGGL(k_frame_axis, dim3((unsigned)((ng + FR_BLOCK - 1) / FR_BLOCK)), dim3(FR_BLOCK), 0, s, k, m, dim,
                     N, Q, xq, cw, p->fa_G.as<double>());
  hipLaunchKernelGGL(k_frame_assemble, dim3((unsigned)((m * NM + FR_BLOCK - 1) / FR_BLOCK)), dim3(FR_BLOCK), 0, s,
                     p->fa_G.as<double>(), static_cast<const double2*>(fhat), m, dim, N, NM, over ? 1 : 0,
                     p->fa_A.as<double>());
  double* A = p->fa_A.as<double>();
  for (int j = 0; j < c; ++j) {
    hipLaunchKernelGGL(k_house, dim3(1), dim3(FR_BLOCK), 0, s, A, r, j, p->fa_diag.as<double>());
    if (cols - j - 1 > 0)
      hipLaunchKernelGGL(k_reflect, dim3((unsigned)(cols - j - 1)), dim3(FR_BLOCK), 0, s, A, r, j);
  }
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, bad, 0);
  if (over)
    hipLaunchKernelGGL(k_backsub, dim3(1), dim3(FR_BLOCK), 0, s, A, r, (int)c, p->fa_diag.as<double>(),
                       p->fa_beta.as<double2>(), bad);
  else
    hipLaunchKernelGGL(k_minnorm, dim3(1), dim3(FR_BLOCK), 0, s, A, r, (int)c, p->fa_diag.as<double>(),
                       static_cast<const double2*>(fhat), p->fa_beta.as<double2>(), bad);
  FTCG_HIP(hipGetLastError());
  // A_fr at the pixels: inverse DFT of beta on the N^dim mode grid (G = N),
  // divided by w(x_p) = Phi(x_p / sigma) (the plan's deapodization factors)
  compute_twiddles(p->fa_tw.p, N, true, s);
  grid_to_image_raw(dim, N, N, true, s, p->fa_tw.p, p->deapod.as<double>(), p->fa_tmp.p, p->fa_beta.p, image);
  timing_end(p, STEP_FRAME);
  int* hb = reinterpret_cast<int*>(p->host_flags + 10);
  FTCG_HIP(hipMemcpyAsync(hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  FTCG_HIP(hipStreamSynchronize(s));
  if (*hb) throw StatusError{FTCG_EINVAL};
}

}  // namespace ftcg
