// Iterative density compensation (the iterative quadrature weights the paper
// cites in Sec. III-A), a comparator to the frame-theoretic weights of
// eq:difopt: starting from w = 1, each iteration spreads the weights onto the
// oversampled grid with the path's own kernel, interpolates the grid back at
// the samples with the same taps (d = Omega^T Omega w) and sets w <- w / d.
// The plan's spreading and interpolation kernels do the two products; the
// weights live in float64 (the plan's alpha) and reach the spread as the
// values (w, 0) in the plan's precision. The result is scaled by
// (pi / (sigma beta))^dim, at which a uniform lattice of spacing h gets h^dim,
// as the frame weights do.
#include "ftcg_internal.h"

namespace ftcg {

constexpr int DEN_BLOCK = 256;

template <class cx>
__global__ __launch_bounds__(DEN_BLOCK) void k_den_init(double* __restrict__ w, cx* __restrict__ val, int64_t m) {
  const int64_t j = (int64_t)blockIdx.x * DEN_BLOCK + threadIdx.x;
  if (j >= m) return;
  w[j] = 1.0;
  cx v;
  v.x = 1;
  v.y = 0;
  val[j] = v;
}

// w <- w / Re(d); the next iteration's values, or (last) the scaled weights
template <class cx>
__global__ __launch_bounds__(DEN_BLOCK) void k_den_update(double* __restrict__ w, const cx* __restrict__ den,
                                                         cx* __restrict__ val, int64_t m, double scale, int last) {
  const int64_t j = (int64_t)blockIdx.x * DEN_BLOCK + threadIdx.x;
  if (j >= m) return;
  const double x = w[j] / (double)den[j].x;
  if (last) {
    w[j] = x * scale;
  } else {
    w[j] = x;
    cx v;
    v.x = (decltype(v.x))x;
    v.y = 0;
    val[j] = v;
  }
}

template <class cx>
static void run_density_t(ftcg_plan p) {
  const int64_t m = p->m;
  const unsigned gb = (unsigned)((m + DEN_BLOCK - 1) / DEN_BLOCK);
  double* w = p->alpha.as<double>();
  cx* val = p->den_val.as<cx>();
  cx* den = p->den_d.as<cx>();
  double scale = 1.0;
  for (int a = 0; a < p->dim; ++a) scale *= WPI / (p->sigma * p->beta);
  hipLaunchKernelGGL(k_den_init<cx>, dim3(gb), dim3(DEN_BLOCK), 0, p->stream, w, val, m);
  for (int it = 0; it < p->den_iters; ++it) {
    spread(p, val, p->grid.p);
    interpolate_grid(p, den);
    hipLaunchKernelGGL(k_den_update<cx>, dim3(gb), dim3(DEN_BLOCK), 0, p->stream, w, den, val, m, scale,
                       it + 1 == p->den_iters ? 1 : 0);
  }
  FTCG_HIP(hipGetLastError());
}

void run_density_weights(ftcg_plan p) {
  const size_t csz = p->dtype == FTCG_F64 ? 16 : 8;
  p->den_val.ensure(csz * (size_t)p->m);
  p->den_d.ensure(csz * (size_t)p->m);
  timing_begin(p, STEP_DENSITY);
  if (p->dtype == FTCG_F64)
    run_density_t<double2>(p);
  else
    run_density_t<float2>(p);
  timing_end(p, STEP_DENSITY);
}

}  // namespace ftcg
