// ftcg_grid_to_image_noalloc: the inverse FFT, deapodization and crop of
// ftcg_grid_to_image without a plan and without any device allocation, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops). Its kernels are those of ftcg_grid_to_image; the workspace a plan
// would own (the n x G intermediate of the two FFT passes, the twiddle
// tables and the deapodization factors) lives in one static device array.
//
// The array is a host-side stand-in in host code: its device address is
// obtained once per device with hipGetSymbolAddress (with that device
// current) and only that address is passed to kernels. Every call on a GPU
// shares that GPU's array: calls that overlap on one GPU (other streams,
// other host threads) race. Nothing in it has to start at zero: every call
// writes the tables and the intermediate before reading them.
#include <math.h>

#include <mutex>

#include "ftcg_internal.h"

namespace {

constexpr size_t NOALLOC_BYTES = size_t(36) << 20;   // 36 MiB per device
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mu;
void* g_scratch_dev[MAX_DEVICES] = {};

// device address of this device's scratch array (looked up once per device)
void* scratch_ptr() {
  int dev = 0;
  FTCG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw ftcg::StatusError{FTCG_EUNSUPPORTED};
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    FTCG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" ftcg_status ftcg_grid_to_image_noalloc(int dim, int64_t n, int half_width, double oversampling,
                                                  ftcg_dtype dtype, const void* grid_dev, void* image_dev,
                                                  void* hip_stream) {
  using namespace ftcg;
  if (!grid_dev || !image_dev) return FTCG_EINVAL;
  if (dim != 1 && dim != 2) return FTCG_EINVAL;
  if (n < 8 || n > 8192 || (n & 1)) return FTCG_EINVAL;
  if (half_width < 2 || half_width > 8) return FTCG_EINVAL;
  if (!(oversampling >= 1.25 && oversampling <= 4.0)) return FTCG_EINVAL;
  if (dtype != FTCG_F32 && dtype != FTCG_F64) return FTCG_EINVAL;
  const double g = oversampling * (double)n;
  if (fabs(g - nearbyint(g)) > 1e-9) return FTCG_EINVAL;
  const int64_t G = (int64_t)nearbyint(g);
  if ((G % 4) != 0 || (G & (G - 1)) != 0) return FTCG_EUNSUPPORTED;
  if (G > (dtype == FTCG_F32 ? 16384 : 8192)) return FTCG_EUNSUPPORTED;
  if (2 * half_width > G) return FTCG_EINVAL;
  const bool f64 = dtype == FTCG_F64;
  const size_t csz = f64 ? 16 : 8;
  const size_t tmp_b = dim == 2 ? align256(csz * (size_t)(n * G)) : 0;
  const size_t tw_b = align256(csz * (size_t)twiddle_entries(G));
  const size_t dp_b = align256(sizeof(double) * (size_t)n);
  if (tmp_b + tw_b + dp_b > NOALLOC_BYTES) return FTCG_EUNSUPPORTED;   // beyond the static scratch
  try {
    unsigned char* base = static_cast<unsigned char*>(scratch_ptr());
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    void* tmp = dim == 2 ? base : nullptr;
    void* tw = base + tmp_b;
    double* dp = reinterpret_cast<double*>(base + tmp_b + tw_b);
    const double beta = M_PI * (oversampling - 0.5) / (oversampling * half_width);
    compute_twiddles(tw, G, f64, s);
    compute_deapod_raw(dp, n, oversampling, beta, s);
    grid_to_image_raw(dim, n, G, f64, s, tw, dp, tmp, grid_dev, image_dev);
    return FTCG_OK;
  } catch (const StatusError& e) {
    return e.status;
  } catch (const HipError&) {
    (void)hipGetLastError();
    return FTCG_EHIP;
  } catch (...) {
    return FTCG_EHIP;
  }
}
