// C ABI of the learned-weight network: lifecycle, parameters, serialisation,
// features, inference, training.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "mlp_internal.h"

using namespace ftcg;

namespace {

template <class F>
ftcg_status guard(F&& f) {
  try {
    f();
    return FTCG_OK;
  } catch (const StatusError& e) {
    return e.status;
  } catch (const HipError&) {
    (void)hipGetLastError();
    return FTCG_EHIP;
  } catch (const std::bad_alloc&) {
    return FTCG_ENOMEM;
  } catch (...) {
    return FTCG_EHIP;
  }
}

constexpr char MAGIC[8] = {'F', 'T', 'C', 'G', 'M', 'L', 'P', '1'};
constexpr uint32_t BLOB_VERSION = 1;
constexpr size_t BLOB_HEADER = 8 + 4 + 4 + 8 + 3 * 4;
constexpr size_t BLOB_BYTES = BLOB_HEADER + 3 * sizeof(float) * MLP_NPARAM;

// internal plan computing plain weights (and neighbour bins) of a raster
void ensure_label_plan(ftcg_mlp m, double R) {
  if (m->labels && m->labels->R == R) return;
  if (m->labels) {
    ftcg_plan_destroy(m->labels);
    m->labels = nullptr;
  }
  const int64_t n[2] = {256, 256};
  ftcg_plan p = nullptr;
  ftcg_status st = ftcg_plan_create(&p, 2, n, 6, 2.0, FTCG_F32, FTCG_W_PLAIN, R, m->stream);
  if (st != FTCG_OK) throw StatusError{st};
  p->weights_only = true;
  m->labels = p;
}

void raster_features(ftcg_mlp m, int64_t n, const double* k, double R, float* feat, double* base, float* target) {
  ensure_label_plan(m, R);
  ftcg_status st = ftcg_set_points(m->labels, n, k);
  if (st != FTCG_OK) throw StatusError{st};
  launch_knn_features(m->labels, k, feat, base, target ? m->labels->alpha.as<double>() : nullptr, target);
}

}  // namespace

extern "C" {

ftcg_status ftcg_mlp_create(ftcg_mlp* out, void* hip_stream) {
  if (!out) return FTCG_EINVAL;
  *out = nullptr;
  ftcg_mlp m = new (std::nothrow) ftcg_mlp_s();
  if (!m) return FTCG_ENOMEM;
  m->stream = static_cast<hipStream_t>(hip_stream);
  ftcg_status st = guard([&] {
    m->params.ensure(sizeof(float) * MLP_NPARAM);
    m->params16.ensure(sizeof(uint16_t) * MLP_NPARAM);
    m->adam_m.ensure(sizeof(float) * MLP_NPARAM);
    m->adam_v.ensure(sizeof(float) * MLP_NPARAM);
    m->grad.ensure(sizeof(float) * MLP_NPARAM);
    m->loss_dev.ensure(sizeof(float) * 1024);
    FTCG_HIP(hipMemsetAsync(m->params.p, 0, sizeof(float) * MLP_NPARAM, m->stream));
    FTCG_HIP(hipMemsetAsync(m->params16.p, 0, sizeof(uint16_t) * MLP_NPARAM, m->stream));
    FTCG_HIP(hipMemsetAsync(m->adam_m.p, 0, sizeof(float) * MLP_NPARAM, m->stream));
    FTCG_HIP(hipMemsetAsync(m->adam_v.p, 0, sizeof(float) * MLP_NPARAM, m->stream));
    if (hipHostMalloc((void**)&m->host, sizeof(float) * 1024, hipHostMallocDefault) != hipSuccess) {
      m->host = nullptr;
      throw StatusError{FTCG_ENOMEM};
    }
  });
  if (st != FTCG_OK) {
    ftcg_mlp_destroy(m);
    return st;
  }
  *out = m;
  return FTCG_OK;
}

ftcg_status ftcg_mlp_destroy(ftcg_mlp m) {
  if (!m) return FTCG_EINVAL;
  (void)hipStreamSynchronize(m->stream);
  if (m->labels) ftcg_plan_destroy(m->labels);
  DevBuf* bufs[] = {&m->params, &m->params16, &m->adam_m, &m->adam_v, &m->grad, &m->partial,
                    &m->loss_dev, &m->feat, &m->base, &m->target};
  for (DevBuf* b : bufs) b->release();
  if (m->host) (void)hipHostFree(m->host);
  delete m;
  return FTCG_OK;
}

ftcg_status ftcg_mlp_set_params(ftcg_mlp m, const float* params_host, int64_t n) {
  if (!m || !params_host) return FTCG_EINVAL;
  if (n != MLP_NPARAM) return FTCG_EINVAL;
  return guard([&] {
    FTCG_HIP(hipMemcpyAsync(m->params.p, params_host, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice,
                            m->stream));
    FTCG_HIP(hipMemsetAsync(m->adam_m.p, 0, sizeof(float) * MLP_NPARAM, m->stream));
    FTCG_HIP(hipMemsetAsync(m->adam_v.p, 0, sizeof(float) * MLP_NPARAM, m->stream));
    m->step = 0;
    launch_params_to_half(m);
    FTCG_HIP(hipStreamSynchronize(m->stream));
  });
}

ftcg_status ftcg_mlp_get_params(ftcg_mlp m, float* params_host, int64_t n) {
  if (!m || !params_host) return FTCG_EINVAL;
  if (n != MLP_NPARAM) return FTCG_EINVAL;
  return guard([&] {
    FTCG_HIP(hipMemcpyAsync(params_host, m->params.p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost,
                            m->stream));
    FTCG_HIP(hipStreamSynchronize(m->stream));
  });
}

ftcg_status ftcg_mlp_save(ftcg_mlp m, void* blob, size_t* bytes) {
  if (!m || !bytes) return FTCG_EINVAL;
  if (!blob) {
    *bytes = BLOB_BYTES;
    return FTCG_OK;
  }
  if (*bytes < BLOB_BYTES) return FTCG_EINVAL;
  return guard([&] {
    unsigned char* b = static_cast<unsigned char*>(blob);
    memcpy(b, MAGIC, 8);
    const uint32_t ver = BLOB_VERSION, np = MLP_NPARAM;
    const int64_t step = m->step;
    memcpy(b + 8, &ver, 4);
    memcpy(b + 12, &np, 4);
    memcpy(b + 16, &step, 8);
    memcpy(b + 24, &m->beta1, 4);
    memcpy(b + 28, &m->beta2, 4);
    memcpy(b + 32, &m->eps, 4);
    float* f = reinterpret_cast<float*>(b + BLOB_HEADER);
    FTCG_HIP(hipMemcpyAsync(f, m->params.p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, m->stream));
    FTCG_HIP(hipMemcpyAsync(f + MLP_NPARAM, m->adam_m.p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost,
                            m->stream));
    FTCG_HIP(hipMemcpyAsync(f + 2 * MLP_NPARAM, m->adam_v.p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost,
                            m->stream));
    FTCG_HIP(hipStreamSynchronize(m->stream));
    *bytes = BLOB_BYTES;
  });
}

ftcg_status ftcg_mlp_load(ftcg_mlp m, const void* blob, size_t bytes) {
  if (!m || !blob) return FTCG_EINVAL;
  if (bytes != BLOB_BYTES) return FTCG_EINVAL;
  const unsigned char* b = static_cast<const unsigned char*>(blob);
  uint32_t ver, np;
  memcpy(&ver, b + 8, 4);
  memcpy(&np, b + 12, 4);
  if (memcmp(b, MAGIC, 8) != 0 || ver != BLOB_VERSION || np != (uint32_t)MLP_NPARAM) return FTCG_EINVAL;
  return guard([&] {
    int64_t step;
    memcpy(&step, b + 16, 8);
    memcpy(&m->beta1, b + 24, 4);
    memcpy(&m->beta2, b + 28, 4);
    memcpy(&m->eps, b + 32, 4);
    m->step = step;
    const float* f = reinterpret_cast<const float*>(b + BLOB_HEADER);
    std::vector<float> tmp(f, f + 3 * MLP_NPARAM);  // the blob may be unaligned
    FTCG_HIP(hipMemcpyAsync(m->params.p, tmp.data(), sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice,
                            m->stream));
    FTCG_HIP(hipMemcpyAsync(m->adam_m.p, tmp.data() + MLP_NPARAM, sizeof(float) * MLP_NPARAM,
                            hipMemcpyHostToDevice, m->stream));
    FTCG_HIP(hipMemcpyAsync(m->adam_v.p, tmp.data() + 2 * MLP_NPARAM, sizeof(float) * MLP_NPARAM,
                            hipMemcpyHostToDevice, m->stream));
    launch_params_to_half(m);
    FTCG_HIP(hipStreamSynchronize(m->stream));
  });
}

ftcg_status ftcg_mlp_features(ftcg_mlp m, int64_t n, const double* k, double R, float* feat, double* base,
                              float* target) {
  if (!m || !k || !feat || !base) return FTCG_EINVAL;
  if (n < 1 || n >= (int64_t(1) << 31)) return FTCG_EINVAL;
  if (!(R > 0.0 && R <= 64.0)) return FTCG_EINVAL;
  return guard([&] { raster_features(m, n, k, R, feat, base, target); });
}

ftcg_status ftcg_mlp_forward(ftcg_mlp m, int64_t n, const float* feat, float* y) {
  if (!m || !feat || !y) return FTCG_EINVAL;
  if (n < 1) return FTCG_EINVAL;
  return guard([&] { launch_mlp_forward(m, feat, n, y); });
}

ftcg_status ftcg_mlp_loss_grad(ftcg_mlp m, int64_t n, const float* feat, const float* target, int fp16,
                               float* grad, double* loss_host) {
  if (!m || !feat || !target || !grad) return FTCG_EINVAL;
  if (n < 1 || n >= (int64_t(1) << 31)) return FTCG_EINVAL;
  return guard([&] {
    m->loss_slot = 0;
    launch_mlp_grad(m, feat, target, n, 0, 1, n, fp16 ? 1 : 0, 0, 0.f, grad);
    if (loss_host) {
      FTCG_HIP(hipMemcpyAsync(m->host, m->loss_dev.p, sizeof(float), hipMemcpyDeviceToHost, m->stream));
      FTCG_HIP(hipStreamSynchronize(m->stream));
      *loss_host = (double)m->host[0] / (double)n;
    }
  });
}

ftcg_status ftcg_mlp_train_batch(ftcg_mlp m, int64_t n, const float* feat, const float* target, int fp16,
                                 float lr, double* loss_host) {
  if (!m || !feat || !target) return FTCG_EINVAL;
  if (n < 1 || n >= (int64_t(1) << 31) || !(lr >= 0.f)) return FTCG_EINVAL;
  return guard([&] {
    m->loss_slot = 0;
    launch_mlp_grad(m, feat, target, n, 0, 1, n, fp16 ? 1 : 0, 1, lr, nullptr);
    if (loss_host) {
      FTCG_HIP(hipMemcpyAsync(m->host, m->loss_dev.p, sizeof(float), hipMemcpyDeviceToHost, m->stream));
      FTCG_HIP(hipStreamSynchronize(m->stream));
      *loss_host = (double)m->host[0] / (double)n;
    }
  });
}

ftcg_status ftcg_mlp_train_raster(ftcg_mlp m, int64_t n, const double* k, double R, int64_t batch, float lr,
                                  int fp16, double* loss_host) {
  if (!m || !k) return FTCG_EINVAL;
  if (n < 1 || n >= (int64_t(1) << 31) || batch < 1 || !(lr >= 0.f)) return FTCG_EINVAL;
  if (!(R > 0.0 && R <= 64.0)) return FTCG_EINVAL;
  return guard([&] {
    m->feat.ensure(sizeof(float) * 32 * n);
    m->base.ensure(sizeof(double) * n);
    m->target.ensure(sizeof(float) * n);
    raster_features(m, n, k, R, m->feat.as<float>(), m->base.as<double>(), m->target.as<float>());
    const int64_t nmb = (n + batch - 1) / batch;
    if (nmb > 1024) throw StatusError{FTCG_EINVAL};
    for (int64_t mb = 0; mb < nmb; ++mb) {
      const int64_t rows = (n - mb + nmb - 1) / nmb;   // samples j = mb + nmb * s < n
      m->loss_slot = (int)mb;
      launch_mlp_grad(m, m->feat.as<float>(), m->target.as<float>(), n, mb, nmb, rows, fp16 ? 1 : 0, 1, lr,
                      nullptr);
    }
    if (loss_host) {
      FTCG_HIP(hipMemcpyAsync(m->host, m->loss_dev.p, sizeof(float) * nmb, hipMemcpyDeviceToHost, m->stream));
      FTCG_HIP(hipStreamSynchronize(m->stream));
      double s = 0.0;
      for (int64_t i = 0; i < nmb; ++i) s += m->host[i];
      *loss_host = s / (double)n;
    }
  });
}

}  // extern "C"
