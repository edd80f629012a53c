// C ABI of libftcg: plan lifecycle, argument checking, step sequencing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "ftcg_internal.h"
#include "wbins.h"
#include "mlp_internal.h"

namespace ftcg {

static hipEvent_t take_event(Timing& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  FTCG_HIP(hipEventCreate(&e));
  return e;
}

void timing_begin(ftcg_plan p, int step) {
  Timing& t = p->timing;
  if (!t.enabled) return;
  t.open_ev = take_event(t);
  t.open_step = step;
  FTCG_HIP(hipEventRecord(t.open_ev, p->stream));
}

void timing_end(ftcg_plan p, int step) {
  Timing& t = p->timing;
  if (!t.enabled || t.open_step != step) return;
  hipEvent_t e = take_event(t);
  FTCG_HIP(hipEventRecord(e, p->stream));
  t.pending.push_back({step, t.open_ev, e});
  t.open_step = -1;
  t.open_ev = nullptr;
}


static bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

// 2D: tile 32. Measured whole steps (binning + spread) on SAS rasters, tile
// 64 / 32 / 16: 2^17 samples at 512^2 0.183 / 0.158 / 0.238 ms, 2^20 at
// 1024^2 0.905 / 0.840 / 0.859 ms, 2^23 at 4096^2 4.75 / 4.57 / 5.26 ms: the
// extra records of the smaller tile (footprints cut by more tile edges) cost
// less than the larger LDS tile's lower occupancy saves.
static int auto_tile(ftcg_plan p) {
  if (p->dim == 1) return (int)(p->G < 1024 ? p->G : 1024);
  return (int)(p->G < 32 ? p->G : 32);
}

static void setup_tiles(ftcg_plan p) {
  int t = p->tile_req ? p->tile_req : auto_tile(p);
  if (t > p->G) t = (int)p->G;
  p->tile = t;
  p->nt = p->G / t;
  p->ntiles = p->dim == 1 ? p->nt : p->nt * p->nt;
}

}  // namespace ftcg

using namespace ftcg;

template <class F>
static ftcg_status guarded(F&& f) {
  try {
    f();
    return FTCG_OK;
  } catch (const StatusError& e) {
    return e.status;
  } catch (const HipError& e) {
    (void)hipGetLastError();
    return FTCG_EHIP;
  } catch (const std::bad_alloc&) {
    return FTCG_ENOMEM;
  } catch (...) {
    return FTCG_EHIP;
  }
}

namespace ftcg {
int64_t plan_nrec(ftcg_plan p) {
  if (p->nrec < 0) {
    FTCG_HIP(hipMemcpyAsync(p->host_flags, p->tile_off.as<int32_t>() + p->ntiles, sizeof(int32_t),
                            hipMemcpyDeviceToHost, p->stream));
    FTCG_HIP(hipStreamSynchronize(p->stream));
    p->nrec = *reinterpret_cast<const int32_t*>(p->host_flags);
  }
  return p->nrec;
}
}  // namespace ftcg

// learned weights, then their audit against the plain weights on a subset of
// samples (one host synchronisation to read its estimate) and the plain
// weights where it fails
static void run_learned_with_audit(ftcg_plan p, const double* k_dev) {
  timing_begin(p, STEP_LEARNED);
  launch_learned_weights(p, k_dev, p->mlp);
  timing_end(p, STEP_LEARNED);
  timing_begin(p, STEP_AUDIT);
  double* est_dev = p->flags.as<double>() + 6;
  launch_audit(p, k_dev, est_dev);
  FTCG_HIP(hipMemcpyAsync(p->host_flags + 6, est_dev, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  FTCG_HIP(hipStreamSynchronize(p->stream));
  timing_end(p, STEP_AUDIT);
  p->audit_estimate = p->host_flags[6];
  p->used_fallback = !(p->audit_estimate <= p->audit_threshold);
  if (p->used_fallback) run_plain_weights(p);
}

namespace ftcg {

// set_points in two parts, so that a batch can enqueue the input checks of
// all its items before the host waits for the first of them.
// set_points_begin enqueues the input check and the binning passes that need
// no host decision (its state is kept in p->pending);
void set_points_begin(ftcg_plan p, int64_t m, const double* k_dev) {
  p->have_points = false;
  p->have_weights = false;
  p->finish_recs = false;
  p->weights_deferred = false;
  p->m = m;
  // 1) input check: finiteness, bounding box and the neighbour-bin
  //    geometry, reduced on the device; the check also zeroes the tile and
  //    bin-row counters of the binning passes
  timing_begin(p, STEP_BIN);
  int32_t* zero_ptr = nullptr;
  int64_t zero_n = 0;
  if (!p->weights_only) {
    setup_tiles(p);
    p->tile_cnt.ensure(sizeof(int32_t) * (p->ntiles + 1));
    zero_ptr = p->tile_cnt.as<int32_t>();
    zero_n = p->ntiles + 1;
  }
  const bool band = p->wmode == FTCG_W_BAND;
  const bool rows2d = p->dim == 2 && (p->wmode == FTCG_W_PLAIN || p->wmode == FTCG_W_LEARNED || band);
  int32_t* zero_b = nullptr;
  int64_t zero_nb = 0;
  if (rows2d) {
    p->wb_cnt.ensure(sizeof(int32_t) * WROW_CNT_ZERO);
    zero_b = p->wb_cnt.as<int32_t>();
    zero_nb = WROW_CNT_ZERO;
  }
  auto* part = p->check_part.as<unsigned long long>();
  const int nparts = launch_check_points(p, k_dev, m, part, zero_ptr, zero_n, zero_b, zero_nb);
  const int seq = ++p->check_seq;
  p->pending.seq = seq;
  launch_check_reduce(p, part, nparts, seq);
  timing_end(p, STEP_BIN);
  FTCG_HIP(hipEventRecord(p->ev_check, p->stream));
  // 2) binning passes that need no host decision are enqueued before the
  //    host waits for the check, and run during the host's turn (their
  //    kernels keep every index in range for any input; rejected points
  //    are reported below):
  //    - 2D weights, tile counters in LDS: tile records and bin rows fused;
  //    - otherwise the tile binning: whole when its counters fit LDS, else
  //      the counting + scan (the tile scatter writes the weights with the
  //      records later; there these passes outlast the host's turn, and
  //      the bin rows follow it).
  //    Records written here get their weights once those are known.
  const bool tiles = !p->weights_only;
  // 2D weights bin their rows with the tiles at any tile count; otherwise the
  // tile scatter runs early only when its counters fit LDS
  const bool early_scatter = tiles && (tile_keys_in_lds(p) || rows2d);
  const bool fused = rows2d && early_scatter;
  const int64_t cap = m << p->dim;  // worst case 2^dim tile records per sample
  if (tiles) {
    p->recs.ensure((p->dtype == FTCG_F64 ? sizeof(Rec<double>) : sizeof(Rec<float>)) * cap);
    p->alpha_s.ensure((p->dtype == FTCG_F64 ? sizeof(double) : sizeof(float)) * cap);
    p->tile_off.ensure(sizeof(int32_t) * (p->ntiles + 1));
    p->tile_scan_tmp.ensure(scan_tmp_bytes(p->ntiles));
  }
  if (rows2d) {
    p->wb_rowoff.ensure(sizeof(int32_t) * (WROW_MAX + 1));
    p->wb_rowbuf.ensure(sizeof(RowRec) * m);
    p->scan_tmp.ensure(scan_tmp_bytes(WROW_MAX));
  }
  if (fused) {
    timing_begin(p, STEP_BIN);
    bin_points_fused(p, k_dev);
    timing_end(p, STEP_BIN);
  } else if (tiles) {
    timing_begin(p, STEP_BIN);
    if (early_scatter)
      bin_points_k(p, k_dev);   // weight 1 until the weights are known
    else
      bin_count_k(p, k_dev);
    timing_end(p, STEP_BIN);
  }
  p->pending.tiles = tiles;
  p->pending.early_scatter = early_scatter;
  p->pending.fused = fused;
  p->pending.band = band;
}

// set_points_end waits for the check (host), then enqueues the weights and the
// rest of the binning
void set_points_end(ftcg_plan p, const double* k_dev) {
  const int64_t m = p->m;
  const int seq = p->pending.seq;
  const bool tiles = p->pending.tiles, early_scatter = p->pending.early_scatter, fused = p->pending.fused;
  const bool band = p->pending.band;
  FTCG_HIP(hipEventSynchronize(p->ev_check));
  const CheckOut chk = *p->host_geo;
  if (chk.seq != seq) throw StatusError{FTCG_EHIP};   // the result of an earlier call: not visible yet
  if (chk.bad) throw StatusError{FTCG_EINVAL};
  p->wgeom = chk.g;
  // 3) weights (caller order)
  p->alpha.ensure(sizeof(double) * m);
  const bool computed = p->wmode == FTCG_W_PLAIN || p->wmode == FTCG_W_LEARNED;
  // records already written, 2D plain weights: the symmetric sum's finish
  // is deferred (the fixed-point spread forms the records' weights from the
  // sums through the caller-to-bin map the bin sort then writes;
  // finish_deferred_weights serves every other reader)
  const bool want_finish = early_scatter && p->dim == 2 && p->wmode == FTCG_W_PLAIN;
  if (computed || band) {
    if (p->wmode == FTCG_W_LEARNED && !p->mlp) throw StatusError{FTCG_ESTATE};
    p->finish_recs = want_finish;
    if (p->dim == 2) {
      setup_weight_bins(p);
      timing_begin(p, STEP_WBIN);
      if (!fused) wrow_bin(p, k_dev, p->wgeom.nb[0]);
      sort_weight_rows(p);
      timing_end(p, STEP_WBIN);
      p->have_wbins = true;
    } else {
      build_weight_bins_1d(p, k_dev);
    }
    if (p->wmode == FTCG_W_PLAIN) {
      run_plain_weights(p);
    } else if (band) {
      // the records carry weight 1; C is applied to the values before the
      // spread (execute)
      fill_ones(p->alpha.as<double>(), m, p->stream);
      run_band_weights(p);
    } else {
      run_learned_with_audit(p, k_dev);
    }
    p->have_weights = true;
  } else if (p->wmode == FTCG_W_NONE) {
    fill_ones(p->alpha.as<double>(), m, p->stream);
    p->have_weights = true;
  }
  // 4) the records' weights
  if (tiles) {
    const bool finished = want_finish && !p->finish_recs;
    if (!early_scatter) {
      timing_begin(p, STEP_BIN);
      bin_scatter_k(p, k_dev);   // with the weights when there are any
      timing_end(p, STEP_BIN);
    } else if ((computed || band) && !finished) {
      timing_begin(p, STEP_BIN);
      refill_alpha_dev(p);
      timing_end(p, STEP_BIN);
    }
  }
  // 5) iterative density compensation: spreads and interpolates through
  //    the records just written (weight 1), then gives them its weights
  if (p->wmode == FTCG_W_DENSITY) {
    if (!tiles) throw StatusError{FTCG_EUNSUPPORTED};
    run_density_weights(p);
    p->have_weights = true;
    timing_begin(p, STEP_BIN);
    refill_alpha_dev(p);
    timing_end(p, STEP_BIN);
  }
  p->finish_recs = false;
  p->nrec = -1;  // on the device (tile_off[ntiles]); read only when asked for
  p->have_points = true;
}

}  // namespace ftcg

extern "C" {

const char* ftcg_status_string(ftcg_status s) {
  switch (s) {
    case FTCG_OK: return "FTCG_OK";
    case FTCG_EINVAL: return "FTCG_EINVAL: invalid argument";
    case FTCG_ENOMEM: return "FTCG_ENOMEM: device allocation failed";
    case FTCG_EHIP: return "FTCG_EHIP: HIP runtime error";
    case FTCG_ESTATE: return "FTCG_ESTATE: call out of order";
    case FTCG_EUNSUPPORTED: return "FTCG_EUNSUPPORTED: not supported by this library";
  }
  return "FTCG_?: unknown status";
}

ftcg_status ftcg_plan_create(ftcg_plan* out, int dim, const int64_t* n, int half_width, double oversampling,
                             ftcg_dtype dtype, ftcg_wmode wmode, double weight_radius, void* hip_stream) {
  if (!out || !n) return FTCG_EINVAL;
  *out = nullptr;
  if (dim != 1 && dim != 2) return FTCG_EINVAL;
  const int64_t n0 = n[0];
  if (dim == 2 && n[1] != n0) return FTCG_EUNSUPPORTED;
  if (n0 < 8 || n0 > 8192 || (n0 & 1)) return FTCG_EINVAL;
  if (half_width < 2 || half_width > 8) return FTCG_EINVAL;
  if (!(oversampling >= 1.25 && oversampling <= 4.0)) return FTCG_EINVAL;
  if (dtype != FTCG_F32 && dtype != FTCG_F64) return FTCG_EINVAL;
  if (wmode < FTCG_W_PLAIN || wmode > FTCG_W_DENSITY) return FTCG_EINVAL;
  if (!(weight_radius > 0.0 && weight_radius <= 64.0)) return FTCG_EINVAL;
  const double g = oversampling * (double)n0;
  if (fabs(g - nearbyint(g)) > 1e-9) return FTCG_EINVAL;
  const int64_t G = (int64_t)nearbyint(g);
  if ((G % 4) != 0 || !is_pow2(G)) return FTCG_EUNSUPPORTED;
  if (G > (dtype == FTCG_F32 ? 16384 : 8192)) return FTCG_EUNSUPPORTED;
  if (2 * half_width > G) return FTCG_EINVAL;
  if (wmode == FTCG_W_LEARNED && dim != 2) return FTCG_EUNSUPPORTED;

  ftcg_plan p = new (std::nothrow) ftcg_plan_s();
  if (!p) return FTCG_ENOMEM;
  p->dim = dim;
  p->n = n0;
  p->W = half_width;
  p->sigma = oversampling;
  p->dtype = dtype;
  p->wmode = wmode;
  p->R = weight_radius;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->G = G;
  p->beta = M_PI * (oversampling - 0.5) / (oversampling * half_width);
  p->accum = dtype == FTCG_F32 ? ACCUM_FIXED : ACCUM_F64;
  ftcg_status st = guarded([&] {
    setup_tiles(p);
    p->flags.ensure(FLAGS_BYTES);
    p->deapod.ensure(sizeof(double) * n0);
    compute_deapod(p);
    p->twiddle.ensure((dtype == FTCG_F64 ? 16 : 8) * (size_t)twiddle_entries(G));
    compute_twiddles(p->twiddle.p, G, dtype == FTCG_F64, p->stream);
    const size_t csz = dtype == FTCG_F64 ? 16 : 8;
    p->grid.ensure(csz * (size_t)(dim == 2 ? G * G : G));
    if (dim == 2) p->fft_tmp.ensure(csz * (size_t)(n0 * G));
    if (hipHostMalloc((void**)&p->host_flags, FLAGS_BYTES, hipHostMallocDefault) != hipSuccess) {
      p->host_flags = nullptr;
      throw StatusError{FTCG_ENOMEM};
    }
    p->check_part.ensure(sizeof(unsigned long long) * 5 * CHECK_PARTS);
    p->geo.ensure(sizeof(CheckOut));
    if (hipHostMalloc((void**)&p->host_geo, sizeof(CheckOut), hipHostMallocCoherent) != hipSuccess) {
      p->host_geo = nullptr;
      throw StatusError{FTCG_ENOMEM};
    }
    FTCG_HIP(hipEventCreateWithFlags(&p->ev_check, hipEventDisableTiming));
  });
  if (st != FTCG_OK) {
    ftcg_plan_destroy(p);
    return st;
  }
  *out = p;
  return FTCG_OK;
}

ftcg_status ftcg_plan_destroy(ftcg_plan p) {
  if (!p) return FTCG_EINVAL;
  (void)hipStreamSynchronize(p->stream);
  DevBuf* bufs[] = {&p->fa_gl, &p->fa_G, &p->fa_A, &p->fa_diag, &p->fa_beta, &p->fa_tw, &p->fa_tmp, &p->den_val, &p->den_d, &p->band_P, &p->band_col, &p->band_row, &p->band_c, &p->alpha,  &p->recs,  &p->alpha_s, &p->tile_cnt, &p->tile_off, &p->scan_tmp, &p->tile_scan_tmp, &p->check_part, &p->geo,
                    &p->flags,  &p->wb_cnt, &p->wb_off, &p->wb_rowoff, &p->wb_rowbuf, &p->ws_k,   &p->ws_idx,   &p->wb_of, &p->ws_inv, &p->ws_sum, &p->audit_buf,
                    &p->grid,   &p->fft_tmp, &p->deapod, &p->twiddle, &p->tile_order};
  for (DevBuf* b : bufs) b->release();
  for (auto& pr : p->timing.pending) {
    (void)hipEventDestroy(pr.a);
    (void)hipEventDestroy(pr.b);
  }
  for (hipEvent_t e : p->timing.pool) (void)hipEventDestroy(e);
  if (p->timing.open_ev) (void)hipEventDestroy(p->timing.open_ev);
  if (p->host_flags) (void)hipHostFree(p->host_flags);
  if (p->host_geo) (void)hipHostFree(p->host_geo);
  if (p->ev_check) (void)hipEventDestroy(p->ev_check);
  delete p;
  return FTCG_OK;
}

ftcg_status ftcg_set_points(ftcg_plan p, int64_t m, const double* k_dev) {
  if (!p || !k_dev) return FTCG_EINVAL;
  if (m < 1 || m >= (int64_t(1) << 31)) return FTCG_EINVAL;
  return guarded([&] {
    set_points_begin(p, m, k_dev);
    set_points_end(p, k_dev);
  });
}

ftcg_status ftcg_set_weights(ftcg_plan p, const double* alpha_dev) {
  if (!p || !alpha_dev) return FTCG_EINVAL;
  if (p->wmode != FTCG_W_USER) return FTCG_ESTATE;
  if (!p->have_points) return FTCG_ESTATE;
  return guarded([&] {
    FTCG_HIP(hipMemcpyAsync(p->alpha.p, alpha_dev, sizeof(double) * p->m, hipMemcpyDeviceToDevice, p->stream));
    refill_alpha(p);
    p->have_weights = true;
  });
}

ftcg_status ftcg_get_weights(ftcg_plan p, double* alpha_dev, int* used_fallback_host) {
  if (!p || !alpha_dev) return FTCG_EINVAL;
  if (!p->have_points || !p->have_weights || p->wmode == FTCG_W_BAND) return FTCG_ESTATE;
  return guarded([&] {
    finish_deferred_weights(p);
    FTCG_HIP(hipMemcpyAsync(alpha_dev, p->alpha.p, sizeof(double) * p->m, hipMemcpyDeviceToDevice, p->stream));
    if (used_fallback_host) {
      FTCG_HIP(hipStreamSynchronize(p->stream));
      *used_fallback_host = p->used_fallback;
    }
  });
}

ftcg_status ftcg_spread_only(ftcg_plan p, const void* fhat_dev, void* grid_dev) {
  if (!p || !fhat_dev || !grid_dev) return FTCG_EINVAL;
  if (!p->have_points || !p->have_weights) return FTCG_ESTATE;
  return guarded([&] {
    if (p->wmode == FTCG_W_BAND) {
      band_apply(p, fhat_dev);
      fhat_dev = p->band_c.p;
    }
    timing_begin(p, STEP_SPREAD);
    spread(p, fhat_dev, grid_dev);
    timing_end(p, STEP_SPREAD);
  });
}

ftcg_status ftcg_grid_to_image(ftcg_plan p, const void* grid_dev, void* image_dev) {
  if (!p || !grid_dev || !image_dev) return FTCG_EINVAL;
  return guarded([&] { grid_to_image(p, grid_dev, image_dev); });
}

ftcg_status ftcg_execute(ftcg_plan p, const void* fhat_dev, void* image_dev) {
  if (!p || !fhat_dev || !image_dev) return FTCG_EINVAL;
  if (!p->have_points || !p->have_weights) return FTCG_ESTATE;
  return guarded([&] {
    if (p->wmode == FTCG_W_BAND) {
      band_apply(p, fhat_dev);
      fhat_dev = p->band_c.p;
    }
    timing_begin(p, STEP_SPREAD);
    spread(p, fhat_dev, p->grid.p);
    timing_end(p, STEP_SPREAD);
    grid_to_image(p, p->grid.p, image_dev);
  });
}

ftcg_status ftcg_forward(ftcg_plan p, const void* image_dev, void* fhat_dev) {
  if (!p || !image_dev || !fhat_dev) return FTCG_EINVAL;
  if (!p->have_points || p->weights_only) return FTCG_ESTATE;
  return guarded([&] { forward_transform(p, image_dev, fhat_dev); });
}

ftcg_status ftcg_frame_approx(ftcg_plan p, int64_t m, const double* k_dev, const void* fhat_dev, void* image_dev) {
  if (!p || !k_dev || !fhat_dev || !image_dev) return FTCG_EINVAL;
  if (m < 1) return FTCG_EINVAL;
  if (p->dtype != FTCG_F64 || (p->n & (p->n - 1)) != 0) return FTCG_EUNSUPPORTED;
  int64_t modes = p->n;
  if (p->dim == 2) modes *= p->n;
  if (p->n > 1024 || modes > 4096 || std::min<int64_t>(m, modes) > 4096 || m * modes > (int64_t(1) << 27))
    return FTCG_EUNSUPPORTED;
  return guarded([&] { frame_approx(p, m, k_dev, fhat_dev, image_dev); });
}

ftcg_status ftcg_plan_set_band(ftcg_plan p, int r) {
  if (!p) return FTCG_EINVAL;
  if (p->wmode != FTCG_W_BAND) return FTCG_ESTATE;
  if (r < 1 || r > 16) return FTCG_EINVAL;
  p->band_r = r;
  p->have_points = false;
  p->have_weights = false;
  return FTCG_OK;
}

ftcg_status ftcg_plan_set_density_iterations(ftcg_plan p, int iters) {
  if (!p) return FTCG_EINVAL;
  if (p->wmode != FTCG_W_DENSITY) return FTCG_ESTATE;
  if (iters < 1 || iters > 1000) return FTCG_EINVAL;
  p->den_iters = iters;
  p->have_points = false;
  p->have_weights = false;
  return FTCG_OK;
}

ftcg_status ftcg_get_band(ftcg_plan p, double* c_dev, int* r_host) {
  if (!p || !c_dev) return FTCG_EINVAL;
  if (p->wmode != FTCG_W_BAND || !p->have_points || !p->have_weights) return FTCG_ESTATE;
  return guarded([&] {
    FTCG_HIP(hipMemcpyAsync(c_dev, p->band_col.p, sizeof(double) * p->m * (2 * p->band_r - 1),
                            hipMemcpyDeviceToDevice, p->stream));
    if (r_host) *r_host = p->band_r;
  });
}

ftcg_status ftcg_plan_set_mlp(ftcg_plan p, ftcg_mlp mlp, double audit_threshold, int64_t audit_samples) {
  if (!p || !mlp) return FTCG_EINVAL;
  if (p->wmode != FTCG_W_LEARNED) return FTCG_ESTATE;
  if (!(audit_threshold >= 0.0) || audit_samples < 1) return FTCG_EINVAL;
  p->mlp = mlp;
  p->audit_threshold = audit_threshold;
  p->audit_samples = audit_samples;
  p->have_points = false;
  return FTCG_OK;
}

ftcg_status ftcg_plan_learned_report(ftcg_plan p, double* audit_estimate, int* used_fallback) {
  if (!p) return FTCG_EINVAL;
  if (p->wmode != FTCG_W_LEARNED || !p->have_weights) return FTCG_ESTATE;
  if (audit_estimate) *audit_estimate = p->audit_estimate;
  if (used_fallback) *used_fallback = p->used_fallback;
  return FTCG_OK;
}

ftcg_status ftcg_plan_info(ftcg_plan p, int64_t* grid_size, int64_t* n_records, int64_t* n_tiles, int* tile) {
  if (!p) return FTCG_EINVAL;
  return guarded([&] {
    if (grid_size) *grid_size = p->G;
    if (n_records) *n_records = p->have_points && !p->weights_only ? plan_nrec(p) : 0;
    if (n_tiles) *n_tiles = p->ntiles;
    if (tile) *tile = p->tile;
  });
}

ftcg_status ftcg_plan_set_weight_tuning(ftcg_plan p, int samples_per_lane, int lanes_per_group) {
  if (!p) return FTCG_EINVAL;
  const int w = samples_per_lane, l = lanes_per_group;
  if (!(w == 0 || w == 1 || w == 2 || w == 4)) return FTCG_EINVAL;
  if (!(l == 0 || l == 1 || l == 2 || l == 4)) return FTCG_EINVAL;
  p->w_samples = w;
  p->w_lanes = l;
  return FTCG_OK;
}

ftcg_status ftcg_plan_set_tuning(ftcg_plan p, int tile, int accum, int lds_copies) {
  if (!p) return FTCG_EINVAL;
  if (tile != 0 && tile != 16 && tile != 32 && tile != 64 && tile != 128 && !(p->dim == 1 && is_pow2(tile)))
    return FTCG_EINVAL;
  if (tile != 0 && tile < 2 * p->W) return FTCG_EINVAL;
  if (accum != FTCG_ACCUM_FIXED && accum != FTCG_ACCUM_F64) return FTCG_EINVAL;
  if (lds_copies != 1 && lds_copies != 2 && lds_copies != 4) return FTCG_EINVAL;
  if (accum == FTCG_ACCUM_FIXED && (p->dtype != FTCG_F32 || lds_copies != 1)) return FTCG_EUNSUPPORTED;
  if (accum == FTCG_ACCUM_F64 && p->dim == 2) {
    const int64_t t = tile ? tile : 64;
    if (t > 64 || (size_t)lds_copies * 2 * t * (t + 1) * sizeof(double) > 160 * 1024) return FTCG_EUNSUPPORTED;
  }
  p->tile_req = tile;
  p->accum = accum;
  p->lds_copies = lds_copies;
  p->have_points = false;
  return FTCG_OK;
}

ftcg_status ftcg_plan_set_spread_layout(ftcg_plan p, int layout) {
  if (!p) return FTCG_EINVAL;
  if (layout != FTCG_SPREAD_AUTO && layout != FTCG_SPREAD_TILES) return FTCG_EINVAL;
  p->spread_segments = layout == FTCG_SPREAD_AUTO;
  return FTCG_OK;
}

ftcg_status ftcg_plan_enable_timing(ftcg_plan p, int enable) {
  if (!p) return FTCG_EINVAL;
  p->timing.enabled = enable != 0;
  return FTCG_OK;
}

ftcg_status ftcg_plan_timing(ftcg_plan p, double* ms, int64_t* count) {
  if (!p || !ms || !count) return FTCG_EINVAL;
  return guarded([&] {
    FTCG_HIP(hipStreamSynchronize(p->stream));
    for (int s = 0; s < N_STEPS; ++s) {
      ms[s] = 0.0;
      count[s] = 0;
    }
    Timing& t = p->timing;
    for (auto& pr : t.pending) {
      float v = 0.f;
      FTCG_HIP(hipEventElapsedTime(&v, pr.a, pr.b));
      ms[pr.step] += v;
      count[pr.step] += 1;
      t.pool.push_back(pr.a);
      t.pool.push_back(pr.b);
    }
    t.pending.clear();
  });
}

}  // extern "C"
