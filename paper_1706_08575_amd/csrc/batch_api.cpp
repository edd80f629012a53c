// C ABI of batched execution (ftcg_batch_*): item plans, task tables, graph
// capture and replay.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>

#include "batch_internal.h"
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

__global__ void k_set_args(BatchArgs* a, const float2* fhat, float2* images, float2* grid, float2* tmp,
                           const double* deapod) {
  if (threadIdx.x == 0) {
    a->fhat = fhat;
    a->images = images;
    a->grid = grid;
    a->tmp = tmp;
    a->deapod = deapod;
  }
}

void drop_graph(ftcg_batch_s* b) {
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->graph_exec = nullptr;
  b->graph = nullptr;
}

void set_args(ftcg_batch_s* b, const void* fhat, void* images) {
  hipLaunchKernelGGL(k_set_args, dim3(1), dim3(64), 0, b->stream, b->args_dev.as<BatchArgs>(),
                     static_cast<const float2*>(fhat), static_cast<float2*>(images), b->grid.as<float2>(),
                     b->tmp.as<float2>(), b->deapod.as<double>());
  FTCG_HIP(hipGetLastError());
}

void enqueue_execute(ftcg_batch_s* b, hipStream_t s) {
  hipStream_t keep = b->stream;
  b->stream = s;
  batch_spread(b);
  batch_fft(b);
  b->stream = keep;
}

// build the tile and task tables from the item plans' tile offsets
void build_tables(ftcg_batch_s* b) {
  std::vector<BatchTile> tiles;
  // every item's tile offsets in one pinned buffer, one wait for all of them
  size_t need = 0;
  for (ftcg_plan p : b->plans) need += (size_t)p->ntiles + 1;
  if (need > b->host_off_len) {
    if (b->host_off) FTCG_HIP(hipHostFree(b->host_off));
    b->host_off = nullptr;
    b->host_off_len = 0;
    FTCG_HIP(hipHostMalloc((void**)&b->host_off, sizeof(int32_t) * need, hipHostMallocDefault));
    b->host_off_len = need;
  }
  {
    size_t at = 0;
    for (ftcg_plan p : b->plans) {
      FTCG_HIP(hipMemcpyAsync(b->host_off + at, p->tile_off.p, sizeof(int32_t) * (p->ntiles + 1),
                              hipMemcpyDeviceToHost, b->stream));
      at += (size_t)p->ntiles + 1;
    }
    FTCG_HIP(hipStreamSynchronize(b->stream));
  }
  size_t at = 0;
  for (int i = 0; i < b->n_items; ++i) {
    ftcg_plan p = b->plans[i];
    const int32_t* off = b->host_off + at;
    at += (size_t)p->ntiles + 1;
    for (int64_t t = 0; t < p->ntiles; ++t) {
      BatchTile tl;
      tl.item = i;
      tl.t0 = (int)(t / p->nt);
      tl.t1 = (int)(t % p->nt);
      tl.beg = off[t];
      tl.end = off[t + 1];
      tl.split = -1;
      tiles.push_back(tl);
    }
  }
  // tasks of at most `chunk` records; order heaviest first by a counting sort
  // on 64 size buckets (empty tiles last)
  const int64_t chunk = b->chunk;
  std::vector<BatchTask> tasks;
  int64_t nsplit = 0;
  std::vector<int> split_tiles;
  for (size_t t = 0; t < tiles.size(); ++t) {
    const int64_t cnt = tiles[t].end - tiles[t].beg;
    const int64_t parts = cnt > chunk ? (cnt + chunk - 1) / chunk : 1;
    if (parts > 1) {
      tiles[t].split = (int)nsplit++;
      split_tiles.push_back((int)t);
    }
    for (int64_t q = 0; q < parts; ++q) {
      BatchTask k;
      k.tile = (int)t;
      k.part = (int)q;
      k.beg = (int)(tiles[t].beg + q * chunk);
      k.end = (int)std::min<int64_t>(tiles[t].end, tiles[t].beg + (q + 1) * chunk);
      tasks.push_back(k);
    }
  }
  const int NB = 65;
  std::vector<int64_t> bucket_count(NB + 1, 0);
  auto bucket = [&](const BatchTask& k) {
    const int64_t c = k.end - k.beg;
    if (c == 0) return NB - 1;                                   // empty: last
    return (int)(NB - 2 - std::min<int64_t>(NB - 2, (c * (NB - 2)) / (chunk + 1)));  // heavy: first
  };
  for (const auto& k : tasks) bucket_count[bucket(k) + 1]++;
  for (int i = 0; i < NB; ++i) bucket_count[i + 1] += bucket_count[i];
  std::vector<BatchTask> ordered(tasks.size());
  for (const auto& k : tasks) ordered[bucket_count[bucket(k)]++] = k;

  b->ntiles = (int64_t)tiles.size();
  b->ntasks = (int64_t)ordered.size();
  b->nsplit = nsplit;
  b->tiles.ensure(sizeof(BatchTile) * std::max<size_t>(1, tiles.size()));
  b->tasks.ensure(sizeof(BatchTask) * std::max<size_t>(1, ordered.size()));
  b->bounds.ensure(sizeof(float) * std::max<size_t>(1, tiles.size()));
  b->split_tiles.ensure(sizeof(int) * std::max<int64_t>(1, nsplit));
  b->scratch.ensure(sizeof(unsigned long long) * std::max<int64_t>(1, nsplit * b->tile * b->tile));
  FTCG_HIP(hipMemcpyAsync(b->tiles.p, tiles.data(), sizeof(BatchTile) * tiles.size(), hipMemcpyHostToDevice,
                          b->stream));
  FTCG_HIP(hipMemcpyAsync(b->tasks.p, ordered.data(), sizeof(BatchTask) * ordered.size(), hipMemcpyHostToDevice,
                          b->stream));
  if (nsplit)
    FTCG_HIP(hipMemcpyAsync(b->split_tiles.p, split_tiles.data(), sizeof(int) * nsplit, hipMemcpyHostToDevice,
                            b->stream));
  FTCG_HIP(hipStreamSynchronize(b->stream));
}

}  // namespace

extern "C" {

ftcg_status ftcg_batch_destroy(ftcg_batch_s* b);

ftcg_status ftcg_batch_create(ftcg_batch_s** out, int n_items, const int64_t* n, int half_width, double sigma,
                              ftcg_wmode wmode, double R, void* hip_stream) {
  if (!out || !n) return FTCG_EINVAL;
  *out = nullptr;
  if (n_items < 1 || n_items > 4096) return FTCG_EINVAL;
  // batches take diagonal weights computed per item by the frame-weight sum
  // or the network, or given by the caller
  if (wmode == FTCG_W_BAND || wmode == FTCG_W_DENSITY) return FTCG_EUNSUPPORTED;
  ftcg_batch_s* b = new (std::nothrow) ftcg_batch_s();
  if (!b) return FTCG_ENOMEM;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->n_items = n_items;
  b->W = half_width;
  b->sigma = sigma;
  b->wmode = wmode;
  b->R = R;
  ftcg_status st = guard([&] {
    int dev = 0, ncu = 0;
    FTCG_HIP(hipGetDevice(&dev));
    FTCG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    b->persistent_blocks = ncu * 8;
    batch_fft_prepare();
    for (int q = 0; q < ftcg_batch_s::BATCH_STREAMS; ++q) {
      FTCG_HIP(hipStreamCreateWithFlags(&b->side[q], hipStreamNonBlocking));
      FTCG_HIP(hipEventCreateWithFlags(&b->ev_side[q], hipEventDisableTiming));
    }
    FTCG_HIP(hipEventCreateWithFlags(&b->ev_start, hipEventDisableTiming));
    for (int i = 0; i < n_items; ++i) {
      ftcg_plan p = nullptr;
      const int64_t nn[2] = {n[i], n[i]};
      ftcg_status s = ftcg_plan_create(&p, 2, nn, half_width, sigma, FTCG_F32, wmode, R, hip_stream);
      if (s != FTCG_OK) throw StatusError{s};
      b->plans.push_back(p);
      b->n.push_back(n[i]);
      s = ftcg_plan_set_tuning(p, b->tile, FTCG_ACCUM_FIXED, 1);
      if (s != FTCG_OK) throw StatusError{s};
    }
    b->items.resize(n_items);
    b->m.assign(n_items, 0);
    b->items_dev.ensure(sizeof(BatchItem) * n_items);
    b->args_dev.ensure(sizeof(BatchArgs));
    b->counter.ensure(64);
    int64_t grid = 0, tmp = 0, img = 0, dp = 0;
    for (int i = 0; i < n_items; ++i) {
      ftcg_plan p = b->plans[i];
      grid += p->G * p->G;
      tmp += p->n * p->G;
      img += p->n * p->n;
      dp += p->n;
    }
    b->grid.ensure(sizeof(float2) * grid);
    b->tmp.ensure(sizeof(float2) * tmp);
    b->deapod.ensure(sizeof(double) * dp);
    b->img_total = img;

    // fft groups by grid size
    std::map<int64_t, std::vector<int>> groups;
    for (int i = 0; i < n_items; ++i) groups[b->plans[i]->G].push_back(i);
    std::vector<int> flat;
    for (auto& kv : groups) {
      b->fft_groups.push_back(kv.second);
      flat.insert(flat.end(), kv.second.begin(), kv.second.end());
    }
    // twiddle tables per grid size, the same as a single plan's (so batch
    // items stay bitwise equal to single plans)
    int64_t ntw = 0;
    for (auto& grp : b->fft_groups) {
      b->twiddle_off.push_back(ntw);
      ntw += twiddle_entries(b->plans[grp[0]]->G);
    }
    b->twiddle.ensure(sizeof(float2) * ntw);
    for (size_t gi = 0; gi < b->fft_groups.size(); ++gi)
      compute_twiddles(b->twiddle.as<float2>() + b->twiddle_off[gi], b->plans[b->fft_groups[gi][0]]->G, false,
                       b->stream);
    b->group_items.ensure(sizeof(int) * flat.size());
    FTCG_HIP(hipMemcpy(b->group_items.p, flat.data(), sizeof(int) * flat.size(), hipMemcpyHostToDevice));
  });
  if (st != FTCG_OK) {
    ftcg_batch_destroy(b);
    return st;
  }
  *out = b;
  return FTCG_OK;
}

ftcg_status ftcg_batch_destroy(ftcg_batch_s* b) {
  if (!b) return FTCG_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (ftcg_plan p : b->plans) ftcg_plan_destroy(p);
  DevBuf* bufs[] = {&b->items_dev, &b->tiles, &b->tasks, &b->bounds, &b->scratch, &b->split_tiles, &b->counter,
                    &b->args_dev, &b->grid, &b->tmp, &b->deapod, &b->group_items, &b->twiddle};
  for (DevBuf* d : bufs) d->release();
  for (int q = 0; q < ftcg_batch_s::BATCH_STREAMS; ++q) {
    if (b->side[q]) {
      (void)hipStreamSynchronize(b->side[q]);
      (void)hipStreamDestroy(b->side[q]);
    }
    if (b->ev_side[q]) (void)hipEventDestroy(b->ev_side[q]);
  }
  if (b->ev_start) (void)hipEventDestroy(b->ev_start);
  if (b->host_off) (void)hipHostFree(b->host_off);
  delete b;
  return FTCG_OK;
}

ftcg_status ftcg_batch_set_tuning(ftcg_batch_s* b, int tile, int64_t chunk_records, int persistent_blocks,
                                  int use_graph) {
  if (!b) return FTCG_EINVAL;
  if (tile != 16 && tile != 32 && tile != 64 && tile != 128) return FTCG_EINVAL;
  if (tile < 2 * b->W) return FTCG_EINVAL;
  if (chunk_records < 64 || persistent_blocks < 1 || persistent_blocks > 65536) return FTCG_EINVAL;
  return guard([&] {
    for (ftcg_plan p : b->plans) {
      ftcg_status s = ftcg_plan_set_tuning(p, tile, FTCG_ACCUM_FIXED, 1);
      if (s != FTCG_OK) throw StatusError{s};
    }
    b->tile = tile;
    b->chunk = chunk_records;
    b->persistent_blocks = persistent_blocks;
    b->use_graph = use_graph != 0;
    b->have_points = false;
    drop_graph(b);
  });
}

ftcg_status ftcg_batch_set_mlp(ftcg_batch_s* b, ftcg_mlp mlp, double audit_threshold, int64_t audit_samples) {
  if (!b || !mlp) return FTCG_EINVAL;
  for (ftcg_plan p : b->plans) {
    ftcg_status s = ftcg_plan_set_mlp(p, mlp, audit_threshold, audit_samples);
    if (s != FTCG_OK) return s;
  }
  b->have_points = false;
  return FTCG_OK;
}

ftcg_status ftcg_batch_set_points(ftcg_batch_s* b, const int64_t* m_host, const double* k_dev) {
  if (!b || !m_host || !k_dev) return FTCG_EINVAL;
  for (int i = 0; i < b->n_items; ++i)
    if (m_host[i] < 1 || m_host[i] >= (int64_t(1) << 31)) return FTCG_EINVAL;
  constexpr int NS = ftcg_batch_s::BATCH_STREAMS;
  // the items' plans enqueue on the side streams for the duration of the
  // call, and on the batch stream again afterwards, also after an error
  struct Restore {
    ftcg_batch_s* b;
    ~Restore() {
      for (ftcg_plan p : b->plans) p->stream = b->stream;
    }
  } restore{b};
  return guard([&] {
    b->have_points = false;
    drop_graph(b);
    // the side streams start after the work already on the batch stream (a
    // previous execute may still read the records rewritten here)
    FTCG_HIP(hipEventRecord(b->ev_start, b->stream));
    for (int q = 0; q < NS; ++q) FTCG_HIP(hipStreamWaitEvent(b->side[q], b->ev_start, 0));
    // items to streams, largest first onto the least loaded (by samples)
    std::vector<int> order(b->n_items);
    for (int i = 0; i < b->n_items; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return m_host[x] > m_host[y]; });
    int64_t load[NS] = {};
    std::vector<int64_t> off(b->n_items);
    {
      int64_t o = 0;
      for (int i = 0; i < b->n_items; ++i) {
        off[i] = o;
        o += m_host[i];
      }
      b->m_total = o;
    }
    for (int i : order) {
      int q = 0;
      for (int r = 1; r < NS; ++r)
        if (load[r] < load[q]) q = r;
      load[q] += m_host[i];
      b->plans[i]->stream = b->side[q];
    }
    // every item's input check and early binning, then the rest of each
    // item once the host has read its check
    for (int i : order) set_points_begin(b->plans[i], m_host[i], k_dev + 2 * off[i]);
    for (int i : order) {
      ftcg_plan p = b->plans[i];
      set_points_end(p, k_dev + 2 * off[i]);
      finish_deferred_weights(p);   // the batched spread reads the records' weights
    }
    for (int q = 0; q < NS; ++q) {
      FTCG_HIP(hipEventRecord(b->ev_side[q], b->side[q]));
      FTCG_HIP(hipStreamWaitEvent(b->stream, b->ev_side[q], 0));
    }
    int64_t grid = 0, tmp = 0, img = 0, dp = 0;
    for (int i = 0; i < b->n_items; ++i) {
      ftcg_plan p = b->plans[i];
      b->m[i] = m_host[i];
      BatchItem& it = b->items[i];
      it.recs = p->recs.as<Rec<float>>();
      it.alpha_s = p->alpha_s.as<float>();
      it.fhat_off = off[i];
      it.grid_off = grid;
      it.tmp_off = tmp;
      it.img_off = img;
      it.deapod_off = dp;
      it.G = p->G;
      it.n = (int)p->n;
      it.nt = (int)p->nt;
      it.beta = (float)p->beta;
      FTCG_HIP(hipMemcpyAsync(b->deapod.as<double>() + dp, p->deapod.p, sizeof(double) * p->n,
                              hipMemcpyDeviceToDevice, b->stream));
      grid += p->G * p->G;
      tmp += p->n * p->G;
      img += p->n * p->n;
      dp += p->n;
    }
    FTCG_HIP(hipMemcpyAsync(b->items_dev.p, b->items.data(), sizeof(BatchItem) * b->n_items,
                            hipMemcpyHostToDevice, b->stream));
    build_tables(b);
    b->have_points = true;
  });
}

ftcg_status ftcg_batch_set_weights(ftcg_batch_s* b, const double* alpha_dev) {
  if (!b || !alpha_dev) return FTCG_EINVAL;
  if (!b->have_points) return FTCG_ESTATE;
  return guard([&] {
    for (int i = 0; i < b->n_items; ++i) {
      ftcg_status s = ftcg_set_weights(b->plans[i], alpha_dev + b->items[i].fhat_off);
      if (s != FTCG_OK) throw StatusError{s};
    }
  });
}

ftcg_status ftcg_batch_get_weights(ftcg_batch_s* b, double* alpha_dev) {
  if (!b || !alpha_dev) return FTCG_EINVAL;
  if (!b->have_points) return FTCG_ESTATE;
  return guard([&] {
    for (int i = 0; i < b->n_items; ++i) {
      ftcg_status s = ftcg_get_weights(b->plans[i], alpha_dev + b->items[i].fhat_off, nullptr);
      if (s != FTCG_OK) throw StatusError{s};
    }
  });
}

ftcg_status ftcg_batch_execute(ftcg_batch_s* b, const void* fhat_dev, void* images_dev) {
  if (!b || !fhat_dev || !images_dev) return FTCG_EINVAL;
  if (!b->have_points) return FTCG_ESTATE;
  for (ftcg_plan p : b->plans)
    if (!p->have_weights) return FTCG_ESTATE;
  return guard([&] {
    set_args(b, fhat_dev, images_dev);
    if (!b->use_graph) {
      enqueue_execute(b, b->stream);
      return;
    }
    if (!b->graph_exec) {
      // capture on a private stream (the null stream cannot be captured),
      // replay on the caller's stream
      hipStream_t cap;
      FTCG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          enqueue_execute(b, cap);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cap, &g);
          if (g) (void)hipGraphDestroy(g);
          (void)hipStreamDestroy(cap);
          throw;
        }
        e = hipStreamEndCapture(cap, &b->graph);
      }
      (void)hipStreamDestroy(cap);
      FTCG_HIP(e);
      FTCG_HIP(hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0));
    }
    FTCG_HIP(hipGraphLaunch(b->graph_exec, b->stream));
  });
}

ftcg_status ftcg_batch_info(ftcg_batch_s* b, int64_t* n_tasks, int64_t* n_split_tiles, int64_t* n_records,
                            int64_t* n_tiles) {
  if (!b) return FTCG_EINVAL;
  return guard([&] {
    int64_t r = 0;
    for (ftcg_plan p : b->plans) r += plan_nrec(p);   // may throw HipError (reads the device)
    if (n_tasks) *n_tasks = b->ntasks;
    if (n_split_tiles) *n_split_tiles = b->nsplit;
    if (n_records) *n_records = r;
    if (n_tiles) *n_tiles = b->ntiles;
  });
}

ftcg_status ftcg_batch_enable_timing(ftcg_batch_s* b, int enable) {
  if (!b) return FTCG_EINVAL;
  for (ftcg_plan p : b->plans) ftcg_plan_enable_timing(p, enable);
  return FTCG_OK;
}

}  // extern "C"
