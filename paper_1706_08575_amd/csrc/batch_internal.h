// Batched execution: descriptors shared by the batch kernels and the batch API.
#pragma once

#include "ftcg_internal.h"

namespace ftcg {

struct BatchItem {
  const Rec<float>* recs;    // the item plan's records
  const float* alpha_s;      // and record weights
  int64_t fhat_off;          // first value of this item in the concatenated values
  int64_t grid_off;          // first cell of this item's grid in the batch grid
  int64_t tmp_off;           // first entry of this item's n x G transposed intermediate
  int64_t img_off;           // first pixel of this item's image in the concatenated images
  int64_t deapod_off;        // first deapodization factor of this item
  int64_t G;                 // grid edge
  int n;                     // image edge
  int nt;                    // tiles per axis
  float beta;
};

struct BatchTile {
  int item;
  int t0, t1;                // tile coordinates
  int beg, end;              // records of the tile in the item plan
  int split;                 // slot in the 64-bit scratch, or -1
};

struct BatchTask {
  int tile;                  // index into the tile table
  int part;                  // chunk number within the tile
  int beg, end;              // records of this chunk
};

// pointers of the current call, read by the kernels (the captured graph never changes)
struct BatchArgs {
  const float2* fhat;
  float2* images;
  float2* grid;
  float2* tmp;
  const double* deapod;
};

}  // namespace ftcg

struct ftcg_batch_s {
  hipStream_t stream = nullptr;
  int n_items = 0;
  int W = 6;
  double sigma = 2.0;
  ftcg_wmode wmode = FTCG_W_PLAIN;
  double R = 8.0;
  int tile = 32;
  int64_t chunk = 4096;          // records per task
  int persistent_blocks = 0;
  std::vector<int64_t> n;        // image edge per item
  std::vector<int64_t> m;        // samples per item
  std::vector<ftcg_plan> plans;  // one plan per item (geometry, weights, records)
  std::vector<ftcg::BatchItem> items;
  std::vector<std::vector<int>> fft_groups;  // item lists per distinct grid size
  ftcg::DevBuf items_dev, tiles, tasks, bounds, scratch, split_tiles, counter, args_dev;
  ftcg::DevBuf grid, tmp, deapod, group_items;
  ftcg::DevBuf twiddle;          // two-level twiddle tables (float2), one per grid size
  std::vector<int64_t> twiddle_off;  // first entry of each fft group's table
  int64_t ntiles = 0, ntasks = 0, nsplit = 0;
  int64_t m_total = 0, img_total = 0;
  bool have_points = false;
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  ftcg::BatchArgs* host_args = nullptr;   // pinned
  struct ftcg_mlp_s* mlp = nullptr;
  double audit_threshold = 1e-4;
  int64_t audit_samples = 4096;
  // set_points runs the items on BATCH_STREAMS streams of default priority
  // (joined back into `stream` by events), so that the small items' launches
  // and short kernels overlap the large items' weight sums
  static constexpr int BATCH_STREAMS = 3;
  hipStream_t side[BATCH_STREAMS] = {};
  hipEvent_t ev_side[BATCH_STREAMS] = {};
  hipEvent_t ev_start = nullptr;
  int32_t* host_off = nullptr;   // pinned: every item's tile offsets
  size_t host_off_len = 0;
};

namespace ftcg {
void batch_spread(ftcg_batch_s* b);
void batch_fft(ftcg_batch_s* b);
void batch_fft_prepare();   // once, outside any graph capture
}  // namespace ftcg
