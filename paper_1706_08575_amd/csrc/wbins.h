// Neighbour bins of the frame-weight sum: bin lookup and the row-grouped
// sample record of the 2D two-level sort (shared by the weight and the
// binning sources).
#pragma once

#include "ftcg_internal.h"

namespace ftcg {

// bin of a sample that passed the input check
template <int DIM>
__device__ inline int wbin_of(const double* x, const WBinGeom& g, int* b) {
  int id = 0;
  for (int a = 0; a < DIM; ++a) {
    int v = (int)floor((x[a] - g.kmin[a]) / g.h);
    v = v < 0 ? 0 : (v >= g.nb[a] ? g.nb[a] - 1 : v);
    b[a] = v;
    id = id * g.nb[a] + v;
  }
  return id;
}

// a sample grouped by bin row: coordinates, caller index, bin column
struct RowRec {
  double k0, k1;
  int32_t j, b1;
};

// bin row and column of sample j, clamped in floating point (a NaN lands in
// the last row or column), so both are in range for any input: the row
// binning runs before the host has seen the input check
__device__ inline int wbin_row_col(const double* __restrict__ k, int64_t j, const WBinGeom& g, int* b1,
                                   double* x) {
  x[0] = k[2 * j];
  x[1] = k[2 * j + 1];
  int b[2];
  for (int a = 0; a < 2; ++a)
    b[a] = (int)fmax(0.0, fmin(floor((x[a] - g.kmin[a]) / g.h), (double)(g.nb[a] - 1)));
  *b1 = b[1];
  return b[0];
}

}  // namespace ftcg
