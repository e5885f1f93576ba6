// Two-level additive Schwarz preconditioner of the collocation BEM system (see precond.hip).
#pragma once
#include "bem.h"

namespace kfmm {

constexpr int kPcFineMax = 32;     // elements per fine block at most (96 x 96 blocks, inverted in LDS)
constexpr int kPcCols = 6;         // coarse columns per aggregate: three translations, three rotations
constexpr int kPcMaxCoarse = 4096; // coarse dimension the default aggregate size stays within

// Aggregate size used when the caller passes 0: 64 elements, doubled while the coarse dimension
// 6 * ceil(T / size) exceeds kPcMaxCoarse.
int pc_default_aggregate(int64_t T);

struct TwoLevelPC {
  int64_t T = 0, nb = 0, na = 0, nc = 0;
  int fine = 32, coarse = 64, n_dropped = 0;
  double t_setup_s = 0;
  Arena arena;
  int* order = nullptr;     // T: element order along the Morton curve of the centroids
  double* binv_t = nullptr; // nb x (3 fine)^2: inverse of each fine block, transposed (column-major)
  double* z = nullptr;      // T x 3 x 6: the element's rows of its aggregate's orthonormal coarse columns
  double* einv = nullptr;   // nc x nc: inverse of E = Z^T A Z (dropped columns padded with identity)
  double *s = nullptr, *g = nullptr;  // nc: Z^T v and E^-1 Z^T v

  void build(const BemSystem& sys, int fine, int coarse);
  // y = M^-1 v (device, 3T each, solver units); y must not alias v
  void apply(const double* v, double* y, hipStream_t st) const;
};

}  // namespace kfmm
