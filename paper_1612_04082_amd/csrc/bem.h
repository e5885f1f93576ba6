// Collocation BEM system on the device (see bem.hip).
#pragma once
#include <memory>
#include <vector>

#include "../../include/kfmm.h"
#include "common.h"
#include "plan.h"
#include "tree.h"

namespace kfmm {

struct TwoLevelPC;

// The plan's cell list of a problem: empty in free space, the periodic cell otherwise.
inline std::vector<double> problem_cells(const bem_problem& p) {
  return p.cell ? std::vector<double>(p.cell, p.cell + 4) : std::vector<double>();
}

// Near pairs (t, e) of the near-singular quadrature (nearfield.hip): CSR by t (off[T + 1], idx sorted by e)
// and the row of every entry.
struct NearPairs {
  int64_t n = 0;
  int *off = nullptr, *idx = nullptr, *row = nullptr;
  signed char* sh = nullptr;  // periodic surface: the image's shift code (sx+1)+3(sy+1)+9(sz+1) per pair
  double cell_L = 0;          // side of the periodic cell, 0 in free space
};
// cell_L > 0: the surface repeats with that period; pairs with an element's images across the faces too
NearPairs find_near_pairs(const double* tri, const double* cen, int64_t T, double radius, Arena& arena,
                          hipStream_t s, double cell_L = 0);
// dU, dP (n x 9 each): upsampled blocks (levels extra midpoint splits) minus the element's 16 quadrature points
void near_blocks(const NearPairs& np, int levels, const double* tri, const double* cen, const double* qp,
                 const double* qn, const double* qw, const Elastic& el, double* dU, double* dP, hipStream_t s);

struct BemSystem {
  hipStream_t stream;
  int64_t T = 0, n = 0;
  Elastic el{};
  const double* tri = nullptr;
  const int8_t* bc_type = nullptr;
  const double* bc_val = nullptr;
  double mean_edge = 0, scale_t = 1;
  Arena arena;
  double *qp = nullptr, *qn = nullptr, *qw = nullptr, *cen = nullptr;  // quadrature sources, collocation points
  double *dU = nullptr, *dP = nullptr;                                 // local-pass blocks (T x 3 x 3)
  int near_levels = 0;                                                 // upsampled near-singular quadrature
  NearPairs near;
  double *near_dU = nullptr, *near_dP = nullptr;                       // near.n x 3 x 3
  double *a16 = nullptr, *b16 = nullptr, *ae = nullptr, *be = nullptr, *fmm_out = nullptr;
  double* partial = nullptr;
  std::unique_ptr<Plan> plan;
  std::unique_ptr<TwoLevelPC> pc;  // right preconditioner of gmres (optional)
  int64_t n_apply = 0;

  BemSystem(const bem_problem& p, const fmm_opts& fo, hipStream_t s);
  ~BemSystem();
  void apply(int mode, const double* x, double* out);  // 0: A x, 1: B y
  double dot(const double* x, const double* y);
  void split(const double* x, double* u, double* t);
  bem_stats gmres(const double* x0, const double* x0_alt, double* x, double tol, int m, int max_iter);
  double* scratch_partial();
};

// Multiplies the traction entries of an unknown vector by factor (scale_t: solver units -> physical).
void scale_traction_unknowns(BemSystem& sys, double* x, double factor);

// Interior stress (eq. stress_1) from boundary u, t through a fresh plan with the lattice as targets.
void stress_from_boundary(const bem_problem& p, const double* u, const double* t, const double* trg, int64_t M,
                          double* out, const fmm_opts& fo, hipStream_t s);

// Pointwise topological derivative (eq. deriv) of M stresses, each plus sig_h (host, 6; NULL for none).
void topological_derivative(const double* sig, int64_t M, const Elastic& el, double* td, hipStream_t s,
                            const double* sig_h = nullptr);

// Quadrature expansion only (16 points per triangle, normals, weights, centroids).
void bem_expand(int64_t T, const double* tri, double* qp, double* qn, double* qw, double* cen, hipStream_t s);

}  // namespace kfmm
