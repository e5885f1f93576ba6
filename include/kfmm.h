/*
 * kfmm.h -- C ABI of the MI355X kernel-independent fast multipole library for 3D isotropic
 * elastostatics (Kelvin kernels) and the collocation BEM it drives.
 *
 * Paper: Ostanin, Tsybulin, Litsarev, Oseledets, Zorin, "What lies beneath the surface:
 * topological-shape optimization with the kernel-independent fast multipole method"
 * (arXiv:1612.04082).  Section references below are to that paper.
 *
 * Conventions for every entry point
 *  - Pointers are DEVICE pointers unless marked (host).  Floating-point I/O is FP64, row-major,
 *    array-of-structures: a point is 3 consecutive doubles (x, y, z).
 *  - All device work is enqueued on the HIP stream passed as `stream` (a hipStream_t; NULL means
 *    the default stream).  fmm_eval returns without waiting for the GPU; fmm_plan, bem_solve and the
 *    ws_* training call synchronise the stream because they need sizes or residuals on the host.
 *  - A plan copies what it needs during fmm_plan and keeps no pointer to caller memory.  The caller
 *    owns every input and output buffer.  A plan must not be used from two streams at once.
 *  - Errors: a negative status is returned; outputs are then undefined (except KFMM_E_NOCONV, which
 *    leaves the best iterate and filled statistics).  kfmm_last_error() returns a message for the
 *    last failing call on the calling thread.
 *  - Elastic moduli are the bulk modulus K and shear modulus G (Sec. 2, eq. elast); internally
 *    nu = (3K - 2G) / (2 (3K + G)).  K <= 0, G <= 0 or non-finite moduli are KFMM_E_ARG.
 */
#ifndef KFMM_H
#define KFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KFMM_OK = 0,
  KFMM_E_ARG = -1,    /* invalid argument (sizes, moduli, non-finite coordinates, ...) */
  KFMM_E_OOM = -2,    /* device allocation failed or exceeds opts.mem_limit */
  KFMM_E_HIP = -3,    /* a HIP runtime call failed */
  KFMM_E_NOCONV = -4, /* GMRES did not reach the tolerance within max_iter */
  KFMM_E_STATE = -5   /* object used in a wrong state (e.g. destroyed plan) */
};

/* Internal arithmetic of fmm_eval. */
enum {
  KFMM_FP64 = 0,          /* everything in FP64 (near field, far field, translations) */
  KFMM_FP32 = 1,          /* near field, check/equivalent evaluations, M2L and translations in FP32; the
                             M2M/L2L chains run on scaled check potentials (smooth fields, no cancellation)
                             and the check-to-equivalent pseudo-inverses are applied in their SVD-factored
                             form (an orthogonal rotation, then a column-scaled one), once per box */
  KFMM_FP32_M2L_BF16 = 2, /* withdrawn: every call given it returns KFMM_E_ARG.  A BF16 M2L (8-bit operands,
                             FP32 accumulation) measured ~1e-2 relative error against its 1e-3 target: the
                             equivalent densities cancel strongly; KFMM_FP32_M2L_SPLIT16 uses the matrix cores
                             at FP32 accuracy instead */
  KFMM_FP32_M2L_SPLIT16 = 3, /* as KFMM_FP32 but the M2L contractions, the M2M/L2L translations on check
                               potentials and the orthogonal factors of the pseudo-inverses on the FP16
                               matrix cores: every operator and every input vector, scaled by a power of
                               two, is split into a high and a low FP16 part and the product is accumulated
                               in FP32 from hi*hi + hi*lo + lo*hi (about 22-bit operands, close to FP32
                               accuracy); the column-scaled pseudo-inverse factors stay FP32 */
  KFMM_FP32_TRANS64 = 4     /* near field, check/equivalent evaluations and M2L in FP32 (as KFMM_FP32), the
                               pseudo-inverses and M2M/L2L translations in FP64 on equivalent densities */
};

/* Target kind of fmm_eval. */
enum {
  KFMM_DISP = 0,  /* displacement: 3 components per target */
  KFMM_STRESS = 1 /* stress: 6 components per target, order xx, yy, zz, yz, xz, xy */
};

typedef struct {
  double K, G;        /* bulk and shear modulus */
  int p;              /* equivalent-surface order: p points per cube edge, 6(p-1)^2+2 points; 0 -> 6 */
  int leaf_max;       /* a box is split while it holds more than leaf_max sources + targets; 0 -> 64 */
  int precision;      /* KFMM_FP64, KFMM_FP32, KFMM_FP32_M2L_SPLIT16 or KFMM_FP32_TRANS64 */
  double svd_eps;     /* relative singular-value cutoff of the check-to-equivalent pseudo-inverse; 0 -> 1e-8 */
  int max_depth;      /* deepest octree level; 0 -> 16 */
  size_t mem_limit;   /* bytes of device memory the plan may use; 0 = no limit */
  double m2l_tol;     /* > 0 compresses the M2L onto one shared basis, keeping the singular directions above
                         m2l_tol (relative) of sum_o K_o K_o^T's square root, their count rounded up to the GEMM
                         padding (fmm_info.m2l_rank); 0 = dense.  Every precision: KFMM_FP64 contracts in FP64
                         (with FP64 translations), the others in FP32 or split FP16.  With KFMM_FP64 and
                         KFMM_FP32_M2L_SPLIT16 each offset's operator is further cut to its leading r_o x r_o
                         block, r_o the smallest multiple of 32 whose dropped part stays below m2l_tol / 3 in the
                         same absolute scale */
} fmm_opts;

typedef struct kfmm_plan* kfmm_plan_t;

/*
 * fmm_plan -- build the octree, interaction lists and translation operators for a fixed set of
 * sources (points y_j with normals n_j and weights w_j) and targets x_i (Sec. 2.2, "Kernel-independent
 * fast multipole method": octree, upward/downward passes, near field; eq. fmm_summation).
 *
 *   src_xyz  N x 3  source points                       (device, FP64)
 *   src_nrm  N x 3  unit normals at the sources, or NULL (then only single-layer densities may be used)
 *   src_w    N      source weights (area x quadrature weight), or NULL for all ones
 *   n_src    N >= 0
 *   trg_xyz  M x 3  target points, or NULL: targets are the sources themselves (M must equal N), or no
 *                   targets (M = 0)
 *   n_trg    M >= 0
 *   batch_src, batch_trg  (host) offsets of n_batch independent geometries, n_batch + 1 entries each,
 *            starting at 0 and ending at N (resp. M); or NULL with n_batch <= 1 for one geometry.
 *            Geometries never interact: each has its own root box.
 *   opts     (host) options; see fmm_opts.
 * Coordinates must be finite (checked on the device; KFMM_E_ARG otherwise).  A source that coincides
 * exactly with a target contributes nothing to that target.
 */
int fmm_plan(kfmm_plan_t* out, const double* src_xyz, const double* src_nrm, const double* src_w, int64_t n_src,
             const double* trg_xyz, int64_t n_trg, const int64_t* batch_src, const int64_t* batch_trg,
             int32_t n_batch, const fmm_opts* opts, void* stream);

/*
 * fmm_plan_periodic -- as fmm_plan, for periodic cubic cells (Sec. 4.3, periodic cell of a metamaterial:
 * the integrals run over the infinite periodic surface, and the FMM tree is periodic at every level).
 * Each geometry g is the cell [c_g, c_g + L_g)^3 repeated over the lattice L_g Z^3; fmm_eval then returns
 * the sums of eq. fmm_summation over every lattice image of every source.
 *   cells  (host) n_batch x 4 doubles (n_batch <= 1: one row): lower corner c_g (x, y, z) and side L_g > 0.
 *          Every source and target of geometry g must lie in its cell (KFMM_E_ARG otherwise).
 * The lattice sum of a point force converges only conditionally; it is defined as its Fourier series
 * without the k = 0 term: the periodic field of zero cell mean (a net force per cell is balanced by a
 * uniform body force; the fast evaluation represents that balance only approximately, so single-layer
 * densities should carry no net force per cell).  The image n = 0 of a source that coincides with a
 * target is left out, all other images are kept.  Every precision mode applies.
 */
int fmm_plan_periodic(kfmm_plan_t* out, const double* src_xyz, const double* src_nrm, const double* src_w,
                      int64_t n_src, const double* trg_xyz, int64_t n_trg, const int64_t* batch_src,
                      const int64_t* batch_trg, int32_t n_batch, const double* cells, const fmm_opts* opts,
                      void* stream);

/*
 * fmm_eval -- fast evaluation of the boundary integrals at the plan's targets (eq. fmm_summation):
 *   KFMM_DISP  : out_i   = sum_j U(x_i, y_j) w_j a_j + P(x_i, y_j, n_j) w_j b_j        (eqs. disp_1, disp_2)
 *   KFMM_STRESS: out_i,kl = sum_j D_mkl(x_i, y_j) w_j a_j,m + S_mkl(x_i, y_j, n_j) w_j b_j,m  (eqs. stress_2, stress_3)
 * With a = t and b = -u these are the right-hand sides of eq. BIE and eq. stress_1.
 *   a_sl  N x 3 single-layer density (device, FP64) or NULL (zero)
 *   b_dl  N x 3 double-layer density (device, FP64) or NULL (zero); needs normals in the plan
 *   out   M x 3 (DISP) or M x 6 (STRESS), overwritten (device, FP64), targets in the caller's order.
 */
int fmm_eval(kfmm_plan_t plan, int kind, const double* a_sl, const double* b_dl, double* out, void* stream);

/* Sizes and counters of a plan (host struct). */
typedef struct {
  int64_t n_src, n_trg, n_box, n_leaf;
  int32_t depth, n_eq;
  int64_t n_u_pairs;   /* near-field source-target point pairs (P2P) */
  int64_t n_v_pairs;   /* M2L box pairs */
  int64_t n_w_pairs, n_x_pairs;
  double plan_seconds;
  size_t device_bytes;
  int32_t m2l_rank;    /* rank of the compressed M2L (0: dense) */
} fmm_info;
int fmm_plan_info(kfmm_plan_t plan, fmm_info* info /* host */);

/*
 * fmm_plan_target_lists -- which far-field paths reach each target (a diagnostic for parity tests; the
 * adaptive lists of Sec. 2.2, "Kernel-independent fast multipole method").  For every target, in the
 * caller's order, flags[i] gets bit 0 if its leaf has a W list (upward densities of smaller boxes
 * evaluated at the target), bit 1 if its leaf has an X list (sources of larger boxes evaluated on the
 * leaf's downward check surface) and bit 2 if an ancestor box of the leaf has an X list.
 *   flags  M int32 (host), overwritten.  Synchronises the device (copies the target permutation).
 */
int fmm_plan_target_lists(kfmm_plan_t plan, int32_t* flags /* host */);

/*
 * Phase timing.  fmm_profile(plan, 1) makes every following fmm_eval record HIP events between its
 * phases on the caller's stream and wait for them at the end of the call (so profiled calls are
 * synchronous); fmm_profile(plan, 0) stops it.  Unprofiled calls run the near field on a second
 * stream of the plan, concurrently with the far-field passes; profiled calls run every phase in turn
 * on the caller's stream.  fmm_profile(plan, 2) times only the M2L contraction launch, with a pair of
 * events around it and no other change to the call (no synchronisation, same streams); its summed
 * milliseconds are reported in the KFMM_PH_M2L entry of fmm_phase_times (which then waits for the
 * recorded events), every other entry 0.  fmm_phase_times writes, for each phase, the summed
 * milliseconds over the profiled calls (host array of KFMM_N_PHASES doubles) and their number.
 * Enabling resets the sums.
 */
enum {
  KFMM_PH_PERMUTE = 0, /* densities into tree order */
  KFMM_PH_S2M,         /* sources -> upward check potentials of leaves */
  KFMM_PH_UC2UE,       /* upward check -> equivalent densities of leaves (FP64 translations only) */
  KFMM_PH_M2M,         /* upward translations, all levels (FP32 translations: and then check ->
                          equivalent densities of every box) */
  KFMM_PH_M2L_PREP,    /* clearing and converting for the M2L */
  KFMM_PH_M2L,         /* M2L contraction (matrix cores), all levels */
  KFMM_PH_M2L_RED,     /* sum of the per-pair M2L outputs of every target box (fixed order) */
  KFMM_PH_S2L,         /* X list: sources -> downward check potentials */
  KFMM_PH_DOWN,        /* downward check -> equivalent, L2L, all levels (FP32 translations: L2L on check
                          potentials, then check -> equivalent at the target leaves) */
  KFMM_PH_NEAR,        /* near field (U list) at the target leaves */
  KFMM_PH_LEAF,        /* far field at the target leaves: L2T + W list */
  KFMM_N_PHASES
};
int fmm_profile(kfmm_plan_t plan, int enable);
int fmm_phase_times(kfmm_plan_t plan, double* ms /* host, KFMM_N_PHASES */, int64_t* calls /* host */);

/*
 * fmm_plan_work -- algorithmic work of one fmm_eval of this plan, per phase (the KFMM_PH_* order): the
 * floating-point operations and the HBM bytes the method itself needs (Sec. 2.2 passes: every operator
 * and coefficient vector read once, every result written once, operand sizes without padding), for the
 * roofline of each phase.  Point-pair costs: U 29, P 45, U+P 65, D 50, S 90, D+S 130 operations.
 *   kind            KFMM_DISP or KFMM_STRESS
 *   with_a, with_b  non-zero if the single-layer (resp. double-layer) density is given
 *   flops, bytes    (host) KFMM_N_PHASES doubles each, overwritten
 */
int fmm_plan_work(kfmm_plan_t plan, int kind, int with_a, int with_b, double* flops /* host */,
                  double* bytes /* host */);

/* Release the plan and its device memory.  NULL is a no-op. */
int fmm_plan_destroy(kfmm_plan_t plan);

/* ---------------------------------------------------------------------------------------------------
 * Collocation BEM (Sec. 2.2, "Discretization of BIE", "Matrix-vector products"; eqs. BIE, num, coef, num2).
 * Flat triangles with piecewise-constant displacement and traction, collocation at centroids (free term
 * 1/2 I), 16 quadrature points per triangle (4 midpoint sub-triangles x symmetric 4-point rule), closed-form
 * self integrals in the local pass, unknowns per element and component: u where the traction is prescribed,
 * t where the displacement is prescribed.
 */
typedef struct {
  int64_t n_tri;          /* T > 0 */
  const double* tri_xyz;  /* T x 3 x 3 vertices (device), counter-clockwise seen from outside the body */
  const int8_t* bc_type;  /* T x 3 (device): 0 = displacement prescribed, 1 = traction prescribed */
  const double* bc_val;   /* T x 3 (device): prescribed displacement or traction */
  double K, G;            /* moduli */
  int near_levels;        /* 0: every off-diagonal block by the 16-point rule.  L in 1..5: the blocks of the
                             near pairs (below) by the upsampled rule of Sec. 2.2 ("Matrix-vector products"):
                             the triangle split at its edge midpoints L more times, the element rule on each
                             of the 4^L pieces (16 4^L points), added in the local pass as the difference to
                             the 16-point blocks the fast summation applies */
  double near_radius;     /* a pair (t, e), t != e, is near when |c_t - c_e|^2 < near_radius^2 l_e^2 (c:
                             centroids, l_e: longest edge of e); 0 -> 1.5 */
  const double* cell;     /* (host) NULL for a body in free space, or 4 doubles (lower corner x, y, z, side L):
                             the surface repeats over the lattice L Z^3 and every integral runs over the
                             infinite periodic surface (Sec. 4.3, periodic cell of a metamaterial; products
                             through fmm_plan_periodic, so fmm.precision must be KFMM_FP64).  With the
                             superposition formulation a cell of cavities under a homogeneous stress s^h is
                             the pure traction problem with bc_val = -s^h n on every element: its solution is
                             the periodic fluctuation field (zero cell mean), added to s^h for the total
                             stress.  Every quadrature point and centroid must lie in [c, c + L)^3 (a
                             face on an upper face of the cell is given on the lower one).  Near pairs then
                             include the images of elements across the cell faces (c_e + L s, s in
                             {-1, 0, 1}^3), so near_radius times the longest edge must be below L
                             (KFMM_E_ARG otherwise); precond must be KFMM_PC_NONE (its exact blocks are
                             free-space). */
} bem_problem;

typedef struct {
  double tol;      /* stop when ||b - A x|| / ||b|| <= tol (true residual) */
  int restart;     /* GMRES restart length m (1..500) */
  int max_iter;    /* maximum number of Arnoldi steps (matrix-vector products); 0 evaluates x0 only */
  fmm_opts fmm;    /* options of the fast summation behind every product (K, G are taken from the problem;
                      svd_eps 0 means 1e-7 here: smaller equivalent densities, lower rounding floor) */
  const double* x0_alt; /* optional second start (device, T x 3, physical units), NULL for none.  GMRES starts
                           from the minimal-residual combination a x0 + c x0_alt (a alone without x0_alt),
                           from the products A x0, A x0_alt (one extra product); a start still worse than
                           zero is replaced by zero. */
  int precond;     /* KFMM_PC_NONE or KFMM_PC_TWO_LEVEL (right preconditioning: the residual GMRES reduces and
                      the stopping test stay the true ||b - A x||) */
  int pc_fine;     /* elements per fine block, 1..32; 0 -> 32 */
  int pc_coarse;   /* elements per coarse aggregate; 0 -> 64, doubled while 6 ceil(T / size) > 4096 */
} bem_opts;

/* Preconditioners of bem_solve (the paper leaves the preconditioning of mixed problems open, Sec. 5,
 * "Discussion and future work"). */
enum {
  KFMM_PC_NONE = 0,
  KFMM_PC_TWO_LEVEL = 1 /* two-level additive Schwarz: M^-1 = sum_b R_b^T (R_b A R_b^T)^-1 R_b + Z (Z^T A Z)^-1 Z^T.
                           Elements ordered along the Morton curve of their centroids (14 bits per axis);
                           fine blocks of pc_fine consecutive elements (their exact 3m x 3m blocks of A,
                           inverted); aggregates of pc_coarse consecutive elements, each contributing its
                           local rigid motions as coarse columns (three translations of every unknown, three
                           rotations about the aggregate's mean centroid at the displacement unknowns),
                           orthonormalised (modified Gram-Schmidt, two passes; a column keeping at most 1e-8
                           of its raw norm is dropped); E = Z^T A Z summed directly in FP64 and inverted. */
};

typedef struct {   /* host */
  int iters, restarts, converged;
  int used_alt;        /* 1 if x0_alt entered the start (c != 0) */
  int used_zero;       /* 1 if both given starts were worse than zero and zero was used */
  double rel_res_alt;  /* true relative residual of x0_alt (if given) */
  double rel_res_start; /* relative residual of the start GMRES iterates from (the minimal-residual combination,
                            or 1 when the guard fell back to zero); 0 without a start */
  double start_coef[2]; /* the coefficients a, c of the start */
  int64_t n_matvec;
  double rel_res;      /* true relative residual of the returned x */
  double rel_res0;     /* true relative residual of x0 */
  double res_estimate; /* last GMRES estimate */
  double b_norm;
  double t_setup_s, t_solve_s;
  double t_precond_s;   /* preconditioner set-up (included in t_setup_s) */
  int64_t pc_coarse_dim; /* columns of Z kept (0 without the preconditioner) */
} bem_stats;

/*
 * bem_solve -- solve A x = B y (eq. num2) by restarted GMRES, every product through fmm_eval plus the local
 * pass.  x0 (device, T x 3) or NULL for zero, and x (device, T x 3), hold the unknowns in physical units
 * (inside the solver traction unknowns are scaled by -l/G, l = mean edge length; residuals refer to that system).  u_full, t_full (device, T x 3, may be NULL) receive the complete
 * boundary displacement and traction.  stats (host) may be NULL.  Returns KFMM_E_NOCONV (x and stats filled)
 * if the tolerance is not reached within max_iter.  Synchronises the stream.
 */
int bem_solve(const bem_problem* prob, const bem_opts* opts, const double* x0, double* x, double* u_full,
              double* t_full, bem_stats* stats, void* stream);

/*
 * bem_stress -- interior stress from a boundary solution (eq. stress_1): sigma = int D t - int S u, with the
 * same 16-point quadrature.  u_full, t_full: T x 3 (device); trg: M x 3 (device); out: M x 6 (device, xx, yy,
 * zz, yz, xz, xy).  Builds and destroys a plan internally.  Synchronises the stream.
 */
int bem_stress(const bem_problem* prob, const double* u_full, const double* t_full, const double* trg, int64_t M,
               double* out, const fmm_opts* fmm, void* stream);

/*
 * bem_matvec -- one product of the discrete system, as used inside bem_solve:
 *   which = 0: y = A x   (x in solver units: traction unknowns scaled by -l/G),
 *   which = 1: y = B y_prescribed (right-hand side; x ignored).
 * x, y: T x 3 (device).  Builds a plan internally.  Synchronises the stream.
 */
int bem_matvec(const bem_problem* prob, const fmm_opts* fmm, int which, const double* x, double* y, void* stream);

/*
 * bem_near_pairs -- the near pairs of prob (near_radius as in bem_problem; near_levels is ignored; a periodic
 * cell is KFMM_E_ARG: the (t, e) rows carry no image shift, so this entry point serves free-space surfaces
 * only, while the solver's own near pairs on a periodic surface include the images), sorted by collocation
 * element t, then by source element e.  *count (host) receives their number; pairs (device,
 * 2 x count int32 as (t, e) rows) may be NULL to query the count, else it must hold *count_capacity pairs
 * (KFMM_E_ARG if fewer).  Synchronises the stream.
 */
int bem_near_pairs(const bem_problem* prob, int64_t* count, int32_t* pairs, int64_t count_capacity, void* stream);

/* ---------------------------------------------------------------------------------------------------
 * Algorithm 1 (Sec. 2.3) on the device: the voxel steps of an optimisation iteration and the adaptive
 * sampling of the interior (Sec. 2.2 end, Sec. 5 "adaptive grid").  A design is a uint8 array (device,
 * nonzero = material) of nx x ny x nz voxels of edge h in C order (i slowest), origin at 0; voxel (i, j, k)
 * spans [i h, (i + 1) h] x [j h, (j + 1) h] x [k h, (k + 1) h].  Outputs follow linear voxel order and are
 * bitwise reproducible.  Calls that return a count take NULL outputs to query it; capacity is the number
 * of rows the output holds (KFMM_E_ARG if fewer).  All synchronise the stream.
 */
typedef struct {
  int nx, ny, nz; /* voxels per axis, nx * ny * nz < 2^31 */
  double h;       /* voxel edge */
} alg1_grid;

/* alg1_surface -- the boundary of the material as triangles with the cantilever's conditions.  Every face of
 * a filled voxel whose neighbour across it is empty or outside gives four triangles (q_e, q_{e+1}, centre),
 * e = 0..3, counter-clockwise seen from outside; faces in six classes (axis 0, +), (axis 0, -), (axis 1, +),
 * ..., each in linear voxel order; corners h p for the grid points p of the face from (0,0), (1,0), (1,1),
 * (0,1) along the axes a + 1, a + 2 (reversed on - faces), centre (((q0 + q1) + q2) + q3) / 4.  The x = 0
 * faces of the voxels with i = 0 are clamped (bc_type 0, value 0), the +x faces of the voxels with
 * i = nx - 1 carry the traction load (host, 3; NULL -> (0, 0, -1)), all other faces are traction-free.
 * tri: T x 3 x 3, bc_type T x 3, bc_val T x 3, owner T x 3 (int32 voxel index, may be NULL). */
int alg1_surface(const alg1_grid* grid, const uint8_t* vox, const double* load, int64_t* n_tri, double* tri,
                 int8_t* bc_type, double* bc_val, int32_t* owner, int64_t capacity, void* stream);

/* alg1_centres -- centres (idx + 1/2) h of the filled voxels (n x 3), the interior points of eq. stress_1. */
int alg1_centres(const alg1_grid* grid, const uint8_t* vox, int64_t* n, double* pts, int64_t capacity, void* stream);

/* alg1_update -- the removal rule of Algorithm 1 with post-processing: td holds one topological derivative
 * per filled voxel (linear order; n_td must equal their number, else KFMM_E_ARG); a filled voxel becomes empty when td < D_min + C (D_max - D_min) (strict),
 * except in the layers i = 0 and i = nx - 1 (the supports); then only the material face-connected to both
 * of those layers is kept.  out (device, nx ny nz, must not alias vox) receives the new design, *n_filled
 * (host, may be NULL) its number of filled voxels. */
int alg1_update(const alg1_grid* grid, const uint8_t* vox, const double* td, int64_t n_td, double C, uint8_t* out,
                int64_t* n_filled, void* stream);

/* Adaptive sampling with blocks of b^3 voxels (block grid ceil(n / b) per axis, linear order):
 * alg1_coarse_blocks -- centres ((I + 1/2) b h, ...) of the blocks all of whose voxels are filled.
 * alg1_refine -- with td_coarse (one value per full block, in that order): a block is refined unless it is
 *   full and its six face neighbours are full blocks with the same decision td < lo + C (hi - lo) (lo, hi
 *   over td_coarse; n_coarse must equal the number of full blocks); returns the centres of the filled voxels of refined blocks (linear order) and, when
 *   refined (device, one byte per block) is not NULL, the mask.
 * alg1_expand -- one value per filled voxel (linear order): its own value from td_fine (in alg1_refine's
 *   order; n_fine must equal their number) in a refined block, else its block's coarse value; alg1_update applies the rule to this field. */
int alg1_coarse_blocks(const alg1_grid* grid, const uint8_t* vox, int block, int64_t* n, double* pts,
                       int64_t capacity, void* stream);
int alg1_refine(const alg1_grid* grid, const uint8_t* vox, int block, const double* td_coarse, int64_t n_coarse,
                double C, int64_t* n, double* pts, int64_t capacity, uint8_t* refined, void* stream);
int alg1_expand(const alg1_grid* grid, const uint8_t* vox, int block, const double* td_coarse, int64_t n_coarse,
                double C, const double* td_fine, int64_t n_fine, double* td_out, void* stream);

/* Periodic cell of a metamaterial (Sec. 4.3), the design a cubic cell [0, nx h) x [0, ny h) x [0, nz h)
 * repeated over the lattice (the cell's own faces are not boundary):
 * alg1_cell_surface -- the void/material faces with neighbours taken periodically (a voxel of the last layer
 *   faces the first layer's image), in alg1_surface's classes, order and corner convention; a face on an
 *   upper plane of the cell is emitted on the lower one (coordinate 0), so every quadrature point and
 *   centroid lies in the cell.  Every element gets the traction of the superposition formulation,
 *   bc_type 1, bc_val = -sig_h n (sig_h host, 6 values xx, yy, zz, yz, xz, xy; n the face normal out of
 *   the material): the problem of the fluctuation field under the homogeneous stress sig_h.
 * alg1_cell_td -- the topological derivative (eq. deriv) of the total stress sig6 + sig_h at M points.
 * alg1_cell_update -- the single-iteration rule of the paper's metamaterial example: keep the material
 *   with the largest td so that round(alpha nx ny nz) voxels stay filled (td one value per filled voxel in
 *   linear order, n_td their number; ties by linear order; nothing is removed when the design already
 *   holds no more).  out (device, must not alias vox) receives the new design, *n_filled (host, may be
 *   NULL) its number of filled voxels. */
int alg1_cell_surface(const alg1_grid* grid, const uint8_t* vox, const double* sig_h, int64_t* n_tri, double* tri,
                      int8_t* bc_type, double* bc_val, int32_t* owner, int64_t capacity, void* stream);
int alg1_cell_td(const double* sig6, int64_t M, const double* sig_h, double K, double G, double* td, void* stream);
int alg1_cell_update(const alg1_grid* grid, const uint8_t* vox, const double* td, int64_t n_td, double alpha,
                     uint8_t* out, int64_t* n_filled, void* stream);

/* alg1_energy -- compliance integrand: *psi (host) = sum over the n stresses (n x 6, device) of
 * (1 / 2E) [(1 + nu) sigma:sigma - nu (tr sigma)^2] (fixed summation order); times h^3 it is the compliance
 * of a voxel design evaluated at the voxel centres. */
int alg1_energy(const double* sig6, int64_t n, double K, double G, double* psi, void* stream);

/* Sizes of a built preconditioner (host). */
typedef struct {
  int64_t n_fine_blocks, n_aggregates, n_coarse; /* n_coarse = 6 n_aggregates (dropped columns included) */
  int fine, coarse, n_dropped;
  double t_setup_s;
} bem_pc_info;

/*
 * bem_precond_apply -- y = M^-1 v for the preconditioner opts->precond (KFMM_PC_TWO_LEVEL) of the system
 * bem_solve builds for prob and opts (solver units: traction unknowns scaled by -l/G).  v, y: T x 3 (device,
 * must not overlap).  info (host) may be NULL.  Builds the system and the preconditioner internally; returns
 * KFMM_E_ARG for KFMM_PC_NONE, block sizes out of range, or a singular block.  Synchronises the stream.
 */
int bem_precond_apply(const bem_problem* prob, const bem_opts* opts, const double* v, double* y, bem_pc_info* info,
                      void* stream);

/* bem_quadrature -- the 16 quadrature points per triangle (device, 16T x 3), their normals (16T x 3),
 * weights (16T) and the collocation points (T x 3).  Synchronises the stream. */
int bem_quadrature(int64_t n_tri, const double* tri_xyz, double* qp, double* qn, double* qw, double* colloc,
                   void* stream);

/*
 * kfmm_topological_derivative -- pointwise topological derivative of the compliance (Sec. 2, eq. deriv):
 *   D = 3 (1 - nu) / (4 E (7 - 5 nu)) [10 (1 + nu) sig:sig - (1 + 5 nu) (tr sig)^2]
 * sig6: M x 6 stresses (xx, yy, zz, yz, xz, xy, device FP64), td: M (device FP64).  E, nu from (K, G).
 */
int kfmm_topological_derivative(const double* sig6, int64_t M, double K, double G, double* td, void* stream);

/* ---------------------------------------------------------------------------------------------------
 * Learned GMRES warm start.  The paper suggests reusing the previous iteration's boundary solution when the
 * boundary changes little (Sec. 5, fast update of the boundary solution); here a point-wise MLP
 * (16 -> 128 -> 128 -> 3, SiLU) learns, online, the correction from the previous solution mapped onto the
 * new surface to the new solution.  Inference uses BF16 matrix cores; training FP32 with Adam.  The solve's
 * accuracy never depends on the network: GMRES runs to the same residual from whatever start it is given.
 */
#define KFMM_WS_DIN 16
typedef struct ws_net* ws_net_t;

/* Create a network (d_in must be KFMM_WS_DIN, width 128); weights drawn from a counter-based generator. */
int ws_create(ws_net_t* out, int d_in, int width, uint64_t seed);
int ws_destroy(ws_net_t net);

/*
 * ws_features -- per element of `next`: the nearest element of `prev` (by centroid, exact matches at
 * distance 0), the previous solution mapped into next's unknown layout (x_mapped, T' x 3, device: the
 * previous t where next prescribes u, the previous u where it prescribes t) and KFMM_WS_DIN features
 * (feat, T' x 16, device FP32).  u_prev, t_prev: previous full boundary solution (T x 3, device).
 * *scale (host) receives the RMS of x_mapped used to normalise features and targets.  Synchronises.
 */
int ws_features(const bem_problem* prev, const double* u_prev, const double* t_prev, const bem_problem* next,
                float* feat, double* x_mapped, double* scale, void* stream);

/* ws_predict -- x0 = x_mapped + scale * net(feat)   (device, n x 3). */
int ws_predict(ws_net_t net, const float* feat, int64_t n, const double* x_mapped, double scale, double* x0,
               void* stream);

/* ws_train -- `epochs` full-batch Adam steps (learning rate lr) on the target (x_target - x_mapped) / scale;
 * *loss (host) receives the last mean squared error.  Synchronises. */
int ws_train(ws_net_t net, const float* feat, const double* x_mapped, const double* x_target, int64_t n,
             double scale, int epochs, float lr, float* loss, void* stream);

/* Parameters as one host FP32 vector: W1 (16x128, [in][out]), b1, W2 (128x128), b2, W3 (128x3), b3. */
int ws_num_params(ws_net_t net, int64_t* n);
int ws_get_params(ws_net_t net, float* host);
int ws_set_params(ws_net_t net, const float* host);
/*
 * ws_train_noalloc -- ws_train for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same arguments, kernels and results
 * as ws_train, but the per-call work buffers (activations, gradients, residual targets, partial sums)
 * live in a static device array of the library (128 MiB, one copy per GPU, held until the process ends)
 * instead of memory the network allocates on first use; the call allocates nothing.
 *   n  1 <= n <= KFMM_WS_NOALLOC_MAX_ROWS (larger n: KFMM_E_ARG, nothing runs)
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (several streams or
 * host threads) race and must be serialised by the caller.  Each call writes every word of the array
 * it reads before reading it, so nothing carries over from an earlier call.  Synchronises the stream
 * (it returns the loss).
 */
#define KFMM_WS_NOALLOC_MAX_ROWS 40000
int ws_train_noalloc(ws_net_t net, const float* feat, const double* x_mapped, const double* x_target, int64_t n,
                     double scale, int epochs, float lr, float* loss /* host, may be NULL */, void* stream);
/* Test hook: loss and gradient (host, ws_num_params entries) for features X and residual targets R
 * (device FP32, n x 16 and n x 3). */
int ws_loss_grad(ws_net_t net, const float* X, const float* R, int64_t n, float* loss, float* grad, void* stream);
/* Save / load parameters and Adam state (host path). */
int ws_save(ws_net_t net, const char* path);
int ws_load(ws_net_t net, const char* path);

/*
 * Test hook: one launch of the batched gather/scatter GEMM used by every translation,
 *   Y[:, out[j]] (=, +=, atomic +=) scale[j] * A[op[j]] * X[:, in[j]]
 * precision 0: A, X, Y FP64; 1: FP32; 3: A, X, Y FP32 with the products on
 * the FP16 matrix cores (A and X split into high and low FP16 parts, see KFMM_FP32_M2L_SPLIT16; NC a
 * multiple of 96 or 64).  A holds NC x NC row-major operators,
 * X and Y hold NC-vectors (stride NC).  op, in, out, scale (scale may be NULL) are HOST arrays of ncols
 * entries with op non-decreasing; NC must be a multiple of 96 or 128.  Synchronises the stream.
 * precision + 16 * k selects the FP64 / FP32 kernel: k = 0 as the library chooses, 1 the LDS-tiled
 * kernel, 2 the split-K kernel used for launches with few columns, 3 / 4 the LDS-tiled kernel with one /
 * two LDS buffers.  With precision 3, k = 1 runs 64-column tiles (the width of the translation passes)
 * instead of the M2L's 128.
 */
int kfmm_selftest_gemm(int precision, const void* A, int NC, const void* X, void* Y, const int* op, const int* in,
                       const int* out, const double* scale, int ncols, int mode, void* stream);

/* Last error message of the calling thread ("" if none); valid until the next call on this thread. */
const char* kfmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KFMM_H */
