// FMM plan object: tree, lists, operator handles, work buffers and per-pass launch descriptors.
#pragma once
#include <memory>
#include <vector>

#include "../../include/kfmm.h"
#include "common.h"
#include "gemm.h"
#include "tree.h"

namespace kfmm {

struct DeviceOps;
struct CompressedM2L;

// Read-only device view of the box arrays passed to kernels by value.
struct TreeView {
  const int *level, *ix, *iy, *iz, *geom;
  const double *root_c, *root_R;
  const int *src_b, *src_e, *trg_b, *trg_e;
};

struct UpLevel {
  GemmJob job;          // T(child) = M2M_octant(child) * phi_up(child), children of one level
  int n_par = 0;        // parents (non-leaf boxes with sources) of that level
  int* parents = nullptr;
};

struct Plan {
  fmm_opts opts{};
  Elastic el{};
  int prec = 0;
  bool alias = false, has_nrm = false, empty = false;
  // FP32 translations (KFMM_FP32, KFMM_FP32_M2L_SPLIT16): M2M and L2L on check potentials and factored
  // pseudo-inverses, in FP32 on FP32 buffers; otherwise the translations run in FP64
  bool f32t = false;
  // split FP16 with the compressed M2L: U q~ and the L2L into a leaf carry the leaf's fd1 (the first factor of
  // DC2DE), so a leaf's row of the downward pass holds fd1 qhat and no separate fd1 product runs
  bool fold_fd1 = false;
  int64_t n_src = 0, n_trg = 0;
  int NC = 0, n_eq = 0;
  std::shared_ptr<DeviceOps> ops;
  // periodic cells: levels 0 and 1 take part in the translations, and job_per adds the far-image operator
  // to the root's downward check potential
  bool periodic = false;
  GemmJob job_per, job_per_c;  // roots in place / into compact rows (FP32 translations: T UC2UE qhat_up)
  float* per_tmp_f = nullptr;  // compact rows of the far images' check potential (FP32 translations)
  double* per_eqm = nullptr;   // the equivalent density's second moments, 6 per root
  // periodic displacement: the cell-mean constant per root (second moments of the sources in chunks of
  // sources, then per root with the equivalent density), subtracted from the root's target rows
  int per_n_roots = 0, per_n_chunks = 0;
  int *per_root = nullptr, *per_chunk_off = nullptr, *per_trg_b = nullptr, *per_trg_e = nullptr;
  int *per_chunk_b = nullptr, *per_chunk_e = nullptr, *per_chunk_root = nullptr;
  double* per_part = nullptr;  // 6 per chunk
  Arena arena;
  Tree tree;
  TreeView tv{};
  // sorted, leaf-local point data (precision-dependent element type)
  void *spos = nullptr, *snrm = nullptr, *tpos = nullptr, *dens = nullptr;
  double* sw = nullptr;
  // launch lists
  int n_leaves_src = 0, n_leaves_trg = 0, n_x_boxes = 0;
  int *leaves_src = nullptr, *leaves_trg = nullptr, *x_boxes = nullptr;
  GemmJob job_uc2ue, job_m2l, job_dc2de;
  // FP32 translations: UC2UE over every box with sources at level >= 2, DC2DE over the target leaves
  GemmJob job_up_all, job_dn_leaf;
  GemmJob job_up_w;  // compressed M2L: the W-list source boxes (the only full equivalent densities read)
  // compressed M2L (FP32 with opts.m2l_tol > 0)
  std::shared_ptr<CompressedM2L> comp;
  GemmJob job_ut, job_dcx;  // U^T projection of source boxes; DC2DE of the X-list rows
  float* phi_t = nullptr;   // U^T phi_up per box (n_box x NCr)
  double* q_t = nullptr;    // reduced compressed check potentials (n_box x NCr)
  // KFMM_FP32_M2L_SPLIT16: M2L source vectors split into FP16 high / low parts, power-of-two scale per box
  uint16_t* phi_h3 = nullptr;
  float* phi_h3_scale = nullptr;
  uint16_t* phi_up_h3 = nullptr;  // compressed case: phi_up split the same way (input of the U^T projection)
  float* phi_up_h3_scale = nullptr;
  // M2L: per-pair output slots (FP64 or FP32) and their fixed-order reduction per target box
  void* m2l_slots = nullptr;
  double* phi_t64 = nullptr;  // KFMM_FP64 with the compressed M2L: phi~ = U^T phi_up per box
  int m2l_red_n = 0;
  int *m2l_red_box = nullptr, *m2l_red_off = nullptr, *m2l_red_idx = nullptr;
  std::vector<UpLevel> up_levels;
  std::vector<GemmJob> dn_levels;

  std::vector<int> dn_lv;  // level of the children of each dn_levels job
  // per-box coefficient buffers (n_box x NC): FP64 translations
  double *q_up = nullptr, *phi_up = nullptr, *phi_dn = nullptr, *tmp = nullptr;
  // FP32 translations: check potentials (upward, then downward qhat), work rows, reduced compressed check
  // potentials (n_box x NCr) and X-list rows; the equivalent densities are phi_up_lo / phi_dn_lo
  float *q_f = nullptr, *tmp_f = nullptr, *q_t_f = nullptr, *qx_f = nullptr;
  float* tmp_w = nullptr;  // fu1 qhat of the W-list source boxes (merged compressed path, second stream)
  void *phi_up_lo = nullptr, *phi_dn_lo = nullptr;
  // W pairs (CSR order of the W lists): one output slot of nt(B) x 6 doubles each
  int n_wp = 0;
  int *wp_b = nullptr, *wp_a = nullptr;
  signed char* wp_s = nullptr;  // lattice shift code of each pair (periodic cells)
  int64_t* wslot_off = nullptr;
  double* wslot = nullptr;
  // X-list check potentials, one compact row per box of x_boxes; computed per X pair (one row each, in
  // list order) and summed per box
  double* qx = nullptr;
  int n_xp = 0;
  int *xp_b = nullptr, *xp_a = nullptr;                       // pair -> target box, source box
  signed char* xp_s = nullptr;                                // pair -> lattice shift code
  int *xr_box = nullptr, *xr_off = nullptr, *xr_idx = nullptr;  // per-box reduction of the pair rows
  void* xslot = nullptr;
  // second stream (near field, X and W lists) and its fork / join events
  hipStream_t near_stream = nullptr;
  hipEvent_t fork_ev = nullptr, phi_ev = nullptr, x_ev = nullptr, join_ev = nullptr;
  hipEvent_t wq_ev = nullptr;  // second stream done reading the upward check potentials
  // optional phase timing with HIP events (see fmm_profile); light: M2L launch only, events in a ring
  bool prof = false;
  bool light = false;
  static constexpr int kLightRing = 64;
  hipEvent_t lev[2 * kLightRing] = {};
  int lev_head = 0, lev_count = 0;
  hipEvent_t ev[KFMM_N_PHASES + 1] = {};
  double phase_ms[KFMM_N_PHASES] = {};
  int64_t prof_calls = 0;
  // counters
  int64_t n_leaf = 0, n_u_pairs = 0, n_v_pairs = 0, n_w_pairs = 0, n_x_pairs = 0;
  double plan_seconds = 0;
  ~Plan();
};

// cells: empty for free space, else n_geom x 4 (lower corner, side) of periodic cubic cells.
Plan* plan_create(const double* src, const double* nrm, const double* w, int64_t n_src, const double* trg,
                  int64_t n_trg, const std::vector<int64_t>& bs, const std::vector<int64_t>& bt, const fmm_opts& o,
                  hipStream_t s, const std::vector<double>& cells = {});
void plan_eval(Plan& P, int kind, const double* a, const double* b, double* out, hipStream_t s);
void plan_profile(Plan& P, int mode);
void plan_light_harvest(Plan& P, bool all);
int plan_m2l_rank(const Plan& P);
void plan_work(const Plan& P, int kind, bool sl, bool dl, double* flops, double* bytes);

}  // namespace kfmm
