// C-ABI entry points (include/kfmm.h): argument validation, status codes and thread-local errors.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>
#include <cstring>
#include <string>

#include "../../include/kfmm.h"
#include "common.h"
#include "bem.h"
#include "learn.h"
#include "precond.h"
#include "plan.h"

namespace kfmm {
static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace kfmm

struct kfmm_plan {
  kfmm::Plan* impl;
};

using namespace kfmm;

template <typename F>
static int guarded(F&& f) {
  try {
    set_last_error("");
    f();
    return KFMM_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return KFMM_E_OOM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return KFMM_E_HIP;
  }
}

static void check_moduli(double K, double G) {
  KFMM_REQUIRE(std::isfinite(K) && std::isfinite(G) && K > 0 && G > 0, "moduli K and G must be finite and positive");
}

static int make_plan(kfmm_plan_t* out, const double* src_xyz, const double* src_nrm, const double* src_w,
                     int64_t n_src, const double* trg_xyz, int64_t n_trg, const int64_t* batch_src,
                     const int64_t* batch_trg, int32_t n_batch, bool periodic, const double* cells,
                     const fmm_opts* opts, void* stream) {
  return guarded([&] {
    KFMM_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    KFMM_REQUIRE(opts != nullptr, "opts is NULL");
    KFMM_REQUIRE(!periodic || cells != nullptr, "cells is NULL");
    check_moduli(opts->K, opts->G);
    KFMM_REQUIRE(n_src >= 0 && n_trg >= 0, "negative size");
    KFMM_REQUIRE(n_src < (int64_t)1 << 31 && n_trg < (int64_t)1 << 31, "too many points (max 2^31 - 1)");
    KFMM_REQUIRE(n_src == 0 || src_xyz != nullptr, "src_xyz is NULL");
    // trg_xyz NULL: the targets are the sources (n_trg == n_src), or there are none (n_trg == 0)
    if (trg_xyz == nullptr) KFMM_REQUIRE(n_trg == n_src || n_trg == 0, "aliased targets need n_trg == n_src");
    KFMM_REQUIRE(opts->precision >= KFMM_FP64 && opts->precision <= KFMM_FP32_TRANS64, "unknown precision");
    KFMM_REQUIRE(opts->precision != KFMM_FP32_M2L_BF16, kBf16Withdrawn);
    KFMM_REQUIRE(opts->p == 0 || (opts->p >= 3 && opts->p <= 12), "p must be in [3, 12]");
    KFMM_REQUIRE(opts->leaf_max >= 0 && opts->max_depth >= 0, "negative leaf_max or max_depth");
    KFMM_REQUIRE(opts->m2l_tol >= 0 && opts->m2l_tol < 1, "m2l_tol must be in [0, 1)");
    KFMM_REQUIRE(n_batch >= 0 && n_batch <= 128, "n_batch must be in [0, 128]");
    std::vector<int64_t> bs, bt;
    if (n_batch <= 1 || batch_src == nullptr) {
      KFMM_REQUIRE(n_batch <= 1, "batch offsets are NULL");
      bs = {0, n_src};
      bt = {0, n_trg};
    } else {
      KFMM_REQUIRE(batch_trg != nullptr || trg_xyz == nullptr, "batch_trg is NULL");
      bs.assign(batch_src, batch_src + n_batch + 1);
      bt = trg_xyz ? std::vector<int64_t>(batch_trg, batch_trg + n_batch + 1)
                   : (n_trg == n_src ? bs : std::vector<int64_t>(n_batch + 1, 0));
      KFMM_REQUIRE(bs.front() == 0 && bs.back() == n_src && bt.front() == 0 && bt.back() == n_trg,
                   "batch offsets must start at 0 and end at the point counts");
      for (int g = 0; g < n_batch; ++g)
        KFMM_REQUIRE(bs[g + 1] >= bs[g] && bt[g + 1] >= bt[g], "batch offsets must be non-decreasing");
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> cv;
    if (cells) cv.assign(cells, cells + 4 * (size_t)(bs.size() - 1));
    Plan* p = plan_create(src_xyz, src_nrm, src_w, n_src, trg_xyz, n_trg, bs, bt, *opts, s, cv);
    *out = new kfmm_plan{p};
  });
}

extern "C" int fmm_plan(kfmm_plan_t* out, const double* src_xyz, const double* src_nrm, const double* src_w,
                        int64_t n_src, const double* trg_xyz, int64_t n_trg, const int64_t* batch_src,
                        const int64_t* batch_trg, int32_t n_batch, const fmm_opts* opts, void* stream) {
  return make_plan(out, src_xyz, src_nrm, src_w, n_src, trg_xyz, n_trg, batch_src, batch_trg, n_batch, false,
                   nullptr, opts, stream);
}

extern "C" int fmm_plan_periodic(kfmm_plan_t* out, const double* src_xyz, const double* src_nrm,
                                 const double* src_w, int64_t n_src, const double* trg_xyz, int64_t n_trg,
                                 const int64_t* batch_src, const int64_t* batch_trg, int32_t n_batch,
                                 const double* cells, const fmm_opts* opts, void* stream) {
  return make_plan(out, src_xyz, src_nrm, src_w, n_src, trg_xyz, n_trg, batch_src, batch_trg, n_batch, true, cells,
                   opts, stream);
}

extern "C" int fmm_eval(kfmm_plan_t plan, int kind, const double* a_sl, const double* b_dl, double* out,
                        void* stream) {
  return guarded([&] {
    KFMM_REQUIRE(plan != nullptr && plan->impl != nullptr, "plan is NULL");
    KFMM_REQUIRE(kind == KFMM_DISP || kind == KFMM_STRESS, "kind must be KFMM_DISP or KFMM_STRESS");
    Plan& P = *plan->impl;
    KFMM_REQUIRE(out != nullptr || P.n_trg == 0, "out is NULL");
    KFMM_REQUIRE(b_dl == nullptr || P.has_nrm || P.n_src == 0, "double-layer density needs normals in the plan");
    plan_eval(P, kind, a_sl, b_dl, out, (hipStream_t)stream);
  });
}

extern "C" int fmm_plan_info(kfmm_plan_t plan, fmm_info* info) {
  return guarded([&] {
    KFMM_REQUIRE(plan != nullptr && plan->impl != nullptr && info != nullptr, "NULL argument");
    Plan& P = *plan->impl;
    std::memset(info, 0, sizeof(*info));
    info->n_src = P.n_src;
    info->n_trg = P.n_trg;
    info->n_box = P.tree.n_box;
    info->n_leaf = P.n_leaf;
    info->depth = P.tree.depth;
    info->n_eq = P.n_eq;
    info->n_u_pairs = P.n_u_pairs;
    info->n_v_pairs = P.n_v_pairs;
    info->n_w_pairs = P.n_w_pairs;
    info->n_x_pairs = P.n_x_pairs;
    info->plan_seconds = P.plan_seconds;
    info->device_bytes = P.arena.bytes;
    info->m2l_rank = plan_m2l_rank(P);
  });
}

extern "C" int fmm_plan_target_lists(kfmm_plan_t plan, int32_t* flags) {
  return guarded([&] {
    KFMM_REQUIRE(plan != nullptr && plan->impl != nullptr && flags != nullptr, "NULL argument");
    Plan& P = *plan->impl;
    if (P.n_trg == 0) return;
    std::memset(flags, 0, sizeof(int32_t) * (size_t)P.n_trg);
    const Tree& t = P.tree;
    if (P.empty || t.n_box == 0 || t.perm_trg == nullptr) return;
    std::vector<int> perm((size_t)P.n_trg);
    KFMM_HIP(hipMemcpy(perm.data(), t.perm_trg, sizeof(int) * perm.size(), hipMemcpyDeviceToHost));
    auto has = [](const std::vector<int>& off, int b) { return off.size() > (size_t)b + 1 && off[b + 1] > off[b]; };
    for (int b = 0; b < t.n_box; ++b) {
      if (!t.h_is_leaf[b]) continue;
      int32_t f = (has(t.h_w_off, b) ? 1 : 0) | (has(t.h_x_off, b) ? 2 : 0);
      for (int a = t.h_parent[b]; a >= 0; a = t.h_parent[a])
        if (has(t.h_x_off, a)) f |= 4;
      for (int i = t.h_trg_b[b]; i < t.h_trg_e[b]; ++i) flags[perm[i]] = f;
    }
  });
}

extern "C" int fmm_plan_work(kfmm_plan_t plan, int kind, int with_a, int with_b, double* flops, double* bytes) {
  return guarded([&] {
    KFMM_REQUIRE(plan != nullptr && plan->impl != nullptr && flops != nullptr && bytes != nullptr, "NULL argument");
    KFMM_REQUIRE(kind == KFMM_DISP || kind == KFMM_STRESS, "kind must be KFMM_DISP or KFMM_STRESS");
    KFMM_REQUIRE(with_b == 0 || plan->impl->has_nrm || plan->impl->n_src == 0,
                 "double-layer density needs normals in the plan");
    plan_work(*plan->impl, kind, with_a != 0, with_b != 0, flops, bytes);
  });
}

extern "C" int fmm_profile(kfmm_plan_t plan, int enable) {
  return guarded([&] {
    KFMM_REQUIRE(plan != nullptr && plan->impl != nullptr, "plan is NULL");
    KFMM_REQUIRE(enable >= 0 && enable <= 2, "enable must be 0, 1 or 2");
    plan_profile(*plan->impl, enable);
  });
}

extern "C" int fmm_phase_times(kfmm_plan_t plan, double* ms, int64_t* calls) {
  return guarded([&] {
    KFMM_REQUIRE(plan != nullptr && plan->impl != nullptr && ms != nullptr, "NULL argument");
    if (plan->impl->light) plan_light_harvest(*plan->impl, true);
    for (int i = 0; i < KFMM_N_PHASES; ++i) ms[i] = plan->impl->phase_ms[i];
    if (calls) *calls = plan->impl->prof_calls;
  });
}

extern "C" int fmm_plan_destroy(kfmm_plan_t plan) {
  return guarded([&] {
    if (!plan) return;
    delete plan->impl;
    plan->impl = nullptr;
    delete plan;
  });
}

static void check_problem(const bem_problem* p) {
  KFMM_REQUIRE(p != nullptr, "problem is NULL");
  KFMM_REQUIRE(p->n_tri > 0 && p->n_tri < ((int64_t)1 << 27), "n_tri must be in [1, 2^27)");
  KFMM_REQUIRE(p->tri_xyz && p->bc_type && p->bc_val, "problem arrays are NULL");
  check_moduli(p->K, p->G);
  KFMM_REQUIRE(p->near_levels >= 0 && p->near_levels <= 5, "near_levels must be in [0, 5]");
  KFMM_REQUIRE(std::isfinite(p->near_radius) && p->near_radius >= 0 && p->near_radius < 16,
               "near_radius must be in [0, 16)");
  if (p->cell) {
    KFMM_REQUIRE(std::isfinite(p->cell[0]) && std::isfinite(p->cell[1]) && std::isfinite(p->cell[2]) &&
                     std::isfinite(p->cell[3]) && p->cell[3] > 0,
                 "cell: finite lower corner and side > 0 required");
  }
}

extern "C" int bem_near_pairs(const bem_problem* prob, int64_t* count, int32_t* pairs, int64_t count_capacity,
                              void* stream) {
  return guarded([&] {
    KFMM_REQUIRE(prob != nullptr && prob->n_tri > 0 && prob->n_tri < ((int64_t)1 << 27) && prob->tri_xyz,
                 "problem with triangles required");
    KFMM_REQUIRE(std::isfinite(prob->near_radius) && prob->near_radius >= 0 && prob->near_radius < 16,
                 "near_radius must be in [0, 16)");
    KFMM_REQUIRE(count != nullptr, "count is NULL");
    KFMM_REQUIRE(prob->cell == nullptr, "bem_near_pairs serves free-space surfaces only (its rows carry no image shift)");
    hipStream_t s = (hipStream_t)stream;
    const int64_t T = prob->n_tri, NQ = 16 * T;
    Arena a;
    double* qp = a.get<double>(3 * NQ);
    double* qn = a.get<double>(3 * NQ);
    double* qw = a.get<double>(NQ);
    double* cen = a.get<double>(3 * T);
    bem_expand(T, prob->tri_xyz, qp, qn, qw, cen, s);
    NearPairs np = find_near_pairs(prob->tri_xyz, cen, T, prob->near_radius > 0 ? prob->near_radius : 1.5, a, s);
    *count = np.n;
    if (pairs) {
      KFMM_REQUIRE(count_capacity >= np.n, "pairs holds fewer than count pairs");
      std::vector<int32_t> h(2 * std::max<int64_t>(np.n, 1));
      std::vector<int32_t> r(np.n), c(np.n);
      if (np.n) {
        KFMM_HIP(hipMemcpyAsync(r.data(), np.row, sizeof(int32_t) * np.n, hipMemcpyDeviceToHost, s));
        KFMM_HIP(hipMemcpyAsync(c.data(), np.idx, sizeof(int32_t) * np.n, hipMemcpyDeviceToHost, s));
        KFMM_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < np.n; ++i) {
          h[2 * i] = r[i];
          h[2 * i + 1] = c[i];
        }
        KFMM_HIP(hipMemcpyAsync(pairs, h.data(), sizeof(int32_t) * 2 * np.n, hipMemcpyHostToDevice, s));
      }
    }
    KFMM_HIP(hipStreamSynchronize(s));
  });
}

extern "C" int bem_solve(const bem_problem* prob, const bem_opts* opts, const double* x0, double* x, double* u_full,
                         double* t_full, bem_stats* stats, void* stream) {
  int rc = KFMM_OK;
  int code = guarded([&] {
    check_problem(prob);
    KFMM_REQUIRE(opts != nullptr && x != nullptr, "opts or x is NULL");
    KFMM_REQUIRE(opts->tol > 0 && opts->restart >= 1 && opts->restart <= 500 && opts->max_iter >= 0,
                 "tol > 0, restart in [1, 500], max_iter >= 0 required");
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    KFMM_REQUIRE(opts->precond == KFMM_PC_NONE || opts->precond == KFMM_PC_TWO_LEVEL, "unknown preconditioner");
    KFMM_REQUIRE(opts->precond == KFMM_PC_NONE || prob->cell == nullptr,
                 "the two-level preconditioner is built for free space (cell must be NULL)");
    BemSystem sys(*prob, opts->fmm, s);
    if (opts->precond == KFMM_PC_TWO_LEVEL) {
      sys.pc = std::make_unique<TwoLevelPC>();
      sys.pc->build(sys, opts->pc_fine, opts->pc_coarse);
    }
    double t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bem_stats st = sys.gmres(x0, opts->x0_alt, x, opts->tol, opts->restart, opts->max_iter);
    st.t_setup_s = t_setup;
    if (sys.pc) {
      st.t_precond_s = sys.pc->t_setup_s;
      st.pc_coarse_dim = sys.pc->nc - sys.pc->n_dropped;
    }
    // traction unknowns back to physical units
    sys.split(x, u_full, t_full);
    scale_traction_unknowns(sys, x, sys.scale_t);
    KFMM_HIP(hipStreamSynchronize(s));
    if (stats) *stats = st;
    if (!st.converged) rc = KFMM_E_NOCONV;
  });
  if (code != KFMM_OK) return code;
  if (rc != KFMM_OK) set_last_error("GMRES did not reach the tolerance within max_iter");
  return rc;
}

extern "C" int bem_stress(const bem_problem* prob, const double* u_full, const double* t_full, const double* trg,
                          int64_t M, double* out, const fmm_opts* fmm, void* stream) {
  return guarded([&] {
    check_problem(prob);
    KFMM_REQUIRE(u_full && t_full && fmm, "NULL argument");
    KFMM_REQUIRE(M >= 0 && (M == 0 || (trg && out)), "bad targets");
    if (M == 0) return;
    stress_from_boundary(*prob, u_full, t_full, trg, M, out, *fmm, (hipStream_t)stream);
  });
}

namespace kfmm {
void alg1_surface_impl(const alg1_grid*, const uint8_t*, const double*, int64_t*, double*, int8_t*, double*,
                       int32_t*, int64_t, hipStream_t);
void alg1_centres_impl(const alg1_grid*, const uint8_t*, int64_t*, double*, int64_t, hipStream_t);
void alg1_update_impl(const alg1_grid*, const uint8_t*, const double*, int64_t, double, uint8_t*, int64_t*,
                      hipStream_t);
void alg1_cell_surface_impl(const alg1_grid*, const uint8_t*, const double*, int64_t*, double*, int8_t*, double*,
                            int32_t*, int64_t, hipStream_t);
void alg1_cell_update_impl(const alg1_grid*, const uint8_t*, const double*, int64_t, double, uint8_t*, int64_t*,
                           hipStream_t);
void alg1_coarse_impl(const alg1_grid*, const uint8_t*, int, int64_t*, double*, int64_t, hipStream_t);
void alg1_refine_impl(const alg1_grid*, const uint8_t*, int, const double*, int64_t, double, int64_t*, double*,
                      int64_t, uint8_t*, hipStream_t);
void alg1_expand_impl(const alg1_grid*, const uint8_t*, int, const double*, int64_t, double, const double*, int64_t,
                      double*, hipStream_t);
void alg1_energy_impl(const double*, int64_t, double, double, double*, hipStream_t);
}  // namespace kfmm

extern "C" int alg1_surface(const alg1_grid* grid, const uint8_t* vox, const double* load, int64_t* n_tri, double* tri,
                            int8_t* bc_type, double* bc_val, int32_t* owner, int64_t capacity, void* stream) {
  return guarded([&] {
    alg1_surface_impl(grid, vox, load, n_tri, tri, bc_type, bc_val, owner, capacity, (hipStream_t)stream);
  });
}

extern "C" int alg1_centres(const alg1_grid* grid, const uint8_t* vox, int64_t* n, double* pts, int64_t capacity,
                            void* stream) {
  return guarded([&] { alg1_centres_impl(grid, vox, n, pts, capacity, (hipStream_t)stream); });
}

extern "C" int alg1_cell_surface(const alg1_grid* grid, const uint8_t* vox, const double* sig_h, int64_t* n_tri,
                                 double* tri, int8_t* bc_type, double* bc_val, int32_t* owner, int64_t capacity,
                                 void* stream) {
  return guarded([&] {
    alg1_cell_surface_impl(grid, vox, sig_h, n_tri, tri, bc_type, bc_val, owner, capacity, (hipStream_t)stream);
  });
}

extern "C" int alg1_cell_update(const alg1_grid* grid, const uint8_t* vox, const double* td, int64_t n_td,
                                double alpha, uint8_t* out, int64_t* n_filled, void* stream) {
  return guarded([&] { alg1_cell_update_impl(grid, vox, td, n_td, alpha, out, n_filled, (hipStream_t)stream); });
}

extern "C" int alg1_update(const alg1_grid* grid, const uint8_t* vox, const double* td, int64_t n_td, double C,
                           uint8_t* out, int64_t* n_filled, void* stream) {
  return guarded([&] { alg1_update_impl(grid, vox, td, n_td, C, out, n_filled, (hipStream_t)stream); });
}

extern "C" int alg1_coarse_blocks(const alg1_grid* grid, const uint8_t* vox, int block, int64_t* n, double* pts,
                                  int64_t capacity, void* stream) {
  return guarded([&] { alg1_coarse_impl(grid, vox, block, n, pts, capacity, (hipStream_t)stream); });
}

extern "C" int alg1_refine(const alg1_grid* grid, const uint8_t* vox, int block, const double* td_coarse,
                           int64_t n_coarse, double C, int64_t* n, double* pts, int64_t capacity, uint8_t* refined,
                           void* stream) {
  return guarded([&] {
    alg1_refine_impl(grid, vox, block, td_coarse, n_coarse, C, n, pts, capacity, refined, (hipStream_t)stream);
  });
}

extern "C" int alg1_expand(const alg1_grid* grid, const uint8_t* vox, int block, const double* td_coarse,
                           int64_t n_coarse, double C, const double* td_fine, int64_t n_fine, double* td_out,
                           void* stream) {
  return guarded([&] {
    alg1_expand_impl(grid, vox, block, td_coarse, n_coarse, C, td_fine, n_fine, td_out, (hipStream_t)stream);
  });
}

extern "C" int alg1_energy(const double* sig6, int64_t n, double K, double G, double* psi, void* stream) {
  return guarded([&] {
    check_moduli(K, G);
    KFMM_REQUIRE(n >= 0, "negative size");
    alg1_energy_impl(sig6, n, K, G, psi, (hipStream_t)stream);
  });
}

extern "C" int bem_precond_apply(const bem_problem* prob, const bem_opts* opts, const double* v, double* y,
                                 bem_pc_info* info, void* stream) {
  return guarded([&] {
    check_problem(prob);
    KFMM_REQUIRE(opts && v && y, "opts, v or y is NULL");
    KFMM_REQUIRE(opts->precond == KFMM_PC_TWO_LEVEL, "bem_precond_apply needs opts->precond = KFMM_PC_TWO_LEVEL");
    KFMM_REQUIRE(prob->cell == nullptr, "the two-level preconditioner is built for free space (cell must be NULL)");
    KFMM_REQUIRE(v != y, "v and y must not overlap");
    hipStream_t s = (hipStream_t)stream;
    BemSystem sys(*prob, opts->fmm, s);
    TwoLevelPC pc;
    pc.build(sys, opts->pc_fine, opts->pc_coarse);
    pc.apply(v, y, s);
    KFMM_HIP(hipStreamSynchronize(s));
    if (info) {
      info->n_fine_blocks = pc.nb;
      info->n_aggregates = pc.na;
      info->n_coarse = pc.nc;
      info->fine = pc.fine;
      info->coarse = pc.coarse;
      info->n_dropped = pc.n_dropped;
      info->t_setup_s = pc.t_setup_s;
    }
  });
}

extern "C" int bem_matvec(const bem_problem* prob, const fmm_opts* fmm, int which, const double* x, double* y,
                          void* stream) {
  return guarded([&] {
    check_problem(prob);
    KFMM_REQUIRE(fmm && y && (which == 1 || (which == 0 && x)), "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    BemSystem sys(*prob, *fmm, s);
    sys.apply(which, x, y);
    KFMM_HIP(hipStreamSynchronize(s));
  });
}

extern "C" int bem_quadrature(int64_t n_tri, const double* tri_xyz, double* qp, double* qn, double* qw,
                              double* colloc, void* stream) {
  return guarded([&] {
    KFMM_REQUIRE(n_tri >= 0 && (n_tri == 0 || (tri_xyz && qp && qn && qw && colloc)), "bad arguments");
    if (n_tri) bem_expand(n_tri, tri_xyz, qp, qn, qw, colloc, (hipStream_t)stream);
  });
}

extern "C" int kfmm_topological_derivative(const double* sig6, int64_t M, double K, double G, double* td,
                                           void* stream) {
  return guarded([&] {
    check_moduli(K, G);
    KFMM_REQUIRE(M >= 0 && (M == 0 || (sig6 && td)), "bad arguments");
    if (M) topological_derivative(sig6, M, Elastic::make(K, G), td, (hipStream_t)stream);
  });
}

extern "C" int alg1_cell_td(const double* sig6, int64_t M, const double* sig_h, double K, double G, double* td,
                            void* stream) {
  return guarded([&] {
    check_moduli(K, G);
    KFMM_REQUIRE(sig_h != nullptr, "sig_h is NULL");
    for (int c = 0; c < 6; ++c) KFMM_REQUIRE(std::isfinite(sig_h[c]), "sig_h must be finite");
    KFMM_REQUIRE(M >= 0 && (M == 0 || (sig6 && td)), "bad arguments");
    if (M) topological_derivative(sig6, M, Elastic::make(K, G), td, (hipStream_t)stream, sig_h);
  });
}

struct ws_net {
  kfmm::WsNet* impl;
};

static WsNet& net_of(ws_net_t n) {
  KFMM_REQUIRE(n != nullptr && n->impl != nullptr, "network is NULL");
  return *n->impl;
}

extern "C" int ws_create(ws_net_t* out, int d_in, int width, uint64_t seed) {
  return guarded([&] {
    KFMM_REQUIRE(out != nullptr, "out is NULL");
    *out = nullptr;
    *out = new ws_net{new WsNet(d_in, width, seed)};
  });
}

extern "C" int ws_destroy(ws_net_t net) {
  return guarded([&] {
    if (!net) return;
    delete net->impl;
    delete net;
  });
}

extern "C" int ws_features(const bem_problem* prev, const double* u_prev, const double* t_prev,
                           const bem_problem* next, float* feat, double* x_mapped, double* scale, void* stream) {
  return guarded([&] {
    check_problem(prev);
    check_problem(next);
    KFMM_REQUIRE(u_prev && t_prev && feat && x_mapped && scale, "NULL argument");
    *scale = ws_make_features(*prev, u_prev, t_prev, *next, feat, x_mapped, (hipStream_t)stream);
  });
}

extern "C" int ws_predict(ws_net_t net, const float* feat, int64_t n, const double* x_mapped, double scale,
                          double* x0, void* stream) {
  return guarded([&] {
    KFMM_REQUIRE(n >= 0 && (n == 0 || (feat && x_mapped && x0)), "bad arguments");
    KFMM_REQUIRE(std::isfinite(scale) && scale > 0, "scale must be positive");
    net_of(net).predict(feat, n, x_mapped, scale, x0, (hipStream_t)stream);
  });
}

extern "C" int ws_train(ws_net_t net, const float* feat, const double* x_mapped, const double* x_target, int64_t n,
                        double scale, int epochs, float lr, float* loss, void* stream) {
  return guarded([&] {
    KFMM_REQUIRE(n > 0 && feat && x_mapped && x_target && epochs >= 0 && lr > 0, "bad arguments");
    KFMM_REQUIRE(std::isfinite(scale) && scale > 0, "scale must be positive");
    float L = net_of(net).train(feat, x_mapped, x_target, n, scale, epochs, lr, (hipStream_t)stream);
    if (loss) *loss = L;
  });
}

extern "C" int ws_train_noalloc(ws_net_t net, const float* feat, const double* x_mapped, const double* x_target,
                                int64_t n, double scale, int epochs, float lr, float* loss, void* stream) {
  return guarded([&] {
    KFMM_REQUIRE(n > 0 && feat && x_mapped && x_target && epochs >= 0 && lr > 0, "bad arguments");
    KFMM_REQUIRE(std::isfinite(scale) && scale > 0, "scale must be positive");
    KFMM_REQUIRE(n <= KFMM_WS_NOALLOC_MAX_ROWS, "n exceeds KFMM_WS_NOALLOC_MAX_ROWS (static scratch size)");
    WsNet& w = net_of(net);
    WsWork b = ws_noalloc_work(w, n);
    float L = w.train(feat, x_mapped, x_target, n, scale, epochs, lr, b, (hipStream_t)stream);
    if (loss) *loss = L;
  });
}

extern "C" int ws_num_params(ws_net_t net, int64_t* n) {
  return guarded([&] {
    KFMM_REQUIRE(n != nullptr, "NULL argument");
    *n = net_of(net).np;
  });
}

extern "C" int ws_get_params(ws_net_t net, float* host) {
  return guarded([&] {
    KFMM_REQUIRE(host != nullptr, "NULL argument");
    WsNet& w = net_of(net);
    KFMM_HIP(hipMemcpy(host, w.params, sizeof(float) * w.np, hipMemcpyDeviceToHost));
  });
}

extern "C" int ws_set_params(ws_net_t net, const float* host) {
  return guarded([&] {
    KFMM_REQUIRE(host != nullptr, "NULL argument");
    WsNet& w = net_of(net);
    KFMM_HIP(hipMemcpy(w.params, host, sizeof(float) * w.np, hipMemcpyHostToDevice));
    w.bf_dirty = true;
  });
}

extern "C" int ws_loss_grad(ws_net_t net, const float* X, const float* R, int64_t n, float* loss, float* grad,
                            void* stream) {
  return guarded([&] {
    KFMM_REQUIRE(n > 0 && X && R, "bad arguments");
    WsNet& w = net_of(net);
    hipStream_t s = (hipStream_t)stream;
    float L = w.loss_grad(X, R, n, s);
    if (loss) *loss = L;
    if (grad) {
      KFMM_HIP(hipMemcpyAsync(grad, w.grads, sizeof(float) * w.np, hipMemcpyDeviceToHost, s));
      KFMM_HIP(hipStreamSynchronize(s));
    }
  });
}

extern "C" int ws_save(ws_net_t net, const char* path) {
  return guarded([&] {
    KFMM_REQUIRE(path != nullptr, "path is NULL");
    WsNet& w = net_of(net);
    std::vector<float> buf(3 * (size_t)w.np);
    KFMM_HIP(hipMemcpy(buf.data(), w.params, sizeof(float) * w.np, hipMemcpyDeviceToHost));
    KFMM_HIP(hipMemcpy(buf.data() + w.np, w.m1, sizeof(float) * w.np, hipMemcpyDeviceToHost));
    KFMM_HIP(hipMemcpy(buf.data() + 2 * w.np, w.m2, sizeof(float) * w.np, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    KFMM_REQUIRE(f != nullptr, std::string("cannot open ") + path);
    int64_t hdr[4] = {0x6b666d6d77730001LL, w.din, w.width, w.step};
    bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1 && std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    KFMM_REQUIRE(ok, "write failed");
  });
}

extern "C" int ws_load(ws_net_t net, const char* path) {
  return guarded([&] {
    KFMM_REQUIRE(path != nullptr, "path is NULL");
    WsNet& w = net_of(net);
    FILE* f = std::fopen(path, "rb");
    KFMM_REQUIRE(f != nullptr, std::string("cannot open ") + path);
    int64_t hdr[4];
    std::vector<float> buf(3 * (size_t)w.np);
    bool ok = std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 0x6b666d6d77730001LL && hdr[1] == w.din &&
              hdr[2] == w.width && std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    KFMM_REQUIRE(ok, "not a network file of this shape");
    KFMM_HIP(hipMemcpy(w.params, buf.data(), sizeof(float) * w.np, hipMemcpyHostToDevice));
    KFMM_HIP(hipMemcpy(w.m1, buf.data() + w.np, sizeof(float) * w.np, hipMemcpyHostToDevice));
    KFMM_HIP(hipMemcpy(w.m2, buf.data() + 2 * w.np, sizeof(float) * w.np, hipMemcpyHostToDevice));
    w.step = hdr[3];
    w.bf_dirty = true;
  });
}

extern "C" int kfmm_selftest_gemm(int precision, const void* A, int NC, const void* X, void* Y, const int* op,
                                  const int* in, const int* out, const double* scale, int ncols, int mode,
                                  void* stream) {
  return guarded([&] {
    const int kernel = precision >> 4;
    precision &= 15;
    KFMM_REQUIRE((precision == 0 || precision == 1 || precision == 3) && mode >= 0 && mode <= 2 && ncols >= 0,
                 "bad arguments");
    KFMM_REQUIRE(kernel >= 0 && kernel <= 4 && (kernel == 0 || precision <= 1 || (precision == 3 && kernel == 1)),
                 "bad kernel selector");
    KFMM_REQUIRE(NC > 0 && gemm_tm(NC) != 0, "NC must be a positive multiple of 96 or 128");
    for (int i = 0; i < ncols; ++i) KFMM_REQUIRE(op[i] >= 0 && in[i] >= 0 && out[i] >= 0, "negative index");
    for (int i = 1; i < ncols; ++i) KFMM_REQUIRE(op[i] >= op[i - 1], "columns must be sorted by op");
    selftest_gemm(precision, A, NC, X, Y, op, in, out, scale, ncols, mode, kernel, (hipStream_t)stream);
  });
}

extern "C" const char* kfmm_last_error(void) { return g_last_error.c_str(); }
