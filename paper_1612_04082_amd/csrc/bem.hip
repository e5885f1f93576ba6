// Collocation BEM for 3D elastostatics driven by the KIFMM (Sec. 2.2, "Discretization of BIE",
// "Matrix-vector products"; eqs. BIE, num, coef, num2).
//
//  * Piecewise-constant u and t per flat triangle, collocation at the centroid (a smooth point: free
//    term 1/2 I, eq. BIE).
//  * Quadrature: every triangle is split at its edge midpoints into four equal triangles, each with the
//    symmetric 4-point degree-3 rule; a quadrature source carries (element value) x (area/4) x (weight).
//    The centroid of the central sub-triangle IS the collocation point (same FP64 value), so the fast
//    summation skips that coincident pair.
//  * Two-pass matrix-vector product: (1) fmm_eval over all quadrature points at all centroids;
//    (2) local pass per element: remove the element's own quadrature contributions and add the
//    closed-form (principal-value) self integrals, then the free term.
//  * Unknowns per element and component: u where the traction is prescribed, t where the displacement is
//    prescribed (eq. num2); the traction unknowns are scaled by -l/G (l = mean edge length): the size
//    balances the single-layer columns against the 1/2 I + P columns and the sign makes those columns +U
//    (positive definite), keeping the spectrum in the right half-plane.
//  * Restarted GMRES(m): Arnoldi with classical Gram-Schmidt applied twice, FP64 vectors on the device,
//    the small Hessenberg problem (Givens rotations) on the host; stop when ||b - A x|| / ||b|| <= tol,
//    checked with a true residual at every restart.  With a preconditioner M (precond.hip) the Arnoldi
//    process runs on A M^-1 and each cycle's correction is M^-1 V y (right preconditioning: the residual
//    is still the true one).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <memory>
#include <vector>

#include "../../include/kfmm.h"
#include "bem.h"
#include "common.h"
#include "precond.h"
#include "plan.h"
#include "tree.h"

namespace kfmm {

// symmetric degree-3 rule: (barycentric, weight); the first point is the centroid
__constant__ double c_rule_bary[4][3] = {
    {1.0 / 3, 1.0 / 3, 1.0 / 3}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
__constant__ double c_rule_w[4] = {-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48};

// Quadrature points (16 per triangle, order: sub-triangle s, rule point q), normals, weights, centroids.
__global__ void k_bem_expand(int64_t T, const double* __restrict__ tri, double* __restrict__ qp,
                             double* __restrict__ qn, double* __restrict__ qw, double* __restrict__ cen,
                             double* __restrict__ edge_sum) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  double v[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) v[a][d] = tri[9 * k + 3 * a + d];
  double c[3], e1[3], e2[3], m[3][3];
  for (int d = 0; d < 3; ++d) {
    c[d] = (v[0][d] + v[1][d] + v[2][d]) / 3.0;
    e1[d] = v[1][d] - v[0][d];
    e2[d] = v[2][d] - v[0][d];
    m[0][d] = 0.5 * (v[0][d] + v[1][d]);  // m01
    m[1][d] = 0.5 * (v[1][d] + v[2][d]);  // m12
    m[2][d] = 0.5 * (v[2][d] + v[0][d]);  // m20
  }
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  double a2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int d = 0; d < 3; ++d) n[d] /= a2;
  double area = 0.5 * a2;
  const double* sub[4][3] = {{v[0], m[0], m[2]}, {m[0], v[1], m[1]}, {m[2], m[1], v[2]}, {m[0], m[1], m[2]}};
  for (int s = 0; s < 4; ++s)
    for (int q = 0; q < 4; ++q) {
      int64_t i = 16 * k + 4 * s + q;
      for (int d = 0; d < 3; ++d) {
        double x = c_rule_bary[q][0] * sub[s][0][d] + c_rule_bary[q][1] * sub[s][1][d] + c_rule_bary[q][2] * sub[s][2][d];
        if (s == 3 && q == 0) x = c[d];  // central centroid == collocation point
        qp[3 * i + d] = x;
        qn[3 * i + d] = n[d];
      }
      qw[i] = 0.25 * area * c_rule_w[q];
    }
  for (int d = 0; d < 3; ++d) cen[3 * k + d] = c[d];
  double l = 0;
  for (int a = 0; a < 3; ++a) {
    double s2 = 0;
    for (int d = 0; d < 3; ++d) {
      double t = v[(a + 1) % 3][d] - v[a][d];
      s2 += t * t;
    }
    l += sqrt(s2);
  }
  edge_sum[k] = l;
}

// Closed-form self integrals at the centroid of a flat triangle, minus the element's own quadrature
// terms (r > 0), for the local pass:  dU = U_self - sum_q U w,  dP = P_self - sum_q P w  (3x3, row-major).
// Polar coordinates about the centroid; per edge with perpendicular distance h, in-plane outward normal m
// and tangent t, angles phi in [phi_a, phi_b], R(phi) = h / cos(phi), L(phi) = ln(sec phi + tan phi):
//   int 1/r          = sum h [L]
//   int r_i r_j / r  = sum h [m m sin - (m t + t m) cos + t t (L - sin)]
//   PV int r_hat/r^2 = sum [m (sin (ln h - ln cos + 1) - L) - t cos (ln h - ln cos + 1)]
__global__ void k_bem_self(int64_t T, const double* __restrict__ tri, const double* __restrict__ qp,
                           const double* __restrict__ qw, Elastic el, double* __restrict__ dU,
                           double* __restrict__ dP) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  const double nu = el.nu;
  double v[3][3], c[3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) v[a][d] = tri[9 * k + 3 * a + d];
  for (int d = 0; d < 3; ++d) c[d] = (v[0][d] + v[1][d] + v[2][d]) / 3.0;
  double e1[3], e2[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = v[1][d] - v[0][d];
    e2[d] = v[2][d] - v[0][d];
  }
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  double inv_r = 0, rr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, V[3] = {0, 0, 0};
  for (int e = 0; e < 3; ++e) {
    const double* A = v[e];
    const double* B = v[(e + 1) % 3];
    double t[3], len = 0;
    for (int d = 0; d < 3; ++d) {
      t[d] = B[d] - A[d];
      len += t[d] * t[d];
    }
    len = sqrt(len);
    for (int d = 0; d < 3; ++d) t[d] /= len;
    double m[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2], t[0] * n[1] - t[1] * n[0]};
    double h = 0, ta = 0, tb = 0;
    for (int d = 0; d < 3; ++d) h += (A[d] - c[d]) * m[d];
    if (h < 0) {
      h = -h;
      for (int d = 0; d < 3; ++d) m[d] = -m[d];
    }
    for (int d = 0; d < 3; ++d) {
      ta += (A[d] - c[d]) * t[d];
      tb += (B[d] - c[d]) * t[d];
    }
    double pa = atan2(ta, h), pb = atan2(tb, h);
    auto L = [](double p) { return log(1.0 / cos(p) + tan(p)); };
    double Lab = L(pb) - L(pa);
    double sab = sin(pb) - sin(pa), cab = cos(pb) - cos(pa);
    inv_r += h * Lab;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        rr[i][j] += h * (m[i] * m[j] * sab - (m[i] * t[j] + t[i] * m[j]) * cab + t[i] * t[j] * (Lab - sab));
    auto Fm = [&](double p) { return sin(p) * (log(h) - log(cos(p)) + 1.0) - L(p); };
    auto Ft = [&](double p) { return -cos(p) * (log(h) - log(cos(p)) + 1.0); };
    double fm = Fm(pb) - Fm(pa), ft = Ft(pb) - Ft(pa);
    for (int d = 0; d < 3; ++d) V[d] += m[d] * fm + t[d] * ft;
  }
  double Us[3][3], Ps[3][3];
  const double cu = 1.0 / (16.0 * kPi * (1.0 - nu) * el.G);
  const double cp = (1.0 - 2.0 * nu) / (8.0 * kPi * (1.0 - nu));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Us[i][j] = cu * ((i == j ? (3.0 - 4.0 * nu) * inv_r : 0.0) + rr[i][j]);
      Ps[i][j] = cp * (V[i] * n[j] - n[i] * V[j]);
    }
  // subtract the element's own quadrature terms (the coincident centroid point is skipped, r = 0)
  for (int q = 0; q < 16; ++q) {
    const int64_t s = 16 * k + q;
    double d[3] = {qp[3 * s] - c[0], qp[3 * s + 1] - c[1], qp[3 * s + 2] - c[2]};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r == 0.0) continue;
    double rh[3] = {d[0] / r, d[1] / r, d[2] / r};
    double drdn = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
    double w = qw[s];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double u = cu / r * ((i == j ? 3.0 - 4.0 * nu : 0.0) + rh[i] * rh[j]);
        double p = -1.0 / (8.0 * kPi * (1.0 - nu) * r * r) *
                   (drdn * ((i == j ? 1.0 - 2.0 * nu : 0.0) + 3.0 * rh[i] * rh[j]) -
                    (1.0 - 2.0 * nu) * (rh[i] * n[j] - rh[j] * n[i]));
        Us[i][j] -= u * w;
        Ps[i][j] -= p * w;
      }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      dU[9 * k + 3 * i + j] = Us[i][j];
      dP[9 * k + 3 * i + j] = Ps[i][j];
    }
}

// Element densities for the fast summation from the unknown vector x or the prescribed values y.
//  mode 0 (matvec of A):   a = -t_unk, b = u_unk     -> FMM gives -U t_unk + P u_unk
//  mode 1 (right side B y): a = t_known, b = -u_known -> FMM gives U t_known - P u_known
// Element e's values go to its 16 quadrature points.  Also writes the element values ae, be (T x 3).
__global__ void k_bem_densities(int64_t T, int mode, const double* __restrict__ x, const double* __restrict__ y,
                                const int8_t* __restrict__ bc_type, double scale_t, double* __restrict__ a,
                                double* __restrict__ b, double* __restrict__ ae, double* __restrict__ be) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * T) return;
  const int64_t k = i / 3;
  const int c = (int)(i % 3);
  const bool u_prescribed = bc_type[i] == 0;  // then t is the unknown
  double av = 0, bv = 0;
  if (mode == 0) {
    if (u_prescribed)
      av = -scale_t * x[i];
    else
      bv = x[i];
  } else {
    if (u_prescribed)
      bv = -y[i];
    else
      av = y[i];
  }
  ae[i] = av;
  be[i] = bv;
  for (int q = 0; q < 16; ++q) {
    a[3 * (16 * k + q) + c] = av;
    b[3 * (16 * k + q) + c] = bv;
  }
}

// Local pass and free term:  out_k = fmm_k + dU_k ae_k + dP_k be_k + half * (+-1/2 u)
//   mode 0: + 1/2 u_unk (= be);  mode 1: - 1/2 u_known (= be, which holds -u_known).
// With the near-singular quadrature (near_off != NULL) also sum_{e near k} nU_ke ae_e + nP_ke be_e, in the
// order of e.
__global__ void k_bem_local(int64_t T, const double* __restrict__ fmm, const double* __restrict__ dU,
                            const double* __restrict__ dP, const double* __restrict__ ae,
                            const double* __restrict__ be, const int* __restrict__ near_off,
                            const int* __restrict__ near_idx, const double* __restrict__ nU,
                            const double* __restrict__ nP, double* __restrict__ out) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  for (int i = 0; i < 3; ++i) {
    double v = fmm[3 * k + i];
    for (int j = 0; j < 3; ++j) v += dU[9 * k + 3 * i + j] * ae[3 * k + j] + dP[9 * k + 3 * i + j] * be[3 * k + j];
    if (near_off)
      for (int p = near_off[k]; p < near_off[k + 1]; ++p) {
        const int64_t e = near_idx[p];
        for (int j = 0; j < 3; ++j) v += nU[9 * p + 3 * i + j] * ae[3 * e + j] + nP[9 * p + 3 * i + j] * be[3 * e + j];
      }
    v += 0.5 * be[3 * k + i];
    out[3 * k + i] = v;
  }
}

// Physical u and t from the unknowns and prescribed values.
__global__ void k_bem_split(int64_t T, const double* __restrict__ x, const double* __restrict__ y,
                            const int8_t* __restrict__ bc_type, double scale_t, double* __restrict__ u,
                            double* __restrict__ t) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * T) return;
  if (bc_type[i] == 0) {
    if (u) u[i] = y[i];
    if (t) t[i] = scale_t * x[i];
  } else {
    if (u) u[i] = x[i];
    if (t) t[i] = y[i];
  }
}

// ----------------------------------------------------------------------------------- BLAS-1 on device

constexpr int kDotChunks = 64;

// partial[i][c] = sum over chunk c of V_i . w   (i < nv); deterministic two-level reduction
__global__ void k_dots(const double* __restrict__ V, int64_t ld, int nv, const double* __restrict__ w, int64_t n,
                       double* __restrict__ partial) {
  const int i = blockIdx.y, c = blockIdx.x;
  const double* vi = V + (size_t)i * ld;
  int64_t per = (n + kDotChunks - 1) / kDotChunks;
  int64_t b = c * per, e = min(n, b + per);
  double s = 0;
  for (int64_t j = b + threadIdx.x; j < e; j += blockDim.x) s += vi[j] * w[j];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)i * kDotChunks + c] = red[0];
}

// w -= sum_i h_i V_i
__global__ void k_sub_many(const double* __restrict__ V, int64_t ld, int nv, const double* __restrict__ h,
                           double* __restrict__ w, int64_t n) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = w[j];
  for (int i = 0; i < nv; ++i) s -= h[i] * V[(size_t)i * ld + j];
  w[j] = s;
}

// x += sum_i y_i V_i
__global__ void k_add_many(const double* __restrict__ V, int64_t ld, int nv, const double* __restrict__ y,
                           double* __restrict__ x, int64_t n) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = x[j];
  for (int i = 0; i < nv; ++i) s += y[i] * V[(size_t)i * ld + j];
  x[j] = s;
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) y[j] = a * x[j] + b * y[j];
}

__global__ void k_scale_copy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) y[j] = a * x[j];
}

__global__ void k_sum(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s += x[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

static unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

void bem_expand(int64_t T, const double* tri, double* qp, double* qn, double* qw, double* cen, hipStream_t s) {
  Arena a;
  double* esum = a.get<double>(T);
  hipLaunchKernelGGL(k_bem_expand, dim3(nblk(T)), dim3(256), 0, s, T, tri, qp, qn, qw, cen, esum);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------------------------------ system

BemSystem::BemSystem(const bem_problem& p, const fmm_opts& fo, hipStream_t s) : stream(s) {
  T = p.n_tri;
  n = 3 * T;
  el = Elastic::make(p.K, p.G);
  tri = p.tri_xyz;
  bc_type = p.bc_type;
  bc_val = p.bc_val;
  const int64_t NQ = 16 * T;
  qp = arena.get<double>(3 * NQ);
  qn = arena.get<double>(3 * NQ);
  qw = arena.get<double>(NQ);
  cen = arena.get<double>(3 * T);
  double* esum = arena.get<double>(T);
  hipLaunchKernelGGL(k_bem_expand, dim3(nblk(T)), dim3(256), 0, s, T, tri, qp, qn, qw, cen, esum);
  KFMM_HIP(hipGetLastError());
  double* d_l = arena.get<double>(1);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, esum, T, d_l);
  double lsum = 0;
  KFMM_HIP(hipMemcpyAsync(&lsum, d_l, sizeof(double), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  mean_edge = lsum / (3.0 * T);
  scale_t = -p.G / mean_edge;
  dU = arena.get<double>(9 * T);
  dP = arena.get<double>(9 * T);
  hipLaunchKernelGGL(k_bem_self, dim3(nblk(T, 128)), dim3(128), 0, s, T, tri, qp, qw, el, dU, dP);
  KFMM_HIP(hipGetLastError());
  near_levels = p.near_levels;
  if (near_levels > 0) {
    near = find_near_pairs(tri, cen, T, p.near_radius > 0 ? p.near_radius : 1.5, arena, s, p.cell ? p.cell[3] : 0.0);
    near_dU = arena.get<double>((size_t)9 * std::max<int64_t>(near.n, 1));
    near_dP = arena.get<double>((size_t)9 * std::max<int64_t>(near.n, 1));
    near_blocks(near, near_levels, tri, cen, qp, qn, qw, el, near_dU, near_dP, s);
  }
  fmm_opts o = fo;
  o.K = p.K;
  o.G = p.G;
  // Solves of ill-conditioned systems: a pseudo-inverse cutoff of 1e-7 keeps the equivalent densities
  // (and their rounding) 10x smaller than the evaluation default 1e-8; with 1e-8 the true residual of the
  // 61k-element cantilever stalls near 2.6e-6, with 1e-7 GMRES reaches 1e-6 in 157 steps.
  if (o.svd_eps == 0) o.svd_eps = 1e-7;
  std::vector<int64_t> bsrc = {0, NQ}, btrg = {0, T};
  plan.reset(plan_create(qp, qn, qw, NQ, cen, T, bsrc, btrg, o, s, problem_cells(p)));
  a16 = arena.get<double>(3 * NQ);
  b16 = arena.get<double>(3 * NQ);
  ae = arena.get<double>(n);
  be = arena.get<double>(n);
  fmm_out = arena.get<double>(n);
}

BemSystem::~BemSystem() = default;

// out = A x (mode 0) or B y (mode 1)
void BemSystem::apply(int mode, const double* xin, double* out) {
  hipStream_t s = stream;
  hipLaunchKernelGGL(k_bem_densities, dim3(nblk(n)), dim3(256), 0, s, T, mode, xin, bc_val, bc_type, scale_t, a16,
                     b16, ae, be);
  KFMM_HIP(hipGetLastError());
  plan_eval(*plan, KFMM_DISP, a16, b16, fmm_out, s);
  hipLaunchKernelGGL(k_bem_local, dim3(nblk(T)), dim3(256), 0, s, T, fmm_out, dU, dP, ae, be,
                     near_levels > 0 ? near.off : nullptr, near.idx, near_dU, near_dP, out);
  KFMM_HIP(hipGetLastError());
  ++n_apply;
}

double BemSystem::dot(const double* x, const double* y) {
  double* part = scratch_partial();
  hipLaunchKernelGGL(k_dots, dim3(kDotChunks, 1), dim3(256), 0, stream, x, (int64_t)0, 1, y, n, part);
  std::vector<double> h(kDotChunks);
  KFMM_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * kDotChunks, hipMemcpyDeviceToHost, stream));
  KFMM_HIP(hipStreamSynchronize(stream));
  double s = 0;
  for (double v : h) s += v;
  return s;
}

double* BemSystem::scratch_partial() {
  if (!partial) partial = arena.get<double>((size_t)kDotChunks * 512);
  return partial;
}

void BemSystem::split(const double* x, double* u, double* t) {
  if (!u && !t) return;
  hipLaunchKernelGGL(k_bem_split, dim3(nblk(n)), dim3(256), 0, stream, T, x, bc_val, bc_type, scale_t, u, t);
  KFMM_HIP(hipGetLastError());
}

// Restarted GMRES(m) with CGS2 Arnoldi (see file header).  Returns the stats; x holds the best iterate.
bem_stats BemSystem::gmres(const double* x0, const double* x0_alt, double* x, double tol, int m, int max_iter) {
  hipStream_t s = stream;
  bem_stats st{};
  auto t0 = std::chrono::steady_clock::now();
  m = std::max(1, std::min(m, 500));
  if (!x0 && x0_alt) {  // a single start given as the alternative
    x0 = x0_alt;
    x0_alt = nullptr;
  }
  double* b = arena.get<double>(n);
  double* r = arena.get<double>(n);
  double* w = arena.get<double>(n);
  double* V = arena.get<double>((size_t)(m + 1) * n);
  double* d_h = arena.get<double>(m + 2);
  double* zb = pc ? arena.get<double>(n) : nullptr;  // M^-1 of an Arnoldi vector or of the correction
  double* part = scratch_partial();
  apply(1, nullptr, b);
  if (x0) {  // x0 in physical units -> traction unknowns divided by the column scale
    KFMM_HIP(hipMemcpyAsync(x, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    scale_traction_unknowns(*this, x, 1.0 / scale_t);
  } else {
    KFMM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
  }
  const double bnorm = std::sqrt(dot(b, b));
  st.b_norm = bnorm;
  auto dots_host = [&](int nv, const double* vec) {
    hipLaunchKernelGGL(k_dots, dim3(kDotChunks, nv), dim3(256), 0, s, V, (int64_t)n, nv, vec, n, part);
    KFMM_HIP(hipGetLastError());
    std::vector<double> pr((size_t)nv * kDotChunks), h(nv);
    KFMM_HIP(hipMemcpyAsync(pr.data(), part, sizeof(double) * pr.size(), hipMemcpyDeviceToHost, s));
    KFMM_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nv; ++i) {
      double acc = 0;
      for (int c = 0; c < kDotChunks; ++c) acc += pr[(size_t)i * kDotChunks + c];
      h[i] = acc;
    }
    return h;
  };
  if (bnorm == 0.0) {
    KFMM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    st.converged = 1;
    st.rel_res = 0;
    return st;
  }
  // guard: a second start is kept if its true residual is smaller (one extra product)
  double* xa = nullptr;
  double* ra = nullptr;
  double rel_alt = INFINITY;
  if (x0_alt) {
    xa = arena.get<double>(n);
    ra = arena.get<double>(n);
    KFMM_HIP(hipMemcpyAsync(xa, x0_alt, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    scale_traction_unknowns(*this, xa, 1.0 / scale_t);
    apply(0, xa, ra);
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, 1.0, b, -1.0, ra);
    rel_alt = std::sqrt(dot(ra, ra)) / bnorm;
    if (!std::isfinite(rel_alt)) rel_alt = INFINITY;
    st.rel_res_alt = rel_alt;
  }
  int it = 0, stalled = 0;
  double rel = 0, prev_rel = INFINITY;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  while (true) {
    // true residual
    apply(0, x, r);
    hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, 1.0, b, -1.0, r);  // r = b - A x
    double beta = std::sqrt(dot(r, r));
    rel = beta / bnorm;
    if (it == 0 && st.restarts == 0) {
      st.rel_res0 = rel;
      if (x0 && std::isfinite(rel)) {
        // minimal-residual start in span{x0, x0_alt}: with u = A x0 = b - r, v = A xa = b - ra, minimise
        // ||b - a u - c v|| (2 x 2 normal equations); without xa only the scale a.  Both products were
        // computed already, so the projection costs dot products only.
        hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, 1.0, b, -1.0, r);  // r <- A x0
        const double uu = dot(r, r), ub = dot(r, b);
        double a = uu > 0 ? ub / uu : 0.0, c = 0.0;
        if (xa && std::isfinite(rel_alt)) {
          hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, 1.0, b, -1.0, ra);  // ra <- A xa
          const double vv = dot(ra, ra), uv = dot(r, ra), vb = dot(ra, b);
          const double det = uu * vv - uv * uv;
          if (det > 1e-14 * uu * vv) {
            a = (ub * vv - vb * uv) / det;
            c = (vb * uu - ub * uv) / det;
          } else if (vv > 0 && vb * vb / vv > ub * ub / std::max(uu, 1e-300)) {
            a = 0.0;
            c = vb / vv;
          }
        }
        // x <- a x0 + c xa,  r <- b - a A x0 - c A xa
        hipLaunchKernelGGL(k_scale_copy, dim3(nblk(n)), dim3(256), 0, s, n, a, x, x);
        hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, -a, r, 0.0, r);
        if (c != 0.0) {
          hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, c, xa, 1.0, x);
          hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, -c, ra, 1.0, r);
          st.used_alt = 1;
        }
        hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, 1.0, b, 1.0, r);
        KFMM_HIP(hipGetLastError());
        st.start_coef[0] = a;
        st.start_coef[1] = c;
        beta = std::sqrt(dot(r, r));
        rel = beta / bnorm;
        st.rel_res_start = rel;
      }
      // a start whose residual exceeds the zero start's (relative residual 1) is replaced by zero
      if ((x0 || xa) && !(rel <= 1.0)) {
        KFMM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
        KFMM_HIP(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        rel = 1.0;
        beta = bnorm;
        st.used_zero = 1;
        st.rel_res_start = 1.0;
      }
    }
    if (rel <= tol || it >= max_iter || !std::isfinite(rel)) break;
    // stagnation (operator noise floor): five restarts in a row without a 1% decrease of the true residual
    stalled = (it > 0 && rel > 0.99 * prev_rel) ? stalled + 1 : 0;
    prev_rel = rel;
    if (stalled >= 5) break;
    st.restarts++;
    hipLaunchKernelGGL(k_scale_copy, dim3(nblk(n)), dim3(256), 0, s, n, 1.0 / beta, r, V);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m && it < max_iter; ++j) {
      double* vj1 = V + (size_t)(j + 1) * n;
      const double* vin = V + (size_t)j * n;
      if (pc) {
        pc->apply(vin, zb, s);
        vin = zb;
      }
      apply(0, vin, vj1);
      ++it;
      // classical Gram-Schmidt, twice
      std::vector<double> hcol(j + 2, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<double> h = dots_host(j + 1, vj1);
        KFMM_HIP(hipMemcpyAsync(d_h, h.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_sub_many, dim3(nblk(n)), dim3(256), 0, s, V, (int64_t)n, j + 1, d_h, vj1, n);
        KFMM_HIP(hipGetLastError());
        for (int i = 0; i <= j; ++i) hcol[i] += h[i];
      }
      double hn = std::sqrt(dot(vj1, vj1));
      hcol[j + 1] = hn;
      if (hn > 0) hipLaunchKernelGGL(k_scale_copy, dim3(nblk(n)), dim3(256), 0, s, n, 1.0 / hn, vj1, vj1);
      for (int i = 0; i < j; ++i) {
        double a = hcol[i], c = hcol[i + 1];
        hcol[i] = cs[i] * a + sn[i] * c;
        hcol[i + 1] = -sn[i] * a + cs[i] * c;
      }
      double den = std::hypot(hcol[j], hcol[j + 1]);
      cs[j] = den > 0 ? hcol[j] / den : 1.0;
      sn[j] = den > 0 ? hcol[j + 1] / den : 0.0;
      hcol[j] = den;
      hcol[j + 1] = 0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hcol[i];
      k = j + 1;
      st.res_estimate = std::fabs(g[j + 1]) / bnorm;
      if (st.res_estimate <= tol || hn == 0.0) break;
    }
    // y = H^-1 g (upper triangular k x k); x += V y
    std::vector<double> y(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int j2 = i + 1; j2 < k; ++j2) acc -= H[(size_t)i * m + j2] * y[j2];
      y[i] = H[(size_t)i * m + i] != 0 ? acc / H[(size_t)i * m + i] : 0.0;
    }
    KFMM_HIP(hipMemcpyAsync(d_h, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    if (pc) {  // x += M^-1 (V y)
      KFMM_HIP(hipMemsetAsync(w, 0, sizeof(double) * n, s));
      hipLaunchKernelGGL(k_add_many, dim3(nblk(n)), dim3(256), 0, s, V, (int64_t)n, k, d_h, w, n);
      pc->apply(w, zb, s);
      hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(256), 0, s, n, 1.0, zb, 1.0, x);
    } else {
      hipLaunchKernelGGL(k_add_many, dim3(nblk(n)), dim3(256), 0, s, V, (int64_t)n, k, d_h, x, n);
    }
    KFMM_HIP(hipGetLastError());
    st.iters = it;
  }
  st.iters = it;
  st.rel_res = rel;
  st.converged = rel <= tol ? 1 : 0;
  st.n_matvec = n_apply;
  st.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

}  // namespace kfmm

namespace kfmm {

__global__ void k_bem_unscale(int64_t n, const int8_t* __restrict__ bc_type, double scale_t, double* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && bc_type[i] == 0) x[i] *= scale_t;
}

void scale_traction_unknowns(BemSystem& sys, double* x, double factor) {
  hipLaunchKernelGGL(k_bem_unscale, dim3(nblk(sys.n)), dim3(256), 0, sys.stream, sys.n, sys.bc_type, factor, x);
  KFMM_HIP(hipGetLastError());
}

// a = t, b = -u replicated to the 16 quadrature points of each element
__global__ void k_bem_stress_dens(int64_t T, const double* __restrict__ u, const double* __restrict__ t,
                                  double* __restrict__ a, double* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * T) return;
  const int64_t k = i / 3;
  const int c = (int)(i % 3);
  for (int q = 0; q < 16; ++q) {
    a[3 * (16 * k + q) + c] = t[i];
    b[3 * (16 * k + q) + c] = -u[i];
  }
}

void stress_from_boundary(const bem_problem& p, const double* u, const double* t, const double* trg, int64_t M,
                          double* out, const fmm_opts& fo, hipStream_t s) {
  Arena a;
  const int64_t T = p.n_tri, NQ = 16 * T;
  double* qp = a.get<double>(3 * NQ);
  double* qn = a.get<double>(3 * NQ);
  double* qw = a.get<double>(NQ);
  double* cen = a.get<double>(3 * T);
  bem_expand(T, p.tri_xyz, qp, qn, qw, cen, s);
  double* da = a.get<double>(3 * NQ);
  double* db = a.get<double>(3 * NQ);
  hipLaunchKernelGGL(k_bem_stress_dens, dim3(nblk(3 * T)), dim3(256), 0, s, T, u, t, da, db);
  KFMM_HIP(hipGetLastError());
  fmm_opts o = fo;
  o.K = p.K;
  o.G = p.G;
  std::vector<int64_t> bs = {0, NQ}, bt = {0, M};
  std::unique_ptr<Plan> plan(plan_create(qp, qn, qw, NQ, trg, M, bs, bt, o, s, problem_cells(p)));
  plan_eval(*plan, KFMM_STRESS, da, db, out, s);
  KFMM_HIP(hipStreamSynchronize(s));
}

}  // namespace kfmm

namespace kfmm {

// Topological derivative of the compliance at a point with stress sig (eq. deriv; "tr sigma^2" read as the
// square of the trace).
struct Stress6 {
  double v[6];
};

__global__ void k_topo_derivative(const double* __restrict__ sig, int64_t M, double E, double nu, Stress6 off,
                                  double* __restrict__ td) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  double s[6];
  for (int c = 0; c < 6; ++c) s[c] = sig[6 * i + c] + off.v[c];
  double ss = s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
  double tr = s[0] + s[1] + s[2];
  td[i] = 3.0 * (1.0 - nu) / (4.0 * E * (7.0 - 5.0 * nu)) * (10.0 * (1.0 + nu) * ss - (1.0 + 5.0 * nu) * tr * tr);
}

void topological_derivative(const double* sig, int64_t M, const Elastic& el, double* td, hipStream_t s,
                            const double* sig_h) {
  const double E = 9.0 * el.K * el.G / (3.0 * el.K + el.G);
  Stress6 off{};
  if (sig_h)
    for (int c = 0; c < 6; ++c) off.v[c] = sig_h[c];
  hipLaunchKernelGGL(k_topo_derivative, dim3(nblk(M)), dim3(256), 0, s, sig, M, E, el.nu, off, td);
  KFMM_HIP(hipGetLastError());
}

}  // namespace kfmm
