/*
 * Oracle (test infrastructure only): plain FP64 direct summation of the Kelvin
 * elastostatic kernels.  Only tests/, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library; the product path never does.
 *
 * Follows the paper's summation contract (eq. fmm_summation, Sec. 2.2, "Numerical
 * solution"): t_i = sum_j K(x_i, y_j, n_j) s_j, with the double-layer normal taken at
 * the source.  Kernels:
 *   U_ij  eq. disp_1 (Sec. 2.1, as printed),
 *   P_ij  eq. disp_2, read with the textbook leading minus and r_hat = (source - target)/r,
 *   D_kij eq. stress_2, read with denominator 8*pi*(1-nu)*r^2 (the printed 2*pi is taken
 *         as a typo: only 8*pi makes D the stress of U),
 *   S_kij eq. stress_3, read with the shear modulus G as an overall factor (the printed
 *         form is exact only for G = 1).
 * Moduli: nu = (3K - 2G) / (2(3K + G)), from the stiffness tensor of eq. elast.
 *
 * Result definition (no blocking, no reordering beyond a parallel loop over targets):
 *   DISP   : v_t,i   = sum_{s : y_s != x_t} U_ij (w_s a_s)_j + P_ij (w_s b_s)_j
 *   STRESS : sig_t,ij = sum_{s : y_s != x_t} D_kij (w_s a_s)_k + S_kij (w_s b_s)_k
 * Stress output order: xx, yy, zz, yz, xz, xy.
 * Parity pinned by tests/test_oracle_kernels.py (finite-difference and integral identities).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846;

static double poisson_ratio(double K, double G) { return (3.0 * K - 2.0 * G) / (2.0 * (3.0 * K + G)); }

static double kron(int i, int j) { return i == j ? 1.0 : 0.0; }

/* U_ij(target, source) of eq. disp_1.  rh = unit vector source - target, r = distance. */
static void kernel_U(const double rh[3], double r, double nu, double G, double U[3][3]) {
  double c = 1.0 / (16.0 * PI * (1.0 - nu) * G * r);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) U[i][j] = c * ((3.0 - 4.0 * nu) * kron(i, j) + rh[i] * rh[j]);
}

/* P_ij(target, source, n_source) of eq. disp_2 with the leading minus (reading above). */
static void kernel_P(const double rh[3], double r, const double n[3], double nu, double P[3][3]) {
  double drdn = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
  double c = -1.0 / (8.0 * PI * (1.0 - nu) * r * r);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      P[i][j] = c * (drdn * ((1.0 - 2.0 * nu) * kron(i, j) + 3.0 * rh[i] * rh[j]) -
                     (1.0 - 2.0 * nu) * (rh[i] * n[j] - rh[j] * n[i]));
}

/* D_kij of eq. stress_2 with the 8*pi denominator. */
static void kernel_D(const double rh[3], double r, double nu, double D[3][3][3]) {
  double c = 1.0 / (8.0 * PI * (1.0 - nu) * r * r);
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        D[k][i][j] = c * ((1.0 - 2.0 * nu) * (kron(k, i) * rh[j] + kron(k, j) * rh[i] - kron(i, j) * rh[k]) +
                          3.0 * rh[i] * rh[j] * rh[k]);
}

/* S_kij of eq. stress_3, times G. */
static void kernel_S(const double rh[3], double r, const double n[3], double nu, double G, double S[3][3][3]) {
  double drdn = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
  double c = G / (4.0 * PI * (1.0 - nu) * r * r * r);
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double t1 = 3.0 * drdn *
                    ((1.0 - 2.0 * nu) * kron(i, j) * rh[k] + nu * (kron(i, k) * rh[j] + kron(j, k) * rh[i]) -
                     5.0 * rh[i] * rh[j] * rh[k]);
        double t2 = 3.0 * nu * (n[i] * rh[j] * rh[k] + n[j] * rh[i] * rh[k]);
        double t3 = (1.0 - 2.0 * nu) * (3.0 * n[k] * rh[i] * rh[j] + n[j] * kron(i, k) + n[i] * kron(j, k));
        double t4 = -(1.0 - 4.0 * nu) * n[k] * kron(i, j);
        S[k][i][j] = c * (t1 + t2 + t3 + t4);
      }
}

static const int VOIGT_I[6] = {0, 1, 2, 1, 0, 0};
static const int VOIGT_J[6] = {0, 1, 2, 2, 2, 1};

/* Geometry of one pair: returns 0 when the source coincides with the target (pair skipped). */
static int pair_geometry(const double* x, const double* y, double rh[3], double* r) {
  double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
  double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (rr == 0.0) return 0;
  for (int i = 0; i < 3; ++i) rh[i] = d[i] / rr;
  *r = rr;
  return 1;
}

/*
 * Direct sum.  kind 0 = DISP (out M x 3), kind 1 = STRESS (out M x 6).
 * a, b may be NULL (treated as zero); nrm may be NULL only when b is NULL.
 * Returns 0 on success, -1 on bad arguments.
 */
int oracle_direct(int kind, double K, double G, const double* trg, int64_t M, const double* src, const double* nrm,
                  const double* w, const double* a, const double* b, int64_t N, double* out, int nthreads) {
  if (kind != 0 && kind != 1) return -1;
  if (!(K > 0.0) || !(G > 0.0)) return -1;
  if (b && !nrm) return -1;
  double nu = poisson_ratio(K, G);
  int nout = kind == 0 ? 3 : 6;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < M; ++t) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t s = 0; s < N; ++s) {
      double rh[3], r;
      if (!pair_geometry(trg + 3 * t, src + 3 * s, rh, &r)) continue;
      double wa[3] = {0, 0, 0}, wb[3] = {0, 0, 0};
      for (int k = 0; k < 3; ++k) {
        if (a) wa[k] = w[s] * a[3 * s + k];
        if (b) wb[k] = w[s] * b[3 * s + k];
      }
      if (kind == 0) {
        if (a) {
          double U[3][3];
          kernel_U(rh, r, nu, G, U);
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc[i] += U[i][j] * wa[j];
        }
        if (b) {
          double P[3][3];
          kernel_P(rh, r, nrm + 3 * s, nu, P);
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc[i] += P[i][j] * wb[j];
        }
      } else {
        if (a) {
          double D[3][3][3];
          kernel_D(rh, r, nu, D);
          for (int v = 0; v < 6; ++v)
            for (int k = 0; k < 3; ++k) acc[v] += D[k][VOIGT_I[v]][VOIGT_J[v]] * wa[k];
        }
        if (b) {
          double S[3][3][3];
          kernel_S(rh, r, nrm + 3 * s, nu, G, S);
          for (int v = 0; v < 6; ++v)
            for (int k = 0; k < 3; ++k) acc[v] += S[k][VOIGT_I[v]][VOIGT_J[v]] * wb[k];
        }
      }
    }
    for (int v = 0; v < nout; ++v) out[nout * t + v] = acc[v];
  }
  return 0;
}

/*
 * Dense quadrature blocks of the collocation BEM (eq. coef, Sec. 2.2): for collocation point t
 * and element e,  Umat[3t+i, 3e+j] = sum_{s in e} U_ij(x_t, y_s) w_s  and likewise Pmat with P.
 * elem[s] names the element that quadrature point s belongs to.  Coincident pairs are skipped.
 * Matrices are row-major (3M) x (3E) and are overwritten.
 */
int oracle_quad_blocks(double K, double G, const double* trg, int64_t M, const double* src, const double* nrm,
                       const double* w, const int64_t* elem, int64_t N, int64_t E, double* Umat, double* Pmat,
                       int nthreads) {
  if (!(K > 0.0) || !(G > 0.0)) return -1;
  double nu = poisson_ratio(K, G);
  int64_t ncol = 3 * E;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t t = 0; t < M; ++t) {
    double* urow[3];
    double* prow[3];
    for (int i = 0; i < 3; ++i) {
      urow[i] = Umat + (3 * t + i) * ncol;
      prow[i] = Pmat + (3 * t + i) * ncol;
      memset(urow[i], 0, sizeof(double) * ncol);
      memset(prow[i], 0, sizeof(double) * ncol);
    }
    for (int64_t s = 0; s < N; ++s) {
      double rh[3], r;
      if (!pair_geometry(trg + 3 * t, src + 3 * s, rh, &r)) continue;
      double U[3][3], P[3][3];
      kernel_U(rh, r, nu, G, U);
      kernel_P(rh, r, nrm + 3 * s, nu, P);
      int64_t e = elem[s];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          urow[i][3 * e + j] += U[i][j] * w[s];
          prow[i][3 * e + j] += P[i][j] * w[s];
        }
    }
  }
  return 0;
}

/* Kernel values for a list of single pairs (for identity checks): U, P (9 each) and D, S (27 each, [k][i][j]). */
int oracle_pair_kernels(double K, double G, const double* trg, const double* src, const double* nrm, int64_t n,
                        double* U, double* P, double* D, double* S) {
  if (!(K > 0.0) || !(G > 0.0)) return -1;
  double nu = poisson_ratio(K, G);
  for (int64_t p = 0; p < n; ++p) {
    double rh[3], r;
    if (!pair_geometry(trg + 3 * p, src + 3 * p, rh, &r)) return -1;
    kernel_U(rh, r, nu, G, (double(*)[3])(U + 9 * p));
    kernel_P(rh, r, nrm + 3 * p, nu, (double(*)[3])(P + 9 * p));
    kernel_D(rh, r, nu, (double(*)[3][3])(D + 27 * p));
    kernel_S(rh, r, nrm + 3 * p, nu, G, (double(*)[3][3])(S + 27 * p));
  }
  return 0;
}

/*
 * Upsampled quadrature of near-singular blocks (Sec. 2.2, "Matrix-vector products": near the collocation
 * point the element's 16-point rule loses accuracy, and an upsampled quadrature is used on the triangles
 * close to it).  For each pair (t, e): the triangle e (tri + 9e, vertices v0 v1 v2) is split at its edge
 * midpoints L + 1 times, each split giving the four children (v0, m01, m20), (m01, v1, m12),
 * (m20, m12, v2), (m01, m12, m20) in that order; on each of the 4^(L+1) leaves the symmetric degree-3
 * four-point rule (centroid weight -27/48; barycentric (3/5, 1/5, 1/5) and permutations, 25/48) is
 * applied with weights (leaf area) x (rule weight).  L = 0 is the element's own 16-point rule.  Leaves
 * are visited in the order of their base-4 child index (first split most significant).
 *   U[9p + 3i + j] = sum_q U_ij(x_t, y_q) w_q,  P likewise with P_ij and the normal of e (right-hand rule).
 * Coincident points are skipped.  Returns 0, or -1 on bad arguments.
 */
int oracle_near_blocks(double K, double G, const double* colloc, const double* tri, const int64_t* pairs,
                       int64_t n, int L, double* U, double* P, int nthreads) {
  if (!(K > 0.0) || !(G > 0.0) || L < 0 || L > 8) return -1;
  double nu = poisson_ratio(K, G);
  static const double bary[4][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
  static const double rw[4] = {-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48};
  int64_t nleaf = 1;
  for (int d = 0; d <= L; ++d) nleaf *= 4;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < n; ++p) {
    const double* x = colloc + 3 * pairs[2 * p];
    const double* v = tri + 9 * pairs[2 * p + 1];
    double e1[3], e2[3], nr[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = v[3 + d] - v[d];
      e2[d] = v[6 + d] - v[d];
    }
    nr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    nr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    nr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double a2 = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
    for (int d = 0; d < 3; ++d) nr[d] /= a2;
    double leaf_area = 0.5 * a2 / (double)nleaf;
    double Ua[3][3] = {{0}}, Pa[3][3] = {{0}};
    for (int64_t k = 0; k < nleaf; ++k) {
      double c[3][3];
      memcpy(c, v, sizeof(c));
      for (int64_t div = nleaf / 4; div >= 1; div /= 4) {
        int child = (int)((k / div) % 4);
        double m01[3], m12[3], m20[3];
        for (int d = 0; d < 3; ++d) {
          m01[d] = 0.5 * (c[0][d] + c[1][d]);
          m12[d] = 0.5 * (c[1][d] + c[2][d]);
          m20[d] = 0.5 * (c[2][d] + c[0][d]);
        }
        for (int d = 0; d < 3; ++d) {
          double a = c[0][d], b = c[1][d], cc = c[2][d];
          if (child == 0) { c[0][d] = a;       c[1][d] = m01[d]; c[2][d] = m20[d]; }
          if (child == 1) { c[0][d] = m01[d];  c[1][d] = b;      c[2][d] = m12[d]; }
          if (child == 2) { c[0][d] = m20[d];  c[1][d] = m12[d]; c[2][d] = cc;     }
          if (child == 3) { c[0][d] = m01[d];  c[1][d] = m12[d]; c[2][d] = m20[d]; }
        }
      }
      for (int q = 0; q < 4; ++q) {
        double y[3], rh[3], r;
        for (int d = 0; d < 3; ++d) y[d] = bary[q][0] * c[0][d] + bary[q][1] * c[1][d] + bary[q][2] * c[2][d];
        if (!pair_geometry(x, y, rh, &r)) continue;
        double Uq[3][3], Pq[3][3], w = leaf_area * rw[q];
        kernel_U(rh, r, nu, G, Uq);
        kernel_P(rh, r, nr, nu, Pq);
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            Ua[i][j] += Uq[i][j] * w;
            Pa[i][j] += Pq[i][j] * w;
          }
      }
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        U[9 * p + 3 * i + j] = Ua[i][j];
        P[9 * p + 3 * i + j] = Pa[i][j];
      }
  }
  return 0;
}
