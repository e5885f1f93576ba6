/*
 * Oracle (test infrastructure only): FP64 periodic sums of the Kelvin kernels by Ewald summation.
 * Only tests/, the smoke check and the CPU-baseline leg of the benchmark may load this library.
 *
 * What is summed (Sec. 4.3, periodic cell of a metamaterial): the boundary integrals of eq. fmm_summation
 * taken over the infinite periodic surface, i.e. over every lattice image y + nL (n in Z^3) of every
 * source of a cubic cell of side L:
 *   DISP   : v(xi)   = sum_s sum_n U(y_s + nL - xi) w_s a_s + P(y_s + nL - xi, n_s) w_s b_s
 *   STRESS : sig(xi) = the same with D and S (the stress of that displacement field).
 * Reading (the paper names no summation order): the lattice sum of the point-force field converges only
 * conditionally; it is defined by its Fourier series over the reciprocal lattice k = 2 pi m / L with the
 * k = 0 term left out.  That is the periodic field with zero cell mean (a net force per cell is balanced
 * by a uniform body force).  P, D and S are the same derivatives of that periodic point-force field as
 * in free space.  The image n = 0 of a source that coincides with the target is left out (as in free
 * space), all other images are kept.
 *
 * Method (plain Ewald splitting, every step a closed form):
 *   U_ij = delta_ij Phi / (4 pi G) - c_B d_i d_j B,   Phi = 1/r,  B = r,  c_B = 1 / (16 pi (1 - nu) G),
 * which is the Kelvin solution since d_i d_j r = delta_ij / r - x_i x_j / r^3.
 *   Phi = erfc(a r)/r                          + [Fourier: 4 pi exp(-s) / k^2]
 *   B   = r erfc(a r) - exp(-a^2 r^2)/(a sqrt(pi)) + [Fourier: -8 pi (1 + s) exp(-s) / k^4],  s = k^2/(4a^2)
 * The real-space parts decay like exp(-a^2 r^2) and are summed over nearby images; the Fourier parts
 * decay like exp(-s) and are summed over |m| <= kmax with structure factors.  Leaving out k = 0 adds the
 * constant -pi/(a^2 V) to Phi (the k -> 0 limit of the real-space part's transform); no other
 * derivative order has one.  Derivative tensors of a radial F(r) come from the operator Dr = (1/r) d/dr:
 *   d_i F = x_i Dr F,  d_i d_j F = delta_ij Dr F + x_i x_j Dr^2 F, ... (orders 3 and 4 likewise),
 * and Dr maps r^p erfc(a r) and r^p exp(-a^2 r^2) into the same family, so every Dr^m F is kept as
 * coefficient lists and evaluated at r.
 *
 * Assembly from U and its derivatives (d = source - target):
 *   P_ij b_j  = d_m U_il Q_lm,   Q_lm = C_lmjk b_j n_k           (traction of the point-force field)
 *   grad_xi v = -d_q (...),      sig_ij = lambda delta_ij tr(g) + G (g_ij + g_ji)   (eq. elast)
 * Pinned by tests/test_oracle_periodic.py.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI_E = 3.14159265358979323846;

#define PMIN (-14)
#define PMAX 3
#define NPW (PMAX - PMIN + 1)

/* F(r) = sum_p ce[p] r^p erfc(a r) + sum_p cg[p] r^p exp(-a^2 r^2) */
typedef struct {
  double ce[NPW], cg[NPW];
} radial;

static void rad_dr(const radial* f, radial* out, double a) {
  const double c = 2.0 * a / sqrt(PI_E);
  memset(out, 0, sizeof(*out));
  for (int i = 0; i < NPW; ++i) {
    const int p = i + PMIN;
    if (f->ce[i] != 0.0) {
      /* Dr (r^p erfc) = p r^(p-2) erfc - c r^(p-1) exp */
      if (p != 0) out->ce[i - 2] += p * f->ce[i];
      out->cg[i - 1] += -c * f->ce[i];
    }
    if (f->cg[i] != 0.0) {
      /* Dr (r^p exp) = p r^(p-2) exp - 2 a^2 r^p exp */
      if (p != 0) out->cg[i - 2] += p * f->cg[i];
      out->cg[i] += -2.0 * a * a * f->cg[i];
    }
  }
}

static double rad_eval(const radial* f, double r, double a) {
  const double ec = erfc(a * r), eg = exp(-a * a * r * r);
  double s = 0.0;
  for (int i = 0; i < NPW; ++i) {
    const int p = i + PMIN;
    if (f->ce[i] != 0.0) s += f->ce[i] * pow(r, p) * ec;
    if (f->cg[i] != 0.0) s += f->cg[i] * pow(r, p) * eg;
  }
  return s;
}

/* Derivative tensors of a radial function at x (|x| = r) from f[m] = Dr^m F (m = 0..4).
   t1[i], t2[i][j], t3[i][j][k], t4[i][j][k][l] as requested by `order`. */
static double dl(int i, int j) { return i == j ? 1.0 : 0.0; }

typedef struct {
  double t0, t1[3], t2[3][3], t3[3][3][3], t4[3][3][3][3];
} dtens;

static void radial_tensors(const double x[3], const double f[5], int order, dtens* T) {
  T->t0 = f[0];
  for (int i = 0; i < 3; ++i) T->t1[i] = x[i] * f[1];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T->t2[i][j] = dl(i, j) * f[1] + x[i] * x[j] * f[2];
  if (order < 3) return;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        T->t3[i][j][k] = (dl(i, j) * x[k] + dl(i, k) * x[j] + dl(j, k) * x[i]) * f[2] + x[i] * x[j] * x[k] * f[3];
  if (order < 4) return;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
          T->t4[i][j][k][l] =
              (dl(i, j) * dl(k, l) + dl(i, k) * dl(j, l) + dl(i, l) * dl(j, k)) * f[2] +
              (dl(i, j) * x[k] * x[l] + dl(i, k) * x[j] * x[l] + dl(i, l) * x[j] * x[k] + dl(j, k) * x[i] * x[l] +
               dl(j, l) * x[i] * x[k] + dl(k, l) * x[i] * x[j]) * f[3] +
              x[i] * x[j] * x[k] * x[l] * f[4];
}

/* U, dU (U1[l][k][m] = d_m U_lk), d2U (U2[l][k][m][q]) from the tensors of Phi and B. */
typedef struct {
  double U[3][3], U1[3][3][3], U2[3][3][3][3];
} ukern;

static void assemble_u(const dtens* ph, const dtens* bb, double G, double cB, int need2, ukern* K) {
  const double cp = 1.0 / (4.0 * PI_E * G);
  for (int l = 0; l < 3; ++l)
    for (int k = 0; k < 3; ++k) {
      K->U[l][k] = dl(l, k) * cp * ph->t0 - cB * bb->t2[l][k];
      for (int m = 0; m < 3; ++m) {
        K->U1[l][k][m] = dl(l, k) * cp * ph->t1[m] - cB * bb->t3[l][k][m];
        if (need2)
          for (int q = 0; q < 3; ++q) K->U2[l][k][m][q] = dl(l, k) * cp * ph->t2[m][q] - cB * bb->t4[l][k][m][q];
      }
    }
}

/* Accumulate one source image: displacement v (DISP) or displacement gradient g[l][q] = d v_l / d xi_q
   (STRESS) from U-tensors K, single-layer weight wa and dipole tensor Q. */
static void accumulate(int kind, const ukern* K, const double* wa, const double Q[3][3], double* v, double g[3][3]) {
  if (kind == 0) {
    for (int l = 0; l < 3; ++l) {
      double s = 0.0;
      if (wa)
        for (int k = 0; k < 3; ++k) s += K->U[l][k] * wa[k];
      if (Q)
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) s += K->U1[l][a][b] * Q[a][b];
      v[l] += s;
    }
  } else {
    for (int l = 0; l < 3; ++l)
      for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        if (wa)
          for (int k = 0; k < 3; ++k) s -= K->U1[l][k][q] * wa[k];
        if (Q)
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) s -= K->U2[l][a][b][q] * Q[a][b];
        g[l][q] += s;
      }
  }
}

static const int VI[6] = {0, 1, 2, 1, 0, 0};
static const int VJ[6] = {0, 1, 2, 2, 2, 1};

/*
 * oracle_periodic -- Ewald sum as described above.
 *   kind 0 DISP (out M x 3), 1 STRESS (out M x 6: xx, yy, zz, yz, xz, xy)
 *   L cell side; alpha splitting parameter (1/length); nreal images |n_i| <= nreal in real space, pairs
 *   farther than rcut skipped; kmax reciprocal vectors |m_i| <= kmax.
 *   free_space != 0: no images, no Fourier part, Phi = 1/r and B = r exactly (the free-space kernels
 *   through the same tensor algebra; a check of that algebra).
 * Returns 0, or -1 on bad arguments.
 */
int oracle_periodic(int kind, double K, double G, double L, const double* trg, int64_t M, const double* src,
                    const double* nrm, const double* w, const double* a, const double* b, int64_t N, double alpha,
                    int nreal, double rcut, int kmax, int free_space, double* out, int nthreads) {
  if (kind != 0 && kind != 1) return -1;
  if (!(K > 0.0) || !(G > 0.0) || !(L > 0.0)) return -1;
  if (b && !nrm) return -1;
  if (!free_space && !(alpha > 0.0)) return -1;
  const double nu = (3.0 * K - 2.0 * G) / (2.0 * (3.0 * K + G));
  const double lam = K - 2.0 * G / 3.0;
  const double cB = 1.0 / (16.0 * PI_E * (1.0 - nu) * G);
  const double V = L * L * L;
  const int nout = kind == 0 ? 3 : 6;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  /* radial families and their Dr powers */
  radial phi[5], bb[5];
  memset(phi, 0, sizeof(phi));
  memset(bb, 0, sizeof(bb));
  phi[0].ce[-1 - PMIN] = 1.0;
  bb[0].ce[1 - PMIN] = 1.0;
  if (!free_space) bb[0].cg[0 - PMIN] = -1.0 / (alpha * sqrt(PI_E));
  for (int m = 1; m < 5; ++m) {
    rad_dr(&phi[m - 1], &phi[m], free_space ? 0.0 : alpha);
    rad_dr(&bb[m - 1], &bb[m], free_space ? 0.0 : alpha);
  }
  const double ae = free_space ? 0.0 : alpha;
  /* per-source weights: wa = w a, Q_lm = C_lmjk (w b)_j n_k = lambda delta_lm (wb.n) + G ((wb)_l n_m + (wb)_m n_l) */
  double* WA = a ? (double*)malloc(sizeof(double) * 3 * (size_t)(N > 0 ? N : 1)) : NULL;
  double* WQ = b ? (double*)malloc(sizeof(double) * 9 * (size_t)(N > 0 ? N : 1)) : NULL;
  for (int64_t s = 0; s < N; ++s) {
    if (a)
      for (int k = 0; k < 3; ++k) WA[3 * s + k] = w[s] * a[3 * s + k];
    if (b) {
      const double* n = nrm + 3 * s;
      double wb[3], bn = 0.0;
      for (int k = 0; k < 3; ++k) {
        wb[k] = w[s] * b[3 * s + k];
        bn += wb[k] * n[k];
      }
      for (int l = 0; l < 3; ++l)
        for (int m = 0; m < 3; ++m) WQ[9 * s + 3 * l + m] = lam * dl(l, m) * bn + G * (wb[l] * n[m] + wb[m] * n[l]);
    }
  }
  /* limits of U^real - U at coincidence (Taylor series of erf and exp at 0): U -> (2a/sqrt(pi)) (c_B - 1/(4 pi G))
     delta, dU -> 0, d2U_lkmq -> (4a^3/(3 sqrt(pi))) [delta_lk delta_mq / (4 pi G) - c_B (delta_lk delta_mq +
     delta_lm delta_kq + delta_lq delta_km)] */
  ukern Kreg;
  memset(&Kreg, 0, sizeof(Kreg));
  if (!free_space) {
    const double c1 = 2.0 * alpha / sqrt(PI_E), c3 = 4.0 * alpha * alpha * alpha / (3.0 * sqrt(PI_E));
    for (int l = 0; l < 3; ++l)
      for (int k = 0; k < 3; ++k) {
        Kreg.U[l][k] = dl(l, k) * c1 * (cB - 1.0 / (4.0 * PI_E * G));
        for (int m = 0; m < 3; ++m)
          for (int q = 0; q < 3; ++q)
            Kreg.U2[l][k][m][q] = c3 * (dl(l, k) * dl(m, q) / (4.0 * PI_E * G) -
                                        cB * (dl(l, k) * dl(m, q) + dl(l, m) * dl(k, q) + dl(l, q) * dl(k, m)));
      }
  }
  const int nr = free_space ? 0 : nreal;
  const int need2 = kind == 1 && b != NULL;
  double* acc = (double*)calloc((size_t)(M > 0 ? M : 1) * 12, sizeof(double)); /* v (3) and g (9) per target */
  /* ---- real space */
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t t = 0; t < M; ++t) {
    const double* xi = trg + 3 * t;
    double v[3] = {0, 0, 0}, g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int64_t s = 0; s < N; ++s) {
      const double* wa = a ? WA + 3 * s : NULL;
      double Q[3][3];
      if (b)
        for (int l = 0; l < 3; ++l)
          for (int m = 0; m < 3; ++m) Q[l][m] = WQ[9 * s + 3 * l + m];
      for (int nx = -nr; nx <= nr; ++nx)
        for (int ny = -nr; ny <= nr; ++ny)
          for (int nz = -nr; nz <= nr; ++nz) {
            double d[3] = {src[3 * s] + nx * L - xi[0], src[3 * s + 1] + ny * L - xi[1], src[3 * s + 2] + nz * L - xi[2]};
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 == 0.0) {
              if (!free_space) accumulate(kind, &Kreg, wa, b ? (const double(*)[3])Q : NULL, v, g);
              continue;
            }
            if (!free_space && r2 > rcut * rcut) continue;
            const double r = sqrt(r2);
            double fp[5] = {0, 0, 0, 0, 0}, fb[5] = {0, 0, 0, 0, 0};
            for (int m = 0; m < 3; ++m) fp[m] = rad_eval(&phi[m], r, ae);
            for (int m = 1; m < 5; ++m)
              if (m < 4 || need2) fb[m] = rad_eval(&bb[m], r, ae);
            dtens tp, tb;
            radial_tensors(d, fp, 2, &tp);
            radial_tensors(d, fb, need2 ? 4 : 3, &tb);
            ukern Kk;
            assemble_u(&tp, &tb, G, cB, need2, &Kk);
            accumulate(kind, &Kk, wa, b ? (const double(*)[3])Q : NULL, v, g);
          }
    }
    double* o = acc + 12 * t;
    for (int l = 0; l < 3; ++l) {
      o[l] += v[l];
      for (int q = 0; q < 3; ++q) o[3 + 3 * l + q] += g[l][q];
    }
  }
  /* ---- reciprocal space: half of the vectors m != 0 (m and -m give complex conjugates) */
  if (!free_space && kmax > 0) {
    const int side = 2 * kmax + 1;
    int64_t nk = 0;
    int* mv = (int*)malloc(sizeof(int) * 3 * (size_t)side * side * side);
    for (int mx = -kmax; mx <= kmax; ++mx)
      for (int my = -kmax; my <= kmax; ++my)
        for (int mz = -kmax; mz <= kmax; ++mz) {
          const int pos = mx > 0 || (mx == 0 && my > 0) || (mx == 0 && my == 0 && mz > 0);
          if (!pos) continue;
          mv[3 * nk] = mx;
          mv[3 * nk + 1] = my;
          mv[3 * nk + 2] = mz;
          ++nk;
        }
    /* c(k) = Uhat(k) z(k), z(k) = sum_s exp(i k.y_s) (wa_s + i Q_s k), Uhat z = Phihat/(4 pi G) z + c_B Bhat k (k.z) */
    double* cre = (double*)calloc((size_t)nk * 3, sizeof(double));
    double* cim = (double*)calloc((size_t)nk * 3, sizeof(double));
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t j = 0; j < nk; ++j) {
      const double k[3] = {2.0 * PI_E * mv[3 * j] / L, 2.0 * PI_E * mv[3 * j + 1] / L, 2.0 * PI_E * mv[3 * j + 2] / L};
      const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
      const double sx = k2 / (4.0 * alpha * alpha);
      const double ph = 4.0 * PI_E * exp(-sx) / k2;
      const double bh = -8.0 * PI_E * (1.0 + sx) * exp(-sx) / (k2 * k2);
      double zr[3] = {0, 0, 0}, zi[3] = {0, 0, 0};
      for (int64_t s = 0; s < N; ++s) {
        const double th = k[0] * src[3 * s] + k[1] * src[3 * s + 1] + k[2] * src[3 * s + 2];
        const double cs = cos(th), sn = sin(th);
        double ur[3] = {0, 0, 0}, ui[3] = {0, 0, 0}; /* wa + i Q k */
        if (a)
          for (int l = 0; l < 3; ++l) ur[l] = WA[3 * s + l];
        if (b)
          for (int l = 0; l < 3; ++l)
            for (int m = 0; m < 3; ++m) ui[l] += WQ[9 * s + 3 * l + m] * k[m];
        for (int l = 0; l < 3; ++l) {
          zr[l] += cs * ur[l] - sn * ui[l];
          zi[l] += cs * ui[l] + sn * ur[l];
        }
      }
      const double kzr = k[0] * zr[0] + k[1] * zr[1] + k[2] * zr[2], kzi = k[0] * zi[0] + k[1] * zi[1] + k[2] * zi[2];
      for (int l = 0; l < 3; ++l) {
        cre[3 * j + l] = ph / (4.0 * PI_E * G) * zr[l] + cB * bh * k[l] * kzr;
        cim[3 * j + l] = ph / (4.0 * PI_E * G) * zi[l] + cB * bh * k[l] * kzi;
      }
    }
    /* field at xi: (2/V) Re sum c(k) exp(-i k.xi); gradient: (2/V) Re sum c(k) (-i k_q) exp(-i k.xi) */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < M; ++t) {
      const double* xi = trg + 3 * t;
      double v[3] = {0, 0, 0}, g[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int64_t j = 0; j < nk; ++j) {
        const double k[3] = {2.0 * PI_E * mv[3 * j] / L, 2.0 * PI_E * mv[3 * j + 1] / L, 2.0 * PI_E * mv[3 * j + 2] / L};
        const double th = k[0] * xi[0] + k[1] * xi[1] + k[2] * xi[2];
        const double cs = cos(th), sn = -sin(th); /* exp(-i th) = cs + i sn */
        for (int l = 0; l < 3; ++l) {
          const double er = cre[3 * j + l] * cs - cim[3 * j + l] * sn; /* Re(c e) */
          const double ei = cre[3 * j + l] * sn + cim[3 * j + l] * cs; /* Im(c e) */
          if (kind == 0) {
            v[l] += er;
          } else {
            for (int q = 0; q < 3; ++q) g[l][q] += k[q] * ei; /* Re(-i k_q c e) = k_q Im(c e) */
          }
        }
      }
      double* o = acc + 12 * t;
      for (int l = 0; l < 3; ++l) {
        o[l] += 2.0 / V * v[l];
        for (int q = 0; q < 3; ++q) o[3 + 3 * l + q] += 2.0 / V * g[l][q];
      }
    }
    free(cre);
    free(cim);
    free(mv);
  }
  /* ---- constant of Phi (k = 0 left out): U gets -delta / (4 a^2 G V); only the single-layer displacement */
  double cst[3] = {0, 0, 0};
  if (!free_space && a && kind == 0)
    for (int64_t s = 0; s < N; ++s)
      for (int l = 0; l < 3; ++l) cst[l] -= WA[3 * s + l] / (4.0 * alpha * alpha * G * V);
  for (int64_t t = 0; t < M; ++t) {
    const double* o = acc + 12 * t;
    if (kind == 0) {
      for (int l = 0; l < 3; ++l) out[3 * t + l] = o[l] + cst[l];
    } else {
      const double* g = o + 3; /* g[l][q] at g[3 l + q] */
      const double tr = g[0] + g[4] + g[8];
      for (int c = 0; c < 6; ++c) {
        const int i = VI[c], j = VJ[c];
        out[6 * t + c] = lam * dl(i, j) * tr + G * (g[3 * i + j] + g[3 * j + i]);
      }
    }
  }
  free(acc);
  free(WA);
  free(WQ);
  (void)nout;
  return 0;
}
