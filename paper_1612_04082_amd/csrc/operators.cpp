// Host-side FP64 precompute of the KIFMM translation operators (Sec. 2.2, "Kernel-independent fast
// multipole method": far and local fields are densities on equivalent surfaces; M2M, M2L and L2L are
// matrices computed from the kernel alone).
//
// Surfaces are cube surfaces with p points per edge (6(p-1)^2+2 points) around a box of half-width r:
//   upward equivalent 1.05 r, upward check 2.95 r, downward check 1.05 r, downward equivalent 2.95 r.
// The equivalent density is always a single-layer (Kelvin U) density.  Because U is homogeneous of
// degree -1, every operator below is computed once at unit half-width and is level-invariant:
//   UC2UE  = pinv(U[uc <- ue])                      leaf:   phi_up = r_l * UC2UE * q_check
//   M2M_c  = UC2UE * U[parent uc <- child c ue]     parent: phi_up = sum_c M2M_c * phi_up(child c)
//   M2L_d  = U[dc <- ue shifted by 2d]              qhat(B) += M2L_d * phi_up(A),  d = index offset A - B
//   DC2DE  = pinv(U[dc <- de]) = UC2UE^T            phi_down = DC2DE * qhat
//   L2L_c  = DC2DE * U[child c dc <- parent de]     phi_down(child) += L2L_c * phi_down(parent)
// where qhat = r_l * (downward check potential).  U is symmetric and reciprocal, so U[dc<-de] is the
// transpose of U[uc<-ue] and one SVD serves both pseudo-inverses.
//
// The pseudo-inverses are also kept in factored form, U[uc<-ue] = Us S Vs^T:
//   UC2UE = (Vs S^-1) Us^T,   DC2DE = (Us S^-1) Vs^T.
// Applied as the two factors in turn, each product rounds relative to its own terms (an orthogonal
// rotation, then a column-scaled one), so they can run in FP32: the explicit UC2UE has entries up to
// 1/s_min with heavy cancellation against a smooth check potential, and FP32 rounding of those entries
// or of their running sum leaves errors far above the field itself.
//
// The same translations written on check potentials (qhat = r_l * check potential, phi = UC2UE qhat up,
// phi = DC2DE qhat down):
//   M2M_q_c = U[parent uc <- child c ue] * UC2UE     qhat_up(parent) = sum_c M2M_q_c * qhat_up(child c)
//   L2L_q_c = U[child c dc <- parent de] * DC2DE     qhat_dn(child) += L2L_q_c * qhat_dn(parent)
// A check potential is a smooth field sample, and these operators map smooth fields to smooth fields
// without cancellation, so chains of them run in FP32; an equivalent density carries the pinv's
// amplified high-order modes, and every product with it (M2M_c, L2L_c) cancels them in its sum.
#include <sys/stat.h>
#include <sys/types.h>

#include <cerrno>
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "operators.h"

namespace kfmm {

std::vector<double> cube_surface(int p) {
  std::vector<double> pts;
  for (int k = 0; k < p; ++k)
    for (int j = 0; j < p; ++j)
      for (int i = 0; i < p; ++i) {
        if (i != 0 && i != p - 1 && j != 0 && j != p - 1 && k != 0 && k != p - 1) continue;
        pts.push_back(-1.0 + 2.0 * i / (p - 1));
        pts.push_back(-1.0 + 2.0 * j / (p - 1));
        pts.push_back(-1.0 + 2.0 * k / (p - 1));
      }
  return pts;
}

// Runs body(i) for i in [0, count) on up to 16 threads (contiguous ranges; each i is done once, by one thread,
// so results do not depend on the thread count).
template <typename F>
static void parallel_for(int count, F body) {
  const unsigned hw = std::thread::hardware_concurrency();
  const int nth = std::max(1, std::min({count, 16, (int)(hw == 0 ? 1 : hw)}));
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t)
    pool.emplace_back([&, t] {
      for (int i = count * t / nth; i < count * (t + 1) / nth; ++i) body(i);
    });
  for (auto& th : pool) th.join();
}

// Dense U-kernel matrix, row-major (3 nx) x (3 ny): entry [3a+i][3b+j] = U_ij(x_a, y_b)  (eq. disp_1).
static void kernel_matrix_U(const Elastic& e, const double* X, int nx, const double* Y, int ny, double* out) {
  const int ld = 3 * ny;
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < ny; ++b) {
      double d[3] = {Y[3 * b] - X[3 * a], Y[3 * b + 1] - X[3 * a + 1], Y[3 * b + 2] - X[3 * a + 2]};
      double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double rr = d[i] * d[j] / (r * r);
          out[(size_t)(3 * a + i) * ld + 3 * b + j] = e.cU / r * ((i == j ? (3.0 - 4.0 * e.nu) : 0.0) + rr);
        }
    }
}

// One-sided (Hestenes) Jacobi SVD of a square n x n row-major matrix A in FP64: on return W = A V has
// mutually orthogonal columns (column-major, W_j = s_j u_j), V is orthogonal (column-major) and sig holds
// the column norms s_j.  Columns are processed in a round-robin ordering so that the n/2 rotations of one
// round touch disjoint column pairs and run on several threads.
static void jacobi_svd(const std::vector<double>& A, int n, std::vector<double>& W, std::vector<double>& V,
                       std::vector<double>& sig) {
  W.assign((size_t)n * n, 0.0);
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) W[(size_t)j * n + i] = A[(size_t)i * n + j];
  for (int j = 0; j < n; ++j) V[(size_t)j * n + j] = 1.0;
  const int m = n + (n & 1);  // even number of slots for the tournament
  std::vector<int> slot(m);
  for (int i = 0; i < m; ++i) slot[i] = i;
  unsigned hw = std::thread::hardware_concurrency();
  int nthreads = (int)std::max(1u, std::min(hw == 0 ? 1u : hw, 16u));
  const double tol = 1e-15;
  // persistent workers; a sense-reversing spin barrier separates the rounds of the tournament
  std::atomic<int> arrived{0};
  std::atomic<int> sense{0};
  auto barrier = [&](int& local_sense) {
    local_sense ^= 1;
    if (arrived.fetch_add(1) == nthreads - 1) {
      arrived.store(0);
      sense.store(local_sense);
    } else {
      while (sense.load() != local_sense) std::this_thread::yield();
    }
  };
  std::vector<int> rotated(nthreads, 0);
  std::atomic<bool> done{false};
  auto worker = [&](int tid) {
    int ls = 0;
    for (int sweep = 0; sweep < 60; ++sweep) {
      for (int round = 0; round < m - 1; ++round) {
        for (int k = tid; k < m / 2; k += nthreads) {
          int p = slot[k], q = slot[m - 1 - k];
          if (p >= n || q >= n) continue;
          if (p > q) std::swap(p, q);
          double* wp = &W[(size_t)p * n];
          double* wq = &W[(size_t)q * n];
          double al = 0, be = 0, ga = 0;
          for (int i = 0; i < n; ++i) {
            al += wp[i] * wp[i];
            be += wq[i] * wq[i];
            ga += wp[i] * wq[i];
          }
          if (ga == 0.0 || std::fabs(ga) <= tol * std::sqrt(al * be)) continue;
          rotated[tid]++;
          double zeta = (be - al) / (2.0 * ga);
          double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
          double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
          for (int i = 0; i < n; ++i) {
            double a = wp[i], b = wq[i];
            wp[i] = c * a - s * b;
            wq[i] = s * a + c * b;
          }
          double* vp = &V[(size_t)p * n];
          double* vq = &V[(size_t)q * n];
          for (int i = 0; i < n; ++i) {
            double a = vp[i], b = vq[i];
            vp[i] = c * a - s * b;
            vq[i] = s * a + c * b;
          }
        }
        barrier(ls);
        if (tid == 0) {  // rotate the tournament (slot 0 fixed)
          int last = slot[m - 1];
          for (int i = m - 1; i > 1; --i) slot[i] = slot[i - 1];
          slot[1] = last;
        }
        barrier(ls);
      }
      if (tid == 0) {
        int tot = 0;
        for (int& r : rotated) {
          tot += r;
          r = 0;
        }
        done.store(tot == 0);
      }
      barrier(ls);
      if (done.load()) break;
      barrier(ls);
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 1; t < nthreads; ++t) th.emplace_back(worker, t);
    worker(0);
    for (auto& t : th) t.join();
  }
  sig.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += W[(size_t)j * n + i] * W[(size_t)j * n + i];
    sig[j] = std::sqrt(s);
  }
}

// Pseudo-inverse of a square n x n row-major matrix from its one-sided Jacobi SVD (W = A V, column j of
// W = s_j u_j, V[j n + i] = (v_j)_i), singular values below eps * s_max discarded.
static std::vector<double> pinv_from_svd(const std::vector<double>& W, const std::vector<double>& V,
                                         const std::vector<double>& sig, int n, double eps, int* rank_out) {
  double smax = 0;
  for (double v : sig) smax = std::max(smax, v);
  // pinv = V diag(1/s) U^T with U_j = W_j / s_j  ->  pinv[i][k] = sum_j V[i][j] W[k][j] / s_j^2
  std::vector<double> P((size_t)n * n, 0.0);
  int rank = 0;
  std::vector<int> keep;
  for (int j = 0; j < n; ++j)
    if (sig[j] > eps * smax) {
      keep.push_back(j);
      ++rank;
    }
  parallel_for(n, [&](int i) {
    for (int k = 0; k < n; ++k) {
      double acc = 0;
      for (int j : keep) acc += V[(size_t)j * n + i] * W[(size_t)j * n + k] / (sig[j] * sig[j]);
      P[(size_t)i * n + k] = acc;
    }
  });
  if (rank_out) *rank_out = rank;
  return P;
}

// The two factors of UC2UE and of DC2DE (row-major n x n, discarded directions as zero rows / columns):
//   fu1 = Us^T, fu2 = Vs S^-1 (UC2UE = fu2 fu1);  fd1 = Vs^T, fd2 = Us S^-1 (DC2DE = fd2 fd1).
static void pinv_factors(const std::vector<double>& W, const std::vector<double>& V, const std::vector<double>& sig,
                         int n, double eps, Operators& op) {
  double smax = 0;
  for (double v : sig) smax = std::max(smax, v);
  for (auto* m : {&op.fu1, &op.fu2, &op.fd1, &op.fd2, &op.vs, &op.us}) m->assign((size_t)n * n, 0.0);
  op.inv_sig.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    if (!(sig[j] > eps * smax)) continue;
    const double s = sig[j];
    for (int k = 0; k < n; ++k) {
      const double u = W[(size_t)j * n + k] / s;  // (u_j)_k
      const double v = V[(size_t)j * n + k];      // (v_j)_k
      op.fu1[(size_t)j * n + k] = u;
      op.fu2[(size_t)k * n + j] = v / s;
      op.fd1[(size_t)j * n + k] = v;
      op.fd2[(size_t)k * n + j] = u / s;
      op.vs[(size_t)k * n + j] = v;
      op.us[(size_t)k * n + j] = u;
    }
    op.inv_sig[j] = 1.0 / s;
  }
}

// C = A B for n x n row-major FP64 matrices (rows in parallel; every entry summed in k order).
static std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n) {
  std::vector<double> C((size_t)n * n, 0.0);
  parallel_for(n, [&](int i) {
    double* c = &C[(size_t)i * n];
    for (int k = 0; k < n; ++k) {
      double a = A[(size_t)i * n + k];
      const double* b = &B[(size_t)k * n];
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
  });
  return C;
}

static std::string cache_dir() {
  const char* dir = std::getenv("KFMM_CACHE_DIR");
  if (dir && *dir) return dir;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/kfmm";
}

static std::string cache_path(int p, const Elastic& e, double eps) {
  const std::string d = cache_dir();
  char name[256];
  std::snprintf(name, sizeof(name), "/svd_uc_ue_p%d_nu%.17g_G%.17g_r1.05_2.95.bin", p, e.nu, e.G);
  (void)eps;  // the SVD does not depend on the cutoff
  return d + name;
}

// Cache file: n, then one array of doubles (the SVD: W, V, sig, 2 n^2 + n values by default), then a checksum.
static bool load_cache(const std::string& path, int n, std::vector<double>& P, size_t count = 0) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  int nn = 0;
  f.read((char*)&nn, sizeof(int));
  if (nn != n) return false;
  P.resize(count ? count : (size_t)2 * n * n + n);
  f.read((char*)P.data(), sizeof(double) * P.size());
  uint64_t chk = 0, ref = 0;
  f.read((char*)&ref, sizeof(ref));
  if (!f) return false;
  for (double v : P) {
    uint64_t u;
    std::memcpy(&u, &v, 8);
    chk = chk * 1099511628211ull ^ u;
  }
  return chk == ref;
}

static void save_cache(const std::string& path, int n, const std::vector<double>& P) {
  // create the cache directory with mkdir(2), one path component at a time (no shell, no child process)
  std::string dir = path.substr(0, path.rfind('/'));
  for (size_t pos = 1; pos <= dir.size(); ++pos) {
    if (pos == dir.size() || dir[pos] == '/') {
      std::string part = dir.substr(0, pos);
      if (::mkdir(part.c_str(), 0755) != 0 && errno != EEXIST) return;
    }
  }
  std::string tmp = path + ".tmp" + std::to_string((long)std::rand());
  std::ofstream f(tmp, std::ios::binary);
  if (!f) return;
  f.write((const char*)&n, sizeof(int));
  f.write((const char*)P.data(), sizeof(double) * P.size());
  uint64_t chk = 0;
  for (double v : P) {
    uint64_t u;
    std::memcpy(&u, &v, 8);
    chk = chk * 1099511628211ull ^ u;
  }
  f.write((const char*)&chk, sizeof(chk));
  f.close();
  std::rename(tmp.c_str(), path.c_str());
}

Operators build_operators(int p, const Elastic& e, double svd_eps) {
  Operators op;
  op.p = p;
  op.n_eq = surface_count(p);
  const int n = 3 * op.n_eq;
  op.n = n;
  std::vector<double> S = cube_surface(p);
  op.surf = S;
  auto scaled = [&](double a, double ox, double oy, double oz) {
    std::vector<double> v(S.size());
    for (int i = 0; i < op.n_eq; ++i) {
      v[3 * i] = ox + a * S[3 * i];
      v[3 * i + 1] = oy + a * S[3 * i + 1];
      v[3 * i + 2] = oz + a * S[3 * i + 2];
    }
    return v;
  };
  const double RE_UP = 1.05, RC_UP = 2.95, RC_DN = 1.05, RE_DN = 2.95;
  op.r_up_equiv = RE_UP;
  op.r_up_check = RC_UP;
  op.r_dn_check = RC_DN;
  op.r_dn_equiv = RE_DN;
  std::vector<double> uc = scaled(RC_UP, 0, 0, 0), ue = scaled(RE_UP, 0, 0, 0);
  std::vector<double> K((size_t)n * n);
  kernel_matrix_U(e, uc.data(), op.n_eq, ue.data(), op.n_eq, K.data());
  std::string path = cache_path(p, e, svd_eps);
  std::vector<double> W, V, sig, packed;
  if (load_cache(path, n, packed)) {
    const size_t nn = (size_t)n * n;
    W.assign(packed.begin(), packed.begin() + nn);
    V.assign(packed.begin() + nn, packed.begin() + 2 * nn);
    sig.assign(packed.begin() + 2 * nn, packed.end());
  } else {
    jacobi_svd(K, n, W, V, sig);
    packed = W;
    packed.insert(packed.end(), V.begin(), V.end());
    packed.insert(packed.end(), sig.begin(), sig.end());
    save_cache(path, n, packed);
  }
  op.uc2ue = pinv_from_svd(W, V, sig, n, svd_eps, &op.rank);
  pinv_factors(W, V, sig, n, svd_eps, op);
  op.dc2de.resize((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) op.dc2de[(size_t)i * n + j] = op.uc2ue[(size_t)j * n + i];
  // M2M and L2L per child octant c (bit0 x, bit1 y, bit2 z; child centre = parent centre + 0.5 o r_parent)
  op.m2m.resize(8);
  op.l2l.resize(8);
  op.m2m_q.resize(8);
  op.l2l_q.resize(8);
  for (int c = 0; c < 8; ++c) {
    double o[3] = {(c & 1) ? 1.0 : -1.0, (c & 2) ? 1.0 : -1.0, (c & 4) ? 1.0 : -1.0};
    // parent frame (unit parent half-width): child upward equivalent surface
    std::vector<double> che = scaled(0.5 * RE_UP, 0.5 * o[0], 0.5 * o[1], 0.5 * o[2]);
    std::vector<double> Kc((size_t)n * n);
    kernel_matrix_U(e, uc.data(), op.n_eq, che.data(), op.n_eq, Kc.data());
    op.m2m[c] = matmul(op.uc2ue, Kc, n);
    op.m2m_q[c] = matmul(Kc, op.uc2ue, n);
    // child frame (unit child half-width): parent downward equivalent surface at -o with half-width 2*RE_DN
    std::vector<double> cdc = scaled(RC_DN, 0, 0, 0);
    std::vector<double> pde = scaled(2.0 * RE_DN, -o[0], -o[1], -o[2]);
    std::vector<double> Kl((size_t)n * n);
    kernel_matrix_U(e, cdc.data(), op.n_eq, pde.data(), op.n_eq, Kl.data());
    op.l2l[c] = matmul(op.dc2de, Kl, n);
    op.l2l_q[c] = matmul(Kl, op.dc2de, n);
  }
  // M2L for every index offset d in [-3,3]^3 with max |d_i| >= 2 (316 offsets)
  std::vector<double> dc = scaled(RC_DN, 0, 0, 0);
  op.m2l_index.assign(343, -1);
  std::vector<int> offs;
  for (int dz = -3; dz <= 3; ++dz)
    for (int dy = -3; dy <= 3; ++dy)
      for (int dx = -3; dx <= 3; ++dx) {
        if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) < 2) continue;
        int idx = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
        op.m2l_index[idx] = (int)offs.size();
        offs.push_back(idx);
      }
  op.m2l.resize(offs.size());
  parallel_for((int)offs.size(), [&](int o) {
    const int idx = offs[o], dx = idx % 7 - 3, dy = (idx / 7) % 7 - 3, dz = idx / 49 - 3;
    std::vector<double> se = scaled(RE_UP, 2.0 * dx, 2.0 * dy, 2.0 * dz);
    op.m2l[o].resize((size_t)n * n);
    kernel_matrix_U(e, dc.data(), op.n_eq, se.data(), op.n_eq, op.m2l[o].data());
  });
  return op;
}

// Eigen-decomposition of a symmetric positive semi-definite n x n matrix (row-major): eigenvalues in
// decreasing order and the matching unit eigenvectors (column-major n x n).  For such a matrix the one-sided
// Jacobi iteration converges to W = A V = V diag(lambda), so the column norms are the eigenvalues.
void sym_eig_psd(const std::vector<double>& A, int n, std::vector<double>& lambda, std::vector<double>& vecs) {
  std::vector<double> W, V, sig;
  jacobi_svd(A, n, W, V, sig);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return sig[a] > sig[b]; });
  lambda.resize(n);
  vecs.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    lambda[k] = sig[order[k]];
    for (int i = 0; i < n; ++i) vecs[(size_t)k * n + i] = V[(size_t)order[k] * n + i];
  }
}

// sym_eig_psd with the result kept in the operator cache directory, keyed by a hash of the matrix's bits (the
// same matrix gives the same file; any change of the input, a new file).
void sym_eig_psd_cached(const std::vector<double>& A, int n, const char* tag, std::vector<double>& lambda,
                        std::vector<double>& vecs) {
  uint64_t h = 1469598103934665603ull;
  for (double v : A) {
    uint64_t u;
    std::memcpy(&u, &v, 8);
    h = (h ^ u) * 1099511628211ull;
  }
  char name[128];
  std::snprintf(name, sizeof(name), "/eig_%s_n%d_%016llx.bin", tag, n, (unsigned long long)h);
  const std::string path = cache_dir() + name;
  std::vector<double> P;
  if (load_cache(path, n, P, (size_t)n + (size_t)n * n)) {
    lambda.assign(P.begin(), P.begin() + n);
    vecs.assign(P.begin() + n, P.end());
    return;
  }
  sym_eig_psd(A, n, lambda, vecs);
  P = lambda;
  P.insert(P.end(), vecs.begin(), vecs.end());
  save_cache(path, n, P);
}

// Far-image operator of a periodic cell (Sec. 4.3: the multipole expansions are periodic, so the tree is
// made periodic at every level).  The lists of a periodic tree cover the 3 x 3 x 3 block of cell images
// around the cell; the images beyond act on the root alone, through
//   T = sum_{n not in {-1,0,1}^3} U[dc <- ue + 2n]      (unit half-width frame, cell side 2)
// added to the root's downward check potential like an M2L.  The lattice sum converges only conditionally;
// it is taken as the Fourier series without its k = 0 term (the zero-mean periodic field, a net force per
// cell balanced by a uniform body force), evaluated by Ewald splitting U = U_r + U_f + constant:
//   U_r(x) = cU [(3 - 4nu) delta erfc(a r) / r + (erfc(a r) / r + 2a/sqrt(pi) exp(-a^2 r^2)) x x^T / r^2]
//   U_f    = (1/V) sum_{k != 0} exp(-s) [delta / (G k^2) - (1 + s) k k^T / (2 (1 - nu) G k^4)] cos(k.x),
//            k = 2 pi m / L, s = k^2 / (4 a^2)
//   constant -delta / (4 a^2 G V)  (the k -> 0 limit of U_r's transform, left out with k = 0)
// (U_r carries the Kelvin singularity; U_r - U is smooth, -(3 - 4nu) cU 2a/sqrt(pi) delta at x = 0).  So
//   T(x) = sum_{n in 27} (U_r - U)(x + 2n) + sum_{n not in 27} U_r(x + 2n) + U_f(x) + constant.
// With a = 1.5 (L = 2) the real-space terms beyond |n_i| <= 2 and the Fourier terms beyond |m_i| <= 7 are
// below 1e-16 of the entries.
std::vector<double> periodic_far_operator(int p, const Elastic& e) {
  const int ne = surface_count(p), n = 3 * ne;
  const double L = 2.0, V = L * L * L, a = 1.5, RE = 1.05, RC = 1.05;
  const double sqpi = std::sqrt(kPi), c_e = 2.0 * a / sqpi;
  const std::vector<double> S = cube_surface(p);
  std::vector<double> X(3 * ne), Y(3 * ne);  // downward check points, upward equivalent points
  for (int i = 0; i < 3 * ne; ++i) {
    X[i] = RC * S[i];
    Y[i] = RE * S[i];
  }
  std::vector<double> T((size_t)n * n, 0.0);
  // ---- real space and constant
  const int NR = 2;
  const double rcut = 6.0 / a;
  for (int ia = 0; ia < ne; ++ia)
    for (int ib = 0; ib < ne; ++ib) {
      double acc[3][3] = {};
      for (int nx = -NR; nx <= NR; ++nx)
        for (int ny = -NR; ny <= NR; ++ny)
          for (int nz = -NR; nz <= NR; ++nz) {
            const bool near = std::abs(nx) <= 1 && std::abs(ny) <= 1 && std::abs(nz) <= 1;
            const double d[3] = {Y[3 * ib] + L * nx - X[3 * ia], Y[3 * ib + 1] + L * ny - X[3 * ia + 1],
                                 Y[3 * ib + 2] + L * nz - X[3 * ia + 2]};
            const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!near && r > rcut) continue;
            double cd, cx;  // coefficients of delta and of x x^T / r^2
            if (near) {     // U_r - U
              const double ef = r > 0 ? std::erf(a * r) / r : c_e;
              cd = -(3.0 - 4.0 * e.nu) * ef;
              cx = r > 0 ? -ef + c_e * std::exp(-a * a * r * r) : 0.0;
            } else {
              const double ec = std::erfc(a * r) / r;
              cd = (3.0 - 4.0 * e.nu) * ec;
              cx = ec + c_e * std::exp(-a * a * r * r);
            }
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j)
                acc[i][j] += e.cU * ((i == j ? cd : 0.0) + (r > 0 ? cx * d[i] * d[j] / (r * r) : 0.0));
          }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          T[(size_t)(3 * ia + i) * n + 3 * ib + j] = acc[i][j] - (i == j ? 1.0 / (4.0 * a * a * e.G * V) : 0.0);
    }
  // ---- reciprocal space: half of the vectors m != 0 (m and -m give the same cosine), weight 2/V
  const int KM = 7;
  std::vector<double> kv;
  for (int mx = -KM; mx <= KM; ++mx)
    for (int my = -KM; my <= KM; ++my)
      for (int mz = -KM; mz <= KM; ++mz)
        if (mx > 0 || (mx == 0 && my > 0) || (mx == 0 && my == 0 && mz > 0)) {
          kv.push_back(2.0 * kPi * mx / L);
          kv.push_back(2.0 * kPi * my / L);
          kv.push_back(2.0 * kPi * mz / L);
        }
  const int nk = (int)kv.size() / 3;
  std::vector<double> w6((size_t)nk * 6);  // (2/V) U_f(k) components xx, yy, zz, xy, xz, yz
  for (int q = 0; q < nk; ++q) {
    const double* k = &kv[3 * q];
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2], sx = k2 / (4.0 * a * a), ex = std::exp(-sx);
    const double cdel = 2.0 / V * ex / (e.G * k2), ckk = -2.0 / V * ex * (1.0 + sx) / (2.0 * (1.0 - e.nu) * e.G * k2 * k2);
    const int pi6[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    for (int c = 0; c < 6; ++c) {
      const int i = pi6[c][0], j = pi6[c][1];
      w6[6 * q + c] = (i == j ? cdel : 0.0) + ckk * k[i] * k[j];
    }
  }
  std::vector<double> cxa((size_t)ne * nk), sxa((size_t)ne * nk), cyb((size_t)ne * nk), syb((size_t)ne * nk);
  for (int i = 0; i < ne; ++i)
    for (int q = 0; q < nk; ++q) {
      const double* k = &kv[3 * q];
      const double tx = k[0] * X[3 * i] + k[1] * X[3 * i + 1] + k[2] * X[3 * i + 2];
      const double ty = k[0] * Y[3 * i] + k[1] * Y[3 * i + 1] + k[2] * Y[3 * i + 2];
      cxa[(size_t)i * nk + q] = std::cos(tx);
      sxa[(size_t)i * nk + q] = std::sin(tx);
      cyb[(size_t)i * nk + q] = std::cos(ty);
      syb[(size_t)i * nk + q] = std::sin(ty);
    }
  auto rows = [&](int a0, int a1) {
    for (int ia = a0; ia < a1; ++ia)
      for (int ib = 0; ib < ne; ++ib) {
        double acc[6] = {0, 0, 0, 0, 0, 0};
        const double *ca = &cxa[(size_t)ia * nk], *sa = &sxa[(size_t)ia * nk];
        const double *cb = &cyb[(size_t)ib * nk], *sb = &syb[(size_t)ib * nk];
        for (int q = 0; q < nk; ++q) {
          const double c = cb[q] * ca[q] + sb[q] * sa[q];  // cos(k.(y - x))
          for (int m = 0; m < 6; ++m) acc[m] += w6[6 * q + m] * c;
        }
        const double M[3][3] = {{acc[0], acc[3], acc[4]}, {acc[3], acc[1], acc[5]}, {acc[4], acc[5], acc[2]}};
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) T[(size_t)(3 * ia + i) * n + 3 * ib + j] += M[i][j];
      }
  };
  const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t) pool.emplace_back(rows, ne * t / nth, ne * (t + 1) / nth);
  for (auto& th : pool) th.join();
  return T;
}

}  // namespace kfmm
