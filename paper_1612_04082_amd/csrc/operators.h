// Level-invariant KIFMM translation operators (host, FP64); see operators.cpp.
#pragma once
#include <vector>

#include "common.h"

namespace kfmm {

struct Operators {
  int p = 0, n_eq = 0, n = 0, rank = 0;  // n = 3 n_eq coefficients per box
  double r_up_equiv = 0, r_up_check = 0, r_dn_check = 0, r_dn_equiv = 0;
  std::vector<double> surf;                 // n_eq x 3 unit cube-surface points
  std::vector<double> uc2ue, dc2de;         // n x n
  std::vector<double> fu1, fu2, fd1, fd2;   // n x n factors: UC2UE = fu2 fu1, DC2DE = fd2 fd1
  std::vector<double> vs, us, inv_sig;      // fu2 = vs diag(inv_sig), fd2 = us diag(inv_sig) (orthogonal vs, us)
  std::vector<std::vector<double>> m2m;     // 8 x (n x n)
  std::vector<std::vector<double>> l2l;     // 8 x (n x n)
  std::vector<std::vector<double>> m2m_q;   // 8 x (n x n): the same translations on check potentials
  std::vector<std::vector<double>> l2l_q;   // 8 x (n x n)
  std::vector<std::vector<double>> m2l;     // 316 x (n x n)
  std::vector<int> m2l_index;               // 343 -> compact index (or -1), key (dx+3)+7(dy+3)+49(dz+3)
};

std::vector<double> cube_surface(int p);
Operators build_operators(int p, const Elastic& e, double svd_eps);
void sym_eig_psd(const std::vector<double>& A, int n, std::vector<double>& lambda, std::vector<double>& vecs);
// The same, cached on disk with the operators (file name from a hash of A).
void sym_eig_psd_cached(const std::vector<double>& A, int n, const char* tag, std::vector<double>& lambda,
                        std::vector<double>& vecs);
// Far-image operator of a periodic cell at unit half-width (cell side 2), n x n row-major: the downward check
// potential of the root from the upward equivalent densities of every lattice image outside the 3 x 3 x 3
// block around the cell (see operators.cpp).
std::vector<double> periodic_far_operator(int p, const Elastic& e);

}  // namespace kfmm
