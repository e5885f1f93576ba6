// Two-level additive Schwarz preconditioner of the collocation BEM system (eq. num2), applied on the
// right inside GMRES so that the residual it reduces stays the true ||b - A x||.  The paper leaves the
// preconditioning of mixed boundary-value problems open (Sec. 5, "Discussion and future work").
//
//     M^-1 v = sum_b R_b^T (R_b A R_b^T)^-1 R_b v  +  Z (Z^T A Z)^-1 Z^T v
//
//  * Elements are ordered along a Morton curve of their centroids (14 bits per axis over the centroids'
//    bounding cube, x in the lowest bit of each triple, ties in element order).
//  * Fine level: runs of `fine` (<= 32) consecutive elements of that order; each block of A (3m x 3m: the
//    16-point quadrature between the block's elements, the near-singular corrections of its near pairs,
//    closed-form self blocks and the free term on the diagonal, the traction columns scaled like the
//    system's) is assembled and inverted (Gauss-Jordan, partial pivoting, FP64) in LDS by one workgroup.
//  * Coarse level: runs of `coarse` elements ("aggregates"), each with the local rigid motions as columns:
//    three translations (every unknown of a component) and three rotations about the aggregate's mean
//    centroid (at the displacement unknowns only), orthonormalised by two passes of modified Gram-Schmidt;
//    a column that keeps at most 1e-8 of its raw norm is dropped (a zero column, identity in E).  Rigid
//    displacements are the null space of 1/2 I + P on a closed surface, and the bending modes of slender
//    bodies are close to them locally, which is what slows unpreconditioned GMRES down.
//  * E = Z^T A Z is summed directly: one wave per (target aggregate, source aggregate) pair evaluates the
//    quadrature between their elements against the six coarse columns and contracts with the target's
//    columns; E is inverted by Gauss-Jordan with partial pivoting in device memory (one pivot step per
//    launch pair).
//  * Application: Z^T v per aggregate, g = E^-1 (Z^T v) (one wave per row), then per fine block the
//    block inverse times v plus Z g, written once per unknown.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "precond.h"

namespace kfmm {

namespace {

constexpr int kQ = 16;           // quadrature points per element
constexpr int kMortonQBits = 14; // bits per axis of the element order
constexpr double kDrop = 1e-8;   // relative norm below which a coarse column is dropped

unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Full 3x3 Kelvin blocks for one quadrature source (d = source - target, r2 > 0, n = source normal):
//   U_ij = cU / r ((3 - 4 nu) d_ij + rh_i rh_j)                                         (eq. disp_1)
//   P_ij = -cP / r^2 ((rh.n) ((1 - 2 nu) d_ij + 3 rh_i rh_j) - (1 - 2 nu)(rh_i n_j - rh_j n_i))  (eq. disp_2)
// accumulated with the quadrature weight w.
__device__ __forceinline__ void add_kelvin(const double d[3], double r2, const double n[3], double w,
                                           const Elastic& el, double KU[3][3], double KP[3][3]) {
  const double r = sqrt(r2), ir = 1.0 / r;
  const double rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
  const double drdn = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
  const double a34 = 3.0 - 4.0 * el.nu, a12 = 1.0 - 2.0 * el.nu;
  const double cu = el.cU * ir * w, cp = -el.cP * ir * ir * w;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double rr = rh[i] * rh[j];
      KU[i][j] += cu * ((i == j ? a34 : 0.0) + rr);
      KP[i][j] += cp * (drdn * ((i == j ? a12 : 0.0) + 3.0 * rr) - a12 * (rh[i] * n[j] - rh[j] * n[i]));
    }
}

// The 3x3 block A[(i, .), (j, .)] of the rearranged system (solver units): the quadrature of element j
// at the centroid of element i (coincident point skipped), with the self correction and the free term
// when i == j; traction-unknown columns take -scale_t U, displacement-unknown columns P (+ 1/2 I).
struct BlockArgs {
  const double *qp, *qn, *qw, *cen, *dU, *dP;
  const int8_t* bc_type;
  double scale_t;
  Elastic el;
  // near-singular quadrature (NULL when off): CSR of near pairs and their corrections
  const int *near_off, *near_idx;
  const double *near_dU, *near_dP;
};

// 3x3 block M[u][v] from the kernel sums KU, KP: traction-unknown columns -scale_t U, others P
__device__ __forceinline__ void column_map(const BlockArgs& a, int64_t j, const double KU[3][3], const double KP[3][3],
                                           double M[3][3]) {
  for (int v = 0; v < 3; ++v) {
    const bool t_unknown = a.bc_type[3 * j + v] == 0;
    for (int u = 0; u < 3; ++u) M[u][v] = t_unknown ? -a.scale_t * KU[u][v] : KP[u][v];
  }
}

// The block of the pair (i, j) with its near-singular correction when with_near and (i, j) is a near pair.
__device__ void system_block(const BlockArgs& a, int64_t i, int64_t j, double M[3][3], bool with_near) {
  double KU[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, KP[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  const double c[3] = {a.cen[3 * i], a.cen[3 * i + 1], a.cen[3 * i + 2]};
  const double n[3] = {a.qn[3 * kQ * j], a.qn[3 * kQ * j + 1], a.qn[3 * kQ * j + 2]};
  for (int q = 0; q < kQ; ++q) {
    const int64_t s = kQ * j + q;
    const double d[3] = {a.qp[3 * s] - c[0], a.qp[3 * s + 1] - c[1], a.qp[3 * s + 2] - c[2]};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) continue;
    add_kelvin(d, r2, n, a.qw[s], a.el, KU, KP);
  }
  if (i == j) {
    for (int u = 0; u < 3; ++u)
      for (int v = 0; v < 3; ++v) {
        KU[u][v] += a.dU[9 * i + 3 * u + v];
        KP[u][v] += a.dP[9 * i + 3 * u + v] + (u == v ? 0.5 : 0.0);
      }
  }
  if (with_near && a.near_off)
    for (int p = a.near_off[i]; p < a.near_off[i + 1]; ++p)
      if (a.near_idx[p] == j) {
        for (int u = 0; u < 3; ++u)
          for (int v = 0; v < 3; ++v) {
            KU[u][v] += a.near_dU[9 * p + 3 * u + v];
            KP[u][v] += a.near_dP[9 * p + 3 * u + v];
          }
        break;
      }
  column_map(a, j, KU, KP, M);
}

// ------------------------------------------------------------------------------------------- order

// Per-axis minimum and maximum of the centroids (one workgroup).
__global__ __launch_bounds__(256) void k_pc_bounds(const double* __restrict__ cen, int64_t T, double* __restrict__ out) {
  __shared__ double lo[3][256], hi[3][256];
  double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t e = threadIdx.x; e < T; e += blockDim.x)
    for (int d = 0; d < 3; ++d) {
      const double v = cen[3 * e + d];
      l[d] = fmin(l[d], v);
      h[d] = fmax(h[d], v);
    }
  for (int d = 0; d < 3; ++d) {
    lo[d][threadIdx.x] = l[d];
    hi[d][threadIdx.x] = h[d];
  }
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int d = 0; d < 3; ++d) {
        lo[d][threadIdx.x] = fmin(lo[d][threadIdx.x], lo[d][threadIdx.x + st]);
        hi[d][threadIdx.x] = fmax(hi[d][threadIdx.x], hi[d][threadIdx.x + st]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) {
      out[d] = lo[d][0];
      out[3 + d] = hi[d][0];
    }
}

// key = (interleaved 14-bit cell coordinates) << 22 | element: unique keys, so the sort keeps ties in
// element order.
__global__ void k_pc_keys(const double* __restrict__ cen, int64_t T, const double* __restrict__ bounds,
                          uint64_t* __restrict__ key, int* __restrict__ idx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) ext = fmax(ext, bounds[3 + d] - bounds[d]);
  if (ext == 0.0) ext = 1.0;
  uint64_t m = 0;
  for (int d = 0; d < 3; ++d) {
    double f = floor((cen[3 * e + d] - bounds[d]) / ext * (double)(1 << kMortonQBits));
    int64_t q = (int64_t)f;
    q = q < 0 ? 0 : (q > (1 << kMortonQBits) - 1 ? (1 << kMortonQBits) - 1 : q);
    for (int b = 0; b < kMortonQBits; ++b) m |= (uint64_t)((q >> b) & 1) << (3 * b + d);
  }
  key[e] = (m << 22) | (uint64_t)e;
  idx[e] = (int)e;
}

// -------------------------------------------------------------------------------------- fine level

// One workgroup per fine block: assemble the block (3m x 3m) in LDS, invert it in place by Gauss-Jordan
// with partial pivoting (row swaps, columns unscrambled in reverse order at the end), write the inverse
// transposed.  A zero pivot sets *singular.
constexpr int kFineN = 3 * kPcFineMax;

__global__ __launch_bounds__(256) void k_pc_fine(BlockArgs a, const int* __restrict__ order, int64_t T, int fine,
                                                 double* __restrict__ binv_t, int* __restrict__ singular) {
  __shared__ double A[kFineN][kFineN + 1];
  __shared__ double fcol[kFineN];
  __shared__ int piv[kFineN];
  __shared__ int sh_p;
  const int64_t first = (int64_t)blockIdx.x * fine;
  const int m = (int)min((int64_t)fine, T - first);
  const int n = 3 * m;
  const int tid = threadIdx.x;
  for (int pr = tid; pr < m * m; pr += blockDim.x) {
    const int bi = pr / m, bj = pr % m;
    double M[3][3];
    system_block(a, order[first + bi], order[first + bj], M, true);
    for (int u = 0; u < 3; ++u)
      for (int v = 0; v < 3; ++v) A[3 * bi + u][3 * bj + v] = M[u][v];
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (tid < 64) {  // pivot: largest |A[i][k]|, i >= k, the first on ties
      double best = -1.0;
      int bi = n;
      for (int i = k + tid; i < n; i += 64) {
        const double v = fabs(A[i][k]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) {
        sh_p = bi;
        piv[k] = bi;
      }
    }
    __syncthreads();
    const int p = sh_p;
    if (p != k)
      for (int t = tid; t < n; t += blockDim.x) {
        const double x = A[k][t];
        A[k][t] = A[p][t];
        A[p][t] = x;
      }
    __syncthreads();
    for (int t = tid; t < n; t += blockDim.x) fcol[t] = A[t][k];
    __syncthreads();
    const double pv = fcol[k];
    if (tid == 0 && pv == 0.0) atomicExch(singular, 1);
    for (int t = tid; t < n; t += blockDim.x) A[k][t] = (t == k) ? 1.0 / pv : A[k][t] / pv;
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e % n;
      if (i == k) continue;
      A[i][j] = (j == k ? 0.0 : A[i][j]) - fcol[i] * A[k][j];
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += blockDim.x)
    for (int k = n - 1; k >= 0; --k) {
      const int p = piv[k];
      if (p != k) {
        const double x = A[i][k];
        A[i][k] = A[i][p];
        A[i][p] = x;
      }
    }
  __syncthreads();
  double* out = binv_t + (size_t)blockIdx.x * kFineN * kFineN;
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int c = e / n, r = e % n;  // out[c][r] = inverse[r][c]
    out[(size_t)c * kFineN + r] = A[r][c];
  }
}

// ------------------------------------------------------------------------------------ coarse level

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One wave per aggregate: the six raw columns, two passes of modified Gram-Schmidt in column order, drop
// test; written to z[e][c][k] for the aggregate's elements (zeros for a dropped column), kept[a*6+k].
__global__ __launch_bounds__(64) void k_pc_coarse_cols(const double* __restrict__ cen, const int8_t* __restrict__ bc_type,
                                                       const int* __restrict__ order, int64_t T, int coarse,
                                                       double* __restrict__ z, int* __restrict__ kept) {
  const int64_t first = (int64_t)blockIdx.x * coarse;
  const int m = (int)min((int64_t)coarse, T - first);
  const int lane = threadIdx.x;
  double cs[3] = {0, 0, 0};
  for (int i = lane; i < m; i += 64) {
    const int64_t e = order[first + i];
    for (int d = 0; d < 3; ++d) cs[d] += cen[3 * e + d];
  }
  double ca[3];
  for (int d = 0; d < 3; ++d) ca[d] = wave_sum(cs[d]) / (double)m;
  unsigned keep = 0;  // bit k: column k kept
  for (int k = 0; k < kPcCols; ++k) {
    double raw2 = 0.0;
    for (int i = lane; i < m; i += 64) {
      const int64_t e = order[first + i];
      const double dd[3] = {cen[3 * e] - ca[0], cen[3 * e + 1] - ca[1], cen[3 * e + 2] - ca[2]};
      for (int c = 0; c < 3; ++c) {
        double v;
        if (k < 3) {
          v = (c == k) ? 1.0 : 0.0;
        } else {
          // (e_w x d)_c with w = k - 3
          const int w = k - 3;
          const double ew[3] = {w == 0 ? 1.0 : 0.0, w == 1 ? 1.0 : 0.0, w == 2 ? 1.0 : 0.0};
          const double cr[3] = {ew[1] * dd[2] - ew[2] * dd[1], ew[2] * dd[0] - ew[0] * dd[2],
                                ew[0] * dd[1] - ew[1] * dd[0]};
          v = bc_type[3 * e + c] == 1 ? cr[c] : 0.0;
        }
        z[(3 * e + c) * kPcCols + k] = v;
        raw2 += v * v;
      }
    }
    const double raw = sqrt(wave_sum(raw2));
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 0; q < k; ++q) {
        if (!((keep >> q) & 1u)) continue;
        double dp = 0.0;
        for (int i = lane; i < m; i += 64) {
          const int64_t e = order[first + i];
          for (int c = 0; c < 3; ++c) dp += z[(3 * e + c) * kPcCols + q] * z[(3 * e + c) * kPcCols + k];
        }
        dp = wave_sum(dp);
        for (int i = lane; i < m; i += 64) {
          const int64_t e = order[first + i];
          for (int c = 0; c < 3; ++c) z[(3 * e + c) * kPcCols + k] -= dp * z[(3 * e + c) * kPcCols + q];
        }
      }
    double nv2 = 0.0;
    for (int i = lane; i < m; i += 64) {
      const int64_t e = order[first + i];
      for (int c = 0; c < 3; ++c) nv2 += z[(3 * e + c) * kPcCols + k] * z[(3 * e + c) * kPcCols + k];
    }
    const double nv = sqrt(wave_sum(nv2));
    const bool kk = !(raw == 0.0 || nv <= kDrop * raw);
    if (kk) keep |= 1u << k;
    const double f = kk ? 1.0 / nv : 0.0;
    for (int i = lane; i < m; i += 64) {
      const int64_t e = order[first + i];
      for (int c = 0; c < 3; ++c) z[(3 * e + c) * kPcCols + k] *= f;
    }
    if (lane == 0) kept[blockIdx.x * kPcCols + k] = kk ? 1 : 0;
  }
}

// E[(a, k), (a', k')] = sum_{i in a} sum_c z[i][c][k] (A Z)[(i, c), (a', k')]: one wave per (a', a) pair.
__global__ __launch_bounds__(64) void k_pc_coarse_E(BlockArgs a, const int* __restrict__ order, int64_t T, int coarse,
                                                    const double* __restrict__ z, int64_t nc, double* __restrict__ E) {
  const int64_t src_first = (int64_t)blockIdx.x * coarse, trg_first = (int64_t)blockIdx.y * coarse;
  const int ms = (int)min((int64_t)coarse, T - src_first), mt = (int)min((int64_t)coarse, T - trg_first);
  const int lane = threadIdx.x;
  double acc[kPcCols][kPcCols];
  for (int k = 0; k < kPcCols; ++k)
    for (int k2 = 0; k2 < kPcCols; ++k2) acc[k][k2] = 0.0;
  for (int ti = lane; ti < mt; ti += 64) {
    const int64_t i = order[trg_first + ti];
    double V[3][kPcCols];
    for (int c = 0; c < 3; ++c)
      for (int k2 = 0; k2 < kPcCols; ++k2) V[c][k2] = 0.0;
    for (int sj = 0; sj < ms; ++sj) {
      const int64_t j = order[src_first + sj];
      double M[3][3];
      system_block(a, i, j, M, false);  // near corrections are added by k_pc_coarse_E_near
      for (int cj = 0; cj < 3; ++cj)
        for (int k2 = 0; k2 < kPcCols; ++k2) {
          const double zz = z[(3 * j + cj) * kPcCols + k2];
          for (int c = 0; c < 3; ++c) V[c][k2] += M[c][cj] * zz;
        }
    }
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < kPcCols; ++k) {
        const double zi = z[(3 * i + c) * kPcCols + k];
        for (int k2 = 0; k2 < kPcCols; ++k2) acc[k][k2] += zi * V[c][k2];
      }
  }
  for (int k = 0; k < kPcCols; ++k)
    for (int k2 = 0; k2 < kPcCols; ++k2) {
      const double v = wave_sum(acc[k][k2]);
      if (lane == 0) E[(blockIdx.y * kPcCols + k) * nc + blockIdx.x * kPcCols + k2] = v;
    }
}

// Near-singular corrections of E: for the elements i of aggregate a (one wave) and their near elements j,
// E[(a, k), (agg j, k')] += z_i[., k]^T dM_ij z_j[., k'].  Lane k * 6 + k' owns those entries of row block a
// and applies the pairs in order (i by position, j by index), so the sums are deterministic.
__global__ __launch_bounds__(64) void k_pc_coarse_E_near(BlockArgs a, const int* __restrict__ order,
                                                         const int* __restrict__ rank, int64_t T, int coarse,
                                                         const double* __restrict__ z, int64_t nc,
                                                         double* __restrict__ E) {
  const int64_t first = (int64_t)blockIdx.x * coarse;
  const int m = (int)min((int64_t)coarse, T - first);
  const int lane = threadIdx.x;
  if (lane >= kPcCols * kPcCols) return;
  const int k = lane / kPcCols, k2 = lane % kPcCols;
  for (int ti = 0; ti < m; ++ti) {
    const int64_t i = order[first + ti];
    for (int p = a.near_off[i]; p < a.near_off[i + 1]; ++p) {
      const int64_t j = a.near_idx[p];
      double KU[3][3], KP[3][3], M[3][3];
      for (int u = 0; u < 3; ++u)
        for (int v = 0; v < 3; ++v) {
          KU[u][v] = a.near_dU[9 * p + 3 * u + v];
          KP[u][v] = a.near_dP[9 * p + 3 * u + v];
        }
      column_map(a, j, KU, KP, M);
      double acc = 0.0;
      for (int u = 0; u < 3; ++u) {
        double t = 0.0;
        for (int v = 0; v < 3; ++v) t += M[u][v] * z[(3 * j + v) * kPcCols + k2];
        acc += z[(3 * i + u) * kPcCols + k] * t;
      }
      const int64_t aj = rank[j] / coarse;
      E[(blockIdx.x * kPcCols + k) * nc + aj * kPcCols + k2] += acc;
    }
  }
}

__global__ void k_pc_rank(const int* __restrict__ order, int64_t T, int* __restrict__ rank) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < T) rank[order[p]] = (int)p;
}

// Dropped columns: identity on their row and column (both are zero), so E stays invertible and the
// column contributes nothing.
__global__ void k_pc_pad(const int* __restrict__ kept, int64_t nc, double* __restrict__ E) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nc && !kept[r]) E[r * nc + r] = 1.0;
}

// Gauss-Jordan in device memory: pivot search, row swap, column copy and row scaling of step k (one
// workgroup) ...
__global__ __launch_bounds__(256) void k_gj_pivot(double* __restrict__ E, int64_t n, int64_t k, int* __restrict__ piv,
                                                  double* __restrict__ col, int* __restrict__ singular) {
  __shared__ double sb[256];
  __shared__ int64_t si[256];
  double best = -1.0;
  int64_t bi = n;
  for (int64_t i = k + threadIdx.x; i < n; i += blockDim.x) {
    const double v = fabs(E[i * n + k]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  sb[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      const double ob = sb[threadIdx.x + st];
      const int64_t oi = si[threadIdx.x + st];
      if (ob > sb[threadIdx.x] || (ob == sb[threadIdx.x] && oi < si[threadIdx.x])) {
        sb[threadIdx.x] = ob;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int64_t p = si[0];
  if (threadIdx.x == 0) piv[k] = (int)p;
  if (p != k)
    for (int64_t t = threadIdx.x; t < n; t += blockDim.x) {
      const double x = E[k * n + t];
      E[k * n + t] = E[p * n + t];
      E[p * n + t] = x;
    }
  __syncthreads();
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) col[t] = E[t * n + k];
  __syncthreads();
  const double pv = col[k];
  if (threadIdx.x == 0 && pv == 0.0) atomicExch(singular, 1);
  for (int64_t t = threadIdx.x; t < n; t += blockDim.x) E[k * n + t] = (t == k) ? 1.0 / pv : E[k * n + t] / pv;
}

// ... and the elimination of column k from every other row.
__global__ void k_gj_update(double* __restrict__ E, int64_t n, int64_t k, const double* __restrict__ col) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= n || i == k) return;
  const double f = col[i];
  E[i * n + j] = (j == k ? 0.0 : E[i * n + j]) - f * E[k * n + j];
}

__global__ void k_gj_unscramble(double* __restrict__ E, int64_t n, const int* __restrict__ piv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t k = n - 1; k >= 0; --k) {
    const int64_t p = piv[k];
    if (p != k) {
      const double x = E[i * n + k];
      E[i * n + k] = E[i * n + p];
      E[i * n + p] = x;
    }
  }
}

// ---------------------------------------------------------------------------------------- apply

// s[a*6+k] = sum over the aggregate's unknowns of z[.][k] v
__global__ __launch_bounds__(64) void k_pc_zt(const double* __restrict__ v, const double* __restrict__ z,
                                              const int* __restrict__ order, int64_t T, int coarse,
                                              double* __restrict__ s) {
  const int64_t first = (int64_t)blockIdx.x * coarse;
  const int m = (int)min((int64_t)coarse, T - first);
  double acc[kPcCols] = {0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < m; i += 64) {
    const int64_t e = order[first + i];
    for (int c = 0; c < 3; ++c) {
      const double x = v[3 * e + c];
      for (int k = 0; k < kPcCols; ++k) acc[k] += z[(3 * e + c) * kPcCols + k] * x;
    }
  }
  for (int k = 0; k < kPcCols; ++k) {
    const double t = wave_sum(acc[k]);
    if (threadIdx.x == 0) s[blockIdx.x * kPcCols + k] = t;
  }
}

// g = E^-1 s, one wave per row
__global__ __launch_bounds__(256) void k_pc_gemv(const double* __restrict__ Einv, const double* __restrict__ s, int64_t n,
                                                 double* __restrict__ g) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (r >= n) return;
  double acc = 0.0;
  for (int64_t c = lane; c < n; c += 64) acc += Einv[r * n + c] * s[c];
  acc = wave_sum(acc);
  if (lane == 0) g[r] = acc;
}

// y = (fine block inverse) v + Z g, one workgroup per fine block
__global__ __launch_bounds__(128) void k_pc_fine_apply(const double* __restrict__ v, const double* __restrict__ binv_t,
                                                       const double* __restrict__ z, const double* __restrict__ g,
                                                       const int* __restrict__ order, int64_t T, int fine, int coarse,
                                                       double* __restrict__ y) {
  __shared__ double vl[kFineN];
  const int64_t first = (int64_t)blockIdx.x * fine;
  const int m = (int)min((int64_t)fine, T - first);
  const int n = 3 * m;
  for (int t = threadIdx.x; t < n; t += blockDim.x) vl[t] = v[3 * (int64_t)order[first + t / 3] + t % 3];
  __syncthreads();
  const double* B = binv_t + (size_t)blockIdx.x * kFineN * kFineN;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < n; ++c) acc += B[(size_t)c * kFineN + r] * vl[c];
    const int64_t pos = first + r / 3;
    const int64_t e = order[pos];
    const int comp = r % 3;
    const double* zr = z + (3 * e + comp) * kPcCols;
    const double* ga = g + (pos / coarse) * kPcCols;
    for (int k = 0; k < kPcCols; ++k) acc += zr[k] * ga[k];
    y[3 * e + comp] = acc;
  }
}

}  // namespace

int pc_default_aggregate(int64_t T) {
  int64_t c = 64;
  while (kPcCols * ((T + c - 1) / c) > kPcMaxCoarse) c *= 2;
  return (int)c;
}

void TwoLevelPC::build(const BemSystem& sys, int fine_, int coarse_) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = sys.stream;
  T = sys.T;
  fine = fine_ > 0 ? fine_ : kPcFineMax;
  coarse = coarse_ > 0 ? coarse_ : pc_default_aggregate(T);
  KFMM_REQUIRE(fine >= 1 && fine <= kPcFineMax, "preconditioner fine block size must be in [1, 32]");
  KFMM_REQUIRE(coarse >= 1, "preconditioner aggregate size must be positive");
  KFMM_REQUIRE(T < (int64_t(1) << 22), "the preconditioner supports fewer than 2^22 elements");
  nb = (T + fine - 1) / fine;
  na = (T + coarse - 1) / coarse;
  nc = kPcCols * na;
  KFMM_REQUIRE(nc <= 16384, "coarse dimension above 16384: raise the aggregate size");

  Arena scratch;
  // Morton order of the centroids
  int64_t n_pad = 2048;
  while (n_pad < T) n_pad *= 2;
  double* bounds = scratch.get<double>(6);
  uint64_t* key = scratch.get<uint64_t>(n_pad);
  int* idx = scratch.get<int>(n_pad);
  hipLaunchKernelGGL(k_pc_bounds, dim3(1), dim3(256), 0, st, sys.cen, T, bounds);
  hipLaunchKernelGGL(k_pc_keys, dim3(nblocks(T, 256)), dim3(256), 0, st, sys.cen, T, bounds, key, idx);
  KFMM_HIP(hipGetLastError());
  sort_keys(key, idx, T, n_pad, st);
  order = arena.get<int>(T);
  KFMM_HIP(hipMemcpyAsync(order, idx, sizeof(int) * T, hipMemcpyDeviceToDevice, st));

  const bool with_near = sys.near_levels > 0 && sys.near.n > 0;
  BlockArgs a{sys.qp,      sys.qn,
              sys.qw,      sys.cen,
              sys.dU,      sys.dP,
              sys.bc_type, sys.scale_t,
              sys.el,      with_near ? sys.near.off : nullptr,
              sys.near.idx, sys.near_dU,
              sys.near_dP};
  int* singular = scratch.get<int>(2);
  KFMM_HIP(hipMemsetAsync(singular, 0, 2 * sizeof(int), st));
  binv_t = arena.get<double>((size_t)nb * kFineN * kFineN);
  hipLaunchKernelGGL(k_pc_fine, dim3((unsigned)nb), dim3(256), 0, st, a, order, T, fine, binv_t, singular);
  KFMM_HIP(hipGetLastError());

  z = arena.get<double>((size_t)T * 3 * kPcCols);
  int* kept = scratch.get<int>(nc);
  hipLaunchKernelGGL(k_pc_coarse_cols, dim3((unsigned)na), dim3(64), 0, st, sys.cen, sys.bc_type, order, T, coarse, z,
                     kept);
  KFMM_HIP(hipGetLastError());
  einv = arena.get<double>((size_t)nc * nc);
  hipLaunchKernelGGL(k_pc_coarse_E, dim3((unsigned)na, (unsigned)na), dim3(64), 0, st, a, order, T, coarse, z, nc,
                     einv);
  KFMM_HIP(hipGetLastError());
  if (with_near) {
    int* rank = scratch.get<int>(T);
    hipLaunchKernelGGL(k_pc_rank, dim3(nblocks(T, 256)), dim3(256), 0, st, order, T, rank);
    hipLaunchKernelGGL(k_pc_coarse_E_near, dim3((unsigned)na), dim3(64), 0, st, a, order, rank, T, coarse, z, nc,
                       einv);
    KFMM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_pc_pad, dim3(nblocks(nc, 256)), dim3(256), 0, st, kept, nc, einv);
  int* piv = scratch.get<int>(nc);
  double* col = scratch.get<double>(nc);
  for (int64_t k = 0; k < nc; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, st, einv, nc, k, piv, col, singular + 1);
    hipLaunchKernelGGL(k_gj_update, dim3(nblocks(nc, 256), (unsigned)nc), dim3(256), 0, st, einv, nc, k, col);
  }
  hipLaunchKernelGGL(k_gj_unscramble, dim3(nblocks(nc, 256)), dim3(256), 0, st, einv, nc, piv);
  KFMM_HIP(hipGetLastError());
  s = arena.get<double>(nc);
  g = arena.get<double>(nc);

  int h_sing[2] = {0, 0};
  std::vector<int> h_kept(nc);
  KFMM_HIP(hipMemcpyAsync(h_sing, singular, sizeof(h_sing), hipMemcpyDeviceToHost, st));
  KFMM_HIP(hipMemcpyAsync(h_kept.data(), kept, sizeof(int) * nc, hipMemcpyDeviceToHost, st));
  KFMM_HIP(hipStreamSynchronize(st));
  KFMM_REQUIRE(!h_sing[0], "preconditioner: a fine block of the system is singular");
  KFMM_REQUIRE(!h_sing[1], "preconditioner: the coarse matrix Z^T A Z is singular");
  n_dropped = (int)std::count(h_kept.begin(), h_kept.end(), 0);
  t_setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

void TwoLevelPC::apply(const double* v, double* y, hipStream_t st) const {
  hipLaunchKernelGGL(k_pc_zt, dim3((unsigned)na), dim3(64), 0, st, v, z, order, T, coarse, s);
  hipLaunchKernelGGL(k_pc_gemv, dim3(nblocks(nc, 4)), dim3(256), 0, st, einv, s, nc, g);
  hipLaunchKernelGGL(k_pc_fine_apply, dim3((unsigned)nb), dim3(128), 0, st, v, binv_t, z, g, order, T, fine, coarse, y);
  KFMM_HIP(hipGetLastError());
}

}  // namespace kfmm
