// Near-singular quadrature of the collocation BEM (Sec. 2.2, "Matrix-vector products": the 16-point rule
// loses accuracy on the triangles next to the collocation point, and an upsampled quadrature is used there).
//
//  * Near pairs (t, e), t != e: |c_t - c_e|^2 < radius^2 l_e^2 with c the centroids and l_e the longest edge
//    of e.  Found on a uniform grid of cells of size radius * max_e l_e (a near pair lies in the same or an
//    adjacent cell): centroids sorted by cell key, then per element the 27 neighbouring cells searched by
//    binary search; each element's list is sorted by e.  Squared distances are summed as
//    dx*dx + dy*dy + dz*dz without fused multiply-adds, so the decision matches a plain FP64 evaluation.
//  * Periodic surface (a cell of side L): also the images c_e + L s, s in {-1, 0, 1}^3, are tested (the
//    element itself only at s != 0), found by searching around c_t - L s; a pair keeps its shift code
//    (sx+1) + 3 (sy+1) + 9 (sz+1), and a row is sorted by e, then code.  The blocks of an image are those of
//    e seen from c_t - L s (translation invariance).
//  * Per near pair the upsampled blocks: the triangle e split at its edge midpoints L + 1 times (children
//    (v0, m01, m20), (m01, v1, m12), (m20, m12, v2), (m01, m12, m20)), the symmetric 4-point rule on each of
//    the 4^(L+1) leaves (weights: leaf area x rule weight), leaves in the order of their base-4 index; minus
//    the element's 16 quadrature points as the fast summation applies them.  The local pass adds
//    dU a_e + dP b_e for every near e.
#include <hip/hip_runtime.h>

#include <vector>

#include "bem.h"
#include "common.h"
#include "tree.h"

namespace kfmm {

namespace {

unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// squared length ((x*x) + (y*y)) + (z*z), each operation rounded on its own (no fused multiply-add: the
// device compiler contracts by default, and these sums decide which pairs are near)
__device__ __forceinline__ double sq3(double x, double y, double z) {
#pragma clang fp contract(off)
  return x * x + y * y + z * z;
}

__global__ void k_near_l2(const double* __restrict__ tri, int64_t T, double* __restrict__ l2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  const double* v = tri + 9 * e;
  double m = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3;
    m = fmax(m, sq3(v[3 * b] - v[3 * a], v[3 * b + 1] - v[3 * a + 1], v[3 * b + 2] - v[3 * a + 2]));
  }
  l2[e] = m;
}

// out[0..2] = per-axis minimum of the centroids, out[3] = largest l2 (one workgroup)
__global__ __launch_bounds__(256) void k_near_bounds(const double* __restrict__ cen, const double* __restrict__ l2,
                                                     int64_t T, double* __restrict__ out) {
  __shared__ double red[4][256];
  double m[4] = {INFINITY, INFINITY, INFINITY, 0.0};
  for (int64_t e = threadIdx.x; e < T; e += blockDim.x) {
    for (int d = 0; d < 3; ++d) m[d] = fmin(m[d], cen[3 * e + d]);
    m[3] = fmax(m[3], l2[e]);
  }
  for (int d = 0; d < 4; ++d) red[d][threadIdx.x] = m[d];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + st]);
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 4; ++d) out[d] = red[d][0];
}

constexpr int kCellBits = 21;

__device__ __forceinline__ int64_t cell_of(double x, double lo, double cs) {
  int64_t q = (int64_t)floor((x - lo) / cs);
  return q < 0 ? 0 : (q > (1 << kCellBits) - 1 ? (1 << kCellBits) - 1 : q);
}

__device__ __forceinline__ uint64_t cell_key(int64_t qx, int64_t qy, int64_t qz) {
  return ((uint64_t)qx << (2 * kCellBits)) | ((uint64_t)qy << kCellBits) | (uint64_t)qz;
}

__global__ void k_near_keys(const double* __restrict__ cen, int64_t T, const double* __restrict__ bounds, double cs,
                            uint64_t* __restrict__ key, int* __restrict__ idx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  key[e] = cell_key(cell_of(cen[3 * e], bounds[0], cs), cell_of(cen[3 * e + 1], bounds[1], cs),
                    cell_of(cen[3 * e + 2], bounds[2], cs));
  idx[e] = (int)e;
}

// first position in sorted keys[0, n) with keys[pos] >= k
__device__ __forceinline__ int64_t lower_bound(const uint64_t* keys, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (keys[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Pass 0 counts the near elements of each t into cnt[t]; pass 1 writes them at idx[off[t]...] (with the
// row t in row[] and, on a periodic surface of side L > 0, the shift code in sh[]) and sorts the row by e,
// then code.
__global__ void k_near_scan(int pass, const double* __restrict__ cen, const double* __restrict__ l2, int64_t T,
                            const double* __restrict__ bounds, double cs, double r2, const uint64_t* __restrict__ keys,
                            const int* __restrict__ sorted, int* __restrict__ cnt, const int* __restrict__ off,
                            int* __restrict__ idx, int* __restrict__ row, double L, signed char* __restrict__ sh) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  int n = 0;
  const int64_t base = pass ? off[t] : 0;
  const int s_lo = L > 0 ? -1 : 0, s_hi = L > 0 ? 1 : 0;
  for (int sz = s_lo; sz <= s_hi; ++sz)
    for (int sy = s_lo; sy <= s_hi; ++sy)
      for (int sx = s_lo; sx <= s_hi; ++sx) {
        const int code = (sx + 1) + 3 * (sy + 1) + 9 * (sz + 1);
        // cells searched around c_t - L s; the decision on (c_e + L s) - c_t, each sum rounded on its own
        const double cx = cen[3 * t] - L * sx, cy = cen[3 * t + 1] - L * sy, cz = cen[3 * t + 2] - L * sz;
        const double ox = L * sx, oy = L * sy, oz = L * sz;
        const int64_t qx = cell_of(cx, bounds[0], cs), qy = cell_of(cy, bounds[1], cs), qz = cell_of(cz, bounds[2], cs);
        for (int64_t dx = -1; dx <= 1; ++dx)
          for (int64_t dy = -1; dy <= 1; ++dy)
            for (int64_t dz = -1; dz <= 1; ++dz) {
              const int64_t ax = qx + dx, ay = qy + dy, az = qz + dz;
              if (ax < 0 || ay < 0 || az < 0 || ax >= (1 << kCellBits) || ay >= (1 << kCellBits) ||
                  az >= (1 << kCellBits))
                continue;
              const uint64_t k = cell_key(ax, ay, az);
              for (int64_t p = lower_bound(keys, T, k); p < T && keys[p] == k; ++p) {
                const int e = sorted[p];
                if (e == t && code == 13) continue;
                const double d2 = sq3(__dsub_rn(__dadd_rn(cen[3 * e], ox), cen[3 * t]),
                                      __dsub_rn(__dadd_rn(cen[3 * e + 1], oy), cen[3 * t + 1]),
                                      __dsub_rn(__dadd_rn(cen[3 * e + 2], oz), cen[3 * t + 2]));
                if (d2 < __dmul_rn(r2, l2[e])) {
                  if (pass) {
                    idx[base + n] = e;
                    row[base + n] = (int)t;
                    if (sh) sh[base + n] = (signed char)code;
                  }
                  ++n;
                }
              }
            }
      }
  if (!pass) {
    cnt[t] = n;
    return;
  }
  for (int a = 1; a < n; ++a) {  // insertion sort of the row by e, then code
    const int v = idx[base + a];
    const signed char c = sh ? sh[base + a] : 0;
    int b = a - 1;
    while (b >= 0 && (idx[base + b] > v || (idx[base + b] == v && sh && sh[base + b] > c))) {
      idx[base + b + 1] = idx[base + b];
      if (sh) sh[base + b + 1] = sh[base + b];
      --b;
    }
    idx[base + b + 1] = v;
    if (sh) sh[base + b + 1] = c;
  }
}

// Kelvin blocks of one point: U, P (eq. disp_1, eq. disp_2 with the leading minus), d = source - target
__device__ __forceinline__ void kelvin_add(const double* x, const double* y, const double* n, double w,
                                           const Elastic& el, double U[3][3], double P[3][3]) {
  const double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (r2 == 0.0) return;
  const double r = sqrt(r2), ir = 1.0 / r;
  const double rh[3] = {d[0] * ir, d[1] * ir, d[2] * ir};
  const double drdn = rh[0] * n[0] + rh[1] * n[1] + rh[2] * n[2];
  const double a34 = 3.0 - 4.0 * el.nu, a12 = 1.0 - 2.0 * el.nu;
  const double cu = el.cU * ir * w, cp = -el.cP * ir * ir * w;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double rr = rh[i] * rh[j];
      U[i][j] += cu * ((i == j ? a34 : 0.0) + rr);
      P[i][j] += cp * (drdn * ((i == j ? a12 : 0.0) + 3.0 * rr) - a12 * (rh[i] * n[j] - rh[j] * n[i]));
    }
}

__constant__ double c_bary[4][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
__constant__ double c_rw[4] = {-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48};

// dU, dP of each near pair: upsampled blocks minus the element's 16 quadrature points
__global__ void k_near_blocks(int64_t n, const int* __restrict__ row, const int* __restrict__ col, int levels,
                              const double* __restrict__ tri, const double* __restrict__ cen,
                              const double* __restrict__ qp, const double* __restrict__ qn,
                              const double* __restrict__ qw, Elastic el, double* __restrict__ dU,
                              double* __restrict__ dP, const signed char* __restrict__ sh, double L) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t t = row[p], e = col[p];
  // an image shifted by L s is e seen from c_t - L s
  const int code = sh ? sh[p] : 13;
  const double x[3] = {cen[3 * t] - L * (code % 3 - 1), cen[3 * t + 1] - L * ((code / 3) % 3 - 1),
                       cen[3 * t + 2] - L * (code / 9 - 1)};
  const double* v = tri + 9 * e;
  double e1[3], e2[3], nr[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = v[3 + d] - v[d];
    e2[d] = v[6 + d] - v[d];
  }
  nr[0] = e1[1] * e2[2] - e1[2] * e2[1];
  nr[1] = e1[2] * e2[0] - e1[0] * e2[2];
  nr[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double a2 = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
  for (int d = 0; d < 3; ++d) nr[d] /= a2;
  int64_t nleaf = 1;
  for (int d = 0; d <= levels; ++d) nleaf *= 4;
  const double leaf_area = 0.5 * a2 / (double)nleaf;
  double U[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, P[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int64_t k = 0; k < nleaf; ++k) {
    double c[3][3];
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) c[a][d] = v[3 * a + d];
    for (int64_t div = nleaf / 4; div >= 1; div /= 4) {
      const int child = (int)((k / div) % 4);
      double m01[3], m12[3], m20[3];
      for (int d = 0; d < 3; ++d) {
        m01[d] = 0.5 * (c[0][d] + c[1][d]);
        m12[d] = 0.5 * (c[1][d] + c[2][d]);
        m20[d] = 0.5 * (c[2][d] + c[0][d]);
      }
      for (int d = 0; d < 3; ++d) {
        const double a = c[0][d], b = c[1][d], cc = c[2][d];
        if (child == 0) {
          c[0][d] = a;
          c[1][d] = m01[d];
          c[2][d] = m20[d];
        } else if (child == 1) {
          c[0][d] = m01[d];
          c[1][d] = b;
          c[2][d] = m12[d];
        } else if (child == 2) {
          c[0][d] = m20[d];
          c[1][d] = m12[d];
          c[2][d] = cc;
        } else {
          c[0][d] = m01[d];
          c[1][d] = m12[d];
          c[2][d] = m20[d];
        }
      }
    }
    for (int q = 0; q < 4; ++q) {
      double y[3];
      for (int d = 0; d < 3; ++d) y[d] = c_bary[q][0] * c[0][d] + c_bary[q][1] * c[1][d] + c_bary[q][2] * c[2][d];
      kelvin_add(x, y, nr, leaf_area * c_rw[q], el, U, P);
    }
  }
  double U16[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, P16[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int q = 0; q < 16; ++q) {
    const int64_t s = 16 * e + q;
    kelvin_add(x, qp + 3 * s, qn + 3 * s, qw[s], el, U16, P16);
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      dU[9 * p + 3 * i + j] = U[i][j] - U16[i][j];
      dP[9 * p + 3 * i + j] = P[i][j] - P16[i][j];
    }
}

}  // namespace

NearPairs find_near_pairs(const double* tri, const double* cen, int64_t T, double radius, Arena& arena,
                          hipStream_t s, double cell_L) {
  KFMM_REQUIRE(radius > 0 && radius < 16, "near_radius must be in (0, 16)");
  KFMM_REQUIRE(cell_L >= 0, "near pairs: bad cell side");
  NearPairs np;
  np.cell_L = cell_L;
  Arena scratch;
  double* l2 = arena.get<double>(T);
  hipLaunchKernelGGL(k_near_l2, dim3(nblk(T, 256)), dim3(256), 0, s, tri, T, l2);
  double* bounds = scratch.get<double>(4);
  hipLaunchKernelGGL(k_near_bounds, dim3(1), dim3(256), 0, s, cen, l2, T, bounds);
  KFMM_HIP(hipGetLastError());
  double hb[4];
  KFMM_HIP(hipMemcpyAsync(hb, bounds, sizeof(hb), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  // cells no smaller than the largest near distance (slightly enlarged against rounding in the cell index)
  double cs = radius * std::sqrt(hb[3]) * (1.0 + 1e-9);
  // on a periodic surface only the 27 images around the cell are searched: every near distance must stay
  // below the cell side
  KFMM_REQUIRE(cell_L == 0 || cs < cell_L,
               "near pairs: near_radius times the longest element edge must be below the periodic cell's side");
  if (!(cs > 0)) cs = 1.0;
  int64_t n_pad = 2048;
  while (n_pad < T) n_pad *= 2;
  uint64_t* keys = scratch.get<uint64_t>(n_pad);
  int* sorted = scratch.get<int>(n_pad);
  hipLaunchKernelGGL(k_near_keys, dim3(nblk(T, 256)), dim3(256), 0, s, cen, T, bounds, cs, keys, sorted);
  KFMM_HIP(hipGetLastError());
  sort_keys(keys, sorted, T, n_pad, s);
  int* cnt = scratch.get<int>(T);
  const double r2 = radius * radius;
  hipLaunchKernelGGL(k_near_scan, dim3(nblk(T, 128)), dim3(128), 0, s, 0, cen, l2, T, bounds, cs, r2, keys, sorted, cnt,
                     (const int*)nullptr, (int*)nullptr, (int*)nullptr, cell_L, (signed char*)nullptr);
  KFMM_HIP(hipGetLastError());
  std::vector<int> hc(T);
  KFMM_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int) * T, hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  std::vector<int> ho(T + 1, 0);
  for (int64_t t = 0; t < T; ++t) {
    KFMM_REQUIRE((int64_t)ho[t] + hc[t] < ((int64_t)1 << 31), "too many near pairs");
    ho[t + 1] = ho[t] + hc[t];
  }
  np.n = ho[T];
  np.off = arena.get<int>(T + 1);
  KFMM_HIP(hipMemcpyAsync(np.off, ho.data(), sizeof(int) * (T + 1), hipMemcpyHostToDevice, s));
  np.idx = arena.get<int>(std::max<int64_t>(np.n, 1));
  np.row = arena.get<int>(std::max<int64_t>(np.n, 1));
  if (cell_L > 0) np.sh = arena.get<signed char>(std::max<int64_t>(np.n, 1));
  hipLaunchKernelGGL(k_near_scan, dim3(nblk(T, 128)), dim3(128), 0, s, 1, cen, l2, T, bounds, cs, r2, keys, sorted, cnt,
                     np.off, np.idx, np.row, cell_L, np.sh);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));  // scratch (keys, sorted) is released on return
  return np;
}

void near_blocks(const NearPairs& np, int levels, const double* tri, const double* cen, const double* qp,
                 const double* qn, const double* qw, const Elastic& el, double* dU, double* dP, hipStream_t s) {
  KFMM_REQUIRE(levels >= 1 && levels <= 5, "near_levels must be in [0, 5]");
  if (np.n == 0) return;
  hipLaunchKernelGGL(k_near_blocks, dim3(nblk(np.n, 64)), dim3(64), 0, s, np.n, np.row, np.idx, levels, tri, cen,
                     qp, qn, qw, el, dU, dP, (const signed char*)np.sh, np.cell_L);
  KFMM_HIP(hipGetLastError());
}

}  // namespace kfmm
