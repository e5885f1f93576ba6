// The voxel steps of Algorithm 1 (Sec. 2.3, hard-kill topology optimisation) and the adaptive sampling of
// the interior (Sec. 2.2 end, Sec. 5 "adaptive grid") on the device, so that an optimisation iteration runs
// without the host: boundary extraction, targets, the removal rule with face-connected post-processing,
// and the two-scale (coarse blocks, then refined voxels) choice of stress targets.
//
// A design is a uint8 array (nonzero = material) of nx x ny x nz voxels of edge h, C order (i slowest),
// origin at 0.  Conventions (face classes, corner order, boundary conditions, rule, blocks) are those of
// include/kfmm.h; every compaction keeps linear voxel order (device exclusive scans), so the outputs are
// deterministic and independent of scheduling.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/kfmm.h"

// Every coordinate here is a product or a sum rounded on its own, as written (the device compiler would
// otherwise fuse a multiply and an add, and the triangles would differ in the last bit from the definition).
#pragma clang fp contract(off)
#include "common.h"
#include "tree.h"

#include <cmath>

namespace kfmm {

namespace {

unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

struct Grid {
  int nx, ny, nz;
  double h;
  __host__ __device__ int64_t n() const { return (int64_t)nx * ny * nz; }
  __host__ __device__ int64_t lin(int i, int j, int k) const { return ((int64_t)i * ny + j) * nz + k; }
  __host__ __device__ bool inside(int i, int j, int k) const {
    return i >= 0 && j >= 0 && k >= 0 && i < nx && j < ny && k < nz;
  }
};

__device__ __forceinline__ void unlin(const Grid& g, int64_t v, int& i, int& j, int& k) {
  k = (int)(v % g.nz);
  j = (int)((v / g.nz) % g.ny);
  i = (int)(v / ((int64_t)g.ny * g.nz));
}

// ------------------------------------------------------------------------- exclusive scan (one workgroup)

// out[i] = sum_{j < i} in[j] (int64), total in out[n]; 1024 threads, each a contiguous chunk.
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024, b = t * per, e = b + per < n ? b + per : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan of the chunk sums
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = b; i < e; ++i) {
    out[i] = run;
    run += in[i];
  }
  if (t == 1023) out[n] = part[1023];
}

// ------------------------------------------------------------------------------------------ surface

constexpr int kClasses = 6;  // (axis 0, +), (axis 0, -), (axis 1, +), ...

__device__ __forceinline__ bool filled(const Grid& g, const uint8_t* vox, int i, int j, int k) {
  return g.inside(i, j, k) && vox[g.lin(i, j, k)] != 0;
}

// Boundary conditions of the emitted faces.  Cantilever (periodic == 0): clamped x = 0 faces of the first
// layer, the load on the +x faces of the last layer, traction-free elsewhere.  Periodic cell (periodic ==
// 1): neighbours wrap around the cell, and every face carries the traction -sig n of the superposition
// formulation (sig row-major 3 x 3, n the face normal out of the material).
struct FaceBC {
  int periodic;
  double load[3];
  double sig[9];
};

// flag[c * n + v] = 1 when voxel v has an exposed face of class c
__global__ void k_face_flags(Grid g, const uint8_t* __restrict__ vox, int periodic, int* __restrict__ flag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n()) return;
  int i, j, k;
  unlin(g, v, i, j, k);
  const bool f = vox[v] != 0;
  const int dims[3] = {g.nx, g.ny, g.nz};
  for (int c = 0; c < kClasses; ++c) {
    const int a = c / 2, s = (c % 2 == 0) ? 1 : -1;
    int nb[3] = {i, j, k};
    nb[a] += s;
    if (periodic) nb[a] = (nb[a] + dims[a]) % dims[a];
    flag[c * g.n() + v] = (f && !filled(g, vox, nb[0], nb[1], nb[2])) ? 1 : 0;
  }
}

__global__ void k_face_emit(Grid g, const uint8_t* __restrict__ vox, const int* __restrict__ flag,
                            const int64_t* __restrict__ pos, FaceBC fb, double* __restrict__ tri,
                            int8_t* __restrict__ bct, double* __restrict__ bcv, int32_t* __restrict__ owner) {
  const int64_t cv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cv >= kClasses * g.n() || !flag[cv]) return;
  const int c = (int)(cv / g.n());
  const int64_t v = cv % g.n();
  int idx[3];
  unlin(g, v, idx[0], idx[1], idx[2]);
  const int a = c / 2, s = (c % 2 == 0) ? 1 : -1, b = (a + 1) % 3, cc = (a + 2) % 3;
  int base[3] = {idx[0], idx[1], idx[2]};
  if (s > 0) base[a] += 1;
  const int dims[3] = {g.nx, g.ny, g.nz};
  if (fb.periodic && base[a] == dims[a]) base[a] = 0;  // the upper face of the cell is its lower face
  const int offs[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
  double q[4][3];
  for (int e = 0; e < 4; ++e) {
    const int o = s > 0 ? e : 3 - e;
    int p[3] = {base[0], base[1], base[2]};
    p[b] += offs[o][0];
    p[cc] += offs[o][1];
    for (int d = 0; d < 3; ++d) q[e][d] = g.h * (double)p[d];
  }
  double cen[3];
  for (int d = 0; d < 3; ++d) cen[d] = (((q[0][d] + q[1][d]) + q[2][d]) + q[3][d]) / 4.0;
  const bool clamp = !fb.periodic && a == 0 && s < 0 && idx[0] == 0;
  const bool loaded = !fb.periodic && a == 0 && s > 0 && idx[0] == g.nx - 1;
  double val[3];
  for (int d = 0; d < 3; ++d) val[d] = fb.periodic ? -(double)s * fb.sig[3 * d + a] : (loaded ? fb.load[d] : 0.0);
  const int64_t t0 = 4 * pos[cv];
  for (int e = 0; e < 4; ++e) {
    const int64_t t = t0 + e;
    for (int d = 0; d < 3; ++d) {
      tri[9 * t + d] = q[e][d];
      tri[9 * t + 3 + d] = q[(e + 1) % 4][d];
      tri[9 * t + 6 + d] = cen[d];
      bct[3 * t + d] = clamp ? 0 : 1;
      bcv[3 * t + d] = val[d];
      if (owner) owner[3 * t + d] = idx[d];
    }
  }
}

// ---------------------------------------------------------------------------------- voxel selection

__global__ void k_filled_flags(int64_t n, const uint8_t* __restrict__ vox, int* __restrict__ flag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = vox[v] != 0 ? 1 : 0;
}

// centres (idx + 1/2) h of the flagged voxels at their scan positions
__global__ void k_emit_centres(Grid g, const int* __restrict__ flag, const int64_t* __restrict__ pos,
                               double* __restrict__ pts) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n() || !flag[v]) return;
  int i, j, k;
  unlin(g, v, i, j, k);
  const int64_t r = pos[v];
  pts[3 * r] = ((double)i + 0.5) * g.h;
  pts[3 * r + 1] = ((double)j + 0.5) * g.h;
  pts[3 * r + 2] = ((double)k + 0.5) * g.h;
}

// minimum and maximum of x[0, n) (one workgroup): out[0] = min, out[1] = max
__global__ __launch_bounds__(256) void k_minmax(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
  __shared__ double lo[256], hi[256];
  double a = INFINITY, b = -INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    a = fmin(a, x[i]);
    b = fmax(b, x[i]);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + st]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = lo[0];
    out[1] = hi[0];
  }
}

// removal rule: material stays unless td < thr (strict) outside the two end layers; labels initialised
__global__ void k_remove(Grid g, const uint8_t* __restrict__ vox, const int64_t* __restrict__ rank,
                         const double* __restrict__ td, double thr, uint8_t* __restrict__ out, int64_t* __restrict__ lab) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n()) return;
  int i, j, k;
  unlin(g, v, i, j, k);
  bool keep = vox[v] != 0;
  if (keep && i > 0 && i < g.nx - 1 && td[rank[v]] < thr) keep = false;
  out[v] = keep ? 1 : 0;
  lab[v] = keep ? v : -1;
}

// one round of face-neighbour minimum and pointer jumping; *changed set when a label moved
__global__ void k_label_round(Grid g, const uint8_t* __restrict__ m, int64_t* __restrict__ lab, int* __restrict__ changed) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n() || !m[v]) return;
  int i, j, k;
  unlin(g, v, i, j, k);
  int64_t best = lab[v];
  const int d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  for (int q = 0; q < 6; ++q) {
    const int u = i + d[q][0], w = j + d[q][1], z = k + d[q][2];
    if (g.inside(u, w, z) && m[g.lin(u, w, z)]) {
      const int64_t l = lab[g.lin(u, w, z)];
      if (l < best) best = l;
    }
  }
  const int64_t jump = lab[best];  // best is a filled voxel of the same component
  if (jump < best) best = jump;
  if (best < lab[v]) {
    lab[v] = best;
    *changed = 1;
  }
}

// labels present in the first (x = 0) and last (x = nx - 1) layers
__global__ void k_end_labels(Grid g, const uint8_t* __restrict__ m, const int64_t* __restrict__ lab,
                             uint8_t* __restrict__ at0, uint8_t* __restrict__ at1) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n() || !m[v]) return;
  int i, j, k;
  unlin(g, v, i, j, k);
  if (i == 0) at0[lab[v]] = 1;
  if (i == g.nx - 1) at1[lab[v]] = 1;
}

__global__ void k_keep_connected(int64_t n, const int64_t* __restrict__ lab, const uint8_t* __restrict__ at0,
                                 const uint8_t* __restrict__ at1, uint8_t* __restrict__ m, int* __restrict__ flag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (m[v] && !(at0[lab[v]] && at1[lab[v]])) m[v] = 0;
  flag[v] = m[v] ? 1 : 0;
}

// ------------------------------------------------------------------------------------------- blocks

struct Blocks {
  int b, bx, by, bz;
  __host__ __device__ int64_t n() const { return (int64_t)bx * by * bz; }
  __host__ __device__ int64_t lin(int I, int J, int K) const { return ((int64_t)I * by + J) * bz + K; }
};

__global__ void k_block_full(Grid g, Blocks B, const uint8_t* __restrict__ vox, int* __restrict__ full) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= B.n()) return;
  const int K = (int)(q % B.bz), J = (int)((q / B.bz) % B.by), I = (int)(q / ((int64_t)B.by * B.bz));
  bool f = true;
  for (int di = 0; di < B.b && f; ++di)
    for (int dj = 0; dj < B.b && f; ++dj)
      for (int dk = 0; dk < B.b && f; ++dk) f = filled(g, vox, I * B.b + di, J * B.b + dj, K * B.b + dk);
  full[q] = f ? 1 : 0;
}

__global__ void k_block_centres(Blocks B, double h, const int* __restrict__ full, const int64_t* __restrict__ pos,
                                double* __restrict__ pts) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= B.n() || !full[q]) return;
  const int K = (int)(q % B.bz), J = (int)((q / B.bz) % B.by), I = (int)(q / ((int64_t)B.by * B.bz));
  const double bh = (double)B.b * h;
  const int64_t r = pos[q];
  pts[3 * r] = ((double)I + 0.5) * bh;
  pts[3 * r + 1] = ((double)J + 0.5) * bh;
  pts[3 * r + 2] = ((double)K + 0.5) * bh;
}

// refined[q] = 0 only for a full block whose six neighbours are full blocks with the same decision
__global__ void k_block_refine(Blocks B, const int* __restrict__ full, const int64_t* __restrict__ pos,
                               const double* __restrict__ td_c, double thr, uint8_t* __restrict__ refined) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= B.n()) return;
  if (!full[q]) {
    refined[q] = 1;
    return;
  }
  const int K = (int)(q % B.bz), J = (int)((q / B.bz) % B.by), I = (int)(q / ((int64_t)B.by * B.bz));
  const bool kill = td_c[pos[q]] < thr;
  bool settled = true;
  const int d[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  for (int s = 0; s < 6 && settled; ++s) {
    const int u = I + d[s][0], w = J + d[s][1], z = K + d[s][2];
    if (u < 0 || w < 0 || z < 0 || u >= B.bx || w >= B.by || z >= B.bz) {
      settled = false;
      break;
    }
    const int64_t qn = B.lin(u, w, z);
    if (!full[qn] || (td_c[pos[qn]] < thr) != kill) settled = false;
  }
  refined[q] = settled ? 0 : 1;
}

// flag of the filled voxels in refined blocks
__global__ void k_fine_flags(Grid g, Blocks B, const uint8_t* __restrict__ vox, const uint8_t* __restrict__ refined,
                             int* __restrict__ flag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n()) return;
  int i, j, k;
  unlin(g, v, i, j, k);
  flag[v] = (vox[v] && refined[B.lin(i / B.b, j / B.b, k / B.b)]) ? 1 : 0;
}

// expanded field: one value per filled voxel (linear order)
__global__ void k_expand(Grid g, Blocks B, const uint8_t* __restrict__ vox, const int64_t* __restrict__ rank,
                         const uint8_t* __restrict__ refined, const int64_t* __restrict__ fine_pos,
                         const int64_t* __restrict__ block_pos, const double* __restrict__ td_c,
                         const double* __restrict__ td_f, double* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n() || !vox[v]) return;
  int i, j, k;
  unlin(g, v, i, j, k);
  const int64_t q = B.lin(i / B.b, j / B.b, k / B.b);
  out[rank[v]] = refined[q] ? td_f[fine_pos[v]] : td_c[block_pos[q]];
}

// ------------------------------------------------------------------------------------------ energy

// sum over points of the strain energy density (1/2E)[(1 + nu) sig:sig - nu (tr sig)^2] (one workgroup,
// fixed order)
__global__ __launch_bounds__(256) void k_energy(const double* __restrict__ sig, int64_t n, double E, double nu,
                                                double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
    const double* s = sig + 6 * p;
    const double ss = s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
    const double tr = s[0] + s[1] + s[2];
    acc += 0.5 * ((1.0 + nu) * ss - nu * tr * tr) / E;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------------ periodic cell: volume-fraction rule

// Ascending keys <=> ascending values of finite doubles (sign-magnitude bits to an unsigned order; -0 is
// taken as +0 first).
__device__ __forceinline__ uint64_t order_key(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x + 0.0);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void k_td_keys(int64_t n, const double* __restrict__ td, uint64_t* __restrict__ key, int* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = order_key(td[i]);
  idx[i] = (int)i;
}

// lin[rank] = linear index of the rank-th filled voxel
__global__ void k_rank_lin(Grid g, const int* __restrict__ flag, const int64_t* __restrict__ pos,
                           int64_t* __restrict__ lin) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < g.n() && flag[v]) lin[pos[v]] = v;
}

__global__ void k_copy_u8(int64_t n, const uint8_t* __restrict__ in, uint8_t* __restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) out[v] = in[v] != 0 ? 1 : 0;
}

// the n_remove filled voxels first in (td, rank) order become empty
__global__ void k_remove_lowest(int64_t n_remove, const int* __restrict__ order, const int64_t* __restrict__ lin,
                                uint8_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_remove) out[lin[order[r]]] = 0;
}

Grid grid_of(const alg1_grid* g) {
  KFMM_REQUIRE(g != nullptr, "grid is NULL");
  KFMM_REQUIRE(g->nx > 0 && g->ny > 0 && g->nz > 0 && (int64_t)g->nx * g->ny * g->nz < ((int64_t)1 << 31),
               "grid sizes must be positive, fewer than 2^31 voxels");
  KFMM_REQUIRE(std::isfinite(g->h) && g->h > 0, "voxel edge h must be finite and positive");
  return Grid{g->nx, g->ny, g->nz, g->h};
}

Blocks blocks_of(const Grid& g, int b) {
  KFMM_REQUIRE(b >= 1 && b <= 64, "block size must be in [1, 64]");
  return Blocks{b, (g.nx + b - 1) / b, (g.ny + b - 1) / b, (g.nz + b - 1) / b};
}

int64_t scan(Arena& a, const int* flag, int64_t n, int64_t*& pos, hipStream_t s) {
  pos = a.get<int64_t>(n + 1);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, flag, n, pos);
  KFMM_HIP(hipGetLastError());
  int64_t tot = 0;
  KFMM_HIP(hipMemcpyAsync(&tot, pos + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  return tot;
}

}  // namespace

static void surface(const Grid& g, const uint8_t* vox, const FaceBC& fb, int64_t* n_tri, double* tri, int8_t* bct,
                    double* bcv, int32_t* owner, int64_t capacity, hipStream_t s) {
  KFMM_REQUIRE(vox && n_tri, "vox or n_tri is NULL");
  Arena a;
  int* flag = a.get<int>(kClasses * g.n());
  hipLaunchKernelGGL(k_face_flags, dim3(nblk(g.n(), 256)), dim3(256), 0, s, g, vox, fb.periodic, flag);
  KFMM_HIP(hipGetLastError());
  int64_t* pos = nullptr;
  const int64_t faces = scan(a, flag, kClasses * g.n(), pos, s);
  *n_tri = 4 * faces;
  if (!tri) return;
  KFMM_REQUIRE(capacity >= 4 * faces, "output holds fewer triangles than the surface has");
  KFMM_REQUIRE(bct && bcv, "bc_type or bc_val is NULL");
  hipLaunchKernelGGL(k_face_emit, dim3(nblk(kClasses * g.n(), 256)), dim3(256), 0, s, g, vox, flag, pos, fb, tri, bct,
                     bcv, owner);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));
}

void alg1_surface_impl(const alg1_grid* gp, const uint8_t* vox, const double* load, int64_t* n_tri, double* tri,
                       int8_t* bct, double* bcv, int32_t* owner, int64_t capacity, hipStream_t s) {
  const Grid g = grid_of(gp);
  FaceBC fb{};
  fb.periodic = 0;
  fb.load[0] = load ? load[0] : 0.0;
  fb.load[1] = load ? load[1] : 0.0;
  fb.load[2] = load ? load[2] : -1.0;
  surface(g, vox, fb, n_tri, tri, bct, bcv, owner, capacity, s);
}

void alg1_cell_surface_impl(const alg1_grid* gp, const uint8_t* vox, const double* sig_h, int64_t* n_tri,
                            double* tri, int8_t* bct, double* bcv, int32_t* owner, int64_t capacity, hipStream_t s) {
  const Grid g = grid_of(gp);
  KFMM_REQUIRE(sig_h != nullptr, "sig_h is NULL");
  FaceBC fb{};
  fb.periodic = 1;
  const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};  // Voigt xx, yy, zz, yz, xz, xy
  for (int c = 0; c < 6; ++c) {
    KFMM_REQUIRE(std::isfinite(sig_h[c]), "sig_h must be finite");
    fb.sig[3 * vi[c] + vj[c]] = sig_h[c];
    fb.sig[3 * vj[c] + vi[c]] = sig_h[c];
  }
  surface(g, vox, fb, n_tri, tri, bct, bcv, owner, capacity, s);
}

void alg1_centres_impl(const alg1_grid* gp, const uint8_t* vox, int64_t* n, double* pts, int64_t capacity,
                       hipStream_t s) {
  const Grid g = grid_of(gp);
  KFMM_REQUIRE(vox && n, "vox or n is NULL");
  Arena a;
  int* flag = a.get<int>(g.n());
  hipLaunchKernelGGL(k_filled_flags, dim3(nblk(g.n(), 256)), dim3(256), 0, s, g.n(), vox, flag);
  int64_t* pos = nullptr;
  *n = scan(a, flag, g.n(), pos, s);
  if (!pts) return;
  KFMM_REQUIRE(capacity >= *n, "output holds fewer points than there are filled voxels");
  hipLaunchKernelGGL(k_emit_centres, dim3(nblk(g.n(), 256)), dim3(256), 0, s, g, flag, pos, pts);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));
}

void alg1_update_impl(const alg1_grid* gp, const uint8_t* vox, const double* td, int64_t n_td, double C,
                      uint8_t* out, int64_t* n_out, hipStream_t s) {
  const Grid g = grid_of(gp);
  KFMM_REQUIRE(vox && td && out && vox != out, "vox, td or out is NULL, or out aliases vox");
  KFMM_REQUIRE(std::isfinite(C) && C >= 0 && C <= 1, "C must be in [0, 1]");
  Arena a;
  const int64_t n = g.n();
  int* flag = a.get<int>(n);
  hipLaunchKernelGGL(k_filled_flags, dim3(nblk(n, 256)), dim3(256), 0, s, n, vox, flag);
  int64_t* rank = nullptr;
  const int64_t nf = scan(a, flag, n, rank, s);
  KFMM_REQUIRE(nf > 0, "the design holds no material");
  KFMM_REQUIRE(n_td == nf, "td must hold one value per filled voxel");
  double* mm = a.get<double>(2);
  hipLaunchKernelGGL(k_minmax, dim3(1), dim3(256), 0, s, td, nf, mm);
  double hmm[2];
  KFMM_HIP(hipMemcpyAsync(hmm, mm, sizeof(hmm), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  KFMM_REQUIRE(std::isfinite(hmm[0]) && std::isfinite(hmm[1]), "non-finite topological derivative");
  const double thr = hmm[0] + C * (hmm[1] - hmm[0]);
  int64_t* lab = a.get<int64_t>(n);
  hipLaunchKernelGGL(k_remove, dim3(nblk(n, 256)), dim3(256), 0, s, g, vox, rank, td, thr, out, lab);
  KFMM_HIP(hipGetLastError());
  int* changed = a.get<int>(1);
  for (int64_t round = 0;; ++round) {
    KFMM_REQUIRE(round <= n, "internal: labels did not settle");
    int h = 0;
    KFMM_HIP(hipMemsetAsync(changed, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_label_round, dim3(nblk(n, 256)), dim3(256), 0, s, g, out, lab, changed);
    KFMM_HIP(hipGetLastError());
    KFMM_HIP(hipMemcpyAsync(&h, changed, sizeof(int), hipMemcpyDeviceToHost, s));
    KFMM_HIP(hipStreamSynchronize(s));
    if (!h) break;
  }
  uint8_t* at0 = a.get<uint8_t>(n);
  uint8_t* at1 = a.get<uint8_t>(n);
  KFMM_HIP(hipMemsetAsync(at0, 0, n, s));
  KFMM_HIP(hipMemsetAsync(at1, 0, n, s));
  hipLaunchKernelGGL(k_end_labels, dim3(nblk(n, 256)), dim3(256), 0, s, g, out, lab, at0, at1);
  hipLaunchKernelGGL(k_keep_connected, dim3(nblk(n, 256)), dim3(256), 0, s, n, lab, at0, at1, out, flag);
  KFMM_HIP(hipGetLastError());
  int64_t* pos = nullptr;
  const int64_t kept = scan(a, flag, n, pos, s);
  if (n_out) *n_out = kept;
}

void alg1_cell_update_impl(const alg1_grid* gp, const uint8_t* vox, const double* td, int64_t n_td, double alpha,
                           uint8_t* out, int64_t* n_out, hipStream_t s) {
  const Grid g = grid_of(gp);
  KFMM_REQUIRE(vox && td && out && vox != out, "vox, td or out is NULL, or out aliases vox");
  KFMM_REQUIRE(std::isfinite(alpha) && alpha > 0 && alpha <= 1, "alpha must be in (0, 1]");
  Arena a;
  const int64_t n = g.n();
  int* flag = a.get<int>(n);
  hipLaunchKernelGGL(k_filled_flags, dim3(nblk(n, 256)), dim3(256), 0, s, n, vox, flag);
  int64_t* rank = nullptr;
  const int64_t nf = scan(a, flag, n, rank, s);
  KFMM_REQUIRE(nf > 0, "the design holds no material");
  KFMM_REQUIRE(n_td == nf, "td must hold one value per filled voxel");
  double* mm = a.get<double>(2);
  hipLaunchKernelGGL(k_minmax, dim3(1), dim3(256), 0, s, td, nf, mm);
  double hmm[2];
  KFMM_HIP(hipMemcpyAsync(hmm, mm, sizeof(hmm), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  KFMM_REQUIRE(std::isfinite(hmm[0]) && std::isfinite(hmm[1]), "non-finite topological derivative");
  const int64_t n_keep = std::llround(alpha * (double)n);
  const int64_t n_remove = nf > n_keep ? nf - n_keep : 0;
  int64_t n_pad = 2048;
  while (n_pad < nf) n_pad *= 2;
  uint64_t* key = a.get<uint64_t>(n_pad);
  int* order = a.get<int>(n_pad);
  hipLaunchKernelGGL(k_td_keys, dim3(nblk(nf, 256)), dim3(256), 0, s, nf, td, key, order);
  KFMM_HIP(hipGetLastError());
  sort_keys(key, order, nf, n_pad, s);
  int64_t* lin = a.get<int64_t>(nf);
  hipLaunchKernelGGL(k_rank_lin, dim3(nblk(n, 256)), dim3(256), 0, s, g, flag, rank, lin);
  hipLaunchKernelGGL(k_copy_u8, dim3(nblk(n, 256)), dim3(256), 0, s, n, vox, out);
  if (n_remove > 0)
    hipLaunchKernelGGL(k_remove_lowest, dim3(nblk(n_remove, 256)), dim3(256), 0, s, n_remove, order, lin, out);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));
  if (n_out) *n_out = nf - n_remove;
}

void alg1_coarse_impl(const alg1_grid* gp, const uint8_t* vox, int block, int64_t* n, double* pts, int64_t capacity,
                      hipStream_t s) {
  const Grid g = grid_of(gp);
  const Blocks B = blocks_of(g, block);
  KFMM_REQUIRE(vox && n, "vox or n is NULL");
  Arena a;
  int* full = a.get<int>(B.n());
  hipLaunchKernelGGL(k_block_full, dim3(nblk(B.n(), 128)), dim3(128), 0, s, g, B, vox, full);
  KFMM_HIP(hipGetLastError());
  int64_t* pos = nullptr;
  *n = scan(a, full, B.n(), pos, s);
  if (!pts) return;
  KFMM_REQUIRE(capacity >= *n, "output holds fewer points than there are full blocks");
  hipLaunchKernelGGL(k_block_centres, dim3(nblk(B.n(), 256)), dim3(256), 0, s, B, g.h, full, pos, pts);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));
}

// Shared by refine and expand: full blocks, their scan, the coarse threshold and the refined mask.
struct Refinement {
  Arena a;
  int* full = nullptr;
  int64_t* block_pos = nullptr;
  int64_t n_full = 0;
  uint8_t* refined = nullptr;
  int* fine_flag = nullptr;
  int64_t* fine_pos = nullptr;
  int64_t n_fine = 0;
};

static void refinement(const Grid& g, const Blocks& B, const uint8_t* vox, const double* td_c, int64_t n_c,
                       double C, Refinement& R, hipStream_t s) {
  R.full = R.a.get<int>(B.n());
  hipLaunchKernelGGL(k_block_full, dim3(nblk(B.n(), 128)), dim3(128), 0, s, g, B, vox, R.full);
  KFMM_HIP(hipGetLastError());
  R.n_full = scan(R.a, R.full, B.n(), R.block_pos, s);
  KFMM_REQUIRE(n_c == R.n_full, "td_coarse must hold one value per full block");
  double thr = 0.0;
  if (R.n_full > 0) {
    KFMM_REQUIRE(td_c != nullptr, "td_coarse is NULL");
    double* mm = R.a.get<double>(2);
    hipLaunchKernelGGL(k_minmax, dim3(1), dim3(256), 0, s, td_c, R.n_full, mm);
    double hmm[2];
    KFMM_HIP(hipMemcpyAsync(hmm, mm, sizeof(hmm), hipMemcpyDeviceToHost, s));
    KFMM_HIP(hipStreamSynchronize(s));
    KFMM_REQUIRE(std::isfinite(hmm[0]) && std::isfinite(hmm[1]), "non-finite topological derivative");
    thr = hmm[0] + C * (hmm[1] - hmm[0]);
  }
  R.refined = R.a.get<uint8_t>(B.n());
  hipLaunchKernelGGL(k_block_refine, dim3(nblk(B.n(), 256)), dim3(256), 0, s, B, R.full, R.block_pos, td_c, thr,
                     R.refined);
  R.fine_flag = R.a.get<int>(g.n());
  hipLaunchKernelGGL(k_fine_flags, dim3(nblk(g.n(), 256)), dim3(256), 0, s, g, B, vox, R.refined, R.fine_flag);
  KFMM_HIP(hipGetLastError());
  R.n_fine = scan(R.a, R.fine_flag, g.n(), R.fine_pos, s);
}

void alg1_refine_impl(const alg1_grid* gp, const uint8_t* vox, int block, const double* td_c, int64_t n_c, double C,
                      int64_t* n, double* pts, int64_t capacity, uint8_t* refined_out, hipStream_t s) {
  const Grid g = grid_of(gp);
  const Blocks B = blocks_of(g, block);
  KFMM_REQUIRE(vox && n, "vox or n is NULL");
  KFMM_REQUIRE(std::isfinite(C) && C >= 0 && C <= 1, "C must be in [0, 1]");
  Refinement R;
  refinement(g, B, vox, td_c, n_c, C, R, s);
  *n = R.n_fine;
  if (refined_out) KFMM_HIP(hipMemcpyAsync(refined_out, R.refined, B.n(), hipMemcpyDeviceToDevice, s));
  if (pts) {
    KFMM_REQUIRE(capacity >= R.n_fine, "output holds fewer points than there are refined voxels");
    hipLaunchKernelGGL(k_emit_centres, dim3(nblk(g.n(), 256)), dim3(256), 0, s, g, R.fine_flag, R.fine_pos, pts);
    KFMM_HIP(hipGetLastError());
  }
  KFMM_HIP(hipStreamSynchronize(s));
}

void alg1_expand_impl(const alg1_grid* gp, const uint8_t* vox, int block, const double* td_c, int64_t n_c, double C,
                      const double* td_f, int64_t n_f, double* out, hipStream_t s) {
  const Grid g = grid_of(gp);
  const Blocks B = blocks_of(g, block);
  KFMM_REQUIRE(vox && out, "vox or out is NULL");
  KFMM_REQUIRE(std::isfinite(C) && C >= 0 && C <= 1, "C must be in [0, 1]");
  Refinement R;
  refinement(g, B, vox, td_c, n_c, C, R, s);
  KFMM_REQUIRE(n_f == R.n_fine, "td_fine must hold one value per refined voxel");
  KFMM_REQUIRE(R.n_fine == 0 || td_f != nullptr, "td_fine is NULL");
  int* flag = R.a.get<int>(g.n());
  hipLaunchKernelGGL(k_filled_flags, dim3(nblk(g.n(), 256)), dim3(256), 0, s, g.n(), vox, flag);
  int64_t* rank = nullptr;
  scan(R.a, flag, g.n(), rank, s);
  hipLaunchKernelGGL(k_expand, dim3(nblk(g.n(), 256)), dim3(256), 0, s, g, B, vox, rank, R.refined, R.fine_pos,
                     R.block_pos, td_c, td_f, out);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));
}

void alg1_energy_impl(const double* sig, int64_t n, double K, double G, double* psi, hipStream_t s) {
  KFMM_REQUIRE(psi != nullptr && (n == 0 || sig != nullptr), "sig or psi is NULL");
  const double E = 9.0 * K * G / (3.0 * K + G), nu = (3.0 * K - 2.0 * G) / (2.0 * (3.0 * K + G));
  Arena a;
  double* d = a.get<double>(1);
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, s, sig, n, E, nu, d);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipMemcpyAsync(psi, d, sizeof(double), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
}

}  // namespace kfmm
