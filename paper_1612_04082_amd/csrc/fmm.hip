// KIFMM evaluation of the Kelvin elastostatic boundary integrals on one GPU (Sec. 2.2).
//
// fmm_eval pipeline (all on one stream):
//   permute-in   densities w*a, w*b gathered into tree (Morton) order
//   S2M          sources of every leaf -> displacement at its upward check surface (source kernel U/P)
//   UC2UE        phi_up = r_l * UC2UE * q                                (FP64 MFMA)
//   M2M          level by level: T = M2M_c * phi_up(child); phi_up(parent) = sum over children
//   M2L          qhat(B) += M2L_d * phi_up(A) for V pairs, grouped by offset d over all levels (MFMA)
//   S2L (X)      qhat(B) += r_l * (sources of coarse adjacent leaves at B's downward check surface)
//   DC2DE, L2L   phi_dn = DC2DE * qhat + L2L_c * phi_dn(parent), top-down  (FP64 MFMA)
//   leaf eval    per target leaf: L2T (phi_dn), M2T over W, direct sum over U; result written in the
//                caller's order (U or D kernel for far fields; U+P or D+S near field)
// Coordinates are stored relative to the leaf centre; box-centre offsets are exact dyadic numbers
// (power-of-two root), which keeps FP32 near-field differences accurate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>

#include "../../include/kfmm.h"
#include "common.h"
#include "gemm.h"
#include "operators.h"
#include "plan.h"
#include "tree.h"

namespace kfmm {

// ------------------------------------------------------------------------ process-wide operator cache

static GemmJob upload_job(Arena& a, const GemmCols& cols, hipStream_t s, int tile_cols = kGemmBN,
                          const std::vector<int>* op_rank = nullptr);

// Shared-basis compression of the M2L operators: K_o ~ U C_o U^T with one orthonormal basis U (n x r)
// for every offset o.  U spans the dominant left singular space of [K_1 ... K_316]: the eigenvectors of
// sum_o K_o K_o^T above a relative singular-value cutoff.  The U kernel is even and symmetric, so
// K_{-o} = K_o^T and the right singular space is the same; C_{-o} = C_o^T.
struct CompressedM2L {
  double tol = 0;
  int r = 0, NCr = 0;
  double* Ut64 = nullptr;  // NCr x NC row-major (row k = k-th basis vector, rows >= r zero)
  double* DU64 = nullptr;  // DC2DE * U, NC x NCr row-major: downward equivalent densities from q~ directly
  float* U32 = nullptr;    // U, NC x NCr row-major (FP32 translations: qhat = U q~)
  float* G32 = nullptr;    // U^T fu2, NCr x NC row-major (FP32 translations: phi~ = U^T UC2UE qhat = G (fu1 qhat))
  float* Gv32 = nullptr;   // U^T vs = G diag(sigma) (split FP16: phi~ = Gv (diag(inv_sig) fu1 qhat))
  uint16_t* Gv_h3 = nullptr;
  float* Gv_h3_scale = nullptr;
  // U^T UC2UE (NCr x NC): phi~ straight from the upward check potentials in one product (split FP16); the
  // pseudo-inverse's large entries 1/sigma sit on density modes that the far field barely sees, and
  // projected onto the M2L basis they stay of the size of the result
  float* Mu32 = nullptr;
  uint16_t* Mu_h3 = nullptr;
  float* Mu_h3_scale = nullptr;
  float* Ut32 = nullptr;   // NCr x NC
  float* C32 = nullptr;    // 316 x NCr x NCr row-major
  // Per-offset rank (split FP16): C_o truncated to its leading r_o x r_o block (the basis is ordered by the
  // singular values of all offsets together, and a far offset needs fewer of its vectors), r_o the smallest
  // multiple of 32 whose dropped entries have a Frobenius norm below a third of the basis cutoff (absolute,
  // like the cutoff itself).  Crk32 holds operator o in an NCr^2 slot as an r_o x r_o row-major block, the rest
  // of the slot zero; the M2L tiles carry r_o (see k_gemm_h3).
  std::vector<int> rank_o;  // per compact offset
  float* Crk32 = nullptr;
  double* C64 = nullptr;     // 316 x NCr x NCr row-major, FP64
  double* Crk64 = nullptr;   // the same truncated layout as Crk32 in FP64 (KFMM_FP64), made on first use
  uint16_t* Crk_h3 = nullptr;  // Crk32 split, made on first use
  float* Crk_h3_scale = nullptr;
  uint16_t* U_h3 = nullptr;     // U32 split likewise (one operator)
  float* U_h3_scale = nullptr;
  // U and fd1 U (two NC x NCr operators, split FP16): the downward check potential of a box with children,
  // and the first pseudo-inverse factor already applied for a leaf (whose check potential nothing else reads)
  uint16_t* UF_h3 = nullptr;
  float* UF_h3_scale = nullptr;
};

struct DeviceOps {
  int device = -1;
  int p = 0, n = 0, NC = 0, n_eq = 0;
  double *uc2ue = nullptr, *dc2de = nullptr, *m2m = nullptr, *l2l = nullptr, *m2l64 = nullptr;
  // FP32 translations: factored pseudo-inverses (UC2UE = fu2 fu1, DC2DE = fd2 fd1) and the M2M / L2L
  // translations on check potentials (8 each)
  float *fu1 = nullptr, *fu2 = nullptr, *fd1 = nullptr, *fd2 = nullptr, *m2mq32 = nullptr, *l2lq32 = nullptr;
  double* fu2t_64 = nullptr;  // fu2 transposed, FP64 (rows = columns of fu2), for U^T fu2
  // fu2 = vs diag(inv_sig), fd2 = us diag(inv_sig): the orthogonal parts (FP32) and 1/sigma (host, device)
  float *vs32 = nullptr, *us32 = nullptr, *inv_sig32 = nullptr;
  std::vector<double> inv_sig;
  uint16_t *vs_h3 = nullptr, *us_h3 = nullptr;  // split-FP16 copies (one scale each), made on first use
  float *vs_h3_scale = nullptr, *us_h3_scale = nullptr;
  float* m2l32 = nullptr;
  uint16_t* m2l_h3 = nullptr;     // m2l64 split into FP16 high / low parts, made on first use
  float* m2l_h3_scale = nullptr;  // power-of-two scale per operator
  // split-FP16 copies (one scale per operator) of M2M_q, L2L_q (8 each) and of the orthogonal pseudo-inverse
  // factors fu1, fd1, made on first use
  uint16_t *m2mq_h3 = nullptr, *l2lq_h3 = nullptr, *fu1_h3 = nullptr, *fd1_h3 = nullptr;
  float *m2mq_h3_scale = nullptr, *l2lq_h3_scale = nullptr, *fu1_h3_scale = nullptr, *fd1_h3_scale = nullptr;
  // fd1 and the transposed L2L_q in FP64, and the 16 operators [L2L_q | fd1 L2L_q] (FP32 and split FP16):
  // an L2L into a leaf applies the first factor of its DC2DE at once (made on first use)
  double *fd1_64 = nullptr, *l2lqT64 = nullptr;
  float* l2lq_fold32 = nullptr;
  uint16_t* l2lq_fold_h3 = nullptr;
  float* l2lq_fold_h3_scale = nullptr;
  std::mutex h3_mutex;
  double* surf = nullptr;  // n_eq x 3
  std::vector<int> m2l_index;
  std::map<double, std::shared_ptr<CompressedM2L>> comp;  // by relative cutoff
  // periodic cells, made on first use: the far-image operator T of the root (NC x NC, FP64), the same on
  // check potentials T UC2UE (FP32) and onto the downward density DC2DE T (FP64), and the second-moment rows
  // of the upward equivalent density (6 x NC, unit half-width) on phi_up and on qhat_up (times UC2UE)
  double* per_far64 = nullptr;
  float* per_farq32 = nullptr;
  double *per_fardn64 = nullptr, *per_mom_phi = nullptr, *per_mom_q = nullptr;
  std::mutex per_mutex;
  Arena arena;
};

static std::mutex g_ops_mutex;
static std::map<std::tuple<int, int, double, double, double>, std::shared_ptr<DeviceOps>> g_ops;

static std::vector<double> pad_square(const std::vector<double>& M, int n, int NC) {
  std::vector<double> out((size_t)NC * NC, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[(size_t)i * NC + j] = M[(size_t)i * n + j];
  return out;
}

static std::shared_ptr<DeviceOps> get_ops(int p, const Elastic& el, double eps, int precision, hipStream_t s) {
  int dev = 0;
  KFMM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_ops_mutex);
  auto key = std::make_tuple(dev, p, el.nu, el.G, eps);
  std::shared_ptr<DeviceOps> d;
  auto it = g_ops.find(key);
  if (it != g_ops.end()) d = it->second;
  if (!d) {
    Operators op = build_operators(p, el, eps);
    d = std::make_shared<DeviceOps>();
    d->device = dev;
    d->p = p;
    d->n = op.n;
    d->n_eq = op.n_eq;
    d->NC = gemm_pad(op.n);
    d->m2l_index = op.m2l_index;
    const int NC = d->NC;
    auto up = [&](const std::vector<double>& v) {
      double* ptr = d->arena.get<double>(v.size());
      KFMM_HIP(hipMemcpy(ptr, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
      return ptr;
    };
    std::vector<double> cat = pad_square(op.uc2ue, op.n, NC);
    d->uc2ue = up(cat);
    cat = pad_square(op.dc2de, op.n, NC);
    d->dc2de = up(cat);
    cat.clear();
    for (int c = 0; c < 8; ++c) {
      auto v = pad_square(op.m2m[c], op.n, NC);
      cat.insert(cat.end(), v.begin(), v.end());
    }
    d->m2m = up(cat);
    cat.clear();
    for (int c = 0; c < 8; ++c) {
      auto v = pad_square(op.l2l[c], op.n, NC);
      cat.insert(cat.end(), v.begin(), v.end());
    }
    d->l2l = up(cat);
    d->surf = up(op.surf);
    auto up32 = [&](const std::vector<double>& v) {
      std::vector<float> f(v.begin(), v.end());
      float* ptr = d->arena.get<float>(f.size());
      KFMM_HIP(hipMemcpy(ptr, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
      return ptr;
    };
    auto cat8 = [&](const std::vector<std::vector<double>>& m) {
      std::vector<double> all;
      for (int c = 0; c < 8; ++c) {
        auto v = pad_square(m[c], op.n, NC);
        all.insert(all.end(), v.begin(), v.end());
      }
      return all;
    };
    d->m2mq32 = up32(cat8(op.m2m_q));
    d->l2lq32 = up32(cat8(op.l2l_q));
    d->fu1 = up32(pad_square(op.fu1, op.n, NC));
    d->fu2 = up32(pad_square(op.fu2, op.n, NC));
    d->fd1 = up32(pad_square(op.fd1, op.n, NC));
    d->fd1_64 = up(pad_square(op.fd1, op.n, NC));
    {
      std::vector<double> lt = cat8(op.l2l_q), tr(lt.size());
      for (int c = 0; c < 8; ++c)
        for (int i = 0; i < NC; ++i)
          for (int j = 0; j < NC; ++j) tr[((size_t)c * NC + j) * NC + i] = lt[((size_t)c * NC + i) * NC + j];
      d->l2lqT64 = up(tr);
    }
    d->fd2 = up32(pad_square(op.fd2, op.n, NC));
    d->vs32 = up32(pad_square(op.vs, op.n, NC));
    d->us32 = up32(pad_square(op.us, op.n, NC));
    d->inv_sig.assign(NC, 0.0);
    for (int j = 0; j < op.n; ++j) d->inv_sig[j] = op.inv_sig[j];
    d->inv_sig32 = up32(d->inv_sig);
    {
      std::vector<double> f = pad_square(op.fu2, op.n, NC), ft((size_t)NC * NC);
      for (int i = 0; i < NC; ++i)
        for (int j = 0; j < NC; ++j) ft[(size_t)j * NC + i] = f[(size_t)i * NC + j];
      d->fu2t_64 = up(ft);
    }
    // M2L operators in the requested precisions are uploaded lazily below
    std::vector<double> m2l_all;
    m2l_all.reserve(op.m2l.size() * (size_t)NC * NC);
    for (auto& m : op.m2l) {
      auto v = pad_square(m, op.n, NC);
      m2l_all.insert(m2l_all.end(), v.begin(), v.end());
    }
    // keep host copy only as long as needed: convert now for every precision
    d->m2l64 = up(m2l_all);
    {
      std::vector<float> f(m2l_all.size());
      for (size_t i = 0; i < f.size(); ++i) f[i] = (float)m2l_all[i];
      d->m2l32 = d->arena.get<float>(f.size());
      KFMM_HIP(hipMemcpy(d->m2l32, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    g_ops[key] = d;
  }
  return d;
}

// ------------------------------------------------------------------------------------ small kernels

__device__ __forceinline__ void box_offset(const int* level, const int* ix, const int* iy, const int* iz,
                                           const int* geom, const double* root_R, int A, int B, double* o) {
  int la = level[A], lb = level[B];
  int L = la > lb ? la : lb;
  double R = root_R[geom[B]];
  double sc = ldexp(R, -L);
  long na[3] = {ix[A], iy[A], iz[A]}, nb[3] = {ix[B], iy[B], iz[B]};
  for (int d = 0; d < 3; ++d) {
    long num = ((2 * na[d] + 1) << (L - la)) - ((2 * nb[d] + 1) << (L - lb));
    o[d] = (double)num * sc;
  }
}

__device__ __forceinline__ double box_half(const int* level, const int* geom, const double* root_R, int B) {
  return ldexp(root_R[geom[B]], -level[B]);
}

// Adds the lattice shift of a list entry (code (sx+1)+3(sy+1)+9(sz+1), periodic cells) in cell sides.
__device__ __forceinline__ void add_lattice_shift(double* o, int code, const int* geom, const double* root_R, int B) {
  if (code == kNoShift) return;
  const double side = 2.0 * root_R[geom[B]];
  o[0] += (code % 3 - 1) * side;
  o[1] += ((code / 3) % 3 - 1) * side;
  o[2] += (code / 9 - 1) * side;
}

__device__ __forceinline__ void box_center(const int* level, const int* ix, const int* iy, const int* iz,
                                           const int* geom, const double* root_c, const double* root_R, int B,
                                           double* c) {
  int g = geom[B];
  double R = root_R[g];
  double r = ldexp(R, -level[B]);
  int q[3] = {ix[B], iy[B], iz[B]};
  for (int d = 0; d < 3; ++d) c[d] = root_c[3 * g + d] - R + (2.0 * q[d] + 1.0) * r;
}

// Local (leaf-relative) coordinates and normals of the sorted points.
template <typename T>
__global__ void k_local_points(int64_t n, const int* perm, const int* leaf_of, const double* xyz, const double* nrm,
                               const double* w, TreeView tv, T* pos4, T* nrm4, double* w_sorted) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = perm[i];
  int leaf = leaf_of[i];
  double c[3];
  box_center(tv.level, tv.ix, tv.iy, tv.iz, tv.geom, tv.root_c, tv.root_R, leaf, c);
  for (int d = 0; d < 3; ++d) pos4[4 * i + d] = (T)(xyz[3 * o + d] - c[d]);
  pos4[4 * i + 3] = T(0);
  if (nrm4) {
    for (int d = 0; d < 3; ++d) nrm4[4 * i + d] = nrm ? (T)nrm[3 * o + d] : T(0);
    nrm4[4 * i + 3] = T(0);
  }
  if (w_sorted) w_sorted[i] = w ? w[o] : 1.0;
}

template <typename T>
__global__ void k_permute_in(int64_t n, const int* perm, const double* w_sorted, const double* a, const double* b,
                             T* dens8) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = perm[i];
  double w = w_sorted[i];
  for (int d = 0; d < 3; ++d) {
    dens8[8 * i + d] = a ? (T)(w * a[3 * o + d]) : T(0);
    dens8[8 * i + 4 + d] = b ? (T)(w * b[3 * o + d]) : T(0);
  }
  dens8[8 * i + 3] = T(0);
  dens8[8 * i + 7] = T(0);
}

template <typename TI, typename TO>
__global__ void k_convert(int64_t n, const TI* in, TO* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (TO)in[i];
}

template <typename T>
__global__ void k_fill_zero(int64_t n, T* p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// dst(boxes[i]) += src(i): the X-list check potentials (compact rows) added to qhat
template <typename T>
__global__ __launch_bounds__(256) void k_add_rows(const int* __restrict__ boxes, const T* __restrict__ src,
                                                  T* __restrict__ dst, int NC) {
  const int i = blockIdx.x, B = boxes[i];
  for (int c = threadIdx.x; c < NC; c += blockDim.x) dst[(size_t)B * NC + c] += src[(size_t)i * NC + c];
}

// Sums of NC-vectors in a fixed order (FP64 accumulation), 16 bytes per lane and per load, four loads in
// flight.  NC is a multiple of 32.
template <typename TS>
struct Vec16 {
  static constexpr int V = 16 / sizeof(TS);
  TS v[V];
};

template <typename TS>
__device__ __forceinline__ Vec16<TS> load16(const TS* p) {
  return *(const Vec16<TS>*)p;
}

// out(box) = sum of the box's M2L slots in list order
template <typename TS, typename TO>
__global__ __launch_bounds__(256) void k_slot_reduce(const int* __restrict__ boxes, const int* __restrict__ off,
                                                     const int* __restrict__ idx, const TS* __restrict__ slots,
                                                     TO* __restrict__ out, int NC) {
  constexpr int V = Vec16<TS>::V;
  const int i = blockIdx.x;
  const int B = boxes[i], k0 = off[i], k1 = off[i + 1];
  for (int c = threadIdx.x * V; c < NC; c += blockDim.x * V) {
    double acc[V] = {};
    int k = k0;
    for (; k + 4 <= k1; k += 4) {
      Vec16<TS> v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = load16(slots + (size_t)idx[k + u] * NC + c);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] += (double)v[u].v[e];
    }
    for (; k < k1; ++k) {
      Vec16<TS> v = load16(slots + (size_t)idx[k] * NC + c);
#pragma unroll
      for (int e = 0; e < V; ++e) acc[e] += (double)v.v[e];
    }
#pragma unroll
    for (int e = 0; e < V; ++e) out[(size_t)B * NC + c + e] = (TO)acc[e];
  }
}

// phi_up(parent) = sum over children with sources of T(child), children in order.  With split != nullptr
// (FP32 only) the parent's row is also written in split-FP16 form (see split_h3: power-of-two scale from
// the row's largest magnitude, [hi 8 | lo 8] chunks), for the split-FP16 products of the next level.
template <typename T>
__global__ __launch_bounds__(256) void k_m2m_reduce(const int* parents, int n_par, const int* child_first,
                                                    const int* child_count, const int* src_b, const int* src_e,
                                                    const T* __restrict__ tmp, T* __restrict__ phi, int NC,
                                                    uint16_t* __restrict__ split = nullptr,
                                                    float* __restrict__ split_scale = nullptr,
                                                    const signed char* __restrict__ pair_sh = nullptr) {
  constexpr int V = Vec16<T>::V;
  int pi = blockIdx.x;
  if (pi >= n_par) return;
  int P = parents[pi];
  int f = child_first[P], nc = child_count[P];
  float m = 0.0f;
  for (int c = threadIdx.x * V; c < NC; c += blockDim.x * V) {
    double acc[V] = {};
    for (int k = 0; k < nc; ++k) {
      int C = f + k;
      if (src_e[C] > src_b[C]) {
        Vec16<T> v = load16(tmp + (size_t)C * NC + c);
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] += (double)v.v[e];
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      phi[(size_t)P * NC + c + e] = (T)acc[e];
      m = fmaxf(m, fabsf((float)(T)acc[e]));
    }
  }
  if constexpr (sizeof(T) == 4) {
    if (!split) return;
    // block maximum: waves by shuffles, then across the (at most 4) waves through LDS
    __shared__ float wmax[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    m = wmax[0];
    for (int w = 1; w < (int)(blockDim.x + 63) / 64; ++w) m = fmaxf(m, wmax[w]);
    int e2 = 0;
    float sc = 1.0f;
    if (m > 0.0f && m < INFINITY) {
      frexpf(m, &e2);  // m = f 2^e2, f in [0.5, 1): scale to put m in [2^14, 2^15)
      sc = ldexpf(1.0f, max(-126, min(127, e2 - 15)));
    }
    if (threadIdx.x == 0) split_scale[P] = sc;
    const float inv = 1.0f / sc;
    _Float16* d = (_Float16*)split + (size_t)P * 2 * NC;
    for (int c = threadIdx.x * V; c < NC; c += blockDim.x * V) {  // 4 values: half of one 8-value chunk
      const float* x = (const float*)phi + (size_t)P * NC + c;     // this thread's own writes
      _Float16* hi = d + 16 * (c / 8) + (c % 8);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const float v = x[e] * inv;
        const _Float16 h = (_Float16)v;
        hi[e] = h;
        hi[8 + e] = (_Float16)(v - (float)h);
      }
    }
  }
}

// threads for one vector sum over NC entries of type T (16 bytes per lane)
template <typename T>
static int reduce_block(int NC) {
  return std::min(256, round_up(NC / Vec16<T>::V, 64));
}

static std::shared_ptr<CompressedM2L> get_compressed(DeviceOps& d, double tol, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_ops_mutex);
  auto it = d.comp.find(tol);
  if (it != d.comp.end()) return it->second;
  const int NC = d.NC, n = d.n, nops = 316;
  auto c = std::make_shared<CompressedM2L>();
  c->tol = tol;
  Arena tmp;
  // Gram matrix G = sum_o K_o K_o^T: column j of K_o K_o^T is K_o times row j of K_o (one launch per o,
  // fixed order, so the basis is reproducible)
  double* gram = tmp.get<double>((size_t)NC * NC);
  KFMM_HIP(hipMemsetAsync(gram, 0, sizeof(double) * NC * NC, s));
  for (int o = 0; o < nops; ++o) {
    GemmCols cols;
    for (int j = 0; j < n; ++j) cols.add(o, o * NC + j, j);
    Arena ja;
    GemmJob job = upload_job(ja, cols, s, kGemmBN);
    gemm_f64(job, d.m2l64, GemmDims::Sq(NC), d.m2l64, gram, kAdd, s);
    KFMM_HIP(hipStreamSynchronize(s));
  }
  std::vector<double> hg((size_t)NC * NC), G((size_t)n * n);
  KFMM_HIP(hipMemcpy(hg.data(), gram, sizeof(double) * NC * NC, hipMemcpyDeviceToHost));
  for (int j = 0; j < n; ++j)  // stored by columns; G is symmetric
    for (int i = 0; i < n; ++i) G[(size_t)i * n + j] = 0.5 * (hg[(size_t)j * NC + i] + hg[(size_t)i * NC + j]);
  std::vector<double> lam, vecs;
  sym_eig_psd_cached(G, n, "m2l_gram", lam, vecs);
  int r = 0;
  while (r < n && lam[r] > 0 && std::sqrt(lam[r] / lam[0]) > tol) ++r;
  r = std::max(r, 1);
  // the contractions run on r padded to the GEMM granularity anyway: keep that many basis vectors
  c->NCr = gemm_pad(r);
  r = std::min(n, c->NCr);
  c->r = r;
  const int NCr = c->NCr;
  std::vector<double> Ut((size_t)NCr * NC, 0.0);
  for (int k = 0; k < r; ++k)
    for (int i = 0; i < n; ++i) Ut[(size_t)k * NC + i] = vecs[(size_t)k * n + i];
  c->Ut64 = d.arena.get<double>(Ut.size());
  KFMM_HIP(hipMemcpy(c->Ut64, Ut.data(), sizeof(double) * Ut.size(), hipMemcpyHostToDevice));
  std::vector<float> Ut32(Ut.begin(), Ut.end());
  c->Ut32 = d.arena.get<float>(Ut32.size());
  KFMM_HIP(hipMemcpy(c->Ut32, Ut32.data(), sizeof(float) * Ut32.size(), hipMemcpyHostToDevice));
  // T_o = K_o U (columns j < r), then C_o(:, j) = U^T T_o(:, j) written as row j of C_{-o}
  double* T = tmp.get<double>((size_t)nops * r * NC);
  double* C64 = c->C64 = d.arena.get<double>((size_t)nops * NCr * NCr);
  KFMM_HIP(hipMemsetAsync(C64, 0, sizeof(double) * nops * NCr * NCr, s));
  std::vector<int> neg(nops, -1);
  for (int k343 = 0; k343 < 343; ++k343)
    if (d.m2l_index[k343] >= 0) neg[d.m2l_index[k343]] = d.m2l_index[342 - k343];
  {
    GemmCols c1, c2;
    for (int o = 0; o < nops; ++o)
      for (int j = 0; j < r; ++j) {
        c1.add(o, j, o * r + j);
        c2.add(0, o * r + j, neg[o] * NCr + j);
      }
    GemmJob j1 = upload_job(tmp, c1, s, kGemmBN), j2 = upload_job(tmp, c2, s, kGemmBN);
    gemm_f64(j1, d.m2l64, GemmDims::Sq(NC), c->Ut64, T, kStore, s);
    gemm_f64(j2, c->Ut64, GemmDims{NCr, NC, NC, NCr}, T, C64, kStore, s);
  }
  {  // per-offset ranks and the truncated operators
    std::vector<double> hc((size_t)nops * NCr * NCr);
    KFMM_HIP(hipStreamSynchronize(s));
    KFMM_HIP(hipMemcpy(hc.data(), C64, sizeof(double) * hc.size(), hipMemcpyDeviceToHost));
    const double drop2 = std::pow(tol / 3.0 * std::sqrt(lam[0]), 2);
    c->rank_o.assign(nops, NCr);
    std::vector<float> f((size_t)nops * NCr * NCr, 0.0f);
    auto ranks = [&](int o0, int o1) {
      for (int o = o0; o < o1; ++o) {
        const double* C = hc.data() + (size_t)o * NCr * NCr;
        double tot = 0;
        for (size_t i = 0; i < (size_t)NCr * NCr; ++i) tot += C[i] * C[i];
        int m = 64;
        for (; m < NCr; m += 32) {
          double kept = 0;
          for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) kept += C[(size_t)i * NCr + j] * C[(size_t)i * NCr + j];
          if (tot - kept <= drop2) break;
        }
        m = std::min(m, NCr);
        c->rank_o[o] = m;
        float* F = f.data() + (size_t)o * NCr * NCr;
        for (int i = 0; i < m; ++i)
          for (int j = 0; j < m; ++j) F[(size_t)i * m + j] = (float)C[(size_t)i * NCr + j];
      }
    };
    const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int t = 0; t < nth; ++t) pool.emplace_back(ranks, nops * t / nth, nops * (t + 1) / nth);
    for (auto& th : pool) th.join();
    c->Crk32 = d.arena.get<float>(f.size());
    KFMM_HIP(hipMemcpy(c->Crk32, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice));
  }
  // DC2DE * U (columns k < r): rows k of Y = DC2DE u_k, transposed on the host
  {
    GemmCols cd;
    for (int k = 0; k < r; ++k) cd.add(0, k, k);
    GemmJob jd = upload_job(tmp, cd, s, kGemmBN);
    double* Y = tmp.get<double>((size_t)NCr * NC);
    KFMM_HIP(hipMemsetAsync(Y, 0, sizeof(double) * NCr * NC, s));
    gemm_f64(jd, d.dc2de, GemmDims::Sq(NC), c->Ut64, Y, kStore, s);
    std::vector<double> hy((size_t)NCr * NC), du((size_t)NC * NCr, 0.0);
    KFMM_HIP(hipMemcpyAsync(hy.data(), Y, sizeof(double) * hy.size(), hipMemcpyDeviceToHost, s));
    KFMM_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < r; ++k)
      for (int i = 0; i < NC; ++i) du[(size_t)i * NCr + k] = hy[(size_t)k * NC + i];
    c->DU64 = d.arena.get<double>(du.size());
    KFMM_HIP(hipMemcpy(c->DU64, du.data(), sizeof(double) * du.size(), hipMemcpyHostToDevice));
  }
  {  // G = U^T fu2 (NCr x NC): column c = U^T (fu2 e_c) from the rows of fu2^T, transposed on the host
    GemmCols cg;
    for (int c2 = 0; c2 < NC; ++c2) cg.add(0, c2, c2);
    GemmJob jg = upload_job(tmp, cg, s, kGemmBN);
    double* Yg = tmp.get<double>((size_t)NC * NCr);
    gemm_f64(jg, c->Ut64, GemmDims{NCr, NC, NC, NCr}, d.fu2t_64, Yg, kStore, s);
    std::vector<double> hg((size_t)NC * NCr);
    KFMM_HIP(hipMemcpyAsync(hg.data(), Yg, sizeof(double) * hg.size(), hipMemcpyDeviceToHost, s));
    KFMM_HIP(hipStreamSynchronize(s));
    std::vector<float> g32((size_t)NCr * NC, 0.0f), gv32((size_t)NCr * NC, 0.0f);
    for (int c2 = 0; c2 < NC; ++c2)
      for (int k = 0; k < NCr; ++k) {
        const double gkc = hg[(size_t)c2 * NCr + k];
        g32[(size_t)k * NC + c2] = (float)gkc;
        if (d.inv_sig[c2] > 0) gv32[(size_t)k * NC + c2] = (float)(gkc / d.inv_sig[c2]);
      }
    c->G32 = d.arena.get<float>(g32.size());
    KFMM_HIP(hipMemcpy(c->G32, g32.data(), sizeof(float) * g32.size(), hipMemcpyHostToDevice));
    c->Gv32 = d.arena.get<float>(gv32.size());
    KFMM_HIP(hipMemcpy(c->Gv32, gv32.data(), sizeof(float) * gv32.size(), hipMemcpyHostToDevice));
  }
  {  // Mu = U^T UC2UE (NCr x NC): column c = U^T (UC2UE e_c), from the rows of UC2UE^T
    std::vector<double> h((size_t)NC * NC), ht((size_t)NC * NC);
    KFMM_HIP(hipMemcpy(h.data(), d.uc2ue, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < NC; ++i)
      for (int j = 0; j < NC; ++j) ht[(size_t)j * NC + i] = h[(size_t)i * NC + j];
    double* uct = tmp.get<double>(ht.size());
    KFMM_HIP(hipMemcpy(uct, ht.data(), sizeof(double) * ht.size(), hipMemcpyHostToDevice));
    GemmCols cm;
    for (int c2 = 0; c2 < NC; ++c2) cm.add(0, c2, c2);
    GemmJob jm = upload_job(tmp, cm, s, kGemmBN);
    double* Ym = tmp.get<double>((size_t)NC * NCr);
    gemm_f64(jm, c->Ut64, GemmDims{NCr, NC, NC, NCr}, uct, Ym, kStore, s);
    std::vector<double> hm((size_t)NC * NCr);
    KFMM_HIP(hipMemcpyAsync(hm.data(), Ym, sizeof(double) * hm.size(), hipMemcpyDeviceToHost, s));
    KFMM_HIP(hipStreamSynchronize(s));
    std::vector<float> m32((size_t)NCr * NC, 0.0f);
    for (int c2 = 0; c2 < NC; ++c2)
      for (int k = 0; k < NCr; ++k) m32[(size_t)k * NC + c2] = (float)hm[(size_t)c2 * NCr + k];
    c->Mu32 = d.arena.get<float>(m32.size());
    KFMM_HIP(hipMemcpy(c->Mu32, m32.data(), sizeof(float) * m32.size(), hipMemcpyHostToDevice));
  }
  {  // U itself (NC x NCr, column k = k-th basis vector) for the FP32 translations
    std::vector<float> u32((size_t)NC * NCr, 0.0f);
    for (int k = 0; k < r; ++k)
      for (int i = 0; i < NC; ++i) u32[(size_t)i * NCr + k] = (float)Ut[(size_t)k * NC + i];
    c->U32 = d.arena.get<float>(u32.size());
    KFMM_HIP(hipMemcpy(c->U32, u32.data(), sizeof(float) * u32.size(), hipMemcpyHostToDevice));
  }
  c->C32 = d.arena.get<float>((size_t)nops * NCr * NCr);
  const int64_t nc = (int64_t)nops * NCr * NCr;
  hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, nc,
                     (const double*)C64, c->C32);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));
  d.comp[tol] = c;
  return c;
}

// Operators of the folded downward pass (split FP16, compressed M2L): the 16 L2L operators [L2L_q | fd1 L2L_q]
// and the two [U | fd1 U], products in FP64 on the device, rounded to FP32 and split; made once per device
// and basis.
static void ensure_fold_ops(DeviceOps& d, CompressedM2L* c, hipStream_t s) {
  std::lock_guard<std::mutex> lock(d.h3_mutex);
  const int NC = d.NC;
  const int64_t sq = (int64_t)NC * NC;
  Arena tmp;
  // fd1 applied to n NC-vectors stored as rows; row j of the result is fd1 times row j of the input
  auto fd1_rows = [&](const double* rows, int n) {
    GemmCols cols;
    for (int j = 0; j < n; ++j) cols.add(0, j, j);
    GemmJob job = upload_job(tmp, cols, s, kGemmBN);
    double* Y = tmp.get<double>((size_t)n * NC);
    gemm_f64(job, d.fd1_64, GemmDims::Sq(NC), rows, Y, kStore, s);
    std::vector<double> h((size_t)n * NC);
    KFMM_HIP(hipStreamSynchronize(s));
    KFMM_HIP(hipMemcpy(h.data(), Y, sizeof(double) * h.size(), hipMemcpyDeviceToHost));
    return h;
  };
  if (!d.l2lq_fold32) {
    // rows of L2L_q[c]^T are its columns: row c NC + j of h is column j of fd1 L2L_q[c]
    const std::vector<double> h = fd1_rows(d.l2lqT64, 8 * NC);
    std::vector<float> f((size_t)8 * sq);
    for (int c2 = 0; c2 < 8; ++c2)
      for (int j = 0; j < NC; ++j)
        for (int i = 0; i < NC; ++i)
          f[(size_t)c2 * sq + (size_t)i * NC + j] = (float)h[((size_t)c2 * NC + j) * NC + i];
    d.l2lq_fold32 = d.arena.get<float>((size_t)16 * sq);
    KFMM_HIP(hipMemcpy(d.l2lq_fold32, d.l2lq32, sizeof(float) * 8 * sq, hipMemcpyDeviceToDevice));
    KFMM_HIP(hipMemcpy(d.l2lq_fold32 + 8 * sq, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice));
    d.l2lq_fold_h3 = d.arena.get<uint16_t>((size_t)16 * 2 * sq);
    d.l2lq_fold_h3_scale = d.arena.get<float>(16);
    split_h3(d.l2lq_fold32, 16, sq, sq, d.l2lq_fold_h3, d.l2lq_fold_h3_scale, s);
  }
  if (!c->UF_h3) {
    const int NCr = c->NCr;
    const int64_t len = (int64_t)NC * NCr;
    const std::vector<double> h = fd1_rows(c->Ut64, NCr);  // row k: fd1 u_k (zero past the rank)
    std::vector<float> f((size_t)len);
    for (int k = 0; k < NCr; ++k)
      for (int i = 0; i < NC; ++i) f[(size_t)i * NCr + k] = (float)h[(size_t)k * NC + i];
    float* uf = tmp.get<float>((size_t)2 * len);
    KFMM_HIP(hipMemcpy(uf, c->U32, sizeof(float) * len, hipMemcpyDeviceToDevice));
    KFMM_HIP(hipMemcpy(uf + len, f.data(), sizeof(float) * len, hipMemcpyHostToDevice));
    c->UF_h3 = d.arena.get<uint16_t>((size_t)2 * 2 * len);
    c->UF_h3_scale = d.arena.get<float>(2);
    split_h3(uf, 2, len, len, c->UF_h3, c->UF_h3_scale, s);
  }
  KFMM_HIP(hipStreamSynchronize(s));
}

// The per-offset truncated operators in FP64 (KFMM_FP64 with the compressed M2L), made once per device and basis.
static void ensure_rank64(DeviceOps& d, CompressedM2L* c, hipStream_t s) {
  std::lock_guard<std::mutex> lock(d.h3_mutex);
  if (c->Crk64) return;
  const int nops = 316, NCr = c->NCr;
  const size_t sq = (size_t)NCr * NCr;
  std::vector<double> hc((size_t)nops * sq), f((size_t)nops * sq, 0.0);
  KFMM_HIP(hipStreamSynchronize(s));
  KFMM_HIP(hipMemcpy(hc.data(), c->C64, sizeof(double) * hc.size(), hipMemcpyDeviceToHost));
  for (int o = 0; o < nops; ++o) {
    const int m = c->rank_o[o];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) f[o * sq + (size_t)i * m + j] = hc[o * sq + (size_t)i * NCr + j];
  }
  c->Crk64 = d.arena.get<double>(f.size());
  KFMM_HIP(hipMemcpy(c->Crk64, f.data(), sizeof(double) * f.size(), hipMemcpyHostToDevice));
}

// Split-FP16 copies of the M2L operators (dense, or the compressed C_o of c), made once per device.
static void ensure_split_ops(DeviceOps& d, CompressedM2L* c, hipStream_t s) {
  std::lock_guard<std::mutex> lock(d.h3_mutex);
  const int nops = 316;
  const int64_t sq = (int64_t)d.NC * d.NC;
  auto split_set = [&](const float* src, int n, int64_t len, uint16_t*& dst, float*& sc) {
    dst = d.arena.get<uint16_t>((size_t)n * 2 * len);
    sc = d.arena.get<float>(n);
    split_h3(src, n, len, len, dst, sc, s);
  };
  if (!d.m2mq_h3) {
    split_set(d.vs32, 1, sq, d.vs_h3, d.vs_h3_scale);
    split_set(d.us32, 1, sq, d.us_h3, d.us_h3_scale);
    split_set(d.m2mq32, 8, sq, d.m2mq_h3, d.m2mq_h3_scale);
    split_set(d.l2lq32, 8, sq, d.l2lq_h3, d.l2lq_h3_scale);
    split_set(d.fu1, 1, sq, d.fu1_h3, d.fu1_h3_scale);
    split_set(d.fd1, 1, sq, d.fd1_h3, d.fd1_h3_scale);
  }
  if (c) {
    if (c->Crk_h3) {
      KFMM_HIP(hipStreamSynchronize(s));
      return;
    }
    split_set(c->U32, 1, (int64_t)d.NC * c->NCr, c->U_h3, c->U_h3_scale);
    split_set(c->Gv32, 1, (int64_t)c->NCr * d.NC, c->Gv_h3, c->Gv_h3_scale);
    split_set(c->Mu32, 1, (int64_t)c->NCr * d.NC, c->Mu_h3, c->Mu_h3_scale);
    const int64_t len = (int64_t)c->NCr * c->NCr;
    c->Crk_h3 = d.arena.get<uint16_t>((size_t)nops * 2 * len);
    c->Crk_h3_scale = d.arena.get<float>(nops);
    split_h3(c->Crk32, nops, len, len, c->Crk_h3, c->Crk_h3_scale, s);
  } else if (!d.m2l_h3) {
    const int64_t len = (int64_t)d.NC * d.NC;
    d.m2l_h3 = d.arena.get<uint16_t>((size_t)nops * 2 * len);
    d.m2l_h3_scale = d.arena.get<float>(nops);
    split_h3(d.m2l64, nops, len, len, d.m2l_h3, d.m2l_h3_scale, s);
  }
  KFMM_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ check-surface evaluations (S2M, X)

constexpr int kStage = 256;  // points staged in LDS per round

// One source point into LDS for the displacement kernels: position (plus the box offset o), normal, and the
// densities with the kernel prefactors folded in: (cU w a, n . cP w b, cP w b, 0) (see disp_pair_f).
template <typename T>
__device__ __forceinline__ void stage_source(T* p, T* n, T* dd, const double* o, const T* __restrict__ spos4,
                                             const T* __restrict__ snrm4, const T* __restrict__ dens8, int64_t g,
                                             const KConst<T>& kc) {
  for (int d = 0; d < 3; ++d) {
    p[d] = (T)o[d] + spos4[4 * g + d];
    n[d] = snrm4[4 * g + d];
  }
  T nb = T(0);
  for (int d = 0; d < 3; ++d) {
    dd[d] = kc.cU * dens8[8 * g + d];
    dd[4 + d] = kc.cP * dens8[8 * g + 4 + d];
    nb += n[d] * dd[4 + d];
  }
  dd[3] = nb;
  dd[7] = T(0);
}

// Evaluate the sources of a list of leaves at the check surface of box B (displacement, U and/or P).
//   S2M: B's own sources at its upward check surface (radius r_up_check), written to row B of q (times
//        r_B with s2m_r: the scaled check potential qhat of the check-potential translations).
//   S2L: sources of X(B) at B's downward check surface (radius r_dn_check), r_B * value written to row
//        blockIdx.x of a compact buffer (added to qhat afterwards).  With pair_src, one workgroup per X pair
//        (boxes[i], pair_src[i]), row i of a per-pair buffer (summed per box in list order afterwards): the
//        X lists differ in length by an order of magnitude, so per-box workgroups left a long tail.
template <typename T, typename TQ, bool SL, bool DL, bool S2M>
__global__ __launch_bounds__(1024) void k_check_eval(const int* __restrict__ boxes, TreeView tv,
                                                    const int* __restrict__ list_off,
                                                    const int* __restrict__ list_idx, const T* __restrict__ spos4,
                                                    const T* __restrict__ snrm4, const T* __restrict__ dens8,
                                                    const double* __restrict__ surf, int n_eq, double radius, int NC,
                                                    KConst<T> kc, TQ* __restrict__ out, int s2m_r = 0,
                                                    const int* __restrict__ pair_src = nullptr,
                                                    uint16_t* __restrict__ split = nullptr,
                                                    float* __restrict__ split_scale = nullptr,
                                                    const signed char* __restrict__ pair_sh = nullptr) {
  __shared__ T sp[kStage][4];
  __shared__ T sn[kStage][4];
  __shared__ T sd[kStage][8];
  const int B = boxes[blockIdx.x];
  const int tid = threadIdx.x;
  const double rB = box_half(tv.level, tv.geom, tv.root_R, B);
  T x[3] = {0, 0, 0};
  if (tid < n_eq)
    for (int d = 0; d < 3; ++d) x[d] = (T)(radius * rB * surf[3 * tid + d]);
  // S2M: U and P brackets apart, prefactors at the end (see disp_pair); S2L: one accumulator on
  // prefactor-scaled densities (disp_pair_f)
  T vU[3] = {0, 0, 0}, vP[3] = {0, 0, 0};
  int fill = 0;
  auto flush = [&](int n) {
    __syncthreads();
    if (tid < n_eq) {
      for (int j = 0; j < n; ++j) {
        T dx = sp[j][0] - x[0], dy = sp[j][1] - x[1], dz = sp[j][2] - x[2];
        T r2 = dx * dx + dy * dy + dz * dz;
        if (r2 == T(0)) continue;
        if (S2M)
          disp_pair<T, SL, DL>(dx, dy, dz, r2, sd[j], sd[j] + 4, sn[j][0], sn[j][1], sn[j][2], kc, vU, vP);
        else
          disp_pair_f<T, SL, DL>(dx, dy, dz, r2, sd[j], sd[j] + 4, sd[j][3], sn[j][0], sn[j][1], sn[j][2], kc,
                                 vU);
      }
    }
    __syncthreads();
  };
  const int nl = S2M || pair_src ? 1 : list_off[B + 1] - list_off[B];
  for (int li = 0; li < nl; ++li) {
    const int A = S2M ? B : (pair_src ? pair_src[blockIdx.x] : list_idx[list_off[B] + li]);
    double o[3] = {0, 0, 0};
    if (!S2M) box_offset(tv.level, tv.ix, tv.iy, tv.iz, tv.geom, tv.root_R, A, B, o);
    if (pair_sh) add_lattice_shift(o, pair_sh[blockIdx.x], tv.geom, tv.root_R, B);
    const int s0 = tv.src_b[A], ns = tv.src_e[A] - s0;
    for (int base = 0; base < ns; base += kStage) {
      int cnt = min(kStage, ns - base);
      if (fill + cnt > kStage) {
        flush(fill);
        fill = 0;
      }
      for (int i = tid; i < cnt; i += blockDim.x) {
        const int64_t g = s0 + base + i;
        if (S2M) {
          for (int d = 0; d < 3; ++d) {
            sp[fill + i][d] = (T)o[d] + spos4[4 * g + d];
            sn[fill + i][d] = snrm4[4 * g + d];
          }
          for (int d = 0; d < 8; ++d) sd[fill + i][d] = dens8[8 * g + d];
        } else {
          stage_source(sp[fill + i], sn[fill + i], sd[fill + i], o, spos4, snrm4, dens8, g, kc);
        }
      }
      fill += cnt;
    }
  }
  flush(fill);
  TQ qv[3] = {0, 0, 0};
  if (tid < n_eq) {
    for (int d = 0; d < 3; ++d) {
      const double vd = S2M ? (double)(kc.cU * vU[d] - kc.cP * vP[d]) : (double)vU[d];
      if (S2M) {
        qv[d] = (TQ)(s2m_r ? rB * vd : vd);
        out[(size_t)B * NC + 3 * tid + d] = qv[d];
      } else {
        out[(size_t)blockIdx.x * NC + 3 * tid + d] = (TQ)(rB * vd);
      }
    }
  }
  if constexpr (S2M && sizeof(TQ) == 4) {
    // S2M with split != nullptr: the row's split-FP16 copy as split_h3 writes it (power-of-two scale from
    // the row's largest magnitude, [hi 8 | lo 8] chunks); the padding entries past 3 n_eq are zero
    if (split) {
      __shared__ float wmax[16];
      float m = fmaxf(fabsf((float)qv[0]), fmaxf(fabsf((float)qv[1]), fabsf((float)qv[2])));
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
      if ((tid & 63) == 0) wmax[tid >> 6] = m;
      __syncthreads();
      m = wmax[0];
      for (int w = 1; w < (int)(blockDim.x + 63) / 64; ++w) m = fmaxf(m, wmax[w]);
      int e2 = 0;
      float sc = 1.0f;
      if (m > 0.0f && m < INFINITY) {
        frexpf(m, &e2);  // m = f 2^e2, f in [0.5, 1): scale to put m in [2^14, 2^15)
        sc = ldexpf(1.0f, max(-126, min(127, e2 - 15)));
      }
      if (tid == 0) split_scale[B] = sc;
      const float inv = 1.0f / sc;
      _Float16* d = (_Float16*)split + (size_t)B * 2 * NC;
      auto put = [&](int k, float v) {
        const float y = v * inv;
        const _Float16 h = (_Float16)y;
        d[16 * (k / 8) + (k % 8)] = h;
        d[16 * (k / 8) + 8 + (k % 8)] = (_Float16)(y - (float)h);
      };
      if (tid < n_eq)
        for (int dd = 0; dd < 3; ++dd) put(3 * tid + dd, (float)qv[dd]);
      for (int k = 3 * n_eq + tid; k < NC; k += blockDim.x) put(k, 0.0f);
    }
  }
}

// ------------------------------------------------------------------------------- leaf evaluation

// One workgroup per target leaf B.  Every lane owns two targets (register blocking: each staged point is
// read from LDS once per two targets) and the lanes are split into S slices over the staged points; slice
// partial sums are reduced in LDS at the end.  KIND 0 = displacement (3), 1 = stress (6).
// far_field: L2T from B's downward equivalent surface, plus the W(B) contributions computed by k_w_eval
// (one output slot per W pair, summed here in list order); near_field: U(B) directly; accumulate: add
// to out instead of storing.
template <typename T, int KIND, bool SL, bool DL>
__global__ __launch_bounds__(256) void k_leaf_eval(
    const int* __restrict__ leaves, TreeView tv, const int* __restrict__ u_off, const int* __restrict__ u_idx,
    const signed char* __restrict__ u_sh, const int* __restrict__ w_off, const int64_t* __restrict__ wslot_off,
    const double* __restrict__ wslot,
    const T* __restrict__ spos4,
    const T* __restrict__ snrm4, const T* __restrict__ dens8, const T* __restrict__ tpos4,
    const int* __restrict__ perm_trg, const T* __restrict__ phi_dn, const T* __restrict__ phi_up,
    const double* __restrict__ surf, int n_eq, double r_up_equiv, double r_dn_equiv, int NC, int far_field,
    int near_field, int accumulate, KConst<T> kc, double* __restrict__ out) {
  constexpr int NO = KIND == 0 ? 3 : 6;
  constexpr int TPL = 2;  // targets per lane
  __shared__ T sp[kStage][4];
  __shared__ T sn[kStage][4];
  __shared__ T sd[kStage][8];
  __shared__ double red[256][TPL * NO];
  const int B = leaves[blockIdx.x];
  const int tid = threadIdx.x;
  const double rB = box_half(tv.level, tv.geom, tv.root_R, B);
  const int t0 = tv.trg_b[B], nt_all = tv.trg_e[B] - t0;
  for (int tc = 0; tc < nt_all; tc += 256 * TPL) {
    const int nt = min(256 * TPL, nt_all - tc);
    const int ntp = (nt + TPL - 1) / TPL;  // lanes per slice
    const int S = 256 / ntp;
    const int tp = tid % ntp, sl = tid / ntp;
    const bool act = sl < S;
    T x[TPL][3];
    bool valid[TPL];
    for (int q = 0; q < TPL; ++q) {
      const int t = TPL * tp + q;
      valid[q] = t < nt;
      const int64_t g = t0 + tc + (valid[q] ? t : 0);
      for (int d = 0; d < 3; ++d) x[q][d] = tpos4[4 * g + d];
    }
    T aU[TPL][NO], aP[TPL][NO];
    for (int q = 0; q < TPL; ++q)
      for (int c = 0; c < NO; ++c) aU[q][c] = aP[q][c] = T(0);
    int fill = 0;
    // far-field points carry only a single-layer density (in sd[0..2])
    auto flush = [&](int n, bool near) {
      __syncthreads();
      if (act && !near && KIND == 0) {
        // L2T: each equivalent point read once for both targets, no branch (a target on the point, which the
        // check radius rules out anyway, would add zeros; targets past nt are computed and never stored).
        // The near field keeps its branches: alone it would run faster without them, but beside the main
        // stream's matrix-core work the evaluation as a whole ran slower.
        for (int j = sl; j < n; j += S) {
          const T px = sp[j][0], py = sp[j][1], pz = sp[j][2];
          const T wa[3] = {sd[j][0], sd[j][1], sd[j][2]};
#pragma unroll
          for (int q = 0; q < TPL; ++q) {
            const T dx = px - x[q][0], dy = py - x[q][1], dz = pz - x[q][2];
            const T ir = rsqrt_or_zero(dx * dx + dy * dy + dz * dz);
            disp_pair_f_ir<T, true, false>(dx, dy, dz, ir, wa, wa, T(0), T(0), T(0), T(0), kc, aP[q]);
          }
        }
      } else if (act) {
        for (int j = sl; j < n; j += S) {
          const T px = sp[j][0], py = sp[j][1], pz = sp[j][2];
#pragma unroll
          for (int q = 0; q < TPL; ++q) {
            if (!valid[q]) continue;
            T dx = px - x[q][0], dy = py - x[q][1], dz = pz - x[q][2];
            T r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == T(0)) continue;
            if (near) {
              if (KIND == 0)
                disp_pair_f<T, SL, DL>(dx, dy, dz, r2, sd[j], sd[j] + 4, sd[j][3], sn[j][0], sn[j][1], sn[j][2], kc,
                                       aU[q]);
              else
                stress_pair<T, SL, DL>(dx, dy, dz, r2, sd[j], sd[j] + 4, sn[j][0], sn[j][1], sn[j][2], kc, aU[q],
                                       aP[q]);
            } else {
              // far field: unscaled equivalent density, U bracket in aP (times cU at the end)
              if (KIND == 0)
                disp_pair_f<T, true, false>(dx, dy, dz, r2, sd[j], sd[j], T(0), T(0), T(0), T(0), kc, aP[q]);
              else
                stress_pair<T, true, false>(dx, dy, dz, r2, sd[j], sd[j], T(0), T(0), T(0), kc, aU[q], aP[q]);
            }
          }
        }
      }
      __syncthreads();
    };
    if (far_field) {
      // L2T: B's downward equivalent surface
      const double rad = r_dn_equiv * rB;
      for (int base = 0; base < n_eq; base += kStage) {
        const int cnt = min(kStage, n_eq - base);
        if (fill + cnt > kStage) {
          flush(fill, false);
          fill = 0;
        }
        for (int i = tid; i < cnt; i += blockDim.x) {
          const int e = base + i;
          for (int d = 0; d < 3; ++d) {
            sp[fill + i][d] = (T)(rad * surf[3 * e + d]);
            sd[fill + i][d] = phi_dn[(size_t)B * NC + 3 * e + d];
          }
        }
        fill += cnt;
      }
      flush(fill, false);
      fill = 0;
    }
    // near field: U(B)
    const int u_end = near_field ? u_off[B + 1] : u_off[B];
    for (int li = u_off[B]; li < u_end; ++li) {
      const int A = u_idx[li];
      double o[3];
      box_offset(tv.level, tv.ix, tv.iy, tv.iz, tv.geom, tv.root_R, A, B, o);
      add_lattice_shift(o, u_sh[li], tv.geom, tv.root_R, B);
      const int s0 = tv.src_b[A], ns = tv.src_e[A] - s0;
      for (int base = 0; base < ns; base += kStage) {
        int cnt = min(kStage, ns - base);
        if (fill + cnt > kStage) {
          flush(fill, true);
          fill = 0;
        }
        for (int i = tid; i < cnt; i += blockDim.x) {
          int64_t g = s0 + base + i;
          if (KIND == 0) {
            stage_source(sp[fill + i], sn[fill + i], sd[fill + i], o, spos4, snrm4, dens8, g, kc);
          } else {
            for (int d = 0; d < 3; ++d) {
              sp[fill + i][d] = (T)o[d] + spos4[4 * g + d];
              sn[fill + i][d] = snrm4[4 * g + d];
            }
            for (int d = 0; d < 8; ++d) sd[fill + i][d] = dens8[8 * g + d];
          }
        }
        fill += cnt;
      }
    }
    flush(fill, true);
    // combine prefactors, reduce the slices
    for (int q = 0; q < TPL; ++q)
      for (int c = 0; c < NO; ++c) {
        double v;
        if (KIND == 0)  // near field: prefactors folded into the staged densities; far field: times cU here
          v = (double)aU[q][c] + (double)kc.cU * (double)aP[q][c];
        else
          v = (double)kc.cD * (double)aU[q][c] + (double)kc.cS * (double)aP[q][c];
        red[tid][q * NO + c] = act ? v : 0.0;
      }
    __syncthreads();
    for (int t = tid; t < nt; t += blockDim.x) {
      double acc[NO];
      for (int c = 0; c < NO; ++c) acc[c] = 0;
      const int lt = t / TPL, q = t % TPL;
      for (int s2 = 0; s2 < S; ++s2)
        for (int c = 0; c < NO; ++c) acc[c] += red[s2 * ntp + lt][q * NO + c];
      if (far_field)  // W(B) slots in list order
        for (int k = w_off[B]; k < w_off[B + 1]; ++k)
          for (int c = 0; c < NO; ++c) acc[c] += wslot[wslot_off[k] + (int64_t)(tc + t) * NO + c];
      int o = perm_trg[t0 + tc + t];
      if (accumulate)
        for (int c = 0; c < NO; ++c) out[(size_t)o * NO + c] += acc[c];
      else
        for (int c = 0; c < NO; ++c) out[(size_t)o * NO + c] = acc[c];
    }
    __syncthreads();
  }
}

// M2T over the W lists, one workgroup per pair (B, A): A's upward equivalent surface evaluated at the
// targets of leaf B, stored in the pair's slot (nt(B) x NO, prefactors applied).  One pair per workgroup
// keeps the work even: a leaf next to a finely refined region can have tens of W boxes.
template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_w_eval(const int* __restrict__ pair_b, const int* __restrict__ pair_a,
                                                const signed char* __restrict__ pair_sh,
                                                const int64_t* __restrict__ slot_off, TreeView tv,
                                                const T* __restrict__ tpos4, const T* __restrict__ phi_up,
                                                const double* __restrict__ surf, int n_eq, double r_up_equiv, int NC,
                                                KConst<T> kc, double* __restrict__ wslot) {
  constexpr int NO = KIND == 0 ? 3 : 6;
  constexpr int TPL = 2;
  __shared__ T sp[kStage][4];
  __shared__ T sd[kStage][4];
  __shared__ double red[256][TPL * NO];
  const int B = pair_b[blockIdx.x], A = pair_a[blockIdx.x];
  const int tid = threadIdx.x;
  double o[3];
  box_offset(tv.level, tv.ix, tv.iy, tv.iz, tv.geom, tv.root_R, A, B, o);
  add_lattice_shift(o, pair_sh[blockIdx.x], tv.geom, tv.root_R, B);
  const double rad = r_up_equiv * box_half(tv.level, tv.geom, tv.root_R, A);
  double* out = wslot + slot_off[blockIdx.x];
  const int t0 = tv.trg_b[B], nt_all = tv.trg_e[B] - t0;
  for (int tc = 0; tc < nt_all; tc += 256 * TPL) {
    const int nt = min(256 * TPL, nt_all - tc);
    const int ntp = (nt + TPL - 1) / TPL;
    const int S = 256 / ntp;
    const int tp = tid % ntp, sl = tid / ntp;
    const bool act = sl < S;
    T x[TPL][3];
    bool valid[TPL];
    for (int q = 0; q < TPL; ++q) {
      const int t = TPL * tp + q;
      valid[q] = t < nt;
      const int64_t g = t0 + tc + (valid[q] ? t : 0);
      for (int d = 0; d < 3; ++d) x[q][d] = tpos4[4 * g + d];
    }
    T aU[TPL][NO], aP[TPL][NO];
    for (int q = 0; q < TPL; ++q)
      for (int c = 0; c < NO; ++c) aU[q][c] = aP[q][c] = T(0);
    for (int base = 0; base < n_eq; base += kStage) {
      const int cnt = min(kStage, n_eq - base);
      __syncthreads();
      for (int i = tid; i < cnt; i += blockDim.x) {
        const int e = base + i;
        for (int d = 0; d < 3; ++d) {
          sp[i][d] = (T)(o[d] + rad * surf[3 * e + d]);
          sd[i][d] = phi_up[(size_t)A * NC + 3 * e + d];
        }
      }
      __syncthreads();
      if (act)
        for (int j = sl; j < cnt; j += S) {
          const T px = sp[j][0], py = sp[j][1], pz = sp[j][2];
#pragma unroll
          for (int q = 0; q < TPL; ++q) {
            if (!valid[q]) continue;
            T dx = px - x[q][0], dy = py - x[q][1], dz = pz - x[q][2];
            T r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == T(0)) continue;
            if (KIND == 0)
              disp_pair_f<T, true, false>(dx, dy, dz, r2, sd[j], sd[j], T(0), T(0), T(0), T(0), kc, aU[q]);
            else
              stress_pair<T, true, false>(dx, dy, dz, r2, sd[j], sd[j], T(0), T(0), T(0), kc, aU[q], aP[q]);
          }
        }
    }
    for (int q = 0; q < TPL; ++q)
      for (int c = 0; c < NO; ++c) {
        double v = KIND == 0 ? (double)kc.cU * (double)aU[q][c] : (double)kc.cD * (double)aU[q][c];
        red[tid][q * NO + c] = act ? v : 0.0;
      }
    __syncthreads();
    for (int t = tid; t < nt; t += blockDim.x) {
      double acc[NO];
      for (int c = 0; c < NO; ++c) acc[c] = 0;
      const int lt = t / TPL, q = t % TPL;
      for (int s2 = 0; s2 < S; ++s2)
        for (int c = 0; c < NO; ++c) acc[c] += red[s2 * ntp + lt][q * NO + c];
      for (int c = 0; c < NO; ++c) out[(int64_t)(tc + t) * NO + c] = acc[c];
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------- periodic cell-mean constant

// Periodic cells, displacement.  The images beyond the 3 x 3 x 3 block reach the root through its upward
// equivalent density.  Image by image that is exact outside the equivalent surface, but the zero-mean
// lattice sum (k = 0 left out) also depends on the field inside: the fast sum exceeds the exact one by
// the cell mean (1/V) int D of D = (field of the sources) - (field of the equivalent density), a field
// that vanishes outside the equivalent surface.  Its transform at k -> 0 follows from the force
// distributions' second moments m2_lbc = sum f_l y_b y_c (y from the root centre; the equivalent density
// matches the lower moments): with Uhat(k) = [delta/k^2 - k k^T / (2 (1-nu) k^4)] / G and averaging over
// the directions of k (the limit does not depend on them),
//   int D_m = -(1 / (2 G)) [dt_m / 3 - (dt_m + 2 ds_m) / (30 (1 - nu))],
//   t_m = sum_b m2_mbb,  s_m = sum_l m2_lml,  d = sources minus equivalent density.
// Point forces f at y give t = f |y|^2, s = y (f . y); a double-layer source, a force dipole of tensor
// Q = C : (w b) (x) n (f = -div(Q delta_y)), gives t = 2 Q y and s = Q y + tr(Q) y.
// k_per_moments: one workgroup per chunk of a root's sources, the chunk's (t, s) into part[6 * chunk].
template <typename T>
__global__ __launch_bounds__(256) void k_per_moments(const int* __restrict__ chunk_root,
                                                     const int* __restrict__ chunk_b, const int* __restrict__ chunk_e,
                                                     TreeView tv, const int* __restrict__ leaf_of,
                                                     const T* __restrict__ spos4, const T* __restrict__ snrm4,
                                                     const T* __restrict__ dens8, double lam, double G,
                                                     double* __restrict__ part) {
  __shared__ double red[256][6];
  const int c = blockIdx.x, root = chunk_root[c];
  const int g = tv.geom[root];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int i = chunk_b[c] + (int)threadIdx.x; i < chunk_e[c]; i += blockDim.x) {
    double cen[3];
    box_center(tv.level, tv.ix, tv.iy, tv.iz, tv.geom, tv.root_c, tv.root_R, leaf_of[i], cen);
    double y[3], f[3];
    for (int d = 0; d < 3; ++d) {
      y[d] = cen[d] - tv.root_c[3 * g + d] + (double)spos4[4 * (int64_t)i + d];
      f[d] = (double)dens8[8 * (int64_t)i + d];
    }
    const double yy = y[0] * y[0] + y[1] * y[1] + y[2] * y[2], fy = f[0] * y[0] + f[1] * y[1] + f[2] * y[2];
    for (int d = 0; d < 3; ++d) {
      acc[d] += f[d] * yy;
      acc[3 + d] += y[d] * fy;
    }
    if (snrm4) {
      double wb[3], n[3], bn = 0.0;
      for (int d = 0; d < 3; ++d) {
        wb[d] = (double)dens8[8 * (int64_t)i + 4 + d];
        n[d] = (double)snrm4[4 * (int64_t)i + d];
        bn += wb[d] * n[d];
      }
      double Qy[3];
      for (int l = 0; l < 3; ++l) {
        Qy[l] = 0.0;
        for (int m = 0; m < 3; ++m) Qy[l] += (lam * (l == m ? bn : 0.0) + G * (wb[l] * n[m] + wb[m] * n[l])) * y[m];
      }
      const double trQ = 3.0 * lam * bn + 2.0 * G * bn;
      for (int d = 0; d < 3; ++d) {
        acc[d] += 2.0 * Qy[d];
        acc[3 + d] += Qy[d] + trQ * y[d];
      }
    }
  }
  for (int k = 0; k < 6; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 6; ++k) red[threadIdx.x][k] += red[threadIdx.x + st][k];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) part[6 * c + k] = red[0][k];
}

// The equivalent density's (t, s) per root: linear in its upward vector (phi_up, or the check potential
// qhat_up with UC2UE folded into the rows), eqm[6 r + k] = R^2 sum_j W[k][j] vec[root][j] (W at unit
// half-width; one workgroup per root, 6 fixed-order block sums).  Taken before the downward pass reuses
// the upward buffers.
template <typename TQ>
__global__ __launch_bounds__(256) void k_per_eqm(const int* __restrict__ roots, const double* __restrict__ W,
                                                 const TQ* __restrict__ vec, int NC, TreeView tv,
                                                 double* __restrict__ eqm) {
  __shared__ double red[256][6];
  const int r = blockIdx.x, root = roots[r];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int j = threadIdx.x; j < NC; j += blockDim.x) {
    const double v = (double)vec[(size_t)root * NC + j];
    for (int k = 0; k < 6; ++k) acc[k] += W[(size_t)k * NC + j] * v;
  }
  for (int k = 0; k < 6; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 6; ++k) red[threadIdx.x][k] += red[threadIdx.x + st][k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double R = tv.root_R[tv.geom[root]];
    for (int k = 0; k < 6; ++k) eqm[6 * r + k] = R * R * red[0][k];
  }
}

// One workgroup per root: the chunk sums in a fixed order, minus the equivalent density's moments, give
// the constant, subtracted from the root's target rows of out (caller order [trg_b, trg_e), 3 per row).
__global__ __launch_bounds__(256) void k_per_shift(const int* __restrict__ roots, const int* __restrict__ chunk_off,
                                                   const int* __restrict__ trg_b, const int* __restrict__ trg_e,
                                                   const double* __restrict__ part, TreeView tv,
                                                   const double* __restrict__ eqm, double nu, double G,
                                                   double* __restrict__ out) {
  __shared__ double sc[3];
  const int r = blockIdx.x, root = roots[r];
  const double R = tv.root_R[tv.geom[root]];
  if (threadIdx.x == 0) {
    double m[6] = {0, 0, 0, 0, 0, 0};
    for (int c = chunk_off[r]; c < chunk_off[r + 1]; ++c)
      for (int k = 0; k < 6; ++k) m[k] += part[6 * c + k];
    for (int k = 0; k < 6; ++k) m[k] -= eqm[6 * r + k];
    const double V = 8.0 * R * R * R;
    for (int d = 0; d < 3; ++d)
      sc[d] = -(m[d] / 3.0 - (m[d] + 2.0 * m[3 + d]) / (30.0 * (1.0 - nu))) / (2.0 * G * V);
  }
  __syncthreads();
  for (int i = trg_b[r] + (int)threadIdx.x; i < trg_e[r]; i += blockDim.x)
    for (int d = 0; d < 3; ++d) out[3 * (int64_t)i + d] -= sc[d];
}

// ------------------------------------------------------------------------------------------ plan

static GemmJob upload_job(Arena& a, const GemmCols& cols, hipStream_t s, int tile_cols,
                          const std::vector<int>* op_rank) {
  GemmJob job;
  job.cols_per_tile = tile_cols;
  const int n = (int)cols.op.size();
  if (n == 0) return job;
  // tiles: consecutive columns with the same op, <= tile_cols each (columns must be grouped by op)
  std::vector<int4> tiles;
  int i = 0;
  while (i < n) {
    int j = i;
    while (j < n && cols.op[j] == cols.op[i] && j - i < tile_cols) ++j;
    tiles.push_back(make_int4(cols.op[i], i, j - i, op_rank ? (*op_rank)[cols.op[i]] : 0));
    job.ranked = job.ranked || op_rank != nullptr;
    i = j;
  }
  job.n_tiles = (int)tiles.size();
  job.tiles = a.get<int4>(tiles.size());
  KFMM_HIP(hipMemcpyAsync(job.tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  job.in_idx = a.get<int>(n);
  job.out_idx = a.get<int>(n);
  job.scale = a.get<double>(n);
  KFMM_HIP(hipMemcpyAsync(job.in_idx, cols.in.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  KFMM_HIP(hipMemcpyAsync(job.out_idx, cols.out.data(), n * sizeof(int), hipMemcpyHostToDevice, s));
  KFMM_HIP(hipMemcpyAsync(job.scale, cols.scale.data(), n * sizeof(double), hipMemcpyHostToDevice, s));
  KFMM_HIP(hipStreamSynchronize(s));  // host vectors may be released after return
  return job;
}

// Sort columns by op (stable) so that tiles share one operator.
static GemmCols sorted_by_op(const GemmCols& c) {
  std::vector<int> order(c.op.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c.op[a] < c.op[b]; });
  GemmCols o;
  for (int i : order) o.add(c.op[i], c.in[i], c.out[i], c.scale[i]);
  return o;
}

template <typename T>
static T* upload_vec(Arena& a, const std::vector<T>& h, hipStream_t s) {
  T* d = a.get<T>(h.empty() ? 1 : h.size());
  if (!h.empty()) {
    KFMM_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    KFMM_HIP(hipStreamSynchronize(s));
  }
  return d;
}

// C = A B for NC x NC row-major host matrices (threads over rows).
static std::vector<double> host_matmul(const std::vector<double>& A, const std::vector<double>& B, int n) {
  std::vector<double> C((size_t)n * n, 0.0);
  auto rows = [&](int i0, int i1) {
    for (int i = i0; i < i1; ++i)
      for (int k = 0; k < n; ++k) {
        const double a = A[(size_t)i * n + k];
        if (a == 0.0) continue;
        for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += a * B[(size_t)k * n + j];
      }
  };
  const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t) pool.emplace_back(rows, n * t / nth, n * (t + 1) / nth);
  for (auto& th : pool) th.join();
  return C;
}

// Periodic-cell operators of an operator set (once per set; see DeviceOps).  fp32: the check-potential
// forms are needed; dn: the downward-density form (FP64 translations with the compressed M2L).
static void ensure_periodic_ops(DeviceOps& D, int p, const Elastic& el, bool fp32, bool dn) {
  std::lock_guard<std::mutex> lock(D.per_mutex);
  const int NC = D.NC, n = 3 * D.n_eq;
  std::vector<double> Tp;
  auto far = [&]() -> const std::vector<double>& {
    if (Tp.empty()) Tp = pad_square(periodic_far_operator(p, el), n, NC);
    return Tp;
  };
  auto down = [&](const double* d) {
    std::vector<double> h((size_t)NC * NC);
    KFMM_HIP(hipMemcpy(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    return h;
  };
  if (!D.per_far64) {
    D.per_far64 = D.arena.get<double>((size_t)NC * NC);
    KFMM_HIP(hipMemcpy(D.per_far64, far().data(), (size_t)NC * NC * sizeof(double), hipMemcpyHostToDevice));
    // second-moment rows on phi_up at unit half-width: t_m = sum_e phi_e,m |z_e|^2, s_m = sum_e z_e,m (phi_e . z_e)
    std::vector<double> surf(3 * (size_t)D.n_eq), W(6 * (size_t)NC, 0.0);
    KFMM_HIP(hipMemcpy(surf.data(), D.surf, surf.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int e = 0; e < D.n_eq; ++e) {
      double z[3];
      for (int d = 0; d < 3; ++d) z[d] = 1.05 * surf[3 * e + d];
      const double zz = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
      for (int m = 0; m < 3; ++m)
        for (int d = 0; d < 3; ++d) {
          if (m == d) W[(size_t)m * NC + 3 * e + d] = zz;
          W[(size_t)(3 + m) * NC + 3 * e + d] = z[m] * z[d];
        }
    }
    D.per_mom_phi = D.arena.get<double>(W.size());
    KFMM_HIP(hipMemcpy(D.per_mom_phi, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  if (fp32 && !D.per_farq32) {
    const std::vector<double> uc = down(D.uc2ue);
    std::vector<double> Tq = host_matmul(far(), uc, NC);
    std::vector<float> Tq32(Tq.begin(), Tq.end());
    D.per_farq32 = D.arena.get<float>(Tq32.size());
    KFMM_HIP(hipMemcpy(D.per_farq32, Tq32.data(), Tq32.size() * sizeof(float), hipMemcpyHostToDevice));
    std::vector<double> Wp(6 * (size_t)NC), Wq(6 * (size_t)NC, 0.0);
    KFMM_HIP(hipMemcpy(Wp.data(), D.per_mom_phi, Wp.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int k = 0; k < 6; ++k)
      for (int i = 0; i < NC; ++i) {
        const double a = Wp[(size_t)k * NC + i];
        if (a == 0.0) continue;
        for (int j = 0; j < NC; ++j) Wq[(size_t)k * NC + j] += a * uc[(size_t)i * NC + j];
      }
    D.per_mom_q = D.arena.get<double>(Wq.size());
    KFMM_HIP(hipMemcpy(D.per_mom_q, Wq.data(), Wq.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  if (dn && !D.per_fardn64) {
    std::vector<double> Td = host_matmul(down(D.dc2de), far(), NC);
    D.per_fardn64 = D.arena.get<double>(Td.size());
    KFMM_HIP(hipMemcpy(D.per_fardn64, Td.data(), Td.size() * sizeof(double), hipMemcpyHostToDevice));
  }
}

Plan* plan_create(const double* src, const double* nrm, const double* w, int64_t n_src, const double* trg,
                  int64_t n_trg, const std::vector<int64_t>& bs, const std::vector<int64_t>& bt, const fmm_opts& o,
                  hipStream_t s, const std::vector<double>& cells) {
  auto t_start = std::chrono::steady_clock::now();
  KFMM_REQUIRE(o.precision == KFMM_FP64 || o.precision == KFMM_FP32 || o.precision == KFMM_FP32_M2L_SPLIT16 ||
                   o.precision == KFMM_FP32_TRANS64,
               o.precision == KFMM_FP32_M2L_BF16 ? kBf16Withdrawn : "unknown precision");
  std::unique_ptr<Plan> P(new Plan());
  P->opts = o;
  P->periodic = !cells.empty();
  P->el = Elastic::make(o.K, o.G);
  P->prec = o.precision;
  P->f32t = o.precision == KFMM_FP32 || o.precision == KFMM_FP32_M2L_SPLIT16;
  P->n_src = n_src;
  P->alias = trg == nullptr && n_trg == n_src;  // NULL with n_trg == 0 (and n_src > 0): no targets
  P->n_trg = P->alias ? n_src : n_trg;
  P->has_nrm = nrm != nullptr;
  P->arena.limit = o.mem_limit;
  const int p = o.p > 0 ? o.p : 6;
  const int leaf_max = o.leaf_max > 0 ? o.leaf_max : 64;
  const int max_depth = std::min(o.max_depth > 0 ? o.max_depth : 16, kMortonBits - 1);
  // relative cutoff of the pseudo-inverse: 1e-8 minimised the measured error for p = 4..10
  double eps = o.svd_eps > 0 ? o.svd_eps : 1e-8;
  P->ops = get_ops(p, P->el, eps, o.precision, s);
  const DeviceOps& D = *P->ops;
  P->NC = D.NC;
  P->n_eq = D.n_eq;
  if (n_src == 0 || P->n_trg == 0) {
    P->empty = true;
    P->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return P.release();
  }
  Tree& t = P->tree;
  build_tree(t, P->arena, src, n_src, trg, n_trg, bs, bt, leaf_max, max_depth, s, cells);
  // a W or X pair with at most n_eq points on its direct side goes to the near field as a direct sum (the
  // near field runs at the VALU issue limit, the W and X kernels at 25-40% of it; measured on 64 periodic
  // cells: 131M target points/s without, 187-189M with a limit of n_eq / 2, n_eq or 2 n_eq; box beam
  // unchanged within noise)
  build_lists(t, P->arena, s, D.n_eq);
  P->tv = TreeView{t.level, t.ix, t.iy, t.iz, t.geom, t.root_c, t.root_R, t.src_b, t.src_e, t.trg_b, t.trg_e};
  const int nb = t.n_box, NC = P->NC;
  // ---- sorted local point data
  const bool f64 = o.precision == KFMM_FP64;
  const size_t ts = f64 ? 8 : 4;
  P->spos = P->arena.alloc(ts * 4 * n_src);
  P->snrm = P->arena.alloc(ts * 4 * n_src);
  P->sw = P->arena.get<double>(n_src);
  P->tpos = P->alias ? P->spos : P->arena.alloc(ts * 4 * P->n_trg);
  P->dens = P->arena.alloc(ts * 8 * n_src);
  unsigned gb = (unsigned)((n_src + 255) / 256), gt = (unsigned)((P->n_trg + 255) / 256);
  if (f64) {
    hipLaunchKernelGGL(k_local_points<double>, dim3(gb), dim3(256), 0, s, n_src, t.perm_src, t.leaf_of_src, src, nrm,
                       w, P->tv, (double*)P->spos, (double*)P->snrm, P->sw);
    if (!P->alias)
      hipLaunchKernelGGL(k_local_points<double>, dim3(gt), dim3(256), 0, s, P->n_trg, t.perm_trg, t.leaf_of_trg, trg,
                         (const double*)nullptr, (const double*)nullptr, P->tv, (double*)P->tpos, (double*)nullptr,
                         (double*)nullptr);
  } else {
    hipLaunchKernelGGL(k_local_points<float>, dim3(gb), dim3(256), 0, s, n_src, t.perm_src, t.leaf_of_src, src, nrm,
                       w, P->tv, (float*)P->spos, (float*)P->snrm, P->sw);
    if (!P->alias)
      hipLaunchKernelGGL(k_local_points<float>, dim3(gt), dim3(256), 0, s, P->n_trg, t.perm_trg, t.leaf_of_trg, trg,
                         (const double*)nullptr, (const double*)nullptr, P->tv, (float*)P->tpos, (float*)nullptr,
                         (double*)nullptr);
  }
  KFMM_HIP(hipGetLastError());
  // ---- work lists
  std::vector<int> leaves_src, leaves_trg, x_boxes;
  for (int b = 0; b < nb; ++b) {
    bool hs = t.h_src_e[b] > t.h_src_b[b], ht = t.h_trg_e[b] > t.h_trg_b[b];
    if (t.h_is_leaf[b] && hs) leaves_src.push_back(b);
    if (t.h_is_leaf[b] && ht) leaves_trg.push_back(b);
    if (t.h_x_off[b + 1] > t.h_x_off[b]) x_boxes.push_back(b);
  }
  P->n_leaves_src = (int)leaves_src.size();
  P->n_leaves_trg = (int)leaves_trg.size();
  P->n_x_boxes = (int)x_boxes.size();
  P->leaves_src = upload_vec(P->arena, leaves_src, s);
  {
    // the leaf passes run one workgroup per target leaf, in this order: leaves with the most near-field pairs
    // first, so that a leaf beside a finely refined region (tens of U-list boxes) does not start last and
    // hold the launch's tail (each leaf writes only its own targets, so the order leaves results unchanged)
    std::vector<int64_t> work(nb, 0);
    for (int b : leaves_trg)
      for (int k = t.h_u_off[b]; k < t.h_u_off[b + 1]; ++k) {
        const int A = t.h_u_idx[k];
        work[b] += (int64_t)(t.h_trg_e[b] - t.h_trg_b[b]) * (t.h_src_e[A] - t.h_src_b[A]);
      }
    std::vector<int> by_work = leaves_trg;
    std::stable_sort(by_work.begin(), by_work.end(), [&](int a, int b) { return work[a] > work[b]; });
    P->leaves_trg = upload_vec(P->arena, by_work, s);
  }
  P->x_boxes = upload_vec(P->arena, x_boxes, s);
  auto half = [&](int b) { return std::ldexp(t.h_root_R[t.h_geom[b]], -t.h_level[b]); };
  // 128-column tiles once a launch has enough columns to fill the chip with them
  auto wide = [](const GemmCols& c) { return c.op.size() >= 4096 ? 2 * kGemmBN : kGemmBN; };
  auto octant = [&](int b) { return (t.h_ix[b] & 1) | ((t.h_iy[b] & 1) << 1) | ((t.h_iz[b] & 1) << 2); };
  auto hs = [&](int b) { return t.h_src_e[b] > t.h_src_b[b]; };
  auto ht = [&](int b) { return t.h_trg_e[b] > t.h_trg_b[b]; };
  // coarsest level of the translations: V and W lists hold boxes of level >= 2 in free space; a periodic
  // tree has them from level 1 (images of the cell) and the root takes the far-image operator
  const int lv0 = P->periodic ? 0 : 2;
  // UC2UE over source leaves
  {
    GemmCols c;
    for (int b : leaves_src) c.add(0, b, b, half(b));
    P->job_uc2ue = upload_job(P->arena, c, s, wide(c));
    if (P->f32t) {  // UC2UE on the check potentials of every box with sources at level >= 2
      GemmCols ca;
      for (int b = 0; b < nb; ++b)
        if (t.h_level[b] >= lv0 && hs(b)) ca.add(0, b, b);
      P->job_up_all = upload_job(P->arena, ca, s, wide(ca));
      // with the compressed M2L, full equivalent densities are only read by the W lists: the second
      // factor runs on the W-list source boxes, the M2L takes U^T UC2UE qhat = G (fu1 qhat) directly
      std::vector<char> isw(nb, 0);
      for (int k : t.h_w_idx) isw[k] = 1;
      GemmCols cw;
      for (int b = 0; b < nb; ++b)
        if (isw[b] && t.h_level[b] >= lv0 && hs(b)) cw.add(0, b, b);
      P->job_up_w = upload_job(P->arena, cw, s, wide(cw));
    }
  }
  // M2M per level (deepest first): children with sources, grouped by octant; parents reduce.  Parents
  // below level lv0 are skipped (no list holds them).
  P->up_levels.clear();
  for (int l = t.depth; l >= lv0 + 1; --l) {
    GemmCols c;
    std::vector<int> parents;
    for (int b = t.level_start[l]; b < t.level_start[l + 1]; ++b)
      if (hs(b)) c.add(octant(b), b, b);
    for (int b = t.level_start[l - 1]; b < t.level_start[l]; ++b)
      if (!t.h_is_leaf[b] && hs(b)) parents.push_back(b);
    if (c.op.empty()) continue;
    UpLevel U;
    U.job = upload_job(P->arena, sorted_by_op(c), s, wide(c));
    U.n_par = (int)parents.size();
    U.parents = upload_vec(P->arena, parents, s);
    P->up_levels.push_back(U);
  }
  // M2L: V pairs grouped by compact offset index
  {
    GemmCols c;
    for (size_t i = 0; i < t.h_v_trg.size(); ++i) {
      int oi = D.m2l_index[t.h_v_off[i]];
      if (oi < 0) throw Error(-5, "internal: V pair with a near offset");
      c.add(oi, t.h_v_src[i], t.h_v_trg[i]);
    }
    GemmCols sc = sorted_by_op(c);
    // Every pair writes its own slot, then each target box sums its slots in a fixed order: repeated
    // products are bitwise identical (atomic accumulation would let the order, and so the rounding, vary
    // between calls, which GMRES on ill-conditioned systems sees as operator noise), and the plain stores
    // are cheaper than FP64 atomics.
    const int np_ = (int)sc.op.size();
    std::vector<std::vector<int>> slots(nb);
    for (int j = 0; j < np_; ++j) {
      slots[sc.out[j]].push_back(j);
      sc.out[j] = j;
    }
    std::vector<int> boxes, off = {0}, idx;
    for (int b2 = 0; b2 < nb; ++b2)
      if (!slots[b2].empty()) {
        boxes.push_back(b2);
        idx.insert(idx.end(), slots[b2].begin(), slots[b2].end());
        off.push_back((int)idx.size());
      }
    P->m2l_red_n = (int)boxes.size();
    P->m2l_red_box = upload_vec(P->arena, boxes, s);
    P->m2l_red_off = upload_vec(P->arena, off, s);
    P->m2l_red_idx = upload_vec(P->arena, idx, s);
    int slot_len = D.NC;
    const bool split16 = o.precision == KFMM_FP32_M2L_SPLIT16;
    const bool fp32m2l = o.precision == KFMM_FP32 || o.precision == KFMM_FP32_TRANS64;
    const bool comp64 = o.precision == KFMM_FP64 && o.m2l_tol > 0;  // FP64 contractions on the basis
    if ((fp32m2l || split16 || comp64) && o.m2l_tol > 0) {
      // compressed M2L: phi~ = U^T phi for every source box, r x r contractions per pair, and the downward
      // pass starts from q~ with DC2DE * U
      P->comp = get_compressed(*P->ops, o.m2l_tol, s);
      slot_len = P->comp->NCr;
      GemmCols cu;
      for (int b2 = 0; b2 < nb; ++b2)
        if (t.h_src_e[b2] > t.h_src_b[b2]) cu.add(0, b2, b2);
      // split FP16: 64-column tiles (a few thousand boxes in 128-column tiles leave most compute units idle)
      P->job_ut = upload_job(P->arena, cu, s, split16 || comp64 ? kGemmBN : 2 * kGemmBN);
      if (comp64) {
        P->phi_t64 = P->arena.get<double>((size_t)nb * slot_len);
        KFMM_HIP(hipMemsetAsync(P->phi_t64, 0, sizeof(double) * nb * slot_len, s));
        ensure_rank64(*P->ops, P->comp.get(), s);
      } else {
        P->phi_t = P->arena.get<float>((size_t)nb * slot_len);
        KFMM_HIP(hipMemsetAsync(P->phi_t, 0, sizeof(float) * nb * slot_len, s));  // boxes without sources
      }
      // rows of boxes without V lists stay zero: the downward pass applies DC2DE * U to every box
      if (P->f32t) {
        P->q_t_f = P->arena.get<float>((size_t)nb * slot_len);
        KFMM_HIP(hipMemsetAsync(P->q_t_f, 0, sizeof(float) * nb * slot_len, s));
      } else {
        P->q_t = P->arena.get<double>((size_t)nb * slot_len);
        KFMM_HIP(hipMemsetAsync(P->q_t, 0, sizeof(double) * nb * slot_len, s));
      }
    }
    const size_t slot_bytes = std::max<size_t>(1, (size_t)np_ * slot_len) * (o.precision == KFMM_FP64 ? 8 : 4);
    P->m2l_slots = P->arena.alloc(slot_bytes);
    KFMM_HIP(hipMemsetAsync(P->m2l_slots, 0, slot_bytes, s));  // rows past a pair's rank stay zero
    // column tiles: 128 (FP32 and split FP16; 160 x 128 workgroup tiles for the split-FP16 compressed
    // contraction when its rank is a multiple of 160), 64 otherwise
    const int m2l_cols = fp32m2l || split16 ? 2 * kGemmBN : kGemmBN;
    // split FP16 with the compressed M2L: every tile carries its offset's rank (k_gemm_h3)
    P->job_m2l = upload_job(P->arena, sc, s, m2l_cols, (split16 || comp64) && P->comp ? &P->comp->rank_o : nullptr);
    if (split16) {
      ensure_split_ops(*P->ops, P->comp.get(), s);
      // a leaf's downward check potential is only ever multiplied by fd1, so that factor can ride on the
      // products that form it, unless something else adds to it: X lists of a leaf, or a periodic root
      // that is a leaf (its far images)
      bool fold = P->comp != nullptr && D.NC <= 1024;
      for (int b2 : x_boxes) fold = fold && !t.h_is_leaf[b2];
      if (P->periodic)
        for (int b2 = t.level_start[0]; b2 < t.level_start[1]; ++b2) fold = fold && !t.h_is_leaf[b2];
      if (fold) ensure_fold_ops(*P->ops, P->comp.get(), s);
      P->fold_fd1 = fold;
      P->phi_h3 = P->arena.get<uint16_t>((size_t)nb * 2 * slot_len);
      P->phi_h3_scale = P->arena.get<float>(std::max(nb, 1));
      // NC-wide split rows per box: check potentials for the translations, phi_up for the U^T projection
      P->phi_up_h3 = P->arena.get<uint16_t>((size_t)nb * 2 * D.NC);
      P->phi_up_h3_scale = P->arena.get<float>(std::max(nb, 1));
    }
    P->n_v_pairs = (int64_t)c.op.size();
    if (std::getenv("KFMM_DEBUG_STATS")) {  // occupancy of target-box blocks x offsets (design statistics)
      for (int bs : {16, 32, 64}) {
        std::vector<int> tb;  // target boxes with V lists, in tree order
        std::vector<std::vector<int>> offs(nb);
        for (size_t i = 0; i < t.h_v_trg.size(); ++i) offs[t.h_v_trg[i]].push_back(D.m2l_index[t.h_v_off[i]]);
        for (int b2 = 0; b2 < nb; ++b2)
          if (!offs[b2].empty()) tb.push_back(b2);
        long cells = 0;
        for (size_t i = 0; i < tb.size(); i += bs) {
          std::vector<char> u(316, 0);
          for (size_t j = i; j < std::min(tb.size(), i + bs); ++j)
            for (int o2 : offs[tb[j]]) u[o2] = 1;
          int cnt = 0;
          for (char x2 : u) cnt += x2;
          cells += (long)cnt * bs;
        }
        std::fprintf(stderr, "[kfmm stats] V pairs %zu, target boxes %zu, block %d: offset-union cells %ld, fill %.3f\n",
                     t.h_v_trg.size(), tb.size(), bs, cells, (double)t.h_v_trg.size() / std::max(1L, cells));
      }
    }
  }
  // DC2DE over all boxes with targets at level >= lv0; L2L per level >= lv0 + 1
  {
    GemmCols c;
    for (int b = 0; b < nb; ++b)
      if (t.h_level[b] >= lv0 && ht(b)) c.add(P->fold_fd1 && t.h_is_leaf[b] ? 1 : 0, b, b);
    P->job_dc2de = upload_job(P->arena, sorted_by_op(c), s, wide(c));
    if (P->f32t) {  // DC2DE at the leaves only: the downward pass carries check potentials
      GemmCols cl;
      for (int b : leaves_trg)
        if (t.h_level[b] >= lv0) cl.add(0, b, b);
      P->job_dn_leaf = upload_job(P->arena, cl, s, wide(cl));
    }
    // compressed M2L: the X-list check potentials get DC2DE on their own (added after DC2DE * U q~)
    if (P->comp) {
      GemmCols cx;
      for (int i = 0; i < (int)x_boxes.size(); ++i)
        if (t.h_level[x_boxes[i]] >= lv0 && ht(x_boxes[i])) cx.add(0, i, x_boxes[i]);
      P->job_dcx = upload_job(P->arena, cx, s, wide(cx));
    }
    P->dn_levels.clear();
    P->dn_lv.clear();
    for (int l = lv0 + 1; l <= t.depth; ++l) {
      GemmCols cl;
      for (int b = t.level_start[l]; b < t.level_start[l + 1]; ++b)
        if (ht(b)) cl.add(octant(b) + (P->fold_fd1 && t.h_is_leaf[b] ? 8 : 0), t.h_parent[b], b);
      if (cl.op.empty()) continue;
      P->dn_levels.push_back(upload_job(P->arena, sorted_by_op(cl), s, wide(cl)));
      P->dn_lv.push_back(l);
    }
  }
  // periodic cells: the images beyond the 3 x 3 x 3 block act on each root through one operator, added
  // to the root's downward check potential like an M2L (unit half-width frame, so no per-box scale)
  if (P->periodic) {
    ensure_periodic_ops(*P->ops, p, P->el, P->f32t, !P->f32t && P->comp != nullptr);
    GemmCols c, cc;
    for (int b = t.level_start[0]; b < t.level_start[1]; ++b)
      if (hs(b) && ht(b)) {
        c.add(0, b, b);
        cc.add(0, b, (int)cc.op.size());  // into compact row i (check-potential form)
      }
    P->job_per = upload_job(P->arena, c, s);
    P->job_per_c = upload_job(P->arena, cc, s);
    if (P->f32t) P->per_tmp_f = P->arena.get<float>(std::max<size_t>(1, cc.op.size()) * NC);
    // cell-mean constant of the displacement: roots with sources and targets, their sources in chunks
    std::vector<int> roots, coff = {0}, tb_, te_, cb, ce, cr;
    const int kChunk = 8192;
    for (int b = t.level_start[0]; b < t.level_start[1]; ++b) {
      if (!hs(b) || !ht(b)) continue;
      const int g = t.h_geom[b];
      const std::vector<int64_t>& bt2 = P->alias ? bs : bt;
      roots.push_back(b);
      tb_.push_back((int)bt2[g]);
      te_.push_back((int)bt2[g + 1]);
      for (int i0 = t.h_src_b[b]; i0 < t.h_src_e[b]; i0 += kChunk) {
        cb.push_back(i0);
        ce.push_back(std::min(i0 + kChunk, t.h_src_e[b]));
        cr.push_back(b);
      }
      coff.push_back((int)cb.size());
    }
    P->per_n_roots = (int)roots.size();
    P->per_n_chunks = (int)cb.size();
    P->per_root = upload_vec(P->arena, roots, s);
    P->per_chunk_off = upload_vec(P->arena, coff, s);
    P->per_trg_b = upload_vec(P->arena, tb_, s);
    P->per_trg_e = upload_vec(P->arena, te_, s);
    P->per_chunk_b = upload_vec(P->arena, cb, s);
    P->per_chunk_e = upload_vec(P->arena, ce, s);
    P->per_chunk_root = upload_vec(P->arena, cr, s);
    P->per_part = P->arena.get<double>(6 * (size_t)std::max(1, P->per_n_chunks));
    P->per_eqm = P->arena.get<double>(6 * (size_t)std::max(1, P->per_n_roots));
  }
  // W pairs and their output slots
  {
    std::vector<int> pb, pa;
    std::vector<signed char> ps;
    std::vector<int64_t> off;
    int64_t tot = 0;
    for (int b = 0; b < nb; ++b)
      for (int k = t.h_w_off[b]; k < t.h_w_off[b + 1]; ++k) {
        pb.push_back(b);
        pa.push_back(t.h_w_idx[k]);
        ps.push_back(t.h_w_sh[k]);
        off.push_back(tot);
        tot += (int64_t)(t.h_trg_e[b] - t.h_trg_b[b]) * 6;
      }
    P->n_wp = (int)pb.size();
    P->wp_b = upload_vec(P->arena, pb, s);
    P->wp_a = upload_vec(P->arena, pa, s);
    P->wp_s = upload_vec(P->arena, ps, s);
    P->wslot_off = upload_vec(P->arena, off, s);
    P->wslot = P->arena.get<double>(std::max<int64_t>(tot, 1));
  }
  // ---- counters
  int64_t up = 0;
  for (int b : leaves_trg)
    for (int k = t.h_u_off[b]; k < t.h_u_off[b + 1]; ++k) {
      int A = t.h_u_idx[k];
      up += (int64_t)(t.h_trg_e[b] - t.h_trg_b[b]) * (t.h_src_e[A] - t.h_src_b[A]);
    }
  P->n_u_pairs = up;
  P->n_w_pairs = (int64_t)t.h_w_idx.size();
  P->n_x_pairs = (int64_t)t.h_x_idx.size();
  {  // X pairs in list order (grouped by box in x_boxes order) and their per-box reduction
    std::vector<int> xb, xa, roff = {0}, ridx, rbox;
    std::vector<signed char> xs;
    for (int i = 0; i < (int)x_boxes.size(); ++i) {
      const int b = x_boxes[i];
      for (int k = t.h_x_off[b]; k < t.h_x_off[b + 1]; ++k) {
        ridx.push_back((int)xb.size());
        xb.push_back(b);
        xa.push_back(t.h_x_idx[k]);
        xs.push_back(t.h_x_sh[k]);
      }
      rbox.push_back(i);
      roff.push_back((int)xb.size());
    }
    P->n_xp = (int)xb.size();
    P->xp_b = upload_vec(P->arena, xb, s);
    P->xp_a = upload_vec(P->arena, xa, s);
    P->xp_s = upload_vec(P->arena, xs, s);
    P->xr_box = upload_vec(P->arena, rbox, s);
    P->xr_off = upload_vec(P->arena, roff, s);
    P->xr_idx = upload_vec(P->arena, ridx, s);
  }
  P->n_leaf = 0;
  for (int b = 0; b < nb; ++b) P->n_leaf += t.h_is_leaf[b];
  // ---- work buffers (zeroed once; padding rows stay zero)
  auto zalloc = [&](size_t bytes) {
    void* p = P->arena.alloc(bytes);
    KFMM_HIP(hipMemsetAsync(p, 0, bytes, s));
    return p;
  };
  const size_t nbc = (size_t)nb * NC;
  const size_t nxc = std::max<size_t>(1, (size_t)P->n_x_boxes * NC);
  P->xslot = zalloc(std::max<size_t>(1, (size_t)P->n_xp * NC) * (P->f32t ? 4 : 8));
  if (P->f32t) {
    P->q_f = (float*)zalloc(nbc * 4);
    P->tmp_f = (float*)zalloc(nbc * 4);
    if (P->comp && o.precision == KFMM_FP32_M2L_SPLIT16) P->tmp_w = (float*)zalloc(nbc * 4);
    P->qx_f = (float*)zalloc(nxc * 4);  // padding rows stay zero
  } else {
    P->q_up = (double*)zalloc(nbc * 8);
    P->phi_up = (double*)zalloc(nbc * 8);
    P->phi_dn = (double*)zalloc(nbc * 8);
    P->tmp = (double*)zalloc(nbc * 8);
    P->qx = (double*)zalloc(nxc * 8);  // padding rows stay zero
  }
  if (!f64) {
    P->phi_up_lo = zalloc(nbc * 4);
    P->phi_dn_lo = zalloc(nbc * 4);
  }
  KFMM_HIP(hipStreamCreateWithFlags(&P->near_stream, hipStreamNonBlocking));
  for (hipEvent_t* e : {&P->fork_ev, &P->phi_ev, &P->x_ev, &P->join_ev, &P->wq_ev})
    KFMM_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  KFMM_HIP(hipStreamSynchronize(s));
  P->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return P.release();
}

// ------------------------------------------------------------------------------------------ eval

// Sums the phase times of a profiled evaluation (events recorded on the evaluation stream).
static void finish_profile(Plan& P) {
  if (!P.prof) return;
  KFMM_HIP(hipEventSynchronize(P.ev[KFMM_N_PHASES]));
  for (int ph = 0; ph < KFMM_N_PHASES; ++ph) {
    float ms = 0;
    KFMM_HIP(hipEventElapsedTime(&ms, P.ev[ph], P.ev[ph + 1]));
    P.phase_ms[ph] += ms;
  }
  P.prof_calls++;
}

template <typename T>
static void eval_t(Plan& P, int kind, const double* a, const double* b, double* out, hipStream_t s) {
  const Tree& t = P.tree;
  const DeviceOps& D = *P.ops;
  const int NC = P.NC, nb = t.n_box, n_eq = P.n_eq;
  const size_t nbc = (size_t)nb * NC;
  const bool SLa = a != nullptr, DLa = b != nullptr;
  KConst<T> kc(P.el);
  auto mark = [&](int i) {
    if (P.prof) KFMM_HIP(hipEventRecord(P.ev[i], s));
  };
  int light_slot = -1;
  auto m2l_begin = [&]() {
    if (!P.light) return;
    if (P.lev_count == Plan::kLightRing) plan_light_harvest(P, false);
    light_slot = (P.lev_head + P.lev_count) % Plan::kLightRing;
    KFMM_HIP(hipEventRecord(P.lev[2 * light_slot], s));
  };
  auto m2l_end = [&]() {
    if (light_slot < 0) return;
    KFMM_HIP(hipEventRecord(P.lev[2 * light_slot + 1], s));
    P.lev_count++;
  };
  // Launches with the single/double-layer variant chosen by which densities are given.
  auto dispatch = [&](auto&& launch) {
    if (SLa && DLa)
      launch(std::true_type(), std::true_type());
    else if (SLa)
      launch(std::true_type(), std::false_type());
    else
      launch(std::false_type(), std::true_type());
    KFMM_HIP(hipGetLastError());
  };
  mark(KFMM_PH_PERMUTE);
  hipLaunchKernelGGL(k_permute_in<T>, dim3((unsigned)((P.n_src + 255) / 256)), dim3(256), 0, s, P.n_src,
                     t.perm_src, P.sw, a, b, (T*)P.dens);
  KFMM_HIP(hipGetLastError());
  const T* spos = (const T*)P.spos;
  const T* snrm = (const T*)P.snrm;
  const T* dens = (const T*)P.dens;
  const bool far = nb > 1 || P.periodic;  // a periodic cell always has far images
  const T* phi_dn = P.prec == KFMM_FP64 ? (const T*)P.phi_dn : (const T*)P.phi_dn_lo;
  const T* phi_up = P.prec == KFMM_FP64 ? (const T*)P.phi_up : (const T*)P.phi_up_lo;
  // leaf evaluation: parts = 1 far field (L2T + W slots, added to out), 2 near field (U lists, stored)
  auto leaf_eval = [&](int parts, hipStream_t st) {
    auto launch = [&](auto kd, auto sl, auto dl) {
      constexpr int KIND = decltype(kd)::value;
      constexpr bool SL = decltype(sl)::value, DL = decltype(dl)::value;
      hipLaunchKernelGGL((k_leaf_eval<T, KIND, SL, DL>), dim3(P.n_leaves_trg), dim3(256), 0, st, P.leaves_trg, P.tv,
                         t.u_off, t.u_idx, (const signed char*)t.u_sh, t.w_off, P.wslot_off, P.wslot, spos, snrm,
                         dens, (const T*)P.tpos,
                         t.perm_trg, phi_dn, phi_up, D.surf, n_eq, 1.05, 2.95, NC, parts & 1, (parts >> 1) & 1,
                         parts & 1, kc, out);
    };
    if (kind == KFMM_DISP)
      dispatch([&](auto sl, auto dl) { launch(std::integral_constant<int, 0>(), sl, dl); });
    else
      dispatch([&](auto sl, auto dl) { launch(std::integral_constant<int, 1>(), sl, dl); });
  };
  mark(KFMM_PH_S2M);
  if (!far) {  // one box: near field only
    for (int ph = KFMM_PH_UC2UE; ph <= KFMM_PH_NEAR; ++ph) mark(ph);
    leaf_eval(2, s);
    mark(KFMM_PH_LEAF);
    mark(KFMM_N_PHASES);
    finish_profile(P);
    return;
  }
  // Work that needs no translation result (near field, X lists) and the W lists run, unprofiled, on the
  // plan's second stream: the near field and the X lists from the start (after the permutation),
  // overlapping S2M and the latency-bound M2M levels; the W lists once phi_up is ready.  Profiled calls run
  // everything here in phase order.
  const bool overlap = !P.prof;
  hipStream_t side = overlap ? P.near_stream : s;
  auto fork = [&](hipEvent_t e) {
    if (!overlap) return;
    KFMM_HIP(hipEventRecord(e, s));
    KFMM_HIP(hipStreamWaitEvent(side, e, 0));
  };
  const int check_block = std::max(64, round_up(n_eq, 64));  // one thread per check point
  auto s2l = [&](hipStream_t st) {  // X pairs -> per-pair rows, summed per box (list order) into qx
    if (!P.n_x_boxes) return;
    dispatch([&](auto sl, auto dl) {
      constexpr bool SL = decltype(sl)::value, DL = decltype(dl)::value;
      if (P.f32t)
        hipLaunchKernelGGL((k_check_eval<T, float, SL, DL, false>), dim3(P.n_xp), dim3(check_block), 0, st, P.xp_b,
                           P.tv, t.x_off, t.x_idx, spos, snrm, dens, D.surf, n_eq, 1.05, NC, kc, (float*)P.xslot, 0,
                           P.xp_a, (uint16_t*)nullptr, (float*)nullptr, (const signed char*)P.xp_s);
      else
        hipLaunchKernelGGL((k_check_eval<T, double, SL, DL, false>), dim3(P.n_xp), dim3(check_block), 0, st,
                           P.xp_b, P.tv, t.x_off, t.x_idx, spos, snrm, dens, D.surf, n_eq, 1.05, NC, kc,
                           (double*)P.xslot, 0, P.xp_a, (uint16_t*)nullptr, (float*)nullptr,
                           (const signed char*)P.xp_s);
    });
    if (P.f32t)
      hipLaunchKernelGGL((k_slot_reduce<float, float>), dim3(P.n_x_boxes), dim3(reduce_block<float>(NC)), 0, st,
                         P.xr_box, P.xr_off, P.xr_idx, (const float*)P.xslot, P.qx_f, NC);
    else
      hipLaunchKernelGGL((k_slot_reduce<double, double>), dim3(P.n_x_boxes), dim3(reduce_block<double>(NC)), 0, st,
                         P.xr_box, P.xr_off, P.xr_idx, (const double*)P.xslot, P.qx, NC);
    KFMM_HIP(hipGetLastError());
  };
  auto w_eval = [&](hipStream_t st) {
    if (!P.n_wp) return;
    if (kind == KFMM_DISP)
      hipLaunchKernelGGL((k_w_eval<T, 0>), dim3(P.n_wp), dim3(256), 0, st, P.wp_b, P.wp_a,
                         (const signed char*)P.wp_s, P.wslot_off, P.tv,
                         (const T*)P.tpos, phi_up, D.surf, n_eq, 1.05, NC, kc, P.wslot);
    else
      hipLaunchKernelGGL((k_w_eval<T, 1>), dim3(P.n_wp), dim3(256), 0, st, P.wp_b, P.wp_a,
                         (const signed char*)P.wp_s, P.wslot_off, P.tv,
                         (const T*)P.tpos, phi_up, D.surf, n_eq, 1.05, NC, kc, P.wslot);
    KFMM_HIP(hipGetLastError());
  };
  // the near field and the X lists need only the points: on the second stream from here
  fork(P.fork_ev);
  if (overlap) {
    leaf_eval(2, side);
    s2l(side);
    KFMM_HIP(hipEventRecord(P.x_ev, side));
  }
  // S2M, UC2UE
  const bool split16 = P.prec == KFMM_FP32_M2L_SPLIT16;
  uint16_t* const xq = P.phi_up_h3;  // split16: NC-wide split rows (check potentials, later phi_up)
  float* const xq_scale = P.phi_up_h3_scale;
  dispatch([&](auto sl, auto dl) {
    constexpr bool SL = decltype(sl)::value, DL = decltype(dl)::value;
    if (P.f32t)  // scaled check potentials qhat = r q; split16: the leaves' split rows too
      hipLaunchKernelGGL((k_check_eval<T, float, SL, DL, true>), dim3(P.n_leaves_src), dim3(check_block), 0, s,
                         P.leaves_src, P.tv, (const int*)nullptr, (const int*)nullptr, spos, snrm, dens, D.surf, n_eq,
                         2.95, NC, kc, P.q_f, 1, (const int*)nullptr, split16 ? xq : nullptr,
                         split16 ? xq_scale : nullptr);
    else
      hipLaunchKernelGGL((k_check_eval<T, double, SL, DL, true>), dim3(P.n_leaves_src), dim3(check_block), 0, s,
                         P.leaves_src, P.tv, (const int*)nullptr, (const int*)nullptr, spos, snrm, dens, D.surf, n_eq,
                         2.95, NC, kc, P.q_up);
  });
  mark(KFMM_PH_UC2UE);
  // split16: the split rows read next are the leaves' (written by S2M above) and the parents' (written by
  // the M2M reductions below); the rows of leaves without sources are never read
  // split-FP16 products pay off on launches of a dozen column tiles or more; smaller ones (the upper levels)
  // run the FP32 split-K kernel, which cuts K across more workgroups
  auto big = [](const GemmJob& J) { return J.n_tiles >= 12; };
  // the 1/sigma-scaled split pass handles rows of up to 1024 values (p <= 8); beyond, fu2 / fd2 / G in FP32
  const bool sig_split = split16 && NC <= 1024;
  float* const phi_up_f = (float*)P.phi_up_lo;
  float* const phi_dn_f = (float*)P.phi_dn_lo;
  // FP32 translations: UC2UE runs after the M2M chain, for every box at once (in the M2M phase)
  if (!P.f32t) gemm_f64(P.job_uc2ue, D.uc2ue, GemmDims::Sq(NC), P.q_up, P.phi_up, kStore, s);
  // M2M
  mark(KFMM_PH_M2M);
  for (const UpLevel& U : P.up_levels) {
    if (P.f32t) {  // qhat_up(parent) = sum_c M2M_q_c qhat_up(child); split16: parents' split rows too
      // (split16: every level as split products, the children's split rows already written by S2M and by the
      // reduction of the level below)
      if (split16)
        gemm_h3(U.job, D.m2mq_h3, D.m2mq_h3_scale, GemmDims{NC, NC, 2 * NC, NC}, xq, xq_scale, P.tmp_f, kStore, s);
      else
        gemm_f32(U.job, D.m2mq32, GemmDims::Sq(NC), P.q_f, P.tmp_f, kStore, s);
      if (U.n_par)
        hipLaunchKernelGGL(k_m2m_reduce<float>, dim3(U.n_par), dim3(reduce_block<float>(NC)), 0, s, U.parents,
                           U.n_par, t.child_first, t.child_count, t.src_b, t.src_e, P.tmp_f, P.q_f, NC,
                           split16 ? xq : nullptr, split16 ? xq_scale : nullptr);
    } else {
      gemm_f64(U.job, D.m2m, GemmDims::Sq(NC), P.phi_up, P.tmp, kStore, s);
      if (U.n_par)
        hipLaunchKernelGGL(k_m2m_reduce<double>, dim3(U.n_par), dim3(reduce_block<double>(NC)), 0, s, U.parents,
                           U.n_par, t.child_first, t.child_count, t.src_b, t.src_e, P.tmp, P.phi_up, NC);
    }
  }
  // split FP16 with the compressed M2L: the M2L input phi~ = (U^T UC2UE) qhat comes in one product from the
  // split check-potential rows (M2L prep below), and the full phi_up of the W-list source boxes, which only
  // the W lists read, is made on the second stream (FP32 fu1 then fu2) ahead of the W evaluation
  const bool merged = split16 && P.comp && P.tmp_w && sig_split;
  if (merged) {
    fork(P.phi_ev);
    gemm_f32(P.job_up_w, D.fu1, GemmDims::Sq(NC), P.q_f, P.tmp_w, kStore, side);
    if (overlap) KFMM_HIP(hipEventRecord(P.wq_ev, side));
    gemm_f32(P.job_up_w, D.fu2, GemmDims::Sq(NC), P.tmp_w, phi_up_f, kStore, side);
  } else if (P.f32t) {  // phi_up = UC2UE qhat_up = fu2 (fu1 qhat_up); fu1 is orthogonal (split16 products)
    if (split16)
      gemm_h3(P.job_up_all, D.fu1_h3, D.fu1_h3_scale, GemmDims{NC, NC, 2 * NC, NC}, xq, xq_scale, P.tmp_f, kStore,
              s);
    else
      gemm_f32(P.job_up_all, D.fu1, GemmDims::Sq(NC), P.q_f, P.tmp_f, kStore, s);
    // fu2: every box for the dense M2L, the W-list boxes only with the compressed one (tmp_f keeps fu1 qhat).
    // split16: fu2 = vs diag(inv_sig), with 1/sigma applied in the split pass and vs as split products
    const GemmJob& J2 = P.comp ? P.job_up_w : P.job_up_all;
    if (sig_split) split_h3(P.tmp_f, nb, NC, NC, xq, xq_scale, s, D.inv_sig32);  // also the input of Gv
    if (sig_split && big(J2))
      gemm_h3(J2, D.vs_h3, D.vs_h3_scale, GemmDims{NC, NC, 2 * NC, NC}, xq, xq_scale, phi_up_f, kStore, s);
    else  // a few W boxes: the FP32 split-K kernel is faster
      gemm_f32(J2, D.fu2, GemmDims::Sq(NC), P.tmp_f, phi_up_f, kStore, s);
  }
  KFMM_HIP(hipGetLastError());
  // periodic cells: the root's upward quantities are read before the M2L and the downward pass reuse their
  // buffers -- the equivalent density's moments (cell-mean constant) and, with FP32 translations, the far
  // images' check potential (T UC2UE) qhat_up, added back at the start of the downward pass
  if (P.periodic && P.per_n_roots) {
    if (P.f32t) {
      hipLaunchKernelGGL(k_per_eqm<float>, dim3(P.per_n_roots), dim3(256), 0, s, P.per_root, D.per_mom_q,
                         (const float*)P.q_f, NC, P.tv, P.per_eqm);
      gemm_f32(P.job_per_c, D.per_farq32, GemmDims::Sq(NC), P.q_f, P.per_tmp_f, kStore, s);
    } else {
      hipLaunchKernelGGL(k_per_eqm<double>, dim3(P.per_n_roots), dim3(256), 0, s, P.per_root, D.per_mom_phi,
                         (const double*)P.phi_up, NC, P.tv, P.per_eqm);
    }
    KFMM_HIP(hipGetLastError());
  }
  // M2L into qhat.  qhat is FP64 in every precision; each box's M2L slots are summed in a fixed order,
  // so repeated products of one operator are bitwise identical (GMRES sees a fixed operator).
  mark(KFMM_PH_M2L_PREP);
  double* qhat = P.q_up;  // reuse: the S2M potentials are consumed (FP64 translations)
  float* qhat_f = P.q_f;  // the same with FP32 translations
  const bool fp32m2l = P.prec == KFMM_FP32 || P.prec == KFMM_FP32_TRANS64;
  const bool comp64 = P.prec == KFMM_FP64 && P.comp;          // FP64 contractions on the basis
  const bool fused_down = (fp32m2l || split16 || comp64) && P.comp;  // DC2DE * U applied to q~ (no qhat)
  if (!fused_down) {
    if (P.f32t)
      hipLaunchKernelGGL(k_fill_zero<float>, dim3((unsigned)((nbc + 255) / 256)), dim3(256), 0, s, (int64_t)nbc,
                         qhat_f);
    else
      hipLaunchKernelGGL(k_fill_zero<double>, dim3((unsigned)((nbc + 255) / 256)), dim3(256), 0, s, (int64_t)nbc,
                         qhat);
  }
  if (P.prec != KFMM_FP64 && !P.f32t)
    hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)((nbc + 255) / 256)), dim3(256), 0, s,
                       (int64_t)nbc, P.phi_up, (float*)P.phi_up_lo);
  KFMM_HIP(hipGetLastError());
  if (!merged) fork(P.phi_ev);  // phi_up ready in the evaluation precision
  if (overlap) {
    w_eval(side);
    KFMM_HIP(hipEventRecord(P.join_ev, side));
  }
  if (P.prec == KFMM_FP64 && !comp64) {  // dense FP64 M2L: slots of NC values, tiles without a rank
    KFMM_REQUIRE(!P.job_m2l.ranked, "internal: dense FP64 M2L with ranked tiles");
    mark(KFMM_PH_M2L);
    m2l_begin();
    gemm_f64(P.job_m2l, D.m2l64, GemmDims::Sq(NC), P.phi_up, (double*)P.m2l_slots, kStore, s);
    m2l_end();
    mark(KFMM_PH_M2L_RED);
    if (P.m2l_red_n)
      hipLaunchKernelGGL((k_slot_reduce<double, double>), dim3(P.m2l_red_n), dim3(reduce_block<double>(NC)), 0, s,
                         P.m2l_red_box, P.m2l_red_off, P.m2l_red_idx, (const double*)P.m2l_slots, qhat, NC);
  } else if (fused_down) {
    const CompressedM2L& C = *P.comp;
    const int NCr = C.NCr;
    if (merged)  // phi~ = (U^T UC2UE) qhat from the split check-potential rows
      gemm_h3(P.job_ut, C.Mu_h3, C.Mu_h3_scale, GemmDims{NCr, NC, 2 * NC, NCr}, xq, xq_scale, P.phi_t, kStore, s);
    else if (sig_split)  // phi~ = Gv (diag(inv_sig) fu1 qhat), the scaled rows split in the UC2UE step above
      gemm_h3(P.job_ut, C.Gv_h3, C.Gv_h3_scale, GemmDims{NCr, NC, 2 * NC, NCr}, xq, xq_scale, P.phi_t, kStore, s);
    else if (P.f32t)  // phi~ = U^T UC2UE qhat = G (fu1 qhat)
      gemm_f32(P.job_ut, C.G32, GemmDims{NCr, NC, NC, NCr}, P.tmp_f, P.phi_t, kStore, s);
    else if (comp64)
      gemm_f64(P.job_ut, C.Ut64, GemmDims{NCr, NC, NC, NCr}, P.phi_up, P.phi_t64, kStore, s);
    else
      gemm_f32(P.job_ut, C.Ut32, GemmDims{NCr, NC, NC, NCr}, (const float*)P.phi_up_lo, P.phi_t, kStore, s);
    if (split16) split_h3(P.phi_t, nb, NCr, NCr, P.phi_h3, P.phi_h3_scale, s);
    mark(KFMM_PH_M2L);
    m2l_begin();
    if (split16)  // tiles of rank r_o: the leading r_o rows of each slot, contraction over r_o
      gemm_h3(P.job_m2l, C.Crk_h3, C.Crk_h3_scale, GemmDims{NCr, NCr, 2 * NCr, NCr}, P.phi_h3, P.phi_h3_scale,
              (float*)P.m2l_slots, kStore, s);
    else if (comp64)  // the same in FP64
      gemm_f64(P.job_m2l, C.Crk64, GemmDims::Sq(NCr), P.phi_t64, (double*)P.m2l_slots, kStore, s);
    else
      gemm_f32(P.job_m2l, C.C32, GemmDims::Sq(NCr), (const float*)P.phi_t, (float*)P.m2l_slots, kStore, s);
    m2l_end();
    mark(KFMM_PH_M2L_RED);
    if (P.m2l_red_n) {
      if (comp64)
        hipLaunchKernelGGL((k_slot_reduce<double, double>), dim3(P.m2l_red_n), dim3(reduce_block<double>(NCr)), 0,
                           s, P.m2l_red_box, P.m2l_red_off, P.m2l_red_idx, (const double*)P.m2l_slots, P.q_t, NCr);
      else if (P.f32t)
        hipLaunchKernelGGL((k_slot_reduce<float, float>), dim3(P.m2l_red_n), dim3(reduce_block<float>(NCr)), 0, s,
                           P.m2l_red_box, P.m2l_red_off, P.m2l_red_idx, (const float*)P.m2l_slots, P.q_t_f, NCr);
      else
        hipLaunchKernelGGL((k_slot_reduce<float, double>), dim3(P.m2l_red_n), dim3(reduce_block<float>(NCr)), 0, s,
                           P.m2l_red_box, P.m2l_red_off, P.m2l_red_idx, (const float*)P.m2l_slots, P.q_t, NCr);
    }
  } else {
    if (fp32m2l) {
      mark(KFMM_PH_M2L);
      m2l_begin();
      gemm_f32(P.job_m2l, D.m2l32, GemmDims::Sq(NC), (const float*)P.phi_up_lo, (float*)P.m2l_slots, kStore, s);
      m2l_end();
    } else if (split16) {
      split_h3((const float*)P.phi_up_lo, nb, NC, NC, P.phi_h3, P.phi_h3_scale, s);
      mark(KFMM_PH_M2L);
      m2l_begin();
      gemm_h3(P.job_m2l, D.m2l_h3, D.m2l_h3_scale, GemmDims{NC, NC, 2 * NC, NC}, P.phi_h3, P.phi_h3_scale,
              (float*)P.m2l_slots, kStore, s);
      m2l_end();
    } else {
      throw Error(KFMM_E_ARG, "unsupported M2L precision");
    }
    mark(KFMM_PH_M2L_RED);
    if (P.m2l_red_n) {
      if (P.f32t)
        hipLaunchKernelGGL((k_slot_reduce<float, float>), dim3(P.m2l_red_n), dim3(reduce_block<float>(NC)), 0, s,
                           P.m2l_red_box, P.m2l_red_off, P.m2l_red_idx, (const float*)P.m2l_slots, qhat_f, NC);
      else
        hipLaunchKernelGGL((k_slot_reduce<float, double>), dim3(P.m2l_red_n), dim3(reduce_block<float>(NC)), 0, s,
                           P.m2l_red_box, P.m2l_red_off, P.m2l_red_idx, (const float*)P.m2l_slots, qhat, NC);
    }
  }
  KFMM_HIP(hipGetLastError());
  // X lists, added to qhat
  mark(KFMM_PH_S2L);
  if (overlap)
    KFMM_HIP(hipStreamWaitEvent(s, P.x_ev, 0));
  else
    s2l(s);
  if (P.n_x_boxes && !fused_down) {
    if (P.f32t)
      hipLaunchKernelGGL(k_add_rows<float>, dim3(P.n_x_boxes), dim3(reduce_block<float>(NC)), 0, s, P.x_boxes,
                         (const float*)P.qx_f, qhat_f, NC);
    else
      hipLaunchKernelGGL(k_add_rows<double>, dim3(P.n_x_boxes), dim3(reduce_block<double>(NC)), 0, s, P.x_boxes,
                         (const double*)P.qx, qhat, NC);
  }
  // periodic cells, FP64 translations on qhat: the far images act on the roots
  if (P.periodic && P.job_per.n_tiles && !P.f32t && !fused_down)
    gemm_f64(P.job_per, D.per_far64, GemmDims::Sq(NC), P.phi_up, qhat, kAdd, s);
  KFMM_HIP(hipGetLastError());
  mark(KFMM_PH_DOWN);
  // the downward pass overwrites the upward check potentials (qhat_f is q_f): wait until the second stream
  // has read the W-list boxes' rows
  if (merged && overlap) KFMM_HIP(hipStreamWaitEvent(s, P.wq_ev, 0));
  if (P.f32t) {
    // downward pass in FP32 on check potentials: qhat = U q~ + X rows (compressed), qhat(child) +=
    // L2L_q qhat(parent) level by level, then phi_dn = DC2DE qhat = fd2 (fd1 qhat) at the target leaves
    // (split16: U, L2L_q and fd1 as split-FP16 products, their inputs split level by level; with fold_fd1
    // the leaves' columns of the U and L2L products use fd1 U and fd1 L2L_q instead)
    if (fused_down) {
      const int NCr = P.comp->NCr;
      if (split16) {
        split_h3(P.q_t_f, nb, NCr, NCr, P.phi_h3, P.phi_h3_scale, s);
        gemm_h3(P.job_dc2de, P.fold_fd1 ? P.comp->UF_h3 : P.comp->U_h3,
                P.fold_fd1 ? P.comp->UF_h3_scale : P.comp->U_h3_scale, GemmDims{NC, NCr, 2 * NCr, NC}, P.phi_h3,
                P.phi_h3_scale, qhat_f, kStore, s);
      } else {
        gemm_f32(P.job_dc2de, P.comp->U32, GemmDims{NC, NCr, NCr, NC}, P.q_t_f, qhat_f, kStore, s);
      }
      if (P.n_x_boxes)
        hipLaunchKernelGGL(k_add_rows<float>, dim3(P.n_x_boxes), dim3(reduce_block<float>(NC)), 0, s, P.x_boxes,
                           (const float*)P.qx_f, qhat_f, NC);
    }
    if (P.periodic && P.per_n_roots)  // the far images' check potential of every root
      hipLaunchKernelGGL(k_add_rows<float>, dim3(P.per_n_roots), dim3(reduce_block<float>(NC)), 0, s, P.per_root,
                         (const float*)P.per_tmp_f, qhat_f, NC);
    for (size_t i = 0; i < P.dn_levels.size(); ++i) {
      if (split16 && big(P.dn_levels[i])) {  // split the parents' level, then qhat(child) += L2L_q qhat(parent)
        const int l = P.dn_lv[i], b0 = t.level_start[l - 1], b1 = t.level_start[l];
        split_h3(qhat_f + (size_t)b0 * NC, b1 - b0, NC, NC, xq + (size_t)b0 * 2 * NC, xq_scale + b0, s);
        gemm_h3(P.dn_levels[i], P.fold_fd1 ? D.l2lq_fold_h3 : D.l2lq_h3,
                P.fold_fd1 ? D.l2lq_fold_h3_scale : D.l2lq_h3_scale, GemmDims{NC, NC, 2 * NC, NC}, xq, xq_scale,
                qhat_f, kAdd, s);
      } else {
        gemm_f32(P.dn_levels[i], P.fold_fd1 ? D.l2lq_fold32 : D.l2lq32, GemmDims::Sq(NC), qhat_f, qhat_f, kAdd, s);
      }
    }
    if (P.fold_fd1) {  // the leaves' rows hold fd1 qhat: 1/sigma in the split pass, then us
      split_h3(qhat_f, nb, NC, NC, xq, xq_scale, s, D.inv_sig32);
      gemm_h3(P.job_dn_leaf, D.us_h3, D.us_h3_scale, GemmDims{NC, NC, 2 * NC, NC}, xq, xq_scale, phi_dn_f, kStore,
              s);
    } else {
      if (split16) {
        split_h3(qhat_f, nb, NC, NC, xq, xq_scale, s);
        gemm_h3(P.job_dn_leaf, D.fd1_h3, D.fd1_h3_scale, GemmDims{NC, NC, 2 * NC, NC}, xq, xq_scale, P.tmp_f,
                kStore, s);
      } else {
        gemm_f32(P.job_dn_leaf, D.fd1, GemmDims::Sq(NC), qhat_f, P.tmp_f, kStore, s);
      }
      if (sig_split) {  // fd2 = us diag(inv_sig): 1/sigma in the split pass, us as split products
        split_h3(P.tmp_f, nb, NC, NC, xq, xq_scale, s, D.inv_sig32);
        gemm_h3(P.job_dn_leaf, D.us_h3, D.us_h3_scale, GemmDims{NC, NC, 2 * NC, NC}, xq, xq_scale, phi_dn_f,
                kStore, s);
      } else {
        gemm_f32(P.job_dn_leaf, D.fd2, GemmDims::Sq(NC), P.tmp_f, phi_dn_f, kStore, s);
      }
    }
  } else {
    // downward pass in FP64
    if (fused_down) {
      const int NCr = P.comp->NCr;
      gemm_f64(P.job_dc2de, P.comp->DU64, GemmDims{NC, NCr, NCr, NC}, P.q_t, P.phi_dn, kStore, s);
      gemm_f64(P.job_dcx, D.dc2de, GemmDims::Sq(NC), P.qx, P.phi_dn, kAdd, s);
      if (P.periodic && P.job_per.n_tiles)  // the far images straight onto the roots' downward densities
        gemm_f64(P.job_per, D.per_fardn64, GemmDims::Sq(NC), P.phi_up, P.phi_dn, kAdd, s);
    } else {
      gemm_f64(P.job_dc2de, D.dc2de, GemmDims::Sq(NC), qhat, P.phi_dn, kStore, s);
    }
    for (const GemmJob& J : P.dn_levels) gemm_f64(J, D.l2l, GemmDims::Sq(NC), P.phi_dn, P.phi_dn, kAdd, s);
    if (P.prec != KFMM_FP64)
      hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)((nbc + 255) / 256)), dim3(256), 0, s,
                         (int64_t)nbc, P.phi_dn, (float*)P.phi_dn_lo);
  }
  KFMM_HIP(hipGetLastError());
  // leaves: near field (already on the side stream when overlapping), W lists, L2T
  mark(KFMM_PH_NEAR);
  if (!overlap) leaf_eval(2, s);
  mark(KFMM_PH_LEAF);
  if (overlap)
    KFMM_HIP(hipStreamWaitEvent(s, P.join_ev, 0));
  else
    w_eval(s);
  leaf_eval(1, s);
  if (P.periodic && kind == KFMM_DISP && P.per_n_roots) {  // zero cell mean (the k = 0 term left out)
    hipLaunchKernelGGL(k_per_moments<T>, dim3(P.per_n_chunks), dim3(256), 0, s, P.per_chunk_root, P.per_chunk_b,
                       P.per_chunk_e, P.tv, t.leaf_of_src, spos, P.has_nrm ? snrm : (const T*)nullptr, dens,
                       P.el.K - 2.0 * P.el.G / 3.0, P.el.G, P.per_part);
    hipLaunchKernelGGL(k_per_shift, dim3(P.per_n_roots), dim3(256), 0, s, P.per_root, P.per_chunk_off, P.per_trg_b,
                       P.per_trg_e, P.per_part, P.tv, (const double*)P.per_eqm, P.el.nu, P.el.G, out);
    KFMM_HIP(hipGetLastError());
  }
  mark(KFMM_N_PHASES);
  finish_profile(P);
}

Plan::~Plan() {
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : lev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {fork_ev, phi_ev, x_ev, join_ev, wq_ev})
    if (e) (void)hipEventDestroy(e);
  if (near_stream) (void)hipStreamDestroy(near_stream);
}

int plan_m2l_rank(const Plan& P) { return P.comp ? P.comp->r : 0; }

// Algorithmic work of one evaluation per phase: the floating-point operations and HBM bytes the method
// itself needs (operand dimensions without the GEMM padding, each operator and each coefficient vector
// read once, each result written once), not what the kernels execute.  Kernel-pair costs per point pair,
// counted from the closed forms of eqs. disp_1, disp_2, stress_2, stress_3: U 29, P 45, U+P 65, D 50,
// S 90, D+S 130 (one reciprocal square root each).  The per-pair M2L slots and their reduction are a
// design choice of this library, so the reduction phase carries no algorithmic work.
void plan_work(const Plan& P, int kind, bool sl, bool dl, double* flops, double* bytes) {
  for (int i = 0; i < KFMM_N_PHASES; ++i) flops[i] = bytes[i] = 0.0;
  if (P.empty || P.n_trg == 0 || (!sl && !dl)) return;
  const Tree& t = P.tree;
  const double n = 3.0 * P.n_eq, neq = P.n_eq;
  const bool f32t = P.f32t, comp = P.comp != nullptr;
  // bytes per coefficient of the translations and of the M2L (split FP16: hi + lo, 4 bytes)
  const double vb = f32t ? 4.0 : 8.0;
  const double mb = P.prec == KFMM_FP64 ? 8.0 : 4.0;
  const double r = comp ? (double)P.comp->r : n;
  const double f_src = sl && dl ? (kind == KFMM_DISP ? 65 : 130) : sl ? (kind == KFMM_DISP ? 29 : 50)
                                                                     : (kind == KFMM_DISP ? 45 : 90);
  const double f_s2m = sl && dl ? 65 : sl ? 29 : 45;  // sources at check points (displacement kernels)
  const double f_l2t = kind == KFMM_DISP ? 29 : 50;   // single-layer equivalent densities at targets
  const double n_src = (double)P.n_src, n_trg = (double)P.n_trg;
  const double dens_in = 3.0 * ((sl ? 1 : 0) + (dl ? 1 : 0));
  flops[KFMM_PH_PERMUTE] = 0;
  bytes[KFMM_PH_PERMUTE] = n_src * (8.0 * dens_in + 8.0 + 4.0 + (P.prec == KFMM_FP64 ? 8.0 : 4.0) * dens_in);
  // box classes
  const int nb = t.n_box;
  double n_up = 0, n_up_child = 0, n_dn = 0, n_dn_child = 0, n_tleaf = 0, src_in_leaves = 0;
  for (int b = 0; b < nb; ++b) {
    const bool hs = t.h_src_e[b] > t.h_src_b[b], ht = t.h_trg_e[b] > t.h_trg_b[b];
    if (hs && t.h_level[b] >= 2) {
      n_up += 1;
      if (t.h_level[b] >= 3) n_up_child += 1;
    }
    if (ht && t.h_level[b] >= 2) {
      n_dn += 1;
      if (t.h_level[b] >= 3) n_dn_child += 1;
    }
    if (t.h_is_leaf[b] && ht) n_tleaf += 1;
    if (t.h_is_leaf[b] && hs) src_in_leaves += t.h_src_e[b] - t.h_src_b[b];
  }
  std::vector<char> vsrc(nb, 0), vtrg(nb, 0), wsrc(nb, 0);
  for (size_t i = 0; i < t.h_v_src.size(); ++i) vsrc[t.h_v_src[i]] = vtrg[t.h_v_trg[i]] = 1;
  double n_vsrc = 0, n_vtrg = 0, n_wsrc = 0, w_pts = 0, x_pts = 0;
  for (int b = 0; b < nb; ++b) {
    n_vsrc += vsrc[b];
    n_vtrg += vtrg[b];
    for (int i = t.h_w_off[b]; i < t.h_w_off[b + 1]; ++i) {
      wsrc[t.h_w_idx[i]] = 1;
      w_pts += t.h_trg_e[b] - t.h_trg_b[b];
    }
    for (int i = t.h_x_off[b]; i < t.h_x_off[b + 1]; ++i) {
      const int a = t.h_x_idx[i];
      x_pts += t.h_src_e[a] - t.h_src_b[a];
    }
  }
  for (int b = 0; b < nb; ++b) n_wsrc += wsrc[b];
  const double pt_bytes = (P.prec == KFMM_FP64 ? 8.0 : 4.0) * (6.0 + dens_in);  // position, normal, densities
  // a product of an (rows x cols) operator with `cnt` vectors
  auto gemm = [&](int ph, double rows, double cols, double cnt, double ob) {
    flops[ph] += 2.0 * rows * cols * cnt;
    bytes[ph] += rows * cols * ob + cnt * (rows + cols) * vb;
  };
  const double ob = vb;  // operators in the evaluation precision (split FP16: 4 bytes per value)
  flops[KFMM_PH_S2M] = src_in_leaves * neq * f_s2m;
  bytes[KFMM_PH_S2M] = src_in_leaves * pt_bytes + n_up * n * vb;
  if (f32t) {
    gemm(KFMM_PH_M2M, n, n, n_up_child, 8 * ob);  // M2M_q, children into parents
    gemm(KFMM_PH_M2M, n, n, n_up, ob);            // fu1
    gemm(KFMM_PH_M2M, n, n, comp ? n_wsrc : n_up, ob);  // fu2 (compressed: W-list source boxes only)
  } else {
    gemm(KFMM_PH_UC2UE, n, n, n_up, ob);
    gemm(KFMM_PH_M2M, n, n, n_up_child, 8 * ob);
  }
  if (comp) gemm(KFMM_PH_M2L_PREP, r, n, n_up, ob);  // phi~ = U^T phi_up
  if (comp && (P.prec == KFMM_FP32_M2L_SPLIT16 || P.prec == KFMM_FP64)) {  // per-offset ranks: r_o^2 per pair
    const CompressedM2L& C = *P.comp;
    double f = 0, ob2 = 0;
    for (size_t i = 0; i < t.h_v_off.size(); ++i) {
      const double m = C.rank_o[P.ops->m2l_index[t.h_v_off[i]]];
      f += 2.0 * m * m;
    }
    for (int m : C.rank_o) ob2 += (double)m * m * mb;
    flops[KFMM_PH_M2L] = f;
    bytes[KFMM_PH_M2L] = ob2 + (n_vsrc + n_vtrg) * r * mb;
  } else {
    flops[KFMM_PH_M2L] = 2.0 * r * r * (double)P.n_v_pairs;
    bytes[KFMM_PH_M2L] = 316.0 * r * r * mb + (n_vsrc + n_vtrg) * r * mb;
  }
  flops[KFMM_PH_S2L] = x_pts * neq * f_s2m;
  bytes[KFMM_PH_S2L] = x_pts * pt_bytes;
  if (comp) gemm(KFMM_PH_DOWN, n, r, n_vtrg, ob);  // qhat = U q~
  else if (!f32t) gemm(KFMM_PH_DOWN, n, n, n_dn, ob);  // DC2DE per box (FP64 translations)
  gemm(KFMM_PH_DOWN, n, n, n_dn_child, 8 * ob);       // L2L, parents into children
  if (f32t) {
    if (!P.fold_fd1) gemm(KFMM_PH_DOWN, n, n, n_tleaf, ob);  // fd1 (folded into U and L2L_q otherwise)
    gemm(KFMM_PH_DOWN, n, n, n_tleaf, ob);  // fd2
  }
  flops[KFMM_PH_NEAR] = (double)P.n_u_pairs * f_src;
  bytes[KFMM_PH_NEAR] = (n_src + n_trg) * pt_bytes + n_trg * 8.0 * (kind == KFMM_DISP ? 3 : 6);
  flops[KFMM_PH_LEAF] = (n_trg + w_pts) * neq * f_l2t;
  bytes[KFMM_PH_LEAF] = n_tleaf * n * vb + (n_wsrc) * n * vb + n_trg * 8.0 * (kind == KFMM_DISP ? 3 : 6);
}

void plan_profile(Plan& P, int mode) {
  if (P.light) plan_light_harvest(P, true);
  if (mode == 1 && !P.ev[0])
    for (auto& e : P.ev) KFMM_HIP(hipEventCreate(&e));
  if (mode == 2 && !P.lev[0])
    for (auto& e : P.lev) KFMM_HIP(hipEventCreate(&e));
  P.prof = mode == 1;
  P.light = mode == 2;
  if (mode != 0) {
    for (double& v : P.phase_ms) v = 0;
    P.prof_calls = 0;
  }
}

// Adds the elapsed times of recorded M2L event pairs (the oldest one, or all) to the M2L phase.
void plan_light_harvest(Plan& P, bool all) {
  while (P.lev_count > 0) {
    const int i = P.lev_head;
    KFMM_HIP(hipEventSynchronize(P.lev[2 * i + 1]));
    float ms = 0;
    KFMM_HIP(hipEventElapsedTime(&ms, P.lev[2 * i], P.lev[2 * i + 1]));
    P.phase_ms[KFMM_PH_M2L] += ms;
    P.prof_calls++;
    P.lev_head = (i + 1) % Plan::kLightRing;
    P.lev_count--;
    if (!all) break;
  }
}

void plan_eval(Plan& P, int kind, const double* a, const double* b, double* out, hipStream_t s) {
  const int no = kind == KFMM_DISP ? 3 : 6;
  if (P.n_trg == 0) return;
  if (P.empty || (!a && !b)) {
    const int64_t n = (int64_t)no * P.n_trg;
    hipLaunchKernelGGL(k_fill_zero<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, out);
    KFMM_HIP(hipGetLastError());
    return;
  }
  if (P.prec == KFMM_FP64)
    eval_t<double>(P, kind, a, b, out, s);
  else
    eval_t<float>(P, kind, a, b, out, s);
}

}  // namespace kfmm
