// GPU octree construction and KIFMM interaction lists (Sec. 2.2: octree partitioning, then upward,
// downward and near-field passes that need, per box, its neighbours and well-separated boxes).
//
// Points get 64-bit keys: geometry id above 57 bits of a Morton code (19 bits per axis, bit order
// x, y, z inside every 3-bit digit), relative to a per-geometry root cube whose half-width is a power
// of two (so box-centre offsets are exact dyadic numbers).  Keys are sorted (bitonic sort of
// key/index pairs), and the tree is grown level by level: a box splits while it holds more than
// leaf_max sources + targets; its non-empty children are found by binary search in the sorted keys.
//
// Lists (standard adaptive KIFMM lists):
//   U(B), leaf B: leaves adjacent to B (and B itself)        -> near field, direct sum
//   V(B): children of the colleagues of parent(B) that are not adjacent to B    -> M2L
//   W(B), leaf B: descendants A of B's colleagues with A not adjacent to B but parent(A) adjacent
//   X(B): leaves A coarser than B, adjacent to parent(B) and not adjacent to B  (dual of W)
// Only boxes that hold sources enter as sources and only boxes that hold targets as targets.
// Cost-based assignment: a W pair whose source box is a leaf with at most direct_max sources, and an X pair
// whose target box is a leaf with at most direct_max targets, joins the U list instead (direct sums over the same
// source-target pairs, exact and cheaper than the route through an equivalent or check surface of
// direct_max points); every source-target interaction is still covered exactly once.
//
// Periodic cells (Sec. 4.3: integrals over the infinite periodic surface; the tree is periodic at every
// level): the root box is the cell, and the neighbours of a box at the cell's faces are boxes of the
// same cell seen through a lattice image.  Every colleague, and so every U, V, W, X entry, carries the
// shift of that image (a code for s in {-1,0,1}^3, in cell sides); at level 0 the 26 colleagues of the
// root are its own images.  The lists then cover exactly the 3 x 3 x 3 block of images around the cell;
// the images farther out reach the root through one precomputed operator (fmm.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "tree.h"

namespace kfmm {

void* Arena::alloc(size_t n) {
  if (n == 0) n = 8;
  n = (n + 255) & ~size_t(255);
  if (limit && bytes + n > limit) throw Error(-2, "device memory limit exceeded (opts.mem_limit)");
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) throw Error(-2, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  ptrs.push_back(p);
  bytes += n;
  return p;
}

void Arena::release() {
  for (void* p : ptrs) (void)hipFree(p);
  ptrs.clear();
  bytes = 0;
}

// ------------------------------------------------------------------------------------------ helpers

__device__ __forceinline__ uint64_t spread3(uint32_t v) {  // 19 bits -> every third bit
  uint64_t x = v & 0x7ffff;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ int find_segment(const int64_t* off, int n_seg, int64_t i) {
  int lo = 0, hi = n_seg;  // last lo with off[lo] <= i
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Per-geometry bounding box and finiteness check. One workgroup per geometry.
__global__ void k_bbox(const double* __restrict__ x, const int64_t* __restrict__ off, double* __restrict__ box,
                       int* __restrict__ bad) {
  int g = blockIdx.x;
  int64_t b = off[g], e = off[g + 1];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  int nonfinite = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    for (int d = 0; d < 3; ++d) {
      double v = x[3 * i + d];
      if (!isfinite(v)) nonfinite = 1;
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
    }
  }
  __shared__ double smn[3][256], smx[3][256];
  __shared__ int sbad[256];
  for (int d = 0; d < 3; ++d) {
    smn[d][threadIdx.x] = mn[d];
    smx[d][threadIdx.x] = mx[d];
  }
  sbad[threadIdx.x] = nonfinite;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int d = 0; d < 3; ++d) {
        smn[d][threadIdx.x] = fmin(smn[d][threadIdx.x], smn[d][threadIdx.x + s]);
        smx[d][threadIdx.x] = fmax(smx[d][threadIdx.x], smx[d][threadIdx.x + s]);
      }
      sbad[threadIdx.x] |= sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) {
      box[6 * g + d] = smn[d][0];
      box[6 * g + 3 + d] = smx[d][0];
    }
    if (sbad[0]) atomicOr(bad, 1);
  }
}

__global__ void k_keys(const double* __restrict__ x, int64_t n, const int64_t* __restrict__ off, int n_seg,
                       const double* __restrict__ root_c, const double* __restrict__ root_R,
                       uint64_t* __restrict__ key, int* __restrict__ idx, int64_t n_pad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pad) return;
  if (i >= n) {
    key[i] = ~0ull;
    idx[i] = 0x7fffffff;
    return;
  }
  int g = find_segment(off, n_seg, i);
  double R = root_R[g];
  const double scale = (double)(1 << kMortonBits);
  uint32_t q[3];
  for (int d = 0; d < 3; ++d) {
    double u = (x[3 * i + d] - (root_c[3 * g + d] - R)) / (2.0 * R);
    double f = floor(u * scale);
    f = fmin(fmax(f, 0.0), scale - 1.0);
    q[d] = (uint32_t)f;
  }
  key[i] = ((uint64_t)g << 57) | spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  idx[i] = (int)i;
}

// ------------------------------------------------------------------------------------ bitonic sort

__device__ __forceinline__ bool kv_less(uint64_t ka, int ia, uint64_t kb, int ib) {
  return ka < kb || (ka == kb && ia < ib);
}

__global__ void k_bitonic_global(uint64_t* key, int* idx, int64_t n, int64_t k, int64_t j) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one thread per pair
  if (t >= n / 2) return;
  int64_t i = 2 * j * (t / j) + (t % j);
  int64_t l = i + j;
  bool asc = (i & k) == 0;
  uint64_t ki = key[i], kl = key[l];
  int ii = idx[i], il = idx[l];
  bool swap = asc ? kv_less(kl, il, ki, ii) : kv_less(ki, ii, kl, il);
  if (swap) {
    key[i] = kl;
    key[l] = ki;
    idx[i] = il;
    idx[l] = ii;
  }
}

constexpr int kSortBlock = 2048;  // elements per workgroup in the LDS stages

// All stages with stride j < kSortBlock for a given k (or, with k_start > 0, the full local sort).
__global__ __launch_bounds__(1024) void k_bitonic_local(uint64_t* key, int* idx, int64_t k_fixed) {
  __shared__ uint64_t sk[kSortBlock];
  __shared__ int si[kSortBlock];
  int64_t base = (int64_t)blockIdx.x * kSortBlock;
  for (int t = threadIdx.x; t < kSortBlock; t += blockDim.x) {
    sk[t] = key[base + t];
    si[t] = idx[base + t];
  }
  __syncthreads();
  int64_t k_lo = k_fixed > 0 ? k_fixed : 2, k_hi = k_fixed > 0 ? k_fixed : kSortBlock;
  for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
    for (int64_t j = (k_fixed > 0 ? kSortBlock / 2 : k / 2); j > 0; j >>= 1) {
      int t = threadIdx.x;  // kSortBlock/2 pairs, one per thread
      int i = 2 * (int)j * (t / (int)j) + (t % (int)j);
      int l = i + (int)j;
      bool asc = ((base + i) & k) == 0;
      uint64_t ki = sk[i], kl = sk[l];
      int ii = si[i], il = si[l];
      bool swap = asc ? kv_less(kl, il, ki, ii) : kv_less(ki, ii, kl, il);
      if (swap) {
        sk[i] = kl;
        sk[l] = ki;
        si[i] = il;
        si[l] = ii;
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < kSortBlock; t += blockDim.x) {
    key[base + t] = sk[t];
    idx[base + t] = si[t];
  }
}

static void bitonic_sort(uint64_t* key, int* idx, int64_t n_pad, hipStream_t s) {
  // n_pad is a power of two >= kSortBlock
  int64_t blocks = n_pad / kSortBlock;
  hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)blocks), dim3(kSortBlock / 2), 0, s, key, idx, (int64_t)0);
  for (int64_t k = 2 * kSortBlock; k <= n_pad; k <<= 1) {
    for (int64_t j = k / 2; j >= kSortBlock; j >>= 1) {
      int64_t pairs = n_pad / 2;
      hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, key, idx, n_pad,
                         k, j);
    }
    hipLaunchKernelGGL(k_bitonic_local, dim3((unsigned)blocks), dim3(kSortBlock / 2), 0, s, key, idx, k);
  }
  KFMM_HIP(hipGetLastError());
}

__global__ void k_pad_keys(uint64_t* key, int* idx, int64_t n, int64_t n_pad) {
  int64_t i = n + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_pad) {
    key[i] = ~0ull;
    idx[i] = 0x7fffffff;
  }
}

void sort_keys(uint64_t* key, int* idx, int64_t n, int64_t n_pad, hipStream_t s) {
  if (n_pad > n)
    hipLaunchKernelGGL(k_pad_keys, dim3((unsigned)((n_pad - n + 255) / 256)), dim3(256), 0, s, key, idx, n, n_pad);
  bitonic_sort(key, idx, n_pad, s);
}

// ------------------------------------------------------------------------------------ tree levels

struct LevelBoxes {  // boxes of one level, device
  int n = 0;
  int *g = nullptr, *ix = nullptr, *iy = nullptr, *iz = nullptr, *sb = nullptr, *se = nullptr, *tb = nullptr,
      *te = nullptr, *parent_local = nullptr;
};

__device__ __forceinline__ int lower_bound_u64(const uint64_t* a, int lo, int hi, uint64_t v) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t box_key(int g, int l, int ix, int iy, int iz) {
  uint64_t m = spread3((uint32_t)ix) | (spread3((uint32_t)iy) << 1) | (spread3((uint32_t)iz) << 2);
  return ((uint64_t)g << 57) | (m << (3 * (kMortonBits - l)));
}

// Count (fill == 0) or write (fill == 1) the non-empty children of the boxes of level l that split.
__global__ void k_children(int n, int l, int leaf_max, int max_depth, const int* g, const int* ix, const int* iy,
                           const int* iz, const int* sb, const int* se, const int* tb, const int* te,
                           const uint64_t* skey, const uint64_t* tkey, int* count, const int* offset, int fill,
                           int* cg, int* cix, int* ciy, int* ciz, int* csb, int* cse, int* ctb, int* cte, int* cpar) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  int npts = (se[b] - sb[b]) + (te[b] - tb[b]);
  if (npts <= leaf_max || l >= max_depth) {
    if (!fill) count[b] = 0;
    return;
  }
  int c_out = fill ? offset[b] : 0;
  int cnt = 0;
  uint64_t span = 1ull << (3 * (kMortonBits - l - 1));
  for (int c = 0; c < 8; ++c) {
    int cx = 2 * ix[b] + (c & 1), cy = 2 * iy[b] + ((c >> 1) & 1), cz = 2 * iz[b] + ((c >> 2) & 1);
    uint64_t lo = box_key(g[b], l + 1, cx, cy, cz), hi = lo + span;
    int s0 = lower_bound_u64(skey, sb[b], se[b], lo), s1 = lower_bound_u64(skey, sb[b], se[b], hi);
    int t0 = tkey ? lower_bound_u64(tkey, tb[b], te[b], lo) : 0, t1 = tkey ? lower_bound_u64(tkey, tb[b], te[b], hi) : 0;
    if (s1 - s0 + t1 - t0 == 0) continue;
    if (fill) {
      int o = c_out + cnt;
      cg[o] = g[b];
      cix[o] = cx;
      ciy[o] = cy;
      ciz[o] = cz;
      csb[o] = s0;
      cse[o] = s1;
      ctb[o] = t0;
      cte[o] = t1;
      cpar[o] = b;
    }
    ++cnt;
  }
  if (!fill) count[b] = cnt;
}

// Exclusive scan of a small int array on the host side (tree sizes are modest; the counts are read
// back anyway to size the next level).
static int host_exclusive_scan(std::vector<int>& v) {
  int acc = 0;
  for (auto& x : v) {
    int t = x;
    x = acc;
    acc += t;
  }
  return acc;
}

__global__ void k_mark_leaf_points(int n_box, const int* is_leaf, const int* b, const int* e, int* leaf_of) {
  int box = blockIdx.x;
  if (box >= n_box || !is_leaf[box]) return;
  for (int i = b[box] + threadIdx.x; i < e[box]; i += blockDim.x) leaf_of[i] = box;
}

__device__ __forceinline__ int wrap_cell(int x, int lim, int& sh) {  // x in [-1, lim] -> [0, lim), shift
  sh = x < 0 ? -1 : (x >= lim ? 1 : 0);
  return x - sh * lim;
}

__global__ void k_colleagues(int n_box, const int* level, const int* ix, const int* iy, const int* iz, const int* g,
                             const int* level_start, const uint64_t* bkey, int periodic, int* colleague,
                             signed char* colleague_sh) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_box) return;
  int l = level[b];
  int lo0 = level_start[l], hi0 = level_start[l + 1];
  int lim = 1 << l;
  for (int c = 0; c < 27; ++c) {
    int dx = c % 3 - 1, dy = (c / 3) % 3 - 1, dz = c / 9 - 1;
    int x = ix[b] + dx, y = iy[b] + dy, z = iz[b] + dz;
    int sx = 0, sy = 0, sz = 0;
    if (periodic) {
      x = wrap_cell(x, lim, sx);
      y = wrap_cell(y, lim, sy);
      z = wrap_cell(z, lim, sz);
    }
    int found = -1;
    if (x >= 0 && y >= 0 && z >= 0 && x < lim && y < lim && z < lim) {
      uint64_t k = box_key(g[b], l, x, y, z);
      int p = lower_bound_u64(bkey, lo0, hi0, k);
      if (p < hi0 && bkey[p] == k) found = p;
    }
    colleague[27 * b + c] = found;
    colleague_sh[27 * b + c] = (signed char)((sx + 1) + 3 * (sy + 1) + 9 * (sz + 1));
  }
}

__global__ void k_box_keys(int n_box, const int* level, const int* ix, const int* iy, const int* iz, const int* g,
                           uint64_t* bkey) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_box) return;
  bkey[b] = box_key(g[b], level[b], ix[b], iy[b], iz[b]);
}

template <typename T>
static T* upload(Arena& a, const std::vector<T>& h, hipStream_t s) {
  T* d = a.get<T>(h.size() ? h.size() : 1);
  if (!h.empty()) KFMM_HIP(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
  return d;
}

template <typename T>
static std::vector<T> download(const T* d, size_t n, hipStream_t s) {
  std::vector<T> h(n);
  if (n) KFMM_HIP(hipMemcpyAsync(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  return h;
}

static int64_t next_pow2(int64_t v) {
  int64_t p = kSortBlock;
  while (p < v) p <<= 1;
  return p;
}

// Sort the points of one set; returns sorted keys (device, padded) and writes the permutation.
static uint64_t* sort_points(Arena& arena, Arena& scratch, const double* x, int64_t n, const int64_t* d_off,
                             int n_seg, const double* root_c, const double* root_R, int* perm_out, hipStream_t s) {
  int64_t n_pad = next_pow2(std::max<int64_t>(n, 1));
  uint64_t* key = arena.get<uint64_t>(n_pad);
  int* idx = scratch.get<int>(n_pad);
  hipLaunchKernelGGL(k_keys, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, s, x, n, d_off, n_seg, root_c,
                     root_R, key, idx, n_pad);
  KFMM_HIP(hipGetLastError());
  bitonic_sort(key, idx, n_pad, s);
  if (n) KFMM_HIP(hipMemcpyAsync(perm_out, idx, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
  return key;
}

void build_tree(Tree& t, Arena& arena, const double* src, int64_t n_src, const double* trg, int64_t n_trg,
                const std::vector<int64_t>& batch_src, const std::vector<int64_t>& batch_trg, int leaf_max,
                int max_depth, hipStream_t s, const std::vector<double>& cells) {
  Arena scratch;
  const int G = (int)batch_src.size() - 1;
  t.n_geom = G;
  t.periodic = !cells.empty();
  if (t.periodic && (int)cells.size() != 4 * G) throw Error(-1, "periodic cells: 4 values per geometry");
  const bool alias = (trg == nullptr);
  // ---- bounding cubes
  int64_t* d_bs = upload(scratch, batch_src, s);
  int64_t* d_bt = alias ? d_bs : upload(scratch, batch_trg, s);
  double* d_bbs = scratch.get<double>(6 * G);
  double* d_bbt = scratch.get<double>(6 * G);
  int* d_bad = scratch.get<int>(1);
  KFMM_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), s));
  if (n_src) hipLaunchKernelGGL(k_bbox, dim3(G), dim3(256), 0, s, src, d_bs, d_bbs, d_bad);
  if (!alias && n_trg) hipLaunchKernelGGL(k_bbox, dim3(G), dim3(256), 0, s, trg, d_bt, d_bbt, d_bad);
  KFMM_HIP(hipGetLastError());
  std::vector<double> hbs = download(d_bbs, 6 * G, s);
  std::vector<double> hbt = (!alias && n_trg) ? download(d_bbt, 6 * G, s) : std::vector<double>();
  int bad = download(d_bad, 1, s)[0];
  if (bad) throw Error(-1, "non-finite source or target coordinate");
  t.h_root_c.assign(3 * G, 0.0);
  t.h_root_R.assign(G, 1.0);
  for (int g = 0; g < G; ++g) {
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool any = false;
    if (batch_src[g + 1] > batch_src[g]) {
      any = true;
      for (int d = 0; d < 3; ++d) {
        mn[d] = std::min(mn[d], hbs[6 * g + d]);
        mx[d] = std::max(mx[d], hbs[6 * g + 3 + d]);
      }
    }
    if (!alias && batch_trg[g + 1] > batch_trg[g]) {
      any = true;
      for (int d = 0; d < 3; ++d) {
        mn[d] = std::min(mn[d], hbt[6 * g + d]);
        mx[d] = std::max(mx[d], hbt[6 * g + 3 + d]);
      }
    }
    if (t.periodic) {  // the root box is the cell; every point must lie in [lo, lo + side)
      const double* c = &cells[4 * g];
      if (!(c[3] > 0.0) || !std::isfinite(c[3]) || !std::isfinite(c[0]) || !std::isfinite(c[1]) ||
          !std::isfinite(c[2]))
        throw Error(-1, "periodic cell: side must be positive and finite");
      for (int d = 0; d < 3; ++d) {
        t.h_root_c[3 * g + d] = c[d] + 0.5 * c[3];
        if (any && (mn[d] < c[d] || mx[d] >= c[d] + c[3])) throw Error(-1, "point outside its periodic cell");
      }
      t.h_root_R[g] = 0.5 * c[3];
      continue;
    }
    if (!any) continue;
    double half = 0;
    for (int d = 0; d < 3; ++d) {
      t.h_root_c[3 * g + d] = 0.5 * (mn[d] + mx[d]);
      half = std::max(half, 0.5 * (mx[d] - mn[d]));
    }
    double R = 1.0;
    half *= (1.0 + 1e-9);
    if (half > 0) R = std::ldexp(1.0, (int)std::ceil(std::log2(half)));
    if (R < half) R *= 2;
    t.h_root_R[g] = R;
  }
  t.root_c = upload(arena, t.h_root_c, s);
  t.root_R = upload(arena, t.h_root_R, s);
  // ---- sort points
  t.perm_src = arena.get<int>(std::max<int64_t>(n_src, 1));
  t.perm_trg = alias ? t.perm_src : arena.get<int>(std::max<int64_t>(n_trg, 1));
  uint64_t* skey = sort_points(scratch, scratch, src, n_src, d_bs, G, t.root_c, t.root_R, t.perm_src, s);
  uint64_t* tkey = alias ? nullptr
                         : sort_points(scratch, scratch, trg, n_trg, d_bt, G, t.root_c, t.root_R, t.perm_trg, s);
  // ---- levels
  std::vector<LevelBoxes> levels;
  {
    std::vector<int> g0, z0, sb0, se0, tb0, te0, p0;
    for (int g = 0; g < G; ++g) {
      int ns = (int)(batch_src[g + 1] - batch_src[g]);
      int nt = alias ? 0 : (int)(batch_trg[g + 1] - batch_trg[g]);
      if (ns + nt == 0) continue;
      g0.push_back(g);
      z0.push_back(0);
      sb0.push_back((int)batch_src[g]);
      se0.push_back((int)batch_src[g + 1]);
      tb0.push_back(alias ? 0 : (int)batch_trg[g]);
      te0.push_back(alias ? 0 : (int)batch_trg[g + 1]);
      p0.push_back(-1);
    }
    LevelBoxes L;
    L.n = (int)g0.size();
    L.g = upload(scratch, g0, s);
    L.ix = upload(scratch, z0, s);
    L.iy = upload(scratch, z0, s);
    L.iz = upload(scratch, z0, s);
    L.sb = upload(scratch, sb0, s);
    L.se = upload(scratch, se0, s);
    L.tb = upload(scratch, tb0, s);
    L.te = upload(scratch, te0, s);
    L.parent_local = upload(scratch, p0, s);
    levels.push_back(L);
  }
  // alias: the target ranges of a box are its source ranges; keep tb/te empty during the build and
  // copy afterwards (the split rule then counts each point once).
  for (int l = 0;; ++l) {
    LevelBoxes& L = levels[l];
    if (L.n == 0) break;
    int* d_cnt = scratch.get<int>(L.n);
    unsigned nb = (unsigned)((L.n + 255) / 256);
    hipLaunchKernelGGL(k_children, dim3(nb), dim3(256), 0, s, L.n, l, leaf_max, max_depth, L.g, L.ix, L.iy, L.iz,
                       L.sb, L.se, L.tb, L.te, skey, tkey, d_cnt, (const int*)nullptr, 0, (int*)nullptr,
                       (int*)nullptr, (int*)nullptr, (int*)nullptr, (int*)nullptr, (int*)nullptr, (int*)nullptr,
                       (int*)nullptr, (int*)nullptr);
    KFMM_HIP(hipGetLastError());
    std::vector<int> cnt = download(d_cnt, L.n, s);
    int total = host_exclusive_scan(cnt);
    if (total == 0) break;
    LevelBoxes C;
    C.n = total;
    C.g = scratch.get<int>(total);
    C.ix = scratch.get<int>(total);
    C.iy = scratch.get<int>(total);
    C.iz = scratch.get<int>(total);
    C.sb = scratch.get<int>(total);
    C.se = scratch.get<int>(total);
    C.tb = scratch.get<int>(total);
    C.te = scratch.get<int>(total);
    C.parent_local = scratch.get<int>(total);
    int* d_off = upload(scratch, cnt, s);
    hipLaunchKernelGGL(k_children, dim3(nb), dim3(256), 0, s, L.n, l, leaf_max, max_depth, L.g, L.ix, L.iy, L.iz,
                       L.sb, L.se, L.tb, L.te, skey, tkey, (int*)nullptr, d_off, 1, C.g, C.ix, C.iy, C.iz, C.sb, C.se,
                       C.tb, C.te, C.parent_local);
    KFMM_HIP(hipGetLastError());
    levels.push_back(C);
  }
  // ---- flatten levels into global box arrays (host side; trees are small)
  const int depth = (int)levels.size() - 1;
  t.depth = depth;
  t.level_start.assign(depth + 2, 0);
  for (int l = 0; l <= depth; ++l) t.level_start[l + 1] = t.level_start[l] + levels[l].n;
  const int nbx = t.level_start[depth + 1];
  t.n_box = nbx;
  t.h_level.resize(nbx);
  t.h_geom.resize(nbx);
  t.h_ix.resize(nbx);
  t.h_iy.resize(nbx);
  t.h_iz.resize(nbx);
  t.h_src_b.resize(nbx);
  t.h_src_e.resize(nbx);
  t.h_trg_b.resize(nbx);
  t.h_trg_e.resize(nbx);
  t.h_parent.resize(nbx);
  t.h_child_first.assign(nbx, -1);
  t.h_child_count.assign(nbx, 0);
  t.h_is_leaf.assign(nbx, 1);
  for (int l = 0; l <= depth; ++l) {
    const LevelBoxes& L = levels[l];
    int o = t.level_start[l];
    auto cp = [&](const int* d, std::vector<int>& h) {
      std::vector<int> v = download(d, L.n, s);
      std::copy(v.begin(), v.end(), h.begin() + o);
    };
    cp(L.g, t.h_geom);
    cp(L.ix, t.h_ix);
    cp(L.iy, t.h_iy);
    cp(L.iz, t.h_iz);
    cp(L.sb, t.h_src_b);
    cp(L.se, t.h_src_e);
    cp(L.tb, t.h_trg_b);
    cp(L.te, t.h_trg_e);
    std::vector<int> par = download(L.parent_local, L.n, s);
    for (int i = 0; i < L.n; ++i) {
      t.h_level[o + i] = l;
      int pb = par[i] < 0 ? -1 : t.level_start[l - 1] + par[i];
      t.h_parent[o + i] = pb;
      if (pb >= 0) {
        if (t.h_child_first[pb] < 0) t.h_child_first[pb] = o + i;
        t.h_child_count[pb]++;
        t.h_is_leaf[pb] = 0;
      }
    }
  }
  if (alias) {
    t.h_trg_b = t.h_src_b;
    t.h_trg_e = t.h_src_e;
  }
  t.level = upload(arena, t.h_level, s);
  t.geom = upload(arena, t.h_geom, s);
  t.ix = upload(arena, t.h_ix, s);
  t.iy = upload(arena, t.h_iy, s);
  t.iz = upload(arena, t.h_iz, s);
  t.src_b = upload(arena, t.h_src_b, s);
  t.src_e = upload(arena, t.h_src_e, s);
  t.trg_b = upload(arena, t.h_trg_b, s);
  t.trg_e = upload(arena, t.h_trg_e, s);
  t.parent = upload(arena, t.h_parent, s);
  t.child_first = upload(arena, t.h_child_first, s);
  t.child_count = upload(arena, t.h_child_count, s);
  t.is_leaf = upload(arena, t.h_is_leaf, s);
  // ---- point -> leaf maps
  t.leaf_of_src = arena.get<int>(std::max<int64_t>(n_src, 1));
  hipLaunchKernelGGL(k_mark_leaf_points, dim3(nbx), dim3(64), 0, s, nbx, t.is_leaf, t.src_b, t.src_e, t.leaf_of_src);
  if (alias) {
    t.leaf_of_trg = t.leaf_of_src;
  } else {
    t.leaf_of_trg = arena.get<int>(std::max<int64_t>(n_trg, 1));
    hipLaunchKernelGGL(k_mark_leaf_points, dim3(nbx), dim3(64), 0, s, nbx, t.is_leaf, t.trg_b, t.trg_e,
                       t.leaf_of_trg);
  }
  KFMM_HIP(hipGetLastError());
  // ---- colleagues
  uint64_t* bkey = scratch.get<uint64_t>(nbx);
  int* d_ls = upload(scratch, t.level_start, s);
  hipLaunchKernelGGL(k_box_keys, dim3((nbx + 255) / 256), dim3(256), 0, s, nbx, t.level, t.ix, t.iy, t.iz, t.geom,
                     bkey);
  t.colleague = arena.get<int>((size_t)27 * nbx);
  t.colleague_sh = arena.get<signed char>((size_t)27 * nbx);
  hipLaunchKernelGGL(k_colleagues, dim3((nbx + 255) / 256), dim3(256), 0, s, nbx, t.level, t.ix, t.iy, t.iz, t.geom,
                     d_ls, bkey, t.periodic ? 1 : 0, t.colleague, t.colleague_sh);
  KFMM_HIP(hipGetLastError());
  KFMM_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------------------------------ lists

struct BoxView {
  const int *level, *ix, *iy, *iz, *parent, *child_first, *child_count, *is_leaf, *colleague;
  const int *src_b, *src_e, *trg_b, *trg_e;
  const signed char* colleague_sh;
};

__device__ __forceinline__ bool has_src(const BoxView& v, int b) { return v.src_e[b] > v.src_b[b]; }
__device__ __forceinline__ bool has_trg(const BoxView& v, int b) { return v.trg_e[b] > v.trg_b[b]; }

__device__ __forceinline__ int shift_of(int code, int d) {  // component d of a lattice shift code
  return d == 0 ? code % 3 - 1 : (d == 1 ? (code / 3) % 3 - 1 : code / 9 - 1);
}

// Closed cubes of box a, seen through the lattice image of shift code sa, and box b touch (boxes of one
// geometry with disjoint interiors).
__device__ __forceinline__ bool adjacent(const BoxView& v, int a, int sa_code, int b) {
  int la = v.level[a], lb = v.level[b];
  int L = la > lb ? la : lb;
  int sa = L - la, sb = L - lb;
  int ca[3] = {v.ix[a], v.iy[a], v.iz[a]}, cb[3] = {v.ix[b], v.iy[b], v.iz[b]};
  for (int d = 0; d < 3; ++d) {
    const long img = (long)shift_of(sa_code, d) * (1L << la);  // one cell side in units of level la
    long a0 = ((long)ca[d] + img) << sa, a1 = ((long)ca[d] + img + 1) << sa;
    long b0 = (long)cb[d] << sb, b1 = ((long)cb[d] + 1) << sb;
    if (a1 < b0 || b1 < a0) return false;
  }
  return true;
}

// One thread per box.  mode 0: count; mode 1: fill.  Each list k in {U, W, X, V} has counts cnt_k[b]
// and offsets off_k[b]; V entries also record the offset index (lattice shift included), U, W, X entries
// the shift code of the image they are seen through.  A descendant is seen through the image of the
// colleague it descends from; colleague 13 of a box is the box itself.
__global__ void k_lists(int n_box, BoxView v, int direct_max, int mode, int* cU, int* cW, int* cX, int* cV,
                        const int* oU, const int* oW, const int* oX, const int* oV, int* lU, int* lW, int* lX,
                        int* lVs, int* lVo, signed char* sU, signed char* sW, signed char* sX) {
  int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= n_box) return;
  int nU = 0, nW = 0, nX = 0, nV = 0;
  const bool trgB = has_trg(v, B);
  const int P = v.parent[B];
#define PUSH(list, shl, cntvar, offarr, val, sh) \
  do {                                            \
    if (mode) {                                   \
      list[offarr[B] + cntvar] = (val);           \
      shl[offarr[B] + cntvar] = (signed char)(sh); \
    }                                             \
    ++cntvar;                                     \
  } while (0)
  if (trgB) {
    // ---- V: children of the colleagues of parent(B), same level, not adjacent
    if (P >= 0) {
      const int l = v.level[B];
      for (int c = 0; c < 27; ++c) {
        int C = v.colleague[27 * P + c];
        if (C < 0) continue;
        const int sc = v.colleague_sh[27 * P + c];
        int f = v.child_first[C], nc = v.child_count[C];
        for (int k = 0; k < nc; ++k) {
          int A = f + k;
          int dx = v.ix[A] + shift_of(sc, 0) * (1 << l) - v.ix[B], dy = v.iy[A] + shift_of(sc, 1) * (1 << l) - v.iy[B],
              dz = v.iz[A] + shift_of(sc, 2) * (1 << l) - v.iz[B];
          int m = max(abs(dx), max(abs(dy), abs(dz)));
          if (m <= 1 || !has_src(v, A)) continue;
          if (mode) {
            lVs[oV[B] + nV] = A;
            lVo[oV[B] + nV] = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
          }
          ++nV;
        }
      }
    }
    // ---- X: leaves coarser than B adjacent to parent(B) but not to B
    if (P >= 0) {
      for (int anc = P; anc >= 0; anc = v.parent[anc]) {
        for (int c = 0; c < 27; ++c) {
          int A = v.colleague[27 * anc + c];
          if (A < 0 || c == 13 || !v.is_leaf[A] || !has_src(v, A)) continue;
          const int sa = v.colleague_sh[27 * anc + c];
          if (adjacent(v, A, sa, P) && !adjacent(v, A, sa, B)) {
            if (v.is_leaf[B] && v.trg_e[B] - v.trg_b[B] <= direct_max)
              PUSH(lU, sU, nU, oU, A, sa);  // direct: cheaper than A's sources at B's check surface
            else
              PUSH(lX, sX, nX, oX, A, sa);
          }
        }
      }
    }
    if (v.is_leaf[B]) {
      // ---- U: B itself, adjacent leaves at B's level and finer (descending colleagues), coarser leaves
      if (has_src(v, B)) PUSH(lU, sU, nU, oU, B, 13);
      int stack[256];
      for (int c = 0; c < 27; ++c) {
        int C = v.colleague[27 * B + c];
        if (C < 0 || c == 13) continue;
        const int sc = v.colleague_sh[27 * B + c];
        if (v.is_leaf[C]) {
          if (has_src(v, C)) PUSH(lU, sU, nU, oU, C, sc);
          continue;
        }
        int sp = 0;
        stack[sp++] = C;
        while (sp > 0) {
          int Q = stack[--sp];
          int f = v.child_first[Q], nc = v.child_count[Q];
          for (int k = 0; k < nc; ++k) {
            int A = f + k;
            if (!has_src(v, A)) continue;
            if (adjacent(v, A, sc, B)) {
              if (v.is_leaf[A])
                PUSH(lU, sU, nU, oU, A, sc);
              else if (sp < 256)
                stack[sp++] = A;
            } else if (v.is_leaf[A] && v.src_e[A] - v.src_b[A] <= direct_max) {
              // direct: cheaper than A's equivalent density at B's targets (leaves only: the near field
              // stages sources from leaf-local coordinates and the offset of their own leaf)
              PUSH(lU, sU, nU, oU, A, sc);
            } else {
              PUSH(lW, sW, nW, oW, A, sc);
            }
          }
        }
      }
      for (int anc = P; anc >= 0; anc = v.parent[anc]) {
        for (int c = 0; c < 27; ++c) {
          int A = v.colleague[27 * anc + c];
          if (A < 0 || c == 13 || !v.is_leaf[A] || !has_src(v, A)) continue;
          const int sa = v.colleague_sh[27 * anc + c];
          if (adjacent(v, A, sa, B)) PUSH(lU, sU, nU, oU, A, sa);
        }
      }
    }
  }
#undef PUSH
  if (!mode) {
    cU[B] = nU;
    cW[B] = nW;
    cX[B] = nX;
    cV[B] = nV;
  }
}

void build_lists(Tree& t, Arena& arena, hipStream_t s, int direct_max) {
  Arena scratch;
  const int n = t.n_box;
  BoxView v{t.level, t.ix, t.iy, t.iz, t.parent, t.child_first, t.child_count, t.is_leaf, t.colleague,
            t.src_b, t.src_e, t.trg_b, t.trg_e, t.colleague_sh};
  int* c4 = scratch.get<int>(4 * (size_t)n);
  unsigned nb = (unsigned)((n + 127) / 128);
  hipLaunchKernelGGL(k_lists, dim3(nb), dim3(128), 0, s, n, v, direct_max, 0, c4, c4 + n, c4 + 2 * n, c4 + 3 * n,
                     (const int*)nullptr, (const int*)nullptr, (const int*)nullptr, (const int*)nullptr, (int*)nullptr,
                     (int*)nullptr, (int*)nullptr, (int*)nullptr, (int*)nullptr, (signed char*)nullptr,
                     (signed char*)nullptr, (signed char*)nullptr);
  KFMM_HIP(hipGetLastError());
  std::vector<int> h = download(c4, 4 * (size_t)n, s);
  std::vector<int> offs[4];
  int tot[4];
  for (int k = 0; k < 4; ++k) {
    offs[k].assign(h.begin() + (size_t)k * n, h.begin() + (size_t)(k + 1) * n);
    tot[k] = host_exclusive_scan(offs[k]);
    offs[k].push_back(tot[k]);
  }
  int* dO[4];
  for (int k = 0; k < 4; ++k) dO[k] = upload(scratch, offs[k], s);
  int* lU = scratch.get<int>(tot[0] + 1);
  int* lW = scratch.get<int>(tot[1] + 1);
  int* lX = scratch.get<int>(tot[2] + 1);
  int* lVs = scratch.get<int>(tot[3] + 1);
  int* lVo = scratch.get<int>(tot[3] + 1);
  signed char* sU = scratch.get<signed char>(tot[0] + 1);
  signed char* sW = scratch.get<signed char>(tot[1] + 1);
  signed char* sX = scratch.get<signed char>(tot[2] + 1);
  hipLaunchKernelGGL(k_lists, dim3(nb), dim3(128), 0, s, n, v, direct_max, 1, (int*)nullptr, (int*)nullptr,
                     (int*)nullptr,
                     (int*)nullptr, dO[0], dO[1], dO[2], dO[3], lU, lW, lX, lVs, lVo, sU, sW, sX);
  KFMM_HIP(hipGetLastError());
  t.h_u_off = offs[0];
  t.h_w_off = offs[1];
  t.h_x_off = offs[2];
  t.h_u_idx = download(lU, tot[0], s);
  t.h_w_idx = download(lW, tot[1], s);
  t.h_x_idx = download(lX, tot[2], s);
  t.h_u_sh = download(sU, tot[0], s);
  t.h_w_sh = download(sW, tot[1], s);
  t.h_x_sh = download(sX, tot[2], s);
  std::vector<int> vs = download(lVs, tot[3], s), vo = download(lVo, tot[3], s);
  t.h_v_trg.resize(tot[3]);
  t.h_v_src = vs;
  t.h_v_off = vo;
  for (int b = 0; b < n; ++b)
    for (int i = offs[3][b]; i < offs[3][b + 1]; ++i) t.h_v_trg[i] = b;
  t.u_off = upload(arena, t.h_u_off, s);
  t.u_idx = upload(arena, t.h_u_idx, s);
  t.w_off = upload(arena, t.h_w_off, s);
  t.w_idx = upload(arena, t.h_w_idx, s);
  t.x_off = upload(arena, t.h_x_off, s);
  t.x_idx = upload(arena, t.h_x_idx, s);
  t.u_sh = upload(arena, t.h_u_sh, s);
  KFMM_HIP(hipStreamSynchronize(s));
}

}  // namespace kfmm
