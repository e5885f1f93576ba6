// Adaptive octree with KIFMM interaction lists, built on the GPU (Sec. 2.2, first pass of the FMM:
// "generation of an octree partitioning of the domain into boxes").
#pragma once
#include <vector>

#include "common.h"

namespace kfmm {

constexpr int kMortonBits = 19;  // bits per axis of a point key; the geometry id sits above 57 bits
constexpr int kNoShift = 13;     // lattice shift code of (0, 0, 0)

// Device arena: owns every allocation of a plan and tracks its size against a limit.
struct Arena {
  std::vector<void*> ptrs;
  size_t bytes = 0, limit = 0;
  void* alloc(size_t n);
  template <typename T>
  T* get(size_t count) {
    return (T*)alloc(count * sizeof(T));
  }
  void release();
  ~Arena() { release(); }
};

struct Tree {
  int n_geom = 0;
  int n_box = 0, depth = 0;
  std::vector<int> level_start;  // host: first box of each level, size depth + 2
  // per box, device
  int *level = nullptr, *ix = nullptr, *iy = nullptr, *iz = nullptr, *geom = nullptr, *parent = nullptr;
  int *child_first = nullptr, *child_count = nullptr;
  int *src_b = nullptr, *src_e = nullptr, *trg_b = nullptr, *trg_e = nullptr;
  int* is_leaf = nullptr;
  int* colleague = nullptr;  // n_box x 27, index (dx+1)+3(dy+1)+9(dz+1), -1 if absent
  // periodic cells: the lattice image of each colleague, as a shift code (sx+1)+3(sy+1)+9(sz+1) with s in
  // {-1,0,1}^3 counted in cell sides (kNoShift in free space)
  signed char* colleague_sh = nullptr;
  bool periodic = false;
  // per geometry root (device)
  double* root_c = nullptr;  // n_geom x 3
  double* root_R = nullptr;  // n_geom: a power of two in free space, half the side of a periodic cell
  // host mirrors
  std::vector<int> h_level, h_parent, h_is_leaf, h_src_b, h_src_e, h_trg_b, h_trg_e, h_ix, h_iy, h_iz, h_geom,
      h_child_first, h_child_count;
  std::vector<double> h_root_c, h_root_R;
  // sorted point permutations (device): sorted position -> caller index
  int *perm_src = nullptr, *perm_trg = nullptr;
  int *leaf_of_src = nullptr, *leaf_of_trg = nullptr;
  // CSR interaction lists (device + host), see build_lists
  std::vector<int> h_u_off, h_u_idx, h_w_off, h_w_idx, h_x_off, h_x_idx;
  std::vector<int> h_v_trg, h_v_src, h_v_off;  // V pairs (target box, source box, offset index 0..342)
  int *u_off = nullptr, *u_idx = nullptr, *w_off = nullptr, *w_idx = nullptr, *x_off = nullptr, *x_idx = nullptr;
  // lattice image of every U, W, X entry (shift codes as for colleague_sh); the V offsets include it
  std::vector<signed char> h_u_sh, h_w_sh, h_x_sh;
  signed char* u_sh = nullptr;
};

// Builds the tree for sources (and targets if trg != nullptr; otherwise targets alias sources).
// batch_src / batch_trg: host offsets of n_geom independent geometries.  cells (host, n_geom x 4: lower
// corner and side) makes every geometry a periodic cubic cell whose root box is the cell (empty: free
// space, root boxes around the points); a point outside its cell is an argument error.
void build_tree(Tree& t, Arena& arena, const double* src, int64_t n_src, const double* trg, int64_t n_trg,
                const std::vector<int64_t>& batch_src, const std::vector<int64_t>& batch_trg, int leaf_max,
                int max_depth, hipStream_t s, const std::vector<double>& cells = {});

// Sorts (key, idx) pairs on the device: n valid entries in arrays of n_pad (a power of two >= 2048)
// elements; the padding is filled with the largest key.
void sort_keys(uint64_t* key, int* idx, int64_t n, int64_t n_pad, hipStream_t s);

// Builds the U, V, W, X lists of the tree; W and X pairs whose direct sum is no dearer than the surface route
// (a leaf with at most direct_max sources, resp. targets) join the U lists (0: none).
void build_lists(Tree& t, Arena& arena, hipStream_t s, int direct_max = 0);

}  // namespace kfmm
