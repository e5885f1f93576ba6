// Batched gather/scatter GEMM on the CDNA matrix cores for every KIFMM translation.
//
//   Y[:, out_idx[j]] (=, +=, atomic +=)  scale[j] * A_op(j) * X[:, in_idx[j]]
//
// A_op are NC x NC row-major operators (op index per tile, stride NC*NC), X and Y hold one
// NC-vector per box (box-major, stride NC).  Columns are grouped in tiles of <= 64 that share one
// operator.  A workgroup of 4 waves computes a (16*TM) x 64 block: every wave owns 16 columns and
// all rows; A and X tiles are staged in LDS, products use v_mfma_*_16x16x4 (FP64/FP32).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace kfmm {

enum GemmMode { kStore = 0, kAdd = 1, kAtomicAdd = 2 };

constexpr int kGemmBN = 64;  // columns per tile

// Rows per workgroup are 16 * TM with TM = 6 (M a multiple of 96) or TM = 8 (M a multiple of 128).
inline int gemm_tm(int M) { return M % 96 == 0 ? 6 : (M % 128 == 0 ? 8 : 0); }

// Padded length of an n-vector of coefficients: the smallest multiple of 32 that is also a multiple of
// 96 or 128 (p = 8: 888 -> 896), else the next multiple of 96.
inline int gemm_pad(int n) {
  const int c = (n + 31) / 32 * 32;
  return gemm_tm(c) ? c : (n + 95) / 96 * 96;
}

struct GemmJob {  // device arrays describing one launch
  int n_tiles = 0;
  int cols_per_tile = 64;   // 64 or 128 (wide tiles: FP32 only)
  int4* tiles = nullptr;    // {op, first column, column count, rank}: rank 0 = the whole operator; a rank m
                            // > 0 takes the leading m x m block (k_gemm_h3 with 128-column tiles, k_gemm_f)
  int* in_idx = nullptr;    // per column: source box (X column)
  int* out_idx = nullptr;   // per column: destination box (Y column)
  double* scale = nullptr;  // per column factor or nullptr
  bool ranked = false;      // some tile has a rank (split FP16: k_gemm_h3; FP64 / FP32: the tiled kernel)
};

// Host-side description: (op, in, out, scale) per column, grouped by op into tiles.
struct GemmCols {
  std::vector<int> op, in, out;
  std::vector<double> scale;
  void add(int o, int i, int u, double s = 1.0) {
    op.push_back(o);
    in.push_back(i);
    out.push_back(u);
    scale.push_back(s);
  }
};

// Shape of one launch: operators are M x K row-major (leading dimension K, stride M*K between
// operators), X vectors have K entries at stride ldx, Y vectors M entries at stride ldy.  M must be a
// multiple of 96 or 128 and K of 32.  Sq(NC) is the square case used by the translations.
struct GemmDims {
  int M, K, ldx, ldy;
  static GemmDims Sq(int NC) { return GemmDims{NC, NC, NC, NC}; }
};

// kernel: kGemmAuto picks the tiled kernel, or the split-K kernel for launches too small to fill the
// chip, and the tiled kernel's LDS buffering by launch size; the other values force a choice (test hook):
// tiled with automatic buffering, split-K, tiled single-buffered, tiled double-buffered.
enum GemmKernel { kGemmAuto = 0, kGemmTiled = 1, kGemmSplitK = 2, kGemmTiled1 = 3, kGemmTiled2 = 4 };
void gemm_f64(const GemmJob& job, const double* A, GemmDims d, const double* X, double* Y, int mode, hipStream_t s,
              int kernel = kGemmAuto);
void gemm_f32(const GemmJob& job, const float* A, GemmDims d, const float* X, float* Y, int mode, hipStream_t s,
              int kernel = kGemmAuto);
void gemm_f32(const GemmJob& job, const float* A, GemmDims d, const float* X, double* Y, int mode, hipStream_t s,
              int kernel = kGemmAuto);

// Split-FP16 products (gemm_h3.hip).  split_h3 writes n_rows rows of len values (a multiple of 8, read at
// stride ld) as split rows of 2 * len FP16 numbers, chunks of [hi of 8 values][lo of the same 8] after
// division by the row's power-of-two scale (written to scale[row]); an operator set is split with one row
// per operator (len = M * K).  gemm_h3 runs the gather/scatter product on such operands: A_op split
// operators with scales a_scale[op], X split vectors (d.ldx = FP16 numbers per split vector, at least
// 2 * d.K) with scales x_scale[box], FP32 outputs.  M must be a multiple of 96 or 64, K of 32 (at least
// 64), at most 128 columns per tile (128-column tiles with M a multiple of 160 use 160-row blocks).
// kscale (optional, FP32 rows of at most 1024 values): value k of every row multiplied by kscale[k] first.
void split_h3(const float* src, int64_t n_rows, int64_t len, int64_t ld, uint16_t* dst, float* scale, hipStream_t s,
              const float* kscale = nullptr);
void split_h3(const double* src, int64_t n_rows, int64_t len, int64_t ld, uint16_t* dst, float* scale,
              hipStream_t s);
void gemm_h3(const GemmJob& job, const uint16_t* A, const float* a_scale, GemmDims d, const uint16_t* X,
             const float* x_scale, float* Y, int mode, hipStream_t s);

// Runs one gather/scatter GEMM launch from host column descriptors (test hook).
void selftest_gemm(int precision, const void* A, int NC, const void* X, void* Y, const int* op, const int* in,
                   const int* out, const double* scale, int ncols, int mode, int kernel, hipStream_t s);

}  // namespace kfmm
