// Batched gather/scatter GEMM on the matrix cores (see gemm.h): FP64 launches and the test hook.
// Compiled with the VGPR form of the MFMA instructions (see build.py).
#include <algorithm>

#include "gemm_kernels.h"

namespace kfmm {

void gemm_f64(const GemmJob& job, const double* A, GemmDims d, const double* X, double* Y, int mode, hipStream_t s,
              int kernel) {
  gemm_t(job, A, d, X, Y, mode, s, kernel);
}
}  // namespace kfmm

// ------------------------------------------------------------------ test hook (see kfmm_selftest_gemm)
namespace kfmm {
void selftest_gemm(int precision, const void* A, int NC, const void* X, void* Y, const int* op, const int* in,
                   const int* out, const double* scale, int ncols, int mode, int kernel, hipStream_t s) {
  Arena a;
  std::vector<int4> tiles;
  // FP32 and split FP16 run the wide tiles used by the M2L; FP64 runs wide tiles when op == 0 only (as in
  // large launches)
  int tile_cols = (precision == 1 || precision == 3 || (precision == 0 && ncols > 0 && op[ncols - 1] == 0))
                      ? 2 * kGemmBN
                      : kGemmBN;
  if (precision == 3 && kernel == 1) tile_cols = kGemmBN;  // the translation passes' 64-column tiles
  int i = 0;
  while (i < ncols) {
    int j = i;
    while (j < ncols && op[j] == op[i] && j - i < tile_cols) ++j;
    tiles.push_back(make_int4(op[i], i, j - i, 0));
    i = j;
  }
  GemmJob job;
  job.cols_per_tile = tile_cols;
  job.n_tiles = (int)tiles.size();
  job.tiles = a.get<int4>(tiles.size() + 1);
  job.in_idx = a.get<int>(ncols + 1);
  job.out_idx = a.get<int>(ncols + 1);
  job.scale = scale ? a.get<double>(ncols + 1) : nullptr;
  KFMM_HIP(hipMemcpyAsync(job.tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  KFMM_HIP(hipMemcpyAsync(job.in_idx, in, ncols * sizeof(int), hipMemcpyHostToDevice, s));
  KFMM_HIP(hipMemcpyAsync(job.out_idx, out, ncols * sizeof(int), hipMemcpyHostToDevice, s));
  if (scale) KFMM_HIP(hipMemcpyAsync(job.scale, scale, ncols * sizeof(double), hipMemcpyHostToDevice, s));
  const GemmDims d = GemmDims::Sq(NC);
  if (precision == 3) {  // FP32 inputs, split on the device
    int n_ops = ncols ? op[ncols - 1] + 1 : 0, n_box = 0;
    for (int j = 0; j < ncols; ++j) n_box = std::max(n_box, in[j] + 1);
    uint16_t* Ah = a.get<uint16_t>((size_t)n_ops * NC * NC * 2 + 8);
    uint16_t* Xh = a.get<uint16_t>((size_t)n_box * NC * 2 + 8);
    float* as = a.get<float>(n_ops + 1);
    float* xs = a.get<float>(n_box + 1);
    split_h3((const float*)A, n_ops, (int64_t)NC * NC, (int64_t)NC * NC, Ah, as, s);
    split_h3((const float*)X, n_box, NC, NC, Xh, xs, s);
    gemm_h3(job, Ah, as, GemmDims{NC, NC, 2 * NC, NC}, Xh, xs, (float*)Y, mode, s);
  } else if (precision == 0)
    gemm_f64(job, (const double*)A, d, (const double*)X, (double*)Y, mode, s, kernel);
  else
    gemm_f32(job, (const float*)A, d, (const float*)X, (float*)Y, mode, s, kernel);
  KFMM_HIP(hipStreamSynchronize(s));
}
}  // namespace kfmm
