// Batched gather/scatter GEMM on the matrix cores (see gemm.h): FP32 launches (the M2L contraction and
// the compressed-basis projections).  Compiled with the default (AGPR) MFMA register form, which
// schedules the 128-column M2L tiles better than the VGPR form used for the FP64 kernels.
#include "gemm_kernels.h"

namespace kfmm {

void gemm_f32(const GemmJob& job, const float* A, GemmDims d, const float* X, float* Y, int mode, hipStream_t s,
              int kernel) {
  gemm_t(job, A, d, X, Y, mode, s, kernel);
}
void gemm_f32(const GemmJob& job, const float* A, GemmDims d, const float* X, double* Y, int mode, hipStream_t s,
              int kernel) {
  gemm_t(job, A, d, X, Y, mode, s, kernel);
}

}  // namespace kfmm
