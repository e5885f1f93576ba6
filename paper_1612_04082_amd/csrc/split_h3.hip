// Split pass of the split-FP16 products (see gemm.h and gemm_h3.hip): a row of values divided by a
// power-of-two scale that puts its largest magnitude in [2^14, 2^15), stored as chunks of 16 FP16 numbers
// [hi of 8 consecutive values][lo of the same 8], hi = fp16(v / s), lo = fp16(v / s - hi).
#include <algorithm>
#include <cstdint>

#include "gemm_kernels.h"

namespace kfmm {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));

// Power-of-two scale s with m / s in [2^14, 2^15) for m > 0 (1 for m = 0 or non-finite m).
template <typename T>
__device__ __forceinline__ float pow2_scale(T m) {
  if (!(m > T(0)) || !(m < T(INFINITY))) return 1.0f;
  int e;
  frexp((double)m, &e);  // m = f 2^e, f in [0.5, 1)
  e = max(-126, min(127, e - 15));
  return ldexpf(1.0f, e);
}

// Split of one 8-value chunk with the multiplier inv (a power of two): [hi of the 8][lo of the 8].
template <typename TIN>
__device__ __forceinline__ void split8(const TIN* v, double inv, uint4* d) {
  union {
    _Float16 h[16];
    uint4 q[2];
  } u;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double x = (double)v[j] * inv;
    const _Float16 hi = (_Float16)(float)x;
    u.h[j] = hi;
    u.h[8 + j] = (_Float16)(float)(x - (double)hi);
  }
  d[0] = u.q[0];
  d[1] = u.q[1];
}

// Short rows (len <= 64 * 8 * CH, rows 16-byte aligned): one wave per row (four rows per workgroup), every
// chunk read once into registers (up to CH per lane), the scale from a wave reduction, then split (in FP32:
// v - fp16(v) is exact) and stored.
// kscale (optional): value k of every row is multiplied by kscale[k] before the split.
template <int CH>
__global__ __launch_bounds__(256) void k_split_h3_short(int64_t n_rows, int64_t len, const float* __restrict__ src,
                                                        int64_t ld, uint4* __restrict__ dst,
                                                        float* __restrict__ scale,
                                                        const float* __restrict__ kscale) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n_rows) return;  // whole waves leave; no barrier follows
  const float* x = src + row * ld;
  const int lane = threadIdx.x & 63, nch = (int)(len / 8);
  float4_t v[CH][2];
  float m = 0.0f;
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int c = lane + 64 * k;
    if (c < nch) {
      v[k][0] = *(const float4_t*)(x + 8 * c);
      v[k][1] = *(const float4_t*)(x + 8 * c + 4);
      if (kscale) {
        v[k][0] *= *(const float4_t*)(kscale + 8 * c);
        v[k][1] *= *(const float4_t*)(kscale + 8 * c + 4);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) m = fmaxf(m, fmaxf(fabsf(v[k][0][q]), fabsf(v[k][1][q])));
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  const float s = pow2_scale(m);
  if (lane == 0) scale[row] = s;
  const float inv = 1.0f / s;  // exact: s is a power of two
  uint4* d = dst + row * (len / 4);
#pragma unroll
  for (int k = 0; k < CH; ++k) {
    const int c = lane + 64 * k;
    if (c < nch) {
      half8_t h, l;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float y = (j < 4 ? v[k][0][j] : v[k][1][j - 4]) * inv;
        h[j] = (_Float16)y;
        l[j] = (_Float16)(y - (float)h[j]);
      }
      d[2 * c] = __builtin_bit_cast(uint4, h);
      d[2 * c + 1] = __builtin_bit_cast(uint4, l);
    }
  }
}

// One wave per row: the row's power-of-two scale (written to scale[row]) and its split copy.
// Rows are `len` values (a multiple of 8) at stride ld; split rows are 2 * len FP16 at stride 2 * len.
template <typename TIN>
__global__ __launch_bounds__(64) void k_split_h3(int64_t len, const TIN* __restrict__ src, int64_t ld,
                                                 uint4* __restrict__ dst, float* __restrict__ scale) {
  const int64_t row = blockIdx.x;
  const TIN* x = src + row * ld;
  const int lane = threadIdx.x;
  TIN m = 0;
  for (int64_t i = lane; i < len; i += 64) m = max(m, (TIN)fabs((double)x[i]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, (TIN)__shfl_xor(m, o, 64));
  const float s = pow2_scale(m);
  if (lane == 0) scale[row] = s;
  const double inv = 1.0 / (double)s;  // exact: s is a power of two
  uint4* d = dst + row * (len / 4);
  for (int64_t c = lane; c < len / 8; c += 64) split8(x + 8 * c, inv, d + 2 * c);
}

void split_h3(const float* src, int64_t n_rows, int64_t len, int64_t ld, uint16_t* dst, float* scale, hipStream_t s,
              const float* kscale) {
  if (n_rows == 0) return;
  KFMM_REQUIRE(len % 8 == 0, "split_h3: row length must be a multiple of 8");
  const bool aligned = ld % 4 == 0 && ((uintptr_t)src & 15) == 0;
  KFMM_REQUIRE(!kscale || (aligned && len <= 64 * 8 * 2 && ((uintptr_t)kscale & 15) == 0),
               "split_h3: per-value scales need aligned rows of at most 1024 values");
  const unsigned nblk = (unsigned)((n_rows + 3) / 4);
  if (aligned && len <= 64 * 8)
    hipLaunchKernelGGL((k_split_h3_short<1>), dim3(nblk), dim3(256), 0, s, n_rows, len, src, ld, (uint4*)dst, scale,
                       kscale);
  else if (aligned && len <= 64 * 8 * 2)
    hipLaunchKernelGGL((k_split_h3_short<2>), dim3(nblk), dim3(256), 0, s, n_rows, len, src, ld, (uint4*)dst, scale,
                       kscale);
  else
    hipLaunchKernelGGL((k_split_h3<float>), dim3((unsigned)n_rows), dim3(64), 0, s, len, src, ld, (uint4*)dst,
                       scale);
  KFMM_HIP(hipGetLastError());
}
void split_h3(const double* src, int64_t n_rows, int64_t len, int64_t ld, uint16_t* dst, float* scale,
              hipStream_t s) {
  if (n_rows == 0) return;
  KFMM_REQUIRE(len % 8 == 0, "split_h3: row length must be a multiple of 8");
  hipLaunchKernelGGL((k_split_h3<double>), dim3((unsigned)n_rows), dim3(64), 0, s, len, src, ld, (uint4*)dst, scale);
  KFMM_HIP(hipGetLastError());
}

}  // namespace kfmm
