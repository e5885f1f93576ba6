// Split-FP16 gather/scatter GEMM (see gemm.h): FP32-accurate products on the FP16 matrix cores.
//
// Every operand value v, divided by a power-of-two scale s (one per operator, one per X vector) that puts
// the largest |v / s| in [2^14, 2^15), is held as two FP16 numbers hi = fp16(v / s), lo = fp16(v / s - hi).
// The scale uses the top of the FP16 range so that lo stays a normal number for every entry down to
// 2^-17 of the largest: those carry about 22 significant bits, smaller ones an absolute error of at most
// 2^-39 of the largest (with the largest mapped to 1 instead, lo would always be subnormal and every
// entry would carry an absolute error of 2^-25 of the largest, which the pseudo-inverse of the downward
// pass amplifies in directions with small entries).  A product is accumulated in FP32 as
// Ah Xh + Ah Xl + Al Xh; the dropped Al Xl term is of relative size 2^-22.  Each product costs three
// v_mfma_f32_16x16x32_f16 (16 cycles each) instead of eight v_mfma_f32_16x16x4_f32 (32 cycles each).
//
// Split layout: a row of K values is stored as K/8 chunks of 16 FP16 numbers, [hi of 8 consecutive
// entries][lo of the same 8], so that one 16-byte load gives one MFMA operand.
#include "gemm_kernels.h"

namespace kfmm {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// Workgroup tile (16*TM) rows x (64*TN) columns, 4 waves side by side: wave w owns columns
// [16 TN w, 16 TN (w+1)) (TN 16-column MFMA blocks) and all rows.  Larger tiles read fewer operand bytes
// per product, which is what limits this kernel (at the M2L shape 160 x 192 tiles took 174 us where
// 96 x 128 took 226 us).  The operator tile (hi and lo) is staged in LDS per 32-value k-stage,
// double-buffered (one barrier per stage); LDS rows are 36 words apart so that the 16-byte operand reads
// of any 16 consecutive lanes fall in distinct banks.  X operands are private to a wave and are loaded
// straight from global memory into registers, one stage ahead.
template <int TM, int TN>
__global__ __launch_bounds__(256) void k_gemm_h3(const u32x4_t* __restrict__ A, GemmDims dm,
                                                 const float* __restrict__ a_scale, const int4* __restrict__ tiles,
                                                 const int* __restrict__ in_idx, const int* __restrict__ out_idx,
                                                 const double* __restrict__ scale, const u32x4_t* __restrict__ X,
                                                 const float* __restrict__ x_scale, float* __restrict__ Y, int mode) {
  constexpr int BM = 16 * TM, RW = 36;
  constexpr int A_PER_THR = BM * 8 / 256;  // 16-byte pieces of the operator tile per thread and stage
  static_assert(BM * 8 % 256 == 0, "operator tile must split into 16-byte pieces");
  __shared__ __attribute__((aligned(16))) uint32_t As[2][BM * RW];
  const int lid = xcd_logical_id();
  const int4 tile = tiles[lid / gridDim.y];
  const int r0 = (lid % gridDim.y) * BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int rowq = dm.K / 4;  // 16-byte pieces per split row
  const u32x4_t* Aop = A + ((size_t)tile.x * dm.M + r0) * rowq;
  const u32x4_t* xc[TN];
  bool ok[TN];
  int src[TN];
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int j = wave * 16 * TN + u * 16 + i16;
    ok[u] = j < tile.z;
    src[u] = ok[u] ? in_idx[tile.y + j] : 0;
    xc[u] = X + (size_t)src[u] * (dm.ldx / 8);
  }
  u32x4_t ra[A_PER_THR], nbh[TN], nbl[TN];
  half8_t bh[TN], bl[TN];
  auto load = [&](int st) {
#pragma unroll
    for (int e = 0; e < A_PER_THR; ++e) {
      const int lin = tid + 256 * e;
      ra[e] = Aop[(size_t)(lin >> 3) * rowq + 8 * st + (lin & 7)];
    }
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      if (ok[u]) {
        nbh[u] = xc[u][8 * st + 2 * g];
        nbl[u] = xc[u][8 * st + 2 * g + 1];
      } else {
        nbh[u] = u32x4_t{0, 0, 0, 0};
        nbl[u] = u32x4_t{0, 0, 0, 0};
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < A_PER_THR; ++e) {
      const int lin = tid + 256 * e;
      *(u32x4_t*)&As[buf][(lin >> 3) * RW + 4 * (lin & 7)] = ra[e];
    }
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      bh[u] = __builtin_bit_cast(half8_t, nbh[u]);
      bl[u] = __builtin_bit_cast(half8_t, nbl[u]);
    }
  };
  float4_t acc[TM][TN];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = float4_t{0, 0, 0, 0};
  auto compute = [&](int cur) {
    // every operator fragment of the stage is read before the first product, so the products of one
    // stage issue back to back
    half8_t ah[TM], al[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int w = (t * 16 + i16) * RW + 8 * g;
      ah[t] = *(const half8_t*)&As[cur][w];
      al[t] = *(const half8_t*)&As[cur][w + 4];
    }
#pragma unroll
    for (int t = 0; t < TM; ++t) {
#pragma unroll
      for (int u = 0; u < TN; ++u) acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[t], bh[u], acc[t][u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < TN; ++u) acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[t], bl[u], acc[t][u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < TN; ++u) acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[t], bh[u], acc[t][u], 0, 0, 0);
    }
    // issue order: the fragments of rows 0 and 1, then the products of row t each followed by the reads
    // of row t + 2, so that LDS latency hides behind products already issued
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      __builtin_amdgcn_sched_group_barrier(0x008, 3 * TN, 0);
      if (t + 2 < TM) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
    }
  };
  const int ns = dm.K / 32;
  load(0);
  stash(0);
  __syncthreads();
  for (int st = 0; st < ns; ++st) {
    const int cur = st & 1;
    if (st + 1 < ns) load(st + 1);
    compute(cur);
    // buffer cur ^ 1 was last read in stage st - 1, which every wave has left (barrier below)
    if (st + 1 < ns) stash(cur ^ 1);
    __syncthreads();
  }
  const float sa = a_scale[tile.x];
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    if (!ok[u]) continue;
    const int col = tile.y + wave * 16 * TN + u * 16 + i16;
    const float sc = x_scale[src[u]] * (scale ? (float)scale[col] : 1.0f);
    float* ycol = Y + (size_t)out_idx[col] * dm.ldy + r0 + 4 * g;
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const float4_t v = (acc[t][u] * sa) * sc;  // scales applied one at a time (no product underflow)
      if (mode == kStore) {
        *(float4_t*)(ycol + t * 16) = v;
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) store_out(ycol + t * 16 + q, v[q], mode);
      }
    }
  }
}

template <int TM>
static void launch_h3(const GemmJob& job, const uint16_t* A, const float* a_scale, GemmDims d, const uint16_t* X,
                      const float* x_scale, float* Y, int mode, hipStream_t s) {
  const dim3 grid(job.n_tiles, d.M / (16 * TM));
  const auto* a = (const u32x4_t*)A;
  const auto* x = (const u32x4_t*)X;
  if (job.cols_per_tile <= 64)
    hipLaunchKernelGGL((k_gemm_h3<TM, 1>), grid, dim3(256), 0, s, a, d, a_scale, job.tiles, job.in_idx, job.out_idx,
                       job.scale, x, x_scale, Y, mode);
  else if (job.cols_per_tile <= 128)
    hipLaunchKernelGGL((k_gemm_h3<TM, 2>), grid, dim3(256), 0, s, a, d, a_scale, job.tiles, job.in_idx, job.out_idx,
                       job.scale, x, x_scale, Y, mode);
  else
    hipLaunchKernelGGL((k_gemm_h3<TM, 3>), grid, dim3(256), 0, s, a, d, a_scale, job.tiles, job.in_idx, job.out_idx,
                       job.scale, x, x_scale, Y, mode);
}

void gemm_h3(const GemmJob& job, const uint16_t* A, const float* a_scale, GemmDims d, const uint16_t* X,
             const float* x_scale, float* Y, int mode, hipStream_t s) {
  if (job.n_tiles == 0) return;
  KFMM_REQUIRE(job.cols_per_tile <= 3 * kGemmBN, "gemm_h3: at most 192 columns per tile");
  KFMM_REQUIRE(d.K % 32 == 0 && d.ldx % 8 == 0 && d.ldx >= 2 * d.K, "gemm_h3: bad K or ldx");
  if (mode == kStore) KFMM_REQUIRE(d.ldy % 4 == 0, "gemm_h3: ldy must be a multiple of 4 for vector stores");
  // 160-row blocks for wide tiles (the M2L contraction at r = 480), else 96- or 64-row blocks
  if (d.M % 160 == 0 && job.cols_per_tile > 2 * kGemmBN)
    launch_h3<10>(job, A, a_scale, d, X, x_scale, Y, mode, s);
  else if (d.M % 96 == 0)
    launch_h3<6>(job, A, a_scale, d, X, x_scale, Y, mode, s);
  else if (d.M % 64 == 0)
    launch_h3<4>(job, A, a_scale, d, X, x_scale, Y, mode, s);
  else
    throw Error(-1, "gemm_h3: M must be a multiple of 96 or 64");
  KFMM_HIP(hipGetLastError());
}

}  // namespace kfmm
