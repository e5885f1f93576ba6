// Batched gather/scatter GEMM on the matrix cores (see gemm.h).
//
// MFMA operand layout used (wave64, 16x16 output block):
//   v_mfma_{f64,f32}_16x16x4 : lane l holds A[l%16][l/16], B[l/16][l%16];
//   v_mfma_f32_16x16x32_bf16 : lane l holds A[l%16][8(l/16)+0..7], B[8(l/16)+0..7][l%16];
//   accumulator (FP32 outputs): lane l holds C[4(l/16)+v][l%16], v = 0..3;
//   accumulator (FP64 output) : lane l holds C[l/16+4v][l%16], v = 0..3.
#include "common.h"
#include "gemm.h"
#include "tree.h"

namespace kfmm {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

template <typename T>
__device__ __forceinline__ void store_out(T* p, T v, int mode) {
  if (mode == kStore)
    *p = v;
  else if (mode == kAdd)
    *p += v;
  else
    unsafeAtomicAdd(p, v);
}

// FP64 / FP32 variant: BK = 16 per LDS stage, 4 MFMA k-steps of 4.  Outputs of type TY (FP32 products
// may be accumulated into FP64 so that atomic scatter order does not change the result beyond FP64 rounding).
template <typename T, typename TY>
__global__ __launch_bounds__(256) void k_gemm_f(const T* __restrict__ A, int NC, const int4* __restrict__ tiles,
                                                const int* __restrict__ in_idx, const int* __restrict__ out_idx,
                                                const double* __restrict__ scale, const T* __restrict__ X,
                                                TY* __restrict__ Y, int mode) {
  constexpr int BK = 16, BM = kGemmBM, BN = kGemmBN, TM = kGemmTM;
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  const int4 tile = tiles[blockIdx.x];
  const int r0 = blockIdx.y * BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T* Aop = A + (size_t)tile.x * NC * NC;
  // global -> register staging: A tile BM x BK (row-major rows of 16), B tile BK x BN (column gathers)
  constexpr int A_ELEMS = BM * BK / 256;  // 6 per thread
  constexpr int B_ELEMS = BK * BN / 256;  // 4 per thread
  T ra[A_ELEMS], rb[B_ELEMS];
  // B: thread -> (column c = tid / 4, k-quad q = tid % 4)
  const int bc = tid >> 2, bq = tid & 3;
  const int col_ok = bc < tile.z;
  const T* xcol = X + (size_t)(col_ok ? in_idx[tile.y + bc] : 0) * NC;
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < A_ELEMS; ++e) {
      int lin = tid + 256 * e;  // over BM*BK, row-major in the tile
      int row = lin / BK, kk = lin % BK;
      ra[e] = Aop[(size_t)(r0 + row) * NC + k0 + kk];
    }
#pragma unroll
    for (int e = 0; e < B_ELEMS; ++e) rb[e] = col_ok ? xcol[k0 + 4 * bq + e] : T(0);
  };
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < A_ELEMS; ++e) {
      int lin = tid + 256 * e;
      As[lin % BK][lin / BK] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < B_ELEMS; ++e) Bs[4 * bq + e][bc] = rb[e];
  };
  typedef typename std::conditional<sizeof(T) == 8, double4_t, float4_t>::type acc_t;
  acc_t acc[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) acc[t] = acc_t{0, 0, 0, 0};
  const int nk = NC / BK;
  load(0);
  stash();
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      T b = Bs[ks * 4 + (lane >> 4)][wave * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        T a = As[ks * 4 + (lane >> 4)][t * 16 + (lane & 15)];
        if constexpr (sizeof(T) == 8)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        else
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      stash();
      __syncthreads();
    }
  }
  const int c = wave * 16 + (lane & 15);
  if (c >= tile.z) return;
  const int col = tile.y + c;
  TY* ycol = Y + (size_t)out_idx[col] * NC + r0;
  const TY sc = scale ? (TY)scale[col] : TY(1);
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = sizeof(T) == 8 ? t * 16 + (lane >> 4) + 4 * v : t * 16 + 4 * (lane >> 4) + v;
      store_out(ycol + row, sc * (TY)acc[t][v], mode);
    }
}

// BF16 inputs, FP32 accumulation: BK = 32 per LDS stage, one MFMA k-step.
template <typename TY>
__global__ __launch_bounds__(256) void k_gemm_bf16(const __bf16* __restrict__ A, int NC, const int4* __restrict__ tiles,
                                                   const int* __restrict__ in_idx, const int* __restrict__ out_idx,
                                                   const double* __restrict__ scale, const __bf16* __restrict__ X,
                                                   TY* __restrict__ Y, int mode) {
  constexpr int BK = 32, BM = kGemmBM, BN = kGemmBN, TM = kGemmTM, PAD = 8;
  __shared__ __attribute__((aligned(16))) __bf16 As[BM][BK + PAD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][BK + PAD];
  const int4 tile = tiles[blockIdx.x];
  const int r0 = blockIdx.y * BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const __bf16* Aop = A + (size_t)tile.x * NC * NC;
  // A tile: BM rows x 32 bf16 = BM*4 chunks of 8 (16 bytes); B tile: 64 columns x 4 chunks
  constexpr int A_CH = BM * BK / 8 / 256;  // 1.5 -> use 2 with guard
  const int bc = tid >> 2, bq = tid & 3;
  const int col_ok = bc < tile.z;
  const __bf16* xcol = X + (size_t)(col_ok ? in_idx[tile.y + bc] : 0) * NC;
  uint4 ra[2], rb;
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      int lin = tid + 256 * e;
      if (lin < BM * 4) {
        int row = lin >> 2, q = lin & 3;
        ra[e] = *(const uint4*)(Aop + (size_t)(r0 + row) * NC + k0 + 8 * q);
      }
    }
    rb = col_ok ? *(const uint4*)(xcol + k0 + 8 * bq) : make_uint4(0, 0, 0, 0);
  };
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      int lin = tid + 256 * e;
      if (lin < BM * 4) *(uint4*)&As[lin >> 2][8 * (lin & 3)] = ra[e];
    }
    *(uint4*)&Bs[bc][8 * bq] = rb;
  };
  (void)A_CH;
  float4_t acc[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) acc[t] = float4_t{0, 0, 0, 0};
  const int nk = NC / BK;
  load(0);
  stash();
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * BK);
    bf16x8_t b = *(const bf16x8_t*)&Bs[wave * 16 + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      bf16x8_t a = *(const bf16x8_t*)&As[t * 16 + (lane & 15)][8 * (lane >> 4)];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
    __syncthreads();
    if (kt + 1 < nk) {
      stash();
      __syncthreads();
    }
  }
  const int c = wave * 16 + (lane & 15);
  if (c >= tile.z) return;
  const int col = tile.y + c;
  TY* ycol = Y + (size_t)out_idx[col] * NC + r0;
  const TY sc = scale ? (TY)scale[col] : TY(1);
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) store_out(ycol + t * 16 + 4 * (lane >> 4) + v, sc * (TY)acc[t][v], mode);
}

static void check_job(const GemmJob& job, int NC) {
  if (NC % kGemmBM != 0) throw Error(-1, "gemm: NC must be a multiple of the row block");
}

void gemm_f64(const GemmJob& job, const double* A, int NC, const double* X, double* Y, int mode, hipStream_t s) {
  if (job.n_tiles == 0) return;
  check_job(job, NC);
  hipLaunchKernelGGL((k_gemm_f<double, double>), dim3(job.n_tiles, NC / kGemmBM), dim3(256), 0, s, A, NC, job.tiles,
                     job.in_idx, job.out_idx, job.scale, X, Y, mode);
  KFMM_HIP(hipGetLastError());
}

template <typename TY>
static void gemm_f32_t(const GemmJob& job, const float* A, int NC, const float* X, TY* Y, int mode, hipStream_t s) {
  if (job.n_tiles == 0) return;
  check_job(job, NC);
  hipLaunchKernelGGL((k_gemm_f<float, TY>), dim3(job.n_tiles, NC / kGemmBM), dim3(256), 0, s, A, NC, job.tiles,
                     job.in_idx, job.out_idx, job.scale, X, Y, mode);
  KFMM_HIP(hipGetLastError());
}
void gemm_f32(const GemmJob& job, const float* A, int NC, const float* X, float* Y, int mode, hipStream_t s) {
  gemm_f32_t(job, A, NC, X, Y, mode, s);
}
void gemm_f32(const GemmJob& job, const float* A, int NC, const float* X, double* Y, int mode, hipStream_t s) {
  gemm_f32_t(job, A, NC, X, Y, mode, s);
}

template <typename TY>
static void gemm_bf16_t(const GemmJob& job, const __hip_bfloat16* A, int NC, const __hip_bfloat16* X, TY* Y, int mode,
                        hipStream_t s) {
  if (job.n_tiles == 0) return;
  check_job(job, NC);
  hipLaunchKernelGGL((k_gemm_bf16<TY>), dim3(job.n_tiles, NC / kGemmBM), dim3(256), 0, s, (const __bf16*)A, NC,
                     job.tiles, job.in_idx, job.out_idx, job.scale, (const __bf16*)X, Y, mode);
  KFMM_HIP(hipGetLastError());
}
void gemm_bf16(const GemmJob& job, const __hip_bfloat16* A, int NC, const __hip_bfloat16* X, float* Y, int mode,
               hipStream_t s) {
  gemm_bf16_t(job, A, NC, X, Y, mode, s);
}
void gemm_bf16(const GemmJob& job, const __hip_bfloat16* A, int NC, const __hip_bfloat16* X, double* Y, int mode,
               hipStream_t s) {
  gemm_bf16_t(job, A, NC, X, Y, mode, s);
}

}  // namespace kfmm

// ------------------------------------------------------------------ test hook (see kfmm_selftest_gemm)
namespace kfmm {
void selftest_gemm(int precision, const void* A, int NC, const void* X, void* Y, const int* op, const int* in,
                   const int* out, const double* scale, int ncols, int mode, hipStream_t s) {
  Arena a;
  std::vector<int4> tiles;
  int i = 0;
  while (i < ncols) {
    int j = i;
    while (j < ncols && op[j] == op[i] && j - i < kGemmBN) ++j;
    tiles.push_back(make_int4(op[i], i, j - i, 0));
    i = j;
  }
  GemmJob job;
  job.n_tiles = (int)tiles.size();
  job.tiles = a.get<int4>(tiles.size() + 1);
  job.in_idx = a.get<int>(ncols + 1);
  job.out_idx = a.get<int>(ncols + 1);
  job.scale = scale ? a.get<double>(ncols + 1) : nullptr;
  KFMM_HIP(hipMemcpyAsync(job.tiles, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  KFMM_HIP(hipMemcpyAsync(job.in_idx, in, ncols * sizeof(int), hipMemcpyHostToDevice, s));
  KFMM_HIP(hipMemcpyAsync(job.out_idx, out, ncols * sizeof(int), hipMemcpyHostToDevice, s));
  if (scale) KFMM_HIP(hipMemcpyAsync(job.scale, scale, ncols * sizeof(double), hipMemcpyHostToDevice, s));
  if (precision == 0)
    gemm_f64(job, (const double*)A, NC, (const double*)X, (double*)Y, mode, s);
  else if (precision == 1)
    gemm_f32(job, (const float*)A, NC, (const float*)X, (float*)Y, mode, s);
  else
    gemm_bf16(job, (const __hip_bfloat16*)A, NC, (const __hip_bfloat16*)X, (float*)Y, mode, s);
  KFMM_HIP(hipStreamSynchronize(s));
}
}  // namespace kfmm
