// Kernels and launch helpers of the batched gather/scatter GEMM (see gemm.h), shared by gemm.hip (FP64,
// test hook) and gemm_f32.hip (FP32), which are compiled with different MFMA register forms.
//
// MFMA operand layout used (wave64, 16x16 output block):
//   v_mfma_{f64,f32}_16x16x4 : lane l holds A[l%16][l/16], B[l/16][l%16];
//   accumulator (FP32 outputs): lane l holds C[4(l/16)+v][l%16], v = 0..3;
//   accumulator (FP64 output) : lane l holds C[l/16+4v][l%16], v = 0..3.
#pragma once
#include "common.h"
#include "gemm.h"
#include "tree.h"

namespace kfmm {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// The dispatcher hands workgroups to the 8 XCDs round-robin by linear id (x fastest).  Remapped so that
// each XCD receives a contiguous range of logical ids: with the row block fastest in the logical order,
// the workgroups of one column tile (same operator, same X columns) share one XCD's L2, and so do the
// consecutive tiles of one operator.
__device__ __forceinline__ int xcd_logical_id() {
  const int n = gridDim.x * gridDim.y;
  const int id = blockIdx.x + blockIdx.y * gridDim.x;
  const int q = n >> 3, r = n & 7, x = id & 7;
  return x * q + min(x, r) + (id >> 3);
}

template <typename T>
__device__ __forceinline__ void store_out(T* p, T v, int mode) {
  if (mode == kStore)
    *p = v;
  else if (mode == kAdd)
    *p += v;
  else
    unsafeAtomicAdd(p, v);
}

// FP64 / FP32 variant.  Workgroup tile (16*TM) x (64*TN): wave w owns columns [16*TN*w, 16*TN*(w+1))
// and all rows; the K dimension advances BK per stage, the next stage being loaded into registers while
// the current one is multiplied.  NBUF = 2: two LDS buffers, stage k+1 is written while stage k is
// multiplied (one barrier per stage; for launches with about one workgroup per compute unit).  NBUF = 1:
// half the LDS, so more workgroups fit on a compute unit (for large launches).  Outputs of type TY (FP32
// products may be accumulated into FP64).
template <typename T, typename TY, int TN, int BK, int NBUF, int TM>
__global__ __launch_bounds__(256) void k_gemm_f(const T* __restrict__ A, GemmDims dm, const int4* __restrict__ tiles,
                                                const int* __restrict__ in_idx, const int* __restrict__ out_idx,
                                                const double* __restrict__ scale, const T* __restrict__ X,
                                                TY* __restrict__ Y, int mode) {
  constexpr int BM = 16 * TM, BN = 64 * TN;
  constexpr int VA = 16 / sizeof(T);  // elements per 16-byte global load
  constexpr int A_VEC = BM * BK / VA / 256;  // vector loads per thread for the A tile
  constexpr int B_THR_PER_COL = 256 / BN;    // threads sharing one column of the X tile
  constexpr int B_ELEMS = BK / B_THR_PER_COL;
  static_assert(BM * BK % (VA * 256) == 0, "A tile must split into 16-byte loads");
  static_assert(B_ELEMS % VA == 0, "B tile must split into 16-byte loads");
  __shared__ T As[NBUF][BM][BK + 1];
  __shared__ T Bs[NBUF][BK][BN + 1];
  const int lid = xcd_logical_id();
  const int4 tile = tiles[lid / gridDim.y];
  const int r0 = (lid % gridDim.y) * BM;
  // a tile of rank m (tile.w = m > 0, a multiple of 32; square operators in M x K slots) multiplies the leading
  // m x m block of its operator, stored row-major with rows of m values at the start of the slot and zeros
  // after it (as in k_gemm_h3)
  const int mr = tile.w > 0 ? tile.w : dm.M, kk = tile.w > 0 ? tile.w : dm.K;
  if (r0 >= mr) return;  // the whole workgroup, before any barrier
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T* Aop = A + (size_t)tile.x * dm.M * dm.K;
  typedef typename std::conditional<sizeof(T) == 8, double2, float4>::type vec_t;
  vec_t ra[A_VEC], rb[B_ELEMS / VA];
  const int bc = tid / B_THR_PER_COL, bq = tid % B_THR_PER_COL;
  const int col_ok = bc < tile.z;
  const T* xcol = X + (size_t)(col_ok ? in_idx[tile.y + bc] : 0) * dm.ldx;
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < A_VEC; ++e) {
      int lin = tid + 256 * e;  // vector index in the tile, row-major
      int row = lin / (BK / VA), kv = lin % (BK / VA);
      ra[e] = *(const vec_t*)(Aop + (size_t)(r0 + row) * kk + k0 + kv * VA);
    }
#pragma unroll
    for (int e = 0; e < B_ELEMS / VA; ++e) {
      if (col_ok)
        rb[e] = *(const vec_t*)(xcol + k0 + bq * B_ELEMS + e * VA);
      else
        rb[e] = vec_t{};
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < A_VEC; ++e) {
      int lin = tid + 256 * e;
      int row = lin / (BK / VA), kv = lin % (BK / VA);
      const T* v = (const T*)&ra[e];
#pragma unroll
      for (int q = 0; q < VA; ++q) As[buf][row][kv * VA + q] = v[q];
    }
#pragma unroll
    for (int e = 0; e < B_ELEMS / VA; ++e) {
      const T* v = (const T*)&rb[e];
#pragma unroll
      for (int q = 0; q < VA; ++q) Bs[buf][bq * B_ELEMS + e * VA + q][bc] = v[q];
    }
  };
  typedef typename std::conditional<sizeof(T) == 8, double4_t, float4_t>::type acc_t;
  acc_t acc[TM][TN];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int u = 0; u < TN; ++u) acc[t][u] = acc_t{0, 0, 0, 0};
  auto compute = [&](int cur) {
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      T b[TN];
#pragma unroll
      for (int u = 0; u < TN; ++u) b[u] = Bs[cur][ks * 4 + (lane >> 4)][(wave * TN + u) * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        T a = As[cur][t * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
#pragma unroll
        for (int u = 0; u < TN; ++u) {
          if constexpr (sizeof(T) == 8)
            acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[u], acc[t][u], 0, 0, 0);
          else
            acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[u], acc[t][u], 0, 0, 0);
        }
      }
    }
  };
  const int nk = kk / BK;
  load(0);
  stash(0);
  if constexpr (NBUF == 2) {
    if (nk > 1) load(BK);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      // buffer cur ^ 1 was last read in iteration kt - 1, which every wave has left (barrier below)
      if (kt + 1 < nk) stash(cur ^ 1);
      if (kt + 2 < nk) load((kt + 2) * BK);
      compute(cur);
      __syncthreads();
    }
  } else {
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      if (kt + 1 < nk) load((kt + 1) * BK);
      compute(0);
      __syncthreads();
      if (kt + 1 < nk) {
        stash(0);
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int u = 0; u < TN; ++u) {
    const int c = (wave * TN + u) * 16 + (lane & 15);
    if (c >= tile.z) continue;
    const int col = tile.y + c;
    TY* ycol = Y + (size_t)out_idx[col] * dm.ldy + r0;
    const TY sc = scale ? (TY)scale[col] : TY(1);
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      if (r0 + 16 * t >= mr) break;  // rows past the tile's rank
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = sizeof(T) == 8 ? t * 16 + (lane >> 4) + 4 * v : t * 16 + 4 * (lane >> 4) + v;
        store_out(ycol + row, sc * (TY)acc[t][u][v], mode);
      }
    }
  }
}

// Split-K variant for launches with few columns (the upper levels of the M2M / L2L passes), where the
// tiled kernel above cannot fill the chip.  A workgroup computes a (16*TM) x 16 block; its four waves
// take contiguous quarters of the K range and read A and X straight from global memory (there is no
// reuse to stage through LDS), keeping PD chunks of loads in flight; the four partial blocks are summed
// in LDS in wave order, so results do not depend on scheduling.  Each lane loads 32 bytes of a row of A
// (a full 128-byte line per row across the four lane groups) and of a column of X, and feeds them to
// consecutive MFMA k-steps: lane group g = l/16 holds k-indices k0 + VA*g + q (q = 0..VA-1), and since
// A and X use the same assignment the products still pair A[i][k] with X[k][j].
// Grid: x = tile * SUB + 16-column sub-block, y = row block of 16*TM rows (remapped per XCD as above).
template <typename T, typename TY, int TM>
__global__ __launch_bounds__(256) void k_gemm_sk(const T* __restrict__ A, GemmDims dm, const int4* __restrict__ tiles,
                                                 int sub_per_tile, const int* __restrict__ in_idx,
                                                 const int* __restrict__ out_idx, const double* __restrict__ scale,
                                                 const T* __restrict__ X, TY* __restrict__ Y, int mode) {
  constexpr int BM = 16 * TM, PD = 2;
  constexpr int VH = 16 / sizeof(T);  // values per 16-byte load
  constexpr int VA = 2 * VH;          // values per lane and row per chunk (two loads)
  constexpr int KC = 4 * VA;          // k-values per chunk (4 lane groups)
  typedef typename std::conditional<sizeof(T) == 8, double2, float4>::type vec_t;
  typedef typename std::conditional<sizeof(T) == 8, double4_t, float4_t>::type acc_t;
  struct Chunk {
    vec_t a[TM][2], b[2];
  };
  __shared__ T red[4][BM][17];
  const int lid = xcd_logical_id();
  const int bx = lid / gridDim.y;
  const int4 tile = tiles[bx / sub_per_tile];
  const int c0 = (bx % sub_per_tile) * 16;
  if (c0 >= tile.z) return;  // whole workgroup: uniform exit before any barrier
  const int ncols = min(16, tile.z - c0);
  const int r0 = (lid % gridDim.y) * BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 15, g = lane >> 4;
  const T* Aop = A + (size_t)tile.x * dm.M * dm.K;
  const bool col_ok = i < ncols;
  const T* xcol = X + (size_t)(col_ok ? in_idx[tile.y + c0 + i] : 0) * dm.ldx;
  // this wave's chunks
  const int nch = dm.K / KC;
  const int ch0 = wave * nch / 4, ch1 = (wave + 1) * nch / 4;
  acc_t acc[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) acc[t] = acc_t{0, 0, 0, 0};
  Chunk buf[PD];
  auto load = [&](Chunk& c, int ch) {
    const int k = ch * KC + VA * g;
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const vec_t* p = (const vec_t*)(Aop + (size_t)(r0 + 16 * t + i) * dm.K + k);
      c.a[t][0] = p[0];
      c.a[t][1] = p[1];
    }
    if (col_ok) {
      c.b[0] = ((const vec_t*)(xcol + k))[0];
      c.b[1] = ((const vec_t*)(xcol + k))[1];
    } else {
      c.b[0] = vec_t{};
      c.b[1] = vec_t{};
    }
  };
  auto compute = [&](const Chunk& c) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < VH; ++q) {
        const T bq = ((const T*)&c.b[h])[q];
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          const T aq = ((const T*)&c.a[t][h])[q];
          if constexpr (sizeof(T) == 8)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq, bq, acc[t], 0, 0, 0);
          else
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq, bq, acc[t], 0, 0, 0);
        }
      }
  };
  // ring of PD chunks in flight; chunk ch lives in buf[(ch - ch0) % PD]
#pragma unroll
  for (int d = 0; d < PD; ++d)
    if (ch0 + d < ch1) load(buf[d], ch0 + d);
  for (int ch = ch0; ch < ch1; ch += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      if (ch + d < ch1) {
        compute(buf[d]);
        if (ch + d + PD < ch1) load(buf[d], ch + d + PD);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = sizeof(T) == 8 ? t * 16 + g + 4 * v : t * 16 + 4 * g + v;
      red[wave][row][i] = acc[t][v];
    }
  __syncthreads();
  for (int e = tid; e < BM * 16; e += 256) {
    const int row = e % BM, c = e / BM;
    if (c >= ncols) continue;
    const T sum = ((red[0][row][c] + red[1][row][c]) + red[2][row][c]) + red[3][row][c];
    const int col = tile.y + c0 + c;
    const TY sc = scale ? (TY)scale[col] : TY(1);
    store_out(Y + (size_t)out_idx[col] * dm.ldy + r0 + row, sc * (TY)sum, mode);
  }
}

inline void check_dims(const GemmDims& d) {
  if (!gemm_tm(d.M) || d.K % 32 != 0) throw Error(-1, "gemm: M must be a multiple of 96 or 128 and K of 32");
}

// A tiled workgroup runs its whole K loop alone (one per compute unit in small launches), so small
// launches are bound by that latency; the split-K kernel cuts them into more, shorter workgroups.  The
// crossover, measured on translation-pass shapes (NC = 960, 1 or 8 operators, FP64 with 64-column and
// FP32 with 128-column tiles), sits near 20k tile columns x row blocks.
inline bool use_split_k(const GemmJob& job, const GemmDims& d, int kernel) {
  if (job.ranked) return false;  // tiles of a given rank run on the tiled kernel only
  if (kernel != kGemmAuto) return kernel == kGemmSplitK;
  return (int64_t)job.n_tiles * job.cols_per_tile * d.M / 96 < 20480;
}

template <typename T, typename TY>
void launch_split_k(const GemmJob& job, const T* A, GemmDims d, const T* X, TY* Y, int mode, hipStream_t s) {
  const int sub = job.cols_per_tile / 16;
  if (d.M % 48 == 0)  // 48-row blocks
    hipLaunchKernelGGL((k_gemm_sk<T, TY, 3>), dim3(job.n_tiles * sub, d.M / 48), dim3(256), 0, s, A, d, job.tiles,
                       sub, job.in_idx, job.out_idx, job.scale, X, Y, mode);
  else  // M a multiple of 128: 64-row blocks
    hipLaunchKernelGGL((k_gemm_sk<T, TY, 4>), dim3(job.n_tiles * sub, d.M / 64), dim3(256), 0, s, A, d, job.tiles,
                       sub, job.in_idx, job.out_idx, job.scale, X, Y, mode);
}

// LDS-tiled launch: 64- or 128-column tiles (TN = 1, 2), 96- or 64-row blocks (TM = 6, 4), BK k-values
// per LDS stage; double-buffered LDS below ~4 workgroups per compute unit, single-buffered (more resident
// workgroups) above.
template <typename T, typename TY, int BK, int TM>
void launch_tiled_tm(const GemmJob& job, const T* A, GemmDims d, const T* X, TY* Y, int mode, hipStream_t s,
                     int kernel) {
  const dim3 grid(job.n_tiles, d.M / (16 * TM));
  const bool big = kernel == kGemmTiled1 || (kernel != kGemmTiled2 && (int64_t)grid.x * grid.y >= 1024);
  if (job.cols_per_tile > kGemmBN) {
    if (big)
      hipLaunchKernelGGL((k_gemm_f<T, TY, 2, BK, 1, TM>), grid, dim3(256), 0, s, A, d, job.tiles, job.in_idx,
                         job.out_idx, job.scale, X, Y, mode);
    else
      hipLaunchKernelGGL((k_gemm_f<T, TY, 2, BK, 2, TM>), grid, dim3(256), 0, s, A, d, job.tiles, job.in_idx,
                         job.out_idx, job.scale, X, Y, mode);
  } else {
    if (big)
      hipLaunchKernelGGL((k_gemm_f<T, TY, 1, BK, 1, TM>), grid, dim3(256), 0, s, A, d, job.tiles, job.in_idx,
                         job.out_idx, job.scale, X, Y, mode);
    else
      hipLaunchKernelGGL((k_gemm_f<T, TY, 1, BK, 2, TM>), grid, dim3(256), 0, s, A, d, job.tiles, job.in_idx,
                         job.out_idx, job.scale, X, Y, mode);
  }
}

template <typename T, typename TY, int BK>
void launch_tiled(const GemmJob& job, const T* A, GemmDims d, const T* X, TY* Y, int mode, hipStream_t s,
                  int kernel) {
  if (gemm_tm(d.M) == 6)
    launch_tiled_tm<T, TY, BK, 6>(job, A, d, X, Y, mode, s, kernel);
  else  // M a multiple of 128: 64-row blocks (twice the workgroups of 128-row blocks)
    launch_tiled_tm<T, TY, BK, 4>(job, A, d, X, Y, mode, s, kernel);
}

template <typename T, typename TY>
void gemm_t(const GemmJob& job, const T* A, GemmDims d, const T* X, TY* Y, int mode, hipStream_t s,
                   int kernel) {
  if (job.n_tiles == 0) return;
  check_dims(d);
  constexpr int BK = sizeof(T) == 8 ? 16 : 32;
  if (use_split_k(job, d, kernel))
    launch_split_k(job, A, d, X, Y, mode, s);
  else
    launch_tiled<T, TY, BK>(job, A, d, X, Y, mode, s, kernel);
  KFMM_HIP(hipGetLastError());
}

}  // namespace kfmm
