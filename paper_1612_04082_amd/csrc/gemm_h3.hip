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
// per product (at the M2L shape, r = 480, 160 x 192 tiles took 174 us where 96 x 128 took 226 us), and
// 160 x 128 tiles beat both in the full evaluation (about 4% below 160 x 192: the same occupancy, half as
// many workgroups again).  The operator tile (hi and lo) is staged in LDS per 32-value k-stage,
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
  // A tile of rank m (tile.w = m > 0, a multiple of 32; operators in M x K slots, square) multiplies the
  // leading m x m block of its operator, stored row-major with rows of m values at the start of the slot and
  // zeros after it: row blocks at or past m have nothing to do, a row block across m reads rows of zeros
  // (inside the slot) and stores only its rows below m, and the contraction runs over m.
  const int mr = tile.w > 0 ? tile.w : dm.M, kk = tile.w > 0 ? tile.w : dm.K;
  if (r0 >= mr) return;  // the whole workgroup, before any barrier
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int rowq = kk / 4;  // 16-byte pieces per split row
  const u32x4_t* Aop = A + (size_t)tile.x * ((size_t)dm.M * dm.K / 4) + (size_t)r0 * rowq;
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
  const int ns = kk / 32;
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
      if (r0 + 16 * t >= mr) break;  // rows past the tile's rank (16-row blocks: m is a multiple of 32)
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

// Variant for launches with few workgroups (fewer than about two per compute unit), where the kernel above
// waits on memory latency: the same tiles and LDS staging, with PD stages of loads in flight in a ring of
// PD register sets.  The loads of stage i + PD are issued before stage i is multiplied (a scheduling
// barrier keeps them there), and stage i + 1 moves to LDS after it.  Every load is unconditional (the
// columns past a ragged tile's end read column 0, whose products are never stored; stage indices clamp
// to the last stage), so the compiler counts the loads in flight exactly instead of draining them at each
// stage.  KW groups of 4 waves take contiguous parts of the k range, each with its own LDS buffers, and
// their partial tiles are summed in LDS in group order, so results do not depend on scheduling.
template <int TM, int TN, int KW, int PD>
__global__ __launch_bounds__(256 * KW) void k_gemm_h3k(const u32x4_t* __restrict__ A, GemmDims dm,
                                                      const float* __restrict__ a_scale,
                                                      const int4* __restrict__ tiles, const int* __restrict__ in_idx,
                                                      const int* __restrict__ out_idx,
                                                      const double* __restrict__ scale, const u32x4_t* __restrict__ X,
                                                      const float* __restrict__ x_scale, float* __restrict__ Y,
                                                      int mode) {
  constexpr int BM = 16 * TM, RW = 36;
  constexpr int NP = BM * 8;                // 16-byte pieces of the operator tile per stage
  constexpr int APT = (NP + 255) / 256;     // pieces per thread (the last round partial when NP % 256 != 0)
  constexpr int LDS_TILE = KW * 2 * BM * RW, LDS_RED = KW > 1 ? BM * 64 * TN : 0;
  __shared__ __attribute__((aligned(16))) uint32_t lds[LDS_TILE > LDS_RED ? LDS_TILE : LDS_RED];
  const int lid = xcd_logical_id();
  const int4 tile = tiles[lid / gridDim.y];
  const int r0 = (lid % gridDim.y) * BM;
  const int tid = threadIdx.x & 255, kg = threadIdx.x >> 8;
  const int lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  uint32_t* const As = lds + kg * 2 * BM * RW;  // this group's two stage buffers
  const int rowq = dm.K / 4;                    // 16-byte pieces per split row
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
  const int ns = dm.K / 32;
  const int s0 = kg * ns / KW, my = (kg + 1) * ns / KW - s0;  // this group's stages (>= 1, see gemm_h3)
  const int nmax = (ns + KW - 1) / KW;                        // stages of the longest group
  struct Stage {
    u32x4_t a[APT], xh[TN], xl[TN];
  };
  Stage ring[PD];
  half8_t bh[TN], bl[TN];
  auto load = [&](Stage& L, int st) {
#pragma unroll
    for (int e = 0; e < APT; ++e) {
      const int lin = NP % 256 == 0 ? tid + 256 * e : min(tid + 256 * e, NP - 1);
      L.a[e] = Aop[(size_t)(lin >> 3) * rowq + 8 * st + (lin & 7)];
    }
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      L.xh[u] = xc[u][8 * st + 2 * g];
      L.xl[u] = xc[u][8 * st + 2 * g + 1];
    }
  };
  auto stash = [&](const Stage& L, int buf) {
#pragma unroll
    for (int e = 0; e < APT; ++e) {
      const int lin = tid + 256 * e;
      if (NP % 256 == 0 || lin < NP) *(u32x4_t*)&As[buf * BM * RW + (lin >> 3) * RW + 4 * (lin & 7)] = L.a[e];
    }
#pragma unroll
    for (int u = 0; u < TN; ++u) {
      bh[u] = __builtin_bit_cast(half8_t, L.xh[u]);
      bl[u] = __builtin_bit_cast(half8_t, L.xl[u]);
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
      const int w = cur * BM * RW + (t * 16 + i16) * RW + 8 * g;
      ah[t] = *(const half8_t*)&As[w];
      al[t] = *(const half8_t*)&As[w + 4];
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
  // stages 0 .. PD-1 in flight, stage 0 staged; ring slot d holds the stages congruent to d mod PD
#pragma unroll
  for (int d = 0; d < PD; ++d) load(ring[d], s0 + min(d, my - 1));
  stash(ring[0], 0);
  __syncthreads();
  for (int i0 = 0; i0 < nmax; i0 += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int i = i0 + d;
      // slot d (stage i) was staged at the end of the previous stage; it now takes stage i + PD
      load(ring[d], s0 + min(i + PD, my - 1));
      __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of the products (else they sink below them)
      if (i < my) compute(i & 1);
      // buffer (i + 1) & 1 was last read in stage i - 1, which every wave has left (barrier below);
      // past the group's last stage this writes a copy nobody reads
      stash(ring[(d + 1) % PD], (i + 1) & 1);
      __syncthreads();
    }
  }
  if constexpr (KW > 1) {  // group partial tiles summed into group 0 in group order
    float4_t* red = (float4_t*)lds;
#pragma unroll 1
    for (int q = 1; q < KW; ++q) {
      if (kg == q) {
#pragma unroll
        for (int t = 0; t < TM; ++t)
#pragma unroll
          for (int u = 0; u < TN; ++u) red[(t * TN + u) * 256 + tid] = acc[t][u];
      }
      __syncthreads();
      if (kg == 0) {
#pragma unroll
        for (int t = 0; t < TM; ++t)
#pragma unroll
          for (int u = 0; u < TN; ++u) acc[t][u] += red[(t * TN + u) * 256 + tid];
      }
      __syncthreads();
    }
    if (kg != 0) return;
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

template <int TM, int TN>
static void launch_h3(const GemmJob& job, const uint16_t* A, const float* a_scale, GemmDims d, const uint16_t* X,
                      const float* x_scale, float* Y, int mode, hipStream_t s) {
  const dim3 grid(job.n_tiles, d.M / (16 * TM));
  hipLaunchKernelGGL((k_gemm_h3<TM, TN>), grid, dim3(256), 0, s, (const u32x4_t*)A, d, a_scale, job.tiles,
                     job.in_idx, job.out_idx, job.scale, (const u32x4_t*)X, x_scale, Y, mode);
}

template <int TM, int TN, int KW, int PD>
static void launch_h3k(const GemmJob& job, const uint16_t* A, const float* a_scale, GemmDims d, const uint16_t* X,
                       const float* x_scale, float* Y, int mode, hipStream_t s) {
  KFMM_REQUIRE(d.K / 32 >= KW, "gemm_h3: fewer k-stages than k groups");
  const dim3 grid(job.n_tiles, d.M / (16 * TM));
  hipLaunchKernelGGL((k_gemm_h3k<TM, TN, KW, PD>), grid, dim3(256 * KW), 0, s, (const u32x4_t*)A, d, a_scale,
                     job.tiles, job.in_idx, job.out_idx, job.scale, (const u32x4_t*)X, x_scale, Y, mode);
}

// Launches with fewer than 512 workgroups (two per compute unit) in 64-column tiles run the latency-hiding
// variant: measured on translation shapes, the upper levels of the M2M / L2L passes (8 operators,
// 896 x 896, 700 columns) take 12.7 instead of 19.3 us and the 480 x 896 U^T product (3000 columns)
// 14.9 instead of 17.5 us; with more workgroups the plain kernel is as fast or faster.
void gemm_h3(const GemmJob& job, const uint16_t* A, const float* a_scale, GemmDims d, const uint16_t* X,
             const float* x_scale, float* Y, int mode, hipStream_t s) {
  if (job.n_tiles == 0) return;
  KFMM_REQUIRE(job.cols_per_tile <= 2 * kGemmBN, "gemm_h3: at most 128 columns per tile");
  KFMM_REQUIRE(!job.ranked || job.cols_per_tile > kGemmBN, "gemm_h3: tiles with a rank need 128-column tiles");
  KFMM_REQUIRE(d.K % 32 == 0 && d.K >= 64 && d.ldx % 8 == 0 && d.ldx >= 2 * d.K, "gemm_h3: bad K or ldx");
  if (mode == kStore) KFMM_REQUIRE(d.ldy % 4 == 0, "gemm_h3: ldy must be a multiple of 4 for vector stores");
  KFMM_REQUIRE(d.M % 96 == 0 || d.M % 64 == 0, "gemm_h3: M must be a multiple of 96 or 64");
  const int64_t nt = job.n_tiles;
  if (job.cols_per_tile > kGemmBN) {
    // 128-column tiles (the M2L): the tallest row block that divides M, 160 rows at r = 480, 192 at r = 384
    // (standalone, 316 operators x 107,900 columns: 142 us against 144 with 128 and 157 with 96 rows)
    if (d.M % 160 == 0)
      launch_h3<10, 2>(job, A, a_scale, d, X, x_scale, Y, mode, s);
    else if (d.M % 192 == 0)
      launch_h3<12, 2>(job, A, a_scale, d, X, x_scale, Y, mode, s);
    else if (d.M % 128 == 0)
      launch_h3<8, 2>(job, A, a_scale, d, X, x_scale, Y, mode, s);
    else if (d.M % 96 == 0)
      launch_h3<6, 2>(job, A, a_scale, d, X, x_scale, Y, mode, s);
    else
      launch_h3<4, 2>(job, A, a_scale, d, X, x_scale, Y, mode, s);
  } else if (d.M % 96 == 0) {  // 64-column tiles
    if (nt * (d.M / 96) < 512)
      launch_h3k<6, 1, 2, 2>(job, A, a_scale, d, X, x_scale, Y, mode, s);
    else
      launch_h3<6, 1>(job, A, a_scale, d, X, x_scale, Y, mode, s);
  } else {
    if (nt * (d.M / 64) < 160)  // 32-row blocks: twice the workgroups (8 operators, 180 columns: 7.6 vs 9.5 us)
      launch_h3k<2, 1, 2, 2>(job, A, a_scale, d, X, x_scale, Y, mode, s);
    else if (nt * (d.M / 64) < 512)
      launch_h3k<4, 1, 2, 2>(job, A, a_scale, d, X, x_scale, Y, mode, s);
    else
      launch_h3<4, 1>(job, A, a_scale, d, X, x_scale, Y, mode, s);
  }
  KFMM_HIP(hipGetLastError());
}

}  // namespace kfmm
