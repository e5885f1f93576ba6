// Learned GMRES warm start: a point-wise MLP that maps features of each new boundary element to a
// correction of the previous iteration's solution mapped onto the new surface.  The paper proposes to
// reuse the previous solution when the boundary changes little (Sec. 5, fast update of the boundary
// solution); here the update is learned online from the iterations the optimisation itself produces.
//
// Network: h1 = silu(X W1 + b1), h2 = silu(h1 W2 + b2), y = h2 W3 + b3 (W stored [in][out], row-major).
// Training: FP32 forward / backward, loss mean((y - r)^2) with r = (x_target - x_mapped) / scale,
// Adam with bias correction.  Inference: layer 2 on the matrix cores in BF16 (FP32 accumulation),
// layers 1 and 3 in FP32.  Features (16 per element): offset to the matched previous centroid / l (3),
// its length (1), unit normal (3), boundary-condition type per component (3), mapped previous unknown /
// scale (3), centroid in the bounding box mapped to [-1, 1] (3).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/kfmm.h"
#include "common.h"
#include "learn.h"
#include "tree.h"

namespace kfmm {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

static unsigned nb(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }

// ---------------------------------------------------------------------------------------- dense layers

// Z = X W + b  (X: n x k, W: k x m), H = act(Z).  Block: 16 rows x m columns, one thread per column.
template <bool ACT>
__global__ void k_dense_fwd(const float* __restrict__ X, int64_t n, int k, const float* __restrict__ W,
                            const float* __restrict__ b, int m, float* __restrict__ Z, float* __restrict__ H) {
  constexpr int R = 16;
  __shared__ float xs[R][129];
  const int64_t r0 = (int64_t)blockIdx.x * R;
  for (int i = threadIdx.x; i < R * k; i += blockDim.x) {
    int r = i / k, c = i % k;
    xs[r][c] = r0 + r < n ? X[(r0 + r) * k + c] : 0.f;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < m; c += blockDim.x) {
    float acc[R];
    for (int r = 0; r < R; ++r) acc[r] = b[c];
    for (int kk = 0; kk < k; ++kk) {
      float w = W[kk * m + c];
      for (int r = 0; r < R; ++r) acc[r] += xs[r][kk] * w;
    }
    for (int r = 0; r < R; ++r) {
      if (r0 + r >= n) break;
      if (Z) Z[(r0 + r) * m + c] = acc[r];
      if (H) H[(r0 + r) * m + c] = ACT ? acc[r] * sigm(acc[r]) : acc[r];
    }
  }
}

// dX = (dZ W^T) * silu'(Zprev)   (dZ: n x m, W: k x m -> dX: n x k).  Zprev may be null (no activation).
__global__ void k_dense_bwd(const float* __restrict__ dZ, int64_t n, int m, const float* __restrict__ W, int k,
                            const float* __restrict__ Zprev, float* __restrict__ dX) {
  constexpr int R = 16;
  __shared__ float ds[R][129];
  const int64_t r0 = (int64_t)blockIdx.x * R;
  for (int i = threadIdx.x; i < R * m; i += blockDim.x) {
    int r = i / m, c = i % m;
    ds[r][c] = r0 + r < n ? dZ[(r0 + r) * m + c] : 0.f;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    float acc[R];
    for (int r = 0; r < R; ++r) acc[r] = 0.f;
    for (int j = 0; j < m; ++j) {
      float w = W[c * m + j];
      for (int r = 0; r < R; ++r) acc[r] += ds[r][j] * w;
    }
    for (int r = 0; r < R; ++r) {
      int64_t row = r0 + r;
      if (row >= n) break;
      float g = acc[r];
      if (Zprev) {
        float z = Zprev[row * k + c], s = sigm(z);
        g *= s * (1.f + z * (1.f - s));
      }
      dX[row * k + c] = g;
    }
  }
}

constexpr int kGradChunks = 128;

// Partial gradients of one dense layer over a chunk of rows, packed as [chunk][k*m weights, m biases]
// (the parameter vector stores each layer's W and b adjacently, so the packed sum lands in place):
//   dW[i][j] = sum_r A[r][i] dZ[r][j],  db[j] = sum_r dZ[r][j].
__global__ void k_weight_grad(const float* __restrict__ A, const float* __restrict__ dZ, int64_t n, int k, int m,
                              float* __restrict__ part) {
  const int chunk = blockIdx.x;
  const int64_t per = (n + kGradChunks - 1) / kGradChunks;
  const int64_t b = chunk * per, e = min(n, b + per);
  const int len = k * m + m;
  for (int idx = threadIdx.x; idx < len; idx += blockDim.x) {
    float acc = 0.f;
    if (idx < k * m) {
      int i = idx / m, j = idx % m;
      for (int64_t r = b; r < e; ++r) acc += A[r * k + i] * dZ[r * m + j];
    } else {
      int j = idx - k * m;
      for (int64_t r = b; r < e; ++r) acc += dZ[r * m + j];
    }
    part[(size_t)chunk * len + idx] = acc;
  }
}

// sum the chunk partials in a fixed order
__global__ void k_sum_chunks(const float* __restrict__ p, int len, float* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int c = 0; c < kGradChunks; ++c) s += p[(size_t)c * len + i];
  out[i] = s;
}

// dY = 2 (Y - R) / (3n); per-block loss partials
__global__ void k_loss(const float* __restrict__ Y, const float* __restrict__ Rt, int64_t n3, float* __restrict__ dY,
                       float* __restrict__ lpart) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
    float d = Y[i] - Rt[i];
    dY[i] = 2.f * d / (float)n3;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ void k_adam(int64_t np, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  float gi = g[i];
  float a = b1 * m1[i] + (1.f - b1) * gi;
  float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// r = (x_target - x_mapped) / scale (FP32)
__global__ void k_residual_target(int64_t n3, const double* __restrict__ xt, const double* __restrict__ xm,
                                  double inv_scale, float* __restrict__ r) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) r[i] = (float)((xt[i] - xm[i]) * inv_scale);
}

// ------------------------------------------------------------------------------- BF16 inference

// Fused inference for 64 rows per workgroup (4 waves x 16 rows): layer 1 FP32 into LDS as BF16, layer 2
// on the matrix cores (v_mfma_f32_16x16x32_bf16, W2 in LDS as BF16, [out][in]), SiLU, layer 3 FP32,
// x0 = x_mapped + scale * y.
__global__ __launch_bounds__(256) void k_infer_bf16(const float* __restrict__ X, int64_t n, int din,
                                                    const float* __restrict__ P, const __hip_bfloat16* __restrict__ W2t,
                                                    const double* __restrict__ xm, double scale,
                                                    double* __restrict__ x0, int width) {
  constexpr int WD = 128;  // width (checked on the host)
  __shared__ __attribute__((aligned(16))) __bf16 w2s[WD][WD + 8];  // [out][in]
  __shared__ __attribute__((aligned(16))) __bf16 h1s[64][WD + 8];
  __shared__ float h2s[64][WD + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const float* W1 = P;
  const float* b1 = W1 + din * WD;
  const float* b2 = b1 + WD + WD * WD;
  const float* W3 = b2 + WD;
  const float* b3 = W3 + WD * 3;
  for (int i = tid; i < WD * WD / 8; i += 256) {
    int o = i / (WD / 8), q = i % (WD / 8);
    *(uint4*)&w2s[o][8 * q] = *(const uint4*)(W2t + (size_t)o * WD + 8 * q);
  }
  // layer 1: thread -> (row r = tid / 4, 32 columns)
  {
    int r = tid >> 2, cb = (tid & 3) * 32;
    int64_t row = r0 + r;
    float xr[32];
    for (int kk = 0; kk < din && kk < 32; ++kk) xr[kk] = row < n ? X[row * din + kk] : 0.f;
    for (int c = 0; c < 32; ++c) {
      float acc = b1[cb + c];
      for (int kk = 0; kk < din && kk < 32; ++kk) acc += xr[kk] * W1[kk * WD + cb + c];
      h1s[r][cb + c] = (__bf16)(acc * sigm(acc));
    }
  }
  __syncthreads();
  // layer 2: wave handles rows wave*16 .. +15, all 128 output columns (8 tiles), K = 128 (4 steps of 32)
  float4_t acc[8];
  for (int t = 0; t < 8; ++t) acc[t] = float4_t{0, 0, 0, 0};
  for (int ks = 0; ks < WD / 32; ++ks) {
    bf16x8_t a = *(const bf16x8_t*)&h1s[wave * 16 + (lane & 15)][32 * ks + 8 * (lane >> 4)];
    for (int t = 0; t < 8; ++t) {
      bf16x8_t b = *(const bf16x8_t*)&w2s[t * 16 + (lane & 15)][32 * ks + 8 * (lane >> 4)];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
  for (int t = 0; t < 8; ++t)
    for (int v = 0; v < 4; ++v) {
      int rr = wave * 16 + 4 * (lane >> 4) + v, cc = t * 16 + (lane & 15);
      float z = acc[t][v] + b2[cc];
      h2s[rr][cc] = z * sigm(z);
    }
  __syncthreads();
  // layer 3 + output: thread -> (row, component)
  if (tid < 64 * 3) {
    int r = tid / 3, c = tid % 3;
    int64_t row = r0 + r;
    if (row < n) {
      float y = b3[c];
      for (int kk = 0; kk < WD; ++kk) y += h2s[r][kk] * W3[kk * 3 + c];
      x0[row * 3 + c] = xm[row * 3 + c] + scale * (double)y;
    }
  }
}

__global__ void k_w2_to_bf16t(const float* __restrict__ W2, int wd, __hip_bfloat16* __restrict__ W2t) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= wd * wd) return;
  int in = i / wd, out = i % wd;
  W2t[(size_t)out * wd + in] = __float2bfloat16(W2[i]);
}

// ------------------------------------------------------------------------------------ features

constexpr int kGridBits = 21;

__device__ __forceinline__ uint64_t cell_key(int x, int y, int z) {
  return ((uint64_t)(uint32_t)x << 42) | ((uint64_t)(uint32_t)y << 21) | (uint64_t)(uint32_t)z;
}

__global__ void k_centroids(int64_t T, const double* __restrict__ tri, double* __restrict__ cen,
                            double* __restrict__ nrm, double* __restrict__ elen) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  double v[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) v[a][d] = tri[9 * k + 3 * a + d];
  double e1[3], e2[3], l = 0;
  for (int d = 0; d < 3; ++d) {
    cen[3 * k + d] = (v[0][d] + v[1][d] + v[2][d]) / 3.0;
    e1[d] = v[1][d] - v[0][d];
    e2[d] = v[2][d] - v[0][d];
  }
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int d = 0; d < 3; ++d) nrm[3 * k + d] = n[d] / nn;
  for (int a = 0; a < 3; ++a) {
    double s = 0;
    for (int d = 0; d < 3; ++d) {
      double t = v[(a + 1) % 3][d] - v[a][d];
      s += t * t;
    }
    l += sqrt(s);
  }
  elen[k] = l / 3.0;
}

__global__ void k_cell_keys(int64_t T, const double* __restrict__ cen, const double* __restrict__ lo, double cell,
                            uint64_t* __restrict__ key, int* __restrict__ idx) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  int q[3];
  for (int d = 0; d < 3; ++d) q[d] = (int)floor((cen[3 * k + d] - lo[d]) / cell) + 1;
  key[k] = cell_key(q[0], q[1], q[2]);
  idx[k] = (int)k;
}

__device__ __forceinline__ int64_t lb_u64(const uint64_t* a, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Nearest previous centroid (search the 27 grid cells around the new centroid), the mapped previous
// solution in the new unknown layout, and the feature vector.
__global__ void k_features(int64_t Tn, const double* __restrict__ cen_n, const double* __restrict__ nrm_n,
                           const int8_t* __restrict__ bc_n, int64_t Tp, const double* __restrict__ cen_p,
                           const uint64_t* __restrict__ keys_p, const int* __restrict__ idx_p,
                           const double* __restrict__ u_p, const double* __restrict__ t_p,
                           const double* __restrict__ lo, const double* __restrict__ hi, double cell, double elen,
                           double* __restrict__ xm, double* __restrict__ dist, int* __restrict__ match,
                           float* __restrict__ feat) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Tn) return;
  double c[3] = {cen_n[3 * k], cen_n[3 * k + 1], cen_n[3 * k + 2]};
  int q[3];
  for (int d = 0; d < 3; ++d) q[d] = (int)floor((c[d] - lo[d]) / cell) + 1;
  double best = INFINITY;
  int bi = -1;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        uint64_t key = cell_key(q[0] + dx, q[1] + dy, q[2] + dz);
        for (int64_t p = lb_u64(keys_p, Tp, key); p < Tp && keys_p[p] == key; ++p) {
          int j = idx_p[p];
          double d2 = 0;
          for (int d = 0; d < 3; ++d) {
            double t = cen_p[3 * j + d] - c[d];
            d2 += t * t;
          }
          // tie-break on the lower index for determinism
          if (d2 < best || (d2 == best && j < bi)) {
            best = d2;
            bi = j;
          }
        }
      }
  match[k] = bi;
  double off[3] = {0, 0, 0};
  double xmv[3] = {0, 0, 0};
  if (bi >= 0) {
    for (int d = 0; d < 3; ++d) {
      off[d] = (c[d] - cen_p[3 * bi + d]) / elen;
      // unknown of the new element: u where the traction is prescribed, t where u is prescribed
      xmv[d] = bc_n[3 * k + d] == 0 ? t_p[3 * bi + d] : u_p[3 * bi + d];
    }
  }
  dist[k] = bi >= 0 ? sqrt(best) / elen : 1e30;
  for (int d = 0; d < 3; ++d) xm[3 * k + d] = xmv[d];
  float* f = feat + (size_t)k * kWsDin;
  for (int d = 0; d < 3; ++d) f[d] = (float)off[d];
  f[3] = bi >= 0 ? (float)(sqrt(best) / elen) : 10.f;
  for (int d = 0; d < 3; ++d) f[4 + d] = (float)nrm_n[3 * k + d];
  for (int d = 0; d < 3; ++d) f[7 + d] = (float)bc_n[3 * k + d];
  for (int d = 0; d < 3; ++d) f[13 + d] = (float)(2.0 * (c[d] - lo[d]) / fmax(hi[d] - lo[d], 1e-30) - 1.0);
}

__global__ void k_feat_scale(int64_t Tn, const double* __restrict__ xm, double inv_scale, float* __restrict__ feat) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Tn) return;
  for (int d = 0; d < 3; ++d) feat[(size_t)k * kWsDin + 10 + d] = (float)(xm[3 * k + d] * inv_scale);
}

__global__ void k_sumsq(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i] * x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void k_minmax_mean(const double* __restrict__ c, const double* __restrict__ el, int64_t T,
                              double* __restrict__ out /* lo[3], hi[3], mean edge, max edge */) {
  __shared__ double smin[3][256], smax[3][256], ssum[256], semx[256];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY}, s = 0, emx = 0;
  for (int64_t k = threadIdx.x; k < T; k += blockDim.x) {
    for (int d = 0; d < 3; ++d) {
      mn[d] = fmin(mn[d], c[3 * k + d]);
      mx[d] = fmax(mx[d], c[3 * k + d]);
    }
    s += el[k];
    emx = fmax(emx, el[k]);
  }
  for (int d = 0; d < 3; ++d) {
    smin[d][threadIdx.x] = mn[d];
    smax[d][threadIdx.x] = mx[d];
  }
  ssum[threadIdx.x] = s;
  semx[threadIdx.x] = emx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      for (int d = 0; d < 3; ++d) {
        smin[d][threadIdx.x] = fmin(smin[d][threadIdx.x], smin[d][threadIdx.x + st]);
        smax[d][threadIdx.x] = fmax(smax[d][threadIdx.x], smax[d][threadIdx.x + st]);
      }
      ssum[threadIdx.x] += ssum[threadIdx.x + st];
      semx[threadIdx.x] = fmax(semx[threadIdx.x], semx[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) {
      out[d] = smin[d][0];
      out[3 + d] = smax[d][0];
    }
    out[6] = ssum[0] / (double)T;
    out[7] = semx[0];
  }
}

// ----------------------------------------------------------------------------------------- net

WsNet::WsNet(int din_, int width_, uint64_t seed) : din(din_), width(width_) {
  KFMM_REQUIRE(din == kWsDin, "d_in must equal the feature count (16)");
  KFMM_REQUIRE(width == 128, "width must be 128");
  const int W = width;
  oW1 = 0;
  ob1 = oW1 + din * W;
  oW2 = ob1 + W;
  ob2 = oW2 + W * W;
  oW3 = ob2 + W;
  ob3 = oW3 + W * 3;
  np = ob3 + 3;
  params = arena.get<float>(np);
  grads = arena.get<float>(np);
  m1 = arena.get<float>(np);
  m2 = arena.get<float>(np);
  w2t = arena.get<__hip_bfloat16>((size_t)W * W);
  // counter-based initialisation: splitmix64 (Vigna) -> two uniforms -> Box-Muller normal
  std::vector<float> h(np, 0.f);
  auto splitmix = [](uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
  };
  auto normal = [&](uint64_t i) {
    double u1 = ((splitmix(seed * 0x100000001b3ull + 2 * i) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double u2 = ((splitmix(seed * 0x100000001b3ull + 2 * i + 1) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * kPi * u2);
  };
  for (int i = 0; i < din * W; ++i) h[oW1 + i] = (float)(normal(i) / std::sqrt((double)din));
  for (int i = 0; i < W * W; ++i) h[oW2 + i] = (float)(normal(100000 + i) / std::sqrt((double)W));
  // the last layer starts at zero: the untrained network predicts the mapped previous solution
  KFMM_HIP(hipMemcpy(params, h.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  KFMM_HIP(hipMemset(m1, 0, sizeof(float) * np));
  KFMM_HIP(hipMemset(m2, 0, sizeof(float) * np));
  step = 0;
}

// The buffers of WsWork for n rows, in one fixed order from `take`.
template <typename Take>
static WsWork carve_work(int64_t n, int W, Take&& take) {
  WsWork b;
  b.Z1 = take(n * W);
  b.H1 = take(n * W);
  b.Z2 = take(n * W);
  b.H2 = take(n * W);
  b.Y = take(n * 3);
  b.dY = take(n * 3);
  b.dA = take(n * W);
  b.dB = take(n * W);
  b.Rt = take(n * 3);
  b.pW = take((int64_t)kGradChunks * (W * W + W));
  b.lpart = take(1024);
  return b;
}

void WsNet::ensure(int64_t n) {
  if (n <= rows) return;
  work.release();
  rows = n;
  buf = carve_work(n, width, [&](int64_t cnt) { return work.get<float>((size_t)cnt); });
}

// ------------------------------------------------------------------------- allocation-free training

// Scratch memory of ws_train_noalloc, for callers that cannot allocate device memory: file-scope device
// data, one copy per GPU, held until the process ends.  In host code the array's name is not a device
// address; host code uses the address hipGetSymbolAddress returns for the current device.
constexpr size_t kWsScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) float scratch[kWsScratchBytes / sizeof(float)];

static constexpr int64_t align_floats(int64_t n) { return (n + 63) / 64 * 64; }  // 256-byte pieces

// floats that carve_work takes for n rows at width W, each piece rounded up to 256 bytes
static constexpr int64_t noalloc_floats(int64_t n, int W) {
  return 4 * align_floats(n * W) + 2 * align_floats(n * W) + 3 * align_floats(n * 3) +
         align_floats((int64_t)kGradChunks * (W * W + W)) + align_floats(1024);
}
static_assert(noalloc_floats(KFMM_WS_NOALLOC_MAX_ROWS, 128) * (int64_t)sizeof(float) <= (int64_t)kWsScratchBytes,
              "KFMM_WS_NOALLOC_MAX_ROWS rows of width 128 must fit the static scratch");

static float* scratch_address() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static float* addr[kMaxDevices] = {};
  int dev = 0;
  KFMM_HIP(hipGetDevice(&dev));
  KFMM_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    KFMM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    KFMM_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    addr[dev] = (float*)p;
  }
  return addr[dev];
}

WsWork ws_noalloc_work(const WsNet& net, int64_t n) {
  KFMM_REQUIRE(n > 0 && n <= KFMM_WS_NOALLOC_MAX_ROWS,
               "ws_train_noalloc: n must be in [1, KFMM_WS_NOALLOC_MAX_ROWS] (static scratch size)");
  KFMM_REQUIRE(noalloc_floats(n, net.width) * (int64_t)sizeof(float) <= (int64_t)kWsScratchBytes,
               "ws_train_noalloc: the network does not fit the static scratch");
  float* base = scratch_address();
  int64_t used = 0;
  return carve_work(n, net.width, [&](int64_t cnt) {
    float* p = base + used;
    used += align_floats(cnt);
    return p;
  });
}

// loss and gradients for features X and residual targets Rt (device, FP32), gradients into `grads`
float WsNet::loss_grad(const float* X, const float* R, int64_t n, hipStream_t s) {
  ensure(n);
  return loss_grad(X, R, n, buf, s);
}

float WsNet::loss_grad(const float* X, const float* R, int64_t n, const WsWork& b, hipStream_t s) {
  const int W = width;
  float* P = params;
  unsigned nr = nb(n, 16);
  hipLaunchKernelGGL(k_dense_fwd<true>, dim3(nr), dim3(128), 0, s, X, n, din, P + oW1, P + ob1, W, b.Z1, b.H1);
  hipLaunchKernelGGL(k_dense_fwd<true>, dim3(nr), dim3(128), 0, s, b.H1, n, W, P + oW2, P + ob2, W, b.Z2, b.H2);
  hipLaunchKernelGGL(k_dense_fwd<false>, dim3(nr), dim3(128), 0, s, b.H2, n, W, P + oW3, P + ob3, 3, (float*)nullptr,
                     b.Y);
  constexpr int lb = 256;
  hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, s, b.Y, R, n * 3, b.dY, b.lpart);
  auto wg = [&](const float* A, const float* dZ, int k, int m, int oW) {
    hipLaunchKernelGGL(k_weight_grad, dim3(kGradChunks), dim3(256), 0, s, A, dZ, n, k, m, b.pW);
    hipLaunchKernelGGL(k_sum_chunks, dim3(nb(k * m + m)), dim3(256), 0, s, b.pW, k * m + m, grads + oW);
  };
  wg(b.H2, b.dY, W, 3, oW3);
  hipLaunchKernelGGL(k_dense_bwd, dim3(nr), dim3(128), 0, s, b.dY, n, 3, P + oW3, W, b.Z2, b.dA);  // dZ2
  wg(b.H1, b.dA, W, W, oW2);
  hipLaunchKernelGGL(k_dense_bwd, dim3(nr), dim3(128), 0, s, b.dA, n, W, P + oW2, W, b.Z1, b.dB);  // dZ1
  wg(X, b.dB, din, W, oW1);
  KFMM_HIP(hipGetLastError());
  float lp[lb];
  KFMM_HIP(hipMemcpyAsync(lp, b.lpart, sizeof(float) * lb, hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  double L = 0;
  for (float v : lp) L += v;
  return (float)(L / (3.0 * n));
}

void WsNet::adam(float lr, hipStream_t s) {
  ++step;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nb(np)), dim3(256), 0, s, (int64_t)np, params, grads, m1, m2, lr, b1, b2, eps, c1,
                     c2);
  KFMM_HIP(hipGetLastError());
  bf_dirty = true;
}

void WsNet::predict(const float* X, int64_t n, const double* xm, double scale, double* x0, hipStream_t s) {
  if (n == 0) return;
  if (bf_dirty) {
    hipLaunchKernelGGL(k_w2_to_bf16t, dim3(nb((int64_t)width * width)), dim3(256), 0, s, params + oW2, width, w2t);
    bf_dirty = false;
  }
  hipLaunchKernelGGL(k_infer_bf16, dim3(nb(n, 64)), dim3(256), 0, s, X, n, din, params, w2t, xm, scale, x0, width);
  KFMM_HIP(hipGetLastError());
}

float WsNet::train(const float* X, const double* xm, const double* xt, int64_t n, double scale, int epochs, float lr,
                   hipStream_t s) {
  ensure(n);
  return train(X, xm, xt, n, scale, epochs, lr, buf, s);
}

float WsNet::train(const float* X, const double* xm, const double* xt, int64_t n, double scale, int epochs, float lr,
                   const WsWork& b, hipStream_t s) {
  hipLaunchKernelGGL(k_residual_target, dim3(nb(3 * n)), dim3(256), 0, s, 3 * n, xt, xm, 1.0 / scale, b.Rt);
  KFMM_HIP(hipGetLastError());
  float L = 0;
  for (int e = 0; e < epochs; ++e) {
    L = loss_grad(X, b.Rt, n, b, s);
    adam(lr, s);
  }
  return L;
}

// ------------------------------------------------------------------------------- features driver

double ws_make_features(const bem_problem& prev, const double* u_prev, const double* t_prev, const bem_problem& next,
                        float* feat, double* xm, hipStream_t s) {
  Arena a;
  const int64_t Tp = prev.n_tri, Tn = next.n_tri;
  double* cp = a.get<double>(3 * Tp);
  double* np_ = a.get<double>(3 * Tp);
  double* ep = a.get<double>(Tp);
  double* cn = a.get<double>(3 * Tn);
  double* nn = a.get<double>(3 * Tn);
  double* en = a.get<double>(Tn);
  hipLaunchKernelGGL(k_centroids, dim3(nb(Tp)), dim3(256), 0, s, Tp, prev.tri_xyz, cp, np_, ep);
  hipLaunchKernelGGL(k_centroids, dim3(nb(Tn)), dim3(256), 0, s, Tn, next.tri_xyz, cn, nn, en);
  double* mm = a.get<double>(8);
  double* mmn = a.get<double>(8);
  hipLaunchKernelGGL(k_minmax_mean, dim3(1), dim3(256), 0, s, cp, ep, Tp, mm);
  hipLaunchKernelGGL(k_minmax_mean, dim3(1), dim3(256), 0, s, cn, en, Tn, mmn);
  double hp[8], hn[8];
  KFMM_HIP(hipMemcpyAsync(hp, mm, sizeof(hp), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipMemcpyAsync(hn, mmn, sizeof(hn), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = std::min(hp[d], hn[d]);
    hi[d] = std::max(hp[3 + d], hn[3 + d]);
  }
  const double cell = 2.0 * std::max(hp[7], hn[7]);
  const double elen = hn[6];
  double* dlo = a.get<double>(6);
  double lohi[6] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
  KFMM_HIP(hipMemcpyAsync(dlo, lohi, sizeof(lohi), hipMemcpyHostToDevice, s));
  // sort previous centroids by grid cell
  int64_t npad = 2048;
  while (npad < Tp) npad <<= 1;
  uint64_t* keys = a.get<uint64_t>(npad);
  int* idx = a.get<int>(npad);
  hipLaunchKernelGGL(k_cell_keys, dim3(nb(Tp)), dim3(256), 0, s, Tp, cp, dlo, cell, keys, idx);
  sort_keys(keys, idx, Tp, npad, s);
  double* dist = a.get<double>(Tn);
  int* match = a.get<int>(Tn);
  hipLaunchKernelGGL(k_features, dim3(nb(Tn)), dim3(256), 0, s, Tn, cn, nn, next.bc_type, Tp, cp, keys, idx, u_prev,
                     t_prev, dlo, dlo + 3, cell, elen, xm, dist, match, feat);
  KFMM_HIP(hipGetLastError());
  double* ss = a.get<double>(1);
  hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(256), 0, s, xm, 3 * Tn, ss);
  double sumsq = 0;
  KFMM_HIP(hipMemcpyAsync(&sumsq, ss, sizeof(double), hipMemcpyDeviceToHost, s));
  KFMM_HIP(hipStreamSynchronize(s));
  double scale = std::sqrt(sumsq / (3.0 * Tn));
  if (!(scale > 0)) scale = 1.0;
  hipLaunchKernelGGL(k_feat_scale, dim3(nb(Tn)), dim3(256), 0, s, Tn, xm, 1.0 / scale, feat);
  KFMM_HIP(hipStreamSynchronize(s));
  return scale;
}

}  // namespace kfmm
