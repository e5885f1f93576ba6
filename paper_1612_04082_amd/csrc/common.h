// Shared internals of the kfmm library: error reporting, HIP checks, and the Kelvin kernel
// evaluators used by every far- and near-field kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace kfmm {

// Exception carrying a kfmm status code; caught at the C-ABI boundary.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define KFMM_HIP(call)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      throw ::kfmm::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_) + " at " +       \
                                  __FILE__ + ":" + std::to_string(__LINE__));                   \
  } while (0)

#define KFMM_REQUIRE(cond, msg)                                 \
  do {                                                          \
    if (!(cond)) throw ::kfmm::Error(-1, std::string(msg));     \
  } while (0)

constexpr double kPi = 3.14159265358979323846;

// Message of the withdrawn BF16 M2L precision (precision value 2).
constexpr const char* kBf16Withdrawn =
    "KFMM_FP32_M2L_BF16 is withdrawn (BF16 M2L measured ~1e-2 relative error, above its 1e-3 target); "
    "KFMM_FP32_M2L_SPLIT16 runs the M2L on the FP16 matrix cores at FP32 accuracy";

// Elastic constants derived from (K, G) (Sec. 2, eq. elast): nu and the kernel prefactors.
struct Elastic {
  double K, G, nu;
  double cU;   // 1 / (16 pi (1-nu) G)            eq. disp_1
  double cP;   // 1 / (8 pi (1-nu))               eq. disp_2 (with the textbook leading minus)
  double cD;   // 1 / (8 pi (1-nu))               eq. stress_2 (8 pi denominator)
  double cS;   // G / (4 pi (1-nu))               eq. stress_3 (times G)
  static Elastic make(double K, double G) {
    Elastic e;
    e.K = K;
    e.G = G;
    e.nu = (3.0 * K - 2.0 * G) / (2.0 * (3.0 * K + G));
    e.cU = 1.0 / (16.0 * kPi * (1.0 - e.nu) * G);
    e.cP = 1.0 / (8.0 * kPi * (1.0 - e.nu));
    e.cD = 1.0 / (8.0 * kPi * (1.0 - e.nu));
    e.cS = G / (4.0 * kPi * (1.0 - e.nu));
    return e;
  }
};

// Constants in the arithmetic type of a kernel.
template <typename T>
struct KConst {
  T nu, a34, a12, a14, cU, cP, cD, cS;  // a34 = 3-4nu, a12 = 1-2nu, a14 = 1-4nu
  __host__ __device__ KConst() {}
  explicit KConst(const Elastic& e)
      : nu((T)e.nu), a34((T)(3.0 - 4.0 * e.nu)), a12((T)(1.0 - 2.0 * e.nu)), a14((T)(1.0 - 4.0 * e.nu)),
        cU((T)e.cU), cP((T)e.cP), cD((T)e.cD), cS((T)e.cS) {}
};

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return __frsqrt_rn(x); }
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

// 1/r, or 0 for a coincident pair (r2 = 0): every term of the pair kernels below carries a factor 1/r, so a
// coincident pair then adds exact zeros and a loop over pairs needs no branch.
template <typename T>
__device__ __forceinline__ T rsqrt_or_zero(T r2) {
  const T ir = rsqrt_t<T>(r2);
  return r2 > T(0) ? ir : T(0);
}

// Displacement at a target from one source (d = source - target, r2 = |d|^2 > 0):
//   v += U(d) wa + P(d, n) wb           (eq. disp_1, eq. disp_2 read with the leading minus)
// The prefactors cU, cP are applied by the caller after the sum (they are common to all pairs).
// vU accumulates the bracket of U, vP the bracket of P.  Used for S2M: the upward check potentials carry
// the far field of every source, and at targets many box sizes away that field is a small remainder of
// cancelling contributions, so their rounding matters there (with the one-accumulator form below, on
// prefactor-scaled densities, targets 40 radii from a sphere of sources went from 5.0e-6 to 1.3e-5).
template <typename T, bool SL, bool DL>
__device__ __forceinline__ void disp_pair(T dx, T dy, T dz, T r2, const T* wa, const T* wb, T nx, T ny, T nz,
                                          const KConst<T>& k, T* vU, T* vP) {
  T ir = rsqrt_t<T>(r2);
  T ir2 = ir * ir;
  if (SL) {
    // U wa * 16pi(1-nu)G = (3-4nu) wa / r + d (d.wa) / r^3
    T dwa = dx * wa[0] + dy * wa[1] + dz * wa[2];
    T s = dwa * ir2 * ir;
    vU[0] += k.a34 * wa[0] * ir + dx * s;
    vU[1] += k.a34 * wa[1] * ir + dy * s;
    vU[2] += k.a34 * wa[2] * ir + dz * s;
  }
  if (DL) {
    // -P wb * 8pi(1-nu) = (d.n)/r^3 [(1-2nu) wb + 3 d (d.wb)/r^2] - (1-2nu) [d (n.wb) - n (d.wb)] / r^3
    T dwb = dx * wb[0] + dy * wb[1] + dz * wb[2];
    T nwb = nx * wb[0] + ny * wb[1] + nz * wb[2];
    T dn = dx * nx + dy * ny + dz * nz;
    T ir3 = ir2 * ir;
    T f = dn * ir3;
    T g = T(3) * f * dwb * ir2;
    T h = k.a12 * ir3;
    vP[0] += f * k.a12 * wb[0] + g * dx - h * (dx * nwb - nx * dwb);
    vP[1] += f * k.a12 * wb[1] + g * dy - h * (dy * nwb - ny * dwb);
    vP[2] += f * k.a12 * wb[2] + g * dz - h * (dz * nwb - nz * dwb);
  }
}

// Displacement at a target from one source (d = source - target, r2 = |d|^2 > 0), the kernel prefactors
// folded into the densities (wa' = cU wa, wb' = cP wb, nwb = n . wb'), one accumulator:
//   v += cU U(d) wa + P(d, n) wb   (eq. disp_1, eq. disp_2 read with the leading minus)
//   16 pi (1-nu) G U(d) wa = (3-4nu) wa / r + d (d.wa) / r^3
//   -8 pi (1-nu) P(d, n) wb = (d.n)/r^3 [(1-2nu) wb + 3 d (d.wb)/r^2] - (1-2nu) [d (n.wb) - n (d.wb)] / r^3
// expanded as v_i += t wa'_i + sc d_i - fp wb'_i - c2 n_i with t = (3-4nu)/r, fp = (1-2nu)(d.n)/r^3,
// sc = (d.wa')/r^3 - 3 (d.n)(d.wb')/r^5 + (1-2nu)(n.wb')/r^3, c2 = (1-2nu)(d.wb')/r^3 (about 44 operations per
// pair; separate U and P accumulators with the prefactors applied at the end take about 51).
// With ir = 1/r given (0 for a coincident pair: no contribution).
template <typename T, bool SL, bool DL>
__device__ __forceinline__ void disp_pair_f_ir(T dx, T dy, T dz, T ir, const T* wa, const T* wb, T nwb, T nx, T ny,
                                               T nz, const KConst<T>& k, T* v) {
  const T ir2 = ir * ir, ir3 = ir2 * ir;
  T sc = T(0), t = T(0), fp = T(0), c2 = T(0);
  if (SL) {
    const T dwa = dx * wa[0] + dy * wa[1] + dz * wa[2];
    sc = dwa * ir3;
    t = k.a34 * ir;
  }
  if (DL) {
    const T dwb = dx * wb[0] + dy * wb[1] + dz * wb[2];
    const T dn = dx * nx + dy * ny + dz * nz;
    const T f = dn * ir3;
    const T h = k.a12 * ir3;
    fp = k.a12 * f;
    sc += h * nwb - T(3) * f * dwb * ir2;
    c2 = h * dwb;
  }
  const T d[3] = {dx, dy, dz}, n[3] = {nx, ny, nz};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T acc = v[i] + sc * d[i];
    if (SL) acc += t * wa[i];
    if (DL) acc -= fp * wb[i] + c2 * n[i];
    v[i] = acc;
  }
}
template <typename T, bool SL, bool DL>
__device__ __forceinline__ void disp_pair_f(T dx, T dy, T dz, T r2, const T* wa, const T* wb, T nwb, T nx, T ny,
                                            T nz, const KConst<T>& k, T* v) {
  disp_pair_f_ir<T, SL, DL>(dx, dy, dz, rsqrt_t<T>(r2), wa, wb, nwb, nx, ny, nz, k, v);
}

// Stress at a target from one source:  s_ij += D_kij wa_k + S_kij wb_k   (eq. stress_2 with 8 pi,
// eq. stress_3 times G).  sD and sS accumulate the brackets (prefactors cD and cS applied later).
// Components xx, yy, zz, yz, xz, xy.
template <typename T, bool SL, bool DL>
__device__ __forceinline__ void stress_pair(T dx, T dy, T dz, T r2, const T* wa, const T* wb, T nx, T ny, T nz,
                                            const KConst<T>& k, T* sD, T* sS) {
  T ir = rsqrt_t<T>(r2);
  T rx = dx * ir, ry = dy * ir, rz = dz * ir;
  T ir2 = ir * ir;
  if (SL) {
    // D:a * 8pi(1-nu) r^2 = (1-2nu)(a_i r_j + a_j r_i - delta_ij r.a) + 3 r_i r_j (r.a)
    T ra = rx * wa[0] + ry * wa[1] + rz * wa[2];
    T t3 = T(3) * ra;
    T c = ir2;
    sD[0] += c * (k.a12 * (T(2) * wa[0] * rx - ra) + t3 * rx * rx);
    sD[1] += c * (k.a12 * (T(2) * wa[1] * ry - ra) + t3 * ry * ry);
    sD[2] += c * (k.a12 * (T(2) * wa[2] * rz - ra) + t3 * rz * rz);
    sD[3] += c * (k.a12 * (wa[1] * rz + wa[2] * ry) + t3 * ry * rz);
    sD[4] += c * (k.a12 * (wa[0] * rz + wa[2] * rx) + t3 * rx * rz);
    sD[5] += c * (k.a12 * (wa[0] * ry + wa[1] * rx) + t3 * rx * ry);
  }
  if (DL) {
    // S:b * 4pi(1-nu) r^3 / G =
    //   3 (r.n) [(1-2nu) delta_ij (r.b) + nu (b_i r_j + b_j r_i) - 5 r_i r_j (r.b)]
    //   + 3 nu (n_i r_j + n_j r_i)(r.b) + (1-2nu)(3 (n.b) r_i r_j + n_j b_i + n_i b_j) - (1-4nu)(n.b) delta_ij
    T rb = rx * wb[0] + ry * wb[1] + rz * wb[2];
    T nb = nx * wb[0] + ny * wb[1] + nz * wb[2];
    T rn = rx * nx + ry * ny + rz * nz;
    T c = ir2 * ir;
    T A = T(3) * rn;
    T diag = A * k.a12 * rb - k.a14 * nb;      // coefficient of delta_ij
    T rr = -T(15) * rn * rb + T(3) * k.a12 * nb;  // coefficient of r_i r_j
    T br = A * k.nu;                           // coefficient of (b_i r_j + b_j r_i)
    T nr = T(3) * k.nu * rb;                   // coefficient of (n_i r_j + n_j r_i)
    T nbij = k.a12;                            // coefficient of (n_j b_i + n_i b_j)
    sS[0] += c * (diag + rr * rx * rx + T(2) * (br * wb[0] * rx + nr * nx * rx + nbij * nx * wb[0]));
    sS[1] += c * (diag + rr * ry * ry + T(2) * (br * wb[1] * ry + nr * ny * ry + nbij * ny * wb[1]));
    sS[2] += c * (diag + rr * rz * rz + T(2) * (br * wb[2] * rz + nr * nz * rz + nbij * nz * wb[2]));
    sS[3] += c * (rr * ry * rz + br * (wb[1] * rz + wb[2] * ry) + nr * (ny * rz + nz * ry) + nbij * (nz * wb[1] + ny * wb[2]));
    sS[4] += c * (rr * rx * rz + br * (wb[0] * rz + wb[2] * rx) + nr * (nx * rz + nz * rx) + nbij * (nz * wb[0] + nx * wb[2]));
    sS[5] += c * (rr * rx * ry + br * (wb[0] * ry + wb[1] * rx) + nr * (nx * ry + ny * rx) + nbij * (ny * wb[0] + nx * wb[1]));
  }
}

// Number of points of the cube-surface grid with p points per edge.
inline int surface_count(int p) { return 6 * (p - 1) * (p - 1) + 2; }

// Round v up to a multiple of m.
inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace kfmm
