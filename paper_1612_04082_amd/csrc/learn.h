// Learned GMRES warm start (see learn.hip).
#pragma once
#include <hip/hip_bf16.h>

#include "../../include/kfmm.h"
#include "common.h"
#include "tree.h"

namespace kfmm {

constexpr int kWsDin = 16;  // features per element

// Work buffers of one training call over n rows (device, FP32): pre-activations and activations of the
// two hidden layers, output, output gradient, hidden-layer gradients, residual targets, per-chunk weight
// gradients and per-block loss partials.  Every word a call reads is written earlier in that call.
struct WsWork {
  float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Y = nullptr, *dY = nullptr, *dA = nullptr,
        *dB = nullptr, *Rt = nullptr, *pW = nullptr, *lpart = nullptr;
};

struct WsNet {
  int din, width;
  int oW1, ob1, oW2, ob2, oW3, ob3, np;  // offsets into the parameter vector
  Arena arena, work;
  float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
  __hip_bfloat16* w2t = nullptr;  // BF16 copy of W2, [out][in]
  bool bf_dirty = true;
  int64_t step = 0, rows = 0;
  WsWork buf;  // allocated by ensure() for the largest n seen so far

  WsNet(int din, int width, uint64_t seed);
  void ensure(int64_t n);
  // gradients into grads; the buffers are buf (grown by ensure) or the caller's
  float loss_grad(const float* X, const float* R, int64_t n, hipStream_t s);
  float loss_grad(const float* X, const float* R, int64_t n, const WsWork& b, hipStream_t s);
  void adam(float lr, hipStream_t s);
  void predict(const float* X, int64_t n, const double* xm, double scale, double* x0, hipStream_t s);
  float train(const float* X, const double* xm, const double* xt, int64_t n, double scale, int epochs, float lr,
              hipStream_t s);
  float train(const float* X, const double* xm, const double* xt, int64_t n, double scale, int epochs, float lr,
              const WsWork& b, hipStream_t s);
};

// Training buffers for n rows carved from the library's static device scratch (ws_train_noalloc): no
// allocation.  n must not exceed KFMM_WS_NOALLOC_MAX_ROWS.
WsWork ws_noalloc_work(const WsNet& net, int64_t n);

// Features of the elements of `next` from the previous surface and its solution; returns the scale.
double ws_make_features(const bem_problem& prev, const double* u_prev, const double* t_prev, const bem_problem& next,
                        float* feat, double* xm, hipStream_t s);

}  // namespace kfmm
