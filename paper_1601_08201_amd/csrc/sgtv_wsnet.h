// Internal interface of the warm-start network kernels (64 channels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace sgtv {
namespace wsn {

size_t conv_lds_bytes(int W);

// out = relu(conv(X) + bias); xt (or nullptr): out channel-major in three shifted
// copies (3*B*H*W*C bf16), ready for the next layer's conv_wgrad
hipError_t conv_relu(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H, int W,
                     __bf16 *out, __bf16 *xt, hipStream_t st);
// z = conv(X) + bias (FP32); sp (or nullptr): softplus(z)
hipError_t conv_softplus(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H,
                         int W, float *z, float *sp, hipStream_t st);
// out = conv(X) masked by mask > 0; dt (or nullptr): the same values channel-major
// per image row ([row][channel][x], B*H*W*C bf16), ready for conv_wgrad
hipError_t conv_masked(const __bf16 *X, const __bf16 *Wk, int B, int H, int W, const __bf16 *mask,
                       __bf16 *out, __bf16 *dt, hipStream_t st);
// image rows per weight-gradient block (divides H; H even)
int wgrad_rows(int H);
// weight and bias gradient of one layer into grad (C*9*C weights, then C biases);
// xt: 3*B*H*W*C bf16, dt: B*H*W*C bf16, wpart: (B*H / wgrad_rows(H)) * (C*9*C + C)
// floats (all scratch); xt_ready / dt_ready: xt already holds X's shifted copies
// (conv_relu wrote them) / dt already holds DZ channel-major (conv_masked wrote it)
hipError_t conv_wgrad(const __bf16 *X, const __bf16 *DZ, int B, int H, float *xt, float *dt,
                      float *wpart, float *grad, bool xt_ready, bool dt_ready, hipStream_t st);
hipError_t to_bf16(const float *x, __bf16 *y, int64_t n, hipStream_t st);
// per-image FP64 partial sums (n_blocks per image, image-major)
hipError_t image_partials(const float *x, int64_t img, int n_images, int n_blocks, double *partials,
                          hipStream_t st);
// y = bf16(x / m_b), m_b = sums[b] / img (1 where not positive), b = i / img
hipError_t scale_to_bf16(const float *x, const double *sums, int64_t img, int64_t n, __bf16 *y,
                         hipStream_t st);
// x0 = c_out * s * (ratio ? f : m_b), raised to at least floor * c_out * m_b when floor > 0
hipError_t start_image(const float *f, const float *s, const double *sums, int64_t img, int64_t n,
                       float c_out, int ratio, float floor, float *x0, hipStream_t st);
// dz = bf16(2 (softplus(z) - target) / n * sigmoid(z)), FP64 squared-error partials
hipError_t mse_grad(const float *target, const float *z, int64_t n, __bf16 *dz, double *partials,
                    int n_blocks, hipStream_t st);
// acc[0] += l[0] / cnt, acc[1] += 1 (FP64, one thread)
hipError_t loss_accumulate(const double *l, double cnt, double *acc, hipStream_t st);
hipError_t adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                float b2, float omb1, float omb2, float eps, float c1, float c2, hipStream_t st);
hipError_t weights_bf16(const float *w, __bf16 *wf, __bf16 *wb, hipStream_t st);

}  // namespace wsn
}  // namespace sgtv
