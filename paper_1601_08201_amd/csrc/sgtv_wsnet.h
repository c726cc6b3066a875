// Internal interface of the warm-start network kernels (64 channels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace sgtv {
namespace wsn {

size_t conv_lds_bytes(int W);
size_t wgrad_lds_bytes();

hipError_t conv_relu(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H, int W,
                     __bf16 *out, hipStream_t st);
hipError_t conv_softplus(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H,
                         int W, float *z, float *sp, hipStream_t st);
hipError_t conv_masked(const __bf16 *X, const __bf16 *Wk, int B, int H, int W, const __bf16 *mask,
                       __bf16 *out, hipStream_t st);
hipError_t conv_wgrad(const __bf16 *X, const __bf16 *DZ, int B, int H, int W, int rows_per_block,
                      float *part, float *grad, hipStream_t st);
hipError_t to_bf16(const float *x, __bf16 *y, int64_t n, hipStream_t st);
// per-image FP64 partial sums (n_blocks per image, image-major)
hipError_t image_partials(const float *x, int64_t img, int n_images, int n_blocks, double *partials,
                          hipStream_t st);
// y = bf16(x / m_b), m_b = sums[b] / img (1 where not positive), b = i / img
hipError_t scale_to_bf16(const float *x, const double *sums, int64_t img, int64_t n, __bf16 *y,
                         hipStream_t st);
// x0 = c_out * s * (ratio ? f : m_b)
hipError_t start_image(const float *f, const float *s, const double *sums, int64_t img, int64_t n,
                       float c_out, int ratio, float *x0, hipStream_t st);
hipError_t mse_grad(const float *out, const float *target, const float *z, int64_t n, __bf16 *dz,
                    double *partials, int n_blocks, hipStream_t st);
hipError_t adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t st);
hipError_t weights_bf16(const float *w, __bf16 *wf, __bf16 *wb, hipStream_t st);

}  // namespace wsn
}  // namespace sgtv
