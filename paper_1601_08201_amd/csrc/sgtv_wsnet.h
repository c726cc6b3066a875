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
hipError_t mse_grad(const float *out, const float *target, const float *z, int64_t n, __bf16 *dz,
                    double *partials, int n_blocks, hipStream_t st);
hipError_t adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t st);
hipError_t weights_bf16(const float *w, __bf16 *wf, __bf16 *wb, hipStream_t st);

}  // namespace wsn
}  // namespace sgtv
