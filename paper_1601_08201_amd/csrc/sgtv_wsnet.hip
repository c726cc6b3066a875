// Kernels of the learned warm-start network: 3x3 convolutions with 64
// channels in and out on MFMA (bfloat16 operands, FP32 accumulation), the
// loss and Adam.  Images are NHWC with the spectral bins as channels (the
// voxel order of the reconstruction); weights are [co][ky][kx][ci].
//
// Convolution as implicit GEMM: output pixels x output channels, reduction
// over (tap, input channel), K = 9 * 64 = 576.  One workgroup computes two
// image rows (128 pixels) x 64 channels from LDS copies of the 4 input rows
// it needs and of all weights; a wave owns 32 pixels x 64 channels, i.e. 2 x 4
// tiles of v_mfma_f32_16x16x32_bf16 (lane l holds A[l%16][8(l/16)..+8],
// B[8(l/16)..+8][l%16], D[4(l/16)..+4][l%16]).
#include "sgtv_device.h"
#include "sgtv_wsnet.h"

namespace sgtv {
namespace wsn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kC = 64;                 // channels
constexpr int kK = 9 * kC;             // reduction length of one output
constexpr int kPixPad = kC + 8;        // bf16 per staged pixel (keeps 16-byte alignment)
constexpr int kWPad = kK + 8;          // bf16 per staged weight row

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoidf(float z) {
    return z >= 0.0f ? 1.0f / (1.0f + expf(-z)) : expf(z) / (1.0f + expf(z));
}

size_t conv_lds_bytes(int W) {
    return (static_cast<size_t>(4) * (W + 2) * kPixPad + static_cast<size_t>(kC) * kWPad) * 2;
}

// EP_RELU: out_bf16 = relu(z + b) (hidden layer); EP_SOFTPLUS: out_z = z + b,
// out_sp = softplus(z + b) (last layer); EP_MASK: out_bf16 = z if mask > 0
// else 0 (gradient through the ReLU of the previous layer, no bias).
template <int EP>
__global__ __launch_bounds__(256) void k_conv3x3(const __bf16 *__restrict__ X,
                                                 const __bf16 *__restrict__ Wk,
                                                 const float *__restrict__ bias, int H, int W,
                                                 __bf16 *__restrict__ out_bf16,
                                                 float *__restrict__ out_z,
                                                 float *__restrict__ out_sp,
                                                 const __bf16 *__restrict__ mask) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __bf16 *xs = reinterpret_cast<__bf16 *>(smem);
    __bf16 *ws = xs + static_cast<size_t>(4) * (W + 2) * kPixPad;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rows = H / 2;
    const int n = blockIdx.x / rows, y0 = (blockIdx.x % rows) * 2;

    for (int i = tid; i < kC * kK / 8; i += 256) {
        const int co = i / (kK / 8), k8 = i % (kK / 8);
        *reinterpret_cast<u16x8 *>(ws + co * kWPad + k8 * 8) =
            *reinterpret_cast<const u16x8 *>(Wk + static_cast<size_t>(co) * kK + k8 * 8);
    }
    for (int i = tid; i < 4 * (W + 2) * (kC / 8); i += 256) {
        const int c8 = i % (kC / 8), rest = i / (kC / 8);
        const int xc = rest % (W + 2), r = rest / (W + 2);
        const int sy = y0 - 1 + r, sx = xc - 1;
        u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
        if (sy >= 0 && sy < H && sx >= 0 && sx < W)
            v = *reinterpret_cast<const u16x8 *>(X + ((static_cast<size_t>(n) * H + sy) * W + sx) * kC + c8 * 8);
        *reinterpret_cast<u16x8 *>(xs + (r * (W + 2) + xc) * kPixPad + c8 * 8) = v;
    }
    __syncthreads();

    const int rr = wv >> 1, xb = (wv & 1) * 32;
    const int li = lane & 15, lk = (lane >> 4) * 8;
    f32x4 acc[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[t][u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int tap = 0; tap < 9; ++tap) {
        const int ky = tap / 3, kx = tap % 3;
#pragma unroll
        for (int c0 = 0; c0 < kC; c0 += 32) {
            bf16x8 a[2], b[4];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int px = xb + 16 * t + li;
                a[t] = *reinterpret_cast<const bf16x8 *>(xs + ((rr + ky) * (W + 2) + px + kx) * kPixPad + c0 + lk);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                b[u] = *reinterpret_cast<const bf16x8 *>(ws + (16 * u + li) * kWPad + tap * kC + c0 + lk);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b[u], acc[t][u], 0, 0, 0);
        }
    }
    const int y = y0 + rr;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int px = xb + 16 * t + (lane >> 4) * 4 + r;
                const int co = 16 * u + li;
                const size_t o = ((static_cast<size_t>(n) * H + y) * W + px) * kC + co;
                float z = acc[t][u][r];
                if (EP != 2) z += bias[co];
                if (EP == 0) out_bf16[o] = static_cast<__bf16>(fmaxf(z, 0.0f));
                if (EP == 1) {
                    out_z[o] = z;
                    out_sp[o] = softplusf(z);
                }
                if (EP == 2) out_bf16[o] = static_cast<float>(mask[o]) > 0.0f ? static_cast<__bf16>(z) : static_cast<__bf16>(0.0f);
            }
}

// Weight and bias gradient of one layer over `rows_per_block` image rows:
// dW[co][tap][ci] = sum_pixels dZ[pixel][co] X[pixel + tap][ci], as a GEMM
// with the pixels as reduction; both operands are staged transposed in LDS so
// that eight consecutive pixels of one channel are one 16-byte read.  Eight
// waves: wave w owns output channels 16 (w % 4).. and half of the 36 column
// tiles of (tap, ci).  Each block writes its partial sums; a second kernel adds
// the blocks in a fixed order.
constexpr int kRowPad = 64 + 8;        // bf16 per staged channel row (64 pixels + pad)

size_t wgrad_lds_bytes() {
    return (static_cast<size_t>(kC) * kRowPad + static_cast<size_t>(9) * kC * kRowPad) * 2;
}

__global__ __launch_bounds__(512) void k_conv_wgrad(const __bf16 *__restrict__ X,
                                                    const __bf16 *__restrict__ DZ, int H, int W,
                                                    int rows_per_block, float *__restrict__ part) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __bf16 *dzT = reinterpret_cast<__bf16 *>(smem);              // [co][pix]
    __bf16 *xT = dzT + static_cast<size_t>(kC) * kRowPad;        // [tap][ci][pix]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int blocks_per_img = H / rows_per_block;
    const int n = blockIdx.x / blocks_per_img, yb = (blockIdx.x % blocks_per_img) * rows_per_block;
    const int li = lane & 15, lk = (lane >> 4) * 8;
    const int u = wv & 3, half = wv >> 2;
    f32x4 acc[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    for (int yy = 0; yy < rows_per_block; ++yy) {
        const int y = yb + yy;
        __syncthreads();
        // dZ row, transposed: dzT[co][x]
        for (int i = tid; i < W * kC; i += 512) {
            const int co = i % kC, x = i / kC;
            dzT[co * kRowPad + x] = DZ[((static_cast<size_t>(n) * H + y) * W + x) * kC + co];
        }
        // inputs of every tap, transposed: xT[tap][ci][x] = X[y + ky - 1][x + kx - 1][ci]
        for (int i = tid; i < 9 * W * kC; i += 512) {
            const int ci = i % kC, rest = i / kC;
            const int x = rest % W, tap = rest / W;
            const int sy = y + tap / 3 - 1, sx = x + tap % 3 - 1;
            __bf16 v = static_cast<__bf16>(0.0f);
            if (sy >= 0 && sy < H && sx >= 0 && sx < W)
                v = X[((static_cast<size_t>(n) * H + sy) * W + sx) * kC + ci];
            xT[(tap * kC + ci) * kRowPad + x] = v;
        }
        __syncthreads();
        if (tid < kC)
            for (int x = 0; x < W; ++x) bsum += static_cast<float>(dzT[tid * kRowPad + x]);
        for (int p0 = 0; p0 < W; p0 += 32) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(dzT + (16 * u + li) * kRowPad + p0 + lk);
#pragma unroll
            for (int k = 0; k < 18; ++k) {
                const int nt = half * 18 + k;          // column tile: tap = nt / 4, ci0 = 16 (nt % 4)
                const int col = nt * 16 + li;          // = tap * 64 + ci
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(xT + col * kRowPad + p0 + lk);
                acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
            }
        }
    }
    float *out = part + static_cast<size_t>(blockIdx.x) * (kC * kK + kC);
#pragma unroll
    for (int k = 0; k < 18; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = 16 * u + (lane >> 4) * 4 + r;
            const int col = (half * 18 + k) * 16 + li;
            out[co * kK + col] = acc[k][r];
        }
    if (tid < kC) out[kC * kK + tid] = bsum;
}

// grad[k] = sum over blocks b of part[b][k], fixed order
__global__ __launch_bounds__(256) void k_block_sum(const float *__restrict__ part, int n_blocks,
                                                   int64_t len, float *__restrict__ grad) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (k >= len) return;
    float s = 0.0f;
    for (int b = 0; b < n_blocks; ++b) s += part[static_cast<int64_t>(b) * len + k];
    grad[k] = s;
}

__global__ void k_to_bf16(const float *__restrict__ x, __bf16 *__restrict__ y, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        y[i] = static_cast<__bf16>(x[i]);
}

// FP64 partial sums of each image: grid (n_blocks, images)
__global__ __launch_bounds__(256) void k_image_partials(const float *__restrict__ x, int64_t img,
                                                        double *__restrict__ partials) {
    const float *xi = x + static_cast<int64_t>(blockIdx.y) * img;
    double acc = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < img;
         i += static_cast<int64_t>(gridDim.x) * 256)
        acc += xi[i];
    block_sum_store(acc, partials + static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x);
}

// mean of image b from its sum; 1 where the mean is not positive
__device__ __forceinline__ double image_mean(const double *sums, int64_t b, int64_t img) {
    const double m = sums[b] / static_cast<double>(img);
    return m > 0.0 ? m : 1.0;
}

// network input: x / mean(image), rounded to bfloat16
__global__ void k_scale_to_bf16(const float *__restrict__ x, const double *__restrict__ sums,
                                int64_t img, int64_t n, __bf16 *__restrict__ y) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        y[i] = static_cast<__bf16>(static_cast<float>(x[i] / image_mean(sums, i / img, img)));
}

// start image from the network output s: c_out * s * f (ratio) or c_out * s * mean(f) (direct)
__global__ void k_start_image(const float *__restrict__ f, const float *__restrict__ s,
                              const double *__restrict__ sums, int64_t img, int64_t n, float c_out,
                              int ratio, float *__restrict__ x0) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float base = ratio ? f[i] : static_cast<float>(image_mean(sums, i / img, img));
        x0[i] = c_out * s[i] * base;
    }
}

// dZ of the last layer: 2 (out - target) / n * softplus'(z); FP64 loss partials
__global__ __launch_bounds__(256) void k_mse_grad(const float *__restrict__ out,
                                                  const float *__restrict__ target,
                                                  const float *__restrict__ z, int64_t n,
                                                  __bf16 *__restrict__ dz,
                                                  double *__restrict__ partials) {
    double acc = 0.0;
    const float inv = 2.0f / static_cast<float>(n);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        const float d = out[i] - target[i];
        acc += static_cast<double>(d) * d;
        dz[i] = static_cast<__bf16>(inv * d * sigmoidf(z[i]));
    }
    block_sum_store(acc, partials + blockIdx.x);
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// bfloat16 copies of one layer's weights: forward [co][tap][ci], and the
// backward-data kernel [ci][8 - tap][co] (flipped taps, swapped channels)
__global__ void k_weights_bf16(const float *__restrict__ w, __bf16 *__restrict__ wf,
                               __bf16 *__restrict__ wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kC * kK) return;
    const int co = i / kK, tap = (i % kK) / kC, ci = i % kC;
    const __bf16 h = static_cast<__bf16>(w[i]);
    wf[i] = h;
    wb[(static_cast<size_t>(ci) * 9 + (8 - tap)) * kC + co] = h;
}

// ---------------------------------------------------------------- launchers
template <int EP>
static hipError_t conv_t(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H,
                         int W, __bf16 *ob, float *oz, float *osp, const __bf16 *mask,
                         hipStream_t st) {
    static bool raised = false;
    const size_t lds = conv_lds_bytes(W);
    if (!raised) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv3x3<EP>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
        if (e != hipSuccess) return e;
        raised = true;
    }
    hipLaunchKernelGGL((k_conv3x3<EP>), dim3(static_cast<unsigned>(B * (H / 2))), dim3(256), lds,
                       st, X, Wk, bias, H, W, ob, oz, osp, mask);
    return hipGetLastError();
}

hipError_t conv_relu(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H, int W,
                     __bf16 *out, hipStream_t st) {
    return conv_t<0>(X, Wk, bias, B, H, W, out, nullptr, nullptr, nullptr, st);
}
hipError_t conv_softplus(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H,
                         int W, float *z, float *sp, hipStream_t st) {
    return conv_t<1>(X, Wk, bias, B, H, W, nullptr, z, sp, nullptr, st);
}
hipError_t conv_masked(const __bf16 *X, const __bf16 *Wk, int B, int H, int W, const __bf16 *mask,
                       __bf16 *out, hipStream_t st) {
    return conv_t<2>(X, Wk, nullptr, B, H, W, out, nullptr, nullptr, mask, st);
}

hipError_t conv_wgrad(const __bf16 *X, const __bf16 *DZ, int B, int H, int W, int rows_per_block,
                      float *part, float *grad, hipStream_t st) {
    static bool raised = false;
    if (!raised) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv_wgrad),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
        if (e != hipSuccess) return e;
        raised = true;
    }
    const int nb = B * (H / rows_per_block);
    hipLaunchKernelGGL(k_conv_wgrad, dim3(static_cast<unsigned>(nb)), dim3(512), wgrad_lds_bytes(),
                       st, X, DZ, H, W, rows_per_block, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t len = static_cast<int64_t>(kC) * kK + kC;
    hipLaunchKernelGGL(k_block_sum, dim3(static_cast<unsigned>((len + 255) / 256)), dim3(256), 0, st,
                       part, nb, len, grad);
    return hipGetLastError();
}

hipError_t to_bf16(const float *x, __bf16 *y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, dim3(static_cast<unsigned>(std::min<int64_t>(4096, (n + 255) / 256))),
                       dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

hipError_t image_partials(const float *x, int64_t img, int n_images, int n_blocks, double *partials,
                          hipStream_t st) {
    if (n_images == 0) return hipSuccess;
    hipLaunchKernelGGL(k_image_partials, dim3(static_cast<unsigned>(n_blocks), static_cast<unsigned>(n_images)),
                       dim3(256), 0, st, x, img, partials);
    return hipGetLastError();
}

hipError_t scale_to_bf16(const float *x, const double *sums, int64_t img, int64_t n, __bf16 *y,
                         hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_to_bf16, dim3(static_cast<unsigned>(std::min<int64_t>(4096, (n + 255) / 256))),
                       dim3(256), 0, st, x, sums, img, n, y);
    return hipGetLastError();
}

hipError_t start_image(const float *f, const float *s, const double *sums, int64_t img, int64_t n,
                       float c_out, int ratio, float *x0, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_start_image, dim3(static_cast<unsigned>(std::min<int64_t>(4096, (n + 255) / 256))),
                       dim3(256), 0, st, f, s, sums, img, n, c_out, ratio, x0);
    return hipGetLastError();
}

hipError_t mse_grad(const float *out, const float *target, const float *z, int64_t n, __bf16 *dz,
                    double *partials, int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_mse_grad, dim3(static_cast<unsigned>(n_blocks)), dim3(256), 0, st, out,
                       target, z, n, dz, partials);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>(std::min<int64_t>(4096, (n + 255) / 256))),
                       dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t weights_bf16(const float *w, __bf16 *wf, __bf16 *wb, hipStream_t st) {
    hipLaunchKernelGGL(k_weights_bf16, dim3((kC * kK + 255) / 256), dim3(256), 0, st, w, wf, wb);
    return hipGetLastError();
}

}  // namespace wsn
}  // namespace sgtv
