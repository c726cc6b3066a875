// Kernels of the learned warm-start network: 3x3 convolutions with 64
// channels in and out on MFMA (bfloat16 operands, FP32 accumulation), the
// loss and Adam.  Images are NHWC with the spectral bins as channels (the
// voxel order of the reconstruction); weights are [co][ky][kx][ci].
//
// Convolution as implicit GEMM: output pixels x output channels, reduction
// over (tap, input channel), K = 9 * 64 = 576.  Persistent workgroups of four
// waves stage all weights in LDS once and then walk over steps of eight image
// rows: the ten input rows a step needs are staged in LDS, and wave w
// computes rows 2w and 2w + 1 of the step, 128 pixels x 64 channels, as
// 2 x 4 x 4 tiles of v_mfma_f32_16x16x32_bf16 (lane l holds A[l%16][8(l/16)..+8],
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

__device__ __forceinline__ float softplusf(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ __forceinline__ float sigmoidf(float z) {
    return z >= 0.0f ? 1.0f / (1.0f + expf(-z)) : expf(z) / (1.0f + expf(z));
}

constexpr int kStepRows = 8;                       // output rows per step (two per wave)
constexpr int kStageRows = kStepRows + 2;          // input rows a step reads
constexpr int kRowPix = kC + 2;                    // staged pixels per row (width 64 + halo)
constexpr int kChunks = kC / 8;                    // 16-byte chunks per pixel (8 channels each)

// LDS layout: the weights [co][tap][ci] (576 bf16 per output channel) and the
// step's input rows [row][pixel][ci], both without padding.  A 16-byte chunk
// is stored at its index XOR (row or pixel index mod 8) within each group of
// 8 chunks, so the 16 lanes that read one MFMA fragment (16 pixels or 16
// output channels at the same channel offset) hit 8 distinct 16-byte bank
// groups per half instead of one.
size_t conv_lds_bytes(int) {
    return (static_cast<size_t>(kC) * kK + static_cast<size_t>(kStageRows) * kRowPix * kC) * 2;
}

__device__ __forceinline__ int swz(int chunk, int key) { return (chunk & ~7) | ((chunk ^ key) & 7); }

// EP_RELU: out_bf16 = relu(z + b) (hidden layer); EP_SOFTPLUS: out_z = z + b,
// out_sp = softplus(z + b) (last layer); EP_MASK: out_bf16 = z if mask > 0
// else 0 (gradient through the ReLU of the previous layer, no bias).  When
// cm_out is not null, the bf16 output also goes out channel-major per image
// row, in the layouts the weight gradient reads: for EP_MASK once
// ([row][channel][x], its dZ), for EP_RELU in three copies shifted by
// kx - 1 = -1, 0, 1 pixels ([row][kx][channel][x], zero outside the row:
// the next layer's X).
//
// Workgroup of 8 waves (two per SIMD, so one wave's LDS reads overlap the
// other's MFMAs), one per CU; a step is 8 output rows of one image and wave w
// computes row w of it: 64 pixels x 64 output channels as 4 x 4 tiles of
// 16 x 16, each k-step of 32 (one tap, 32 input channels) reading 4 pixel and
// 4 weight fragments from LDS for 16 MFMAs.
constexpr int kConvThreads = 64 * kStepRows;

template <int EP>
__global__ __launch_bounds__(kConvThreads) void k_conv3x3(const __bf16 *__restrict__ X,
                                                          const __bf16 *__restrict__ Wk,
                                                          const float *__restrict__ bias, int B, int H,
                                                          __bf16 *__restrict__ out_bf16,
                                                          float *__restrict__ out_z,
                                                          float *__restrict__ out_sp,
                                                          const __bf16 *__restrict__ mask,
                                                          __bf16 *__restrict__ cm_out) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __bf16 *ws = reinterpret_cast<__bf16 *>(smem);                  // [co][576], swizzled chunks
    __bf16 *xs = ws + static_cast<size_t>(kC) * kK;                 // [row][pixel][64], swizzled
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int steps_per_img = (H + kStepRows - 1) / kStepRows;
    const int n_steps = B * steps_per_img;

    // the input rows of a step, loaded into registers (all loads in flight at once)
    constexpr int kRChunks = kStageRows * kRowPix * kChunks, kRPer = (kRChunks + kConvThreads - 1) / kConvThreads;
    u16x8 rv[kRPer];
    auto load_rows = [&](int step) {
        const int n = step / steps_per_img, y0 = (step % steps_per_img) * kStepRows;
#pragma unroll
        for (int k = 0; k < kRPer; ++k) {
            const int i = tid + k * kConvThreads;
            const int c8 = i % kChunks, rest = i / kChunks;
            const int xc = rest % kRowPix, r = rest / kRowPix;
            const int sy = y0 - 1 + r, sx = xc - 1;
            u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
            if (i < kRChunks && sy >= 0 && sy < H && sx >= 0 && sx < kC)
                v = *reinterpret_cast<const u16x8 *>(X + ((static_cast<size_t>(n) * H + sy) * kC + sx) * kC + c8 * 8);
            rv[k] = v;
        }
    };

    // the weights and the first step's rows in flight together, then the
    // weights to LDS
    constexpr int kWChunks = kC * (kK / 8), kWPer = kWChunks / kConvThreads;
    static_assert(kWChunks % kConvThreads == 0, "weight chunks per thread");
    {
        u16x8 wr[kWPer];
#pragma unroll
        for (int k = 0; k < kWPer; ++k) {
            const int i = tid + k * kConvThreads, co = i / (kK / 8), k8 = i % (kK / 8);
            wr[k] = *reinterpret_cast<const u16x8 *>(Wk + static_cast<size_t>(co) * kK + k8 * 8);
        }
        if (static_cast<int>(blockIdx.x) < n_steps) load_rows(blockIdx.x);
#pragma unroll
        for (int k = 0; k < kWPer; ++k) {
            const int i = tid + k * kConvThreads, co = i / (kK / 8), k8 = i % (kK / 8);
            *reinterpret_cast<u16x8 *>(ws + co * kK + swz(k8, co) * 8) = wr[k];
        }
    }

    const int li = lane & 15, g = lane >> 4;
    for (int step = blockIdx.x; step < n_steps; step += gridDim.x) {
        const int n = step / steps_per_img, y0 = (step % steps_per_img) * kStepRows;
        __syncthreads();                               // every wave is done with the previous step's LDS
#pragma unroll
        for (int k = 0; k < kRPer; ++k) {
            const int i = tid + k * kConvThreads;
            const int c8 = i % kChunks, rest = i / kChunks, xc = rest % kRowPix;
            if (i < kRChunks) *reinterpret_cast<u16x8 *>(xs + rest * kC + swz(c8, xc) * 8) = rv[k];
        }
        __syncthreads();
        // the next step's rows load while this one computes
        if (step + static_cast<int>(gridDim.x) < n_steps) load_rows(step + gridDim.x);

        const int y = y0 + wv;
        const bool active = y < H;
        f32x4 acc[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[t][u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        if (active) {
#pragma unroll 1
            for (int tap = 0; tap < 9; ++tap) {
                const int ky = tap / 3, kx = tap % 3;
                const __bf16 *row = xs + (wv + ky) * kRowPix * kC;
#pragma unroll
                for (int c0 = 0; c0 < kC; c0 += 32) {
                    const int cc = c0 / 8 + g;         // chunk of this lane's 8 input channels
                    bf16x8 a[4], b[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int px = 16 * t + li + kx;
                        a[t] = *reinterpret_cast<const bf16x8 *>(row + px * kC + swz(cc, px) * 8);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int co = 16 * u + li;
                        b[u] = *reinterpret_cast<const bf16x8 *>(ws + co * kK + swz(tap * kChunks + cc, co) * 8);
                    }
#pragma unroll
                    for (int t = 0; t < 4; ++t)
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b[u], acc[t][u], 0, 0, 0);
                }
            }
        }
        __syncthreads();                               // the staged rows are free: the outputs pass through them

        // Epilogue through LDS: the wave's tile is written to its own part of
        // the row area in the output's layout, then read back and stored as
        // 16-byte chunks, so every store instruction covers whole lines.
        const size_t base = (static_cast<size_t>(n) * H + y) * kC * kC;   // first element of row y
        if (EP != 1) {
            __bf16 *tile = xs + wv * (kC * kC);        // 8 KB per wave
            if (active) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int px = 16 * t + g * 4 + r, co = 16 * u + li;
                            float z = acc[t][u][r];
                            if (EP == 0) z = fmaxf(z + bias[co], 0.0f);
                            tile[px * kC + co] = static_cast<__bf16>(z);
                        }
            }
            __syncthreads();
            if (active) {
#pragma unroll 4
                for (int c = lane; c < kC * kC / 8; c += 64) {
                    u16x8 v = *reinterpret_cast<const u16x8 *>(tile + c * 8);
                    if (EP == 2) {
                        const u16x8 m = *reinterpret_cast<const u16x8 *>(mask + base + c * 8);
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            __bf16 mb;
                            const unsigned short mu = m[e];
                            __builtin_memcpy(&mb, &mu, 2);
                            if (!(static_cast<float>(mb) > 0.0f)) v[e] = 0;
                        }
                        if (cm_out) *reinterpret_cast<u16x8 *>(tile + c * 8) = v;   // masked, for the copy below
                    }
                    *reinterpret_cast<u16x8 *>(out_bf16 + base + c * 8) = v;
                }
            }
            if (cm_out) {
                __syncthreads();
                if (active) {
                    // eight lanes per channel, each eight pixels of the tile's column, so every
                    // store instruction writes eight whole 128-byte channel rows
                    const unsigned short *tu = reinterpret_cast<const unsigned short *>(tile);
                    const int x8 = lane & 7;
#pragma unroll 2
                    for (int k = 0; k < 8; ++k) {
                        const int co = (lane >> 3) + 8 * k;
                        if (EP == 2) {
                            u16x8 w;
#pragma unroll
                            for (int j = 0; j < 8; ++j) w[j] = tu[(x8 * 8 + j) * kC + co];
                            *reinterpret_cast<u16x8 *>(cm_out + base + static_cast<size_t>(co) * kC + x8 * 8) = w;
                        } else {
                            // pixels x8 * 8 - 1 .. x8 * 8 + 8 of the channel, 0 outside the row
                            unsigned short pv[10];
#pragma unroll
                            for (int j = 0; j < 10; ++j) {
                                const int px = x8 * 8 - 1 + j;
                                pv[j] = (px >= 0 && px < kC) ? tu[px * kC + co] : static_cast<unsigned short>(0);
                            }
#pragma unroll
                            for (int sh = 0; sh < 3; ++sh) {
                                u16x8 w;
#pragma unroll
                                for (int j = 0; j < 8; ++j) w[j] = pv[j + sh];
                                *reinterpret_cast<u16x8 *>(cm_out + 3 * base + static_cast<size_t>(sh) * kC * kC +
                                                           static_cast<size_t>(co) * kC + x8 * 8) = w;
                            }
                        }
                    }
                }
            }
        } else {
            // FP32 z and softplus(z), 32 pixels at a time (8 KB of FP32 per wave)
            float *tile = reinterpret_cast<float *>(xs) + wv * (kC * kC / 2);
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                if (active) {
#pragma unroll
                    for (int t = 2 * hh; t < 2 * hh + 2; ++t)
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int px = 16 * t + g * 4 + r - 32 * hh, co = 16 * u + li;
                                tile[px * kC + co] = acc[t][u][r] + bias[co];
                            }
                }
                __syncthreads();
                if (active) {
                    const size_t hb = base + static_cast<size_t>(hh) * 32 * kC;
#pragma unroll 4
                    for (int c = lane; c < 32 * kC / 4; c += 64) {
                        const f32x4 z = *reinterpret_cast<const f32x4 *>(tile + c * 4);
                        *reinterpret_cast<f32x4 *>(out_z + hb + c * 4) = z;
                        if (out_sp) {   // uniform: training leaves softplus(z) to the loss kernel
                            f32x4 sp;
                            sp[0] = softplusf(z[0]);
                            sp[1] = softplusf(z[1]);
                            sp[2] = softplusf(z[2]);
                            sp[3] = softplusf(z[3]);
                            *reinterpret_cast<f32x4 *>(out_sp + hb + c * 4) = sp;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
}

// Weight and bias gradient of one layer: dW[co][tap][ci] = sum over pixels of
// dZ[pixel][co] X[pixel + tap][ci], a GEMM with the pixels as reduction.  The
// matrix cores want eight consecutive pixels of one channel per lane, so both
// operands are first rewritten channel-major per image row (dZ once, X in
// three copies shifted by kx - 1 pixels, zero outside the row); the product
// kernel then loads every fragment with one aligned 16-byte read.

constexpr int kTPad = kC + 8;          // bf16 per channel row of the staged tile

// One block (256 threads) per image row r = n * H + y: out[(r * shifts + k)][c][x]
// = in[r][x + k - (shifts == 3)][c].
__global__ __launch_bounds__(256) void k_rows_cmajor(const __bf16 *__restrict__ in, int shifts,
                                                     __bf16 *__restrict__ out) {
    __shared__ __attribute__((aligned(16))) __bf16 tile[kC * kTPad];   // [c][x]
    const int64_t r = blockIdx.x;
    const __bf16 *src = in + r * kC * kC;                              // width = channels = 64
    for (int i = threadIdx.x; i < kC * kC / 8; i += 256) {
        const int x = i >> 3, c0 = (i & 7) * 8;
        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(src + x * kC + c0);
#pragma unroll
        for (int j = 0; j < 8; ++j) tile[(c0 + j) * kTPad + x] = v[j];
    }
    __syncthreads();
    const int off = shifts == 3 ? 1 : 0;
    for (int k = 0; k < shifts; ++k) {
        __bf16 *dst = out + (r * shifts + k) * kC * kC;
        for (int i = threadIdx.x; i < kC * kC / 8; i += 256) {
            const int c = i >> 3, x0 = (i & 7) * 8;
            bf16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x = x0 + j + k - off;
                v[j] = (x >= 0 && x < kC) ? tile[c * kTPad + x] : static_cast<__bf16>(0.0f);
            }
            *reinterpret_cast<bf16x8 *>(dst + c * kC + x0) = v;
        }
    }
}

// Partial dW over R image rows (block b: rows b R .. b R + R - 1 of one image);
// wave t = tap (ky, kx) accumulates all 64 x 64 (co, ci) outputs of its tap as
// 4 x 4 tiles of v_mfma_f32_16x16x32_bf16.  DT = dZ channel-major [row][co][x],
// XT = X channel-major with the three shifts [row][kx][ci][x].  The block's R
// rows of DT, which every tap's wave reads, are staged in LDS once (16-byte
// chunks at their index XOR (co mod 8)); the X fragments, different for every
// tap, come from memory.  The wave of the centre tap (which reads every row)
// also sums its dZ fragments: the block's bias partials follow its weight
// partials.  Row stride of part: C*9*C + C.
constexpr int kWgradThreads = 9 * 64;
constexpr int kWgradMaxRows = 8;

__global__ __launch_bounds__(kWgradThreads) void k_wgrad_taps(const __bf16 *__restrict__ DT,
                                                              const __bf16 *__restrict__ XT, int H, int R,
                                                              float *__restrict__ part) {
    __shared__ __attribute__((aligned(16))) __bf16 ds[kWgradMaxRows * kC * kC];   // 64 KB
    const int lane = threadIdx.x & 63;
    const int t = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ky = t / 3, kx = t % 3;
    const int li = lane & 15, g = lane >> 4, lk = g * 8;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * R;
    const int64_t n = row0 / H;
    const int y0 = static_cast<int>(row0 - n * H);
    {
        const __bf16 *src = DT + row0 * kC * kC;
        for (int i = threadIdx.x; i < R * kC * kC / 8; i += kWgradThreads) {
            const int x8 = i & 7, co = (i >> 3) & (kC - 1), r = i >> 9;
            *reinterpret_cast<u16x8 *>(ds + (r * kC + co) * kC + ((x8 ^ co) & 7) * 8) =
                *reinterpret_cast<const u16x8 *>(src + static_cast<int64_t>(i) * 8);
        }
    }
    __syncthreads();
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int yy = 0; yy < R; ++yy) {
        const int y = y0 + yy, sy = y + ky - 1;
        if (sy < 0 || sy >= H) continue;
        const __bf16 *drow = ds + yy * kC * kC;
        const __bf16 *xrow = XT + ((n * H + sy) * 3 + kx) * kC * kC;
#pragma unroll
        for (int p0 = 0; p0 < kC; p0 += 32) {
            const int x8 = (p0 + lk) / 8;
            bf16x8 a[4], b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(xrow + (16 * j + li) * kC + p0 + lk);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = 16 * i + li;
                a[i] = *reinterpret_cast<const bf16x8 *>(drow + co * kC + ((x8 ^ co) & 7) * 8);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            if (t == 4) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int e = 0; e < 8; ++e) bs[i] += static_cast<float>(a[i][e]);
            }
        }
    }
    float *out = part + static_cast<int64_t>(blockIdx.x) * (kC * kK + kC);
    if (t == 4) {
        // lanes li, li + 16, li + 32, li + 48 hold pixel quarters of channel 16 i + li
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = bs[i];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (g == 0) out[kC * kK + 16 * i + li] = v;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                out[(16 * i + 4 * g + q) * kK + t * kC + 16 * j + li] = acc[i][j][q];
}

// grad[k] = sum over blocks b of part[b][k] in a fixed order: four contiguous
// quarters of the blocks summed in order, then ((q0 + q1) + (q2 + q3)).
__global__ __launch_bounds__(256) void k_block_sum(const float *__restrict__ part, int n_blocks,
                                                   int64_t len, float *__restrict__ grad) {
    __shared__ float s4[4][64];
    const int kl = threadIdx.x & 63, qt = threadIdx.x >> 6;
    const int64_t k = static_cast<int64_t>(blockIdx.x) * 64 + kl;
    const int per = (n_blocks + 3) / 4;
    const int b0 = qt * per, b1 = min(n_blocks, b0 + per);
    float acc = 0.0f;
    if (k < len) {
        // eight loads in flight, then their additions in block order
        int b = b0;
        for (; b + 8 <= b1; b += 8) {
            float t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = part[static_cast<int64_t>(b + u) * len + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += t[u];
        }
        for (; b < b1; ++b) acc += part[static_cast<int64_t>(b) * len + k];
    }
    s4[qt][kl] = acc;
    __syncthreads();
    if (qt == 0 && k < len) grad[k] = (s4[0][kl] + s4[1][kl]) + (s4[2][kl] + s4[3][kl]);
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
                              int ratio, float floor, float *__restrict__ x0) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float m = static_cast<float>(image_mean(sums, i / img, img));
        const float base = ratio ? f[i] : m;
        const float v = c_out * s[i] * base;
        x0[i] = floor > 0.0f ? fmaxf(v, floor * c_out * m) : v;
    }
}

// dZ of the last layer: 2 (out - target) / n * softplus'(z) with out =
// softplus(z) (the same function as the layer's epilogue); FP64 loss partials
__global__ __launch_bounds__(256) void k_mse_grad(const float *__restrict__ target,
                                                  const float *__restrict__ z, int64_t n,
                                                  __bf16 *__restrict__ dz,
                                                  double *__restrict__ partials) {
    double acc = 0.0;
    const float inv = 2.0f / static_cast<float>(n);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256) {
        // softplusf(z) and sigmoidf(z) from one exp(-|z|): exp(-z) for z >= 0
        // and exp(z) below, bit for bit the values of the two functions
        const float zi = z[i];
        const float e = expf(-fabsf(zi));
        const float sp = fmaxf(zi, 0.0f) + log1pf(e);
        const float sg = zi >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
        const float d = sp - target[i];
        acc += static_cast<double>(d) * d;
        dz[i] = static_cast<__bf16>(inv * d * sg);
    }
    block_sum_store(acc, partials + blockIdx.x);
}

// One training step's mean squared error (its sum l[0] over cnt values) added
// to the running sum acc[0], and the step to the count acc[1].
__global__ void k_loss_accumulate(const double *__restrict__ l, double cnt, double *__restrict__ acc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        acc[0] += l[0] / cnt;
        acc[1] += 1.0;
    }
}

// 1 - beta1 and 1 - beta2 come from the host, formed in FP64: 1 - 0.999f in
// FP32 would be 0.000999987, a 1.3e-5 relative error in every second moment.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float omb1,
                       float omb2, float eps, float c1, float c2) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + omb1 * gi;
        const float vi = b2 * v[i] + omb2 * gi * gi;
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
int conv_workgroups() {
    // computed once (thread-safe initialisation of a function-local static)
    static const int n = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            return cus;
        return 256;
    }();
    return n;
}

template <int EP>
static hipError_t conv_t(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H,
                         int W, __bf16 *ob, float *oz, float *osp, const __bf16 *mask, __bf16 *cm,
                         hipStream_t st) {
    const size_t lds = conv_lds_bytes(W);
    static const hipError_t raised = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&k_conv3x3<EP>), hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
    if (raised != hipSuccess) return raised;
    const int n_steps = B * ((H + kStepRows - 1) / kStepRows);
    if (n_steps == 0) return hipSuccess;
    // one workgroup per CU (the staged weights and rows take 155 KB of LDS)
    const int grid = std::min(n_steps, conv_workgroups());
    hipLaunchKernelGGL((k_conv3x3<EP>), dim3(static_cast<unsigned>(grid)), dim3(kConvThreads), lds, st, X, Wk,
                       bias, B, H, ob, oz, osp, mask, cm);
    return hipGetLastError();
}

hipError_t conv_relu(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H, int W,
                     __bf16 *out, __bf16 *xt, hipStream_t st) {
    return conv_t<0>(X, Wk, bias, B, H, W, out, nullptr, nullptr, nullptr, xt, st);
}
hipError_t conv_softplus(const __bf16 *X, const __bf16 *Wk, const float *bias, int B, int H,
                         int W, float *z, float *sp, hipStream_t st) {
    return conv_t<1>(X, Wk, bias, B, H, W, nullptr, z, sp, nullptr, nullptr, st);
}
hipError_t conv_masked(const __bf16 *X, const __bf16 *Wk, int B, int H, int W, const __bf16 *mask,
                       __bf16 *out, __bf16 *dt, hipStream_t st) {
    return conv_t<2>(X, Wk, nullptr, B, H, W, out, nullptr, nullptr, mask, dt, st);
}

int wgrad_rows(int H) { return H % 8 == 0 ? 8 : (H % 4 == 0 ? 4 : 2); }

hipError_t conv_wgrad(const __bf16 *X, const __bf16 *DZ, int B, int H, float *xt, float *dt,
                      float *wpart, float *grad, bool xt_ready, bool dt_ready, hipStream_t st) {
    const int rows = B * H;
    if (rows == 0) return hipSuccess;
    __bf16 *XT = reinterpret_cast<__bf16 *>(xt);
    __bf16 *DT = reinterpret_cast<__bf16 *>(dt);
    hipError_t e = hipSuccess;
    if (!dt_ready) {
        hipLaunchKernelGGL(k_rows_cmajor, dim3(static_cast<unsigned>(rows)), dim3(256), 0, st, DZ, 1, DT);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!xt_ready) {
        hipLaunchKernelGGL(k_rows_cmajor, dim3(static_cast<unsigned>(rows)), dim3(256), 0, st, X, 3, XT);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int R = wgrad_rows(H);
    const int nb = rows / R;
    if (R > kWgradMaxRows) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wgrad_taps, dim3(static_cast<unsigned>(nb)), dim3(kWgradThreads), 0, st, DT, XT, H, R, wpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t len = static_cast<int64_t>(kC) * kK + kC;
    hipLaunchKernelGGL(k_block_sum, dim3(static_cast<unsigned>((len + 63) / 64)), dim3(256), 0, st,
                       wpart, nb, len, grad);
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
                       float c_out, int ratio, float floor, float *x0, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_start_image, dim3(static_cast<unsigned>(std::min<int64_t>(4096, (n + 255) / 256))),
                       dim3(256), 0, st, f, s, sums, img, n, c_out, ratio, floor, x0);
    return hipGetLastError();
}

hipError_t mse_grad(const float *target, const float *z, int64_t n, __bf16 *dz, double *partials,
                    int n_blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_mse_grad, dim3(static_cast<unsigned>(n_blocks)), dim3(256), 0, st, target, z, n, dz,
                       partials);
    return hipGetLastError();
}

hipError_t loss_accumulate(const double *l, double cnt, double *acc, hipStream_t st) {
    hipLaunchKernelGGL(k_loss_accumulate, dim3(1), dim3(64), 0, st, l, cnt, acc);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                float b2, float omb1, float omb2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>(std::min<int64_t>(4096, (n + 255) / 256))),
                       dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, omb1, omb2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t weights_bf16(const float *w, __bf16 *wf, __bf16 *wb, hipStream_t st) {
    hipLaunchKernelGGL(k_weights_bf16, dim3((kC * kK + 255) / 256), dim3(256), 0, st, w, wf, wb);
    return hipGetLastError();
}

}  // namespace wsn
}  // namespace sgtv
