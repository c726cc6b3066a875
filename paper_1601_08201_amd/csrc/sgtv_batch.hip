// Elementwise kernels of the ADMM iteration for many scans in one launch.
// Block b works on scan blocks[b].scan starting at element blocks[b].start;
// the arithmetic per element is the single-scan kernels' own (shared device
// functions), so a scan of a batch reproduces its single-scan run bit for bit.
#include "sgtv_device.h"

namespace sgtv {

// ratio = y / (sum of forward partials + r)
__global__ __launch_bounds__(kBlock) void k_ratio_batch(const BatchBlock *__restrict__ blocks,
                                                        const ScanDev *__restrict__ scans) {
    const BatchBlock bb = blocks[blockIdx.x];
    const ScanDev &S = scans[bb.scan];
    const int64_t i = bb.start + threadIdx.x;
    if (i >= S.I) return;
    float acc = S.fpart[i];
    for (int k = 1; k < S.ns_f; ++k) acc += S.fpart[static_cast<int64_t>(k) * S.I + i];
    const float p = acc + S.r[i];
    S.ratio[i] = S.y[i] / p;
}

// image update of every voxel (FP32 values)
__global__ __launch_bounds__(kBlock) void k_voxel_batch(const BatchBlock *__restrict__ blocks,
                                                        const ScanDev *__restrict__ scans,
                                                        int fcur, int vcur) {
    const BatchBlock bb = blocks[blockIdx.x];
    const ScanDev &S = scans[bb.scan];
    const int64_t j = bb.start + threadIdx.x;
    if (j >= S.grid.J) return;
    auto e = [&]() {
        float s = S.bpart[j];
        for (int k = 1; k < S.ns_b; ++k) s += S.bpart[static_cast<int64_t>(k) * S.grid.J + j];
        return s;
    };
    const float *g = S.f[fcur], *v = S.v[vcur], *a = S.a[vcur];
    float gnew;
    if (S.grouping == 0)
        gnew = S.wts.full ? voxel_update_value<0, true>(j, e, g, v, a, S.sens, S.H, S.grid, S.wts, S.lam)
                          : voxel_update_value<0, false>(j, e, g, v, a, S.sens, S.H, S.grid, S.wts, S.lam);
    else
        gnew = S.wts.full ? voxel_update_value<1, true>(j, e, g, v, a, S.sens, S.H, S.grid, S.wts, S.lam)
                          : voxel_update_value<1, false>(j, e, g, v, a, S.sens, S.H, S.grid, S.wts, S.lam);
    S.f[fcur ^ 1][j] = gnew;
}

// split and dual update, one segment of 2^seg_log2 lanes per spatial bin
__global__ __launch_bounds__(kBlock) void k_split_batch(const BatchBlock *__restrict__ blocks,
                                                        const ScanDev *__restrict__ scans,
                                                        int fcur, int vcur) {
    const BatchBlock bb = blocks[blockIdx.x];
    const ScanDev &S = scans[bb.scan];
    const int sl = S.seg_log2;
    const int64_t s = bb.start + (threadIdx.x >> sl);
    const int ls = threadIdx.x & ((1 << sl) - 1);
    const float *f = S.f[fcur], *v = S.v[vcur], *a = S.a[vcur];
    float *vn = S.v[vcur ^ 1], *an = S.a[vcur ^ 1];
    const bool act = s < S.grid.S;
    if (S.grouping == 0) {
        if (S.wts.full) split_bin<0, true>(s, act, ls, sl, f, v, a, vn, an, S.grid, S.wts, S.thr);
        else split_bin<0, false>(s, act, ls, sl, f, v, a, vn, an, S.grid, S.wts, S.thr);
    } else {
        if (S.wts.full) split_bin<1, true>(s, act, ls, sl, f, v, a, vn, an, S.grid, S.wts, S.thr);
        else split_bin<1, false>(s, act, ls, sl, f, v, a, vn, an, S.grid, S.wts, S.thr);
    }
}

hipError_t launch_ratio_batch(const BatchBlock *blocks, int64_t n_blocks, const ScanDev *scans,
                              hipStream_t st) {
    if (n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ratio_batch, dim3(static_cast<unsigned>(n_blocks)), dim3(kBlock), 0, st,
                       blocks, scans);
    return hipGetLastError();
}

hipError_t launch_voxel_batch(const BatchBlock *blocks, int64_t n_blocks, const ScanDev *scans,
                              int fcur, int vcur, hipStream_t st) {
    if (n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_voxel_batch, dim3(static_cast<unsigned>(n_blocks)), dim3(kBlock), 0, st,
                       blocks, scans, fcur, vcur);
    return hipGetLastError();
}

hipError_t launch_split_batch(const BatchBlock *blocks, int64_t n_blocks, const ScanDev *scans,
                              int fcur, int vcur, hipStream_t st) {
    if (n_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_batch, dim3(static_cast<unsigned>(n_blocks)), dim3(kBlock), 0, st,
                       blocks, scans, fcur, vcur);
    return hipGetLastError();
}

}  // namespace sgtv
