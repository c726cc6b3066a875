// Elementwise kernels of the ADMM iteration for many scans in one launch.
// Block b works on scan blocks[b].scan starting at element blocks[b].start;
// the arithmetic per element is the single-scan kernels' own (shared device
// functions batch_*_elem / batch_split_block), so a scan of a batch
// reproduces its single-scan run bit for bit.
#include "sgtv_device.h"

namespace sgtv {

__global__ __launch_bounds__(kBlock) void k_ratio_batch(const BatchBlock *__restrict__ blocks,
                                                        const ScanDev *__restrict__ scans) {
    const BatchBlock bb = blocks[blockIdx.x];
    batch_ratio_elem(scans[bb.scan], bb.start + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_voxel_batch(const BatchBlock *__restrict__ blocks,
                                                        const ScanDev *__restrict__ scans,
                                                        int fcur, int vcur) {
    const BatchBlock bb = blocks[blockIdx.x];
    batch_voxel_elem(scans[bb.scan], bb.start + threadIdx.x, fcur, vcur);
}

__global__ __launch_bounds__(kBlock) void k_split_batch(const BatchBlock *__restrict__ blocks,
                                                        const ScanDev *__restrict__ scans,
                                                        int fcur, int vcur) {
    const BatchBlock bb = blocks[blockIdx.x];
    batch_split_block(scans[bb.scan], bb.start, threadIdx.x, fcur, vcur);
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
