// Internal interface between the C-ABI host code and the CDNA4 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sgtv_persistent.h"

namespace sgtv {

constexpr int kWave = 64;          // wavefront width on gfx950
constexpr int kBlock = 256;        // threads per block for every streaming kernel
constexpr int kSliceRows = 64;     // lines (rows or columns) per sliced-ELL slice
constexpr int kDepth = 4;          // entries per lane per 16-byte index load

// Hyperspectral grid: J = S * Q voxels, voxel j = s * Q + q, s = iy * nx + ix.
struct Grid {
    int ny, nx, Q;
    int64_t S, J;
};

// Direction weights: constants per direction, or a full [s][p][q] array.
struct Weights {
    float w[4];
    const float *full;   // nullptr: use w[p]
};

// Sliced-ELL matrix in device memory (slices of 64 lines, depth padded to 4).
// Entry t of line l of slice k sits at sptr[k] + (t / 4) * 256 + (l % 64) * 4 + t % 4.
struct Sell {
    const int64_t *sptr;   // n_slices + 1 element offsets
    const int32_t *idx;    // gathered index per entry (padding: 0)
    const void *val;       // float / bf16 / fp16 codes (padding: 0)
    const float *scale;    // per-column scale for 16-bit values, nullptr for FP32
    int64_t n_lines, n_slices;
};

// LDS-tiled sparse product y = M x with per-slab partial outputs.
// Rows of M are cut into row blocks of waves * rw rows (one workgroup each;
// every wave owns rw rows of the block and keeps their sums in LDS: rows
// [w*rw, (w+1)*rw) for 32-bit indices, rows chosen per tile to even out the
// waves' work in every column block for 24-bit indices, see slot), columns
// into blocks of cb columns (staged in LDS one at a time) and
// the column blocks into ns slabs.  Workgroup b works on row block b / ns and
// slab b % ns, so all workgroups of a slab land on the same XCD and its
// slice of x stays in that XCD's L2.  Entries of one (row block, slab,
// column block, wave) list are stored in groups of 64 with 64 distinct rows,
// four groups interleaved per 16-byte load; packed index = row << 16 | col.
constexpr int kMaxSlabs = 16;

// The 24-bit index format: e = row << c | column with c = 14 column bits for
// up to 1024 rows per wave and c = 13 for up to 2048; the widest block leaves
// code cb for the zero slot (cb a multiple of 4, at most 2^c - 4).
inline int idx24_col_bits(int rw) { return rw <= 1024 ? 14 : 13; }
inline bool idx24_fits(int rw, int cb) {
    return rw >= 64 && rw <= 2048 && cb % 4 == 0 && cb <= (1 << idx24_col_bits(rw)) - 4;
}
// LDS of one tiled workgroup: the row sums (a spare padding row per wave with
// 32-bit indices), then the column block (and the zero slot with 24-bit ones)
inline size_t tiled_lds_bytes(int waves, int rw, int cb, bool idx24) {
    size_t a = static_cast<size_t>(waves) * (rw + (idx24 ? 0 : 1)) * 4;
    a = (a + 15) / 16 * 16;
    return a + static_cast<size_t>(cb) * 4 + (idx24 ? 16 : 0);
}

struct TileMap {
    const int32_t *pk;      // packed (row in wave, column in block), padding: row = rw
    const void *val;        // values or 16-bit codes, padding: 0
    const int32_t *goff;    // group offset of every list, n_lists + 1 entries
    const int32_t *poff;    // 24-bit indices: offset (in dwords) of every list's indices
    const uint16_t *slot;   // 24-bit indices: per tile, the slot w * rw + l (wave w, row l
                            // in the wave) of every row of the row block; nullptr: identity
    int idx24;              // 1: indices row << cbits | column, three dwords per lane and batch;
                            // padding: a row unused in its group, column cb (a zero in LDS)
    int64_t n_rows, n_cols;
    int64_t n_rb;           // row blocks
    int64_t pad;            // entry offset of one all-padding batch (256 entries)
    int rw, waves, cb, ns, cbs_max;
    int variant;            // kernel variant (0 simple, 1 pipelined, 2 + block prefetch)
    int cbits;              // 24-bit indices: column bits (idx24_col_bits(rw))
    int slab_begin[kMaxSlabs + 1];   // first column block of each slab
    size_t lds_bytes() const { return tiled_lds_bytes(waves, rw, cb, idx24 != 0); }
};

// Batched launches: one work item per workgroup.
struct BatchTile {
    int32_t scan;     // index into the per-scan arrays
    int32_t local;    // tile of that scan's map
};

// Per-scan vectors and parameters of the batched elementwise kernels; the
// image and split state are double buffered, the launch passes the parity.
struct ScanDev {
    const float *y, *r;
    float *ratio, *fpart, *bpart;
    float *f[2], *v[2], *a[2];
    const float *sens, *H;
    const float *htab;          // H0 by neighbour pattern (weights constant per direction)
    const float *scale;         // per-column scale of 16-bit values (nullptr: FP32) ...
    float *fs;                  // ... and the scaled image the forward product reads
    Grid grid;
    Weights wts;
    int64_t I;
    int ns_f, ns_b, seg_log2, grouping;
    float lam, thr;
};

// Block of a batched elementwise launch: scan and first element.
struct BatchBlock {
    int32_t scan;
    int32_t pad_;
    int64_t start;
};

// Arguments of the persistent batched iteration (one cooperative launch of
// n iterations over every scan; the order of work: sgtv_persistent.h).
// The tables live in device memory (the kernel indexes them at run time).
struct PersistentDev {
    const BatchTile *tiles_f, *tiles_b;
    const TileMap *maps_f, *maps_b;
    const float *const *xs_f0;      // forward input of every scan for fc = 0 (f[0]) ...
    const float *const *xs_f1;      // ... and fc = 1 (f[1])
    const float *const *xs_b;       // back input (the ratio) of every scan
    float *const *parts_f, *const *parts_b;
    const ScanDev *scans;
    const BatchBlock *rblocks, *vblocks, *sblocks;
    uint32_t *bar;                  // kBarWords counters, all 0 at launch (layout below)
    uint64_t limit;                 // longest wait at a barrier, in wall-clock ticks
    uint64_t *ticks;                // kPhaseSlots clock ticks added by workgroup 0: phases A-D
                                    // (from one barrier exit to the next), the last split
};
constexpr int kPhaseSlots = 5;

// Words of the persistent launch's counter buffer, each on its own 64-byte line:
// barrier arrivals (all workgroups), the error flag, the arrivals of every
// workgroup group g = wg mod 8, and the forward and back tile queues.
constexpr int kBarGlobal = 0, kBarErr = 1, kBarGroup = 16, kBarQueueF = 160, kBarQueueB = 288;
constexpr int kBarWords = 416;

// Image update and split/dual update in one pass over tiles of tw x th
// spatial bins (sgtv_update.hip).
constexpr int kFusedMaxLds = 65536;        // LDS of one workgroup's image tile and ring
struct FusedUpdate {
    const float *part;        // back-product partial sums, ns slabs of J
    int ns;
    const float *scale;       // per-column scale of 16-bit values (nullptr: FP32)
    const float *g;           // image f^k
    float *g_next, *gs_next;  // new image; its scaled copy for 16-bit values (or nullptr)
    const float *v_old, *a_old;
    float *v_new, *a_new;
    const float *sens;
    const float *H;           // curvature array (full weights) ...
    const float *htab;        // ... or 16 values by neighbour pattern (device memory)
    Grid grid;
    Weights wts;
    float lam, thr;
    int tw, th, tiles_x, seg_log2;
};
constexpr int kFusedThreads = 1024;        // default workgroup size
size_t fused_lds_bytes(int tw, int th, int Q);
// threads per workgroup: 256, 512 or 1024
hipError_t launch_update_fused(const FusedUpdate &A, int grouping, int threads, hipStream_t st);

// Launchers (all asynchronous on `st`).
// Workgroups of the persistent launch (all resident at once); *what names the
// call that failed.
hipError_t persistent_grid(int variant, int threads, size_t lds, int *grid, const char **what);
hipError_t launch_admm_persistent(const PersistentDev *D, const PersistentPlan &plan, size_t lds,
                                  int threads, int variant, int grid, hipStream_t st);
hipError_t launch_tiled_batch(const BatchTile *tiles, int64_t n_tiles, const TileMap *maps,
                              const float *const *xs, float *const *parts, int waves, size_t lds,
                              int variant, int vt, hipStream_t st);
hipError_t launch_ratio_batch(const BatchBlock *blocks, int64_t n_blocks, const ScanDev *scans,
                              hipStream_t st);
hipError_t launch_voxel_batch(const BatchBlock *blocks, int64_t n_blocks, const ScanDev *scans,
                              int fcur, int vcur, hipStream_t st);
hipError_t launch_split_batch(const BatchBlock *blocks, int64_t n_blocks, const ScanDev *scans,
                              int fcur, int vcur, hipStream_t st);
hipError_t launch_tiled(const TileMap &M, int vt, const float *x, float *part, hipStream_t st);

// A product whose row blocks are finished by the workgroup that completes
// them (the last of the row block's slabs to arrive at its counter): the
// forward product then computes the ratio of its rows, the back product the
// image update of its rows (voxels), with the arithmetic of
// launch_ratio_combine and launch_voxel_update.  count: n_rb counters, zero
// before the launch and again after it.
struct RatioEpilogue {
    uint32_t *count;
    const float *y, *r;
    float *ratio;
};
struct UpdateEpilogue {
    uint32_t *count;
    const float *scale;       // per-column scale of 16-bit values (nullptr: FP32)
    const float *g;           // image f^k
    float *g_next, *gs_next;  // new image; its scaled copy for 16-bit values (or nullptr)
    const float *v, *a, *sens, *H, *htab;
    Grid grid;
    Weights wts;
    float lam;
};
hipError_t launch_tiled_ratio(const TileMap &M, int vt, const float *x, float *part, const RatioEpilogue &E,
                              hipStream_t st);
hipError_t launch_tiled_update(const TileMap &M, int vt, const float *x, float *part, const UpdateEpilogue &E,
                               int grouping, hipStream_t st);
hipError_t launch_ratio_combine(const float *part, int ns, int64_t n, const float *y,
                                const float *r, float *ratio, double *partials, bool objective,
                                hipStream_t st, int64_t *n_partials);
hipError_t launch_back_combine(const float *part, int ns, int64_t n, const float *scale,
                               float *e, hipStream_t st);
hipError_t launch_voxel_update(const float *part, int ns, const float *scale, const float *g,
                               float *g_next, float *gs_next, const float *v, const float *a,
                               const float *sens, const float *H, const float *htab, const Grid &grid,
                               const Weights &w, int grouping, float lam, hipStream_t st);
hipError_t launch_forward_ratio(const Sell &A, int vt, const float *x, const float *y,
                                const float *r, float *ratio, double *partials, bool objective,
                                hipStream_t st, int64_t *n_partials);
hipError_t launch_back(const Sell &At, int vt, const float *t, float *e, hipStream_t st);
hipError_t launch_back_update(const Sell &At, int vt, const float *ratio, const float *g,
                              float *g_next, float *gs_next, const float *v, const float *a,
                              const float *sens, const float *H, const Grid &grid,
                              const Weights &w, int grouping, float lam, hipStream_t st);
hipError_t launch_split_update(const float *f, const float *v_old, const float *a_old,
                               float *v_new, float *a_new, const Grid &grid, const Weights &w,
                               int grouping, float thr, hipStream_t st);
hipError_t launch_consistent_split(const float *f, float *v, float *a, const Grid &grid,
                                   const Weights &w, int grouping, float thr, hipStream_t st);
hipError_t launch_report(const float *f, const float *v, const float *a, const float *v_prev,
                         const float *a_prev, const Grid &grid, const Weights &w, int grouping,
                         double *partials, hipStream_t st, int64_t *n_blocks);
// lam -> lam / t with lam c unchanged: c <- t c on the state (v, a), d kept
hipError_t launch_rescale_dual(float *v, float *a, const Grid &grid, int grouping, float t,
                               hipStream_t st);
hipError_t launch_reduce(const double *partials, int64_t n, int n_quant, double *out,
                         hipStream_t st);
hipError_t launch_sum_f32(const float *a, int64_t n, double *partials, hipStream_t st,
                          int64_t *n_blocks);
hipError_t launch_fill_ratio(const double *num, const double *den, float *out, int64_t n,
                             hipStream_t st);
hipError_t launch_scale(const float *x, const float *s, float *out, int64_t n, hipStream_t st);
hipError_t launch_split_from_state(const float *v, const float *a, float *d, float *c,
                                   const Grid &grid, int grouping, hipStream_t st);
hipError_t launch_div_safe(const float *num, const float *den, float *out, int64_t n,
                           hipStream_t st);
hipError_t launch_check_range(const float *x, int64_t n, float lo, int strict_lo, float hi,
                              int *flag, hipStream_t st);

}  // namespace sgtv
