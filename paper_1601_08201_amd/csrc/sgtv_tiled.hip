// LDS-tiled sparse products for the forward projection A f and the
// backprojection A^T t of the ADMM iteration (Section III, image update).
//
// Random 4-byte gathers of the projected vector are the cost of a sparse
// product on this matrix family: served from L2 they cap the value stream far
// below HBM speed, served from LDS they do not.  So each workgroup keeps the
// sums of its row block in LDS, stages the gathered vector one column block
// at a time into LDS (read coalesced from L2, where the XCD-pinned slab of
// the vector stays resident) and streams the entries of the block with
// nontemporal 16-byte loads.  Every row of a wave's accumulator range is hit
// by at most one lane per instruction, so read-modify-write needs no atomics
// and each sum has a fixed order.
#include "sgtv_device.h"
#include "sgtv_persistent.h"

namespace sgtv {

typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Float4 chunks of the next column block each thread holds in registers while
// the current block is being processed (blocks larger than this are staged
// without the register prefetch).
constexpr int kXPrefetch = 4;

// Products of one batch (4 groups of 64 entries, 4 entries per lane) into
// the wave's LDS accumulators; rows within a group are distinct.
//
// Index formats.  32-bit: one dword (row << 16 | column) per entry, padding
// in the extra row rw.  24-bit (64 <= rows per wave <= 2048, block columns a
// multiple of 4 up to 2^c - 4): e = row << c | column with c = 14 column bits
// (up to 1024 rows per wave) or 13 (up to 2048), padding in a row the group
// does not use, reading the zero at column cb; and
// the four entries a lane holds in one batch share three dwords
// w0 = e0 | e1 << 24, w1 = e1 >> 8 | e2 << 16, w2 = e2 >> 16 | e3 << 8.  Four
// consecutive batches form a super-batch whose 12 dwords per lane are stored
// as three planes of 64 lanes x 16 bytes (three aligned loads per 16 entries);
// the batches past the last whole super-batch are stored as two planes each
// (64 lanes x (w0, w1), then 64 lanes x w2), and the groups past the last
// whole batch keep one dword per entry.
template <int VT>
__device__ __forceinline__ void tile_batch(const v4i p, const typename Code<VT>::V4 a,
                                           const float *xs, float *my) {
    float t;
    t = xs[p.x & 0xFFFF]; my[p.x >> 16] = fmaf(Code<VT>::dec(a.x), t, my[p.x >> 16]);
    t = xs[p.y & 0xFFFF]; my[p.y >> 16] = fmaf(Code<VT>::dec(a.y), t, my[p.y >> 16]);
    t = xs[p.z & 0xFFFF]; my[p.z >> 16] = fmaf(Code<VT>::dec(a.z), t, my[p.z >> 16]);
    t = xs[p.w & 0xFFFF]; my[p.w >> 16] = fmaf(Code<VT>::dec(a.w), t, my[p.w >> 16]);
}

// A lane's window of N entries with 24-bit indices (lane-owned lists: no
// other lane touches these rows, and equal rows are adjacent): all gathers and
// accumulator reads are issued first, then the running sum of each row is
// carried in a register across adjacent entries and written once per run (the
// sums keep their order: entry after entry).
template <int VT, int N>
__device__ __forceinline__ void window24(const uint32_t (&e)[N], const typename Code<VT>::T (&a)[N],
                                         const float *xs, float *my, uint32_t cbits) {
    const uint32_t cmask = (1u << cbits) - 1u;
    float t[N], m[N];
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = xs[e[i] & cmask];
#pragma unroll
    for (int i = 0; i < N; ++i) m[i] = my[e[i] >> cbits];
    float run = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint32_t row = e[i] >> cbits;
        const bool cont = i > 0 && row == (e[i - 1] >> cbits);
        run = fmaf(Code<VT>::dec(a[i]), t[i], cont ? run : m[i]);
        if (i + 1 == N || (e[i + 1] >> cbits) != row) my[row] = run;
    }
}

__device__ __forceinline__ void unpack4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t *e) {
    e[0] = w0 & 0xFFFFFFu;
    e[1] = ((w0 >> 24) | (w1 << 8)) & 0xFFFFFFu;
    e[2] = ((w1 >> 16) | (w2 << 16)) & 0xFFFFFFu;
    e[3] = w2 >> 8;
}

// one batch (4 entries per lane)
template <int VT>
__device__ __forceinline__ void tile_batch24(uint32_t w0, uint32_t w1, uint32_t w2,
                                             const typename Code<VT>::V4 a, const float *xs,
                                             float *my, uint32_t cbits) {
    uint32_t e[4];
    unpack4(w0, w1, w2, e);
    const typename Code<VT>::T av[4] = {a.x, a.y, a.z, a.w};
    window24<VT, 4>(e, av, xs, my, cbits);
}

// one super-batch (16 entries per lane: three 16-byte index planes, four value batches)
template <int VT, class U4>
__device__ __forceinline__ void tile_super24(const U4 A, const U4 B, const U4 C,
                                             const typename Code<VT>::V4 a0,
                                             const typename Code<VT>::V4 a1,
                                             const typename Code<VT>::V4 a2,
                                             const typename Code<VT>::V4 a3, const float *xs,
                                             float *my, uint32_t cbits) {
    uint32_t e[16];
    unpack4(A.x, A.y, A.z, e);
    unpack4(A.w, B.x, B.y, e + 4);
    unpack4(B.z, B.w, C.x, e + 8);
    unpack4(C.y, C.z, C.w, e + 12);
    const typename Code<VT>::T av[16] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w,
                                         a2.x, a2.y, a2.z, a2.w, a3.x, a3.y, a3.z, a3.w};
    window24<VT, 16>(e, av, xs, my, cbits);
}

// MODE 0: one batch at a time, the next column block staged after the
//         barrier; 32-bit or 24-bit indices.
// MODE 1: two batches in flight per wave (the batch past the end of a list is
//         the all-padding batch, so the loop is straight-line and the wait
//         counts stay exact).
// MODE 2: MODE 1, and the next column block is read into registers (kXPrefetch
//         float4 per thread; needs cb <= 16 * threads) after the last batch
//         of the current block has been issued.
template <int VT, int MODE, bool PREFETCH = true>
__device__ __forceinline__ void tiled_body(const TileMap &M, int64_t tile,
                                           const int32_t *__restrict__ pk,
                                           const typename Code<VT>::T *__restrict__ val,
                                           const int32_t *__restrict__ goff,
                                           const int32_t *__restrict__ poff,
                                           const float *__restrict__ x,
                                           float *__restrict__ part) {
    typedef typename Code<VT>::T T;
    typedef typename Code<VT>::V4 V4;
    extern __shared__ float lds[];
    // row sums: rw per wave, plus the padding row of the 32-bit format
    const int rw1 = M.rw + (M.idx24 ? 0 : 1);
    const uint32_t cbits = static_cast<uint32_t>(M.cbits);
    float *acc = lds;
    const size_t acc_floats = (static_cast<size_t>(M.waves) * rw1 + 3) / 4 * 4;
    float *xs = lds + acc_floats;

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    // the wave index is uniform: scalar list offsets and uniform loop bounds
    const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
    const int lane = tid & (kWave - 1);
    const int slab = static_cast<int>(tile % M.ns);
    const int64_t rb = tile / M.ns;
    float *my = acc + w * rw1;

    for (int i = tid; i < M.waves * rw1; i += nthr) acc[i] = 0.0f;
    // zero slot read by the padding entries of the 24-bit format (the staging
    // of a block, cb a multiple of 4, never writes past xs[cb - 1])
    if (M.idx24 && tid < 4) xs[M.cb + tid] = 0.0f;

    const int cb0 = M.slab_begin[slab];
    const int ncbs = M.slab_begin[slab + 1] - cb0;
    const int64_t list0 = ((rb * M.ns + slab) * M.cbs_max) * M.waves + w;
    const v4i *pad4 = reinterpret_cast<const v4i *>(pk + M.pad) + lane;
    const V4 *padv4 = reinterpret_cast<const V4 *>(val + M.pad) + lane;

    // the gathered vector is padded to a multiple of 4 floats plus 16, so a
    // whole float4 that starts inside it stays inside the allocation
    if (ncbs > 0) {
        const int64_t col0 = static_cast<int64_t>(cb0) * M.cb;
        const int64_t rem = M.n_cols - col0;
        const int ncols = rem < M.cb ? static_cast<int>(rem) : M.cb;
        for (int i4 = tid * 4; i4 < ncols; i4 += nthr * 4)
            *reinterpret_cast<v4f *>(xs + i4) = *reinterpret_cast<const v4f *>(x + col0 + i4);
    }
    __syncthreads();

    // the next column block is read into registers before the block barrier
    // (so its latency overlaps the wait there): MODE 2, and the simple loop on
    // 24-bit lists when the block fits the prefetch registers.  All kXPrefetch
    // loads are issued unconditionally (a chunk past a narrow block rereads
    // the block's first float4; skipping such chunks with a uniform branch
    // made the products 11 % slower)
    const bool pre = PREFETCH && (MODE == 2 || (MODE == 0 && M.idx24 && M.cb <= kXPrefetch * 4 * nthr));
    // The offsets of a block's list (group offset, length, and where its
    // 24-bit indices start) are read one block ahead, while the previous
    // block streams: read after the block barrier, every wave of the
    // workgroup would wait for them at once with nothing else in flight.
    // The reads are unconditional (the last block rereads its own list;
    // 32-bit lists read goff in place of poff and ignore the value).
    const int32_t *lp = M.idx24 ? poff : goff;
    int nx_g0 = 0, nx_g1 = 0, nx_po = 0;
    if (ncbs > 0) {
        nx_g0 = goff[list0];
        nx_g1 = goff[list0 + 1];
        nx_po = lp[list0];
    }
    for (int c = 0; c < ncbs; ++c) {
        const int64_t L = list0 + static_cast<int64_t>(c) * M.waves;
        const int g0 = __builtin_amdgcn_readfirstlane(nx_g0);
        const int ng = __builtin_amdgcn_readfirstlane(nx_g1) - g0;
        const int po = __builtin_amdgcn_readfirstlane(nx_po);
        {
            const int64_t Ln = c + 1 < ncbs ? L + M.waves : L;
            nx_g0 = goff[Ln];
            nx_g1 = goff[Ln + 1];
            nx_po = lp[Ln];
        }
        const int nb4 = ng >> 2;
        const int64_t base = static_cast<int64_t>(g0) * kWave;
        const v4i *p4 = reinterpret_cast<const v4i *>(pk + base) + lane;
        const V4 *v4 = reinterpret_cast<const V4 *>(val + base) + lane;

        const int cn = c + 1 < ncbs ? c + 1 : c;
        const int64_t ncol0 = static_cast<int64_t>(cb0 + cn) * M.cb;
        const int64_t nrem = M.n_cols - ncol0;
        const int nncols = nrem < M.cb ? static_cast<int>(nrem) : M.cb;
        v4f xr[kXPrefetch];
        const bool i24 = MODE == 0 && M.idx24;
        const uint32_t *p3 = nullptr;
        if (i24) p3 = reinterpret_cast<const uint32_t *>(pk + po);
        if (MODE == 0 && i24) {
            const int nsb = nb4 >> 2;
            const v4u *qs = reinterpret_cast<const v4u *>(p3) + lane;
            for (int sb = 0; sb < nsb; ++sb) {
                const v4u A = __builtin_nontemporal_load(qs + sb * 3 * kWave);
                const v4u B = __builtin_nontemporal_load(qs + sb * 3 * kWave + kWave);
                const v4u C = __builtin_nontemporal_load(qs + sb * 3 * kWave + 2 * kWave);
                const V4 a0 = __builtin_nontemporal_load(v4 + (4 * sb) * kWave);
                const V4 a1 = __builtin_nontemporal_load(v4 + (4 * sb + 1) * kWave);
                const V4 a2 = __builtin_nontemporal_load(v4 + (4 * sb + 2) * kWave);
                const V4 a3 = __builtin_nontemporal_load(v4 + (4 * sb + 3) * kWave);
                tile_super24<VT>(A, B, C, a0, a1, a2, a3, xs, my, cbits);
            }
            const uint32_t *q2 = p3 + static_cast<int64_t>(nsb) * 12 * kWave;
            const v2u *qa = reinterpret_cast<const v2u *>(q2) + lane;
            const uint32_t *qb = q2 + 2 * kWave + lane;
            for (int b = nsb * 4; b < nb4; ++b) {
                const int rb4 = b - nsb * 4;
                const v2u w01 = __builtin_nontemporal_load(qa + rb4 * (3 * kWave / 2));
                const uint32_t w2 = __builtin_nontemporal_load(qb + rb4 * 3 * kWave);
                const V4 a = __builtin_nontemporal_load(v4 + b * kWave);
                tile_batch24<VT>(w01.x, w01.y, w2, a, xs, my, cbits);
            }
        } else if (MODE == 0) {
            for (int b = 0; b < nb4; ++b) {
                const v4i p = __builtin_nontemporal_load(p4 + b * kWave);
                const V4 a = __builtin_nontemporal_load(v4 + b * kWave);
                tile_batch<VT>(p, a, xs, my);
            }
        } else {
            v4i pA = __builtin_nontemporal_load(nb4 > 0 ? p4 : pad4);
            V4 aA = __builtin_nontemporal_load(nb4 > 0 ? v4 : padv4);
            for (int b = 0; b < nb4; b += 2) {
                // a batch past the end of the list is the all-padding batch
                // (row = rw, value 0): processing it changes nothing
                const bool h1 = b + 1 < nb4, h2 = b + 2 < nb4;
                const v4i pB = __builtin_nontemporal_load(h1 ? p4 + (b + 1) * kWave : pad4);
                const V4 aB = __builtin_nontemporal_load(h1 ? v4 + (b + 1) * kWave : padv4);
                tile_batch<VT>(pA, aA, xs, my);
                pA = __builtin_nontemporal_load(h2 ? p4 + (b + 2) * kWave : pad4);
                aA = __builtin_nontemporal_load(h2 ? v4 + (b + 2) * kWave : padv4);
                tile_batch<VT>(pB, aB, xs, my);
            }
        }
        if (pre && c + 1 < ncbs) {
#pragma unroll
            for (int k = 0; k < kXPrefetch; ++k) {
                const int i4 = (k * nthr + tid) * 4;
                xr[k] = *reinterpret_cast<const v4f *>(x + ncol0 + (i4 < nncols ? i4 : 0));
            }
        }
        const int64_t tail = base + static_cast<int64_t>(nb4) * 4 * kWave + lane;
        if (i24) {
            const uint32_t *pt = p3 + static_cast<int64_t>(nb4) * 3 * kWave + lane;
            for (int g = nb4 * 4; g < ng; ++g) {
                const uint32_t p = __builtin_nontemporal_load(pt + (g - nb4 * 4) * kWave);
                const T a = __builtin_nontemporal_load(val + tail + static_cast<int64_t>(g - nb4 * 4) * kWave);
                const float t = xs[p & ((1u << cbits) - 1u)];
                my[p >> cbits] = fmaf(Code<VT>::dec(a), t, my[p >> cbits]);
            }
        } else {
            for (int g = nb4 * 4; g < ng; ++g) {
                const int64_t e = tail + static_cast<int64_t>(g - nb4 * 4) * kWave;
                const int p = __builtin_nontemporal_load(pk + e);
                const T a = __builtin_nontemporal_load(val + e);
                const float t = xs[p & 0xFFFF];
                my[p >> 16] = fmaf(Code<VT>::dec(a), t, my[p >> 16]);
            }
        }
        if (c + 1 < ncbs) {
            __syncthreads();   // every wave is done with this block
            if (pre) {
#pragma unroll
                for (int k = 0; k < kXPrefetch; ++k) {
                    const int i4 = (k * nthr + tid) * 4;
                    if (i4 < nncols) *reinterpret_cast<v4f *>(xs + i4) = xr[k];
                }
            } else {
                for (int i4 = tid * 4; i4 < nncols; i4 += nthr * 4)
                    *reinterpret_cast<v4f *>(xs + i4) = *reinterpret_cast<const v4f *>(x + ncol0 + i4);
            }
            __syncthreads();
        }
    }
    __syncthreads();
    const int64_t rb_rows = static_cast<int64_t>(M.waves) * M.rw;
    const int64_t row0 = rb * rb_rows;
    float *out = part + static_cast<int64_t>(slab) * M.n_rows;
    const uint16_t *sl = M.slot ? M.slot + (rb * M.ns + slab) * rb_rows : nullptr;
    for (int64_t i = tid; i < rb_rows && row0 + i < M.n_rows; i += nthr) {
        const int64_t s = sl ? static_cast<int64_t>(sl[i]) : i;
        out[row0 + i] = acc[(s / M.rw) * rw1 + (s % M.rw)];
    }
}

template <int VT, int MODE>
__global__ __launch_bounds__(1024) void k_tiled(TileMap M, const int32_t *__restrict__ pk,
                                                const typename Code<VT>::T *__restrict__ val,
                                                const int32_t *__restrict__ goff,
                                                const int32_t *__restrict__ poff,
                                                const float *__restrict__ x,
                                                float *__restrict__ part) {
    tiled_body<VT, MODE>(M, blockIdx.x, pk, val, goff, poff, x, part);
}

// Many scans in one launch: workgroup b runs tile tiles[b].local of scan
// tiles[b].scan with that scan's map and vectors.
template <int VT, int MODE>
__global__ __launch_bounds__(1024) void k_tiled_batch(const BatchTile *__restrict__ tiles,
                                                      const TileMap *__restrict__ maps,
                                                      const float *const *__restrict__ xs,
                                                      float *const *__restrict__ parts) {
    const BatchTile bt = tiles[blockIdx.x];
    if (bt.local < 0) return;   // alignment filler: the whole workgroup leaves
    // a reference, not a copy: fields (and the slab table indexed at run time)
    // are read with scalar loads instead of living in scratch memory
    const TileMap &M = maps[bt.scan];
    tiled_body<VT, MODE>(M, bt.local, M.pk, static_cast<const typename Code<VT>::T *>(M.val),
                         M.goff, M.poff, xs[bt.scan], parts[bt.scan]);
}

// ---------------------------------------------------------------- persistent batch
// All phases of n ADMM iterations of a batch in one cooperative launch (the
// order of work, its dependences and the tile queues: sgtv_persistent.h).
// Between dependent phases every workgroup waits at a grid barrier: each wave
// waits for its own memory operations, then one thread makes the workgroup's
// writes visible device-wide, adds its arrival to its group's counter (the
// last of a group adds the group to the global count) and waits for the
// phase's count.  The wait is bounded: past `limit` ticks of the constant-rate
// clock, or when another workgroup has already given up, the workgroup sets
// the error flag and leaves the kernel, so every wave ends and the host
// reports the failure.
template <int MODE>
struct PersistentWork {
    const PersistentDev &D;   // in device memory
    uint64_t *last;           // LDS: clock at the last barrier exit (workgroup 0, thread 0)
    __device__ __forceinline__ uint32_t *word(int i) const { return D.bar + i; }
    __device__ __forceinline__ int64_t grab(int phase, uint32_t q) {
        __shared__ int next;
        __syncthreads();   // every thread has read the previous index
        if (threadIdx.x == 0)
            next = static_cast<int>(__hip_atomic_fetch_add(
                word((phase == kPhaseForward ? kBarQueueF : kBarQueueB) + 16 * static_cast<int>(q)), 1u,
                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        __syncthreads();
        return next;
    }
    __device__ __forceinline__ void clear(int phase) {
        if (threadIdx.x < kMaxQueues)
            __hip_atomic_store(word((phase == kPhaseForward ? kBarQueueF : kBarQueueB) + 16 * threadIdx.x), 0u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ __forceinline__ void tile(int phase, int64_t t, int fc) {
        const bool fwd = phase == kPhaseForward;
        const BatchTile bt = (fwd ? D.tiles_f : D.tiles_b)[t];
        if (bt.local < 0) return;   // alignment filler (uniform in the workgroup)
        const TileMap &M = (fwd ? D.maps_f : D.maps_b)[bt.scan];
        const float *x = fwd ? (fc ? D.xs_f1 : D.xs_f0)[bt.scan] : D.xs_b[bt.scan];
        float *part = (fwd ? D.parts_f : D.parts_b)[bt.scan];
        // without the register prefetch of the next column block: its 16
        // registers would push the walk past the 128 of a 16-wave workgroup
        // (same sums in the same order, only the timing of the staging loads
        // differs).  grab() synchronised the workgroup before this tile.
        tiled_body<0, MODE, false>(M, bt.local, M.pk, static_cast<const float *>(M.val), M.goff, M.poff, x,
                                   part);
    }
    __device__ __forceinline__ void blocks(int phase, int64_t first, int64_t stride, int64_t n, int fc, int vc) {
        const int q = threadIdx.x / kBlock, t = threadIdx.x % kBlock;
        const BatchBlock *tab = phase == kPhaseRatio ? D.rblocks : phase == kPhaseVoxel ? D.vblocks : D.sblocks;
        for (int64_t b = first + q; b < n; b += stride) {
            const BatchBlock bb = tab[b];
            const ScanDev &S = D.scans[bb.scan];
            if (phase == kPhaseRatio) batch_ratio_elem(S, bb.start + t);
            else if (phase == kPhaseVoxel) batch_voxel_elem(S, bb.start + t, fc, vc);
            else batch_split_block(S, bb.start, t, fc, vc);
        }
    }
    __device__ __forceinline__ bool barrier(uint32_t target) {
        __shared__ int ok;
        const uint32_t G = gridDim.x, m = target / G;
        const uint32_t ng = persistent_queues(G), g = blockIdx.x % ng, n_g = (G - g + ng - 1) / ng;
        __builtin_amdgcn_s_waitcnt(0);   // this wave's loads and stores have completed
        __syncthreads();
        if (threadIdx.x == 0) {
            int good = __hip_atomic_load(word(kBarErr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
            if (good) {
                // release: the workgroup's writes (now in this XCD's L2) become visible device-wide
                const uint32_t old = __hip_atomic_fetch_add(word(kBarGroup + 16 * static_cast<int>(g)), 1u,
                                                            __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                if (old + 1 == m * n_g)
                    __hip_atomic_fetch_add(word(kBarGlobal), 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(word(kBarGlobal), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < m * ng) {
                    if (__hip_atomic_load(word(kBarErr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        good = 0;
                        break;
                    }
                    if (static_cast<uint64_t>(wall_clock64()) - t0 > D.limit) {
                        __hip_atomic_store(word(kBarErr), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        good = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                // acquire: the other workgroups' writes become visible here
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            ok = good;
            if (blockIdx.x == 0) {   // phase durations as workgroup 0 sees them
                const uint64_t now = wall_clock64();
                D.ticks[(m - 1) % 4] += now - *last;
                *last = now;
            }
        }
        __syncthreads();
        return ok != 0;
    }
};

template <int MODE>
__global__ __launch_bounds__(1024) void k_admm_persistent(const PersistentDev *__restrict__ D,
                                                          PersistentPlan plan) {
    __shared__ uint64_t last;
    if (threadIdx.x == 0) last = wall_clock64();
    PersistentWork<MODE> w{*D, &last};
    persistent_walk(plan, blockIdx.x, gridDim.x, w);
    if (blockIdx.x == 0 && threadIdx.x == 0) D->ticks[4] += wall_clock64() - last;
}

// The same without the objective, four rows per thread (16-byte loads and
// stores; n a multiple of 4 and every array 16-byte aligned).
__global__ __launch_bounds__(kBlock) void k_ratio_combine4(const float *__restrict__ part, int ns,
                                                           int64_t n, const float *__restrict__ y,
                                                           const float *__restrict__ r,
                                                           float *__restrict__ ratio) {
    const int64_t n4 = n >> 2;
    const v4f *p4 = reinterpret_cast<const v4f *>(part);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n4;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        const v4f ri = reinterpret_cast<const v4f *>(r)[i];
        const v4f yi = reinterpret_cast<const v4f *>(y)[i];
        v4f acc = p4[i];
        for (int k = 1; k < ns; ++k) {
            const v4f t = p4[static_cast<int64_t>(k) * n4 + i];
            acc.x += t.x;
            acc.y += t.y;
            acc.z += t.z;
            acc.w += t.w;
        }
        v4f q;
        q.x = yi.x / (acc.x + ri.x);
        q.y = yi.y / (acc.y + ri.y);
        q.z = yi.z / (acc.z + ri.z);
        q.w = yi.w / (acc.w + ri.w);
        reinterpret_cast<v4f *>(ratio)[i] = q;
    }
}

// ratio_i = y_i / (sum_k part[k][i] + r_i), with optional FP64 partials of
// the I-divergence sum_i p_i - y_i + y_i log(y_i / p_i).
template <bool OBJ>
__global__ __launch_bounds__(kBlock) void k_ratio_combine(const float *__restrict__ part, int ns,
                                                          int64_t n, const float *__restrict__ y,
                                                          const float *__restrict__ r,
                                                          float *__restrict__ ratio,
                                                          double *__restrict__ partials) {
    double term = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        float acc = part[i];
        for (int k = 1; k < ns; ++k) acc += part[static_cast<int64_t>(k) * n + i];
        const float p = acc + r[i];
        const float yi = y[i];
        ratio[i] = yi / p;
        if (OBJ) {
            const double pd = p, yd = yi;
            double t = pd - yd;
            if (yd > 0.0) t += yd * log(yd / pd);
            term += t;
        }
    }
    if (OBJ) block_sum_store(term, partials + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_back_combine(const float *__restrict__ part, int ns,
                                                         int64_t n, const float *__restrict__ scale,
                                                         float *__restrict__ e) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock) {
        float acc = part[i];
        for (int k = 1; k < ns; ++k) acc += part[static_cast<int64_t>(k) * n + i];
        e[i] = scale ? acc * scale[i] : acc;
    }
}

// Image update of voxel j from the back-product partial sums (ns slabs of J).
// H0 comes from the array H (full weights) or, for weights constant per
// direction, from the 16-entry table htab by neighbour pattern (the same
// values; the J-float array is not read).
template <int GROUPING, bool WFULL>
__device__ __forceinline__ void voxel_update_elem(int64_t j, const float *__restrict__ part, int ns,
                                                  const float *__restrict__ scale, const float *__restrict__ g,
                                                  float *__restrict__ g_next, float *__restrict__ gs_next,
                                                  const float *__restrict__ v, const float *__restrict__ a,
                                                  const float *__restrict__ sens, const float *__restrict__ H,
                                                  const float *__restrict__ htab, const Grid &grid,
                                                  const Weights &wts, float lam) {
    const int64_t n = grid.J;
    auto e_of = [&]() {
        float e = part[j];
        for (int k = 1; k < ns; ++k) e += part[static_cast<int64_t>(k) * n + j];
        return scale ? e * scale[j] : e;
    };
    const VoxelPos P = voxel_pos(j, grid);
    auto h_of = [&]() { return WFULL ? H[j] : htab[neighbour_mask(grid, P.iy, P.ix)]; };
    const float gnew = voxel_update_at<GROUPING, WFULL>(j, P, e_of, g, v, a, sens, h_of, grid, wts, lam);
    g_next[j] = gnew;
    if (gs_next) gs_next[j] = gnew * scale[j];
}

template <int GROUPING, bool WFULL>
__global__ __launch_bounds__(kBlock) void k_voxel_update(
    const float *__restrict__ part, int ns, const float *__restrict__ scale,
    const float *__restrict__ g, float *__restrict__ g_next, float *__restrict__ gs_next,
    const float *__restrict__ v, const float *__restrict__ a, const float *__restrict__ sens,
    const float *__restrict__ H, const float *__restrict__ htab, Grid grid, Weights wts, float lam) {
    for (int64_t j = static_cast<int64_t>(xcd_block()) * kBlock + threadIdx.x; j < grid.J;
         j += static_cast<int64_t>(gridDim.x) * kBlock)
        voxel_update_elem<GROUPING, WFULL>(j, part, ns, scale, g, g_next, gs_next, v, a, sens, H, htab, grid,
                                           wts, lam);
}

// ---------------------------------------------------------------- row-block epilogues
// The workgroup of one (row block, slab) tile arrives at its row block's
// counter once its partial sums are written; the last of the ns arrivals
// finishes the row block.  Each wave first waits for its own stores, then one
// thread adds the arrival with release semantics at agent scope (the
// workgroup's writes, held in this XCD's L2, become visible device-wide); the
// last arrival then acquires at agent scope (the other slabs' writes become
// visible here) and resets the counter for the next launch.  No workgroup
// waits for another, so the epilogue cannot stall the launch.  flag: one LDS
// word that no thread reads any more.
__device__ __forceinline__ bool last_slab(uint32_t *count, int ns, int *flag) {
    __builtin_amdgcn_s_waitcnt(0);   // this wave's stores have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t old = __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const bool last = old + 1 == static_cast<uint32_t>(ns);
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        *flag = last;
    }
    __syncthreads();
    return *flag != 0;
}

// Forward product, then the ratio y / (A f + r) of the row block's rows (the
// slab sums added in slab order, as launch_ratio_combine).  vec: every
// array 16-byte aligned and n_rows a multiple of 4 (four rows per thread).
template <int VT, int MODE>
__global__ __launch_bounds__(1024) void k_tiled_ratio(TileMap M, const int32_t *__restrict__ pk,
                                                      const typename Code<VT>::T *__restrict__ val,
                                                      const int32_t *__restrict__ goff,
                                                      const int32_t *__restrict__ poff,
                                                      const float *__restrict__ x, float *part,
                                                      RatioEpilogue E, int vec) {
    extern __shared__ float lds[];
    tiled_body<VT, MODE>(M, blockIdx.x, pk, val, goff, poff, x, part);
    const int64_t rb = blockIdx.x / M.ns;
    if (!last_slab(E.count + rb, M.ns, reinterpret_cast<int *>(lds))) return;
    const int64_t rows = static_cast<int64_t>(M.waves) * M.rw, row0 = rb * rows;
    const int64_t end = row0 + rows < M.n_rows ? row0 + rows : M.n_rows;
    const int64_t n = M.n_rows;
    if (vec) {
        const v4f *p4 = reinterpret_cast<const v4f *>(part);
        for (int64_t i = row0 / 4 + threadIdx.x; i < end / 4; i += blockDim.x) {
            const v4f ri = reinterpret_cast<const v4f *>(E.r)[i];
            const v4f yi = reinterpret_cast<const v4f *>(E.y)[i];
            v4f acc = p4[i];
            for (int k = 1; k < M.ns; ++k) {
                const v4f t = p4[static_cast<int64_t>(k) * (n / 4) + i];
                acc.x += t.x;
                acc.y += t.y;
                acc.z += t.z;
                acc.w += t.w;
            }
            v4f q;
            q.x = yi.x / (acc.x + ri.x);
            q.y = yi.y / (acc.y + ri.y);
            q.z = yi.z / (acc.z + ri.z);
            q.w = yi.w / (acc.w + ri.w);
            reinterpret_cast<v4f *>(E.ratio)[i] = q;
        }
    } else {
        for (int64_t i = row0 + threadIdx.x; i < end; i += blockDim.x) {
            float acc = part[i];
            for (int k = 1; k < M.ns; ++k) acc += part[static_cast<int64_t>(k) * n + i];
            E.ratio[i] = E.y[i] / (acc + E.r[i]);
        }
    }
}

// Back product, then the image update of the row block's voxels.
template <int VT, int MODE, int GROUPING, bool WFULL>
__global__ __launch_bounds__(1024) void k_tiled_update(TileMap M, const int32_t *__restrict__ pk,
                                                       const typename Code<VT>::T *__restrict__ val,
                                                       const int32_t *__restrict__ goff,
                                                       const int32_t *__restrict__ poff,
                                                       const float *__restrict__ x, float *part,
                                                       UpdateEpilogue E) {
    extern __shared__ float lds[];
    tiled_body<VT, MODE>(M, blockIdx.x, pk, val, goff, poff, x, part);
    const int64_t rb = blockIdx.x / M.ns;
    if (!last_slab(E.count + rb, M.ns, reinterpret_cast<int *>(lds))) return;
    const int64_t rows = static_cast<int64_t>(M.waves) * M.rw, row0 = rb * rows;
    const int64_t end = row0 + rows < M.n_rows ? row0 + rows : M.n_rows;
    for (int64_t j = row0 + threadIdx.x; j < end; j += blockDim.x)
        voxel_update_elem<GROUPING, WFULL>(j, part, M.ns, E.scale, E.g, E.g_next, E.gs_next, E.v, E.a, E.sens,
                                           E.H, E.htab, E.grid, E.wts, E.lam);
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

static unsigned stride_blocks(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return static_cast<unsigned>(b);
}

// Largest dynamic LDS of one workgroup on gfx950.
constexpr int kMaxLds = 163840;

// Raises a kernel's dynamic-LDS limit once (outside any graph capture that
// may follow: the first launch of a context is never captured); the
// initialisation of a function-local static runs once even when several
// threads launch at the same time.
template <auto KERN>
static hipError_t raise_lds() {
    static const hipError_t raised =
        hipFuncSetAttribute(reinterpret_cast<const void *>(KERN), hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    return raised;
}

// The tiled product's launch: epilogue 0 none, 1 ratio, 2 image update (with
// its grouping and weights as template arguments).
template <int VT, int MODE, int EPI, int GROUPING, bool WFULL>
static hipError_t launch_tiled_t(const TileMap &M, const float *x, float *part, const RatioEpilogue *R,
                                 const UpdateEpilogue *U, hipStream_t st) {
    typedef typename Code<VT>::T T;
    const dim3 grid(static_cast<unsigned>(M.n_rb * M.ns)), block(static_cast<unsigned>(M.waves * kWave));
    const size_t lds = M.lds_bytes();
    const T *val = static_cast<const T *>(M.val);
    if (EPI == 0) {
        if (hipError_t e = raise_lds<&k_tiled<VT, MODE>>()) return e;
        hipLaunchKernelGGL((k_tiled<VT, MODE>), grid, block, lds, st, M, M.pk, val, M.goff, M.poff, x, part);
    } else if (EPI == 1) {
        const auto al = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
        const int vec = M.n_rows % 4 == 0 && al(part) && al(R->y) && al(R->r) && al(R->ratio);
        if (hipError_t e = raise_lds<&k_tiled_ratio<VT, MODE>>()) return e;
        hipLaunchKernelGGL((k_tiled_ratio<VT, MODE>), grid, block, lds, st, M, M.pk, val, M.goff, M.poff, x,
                           part, *R, vec);
    } else {
        if (hipError_t e = raise_lds<&k_tiled_update<VT, MODE, GROUPING, WFULL>>()) return e;
        hipLaunchKernelGGL((k_tiled_update<VT, MODE, GROUPING, WFULL>), grid, block, lds, st, M, M.pk, val,
                           M.goff, M.poff, x, part, *U);
    }
    return hipGetLastError();
}

template <int VT, int EPI, int GROUPING, bool WFULL>
static hipError_t launch_tiled_v(const TileMap &M, const float *x, float *part, const RatioEpilogue *R,
                                 const UpdateEpilogue *U, hipStream_t st) {
    const bool fits = M.cb <= kXPrefetch * 4 * M.waves * kWave;
    if (M.variant == 1) return launch_tiled_t<VT, 1, EPI, GROUPING, WFULL>(M, x, part, R, U, st);
    if (M.variant == 2 && fits) return launch_tiled_t<VT, 2, EPI, GROUPING, WFULL>(M, x, part, R, U, st);
    return launch_tiled_t<VT, 0, EPI, GROUPING, WFULL>(M, x, part, R, U, st);
}

template <int EPI, int GROUPING, bool WFULL>
static hipError_t launch_tiled_e(const TileMap &M, int vt, const float *x, float *part, const RatioEpilogue *R,
                                 const UpdateEpilogue *U, hipStream_t st) {
    if (M.n_rb * M.ns == 0) return hipSuccess;
    if (vt == 0) return launch_tiled_v<0, EPI, GROUPING, WFULL>(M, x, part, R, U, st);
    if (vt == 1) return launch_tiled_v<1, EPI, GROUPING, WFULL>(M, x, part, R, U, st);
    return launch_tiled_v<2, EPI, GROUPING, WFULL>(M, x, part, R, U, st);
}

hipError_t launch_tiled(const TileMap &M, int vt, const float *x, float *part, hipStream_t st) {
    return launch_tiled_e<0, 0, false>(M, vt, x, part, nullptr, nullptr, st);
}

hipError_t launch_tiled_ratio(const TileMap &M, int vt, const float *x, float *part, const RatioEpilogue &E,
                              hipStream_t st) {
    return launch_tiled_e<1, 0, false>(M, vt, x, part, &E, nullptr, st);
}

hipError_t launch_tiled_update(const TileMap &M, int vt, const float *x, float *part, const UpdateEpilogue &E,
                               int grouping, hipStream_t st) {
    const bool wf = E.wts.full != nullptr;
    if (grouping == 0)
        return wf ? launch_tiled_e<2, 0, true>(M, vt, x, part, nullptr, &E, st)
                  : launch_tiled_e<2, 0, false>(M, vt, x, part, nullptr, &E, st);
    return wf ? launch_tiled_e<2, 1, true>(M, vt, x, part, nullptr, &E, st)
              : launch_tiled_e<2, 1, false>(M, vt, x, part, nullptr, &E, st);
}

template <int VT, int MODE>
static hipError_t launch_tiled_batch_t(const BatchTile *tiles, int64_t n_tiles, const TileMap *maps,
                                       const float *const *xs, float *const *parts, int waves,
                                       size_t lds, hipStream_t st) {
    if (hipError_t e = raise_lds<&k_tiled_batch<VT, MODE>>()) return e;
    hipLaunchKernelGGL((k_tiled_batch<VT, MODE>), dim3(static_cast<unsigned>(n_tiles)),
                       dim3(static_cast<unsigned>(waves * kWave)), lds, st, tiles, maps, xs, parts);
    return hipGetLastError();
}

template <int VT>
static hipError_t launch_tiled_batch_v(const BatchTile *tiles, int64_t n_tiles, const TileMap *maps,
                                       const float *const *xs, float *const *parts, int waves, size_t lds,
                                       int variant, hipStream_t st) {
    if (variant == 1) return launch_tiled_batch_t<VT, 1>(tiles, n_tiles, maps, xs, parts, waves, lds, st);
    return launch_tiled_batch_t<VT, 0>(tiles, n_tiles, maps, xs, parts, waves, lds, st);
}

hipError_t launch_tiled_batch(const BatchTile *tiles, int64_t n_tiles, const TileMap *maps,
                              const float *const *xs, float *const *parts, int waves, size_t lds,
                              int variant, int vt, hipStream_t st) {
    if (n_tiles == 0) return hipSuccess;
    if (vt == 1) return launch_tiled_batch_v<1>(tiles, n_tiles, maps, xs, parts, waves, lds, variant, st);
    if (vt == 2) return launch_tiled_batch_v<2>(tiles, n_tiles, maps, xs, parts, waves, lds, variant, st);
    return launch_tiled_batch_v<0>(tiles, n_tiles, maps, xs, parts, waves, lds, variant, st);
}

template <int MODE>
static const void *persistent_fn() {
    return reinterpret_cast<const void *>(&k_admm_persistent<MODE>);
}

hipError_t persistent_grid(int variant, int threads, size_t lds, int *grid, const char **what) {
    const void *fn = variant == 1 ? persistent_fn<1>() : persistent_fn<0>();
    // the dynamic limit leaves room for the kernel's own static LDS (its barrier flag)
    auto raise = [](const void *f) {
        hipFuncAttributes at{};
        hipError_t e = hipFuncGetAttributes(&at, f);
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   kMaxLds - static_cast<int>(at.sharedSizeBytes));
    };
    static const hipError_t r0 = raise(persistent_fn<0>());
    static const hipError_t r1 = raise(persistent_fn<1>());
    *what = "hipFuncGetAttributes / hipFuncSetAttribute";
    if (r0 != hipSuccess) return r0;
    if (r1 != hipSuccess) return r1;
    int dev = 0, cus = 0, per_cu = 0;
    *what = "hipGetDevice";
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    *what = "hipDeviceGetAttribute(multiprocessor count)";
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *what = "hipOccupancyMaxActiveBlocksPerMultiprocessor";
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
    if (e != hipSuccess) return e;
    *what = "occupancy of the persistent kernel (the largest tile's LDS and the kernel's own 16 bytes "
            "must fit the 160 KiB of a CU)";
    if (per_cu < 1 || cus < 1) return hipErrorCooperativeLaunchTooLarge;
    *grid = per_cu * cus;
    return hipSuccess;
}

hipError_t launch_admm_persistent(const PersistentDev *D, const PersistentPlan &plan, size_t lds,
                                  int threads, int variant, int grid, hipStream_t st) {
    const void *fn = variant == 1 ? persistent_fn<1>() : persistent_fn<0>();
    const PersistentDev *a0 = D;
    PersistentPlan a1 = plan;
    void *args[] = {&a0, &a1};
    return hipLaunchCooperativeKernel(fn, dim3(static_cast<unsigned>(grid)), dim3(static_cast<unsigned>(threads)),
                                      args, static_cast<unsigned>(lds), st);
}

hipError_t launch_ratio_combine(const float *part, int ns, int64_t n, const float *y,
                                const float *r, float *ratio, double *partials, bool objective,
                                hipStream_t st, int64_t *n_partials) {
    const unsigned nb = stride_blocks(n) > 4096 ? 4096 : stride_blocks(n);
    if (n_partials) *n_partials = nb;
    if (objective)
        hipLaunchKernelGGL(k_ratio_combine<true>, dim3(nb), dim3(kBlock), 0, st, part, ns, n, y, r,
                           ratio, partials);
    else if (n % 4 == 0 && aligned16(part) && aligned16(y) && aligned16(r) && aligned16(ratio)) {
        const unsigned nb4 = stride_blocks(n / 4) > 4096 ? 4096 : stride_blocks(n / 4);
        hipLaunchKernelGGL(k_ratio_combine4, dim3(nb4), dim3(kBlock), 0, st, part, ns, n, y, r,
                           ratio);
    } else
        hipLaunchKernelGGL(k_ratio_combine<false>, dim3(nb), dim3(kBlock), 0, st, part, ns, n, y,
                           r, ratio, partials);
    return hipGetLastError();
}

hipError_t launch_back_combine(const float *part, int ns, int64_t n, const float *scale,
                               float *e, hipStream_t st) {
    hipLaunchKernelGGL(k_back_combine, dim3(stride_blocks(n)), dim3(kBlock), 0, st, part, ns, n,
                       scale, e);
    return hipGetLastError();
}

hipError_t launch_voxel_update(const float *part, int ns, const float *scale, const float *g,
                               float *g_next, float *gs_next, const float *v, const float *a,
                               const float *sens, const float *H, const float *htab, const Grid &grid,
                               const Weights &w, int grouping, float lam, hipStream_t st) {
    const unsigned nb = stride_blocks(grid.J);
    auto kern = grouping == 0 ? (w.full ? k_voxel_update<0, true> : k_voxel_update<0, false>)
                              : (w.full ? k_voxel_update<1, true> : k_voxel_update<1, false>);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, st, part, ns, scale, g, g_next, gs_next, v,
                       a, sens, H, htab, grid, w, lam);
    return hipGetLastError();
}

}  // namespace sgtv
