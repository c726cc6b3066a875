// Order of work of the persistent batched iteration: one cooperative launch
// runs n ADMM iterations (Section III, Eqs. 4-6) of every scan of a batch,
// each workgroup walking the same sequence of phases with grid-wide barriers
// between dependent ones.  Written for host and device so that the walk can
// be run on CPU threads (every work item once per phase, the same barriers in
// every workgroup) without a GPU.
//
// Iteration k with buffer parities (fc, vc) = (fc0 + k, vc0 + k) mod 2:
//   A  forward tiles (x = f[fc])           and the split blocks of iteration
//      k - 1 (new image f[fc], v from vc ^ 1 to vc): both only read f[fc]
//   |  barrier
//   B  ratio blocks
//   |  barrier
//   C  back tiles
//   |  barrier
//   D  image-update blocks (f[fc] -> f[fc ^ 1], v and a of parity vc)
//   |  barrier
// and after the last iteration the split blocks of that iteration (phase E).
// The split of iteration k - 1 writes (v, a) of parity vc, which the image
// update of iteration k reads after three barriers; it reads (v, a) of parity
// vc ^ 1, last written by the split of iteration k - 2 (phase A of iteration
// k - 1) and read by the image update of iteration k - 1 (before a barrier).
//
// Tiles are handed out through work queues: queue q (q < Nq = min(G, 8))
// holds the tiles t = q (mod Nq) and is served to the workgroups wg = q
// (mod Nq), each taking the next index of the queue's counter when it is free.
// Workgroups are dealt round-robin to the 8 XCDs, so a queue is served by one
// XCD and the tiles of one slab (padded per scan to multiples of 8 in the
// batch tables) stay on it, while the uneven tiles of uneven scans are
// balanced among its workgroups.  The counters of a phase are cleared by
// workgroup 0 two phases later, when no workgroup can still take from them.
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace sgtv {

enum PersistentPhase { kPhaseForward = 0, kPhaseRatio = 1, kPhaseBack = 2, kPhaseVoxel = 3, kPhaseSplit = 4 };

constexpr uint32_t kMaxQueues = 8;

struct PersistentPlan {
    int64_t n_tiles_f, n_tiles_b;     // tiles of the forward and back products
    int64_t n_rblocks, n_vblocks, n_sblocks;   // 256-thread blocks of the elementwise steps
    int n_iters, fcur0, vcur0;
    int quarters;                     // 256-thread blocks per workgroup (waves / 4)
};

// Barriers per launch: four per iteration.
__host__ __device__ inline int64_t persistent_barriers(const PersistentPlan &P) {
    return 4 * static_cast<int64_t>(P.n_iters);
}

__host__ __device__ inline uint32_t persistent_queues(uint32_t G) { return G < kMaxQueues ? G : kMaxQueues; }

// Walks the work of workgroup wg of G for the whole launch.  V provides
//   int64_t grab(int phase, uint32_t queue)    the next index of a queue (from 0)
//   void clear(int phase)                      all queue counters of a phase to 0
//   void tile(int phase, int64_t tile, int fc) a product tile
//   void blocks(int phase, int64_t first, int64_t stride, int64_t n, int fc, int vc)
//        the elementwise blocks first, first + stride, ... below n, per quarter
//        (quarter q of the workgroup starts at first + q)
//   bool barrier(uint32_t target)              false: stop at once
template <class V>
__host__ __device__ inline __attribute__((always_inline)) void persistent_walk(const PersistentPlan &P, uint32_t wg,
                                                                               uint32_t G, V &v) {
    uint32_t target = 0;
    const int64_t first = static_cast<int64_t>(wg) * P.quarters;
    const int64_t stride = static_cast<int64_t>(G) * P.quarters;
    const uint32_t nq = persistent_queues(G), queue = wg % nq;
    for (int k = 0; k < P.n_iters; ++k) {
        const int fc = (P.fcur0 + k) & 1, vc = (P.vcur0 + k) & 1;
        // the four phases A-D; the tiles of A and C go through one call site
        // (a single inlined copy of the tile body)
        for (int step = 0; step < 4; ++step) {
            if (step == 0 || step == 2) {
                const int phase = step == 0 ? kPhaseForward : kPhaseBack;
                const int64_t n = step == 0 ? P.n_tiles_f : P.n_tiles_b;
                for (;;) {
                    const int64_t t = queue + static_cast<int64_t>(nq) * v.grab(phase, queue);
                    if (t >= n) break;
                    v.tile(phase, t, fc);
                }
                // the other product's counters were last taken from two phases ago
                if (wg == 0) v.clear(step == 0 ? kPhaseBack : kPhaseForward);
            }
            if (step == 0 && k > 0) v.blocks(kPhaseSplit, first, stride, P.n_sblocks, fc, vc ^ 1);
            if (step == 1) v.blocks(kPhaseRatio, first, stride, P.n_rblocks, fc, vc);
            if (step == 3) v.blocks(kPhaseVoxel, first, stride, P.n_vblocks, fc, vc);
            target += G;
            if (!v.barrier(target)) return;
        }
    }
    if (P.n_iters > 0) {
        const int k = P.n_iters - 1;
        const int fc = (P.fcur0 + k + 1) & 1, vc = (P.vcur0 + k) & 1;
        v.blocks(kPhaseSplit, first, stride, P.n_sblocks, fc, vc);
    }
}

}  // namespace sgtv
