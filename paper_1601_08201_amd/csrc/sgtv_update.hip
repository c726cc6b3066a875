// Image update and split/dual update in one elementwise-and-stencil pass
// (Section III, Eqs. 4-6): each workgroup owns a tile of tw x th spatial bins
// (all spectral bins) and
//   1. runs the closed-form image update of every hyper-voxel of the tile and
//      of the one-bin ring around it (the four corner bins are not needed),
//      keeping the new image in LDS and writing the tile's own voxels out;
//   2. runs the split and dual update of the tile's groups from that LDS
//      copy (the new image of a group's four neighbour bins is in the ring).
// The ring's new values are computed again by the neighbouring tiles instead
// of being written and read back in a second launch, so the new image and
// the (v, a) state pass through HBM once.  Arithmetic per voxel and per group
// is that of the separate image and split kernels (voxel_update_at, and the
// loop of split_bin over the same values), so the results are bit for bit the
// same.  The curvature H0 comes from a table by neighbour pattern when the
// weights are constant per direction (16 floats instead of a J-float array).
#include "sgtv_device.h"

namespace sgtv {

template <int GROUPING, bool WFULL, int THREADS>
__global__ __launch_bounds__(THREADS) void k_update_fused(FusedUpdate A) {
    extern __shared__ float fl[];   // new image of the tile and its ring: (tw + 2) * (th + 2) bins x Q
    const Grid &gr = A.grid;
    const int Q = gr.Q;
    const int sl = A.seg_log2, G = 1 << sl;
    const int nseg = blockDim.x >> sl;
    const int seg = threadIdx.x >> sl, ls = threadIdx.x & (G - 1);
    const unsigned tile = xcd_block();
    const int ty = static_cast<int>(tile / A.tiles_x), tx = static_cast<int>(tile - ty * A.tiles_x);
    const int rw = A.tw + 2, rh = A.th + 2;
    const int x0 = tx * A.tw - 1, y0 = ty * A.th - 1;   // grid position of ring bin (0, 0)
    const int64_t J = gr.J;

    // 1. image update of the tile and its ring (one segment of G lanes per bin)
    for (int lb = seg; lb < rw * rh; lb += nseg) {
        const int ly = lb / rw, lx = lb - ly * rw;
        const int gx = x0 + lx, gy = y0 + ly;
        const bool corner = (lx == 0 || lx == rw - 1) && (ly == 0 || ly == rh - 1);
        if (corner || gx < 0 || gx >= gr.nx || gy < 0 || gy >= gr.ny) continue;
        const bool own = lx > 0 && lx < rw - 1 && ly > 0 && ly < rh - 1;
        const int64_t s = static_cast<int64_t>(gy) * gr.nx + gx;
        const int mask = neighbour_mask(gr, gy, gx);
        for (int q = ls; q < Q; q += G) {
            const int64_t j = s * Q + q;
            VoxelPos P;
            P.s = s;
            P.q = q;
            P.iy = gy;
            P.ix = gx;
            auto e_of = [&]() {
                float e = A.part[j];
                for (int k = 1; k < A.ns; ++k) e += A.part[static_cast<int64_t>(k) * J + j];
                return A.scale ? e * A.scale[j] : e;
            };
            auto h_of = [&]() { return WFULL ? A.H[j] : A.htab[mask]; };
            const float fn = voxel_update_at<GROUPING, WFULL>(j, P, e_of, A.g, A.v_old, A.a_old, A.sens, h_of, gr,
                                                              A.wts, A.lam);
            fl[lb * Q + q] = fn;
            if (own) {
                A.g_next[j] = fn;
                if (A.gs_next) A.gs_next[j] = fn * A.scale[j];
            }
        }
    }
    __syncthreads();

    // 2. split and dual update of the tile's groups, the new image from LDS
    //    (the arithmetic of split_bin); every lane of a wave takes part in the
    //    segment reduction, so the loop count is the same for all segments
    const int n_own = A.tw * A.th;
    for (int base = 0; base < n_own; base += nseg) {
        const int ob = base + seg;
        const int oy = ob / A.tw, ox = ob - oy * A.tw;
        const int gx = x0 + 1 + ox, gy = y0 + 1 + oy;
        const bool active = ob < n_own && gx < gr.nx && gy < gr.ny;
        float ss = 0.0f;
        int64_t s = 0;
        if (active) {
            s = static_cast<int64_t>(gy) * gr.nx + gx;
            const int lb = (oy + 1) * rw + (ox + 1);
            // neighbour bins in the ring (out of the grid: the bin itself, value replaced by 0)
            const bool in[4] = {gx + 1 < gr.nx, gx > 0, gy + 1 < gr.ny, gy > 0};
            const int nl[4] = {in[0] ? lb + 1 : lb, in[1] ? lb - 1 : lb, in[2] ? lb + rw : lb, in[3] ? lb - rw : lb};
            const float ag = GROUPING == 0 ? A.a_old[s] : 0.0f;
#pragma unroll 2
            for (int q = ls; q < Q; q += G) {
                const float fs = fl[lb * Q + q];
                const float aq = GROUPING == 0 ? ag : A.a_old[s * Q + q];
                float sq = 0.0f;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const float fv = fl[nl[p] * Q + q];
                    const float fn = in[p] ? fv : 0.0f;
                    const int64_t o = (s * 4 + p) * Q + q;
                    const float vo = A.v_old[o];
                    const float c_old = vo - aq * vo;
                    const float vn = fmaf(weight_t<WFULL>(A.wts, gr, s, p, q), fs - fn, c_old);
                    A.v_new[o] = vn;
                    sq = fmaf(vn, vn, sq);
                }
                if (GROUPING == 0) ss += sq;
                else A.a_new[s * Q + q] = shrink_factor(sqrtf(sq), A.thr);
            }
        }
        if (GROUPING == 0) {
            ss = seg_sum(ss, G);
            if (active && ls == 0) A.a_new[s] = shrink_factor(sqrtf(ss), A.thr);
        }
    }
}

size_t fused_lds_bytes(int tw, int th, int Q) {
    return sizeof(float) * static_cast<size_t>(tw + 2) * (th + 2) * Q;
}

template <int THREADS>
static hipError_t launch_fused_t(const FusedUpdate &A, int grouping, size_t lds, unsigned nb, hipStream_t st) {
    const bool wf = A.wts.full != nullptr;
    auto kern = grouping == 0 ? (wf ? k_update_fused<0, true, THREADS> : k_update_fused<0, false, THREADS>)
                              : (wf ? k_update_fused<1, true, THREADS> : k_update_fused<1, false, THREADS>);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(THREADS), lds, st, A);
    return hipGetLastError();
}

hipError_t launch_update_fused(const FusedUpdate &A, int grouping, int threads, hipStream_t st) {
    const size_t lds = fused_lds_bytes(A.tw, A.th, A.grid.Q);
    const int tiles_y = (A.grid.ny + A.th - 1) / A.th;
    const unsigned nb = static_cast<unsigned>(A.tiles_x) * tiles_y;
    if (nb == 0) return hipSuccess;
    if (lds > static_cast<size_t>(kFusedMaxLds)) return hipErrorInvalidValue;
    if (threads == 256) return launch_fused_t<256>(A, grouping, lds, nb, st);
    if (threads == 1024) return launch_fused_t<1024>(A, grouping, lds, nb, st);
    return launch_fused_t<512>(A, grouping, lds, nb, st);
}

}  // namespace sgtv
