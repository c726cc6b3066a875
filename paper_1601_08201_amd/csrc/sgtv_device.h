// Device helpers shared by the kernels of the ADMM iteration.
#pragma once

#include "sgtv_kernels.h"

namespace sgtv {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned short v4u16 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- value codes
template <int VT> struct Code;
template <> struct Code<0> {
    typedef float T;
    typedef v4f V4;
    static __device__ __forceinline__ float dec(float a) { return a; }
};
template <> struct Code<1> {   // bfloat16: upper half of an FP32 word
    typedef unsigned short T;
    typedef v4u16 V4;
    static __device__ __forceinline__ float dec(unsigned short a) {
        return __uint_as_float(static_cast<unsigned>(a) << 16);
    }
};
template <> struct Code<2> {   // IEEE binary16
    typedef unsigned short T;
    typedef v4u16 V4;
    static __device__ __forceinline__ float dec(unsigned short a) {
        return static_cast<float>(__builtin_bit_cast(_Float16, a));
    }
};

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ float seg_sum(float v, int width) {
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double seg_sum(double v, int width) {
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum of one double per thread over the block, written by thread 0.
__device__ __forceinline__ void block_sum_store(double v, double *out) {
    __shared__ double sh[kBlock / kWave];
    v = wave_sum(v);
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += sh[w];
        *out = s;
    }
}

// ---------------------------------------------------------------- block order
// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  This
// renumbers them so that the workgroups of one XCD cover one contiguous range
// of the grid: stencil neighbours (the next spatial bin, the next grid row)
// are then read through the same L2 instead of being fetched again by another
// XCD.  A bijection of [0, gridDim.x) for any grid size.  Used by the
// single-scan image and split updates; the batched ones, whose grids are
// twenty times longer, run faster in dispatch order.
constexpr unsigned kXcds = 8;

__device__ __forceinline__ unsigned xcd_block() {
    const unsigned n = gridDim.x, b = blockIdx.x;
    const unsigned x = b % kXcds, k = b / kXcds, q = n / kXcds, r = n % kXcds;
    return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------- geometry
__device__ __forceinline__ int64_t neighbour(const Grid &g, int64_t s, int iy, int ix, int p) {
    switch (p) {
    case 0: return ix + 1 < g.nx ? s + 1 : -1;
    case 1: return ix > 0 ? s - 1 : -1;
    case 2: return iy + 1 < g.ny ? s + g.nx : -1;
    default: return iy > 0 ? s - g.nx : -1;
    }
}

__device__ __forceinline__ float weight(const Weights &w, const Grid &g, int64_t s, int p, int q) {
    return w.full ? w.full[(s * 4 + p) * g.Q + q] : w.w[p];
}

// The same with the kind of weights fixed at compile time (no branch).
template <bool WFULL>
__device__ __forceinline__ float weight_t(const Weights &w, const Grid &g, int64_t s, int p, int q) {
    return WFULL ? w.full[(s * 4 + p) * g.Q + q] : w.w[p];
}

// Spatial bin s = j / Q, spectral bin q and grid position (iy, ix) of
// hyper-voxel j, with 32-bit divisions: J < 2^31 is checked when the system
// is set.
struct VoxelPos {
    int64_t s;
    int q, iy, ix;
};

__device__ __forceinline__ VoxelPos voxel_pos(int64_t j, const Grid &g) {
    const uint32_t jj = static_cast<uint32_t>(j);
    const uint32_t Q = static_cast<uint32_t>(g.Q), nx = static_cast<uint32_t>(g.nx);
    const uint32_t s = jj / Q, iy = s / nx;
    VoxelPos r;
    r.s = s;
    r.q = static_cast<int>(jj - s * Q);
    r.iy = static_cast<int>(iy);
    r.ix = static_cast<int>(s - iy * nx);
    return r;
}

// Nonnegative root of H t^2 + B t - C = 0, C >= 0, H > 0; branch chosen so
// neither form subtracts nearly equal numbers.
__device__ __forceinline__ float voxel_root(float H, float B, float C) {
    float disc = sqrtf(fmaf(B, B, 4.0f * H * C));
    return B <= 0.0f ? (disc - B) / (2.0f * H) : (2.0f * C) / (B + disc);
}

// Image update of one hyper-voxel j = (s, q) (Section III, Eq. 4, optimisation
// transfer): with e = (A^T ratio)_j,
//   gamma = lam * (D^T t)_j, t = w.*G g - d + c = w.*G g + v - 2 a v   (z = d - c)
//   B = sens_j + gamma - lam H0_j g_j,  C = g_j e
// the new value is the nonnegative root of (lam H0_j) t^2 + B t - C.
// Every load is issued whatever the position of the voxel: a neighbour outside
// the grid reads the voxel's own bin and its terms are then discarded, so the
// loads need no branches.  e = (A^T ratio)_j comes from the callable E, called
// after the stencil loads are issued so that its own loads overlap them.
// The same at a known position, with the curvature H0_j from the callable HF
// (the array H or the table of the neighbour pattern), read where H[j] is.
template <int GROUPING, bool WFULL, class E, class HF>
__device__ __forceinline__ float voxel_update_at(int64_t j, const VoxelPos &P, E e_of, const float *__restrict__ g,
                                                 const float *__restrict__ v,
                                                 const float *__restrict__ a,
                                                 const float *__restrict__ sens, HF h_of,
                                                 const Grid &grid, const Weights &wts, float lam) {
    const int Q = grid.Q;
    const int64_t s = P.s;
    const int q = P.q;
    const float gs = g[j];
    const float as = GROUPING == 0 ? a[s] : a[j];
    float dt = 0.0f;   // (D^T t)_j
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int64_t nb = neighbour(grid, s, P.iy, P.ix, p);
        const bool in = nb >= 0;
        const int64_t nc = in ? nb : s;
        const float gl = g[nc * Q + q];
        const float gn = in ? gl : 0.0f;
        const float wp = weight_t<WFULL>(wts, grid, s, p, q);
        const float vs = v[(s * 4 + p) * Q + q];
        const float ds = as * vs;
        dt = fmaf(wp, fmaf(wp, gs - gn, vs - 2.0f * ds), dt);
        const int pb = p ^ 1;   // direction from the neighbour back to s
        const float wn = weight_t<WFULL>(wts, grid, nc, pb, q);
        const float vn = v[(nc * 4 + pb) * Q + q];
        const float an = GROUPING == 0 ? a[nc] : a[nc * Q + q];
        const float dn = an * vn;
        const float dtn = fmaf(-wn, fmaf(wn, gn - gs, vn - 2.0f * dn), dt);
        dt = in ? dtn : dt;
    }
    const float h = lam * h_of();
    const float B = sens[j] + lam * dt - h * gs;
    const float C = gs * e_of();
    return voxel_root(h, B, C);
}

template <int GROUPING, bool WFULL, class E>
__device__ __forceinline__ float voxel_update_value(int64_t j, E e_of, const float *__restrict__ g,
                                                    const float *__restrict__ v,
                                                    const float *__restrict__ a,
                                                    const float *__restrict__ sens,
                                                    const float *__restrict__ H, const Grid &grid,
                                                    const Weights &wts, float lam) {
    const VoxelPos P = voxel_pos(j, grid);
    return voxel_update_at<GROUPING, WFULL>(j, P, e_of, g, v, a, sens, [&]() { return H[j]; }, grid, wts, lam);
}

// Neighbour pattern of a spatial bin: bit p set when the neighbour in
// direction p (+x, -x, +y, -y) lies inside the grid.  The curvature H0 of a
// voxel depends only on it when the weights are constant per direction.
__device__ __forceinline__ int neighbour_mask(const Grid &g, int iy, int ix) {
    return (ix + 1 < g.nx ? 1 : 0) | (ix > 0 ? 2 : 0) | (iy + 1 < g.ny ? 4 : 0) | (iy > 0 ? 8 : 0);
}

__device__ __forceinline__ float shrink_factor(float nrm, float thr) {
    return nrm > thr ? 1.0f - thr / nrm : 0.0f;
}

// Split and dual update of spatial bin s by a segment of 2^seg_log2 lanes
// (lane ls strides over q): v_new = w.*G f + c_old, c_old = v_old - a_old v_old,
// then the shrink factor of the group (Eq. 5).  Every lane of the wave must
// call this (the segment reduction shuffles), with active = false for bins
// past the end.
template <int GROUPING, bool WFULL>
__device__ __forceinline__ void split_bin(int64_t s, bool active, int ls, int seg_log2,
                                          const float *__restrict__ f,
                                          const float *__restrict__ v_old,
                                          const float *__restrict__ a_old,
                                          float *__restrict__ v_new, float *__restrict__ a_new,
                                          const Grid &grid, const Weights &wts, float thr) {
    const int G = 1 << seg_log2;
    const int Q = grid.Q;
    float ss = 0.0f;
    if (active) {
        // 32-bit division: J < 2^31 is checked when the system is set
        const uint32_t s32 = static_cast<uint32_t>(s), nx = static_cast<uint32_t>(grid.nx);
        const uint32_t y = s32 / nx;
        const int iy = static_cast<int>(y);
        const int ix = static_cast<int>(s32 - y * nx);
        // a neighbour outside the grid reads the bin itself; its value is then
        // replaced by 0, so the loads need no branches
        int64_t nc[4];
        bool in[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int64_t nb = neighbour(grid, s, iy, ix, p);
            in[p] = nb >= 0;
            nc[p] = in[p] ? nb : s;
        }
        const float ag = GROUPING == 0 ? a_old[s] : 0.0f;
#pragma unroll 2
        for (int q = ls; q < Q; q += G) {
            const float fs = f[s * Q + q];
            const float aq = GROUPING == 0 ? ag : a_old[s * Q + q];
            float sq = 0.0f;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const float fl = f[nc[p] * Q + q];
                const float fn = in[p] ? fl : 0.0f;
                const int64_t o = (s * 4 + p) * Q + q;
                const float vo = v_old[o];
                const float c_old = vo - aq * vo;
                const float vn = fmaf(weight_t<WFULL>(wts, grid, s, p, q), fs - fn, c_old);
                v_new[o] = vn;
                sq = fmaf(vn, vn, sq);
            }
            if (GROUPING == 0) ss += sq;
            else a_new[s * Q + q] = shrink_factor(sqrtf(sq), thr);
        }
    }
    if (GROUPING == 0) {
        ss = seg_sum(ss, G);
        if (active && ls == 0) a_new[s] = shrink_factor(sqrtf(ss), thr);
    }
}

// ---------------------------------------------------------------- batched elements
// One element of the batched elementwise steps, on scan S with the image and
// split buffers of parity fcur / vcur (the arithmetic of the single-scan
// kernels, so a scan of a batch reproduces its own run bit for bit).

// ratio_i = y_i / (sum of the forward partials + r_i)
__device__ __forceinline__ void batch_ratio_elem(const ScanDev &S, int64_t i) {
    if (i >= S.I) return;
    float acc = S.fpart[i];
    for (int k = 1; k < S.ns_f; ++k) acc += S.fpart[static_cast<int64_t>(k) * S.I + i];
    const float p = acc + S.r[i];
    S.ratio[i] = S.y[i] / p;
}

// image update of hyper-voxel j: reads f[fcur], writes f[fcur ^ 1] (and, for
// 16-bit values, the scaled copy fs); the arithmetic of the single-scan image
// update (the same H0 source: the table unless the weights are full)
__device__ __forceinline__ void batch_voxel_elem(const ScanDev &S, int64_t j, int fcur, int vcur) {
    if (j >= S.grid.J) return;
    auto e = [&]() {
        float s = S.bpart[j];
        for (int k = 1; k < S.ns_b; ++k) s += S.bpart[static_cast<int64_t>(k) * S.grid.J + j];
        return S.scale ? s * S.scale[j] : s;
    };
    const float *g = S.f[fcur], *v = S.v[vcur], *a = S.a[vcur];
    const VoxelPos P = voxel_pos(j, S.grid);
    auto h = [&]() { return S.wts.full ? S.H[j] : S.htab[neighbour_mask(S.grid, P.iy, P.ix)]; };
    float gnew;
    if (S.grouping == 0)
        gnew = S.wts.full ? voxel_update_at<0, true>(j, P, e, g, v, a, S.sens, h, S.grid, S.wts, S.lam)
                          : voxel_update_at<0, false>(j, P, e, g, v, a, S.sens, h, S.grid, S.wts, S.lam);
    else
        gnew = S.wts.full ? voxel_update_at<1, true>(j, P, e, g, v, a, S.sens, h, S.grid, S.wts, S.lam)
                          : voxel_update_at<1, false>(j, P, e, g, v, a, S.sens, h, S.grid, S.wts, S.lam);
    S.f[fcur ^ 1][j] = gnew;
    if (S.fs) S.fs[j] = gnew * S.scale[j];
}

// split and dual update of the 256-thread block that starts at spatial bin s0
// (one segment of 2^seg_log2 lanes per bin; t = thread within the block): the
// new image is f[fcur], (v, a) is read from parity vcur and written to vcur ^ 1.
// Every lane of the calling waves must take part (segment shuffles).
__device__ __forceinline__ void batch_split_block(const ScanDev &S, int64_t s0, int t, int fcur, int vcur) {
    const int sl = S.seg_log2;
    const int64_t s = s0 + (t >> sl);
    const int ls = t & ((1 << sl) - 1);
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

// Split state that makes image f a fixed point of the split update: with
// d = w.*G f and thr = beta / rho, the scaled dual satisfying the optimality
// condition of Eq. 5 is c_g = thr d_g / ||d_g|| on every group g with d_g != 0
// (0 otherwise).  Stored as v = d + c = d (1 + thr / ||d_g||) and
// a = ||d_g|| / (||d_g|| + thr), so that shrink(v) = a v = d.
template <int GROUPING>
__device__ __forceinline__ void consistent_bin(int64_t s, bool active, int ls, int seg_log2,
                                               const float *__restrict__ f, float *__restrict__ v,
                                               float *__restrict__ a, const Grid &grid,
                                               const Weights &wts, float thr) {
    const int G = 1 << seg_log2;
    const int Q = grid.Q;
    float ss = 0.0f;
    int iy = 0, ix = 0;
    int64_t nb[4] = {-1, -1, -1, -1};
    if (active) {
        iy = static_cast<int>(s / grid.nx);
        ix = static_cast<int>(s - static_cast<int64_t>(iy) * grid.nx);
#pragma unroll
        for (int p = 0; p < 4; ++p) nb[p] = neighbour(grid, s, iy, ix, p);
        for (int q = ls; q < Q; q += G) {
            const float fs = f[s * Q + q];
            float sq = 0.0f;
            float d[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const float fn = nb[p] >= 0 ? f[nb[p] * Q + q] : 0.0f;
                d[p] = weight(wts, grid, s, p, q) * (fs - fn);
                sq = fmaf(d[p], d[p], sq);
            }
            if (GROUPING == 0) {
                ss += sq;
            } else {
                const float nrm = sqrtf(sq);
                const float scale = nrm > 0.0f ? 1.0f + thr / nrm : 0.0f;
#pragma unroll
                for (int p = 0; p < 4; ++p) v[(s * 4 + p) * Q + q] = d[p] * scale;
                a[s * Q + q] = nrm > 0.0f ? nrm / (nrm + thr) : 0.0f;
            }
        }
    }
    if (GROUPING == 0) {
        ss = seg_sum(ss, G);
        const float nrm = sqrtf(ss);
        if (active) {
            const float scale = nrm > 0.0f ? 1.0f + thr / nrm : 0.0f;
            for (int q = ls; q < Q; q += G) {
                const float fs = f[s * Q + q];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const float fn = nb[p] >= 0 ? f[nb[p] * Q + q] : 0.0f;
                    v[(s * 4 + p) * Q + q] = weight(wts, grid, s, p, q) * (fs - fn) * scale;
                }
            }
            if (ls == 0) a[s] = nrm > 0.0f ? nrm / (nrm + thr) : 0.0f;
        }
    }
}

}  // namespace sgtv
