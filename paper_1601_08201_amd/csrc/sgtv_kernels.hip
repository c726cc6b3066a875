// CDNA4 (gfx950) kernels of one ADMM iteration for spectrally grouped TV
// reconstruction (Section III, Eqs. 4-6):
//   forward_ratio : p = A f + r, ratio = y / p (+ FP64 I-divergence partials)
//   back_update   : e = A^T ratio, then the closed-form nonnegative root of the
//                   separable surrogate per hyper-voxel (image update, Eq. 4)
//   split_update  : v = w.*G f + c, group 2-norm, block soft-threshold factor
//                   (split update, Eq. 5) and the dual c = v - d (Eq. 6),
//                   kept implicitly as (v, a) with d = a v
//   report        : FP64 TV, primal and dual residual partials
// The matrix is held twice in sliced-ELL form (64 lines per slice, one lane
// per line, 4 entries per lane per 16-byte load): row slices for A f and
// column slices for A^T t, so neither product needs atomics and every sum has
// a fixed order.
#include "sgtv_device.h"

namespace sgtv {

// ---------------------------------------------------------------- A f, ratio
// One wavefront per row slice; lane l owns row 64k + l and walks its padded
// entries four at a time with 16-byte index loads.
template <int VT, bool OBJ>
__global__ __launch_bounds__(kBlock) void k_forward_ratio(
    const int64_t *__restrict__ sptr, const int32_t *__restrict__ idx,
    const typename Code<VT>::T *__restrict__ val, const float *__restrict__ x,
    const float *__restrict__ y, const float *__restrict__ r, float *__restrict__ ratio,
    double *__restrict__ part, int64_t n_rows, int64_t n_slices) {
    typedef typename Code<VT>::V4 V4;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t slice = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    double term = 0.0;
    if (slice < n_slices) {
        const int64_t beg = sptr[slice];
        const int64_t steps = (sptr[slice + 1] - beg) / (kWave * kDepth);
        const v4i *ip = reinterpret_cast<const v4i *>(idx + beg) + lane;
        const V4 *vp = reinterpret_cast<const V4 *>(val + beg) + lane;
        float acc = 0.0f;
        for (int64_t t = 0; t < steps; ++t) {
            const v4i c = __builtin_nontemporal_load(ip + t * kWave);
            const V4 a = __builtin_nontemporal_load(vp + t * kWave);
            acc = fmaf(Code<VT>::dec(a.x), x[c.x], acc);
            acc = fmaf(Code<VT>::dec(a.y), x[c.y], acc);
            acc = fmaf(Code<VT>::dec(a.z), x[c.z], acc);
            acc = fmaf(Code<VT>::dec(a.w), x[c.w], acc);
        }
        const int64_t row = slice * kWave + lane;
        if (row < n_rows) {
            const float p = acc + r[row];
            const float yi = y[row];
            ratio[row] = yi / p;
            if (OBJ) {
                const double pd = p, yd = yi;
                term = pd - yd;
                if (yd > 0.0) term += yd * log(yd / pd);
            }
        }
    }
    if (OBJ) block_sum_store(term, part + blockIdx.x);
}

// ---------------------------------------------------------------- A^T t
template <int VT>
__device__ __forceinline__ float column_dot(const int64_t *__restrict__ sptr,
                                            const int32_t *__restrict__ idx,
                                            const typename Code<VT>::T *__restrict__ val,
                                            const float *__restrict__ t, int64_t slice, int lane) {
    typedef typename Code<VT>::V4 V4;
    const int64_t beg = sptr[slice];
    const int64_t steps = (sptr[slice + 1] - beg) / (kWave * kDepth);
    const v4i *ip = reinterpret_cast<const v4i *>(idx + beg) + lane;
    const V4 *vp = reinterpret_cast<const V4 *>(val + beg) + lane;
    float acc = 0.0f;
    for (int64_t k = 0; k < steps; ++k) {
        const v4i c = __builtin_nontemporal_load(ip + k * kWave);
        const V4 a = __builtin_nontemporal_load(vp + k * kWave);
        acc = fmaf(Code<VT>::dec(a.x), t[c.x], acc);
        acc = fmaf(Code<VT>::dec(a.y), t[c.y], acc);
        acc = fmaf(Code<VT>::dec(a.z), t[c.z], acc);
        acc = fmaf(Code<VT>::dec(a.w), t[c.w], acc);
    }
    return acc;
}

template <int VT>
__global__ __launch_bounds__(kBlock) void k_back(const int64_t *__restrict__ sptr,
                                                 const int32_t *__restrict__ idx,
                                                 const typename Code<VT>::T *__restrict__ val,
                                                 const float *__restrict__ scale,
                                                 const float *__restrict__ t,
                                                 float *__restrict__ e, int64_t n_cols,
                                                 int64_t n_slices) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t slice = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    if (slice >= n_slices) return;
    float acc = column_dot<VT>(sptr, idx, static_cast<const typename Code<VT>::T *>(val), t, slice, lane);
    const int64_t j = slice * kWave + lane;
    if (j < n_cols) e[j] = VT == 0 ? acc : acc * scale[j];
}

// Backprojection of the ratio fused with the image update of one surrogate
// sweep.  For voxel j = (s, q):
//   e     = (A^T ratio)_j
//   gamma = lam * (D^T t)_j, t = D g - d + c = D g + v - 2 a v   (z = d - c)
//   B     = sens_j + gamma - H_j g_j,   C = g_j e
//   g'_j  = nonnegative root of H t^2 + B t - C
template <int VT, int GROUPING>
__global__ __launch_bounds__(kBlock) void k_back_update(
    const int64_t *__restrict__ sptr, const int32_t *__restrict__ idx,
    const typename Code<VT>::T *__restrict__ val, const float *__restrict__ scale,
    const float *__restrict__ ratio, const float *__restrict__ g, float *__restrict__ g_next,
    float *__restrict__ gs_next, const float *__restrict__ v, const float *__restrict__ a,
    const float *__restrict__ sens, const float *__restrict__ H, Grid grid, Weights wts,
    float lam, int64_t n_slices) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t slice = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    if (slice >= n_slices) return;
    float e = column_dot<VT>(sptr, idx, val, ratio, slice, lane);
    const int64_t j = slice * kWave + lane;
    if (j >= grid.J) return;
    if (VT != 0) e *= scale[j];
    auto e_of = [e]() { return e; };
    const float gnew = wts.full
        ? voxel_update_value<GROUPING, true>(j, e_of, g, v, a, sens, H, grid, wts, lam)
        : voxel_update_value<GROUPING, false>(j, e_of, g, v, a, sens, H, grid, wts, lam);
    g_next[j] = gnew;
    if (VT != 0) gs_next[j] = gnew * scale[j];
}

// ---------------------------------------------------------------- split + dual
// Segments of G = 2^seg_log2 lanes per spatial bin; lanes stride over q.
// v_new = w.*G f + c_old with c_old = v_old - a_old v_old; then the shrink
// factor of the group.  Spectral grouping reduces over the segment; the
// standard grouping keeps one factor per (s, q).
template <int GROUPING, bool WFULL>
__global__ __launch_bounds__(kBlock) void k_split_update(
    const float *__restrict__ f, const float *__restrict__ v_old, const float *__restrict__ a_old,
    float *__restrict__ v_new, float *__restrict__ a_new, Grid grid, Weights wts, float thr,
    int seg_log2) {
    const int64_t s = static_cast<int64_t>(xcd_block()) * (kBlock >> seg_log2) + (threadIdx.x >> seg_log2);
    const int ls = threadIdx.x & ((1 << seg_log2) - 1);
    split_bin<GROUPING, WFULL>(s, s < grid.S, ls, seg_log2, f, v_old, a_old, v_new, a_new, grid, wts,
                               thr);
}

template <int GROUPING>
__global__ __launch_bounds__(kBlock) void k_consistent_split(const float *__restrict__ f,
                                                             float *__restrict__ v,
                                                             float *__restrict__ a, Grid grid,
                                                             Weights wts, float thr, int seg_log2) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * (kBlock >> seg_log2) + (threadIdx.x >> seg_log2);
    const int ls = threadIdx.x & ((1 << seg_log2) - 1);
    consistent_bin<GROUPING>(s, s < grid.S, ls, seg_log2, f, v, a, grid, wts, thr);
}

// ---------------------------------------------------------------- report
// FP64 partials per block: [0] R(w.*G f), [1] ||w.*G f - d||^2,
// [2] ||(w.*G)^T (d - d_prev)||^2 with d = a v, d_prev = a_prev v_prev,
// [3] ||w.*G f||^2, [4] ||d||^2, [5] ||(w.*G)^T c||^2 with c = v - d (the
// norms of the residual stopping rule).
template <int GROUPING>
__global__ __launch_bounds__(kBlock) void k_report(
    const float *__restrict__ f, const float *__restrict__ v, const float *__restrict__ a,
    const float *__restrict__ v_prev, const float *__restrict__ a_prev, Grid grid, Weights wts,
    int seg_log2, double *__restrict__ part, int64_t n_blocks) {
    const int G = 1 << seg_log2;
    const int64_t s = static_cast<int64_t>(blockIdx.x) * (kBlock >> seg_log2) + (threadIdx.x >> seg_log2);
    const int ls = threadIdx.x & (G - 1);
    const int Q = grid.Q;
    double tv = 0.0, grp = 0.0, rp = 0.0, rd = 0.0, gf2 = 0.0, d2 = 0.0, tc2 = 0.0;
    if (s < grid.S) {
        const int iy = static_cast<int>(s / grid.nx), ix = static_cast<int>(s - static_cast<int64_t>(iy) * grid.nx);
        int64_t nb[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) nb[p] = neighbour(grid, s, iy, ix, p);
        for (int q = ls; q < Q; q += G) {
            const float fs = f[s * Q + q];
            const float as = GROUPING == 0 ? a[s] : a[s * Q + q];
            const float aps = GROUPING == 0 ? a_prev[s] : a_prev[s * Q + q];
            double sq = 0.0, dual = 0.0, tc = 0.0;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const float fn = nb[p] >= 0 ? f[nb[p] * Q + q] : 0.0f;
                const float wp = weight(wts, grid, s, p, q);
                const float df = wp * (fs - fn);
                const int64_t o = (s * 4 + p) * Q + q;
                const float vo = v[o];
                const float d = as * vo;
                const double pr = static_cast<double>(df) - d;
                sq += static_cast<double>(df) * df;
                rp += pr * pr;
                d2 += static_cast<double>(d) * d;
                dual += static_cast<double>(wp) * (static_cast<double>(d) - static_cast<double>(aps * v_prev[o]));
                tc += static_cast<double>(wp) * static_cast<double>(vo - d);
                if (nb[p] >= 0) {
                    const int pb = p ^ 1;
                    const int64_t o2 = (nb[p] * 4 + pb) * Q + q;
                    const float an = GROUPING == 0 ? a[nb[p]] : a[nb[p] * Q + q];
                    const float apn = GROUPING == 0 ? a_prev[nb[p]] : a_prev[nb[p] * Q + q];
                    const float wn = weight(wts, grid, nb[p], pb, q);
                    const float v2 = v[o2];
                    dual -= static_cast<double>(wn) *
                            (static_cast<double>(an * v2) - static_cast<double>(apn * v_prev[o2]));
                    tc -= static_cast<double>(wn) * static_cast<double>(v2 - an * v2);
                }
            }
            rd += dual * dual;
            tc2 += tc * tc;
            gf2 += sq;
            if (GROUPING == 0) grp += sq;
            else tv += sqrt(sq);
        }
    }
    if (GROUPING == 0) {
        grp = seg_sum(grp, G);
        if (s < grid.S && ls == 0) tv = sqrt(grp);
    }
    block_sum_store(tv, part + blockIdx.x);
    __syncthreads();
    block_sum_store(rp, part + n_blocks + blockIdx.x);
    __syncthreads();
    block_sum_store(rd, part + 2 * n_blocks + blockIdx.x);
    __syncthreads();
    block_sum_store(gf2, part + 3 * n_blocks + blockIdx.x);
    __syncthreads();
    block_sum_store(d2, part + 4 * n_blocks + blockIdx.x);
    __syncthreads();
    block_sum_store(tc2, part + 5 * n_blocks + blockIdx.x);
}

// Penalty change lam -> lam / t with the unscaled dual lam c kept: c <- t c,
// d unchanged.  Per group, m = a + t (1 - a) > 0; v <- m v, then a <- a / m.
template <int GROUPING>
__global__ void k_rescale_v(float *__restrict__ v, const float *__restrict__ a, Grid grid, float t) {
    const int64_t n = grid.J * 4;
    for (int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; o < n;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t s = o / (4 * static_cast<int64_t>(grid.Q));
        const int64_t gidx = GROUPING == 0 ? s : s * grid.Q + o % grid.Q;
        const float ag = a[gidx];
        v[o] *= ag + t * (1.0f - ag);
    }
}

__global__ void k_rescale_a(float *__restrict__ a, int64_t n, float t) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float ag = a[i];
        a[i] = ag / (ag + t * (1.0f - ag));
    }
}

// ---------------------------------------------------------------- small kernels
// Fixed-order final reduction: out[q] = sum_b part[q * n + b].
__global__ __launch_bounds__(kBlock) void k_reduce(const double *__restrict__ part, int64_t n,
                                                   double *__restrict__ out) {
    const int qi = blockIdx.x;
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < n; b += kBlock) acc += part[qi * n + b];
    block_sum_store(acc, out + qi);
}

__global__ __launch_bounds__(kBlock) void k_sum_f32(const float *__restrict__ a, int64_t n,
                                                    double *__restrict__ part) {
    double acc = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kBlock)
        acc += a[i];
    block_sum_store(acc, part + blockIdx.x);
}

__global__ void k_fill_ratio(const double *__restrict__ num, const double *__restrict__ den,
                             float *__restrict__ out, int64_t n) {
    const double d = *den;
    const float val = d > 0.0 ? static_cast<float>(*num / d) : 0.0f;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        out[i] = val;
}

__global__ void k_scale(const float *__restrict__ x, const float *__restrict__ s,
                        float *__restrict__ out, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        out[i] = x[i] * s[i];
}

__global__ void k_div_safe(const float *__restrict__ num, const float *__restrict__ den,
                           float *__restrict__ out, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        out[i] = den[i] > 0.0f ? num[i] / den[i] : 0.0f;
}

__global__ void k_split_from_state(const float *__restrict__ v, const float *__restrict__ a,
                                   float *__restrict__ d, float *__restrict__ c, Grid grid,
                                   int grouping) {
    const int64_t n = grid.J * 4;
    for (int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; o < n;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t s = o / (4 * grid.Q);
        const int q = static_cast<int>(o % grid.Q);
        const float av = grouping == 0 ? a[s] : a[s * grid.Q + q];
        const float dv = av * v[o];
        if (d) d[o] = dv;
        if (c) c[o] = v[o] - dv;
    }
}

__global__ void k_check_range(const float *__restrict__ x, int64_t n, float lo, int strict_lo,
                              float hi, int *__restrict__ flag) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const float t = x[i];
        const bool ok = (strict_lo ? t > lo : t >= lo) && t <= hi;   // false for NaN
        if (!ok) *flag = 1;
    }
}

// ---------------------------------------------------------------- launchers
static inline unsigned blocks_for(int64_t n, int64_t per_block) {
    return static_cast<unsigned>((n + per_block - 1) / per_block);
}

static inline unsigned grid_stride_blocks(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return static_cast<unsigned>(b);
}

static inline int seg_log2_for(int Q) {
    int l = 0;
    while ((1 << l) < Q && l < 6) ++l;
    return l;
}

hipError_t launch_forward_ratio(const Sell &A, int vt, const float *x, const float *y,
                                const float *r, float *ratio, double *partials, bool objective,
                                hipStream_t st, int64_t *n_partials) {
    const unsigned nb = blocks_for(A.n_slices, kBlock / kWave);
    if (n_partials) *n_partials = nb;
    if (nb == 0) return hipSuccess;
#define SGTV_FWD(VT, OBJ)                                                                          \
    hipLaunchKernelGGL((k_forward_ratio<VT, OBJ>), dim3(nb), dim3(kBlock), 0, st, A.sptr, A.idx,   \
                       static_cast<const typename Code<VT>::T *>(A.val), x, y, r, ratio, partials, \
                       A.n_lines, A.n_slices)
    if (vt == 0) { if (objective) SGTV_FWD(0, true); else SGTV_FWD(0, false); }
    else if (vt == 1) { if (objective) SGTV_FWD(1, true); else SGTV_FWD(1, false); }
    else { if (objective) SGTV_FWD(2, true); else SGTV_FWD(2, false); }
#undef SGTV_FWD
    return hipGetLastError();
}

hipError_t launch_back(const Sell &At, int vt, const float *t, float *e, hipStream_t st) {
    const unsigned nb = blocks_for(At.n_slices, kBlock / kWave);
    if (nb == 0) return hipSuccess;
#define SGTV_BACK(VT)                                                                              \
    hipLaunchKernelGGL((k_back<VT>), dim3(nb), dim3(kBlock), 0, st, At.sptr, At.idx,               \
                       static_cast<const typename Code<VT>::T *>(At.val), At.scale, t, e,          \
                       At.n_lines, At.n_slices)
    if (vt == 0) SGTV_BACK(0);
    else if (vt == 1) SGTV_BACK(1);
    else SGTV_BACK(2);
#undef SGTV_BACK
    return hipGetLastError();
}

hipError_t launch_back_update(const Sell &At, int vt, const float *ratio, const float *g,
                              float *g_next, float *gs_next, const float *v, const float *a,
                              const float *sens, const float *H, const Grid &grid,
                              const Weights &w, int grouping, float lam, hipStream_t st) {
    const unsigned nb = blocks_for(At.n_slices, kBlock / kWave);
    if (nb == 0) return hipSuccess;
#define SGTV_BU(VT, GR)                                                                            \
    hipLaunchKernelGGL((k_back_update<VT, GR>), dim3(nb), dim3(kBlock), 0, st, At.sptr, At.idx,    \
                       static_cast<const typename Code<VT>::T *>(At.val), At.scale, ratio, g,      \
                       g_next, gs_next, v, a, sens, H, grid, w, lam, At.n_slices)
    if (grouping == 0) {
        if (vt == 0) SGTV_BU(0, 0); else if (vt == 1) SGTV_BU(1, 0); else SGTV_BU(2, 0);
    } else {
        if (vt == 0) SGTV_BU(0, 1); else if (vt == 1) SGTV_BU(1, 1); else SGTV_BU(2, 1);
    }
#undef SGTV_BU
    return hipGetLastError();
}

hipError_t launch_split_update(const float *f, const float *v_old, const float *a_old,
                               float *v_new, float *a_new, const Grid &grid, const Weights &w,
                               int grouping, float thr, hipStream_t st) {
    const int sl = seg_log2_for(grid.Q);
    const unsigned nb = blocks_for(grid.S, kBlock >> sl);
    if (nb == 0) return hipSuccess;
    auto kern = grouping == 0 ? (w.full ? k_split_update<0, true> : k_split_update<0, false>)
                              : (w.full ? k_split_update<1, true> : k_split_update<1, false>);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, st, f, v_old, a_old, v_new, a_new, grid, w,
                       thr, sl);
    return hipGetLastError();
}

hipError_t launch_consistent_split(const float *f, float *v, float *a, const Grid &grid,
                                   const Weights &w, int grouping, float thr, hipStream_t st) {
    const int sl = seg_log2_for(grid.Q);
    const unsigned nb = blocks_for(grid.S, kBlock >> sl);
    if (nb == 0) return hipSuccess;
    if (grouping == 0)
        hipLaunchKernelGGL(k_consistent_split<0>, dim3(nb), dim3(kBlock), 0, st, f, v, a, grid, w, thr, sl);
    else
        hipLaunchKernelGGL(k_consistent_split<1>, dim3(nb), dim3(kBlock), 0, st, f, v, a, grid, w, thr, sl);
    return hipGetLastError();
}

hipError_t launch_report(const float *f, const float *v, const float *a, const float *v_prev,
                         const float *a_prev, const Grid &grid, const Weights &w, int grouping,
                         double *partials, hipStream_t st, int64_t *n_blocks) {
    const int sl = seg_log2_for(grid.Q);
    const unsigned nb = blocks_for(grid.S, kBlock >> sl);
    *n_blocks = nb;
    if (grouping == 0)
        hipLaunchKernelGGL(k_report<0>, dim3(nb), dim3(kBlock), 0, st, f, v, a, v_prev, a_prev,
                           grid, w, sl, partials, static_cast<int64_t>(nb));
    else
        hipLaunchKernelGGL(k_report<1>, dim3(nb), dim3(kBlock), 0, st, f, v, a, v_prev, a_prev,
                           grid, w, sl, partials, static_cast<int64_t>(nb));
    return hipGetLastError();
}

hipError_t launch_rescale_dual(float *v, float *a, const Grid &grid, int grouping, float t,
                               hipStream_t st) {
    if (grid.J == 0) return hipSuccess;
    if (grouping == 0)
        hipLaunchKernelGGL(k_rescale_v<0>, dim3(grid_stride_blocks(grid.J * 4)), dim3(kBlock), 0, st, v, a,
                           grid, t);
    else
        hipLaunchKernelGGL(k_rescale_v<1>, dim3(grid_stride_blocks(grid.J * 4)), dim3(kBlock), 0, st, v, a,
                           grid, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ng = grouping == 0 ? grid.S : grid.J;
    hipLaunchKernelGGL(k_rescale_a, dim3(grid_stride_blocks(ng)), dim3(kBlock), 0, st, a, ng, t);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *partials, int64_t n, int n_quant, double *out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(n_quant), dim3(kBlock), 0, st, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_sum_f32(const float *a, int64_t n, double *partials, hipStream_t st,
                          int64_t *n_blocks) {
    const unsigned nb = grid_stride_blocks(n);
    *n_blocks = nb;
    hipLaunchKernelGGL(k_sum_f32, dim3(nb), dim3(kBlock), 0, st, a, n, partials);
    return hipGetLastError();
}

hipError_t launch_fill_ratio(const double *num, const double *den, float *out, int64_t n,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_fill_ratio, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, st, num, den,
                       out, n);
    return hipGetLastError();
}

hipError_t launch_scale(const float *x, const float *s, float *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_scale, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, st, x, s, out, n);
    return hipGetLastError();
}

hipError_t launch_split_from_state(const float *v, const float *a, float *d, float *c,
                                   const Grid &grid, int grouping, hipStream_t st) {
    hipLaunchKernelGGL(k_split_from_state, dim3(grid_stride_blocks(grid.J * 4)), dim3(kBlock), 0,
                       st, v, a, d, c, grid, grouping);
    return hipGetLastError();
}

hipError_t launch_div_safe(const float *num, const float *den, float *out, int64_t n,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_div_safe, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, st, num, den,
                       out, n);
    return hipGetLastError();
}

hipError_t launch_check_range(const float *x, int64_t n, float lo, int strict_lo, float hi,
                              int *flag, hipStream_t st) {
    hipLaunchKernelGGL(k_check_range, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, st, x, n, lo,
                       strict_lo, hi, flag);
    return hipGetLastError();
}

}  // namespace sgtv
