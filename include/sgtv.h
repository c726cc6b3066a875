/*
 * sgtv.h -- C ABI of the MI355X library for spectrally grouped total-variation
 * reconstruction of photon-limited scatter data with ADMM.
 *
 * Problem (Section II, Eqs. 1-2; Section III, Eq. 3):
 *   minimise over f >= 0   L(f) + beta * R(w .* G f)
 *   L(f) = sum_i (A f + r)_i - y_i log (A f + r)_i   (Poisson model of Eq. 1)
 *   R(d) = sum_s || d[s, :, :] ||_2                   (one group per spatial bin,
 *                                                      over all spectral bins q and
 *                                                      all neighbour directions p)
 * solved with the split-Bregman / scaled ADMM iteration of Eqs. 4-6:
 *   image update (Eq. 4)  by optimisation transfer (EM surrogate of L plus
 *                         De Pierro's separable surrogate of the quadratic),
 *                         a closed-form nonnegative root per hyper-voxel;
 *   split update (Eq. 5)  block soft-threshold of v = w.*G f + c per group;
 *   dual update  (Eq. 6)  c = v - d.
 *
 * Conventions fixed by this ABI:
 *   - J = ny * nx * Q hyper-voxels, voxel j = (iy * nx + ix) * Q + q
 *     (spectral bin fastest; "lexicographic order" of Section II).
 *   - Neighbour directions p = 0..3: +x, -x, +y, -y.  A neighbour outside the
 *     grid has value zero (Dirichlet, Section III), so every voxel has N = 4
 *     differences (G_p f)[s, q] = f[s, q] - f[nb_p(s), q].
 *   - Arrays indexed by (s, p, q) are laid out [s][p][q], q fastest (4*J floats).
 *   - The objective is reported with the data term written as the
 *     I-divergence sum_i p_i - y_i + y_i log(y_i / p_i) (0 log 0 = 0), which
 *     differs from L by a constant of the data.
 *
 * Every function returns SGTV_OK (0) or a negative status, never throws, and
 * on error leaves the context exactly as it was.  sgtv_last_error() returns a
 * message for the last failing call on the calling thread.
 *
 * Ownership: every pointer argument belongs to the caller and is read (or
 * written) only during the call; the library copies what it keeps into
 * device memory it allocates itself, or into the caller's workspace after
 * sgtv_commit_system (the one exception: that buffer is used for the
 * context's lifetime).  mem_kind says whether a pointer is host memory
 * (SGTV_HOST) or device memory of the context's GPU (SGTV_DEVICE).  All work
 * is ordered on the stream given to sgtv_create; functions that return data
 * to the host synchronise that stream.
 */
#ifndef SGTV_H
#define SGTV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgtv_ctx_s *sgtv_ctx;

enum {
    SGTV_OK = 0,
    SGTV_EINVAL = -1,   /* an argument is out of range, NaN/Inf, negative, ... */
    SGTV_ESHAPE = -2,   /* sizes or index arrays are inconsistent               */
    SGTV_ESTATE = -3,   /* call order: system or data not set yet               */
    SGTV_EDEVICE = -4,  /* a HIP runtime call failed                            */
    SGTV_ENOMEM = -5    /* device or host allocation failed                     */
};

/* storage type of the system-matrix values */
enum { SGTV_F32 = 0, SGTV_BF16 = 1, SGTV_F16 = 2 };

/* where caller pointers live */
enum { SGTV_HOST = 0, SGTV_DEVICE = 1 };

/* grouping of the total-variation penalty */
enum {
    SGTV_GROUP_SPECTRAL = 0, /* Eq. 2: one group per spatial bin over (q, p)           */
    SGTV_GROUP_STANDARD = 1  /* standard isotropic TV: one group per (s, q) over p     */
};

typedef struct {
    double total;     /* data + beta * tv, for the current image f^k                 */
    double data;      /* sum_i p_i - y_i + y_i log(y_i / p_i), p = A f^k + r         */
    double tv;        /* R(w .* G f^k)                                               */
    double r_primal;  /* || w.*G f^k - d^k ||_2                                      */
    double r_dual;    /* rho * || (w.*G)^T (d^k - d^{k-1}) ||_2  (0 before the first
                         iteration after set_data / set_init / set_state)           */
    int64_t iter;     /* k: ADMM iterations done since set_data / set_init          */
} sgtv_report;

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t of
 * that device (NULL: the null stream).  The stream must outlive the context. */
int sgtv_create(sgtv_ctx *out, int device, void *hip_stream);

/* Free every device buffer of the context.  NULL is ignored. */
void sgtv_destroy(sgtv_ctx ctx);

/* Message of the last failing call on this thread ("" if none). */
const char *sgtv_last_error(void);

/* Library version string, for diagnostics. */
const char *sgtv_version(void);

/*
 * Set the system: an I x J nonnegative matrix A (Section II, A in R_+^{IxJ})
 * in CSR form with int64 row pointer (I+1 entries, row_ptr[0] = 0,
 * row_ptr[I] = nnz, non-decreasing) and int32 column indices in [0, J).
 * Values must be finite and >= 0; explicit zeros are allowed and empty rows
 * and columns are legal.  nnz must be below 2^31.
 * storage_dtype SGTV_BF16 / SGTV_F16 stores every value as a 16-bit code of
 * a / sigma_j with a per-column FP32 scale sigma_j = max_i a_ij; products are
 * accumulated in FP32.
 * w: direction weights w_{s,q,p} of Eq. 2: NULL (all one), w_len = 4 (one
 * positive value per direction) or w_len = 4*J (layout [s][p][q], positive).
 * Resets data and iteration state.
 */
int sgtv_set_system(sgtv_ctx ctx, int64_t I, int32_t ny, int32_t nx, int32_t Q,
                    const int64_t *row_ptr, const int32_t *col_idx, const float *val,
                    int64_t nnz, int storage_dtype, const float *w, int64_t w_len,
                    int mem_kind);

/*
 * Set the data y (I counts, finite, >= 0, real values allowed), the known
 * background r (I values, finite, > 0), the regularisation weight beta >= 0,
 * the ADMM penalty rho = lambda > 0 (Eqs. 4-6) and the number of surrogate
 * sweeps per image update (>= 1).  Resets the state: f = kappa * 1 with
 * kappa = sum(y) / sum(A^T 1) (the count-matched uniform start), d = c = 0,
 * k = 0.  Requires a system.
 */
int sgtv_set_data(sgtv_ctx ctx, const float *y, const float *r, double beta, double rho,
                  int sweeps, int mem_kind);

/* Choose the TV grouping (SGTV_GROUP_*); resets d = c = 0 and k = 0. */
int sgtv_set_grouping(sgtv_ctx ctx, int grouping);

/* Start image: x0 (J values, finite, >= 0) or NULL for the uniform start
 * kappa * 1.  Resets d = c = 0, k = 0. */
int sgtv_set_init(sgtv_ctx ctx, const float *x0, int mem_kind);

/* Start image x0 (J values, finite, >= 0) together with the split and dual
 * variables for which x0 is a fixed point of the split and dual updates
 * (Eqs. 5-6): d = w.*G x0 and, on every group g with d_g != 0, the scaled
 * dual c_g = (beta / rho) d_g / ||d_g|| (0 on the other groups), the
 * optimality condition of Eq. 5.  A start image near the solution then
 * starts near the ADMM fixed point, where d = c = 0 would not.  k = 0. */
int sgtv_set_init_dual(sgtv_ctx ctx, const float *x0, int mem_kind);

/* Run n_iters >= 0 ADMM iterations (Eqs. 4-6) asynchronously on the stream. */
int sgtv_iterate(sgtv_ctx ctx, int n_iters);

/* Capture and instantiate now the graph that sgtv_iterate(ctx, n_iters) would
 * replay from the current state, without running it, so that the next such
 * call only launches the graph (for callers that time or serve the iterations
 * and want the capture outside that call).  Leaves the state unchanged.  No
 * effect when graphs are off, kernel timing is on or n_iters < 2.  The graph
 * is dropped, like every captured graph, by calls that change the system,
 * data, parameters or state.  Errors: SGTV_EINVAL for n_iters < 0, SGTV_ESTATE
 * before system and data are set, SGTV_EDEVICE if capture fails. */
int sgtv_prepare(sgtv_ctx ctx, int n_iters);

/* Graph replay of sgtv_iterate (default on): the launch sequence of n
 * iterations is captured once into a HIP graph per (n, buffer parity) and
 * replayed on the context stream; captured graphs are dropped by every call
 * that changes the system, data, parameters or state.  enable = 0 launches
 * the kernels one by one. */
int sgtv_set_graphs(sgtv_ctx ctx, int enable);

/* Image update and split/dual update of the last surrogate sweep in one
 * elementwise-and-stencil pass over tiles of spatial bins (tiled format;
 * default off): a workgroup updates the image of its tile and of a one-bin
 * ring in LDS, then the groups of its tile from it, so the new image is not
 * read back from memory.  The results are the same bit for bit as with the
 * two launches; on an MI355X the two launches are faster (the ring is
 * computed twice and a tile's LDS allows one workgroup per CU), so they stay
 * the default.  get_fused_update reports whether the pass is used for the
 * current system and its tile (bins in x and y; 0 when a tile's LDS would
 * not fit). */
int sgtv_set_fused_update(sgtv_ctx ctx, int enable);
int sgtv_get_fused_update(sgtv_ctx ctx, int *active, int32_t *tile_x, int32_t *tile_y);

/* Row-block epilogues of the tiled products (Section III: the ratio of the
 * EM step and the image update follow the two products; default off).  The
 * workgroup that writes the last slab's partial sums of a row block of A f
 * computes the ratio y / (A f + r) of its rows in the same launch, and the
 * one that completes a row block of A^T t the image update of its voxels,
 * so an iteration is three launches (forward with ratio, back with image
 * update, split and dual update) instead of five.  The arithmetic and the
 * order of every sum are those of the separate launches: results are the
 * same bit for bit.  Off: the separate launches.  The work of a row block
 * waits for its last slab, so when all row blocks finish together (one wave
 * of workgroups) the epilogues run on as many CUs as there are row blocks;
 * on an MI355X they save a little on the smallest scans (9 x 41 x 54:
 * 0.025 against 0.027 ms per iteration) and lose on larger ones (64^3:
 * 0.067 against 0.051 ms; 128^3: 0.427 against 0.408 ms).  With the fused
 * image and split update on, the last sweep's back product runs without its
 * epilogue. */
int sgtv_set_epilogues(sgtv_ctx ctx, int enable);
int sgtv_get_epilogues(sgtv_ctx ctx, int *enabled);

/* Objective and residuals of the current state (FP64 reductions); synchronises. */
int sgtv_objective(sgtv_ctx ctx, sgtv_report *out);

/* Copy the current image f^k (J floats). */
int sgtv_get_image(sgtv_ctx ctx, float *x, int mem_kind);

/* Copy the split and scaled dual variables d^k and c^k (4*J floats each,
 * layout [s][p][q]).  Either pointer may be NULL. */
int sgtv_get_split(sgtv_ctx ctx, float *d, float *c, int mem_kind);

/*
 * Raw iteration state for bit-exact checkpoint and resume.  The library
 * keeps v^k = w.*G f^k + c^{k-1} (4*J floats, [s][p][q]) and one shrink
 * factor per group a^k (n_groups floats: ny*nx for the spectral grouping,
 * J for the standard one), so that d^k = a^k v^k and c^k = v^k - d^k.
 * sgtv_state_sizes reports the element counts.  set_state requires
 * 0 <= a <= 1 and finite values; it resets the previous-split memory used by
 * r_dual.
 */
int sgtv_state_sizes(sgtv_ctx ctx, int64_t *n_image, int64_t *n_split, int64_t *n_groups);
int sgtv_get_state(sgtv_ctx ctx, float *f, float *v, float *a, int64_t *k, int mem_kind);
int sgtv_set_state(sgtv_ctx ctx, const float *f, const float *v, const float *a, int64_t k,
                   int mem_kind);

/*
 * Penalty adaptation and stopping (Boyd, Parikh, Chu, Peleato, Eckstein,
 * Distributed Optimization and Statistical Learning via ADMM, 2011:
 * Sections 3.3 and 3.4.1), for the constraint d = w.*G f of Eq. 3.
 *
 * sgtv_set_penalty changes the penalty rho (lambda of Eq. 4) of the running
 * iteration: the scaled dual c is rescaled so that rho * c is unchanged, d and
 * f are kept, and the curvature and shrink threshold follow rho.
 *
 * sgtv_iterate_adaptive iterates in chunks of opt->check (the last may be
 * shorter, at most max_iters in all); after each chunk, with r and s the
 * primal and dual residuals of its last iteration (as sgtv_objective),
 *   eps_pri  = sqrt(4 J) eps_abs + eps_rel max(||w.*G f||, ||d||)
 *   eps_dual = sqrt(J)   eps_abs + eps_rel rho ||(w.*G)^T c||
 * it stops when r <= eps_pri and s <= eps_dual; otherwise rho <- tau rho when
 * r > mu s, rho <- rho / tau when s > mu r (tau = 1: fixed rho; eps = 0: no
 * stopping).  checks[m] (up to max_checks) records check m; n_checks,
 * iters_done and converged (1 when the rule stopped the run) may be NULL.
 */
typedef struct {
    int32_t check;     /* iterations between checks, >= 1                          */
    double eps_abs;    /* absolute tolerance, >= 0                                 */
    double eps_rel;    /* relative tolerance, >= 0                                 */
    double mu;         /* residual ratio that triggers a change, >= 1              */
    double tau;        /* factor of a change, >= 1                                 */
} sgtv_adaptive;

typedef struct {
    int64_t iter;      /* iterations of this call done at the check                */
    double r_primal, r_dual, eps_primal, eps_dual;
    double rho;        /* penalty after the check                                  */
} sgtv_check;

int sgtv_set_penalty(sgtv_ctx ctx, double rho);
int sgtv_get_penalty(sgtv_ctx ctx, double *rho);
int sgtv_iterate_adaptive(sgtv_ctx ctx, int64_t max_iters, const sgtv_adaptive *opt,
                          sgtv_check *checks, int32_t max_checks, int32_t *n_checks,
                          int64_t *iters_done, int *converged);

/* Device memory.  With sgtv_set_system the library allocates the context's
 * memory itself (at set_system and set_data).  sgtv_workspace_bytes estimates
 * that amount beforehand (within about 25 % for random matrices of evenly
 * spread entries; -1 for invalid arguments) for a system of I measurements,
 * J hyper-voxels and nnz entries with the automatic schedule;
 * sgtv_device_bytes reports what the library has allocated for the context
 * now (memory in a caller's workspace is not counted). */
int64_t sgtv_workspace_bytes(int64_t I, int64_t J, int64_t nnz, int storage_dtype);
int sgtv_device_bytes(sgtv_ctx ctx, int64_t *bytes);

/*
 * Caller-owned device memory, in two phases.  sgtv_plan_system takes the
 * arguments of sgtv_set_system, checks and packs the system on the host
 * (nothing on the device yet), keeps it in the context and returns in *bytes
 * the exact size of device memory the context will use for this system, its
 * data, its iteration state (either grouping) and the temporaries of single
 * calls.  sgtv_commit_system then puts the planned system into `workspace`,
 * a device buffer of the context's GPU that the caller allocated (a torch
 * tensor, say) of at least that many bytes, aligned to 256 bytes; it replaces
 * the context's system and data like sgtv_set_system.  From then on no call
 * on the context allocates device memory: set_data, set_grouping, set_init,
 * set_init_dual, set_state, get_split, backprojection and iterate use the
 * workspace only.  The library never frees it; the caller keeps it alive
 * and unchanged until sgtv_destroy or the next set_system / commit_system
 * (sgtv_set_system returns the context to library-allocated memory).
 * Errors: commit without a plan SGTV_ESTATE, a smaller or misaligned
 * workspace SGTV_ENOMEM / SGTV_EINVAL (context unchanged).
 */
int sgtv_plan_system(sgtv_ctx ctx, int64_t I, int32_t ny, int32_t nx, int32_t Q, const int64_t *row_ptr,
                     const int32_t *col_idx, const float *val, int64_t nnz, int storage_dtype, const float *w,
                     int64_t w_len, int mem_kind, int64_t *bytes);
int sgtv_commit_system(sgtv_ctx ctx, void *workspace, int64_t bytes);

/*
 * The packed system of a fixed scanner, stored once and loaded afterwards
 * without packing again (packing the system matrix into the tiled layout is
 * the slow part of sgtv_set_system).  sgtv_save_system writes the context's
 * system (its schedule, tile tables, value arrays, H table and weights, not
 * the data or the iteration state) to the file `path`; sgtv_load_system
 * reads such a file into a context and installs it like sgtv_set_system
 * (library-allocated memory, data and state cleared); the sensitivity A^T 1
 * is computed again on the device.  A loaded system gives bit for bit the
 * results of the system that was saved.  The file is for this library
 * version and GPU architecture; it carries a checksum, and a damaged, short
 * or foreign file gives SGTV_EINVAL with the context unchanged.  Its content
 * is trusted beyond that: load only files that sgtv_save_system wrote.
 * Errors: save without a system SGTV_ESTATE, a file that cannot be opened or
 * written SGTV_EINVAL.
 */
int sgtv_save_system(sgtv_ctx ctx, const char *path);
int sgtv_load_system(sgtv_ctx ctx, const char *path);

/* Normalised backprojection x_in = (A^T y) / (A^T 1) (0 where A^T 1 = 0),
 * J floats, of the data currently set. */
int sgtv_backprojection(sgtv_ctx ctx, float *x, int mem_kind);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same result
 * as sgtv_backprojection, computed without any allocation.  Its intermediate
 * vectors live in a static device buffer of the library (8388608 floats,
 * 32 MiB, on every GPU the library runs on, held until the process ends), so
 * J may be at most SGTV_NOALLOC_MAX_VOXELS (SGTV_ESHAPE beyond).  x (J
 * floats) is host or device memory as mem_kind says; the call synchronises
 * the context stream.  Every call on one GPU uses the same buffer: calls that
 * overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller. */
#define SGTV_NOALLOC_MAX_VOXELS 4194304
int sgtv_backprojection_noalloc(sgtv_ctx ctx, float *x, int mem_kind);

/*
 * Launch schedule of the two sparse products A f and A^T t.  Takes effect at
 * the next sgtv_set_system; zero fields are chosen automatically.
 *   format SGTV_FORMAT_TILED: LDS-tiled products.  A workgroup of `waves`
 *     wavefronts owns waves * rows_per_wave output rows with their sums in
 *     LDS, stages `block_cols` entries of the gathered vector at a time into
 *     LDS, and the column blocks are split into `slabs` groups whose partial
 *     sums are added afterwards (each slab is pinned to one XCD).
 *   format SGTV_FORMAT_SELL: sliced ELL, one lane per output row, gathers
 *     straight from memory (no other field applies).
 *   variant: inner loop of the tiled products: 1 one batch of entries in
 *     flight per wave, 2 two batches, 3 two batches plus the next column block
 *     read ahead into registers (0: automatic).  Variant 1 stores the
 *     entries' indices in 24 bits (three bytes per entry instead of four)
 *     when 64 <= rows_per_wave <= 1024 and block_cols <= 16380, or
 *     1024 < rows_per_wave <= 2048 and block_cols <= 8188.
 * Limits: waves in [1, 16]; rows_per_wave in [1, 32767]; block_cols a
 * multiple of 4 in [4, 65536]; slabs in [1, 16]; the LDS of one workgroup,
 * 4 * (waves * rows_per_wave rounded up to 4 + block_cols) + 16 bytes with
 * 24-bit indices, 4 * (waves * (rows_per_wave + 1) rounded up to 4 +
 * block_cols) bytes with 32-bit ones, at most 163840.  Violations give
 * SGTV_EINVAL at set_schedule (field ranges) or set_system (LDS size).  The
 * persistent batch launch keeps 16 bytes of LDS of its own and refuses tiles
 * that leave less (sgtv_batch_iterate returns SGTV_EDEVICE).
 */
enum { SGTV_FORMAT_TILED = 0, SGTV_FORMAT_SELL = 1 };
typedef struct {
    int32_t format;
    int32_t waves;
    int32_t fwd_rows_per_wave, fwd_block_cols, fwd_slabs;
    int32_t back_rows_per_wave, back_block_cols, back_slabs;
    int32_t variant;
} sgtv_schedule;

int sgtv_set_schedule(sgtv_ctx ctx, const sgtv_schedule *s);
/* The schedule in use for the current system (automatic choices resolved),
 * or the requested one if no system is set. */
int sgtv_get_schedule(sgtv_ctx ctx, sgtv_schedule *s);

/*
 * Kernel timing for measurement.  While enabled, sgtv_iterate brackets every
 * kernel launch with HIP events on the context stream.  sgtv_kernel_times
 * synchronises, adds the elapsed milliseconds per kernel class to ms[0..4]
 * and the launch counts to counts[0..4], then clears the record.  Classes:
 * 0 forward projection A f (sliced ELL: fused with the ratio), 1
 * backprojection A^T t (sliced ELL: fused with the image update), 2 split and
 * dual update, 3 ratio y / (A f + r) of the tiled format, 4 image update of
 * the tiled format (with the split and dual update when they run in one pass,
 * see sgtv_set_fused_update).
 */
int sgtv_set_profiling(sgtv_ctx ctx, int enable);
int sgtv_kernel_times(sgtv_ctx ctx, double *ms, int64_t *counts);

/*
 * Batches: many independent scans iterated together.  Each ADMM iteration
 * of the whole batch is five launches (forward products of every scan, the
 * ratios, the backprojections, the image updates, the split and dual
 * updates), each covering all scans; sgtv_batch_iterate captures the n
 * iterations into one HIP graph and launches it once.  All scans of a batch
 * store their matrix values in one type (FP32 unless sgtv_batch_set_storage
 * says otherwise) and use one surrogate sweep; each scan may have its own
 * grid, matrix, weights, grouping, data, beta, rho and schedule.  A scan
 * of a batch gives bit-identical results to the same scan in its own context
 * with the same schedule.
 */
typedef struct sgtv_batch_s *sgtv_batch;

int sgtv_batch_create(sgtv_batch *out, int device, void *hip_stream);
void sgtv_batch_destroy(sgtv_batch b);
/* Value type of the matrices of every scan added afterwards: SGTV_F32
 * (default), SGTV_BF16 or SGTV_F16 with a per-column FP32 scale, as in
 * sgtv_set_system.  Only before the first scan is added (SGTV_ESTATE after);
 * the persistent launch takes FP32 batches only. */
int sgtv_batch_set_storage(sgtv_batch b, int storage_dtype);
/* Add one scan (arguments as sgtv_set_system / sgtv_set_grouping /
 * sgtv_set_data; schedule NULL: automatic; schedules of one batch must agree
 * on waves and variant).  The new scan starts from the uniform image; index
 * receives its position.
 * Several threads may add scans to one batch at the same time (the host-side
 * packing of each matrix runs in the calling thread); the scan order is then
 * the order in which the calls finish. */
int sgtv_batch_add_scan(sgtv_batch b, int64_t I, int32_t ny, int32_t nx, int32_t Q,
                        const int64_t *row_ptr, const int32_t *col_idx, const float *val,
                        int64_t nnz, const float *w, int64_t w_len, const float *y, const float *r,
                        double beta, double rho, int grouping, const sgtv_schedule *schedule,
                        int mem_kind, int32_t *index);
/* Add one scan whose system comes from a file that sgtv_save_system (or
 * sgtv_batch_save_scan) wrote: a tiled system with FP32 values whose
 * schedule agrees with the batch on waves and variant; grouping and data as
 * in sgtv_batch_add_scan.  The scan gives bit for bit the results of one
 * added with the matrix that was saved.  Errors as sgtv_load_system, and
 * SGTV_EINVAL for a system of another format or value type. */
int sgtv_batch_add_system_file(sgtv_batch b, const char *path, const float *y, const float *r, double beta,
                               double rho, int grouping, int mem_kind, int32_t *index);
/* Write the packed system of scan `scan` to a file, as sgtv_save_system. */
int sgtv_batch_save_scan(sgtv_batch b, int32_t scan, const char *path);
int sgtv_batch_size(sgtv_batch b, int32_t *n_scans);
/* n_iters iterations of every scan in batched launches (graph replay). */
int sgtv_batch_iterate(sgtv_batch b, int n_iters);

/* Capture and instantiate now, without running them, the graphs that the
 * next call with n_iters replays: sequential = 0, the graph of
 * sgtv_batch_iterate (building the batch tables first if scans were added);
 * sequential = 1, each scan's own graph of sgtv_batch_iterate_sequential (as
 * sgtv_prepare per scan).  The state is unchanged.  No effect for an empty
 * batch or n_iters = 0.  Errors as sgtv_prepare, and SGTV_EINVAL for a
 * sequential other than 0 or 1. */
int sgtv_batch_prepare(sgtv_batch b, int n_iters, int sequential);
/* How sgtv_batch_iterate runs the iterations.
 *   SGTV_BATCH_GRAPH (default): five batched launches per iteration, the n
 *     iterations captured into one HIP graph (asynchronous).
 *   SGTV_BATCH_PERSISTENT: one cooperative launch (hipLaunchCooperativeKernel:
 *     a grid that cannot be resident at once is refused) of one workgroup per
 *     free slot of every CU runs all n iterations, its workgroups walking the
 *     phases of every scan with grid-wide barriers between dependent phases
 *     (four per iteration).  A barrier wait is bounded (two seconds): past it
 *     the launch is abandoned, the call returns SGTV_EDEVICE and the batch
 *     state is undefined.  The call waits for the launch.  Needs a multiple of
 *     4 waves per workgroup.
 * Both give bitwise the same images.  get_launch also reports the grid of the
 * last persistent launch (0 before the first). */
enum { SGTV_BATCH_GRAPH = 0, SGTV_BATCH_PERSISTENT = 1 };
int sgtv_batch_set_launch(sgtv_batch b, int mode);
int sgtv_batch_get_launch(sgtv_batch b, int *mode, int32_t *grid);
/* Time spent in each phase of the persistent launches since the last call,
 * as workgroup 0 sees it (clock ticks between its barrier exits), in
 * milliseconds: ms[0] forward products with the previous split, ms[1] ratio,
 * ms[2] back products, ms[3] image update, ms[4] the final split of each
 * launch; *iters = the iterations they cover.  Clears the record. */
int sgtv_batch_phase_times(sgtv_batch b, double *ms, int64_t *iters);

/* The same iterations scan after scan, each with its own graph: the
 * reference the batched launch is measured against. */
int sgtv_batch_iterate_sequential(sgtv_batch b, int n_iters);
int sgtv_batch_objective(sgtv_batch b, int32_t scan, sgtv_report *out);
int sgtv_batch_get_image(sgtv_batch b, int32_t scan, float *x, int mem_kind);

/*
 * Learned warm start: a convolutional network that maps an early image of a
 * scan (height x width pixels with one channel per spectral bin, NHWC = the
 * voxel order above) to a nonnegative start image for sgtv_set_init_dual.
 * The early image is either the image after a few plain iterations, from
 * which the network predicts a per-voxel correction factor, or the
 * normalised backprojection (sgtv_backprojection), from which it predicts
 * the image itself (see wsnet_start).  Architecture: `layers`
 * 3x3 convolutions with zero padding 1, 64 channels in and out, weights
 * [co][ky][kx][ci] and one bias per output channel; ReLU after every layer
 * but the last, softplus after the last.  Training minimises the mean
 * squared error against target images (reconstructions of the plain method)
 * with Adam.  Convolutions run on bfloat16 matrix cores with FP32
 * accumulation; master weights, gradients and Adam moments are FP32; the
 * loss is reduced in FP64.  Parameters are flat FP32, layer by layer:
 * weights (64*9*64) then bias (64).
 * Limits: channels = 64, width = 64, height even, 1 <= layers <= 16,
 * 1 <= batch <= max_batch.
 */
typedef struct wsnet_s *wsnet;

int wsnet_create(wsnet *out, int device, void *hip_stream, int32_t layers, int32_t height,
                 int32_t width, int32_t channels, int32_t max_batch);
void wsnet_destroy(wsnet net);
/* Number of parameters of a network with `layers` layers and `channels` channels. */
int64_t wsnet_param_count(int32_t layers, int32_t channels);
int wsnet_set_params(wsnet net, const float *params, int64_t n, int mem_kind);
int wsnet_get_params(wsnet net, float *params, int64_t n, int mem_kind);
/* Parameters to / from a file: a 24-byte header ("WSNT", version 1, layers,
 * channels, parameter count as int32, int32, int32, int32, int64) and the FP32
 * parameters; the Adam moments are not stored.  load requires a file of the
 * same shape and resets Adam as set_params does. */
int wsnet_save(wsnet net, const char *path);
int wsnet_load(wsnet net, const char *path);
/* x0 = network(x_in) for `batch` images (FP32 NHWC in and out). */
int wsnet_forward(wsnet net, const float *x_in, int32_t batch, float *x0, int mem_kind);
/* Start images for the reconstruction (the learned warm start).  For each of
 * `batch` images f (FP32 NHWC, J = height*width*channels values each: the
 * image after a few plain iterations, or the normalised backprojection),
 * m = mean(f) (FP64 sum; 1 where not positive) and s = network(f / m):
 *   WSNET_START_RATIO:  x0 = c_out * s * f   (per-voxel correction factor)
 *   WSNET_START_DIRECT: x0 = c_out * s * m   (the image itself)
 * c_out is the scale the targets were divided by in training (> 0).  With
 * floor > 0 every voxel is raised to at least floor * c_out * m (a fraction
 * of the predicted mean level): the image update is multiplicative, so a
 * voxel started near zero takes many iterations to grow; floor = 0 leaves x0
 * as above.  floor must be finite and >= 0. */
#define WSNET_START_RATIO 0
#define WSNET_START_DIRECT 1
int wsnet_start(wsnet net, const float *f, int32_t batch, int mode, double c_out, double floor, float *x0,
                int mem_kind);
/* Loss and gradient of the mean squared error of network(x_in) against
 * target; the gradient stays in the network for wsnet_adam_step and is
 * copied to grad (n parameters) when grad is not NULL. */
int wsnet_backward(wsnet net, const float *x_in, const float *target, int32_t batch,
                   double *loss, float *grad, int mem_kind);
/* One Adam step with the last gradient (Kingma and Ba); the step counter
 * starts at 1 after set_params or reset. */
int wsnet_adam_step(wsnet net, double lr, double beta1, double beta2, double eps);
/* wsnet_backward followed by wsnet_adam_step without waiting for the
 * device: the step's mean squared error (as wsnet_backward reports it) is
 * added to a running FP64 sum on the device instead of being returned, so a
 * training loop issues its steps back to back.  Parameters, gradients and
 * moments evolve exactly as with the two calls.  wsnet_loss_sum waits for
 * the device and returns the running sum and the number of steps in it
 * (reset != 0: both to zero afterwards). */
int wsnet_train_step(wsnet net, const float *x_in, const float *target, int32_t batch, double lr, double beta1,
                     double beta2, double eps, int mem_kind);
int wsnet_loss_sum(wsnet net, double *sum, int64_t *steps, int reset);
int wsnet_reset_adam(wsnet net);

#ifdef __cplusplus
}
#endif

#endif /* SGTV_H */
