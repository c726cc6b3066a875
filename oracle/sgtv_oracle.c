/*
 * FP64 CPU oracle for spectrally grouped TV reconstruction with ADMM.
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines what the GPU library must
 * compute; it is called by the tests, by the package's smoke check and by the
 * benchmark's CPU-baseline leg, and by nothing on the product path.  It shares
 * no code, header or table with the GPU library.
 *
 * Everything is plain IEEE double arithmetic, loops in fixed index order,
 * built without fast-math.  Loops whose outputs are independent of each
 * other (one row, one column, one voxel or one group per iteration) are
 * shared among OpenMP threads; every sum keeps the order of the serial loop
 * and every reduction over many outputs (objective, residual norms) stays
 * serial, so results are bitwise the same for any number of threads.
 * Conventions:
 *
 *   voxel j = s*Q + q, spatial bin s = iy*nx + ix          (Section II, J = S x Q)
 *   direction p: 0 = +x, 1 = -x, 2 = +y, 3 = -y            (four spatial neighbours)
 *   (D f)[s][p][q] = w[s][p][q] * (f[s][q] - f[nb_p(s)][q]), a neighbour outside
 *   the grid contributes the value zero (Dirichlet, Section III after Eq. 3).
 *   Arrays indexed by (s, p, q) are stored [s][p][q], q fastest.
 *   w == NULL means all weights are one.
 *
 * Groups: grouping 0 is the paper's spectral group (one group per spatial bin,
 * over all q and p, Eq. 2); grouping 1 is standard isotropic TV (one group per
 * (s, q) over p, the comparison regulariser of Section II).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NDIR 4

/* Threads for the loops over independent outputs (1: serial). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* neighbour of spatial bin s in direction p, or -1 when it lies outside */
static int64_t neighbour(int ny, int nx, int64_t s, int p)
{
    int64_t iy = s / nx, ix = s % nx;
    switch (p) {
    case 0: return ix + 1 < nx ? s + 1 : -1;
    case 1: return ix - 1 >= 0 ? s - 1 : -1;
    case 2: return iy + 1 < ny ? s + nx : -1;
    default: return iy - 1 >= 0 ? s - nx : -1;
    }
}

static double weight(const double *w, int Q, int64_t s, int p, int q)
{
    return w ? w[(s * NDIR + p) * Q + q] : 1.0;
}

/* Eq. 1 mean: p = A f + r, A in CSR. */
void or_forward(int64_t I, const int64_t *rowptr, const int32_t *col, const double *val,
                const double *f, const double *r, double *p)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < I; ++i) {
        double acc = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            acc += val[k] * f[col[k]];
        p[i] = acc + (r ? r[i] : 0.0);
    }
}

/* e = A^T t, accumulated row by row in CSR order. */
void or_back(int64_t I, int64_t J, const int64_t *rowptr, const int32_t *col,
             const double *val, const double *t, double *e)
{
    for (int64_t j = 0; j < J; ++j)
        e[j] = 0.0;
    for (int64_t i = 0; i < I; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            e[col[k]] += val[k] * t[i];
}

/* The entries of A column by column: column j holds its entries in the order
 * a row-by-row pass over the CSR form meets them (rows ascending), so
 * e_j = sum over that list of a_ij t_i adds exactly the terms of or_back in
 * the same order, and the columns can be summed independently. */
typedef struct {
    int64_t J;
    int64_t *colptr;
    int32_t *row;
    double *val;
} or_csc;

static int csc_build(int64_t I, int64_t J, const int64_t *rowptr, const int32_t *col,
                     const double *val, or_csc *At)
{
    int64_t nnz = rowptr[I];
    At->J = J;
    At->colptr = calloc((size_t)(J + 1), sizeof(int64_t));
    At->row = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    At->val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int64_t *next = malloc(sizeof(int64_t) * (size_t)(J > 0 ? J : 1));
    if (!At->colptr || !At->row || !At->val || !next) {
        free(next);
        return -1;
    }
    /* each thread counts and fills the columns of its own range, passing over
     * the rows in order: every column list is written by one thread, rows
     * ascending, whatever the number of threads */
#pragma omp parallel
    {
        int64_t nth = 1, me = 0;
#ifdef _OPENMP
        nth = omp_get_num_threads();
        me = omp_get_thread_num();
#endif
        int64_t j0 = J * me / nth, j1 = J * (me + 1) / nth;
        for (int64_t k = 0; k < nnz; ++k)
            if (col[k] >= j0 && col[k] < j1)
                At->colptr[col[k] + 1]++;
#pragma omp barrier
#pragma omp single
        for (int64_t j = 0; j < J; ++j)
            At->colptr[j + 1] += At->colptr[j];
        for (int64_t j = j0; j < j1; ++j)
            next[j] = At->colptr[j];
        for (int64_t i = 0; i < I; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] >= j0 && col[k] < j1) {
                    int64_t pos = next[col[k]]++;
                    At->row[pos] = (int32_t)i;
                    At->val[pos] = val[k];
                }
    }
    free(next);
    return 0;
}

static void csc_free(or_csc *At)
{
    free(At->colptr);
    free(At->row);
    free(At->val);
}

/* e = A^T t from the column lists (the same sums as or_back). */
static void back_csc(const or_csc *At, const double *t, double *e)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < At->J; ++j) {
        double acc = 0.0;
        for (int64_t k = At->colptr[j]; k < At->colptr[j + 1]; ++k)
            acc += At->val[k] * t[At->row[k]];
        e[j] = acc;
    }
}

/* g = w .* (G f), the stacked finite differences of Eq. 3. */
void or_diff(int ny, int nx, int Q, const double *w, const double *f, double *g)
{
    int64_t S = (int64_t)ny * nx;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s)
        for (int p = 0; p < NDIR; ++p) {
            int64_t nb = neighbour(ny, nx, s, p);
            for (int q = 0; q < Q; ++q) {
                double other = nb >= 0 ? f[nb * Q + q] : 0.0;
                g[(s * NDIR + p) * Q + q] = weight(w, Q, s, p, q) * (f[s * Q + q] - other);
            }
        }
}

/* out = (w .* G)^T t: each difference row adds +w*t to its own voxel and -w*t
 * to its in-grid neighbour.  Written per output voxel (s, q), the terms come
 * in the order of a pass over the rows by increasing s and p: the row of the
 * bin below (s - nx, direction +y), of the bin to the left (s - 1, +x), the
 * four rows of s, then the bin to the right (s + 1, -x) and the bin above
 * (s + nx, -y). */
void or_diff_adj(int ny, int nx, int Q, const double *w, const double *t, double *out)
{
    static const int before[2] = {3, 1}, after[2] = {0, 2};
    int64_t S = (int64_t)ny * nx;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < S; ++s)
        for (int q = 0; q < Q; ++q) {
            double acc = 0.0;
            for (int k = 0; k < 2; ++k) {
                int64_t nb = neighbour(ny, nx, s, before[k]);
                int pb = before[k] ^ 1;   /* direction from nb back to s */
                if (nb >= 0)
                    acc -= weight(w, Q, nb, pb, q) * t[(nb * NDIR + pb) * Q + q];
            }
            for (int p = 0; p < NDIR; ++p)
                acc += weight(w, Q, s, p, q) * t[(s * NDIR + p) * Q + q];
            for (int k = 0; k < 2; ++k) {
                int64_t nb = neighbour(ny, nx, s, after[k]);
                int pb = after[k] ^ 1;
                if (nb >= 0)
                    acc -= weight(w, Q, nb, pb, q) * t[(nb * NDIR + pb) * Q + q];
            }
            out[s * Q + q] = acc;
        }
}

/* De Pierro curvature of the quadratic penalty (Section III, image update):
 * every difference row rho spreads over its voxels with weights
 * |D_rho,j| / ||D_rho||_1, which yields H_j = lam * sum_rho |D_rho,j| ||D_rho||_1. */
void or_curv(int ny, int nx, int Q, const double *w, double lam, double *H)
{
    int64_t S = (int64_t)ny * nx;
    for (int64_t j = 0; j < S * Q; ++j)
        H[j] = 0.0;
    for (int64_t s = 0; s < S; ++s)
        for (int p = 0; p < NDIR; ++p) {
            int64_t nb = neighbour(ny, nx, s, p);
            for (int q = 0; q < Q; ++q) {
                double a = fabs(weight(w, Q, s, p, q));
                double l1 = nb >= 0 ? 2.0 * a : a;
                H[s * Q + q] += a * l1;
                if (nb >= 0)
                    H[nb * Q + q] += a * l1;
            }
        }
    for (int64_t j = 0; j < S * Q; ++j)
        H[j] *= lam;
}

/* Nonnegative root of H t^2 + B t - C = 0 (C >= 0, H > 0), the stationary
 * point of the separable surrogate of one hyper-voxel.  The branch choice
 * avoids cancellation.  H == 0 (no penalty curvature) reduces to t = C / B. */
double or_root(double H, double B, double C)
{
    if (H == 0.0)
        return B > 0.0 ? C / B : 0.0;
    double disc = sqrt(B * B + 4.0 * H * C);
    if (B <= 0.0)
        return (-B + disc) / (2.0 * H);
    return 2.0 * C / (B + disc);
}

/* Proximal map of thr * ||.||_2 on one group (Eq. 5): block soft-threshold.
 * Ties (norm == thr) and empty groups give zero. */
static void shrink_group(int n, const double *v, int64_t stride, double thr, double *d)
{
    double ss = 0.0;
    for (int k = 0; k < n; ++k)
        ss += v[k * stride] * v[k * stride];
    double nrm = sqrt(ss);
    double scale = nrm > thr ? 1.0 - thr / nrm : 0.0;
    for (int k = 0; k < n; ++k)
        d[k * stride] = scale * v[k * stride];
}

/* d = prox of (beta/lam) R applied to v, v and d laid out [s][p][q]. */
void or_shrink(int ny, int nx, int Q, int grouping, double thr, const double *v, double *d)
{
    int64_t S = (int64_t)ny * nx;
    if (grouping == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < S; ++s)
            shrink_group(NDIR * Q, v + s * NDIR * Q, 1, thr, d + s * NDIR * Q);
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < S; ++s)
            for (int q = 0; q < Q; ++q)
                shrink_group(NDIR, v + s * NDIR * Q + q, Q, thr, d + s * NDIR * Q + q);
    }
}

/* R applied to a stacked difference vector g: sum of group 2-norms (Eq. 2). */
double or_group_norm_sum(int ny, int nx, int Q, int grouping, const double *g)
{
    int64_t S = (int64_t)ny * nx;
    double tot = 0.0;
    for (int64_t s = 0; s < S; ++s) {
        if (grouping == 0) {
            double ss = 0.0;
            for (int k = 0; k < NDIR * Q; ++k)
                ss += g[s * NDIR * Q + k] * g[s * NDIR * Q + k];
            tot += sqrt(ss);
        } else {
            for (int q = 0; q < Q; ++q) {
                double ss = 0.0;
                for (int p = 0; p < NDIR; ++p) {
                    double v = g[(s * NDIR + p) * Q + q];
                    ss += v * v;
                }
                tot += sqrt(ss);
            }
        }
    }
    return tot;
}

/* Negative Poisson log-likelihood of Eq. 1 written as an I-divergence:
 * sum_i p_i - y_i + y_i log(y_i / p_i), with 0 log 0 = 0.  It differs from
 * the plain negative log-likelihood by a constant of the data only. */
double or_data_term(int64_t I, const double *p, const double *y)
{
    double tot = 0.0;
    for (int64_t i = 0; i < I; ++i) {
        double t = p[i] - y[i];
        if (y[i] > 0.0)
            t += y[i] * log(y[i] / p[i]);
        tot += t;
    }
    return tot;
}

typedef struct {
    int64_t I;
    int ny, nx, Q;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
    const double *y, *r;
    const double *w;
    double beta, lam;
    int grouping;
} or_problem;

static int64_t n_vox(const or_problem *P) { return (int64_t)P->ny * P->nx * P->Q; }

/* objective of Eq. 3 evaluated at d = w.*Gf: data term + beta * R(w.*Gf) */
void or_objective(const or_problem *P, const double *f, double out[3])
{
    int64_t J = n_vox(P);
    double *p = malloc(sizeof(double) * (P->I > 0 ? P->I : 1));
    double *g = malloc(sizeof(double) * (J * NDIR > 0 ? J * NDIR : 1));
    or_forward(P->I, P->rowptr, P->col, P->val, f, P->r, p);
    double data = or_data_term(P->I, p, P->y);
    or_diff(P->ny, P->nx, P->Q, P->w, f, g);
    double tv = or_group_norm_sum(P->ny, P->nx, P->Q, P->grouping, g);
    out[0] = data + P->beta * tv;
    out[1] = data;
    out[2] = tv;
    free(p);
    free(g);
}

/* Image update of Eq. 4, one pass of optimisation transfer from g:
 *   EM surrogate of L at g (sensitivity s = A^T 1, back-projected ratio e),
 *   De Pierro surrogate of (lam/2)||D f - z||^2 at g (gradient gam, curvature H),
 *   every hyper-voxel then solves its own 1-D problem in closed form. */
static void image_sweep(const or_problem *P, const or_csc *At, const double *sens,
                        const double *H, const double *z, double *g)
{
    int64_t J = n_vox(P), I = P->I;
    double *p = malloc(sizeof(double) * (I > 0 ? I : 1));
    double *e = malloc(sizeof(double) * (J > 0 ? J : 1));
    double *t = malloc(sizeof(double) * (J * NDIR > 0 ? J * NDIR : 1));
    double *gam = malloc(sizeof(double) * (J > 0 ? J : 1));
    or_forward(I, P->rowptr, P->col, P->val, g, P->r, p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < I; ++i)
        p[i] = P->y[i] / p[i];
    if (At)
        back_csc(At, p, e);
    else
        or_back(I, J, P->rowptr, P->col, P->val, p, e);
    or_diff(P->ny, P->nx, P->Q, P->w, g, t);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < J * NDIR; ++k)
        t[k] -= z[k];
    or_diff_adj(P->ny, P->nx, P->Q, P->w, t, gam);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < J; ++j) {
        double B = sens[j] + P->lam * gam[j] - H[j] * g[j];
        double C = g[j] * e[j];
        g[j] = or_root(H[j], B, C);
    }
    free(p);
    free(e);
    free(t);
    free(gam);
}

void or_image_sweep(const or_problem *P, const double *sens, const double *H, const double *z,
                    double *g)
{
    image_sweep(P, NULL, sens, H, z, g);
}

/* Sensitivity s = A^T 1. */
void or_sensitivity(const or_problem *P, double *sens)
{
    int64_t J = n_vox(P);
    double *ones = malloc(sizeof(double) * (P->I > 0 ? P->I : 1));
    for (int64_t i = 0; i < P->I; ++i)
        ones[i] = 1.0;
    or_back(P->I, J, P->rowptr, P->col, P->val, ones, sens);
    free(ones);
}

/* Uniform start kappa*1 matching total counts: kappa = sum(y) / sum(s). */
double or_plain_init(const or_problem *P)
{
    int64_t J = n_vox(P);
    double *sens = malloc(sizeof(double) * (J > 0 ? J : 1));
    or_sensitivity(P, sens);
    double sy = 0.0, ss = 0.0;
    for (int64_t i = 0; i < P->I; ++i)
        sy += P->y[i];
    for (int64_t j = 0; j < J; ++j)
        ss += sens[j];
    free(sens);
    return ss > 0.0 ? sy / ss : 0.0;
}

/*
 * ADMM / split Bregman of Eqs. 4-6 for n_iter iterations, state (f, d, c) in
 * place.  Each image update runs `sweeps` passes of optimisation transfer
 * with z = d^k - c^k held fixed.  After iteration k+1 the row
 * report[5k..5k+4] holds the objective of f^{k+1}, its data and TV parts,
 * the primal residual ||w.*Gf - d|| and the dual residual lam ||D^T(d^{k+1}-d^k)||.
 */
static double g_loop_seconds = 0.0;

/* Wall time of the iteration loop of the last or_admm call (set-up excluded). */
double or_last_loop_seconds(void)
{
    return g_loop_seconds;
}

static double now_seconds(void)
{
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

int or_admm(const or_problem *P, int n_iter, int sweeps, double *f, double *d, double *c,
            double *report)
{
    int64_t J = n_vox(P), JN = J * NDIR;
    double *sens = malloc(sizeof(double) * (J > 0 ? J : 1));
    double *H = malloc(sizeof(double) * (J > 0 ? J : 1));
    double *z = malloc(sizeof(double) * (JN > 0 ? JN : 1));
    double *v = malloc(sizeof(double) * (JN > 0 ? JN : 1));
    double *dn = malloc(sizeof(double) * (JN > 0 ? JN : 1));
    double *tmp = malloc(sizeof(double) * (J > 0 ? J : 1));
    double *ones = malloc(sizeof(double) * (P->I > 0 ? P->I : 1));
    or_csc At;
    if (!sens || !H || !z || !v || !dn || !tmp || !ones ||
        csc_build(P->I, J, P->rowptr, P->col, P->val, &At) != 0)
        return -1;
    for (int64_t i = 0; i < P->I; ++i)
        ones[i] = 1.0;
    back_csc(&At, ones, sens);                  /* s = A^T 1, as or_sensitivity */
    free(ones);
    or_curv(P->ny, P->nx, P->Q, P->w, P->lam, H);
    double t0 = now_seconds();
    for (int k = 0; k < n_iter; ++k) {
#pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < JN; ++m)
            z[m] = d[m] - c[m];
        for (int sw = 0; sw < sweeps; ++sw)
            image_sweep(P, &At, sens, H, z, f);
        or_diff(P->ny, P->nx, P->Q, P->w, f, v);
#pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < JN; ++m)
            v[m] += c[m];
        or_shrink(P->ny, P->nx, P->Q, P->grouping, P->beta / P->lam, v, dn);
        double rp = 0.0, rd = 0.0;
        for (int64_t m = 0; m < JN; ++m) {
            double prim = (v[m] - dn[m]) - c[m];   /* = Df^{k+1} - d^{k+1}            */
            rp += prim * prim;
        }
#pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < JN; ++m) {
            double cn = v[m] - dn[m];          /* c^k + Df^{k+1} - d^{k+1}   (Eq. 6) */
            c[m] = cn;
            z[m] = dn[m] - d[m];               /* reuse z for d^{k+1} - d^k       */
            d[m] = dn[m];
        }
        or_diff_adj(P->ny, P->nx, P->Q, P->w, z, tmp);
        for (int64_t j = 0; j < J; ++j)
            rd += tmp[j] * tmp[j];
        if (report) {
            double obj[3];
            or_objective(P, f, obj);
            report[5 * k + 0] = obj[0];
            report[5 * k + 1] = obj[1];
            report[5 * k + 2] = obj[2];
            report[5 * k + 3] = sqrt(rp);
            report[5 * k + 4] = P->lam * sqrt(rd);
        }
    }
    g_loop_seconds = now_seconds() - t0;
    csc_free(&At);
    free(sens);
    free(H);
    free(z);
    free(v);
    free(dn);
    free(tmp);
    return 0;
}

/*
 * ADMM with the penalty adapted by residual balancing and stopped by the
 * primal/dual residual rule (Boyd et al., Distributed Optimization and
 * Statistical Learning via ADMM, 2011: Sections 3.3 and 3.4.1), written for
 * the constraint d = w.*G f of Eq. 3 and the scaled dual c of Eq. 6.
 * Iterations run in chunks of `check` (the last one may be shorter); after
 * each chunk, with r and s the primal and dual residuals of its last
 * iteration (as in or_admm's report),
 *   eps_pri  = sqrt(4J) eps_abs + eps_rel max(||w.*Gf||, ||d||)
 *   eps_dual = sqrt(J)  eps_abs + eps_rel lam ||(w.*G)^T c||
 * the run stops when r <= eps_pri and s <= eps_dual; otherwise
 *   r > mu s:  lam <- tau lam, c <- c / tau
 *   s > mu r:  lam <- lam / tau, c <- c tau
 * (the unscaled dual lam c is unchanged; the curvature follows lam).
 * At most max_iter iterations; returns the number done, -1 on allocation
 * failure.  hist[6m .. 6m+5] for check m: iterations done, r, s, eps_pri,
 * eps_dual, lam after the check; *n_checks = number of checks, *lam_out =
 * final lam, *converged = 1 when the rule stopped the run.
 */
int or_admm_adaptive(const or_problem *P0, int max_iter, int sweeps, int check, double eps_abs,
                     double eps_rel, double mu, double tau, double *f, double *d, double *c,
                     double *hist, int max_checks, int *n_checks, double *lam_out, int *converged)
{
    or_problem P = *P0;
    int64_t J = n_vox(&P), JN = J * NDIR;
    double *g = malloc(sizeof(double) * (JN > 0 ? JN : 1));
    double *t = malloc(sizeof(double) * (J > 0 ? J : 1));
    double rep[5];
    int k = 0, m = 0;
    *converged = 0;
    if (!g || !t)
        return -1;
    while (k < max_iter) {
        int n = max_iter - k < check ? max_iter - k : check;
        if (n > 1 && or_admm(&P, n - 1, sweeps, f, d, c, NULL) != 0)
            return -1;
        if (or_admm(&P, 1, sweeps, f, d, c, rep) != 0)
            return -1;
        k += n;
        double r = rep[3], sd = rep[4];
        double ngf = 0.0, nd = 0.0, ntc = 0.0;
        or_diff(P.ny, P.nx, P.Q, P.w, f, g);
        for (int64_t i = 0; i < JN; ++i) {
            ngf += g[i] * g[i];
            nd += d[i] * d[i];
        }
        or_diff_adj(P.ny, P.nx, P.Q, P.w, c, t);
        for (int64_t j = 0; j < J; ++j)
            ntc += t[j] * t[j];
        double eps_pri = sqrt((double)JN) * eps_abs + eps_rel * fmax(sqrt(ngf), sqrt(nd));
        double eps_dual = sqrt((double)J) * eps_abs + eps_rel * P.lam * sqrt(ntc);
        int stop = r <= eps_pri && sd <= eps_dual;
        if (!stop) {
            double scale = 1.0;
            if (r > mu * sd) {
                P.lam *= tau;
                scale = 1.0 / tau;
            } else if (sd > mu * r) {
                P.lam /= tau;
                scale = tau;
            }
            if (scale != 1.0)
                for (int64_t i = 0; i < JN; ++i)
                    c[i] *= scale;
        }
        if (m < max_checks && hist) {
            hist[6 * m + 0] = k;
            hist[6 * m + 1] = r;
            hist[6 * m + 2] = sd;
            hist[6 * m + 3] = eps_pri;
            hist[6 * m + 4] = eps_dual;
            hist[6 * m + 5] = P.lam;
        }
        ++m;
        if (stop) {
            *converged = 1;
            break;
        }
    }
    *n_checks = m;
    *lam_out = P.lam;
    free(g);
    free(t);
    return k;
}

/* Flat-argument entry points for ctypes. */
static or_problem make_problem(int64_t I, int ny, int nx, int Q, const int64_t *rowptr,
                               const int32_t *col, const double *val, const double *y,
                               const double *r, const double *w, double beta, double lam,
                               int grouping)
{
    or_problem P;
    P.I = I; P.ny = ny; P.nx = nx; P.Q = Q;
    P.rowptr = rowptr; P.col = col; P.val = val;
    P.y = y; P.r = r; P.w = w;
    P.beta = beta; P.lam = lam; P.grouping = grouping;
    return P;
}

int or_admm_flat(int64_t I, int ny, int nx, int Q, const int64_t *rowptr, const int32_t *col,
                 const double *val, const double *y, const double *r, const double *w,
                 double beta, double lam, int grouping, int n_iter, int sweeps,
                 double *f, double *d, double *c, double *report)
{
    or_problem P = make_problem(I, ny, nx, Q, rowptr, col, val, y, r, w, beta, lam, grouping);
    return or_admm(&P, n_iter, sweeps, f, d, c, report);
}

int or_admm_adaptive_flat(int64_t I, int ny, int nx, int Q, const int64_t *rowptr,
                          const int32_t *col, const double *val, const double *y, const double *r,
                          const double *w, double beta, double lam, int grouping, int max_iter,
                          int sweeps, int check, double eps_abs, double eps_rel, double mu, double tau,
                          double *f, double *d, double *c, double *hist, int max_checks,
                          int *n_checks, double *lam_out, int *converged)
{
    or_problem P = make_problem(I, ny, nx, Q, rowptr, col, val, y, r, w, beta, lam, grouping);
    return or_admm_adaptive(&P, max_iter, sweeps, check, eps_abs, eps_rel, mu, tau, f, d, c, hist,
                            max_checks, n_checks, lam_out, converged);
}

void or_objective_flat(int64_t I, int ny, int nx, int Q, const int64_t *rowptr,
                       const int32_t *col, const double *val, const double *y, const double *r,
                       const double *w, double beta, int grouping, const double *f, double *out)
{
    or_problem P = make_problem(I, ny, nx, Q, rowptr, col, val, y, r, w, beta, 1.0, grouping);
    or_objective(&P, f, out);
}

void or_image_sweep_flat(int64_t I, int ny, int nx, int Q, const int64_t *rowptr,
                         const int32_t *col, const double *val, const double *y,
                         const double *r, const double *w, double lam, const double *z,
                         double *g)
{
    or_problem P = make_problem(I, ny, nx, Q, rowptr, col, val, y, r, w, 0.0, lam, 0);
    int64_t J = n_vox(&P);
    double *sens = malloc(sizeof(double) * (J > 0 ? J : 1));
    double *H = malloc(sizeof(double) * (J > 0 ? J : 1));
    or_sensitivity(&P, sens);
    or_curv(ny, nx, Q, w, lam, H);
    or_image_sweep(&P, sens, H, z, g);
    free(sens);
    free(H);
}

double or_plain_init_flat(int64_t I, int ny, int nx, int Q, const int64_t *rowptr,
                          const int32_t *col, const double *val, const double *y)
{
    or_problem P = make_problem(I, ny, nx, Q, rowptr, col, val, y, NULL, NULL, 0.0, 1.0, 0);
    return or_plain_init(&P);
}

/*
 * Reduced-precision storage of the system matrix: every column j gets the
 * FP32 scale sigma_j = max_i a_ij and every value the 16-bit code of the FP32
 * quotient a_ij / sigma_j, rounded to nearest-even (bfloat16: kind 1, IEEE
 * binary16: kind 2).  The quotient is formed in FP32 so that both sides round
 * the same number.  deq receives sigma_j * decode(code) in FP64, the matrix
 * the reduced-precision path effectively multiplies with.
 */
static uint16_t rne_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

static double bf16_value(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* binary16 from the IEEE 754 definition: 1 sign, 5 exponent (bias 15),
 * 10 fraction bits, subnormals below 2^-14; inputs here are finite, >= 0. */
static uint16_t rne_f16(float xf)
{
    double x = (double)xf;           /* exact */
    if (x == 0.0)
        return 0;
    int e;
    (void)frexp(x, &e);              /* x = m 2^e, m in [0.5, 1) */
    int E = e - 1;                   /* x = (2m) 2^E, 2m in [1, 2) */
    if (E < -14) {                   /* subnormal: units of 2^-24 */
        double q = x / ldexp(1.0, -24);
        double r = nearbyint(q);     /* round half to even (default mode) */
        return (uint16_t)r;          /* may round up into the normal range */
    }
    double q = ldexp(x, 10 - E);     /* in [1024, 2048) */
    double r = nearbyint(q);
    if (r == 2048.0) { r = 1024.0; E += 1; }
    if (E > 15)
        return 0x7C00;               /* overflow to infinity (not reached for a / max) */
    return (uint16_t)(((E + 15) << 10) | ((int)r - 1024));
}

static double f16_value(uint16_t h)
{
    int E = (h >> 10) & 0x1F, F = h & 0x3FF;
    if (E == 0)
        return ldexp((double)F, -24);
    return ldexp(1024.0 + F, E - 25);
}

void or_quantise(int64_t nnz, int64_t J, const int32_t *col, const float *val, int kind,
                 float *scale, uint16_t *codes, double *deq)
{
    for (int64_t j = 0; j < J; ++j)
        scale[j] = 0.0f;
    for (int64_t k = 0; k < nnz; ++k)
        if (val[k] > scale[col[k]])
            scale[col[k]] = val[k];
    for (int64_t k = 0; k < nnz; ++k) {
        float s = scale[col[k]];
        float t = s > 0.0f ? val[k] / s : 0.0f;
        uint16_t c = kind == 1 ? rne_bf16(t) : rne_f16(t);
        codes[k] = c;
        deq[k] = (double)s * (kind == 1 ? bf16_value(c) : f16_value(c));
    }
}
