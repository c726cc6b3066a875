"""Pins of the FP64 oracle against facts fixed by the mathematics (CPU only).

Each test checks one step of the method against something other than the
oracle itself: a library routine, an explicitly assembled operator, a closed
form, a 1-D numerical minimisation, an invariant of the iteration, or brute
force on tiny problems.  Constructions here are written independently of the
oracle's loops (geometric offsets, explicit sparse matrices, scipy solvers).
"""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import oracle
from paper_1601_08201_amd import datagen

OFFS = [(0, 1), (0, -1), (1, 0), (-1, 0)]   # (dy, dx) of directions +x, -x, +y, -y


def explicit_D(ny, nx, Q, w=None):
    """Stacked difference operator assembled as a sparse matrix, rows (s, p, q)."""
    rows, cols, vals = [], [], []
    for iy in range(ny):
        for ix in range(nx):
            s = iy * nx + ix
            for p, (dy, dx) in enumerate(OFFS):
                jy, jx = iy + dy, ix + dx
                for q in range(Q):
                    rho = (s * 4 + p) * Q + q
                    wt = 1.0 if w is None else w[rho]
                    rows.append(rho); cols.append(s * Q + q); vals.append(wt)
                    if 0 <= jy < ny and 0 <= jx < nx:
                        rows.append(rho); cols.append((jy * nx + jx) * Q + q); vals.append(-wt)
    return sp.csr_matrix((vals, (rows, cols)), shape=(ny * nx * Q * 4, ny * nx * Q))


def rand_csr(rng, I, J, density=0.3, empty_rows=(), empty_cols=()):
    A = sp.random(I, J, density=density, random_state=np.random.RandomState(rng.integers(1 << 30)),
                  format="csr", dtype=np.float64)
    A = A.tolil()
    for i in empty_rows:
        A[i, :] = 0
    for j in empty_cols:
        A[:, j] = 0
    A = A.tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    A.data = A.data.astype(np.float32).astype(np.float64)
    return A


def group_tv(ny, nx, Q, f, grouping=0):
    """R of Eq. 2 with w = 1 from numpy shifts of the [ny, nx, Q] image."""
    x = f.reshape(ny, nx, Q)
    pad = np.zeros((ny + 2, nx + 2, Q))
    pad[1:-1, 1:-1] = x
    diffs = [x - pad[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx] for dy, dx in OFFS]
    sq = sum(d * d for d in diffs)                  # [ny, nx, Q]
    return np.sqrt(sq.sum(axis=2)).sum() if grouping == 0 else np.sqrt(sq).sum()


def tiny_problem(seed, ny=2, nx=2, Q=2, I=8, beta=0.1, lam=1.0, dense=True):
    rng = np.random.default_rng(seed)
    J = ny * nx * Q
    A = rng.random((I, J)) * (rng.random((I, J)) < (1.0 if dense else 0.5))
    A = A.astype(np.float32).astype(np.float64)
    x = rng.uniform(0, 5, J)
    y = rng.poisson(A @ x + 0.1).astype(np.float64)
    csr = sp.csr_matrix(A)
    csr.sort_indices()
    return datagen.Problem(ny=ny, nx=nx, Q=Q, I=I, rowptr=csr.indptr.astype(np.int64),
                           col=csr.indices.astype(np.int32), val=csr.data, y=y,
                           r=np.full(I, 0.1), x_true=x.astype(np.float32), beta=beta, rho=lam,
                           iters=0, sweeps=1), A


# --- P5: projections against scipy.sparse -----------------------------------------------

@pytest.mark.parametrize("I,J", [(7, 11), (30, 20), (1, 5), (5, 1)])
def test_projections_match_scipy(I, J):
    rng = np.random.default_rng(I * 100 + J)
    A = rand_csr(rng, I, J, empty_rows=(0,) if I > 1 else (), empty_cols=(J - 1,) if J > 1 else ())
    f = rng.random(J)
    r = rng.random(I)
    t = rng.random(I)
    p = oracle.forward(A.indptr, A.indices, A.data, f, r)
    e = oracle.back(A.indptr, A.indices, A.data, t, J)
    np.testing.assert_allclose(p, A @ f + r, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(e, A.T @ t, rtol=1e-14, atol=1e-15)


def test_projections_on_generated_system():
    prob = datagen.make_problem(dict(ny=4, nx=3, Q=5, I=50, nnz_per_col=6, rects=2), seed=3)
    A = prob.csr().astype(np.float64)
    f = prob.x_true.astype(np.float64)
    np.testing.assert_allclose(oracle.forward(prob.rowptr, prob.col, prob.val, f, prob.r),
                               A @ f + prob.r.astype(np.float64), rtol=1e-14)
    np.testing.assert_allclose(oracle.back(prob.rowptr, prob.col, prob.val, prob.y, prob.J),
                               A.T @ prob.y.astype(np.float64), rtol=1e-14)


# --- P4: finite differences --------------------------------------------------------------

@pytest.mark.parametrize("ny,nx,Q", [(1, 1, 1), (1, 5, 3), (4, 3, 2), (3, 3, 1), (5, 2, 4)])
@pytest.mark.parametrize("weighted", [False, True])
def test_diff_matches_explicit_operator(ny, nx, Q, weighted):
    rng = np.random.default_rng(ny * 31 + nx * 7 + Q)
    w = rng.uniform(0.5, 2.0, ny * nx * Q * 4) if weighted else None
    D = explicit_D(ny, nx, Q, w)
    f = rng.normal(size=ny * nx * Q)
    t = rng.normal(size=ny * nx * Q * 4)
    np.testing.assert_allclose(oracle.diff(ny, nx, Q, f, w), D @ f, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(oracle.diff_adj(ny, nx, Q, t, w), D.T @ t, rtol=1e-13, atol=1e-13)
    lhs = np.dot(oracle.diff(ny, nx, Q, f, w), t)
    rhs = np.dot(f, oracle.diff_adj(ny, nx, Q, t, w))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_per_direction_weights_expand():
    ny, nx, Q = 3, 4, 2
    w4 = np.array([1.0, 2.0, 0.5, 3.0])
    full = np.broadcast_to(w4[None, :, None], (ny * nx, 4, Q)).ravel()
    f = np.random.default_rng(0).normal(size=ny * nx * Q)
    np.testing.assert_array_equal(oracle.diff(ny, nx, Q, f, w4), oracle.diff(ny, nx, Q, f, full))


# --- P3: De Pierro curvature ------------------------------------------------------------

@pytest.mark.parametrize("ny,nx,Q", [(1, 1, 2), (1, 4, 1), (3, 4, 3), (5, 5, 1)])
def test_curvature_closed_form(ny, nx, Q):
    lam = 1.7
    H = oracle.curvature(ny, nx, Q, lam)
    D = explicit_D(ny, nx, Q)
    absD = abs(D)
    expl = lam * (absD.T @ (absD @ np.ones(ny * nx * Q)))
    np.testing.assert_allclose(H, expl, rtol=1e-15)
    n_in = np.zeros((ny, nx))
    for iy in range(ny):
        for ix in range(nx):
            n_in[iy, ix] = sum(0 <= iy + dy < ny and 0 <= ix + dx < nx for dy, dx in OFFS)
    closed = lam * (3 * np.repeat(n_in.ravel(), Q) + 4)
    np.testing.assert_allclose(H, closed, rtol=1e-15)


def test_curvature_weighted_matches_explicit():
    ny, nx, Q = 3, 2, 2
    w = np.random.default_rng(5).uniform(0.2, 3.0, ny * nx * Q * 4)
    D = abs(explicit_D(ny, nx, Q, w))
    np.testing.assert_allclose(oracle.curvature(ny, nx, Q, 0.5, w),
                               0.5 * (D.T @ (D @ np.ones(ny * nx * Q))), rtol=1e-14)


def test_curvature_majorises_penalty():
    """(lam/2)||D f - z||^2 <= its separable De Pierro surrogate, equality at the expansion point."""
    ny, nx, Q, lam = 3, 3, 2, 1.3
    rng = np.random.default_rng(7)
    D = explicit_D(ny, nx, Q)
    H = oracle.curvature(ny, nx, Q, lam)
    fn = rng.random(ny * nx * Q)
    z = rng.normal(size=D.shape[0])
    pen = lambda f: 0.5 * lam * np.sum((D @ f - z) ** 2)
    grad = lam * (D.T @ (D @ fn - z))
    for _ in range(50):
        f = rng.random(ny * nx * Q) * 3
        sur = pen(fn) + grad @ (f - fn) + 0.5 * np.sum(H * (f - fn) ** 2)
        assert sur >= pen(f) - 1e-12
    # a majoriser with the wrong curvature (half of H) fails somewhere
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    checker = np.repeat(((-1.0) ** (iy + ix)).ravel(), Q)
    f = fn + checker
    assert pen(fn) + grad @ (f - fn) + 0.25 * np.sum(H * (f - fn) ** 2) < pen(f)


# --- P2 / P7: per-voxel root ------------------------------------------------------------

def phi(t, s, C, H, fn, gam):
    return s * t - (C * math.log(t) if C > 0 else 0.0) + 0.5 * H * (t - fn) ** 2 + gam * (t - fn)


@pytest.mark.parametrize("seed", range(40))
def test_root_minimises_voxel_surrogate(seed):
    rng = np.random.default_rng(seed)
    s, H, fn = rng.uniform(0, 20), rng.uniform(0.5, 16), rng.uniform(0, 10)
    e = rng.uniform(0, 30) if seed % 5 else 0.0
    gam = rng.normal(scale=20)
    if seed % 7 == 0:
        fn = 0.0
    C = fn * e
    B = s + gam - H * fn
    t = oracle.root(H, B, C)
    assert t >= 0.0
    hi = max(10.0, 4 * t + 10)
    res = so.minimize_scalar(lambda u: phi(u, s, C, H, fn, gam), bounds=(1e-300 if C > 0 else 0.0, hi),
                             method="bounded", options=dict(xatol=1e-13))
    assert abs(res.x - t) <= 1e-6 * max(1.0, t)
    assert phi(t, s, C, H, fn, gam) <= res.fun + 1e-12 * max(1.0, abs(res.fun))
    if t > 0:
        assert abs(H * t * t + B * t - C) <= 1e-10 * max(1.0, C, abs(B) * t, H * t * t)


def test_root_reduces_to_mlem_without_curvature():
    """H = 0: the surrogate is the EM one alone and the update is f e / s (MLEM with background)."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        s, f, e = rng.uniform(0.1, 10), rng.uniform(0, 5), rng.uniform(0, 5)
        assert oracle.root(0.0, s, f * e) == pytest.approx(f * e / s, rel=1e-15)


def test_root_stable_branches():
    # large |B|, tiny C: both branches must keep relative accuracy
    assert oracle.root(1.0, 1e8, 1.0) == pytest.approx(1e-8, rel=1e-12)
    assert oracle.root(1.0, -1e8, 1.0) == pytest.approx(1e8, rel=1e-12)
    assert oracle.root(2.0, 0.0, 8.0) == pytest.approx(2.0, rel=1e-15)
    assert oracle.root(3.0, 5.0, 0.0) == 0.0
    assert oracle.root(3.0, -6.0, 0.0) == pytest.approx(2.0, rel=1e-15)


# --- P1: group shrinkage ----------------------------------------------------------------

@pytest.mark.parametrize("grouping", [0, 1])
def test_shrink_is_the_prox(grouping):
    ny, nx, Q = 2, 3, 3
    rng = np.random.default_rng(11 + grouping)
    v = rng.normal(size=ny * nx * Q * 4)
    v[:4 * Q] = 0.0                         # an empty group
    thr = 0.9
    d = oracle.shrink(ny, nx, Q, thr, v, grouping)
    groups = ([np.arange(s * 4 * Q, (s + 1) * 4 * Q) for s in range(ny * nx)] if grouping == 0 else
              [np.array([(s * 4 + p) * Q + q for p in range(4)]) for s in range(ny * nx) for q in range(Q)])
    for g in groups:
        vg, dg = v[g], d[g]
        nv = np.linalg.norm(vg)
        # optimality of min thr*||u|| + 0.5||u - v||^2
        if np.linalg.norm(dg) > 0:
            np.testing.assert_allclose(vg - dg, thr * dg / np.linalg.norm(dg), rtol=1e-13, atol=1e-14)
        else:
            assert nv <= thr + 1e-15
        # brute-force prox along the direction of v
        if nv > 0:
            res = so.minimize_scalar(lambda a: thr * abs(a) + 0.5 * (a - nv) ** 2,
                                     bounds=(-1, nv + 1), method="bounded", options=dict(xatol=1e-12))
            np.testing.assert_allclose(np.linalg.norm(dg), max(res.x, 0.0), atol=1e-8)


def test_shrink_general_prox_by_minimisation():
    rng = np.random.default_rng(2)
    v = rng.normal(size=4 * 3)                # one spatial bin, Q = 3
    d = oracle.shrink(1, 1, 3, 0.7, v, 0)
    assert np.linalg.norm(v) > 0.7
    obj = lambda u: 0.7 * np.linalg.norm(u) + 0.5 * np.sum((u - v) ** 2)
    jac = lambda u: 0.7 * u / np.linalg.norm(u) + (u - v)
    res = so.minimize(obj, np.full_like(v, 0.01), jac=jac, method="BFGS", options=dict(gtol=1e-12))
    assert obj(d) <= res.fun + 1e-12
    np.testing.assert_allclose(d, res.x, atol=1e-7)


def test_shrink_tie_gives_zero():
    v = np.zeros(4 * 2)
    v[0] = 0.5
    np.testing.assert_array_equal(oracle.shrink(1, 1, 2, 0.5, v, 0), np.zeros_like(v))


# --- objective pieces -------------------------------------------------------------------

def test_group_tv_and_standard_tv_match_numpy():
    ny, nx, Q = 4, 5, 3
    f = np.random.default_rng(3).random(ny * nx * Q)
    g = oracle.diff(ny, nx, Q, f)
    assert oracle.group_norm_sum(ny, nx, Q, g, 0) == pytest.approx(group_tv(ny, nx, Q, f, 0), rel=1e-14)
    assert oracle.group_norm_sum(ny, nx, Q, g, 1) == pytest.approx(group_tv(ny, nx, Q, f, 1), rel=1e-14)
    # Q = 1: spectral grouping is classic isotropic TV over the four differences
    f1 = f[: ny * nx]
    g1 = oracle.diff(ny, nx, 1, f1)
    assert oracle.group_norm_sum(ny, nx, 1, g1, 0) == oracle.group_norm_sum(ny, nx, 1, g1, 1)


def test_data_term_is_shifted_negative_loglik():
    """I-divergence = NLL(p) - NLL(y) where NLL(m) = sum m - y log m (0 log 0 = 0)."""
    rng = np.random.default_rng(4)
    y = rng.poisson(3.0, 50).astype(float)
    y[:5] = 0
    p = rng.uniform(0.1, 8, 50)
    nll = lambda m: np.sum(m) - np.sum(np.where(y > 0, y * np.log(np.where(y > 0, m, 1)), 0))
    assert oracle.data_term(p, y) == pytest.approx(nll(p) - nll(y), rel=1e-13)
    assert oracle.data_term(y + (y == 0), y) >= 0


# --- P6: optimisation transfer of the image update -----------------------------------------

def psi(prob, A, D, f, z, lam):
    p = A @ f + prob.r
    return np.sum(p - prob.y * np.log(p)) + 0.5 * lam * np.sum((D @ f - z) ** 2)


@pytest.mark.parametrize("seed", range(4))
def test_image_sweeps_descend_and_reach_subproblem_minimiser(seed):
    prob, A = tiny_problem(seed, ny=2, nx=3, Q=2, I=10, dense=False)
    D = explicit_D(prob.ny, prob.nx, prob.Q)
    rng = np.random.default_rng(100 + seed)
    z = rng.normal(scale=0.5, size=D.shape[0])
    g = rng.uniform(0.1, 3, prob.J)
    vals = [psi(prob, A, D, g, z, 1.0)]
    for _ in range(3000):
        g = oracle.image_sweep(prob, g, z, lam=1.0)
        assert np.all(g >= 0)
        vals.append(psi(prob, A, D, g, z, 1.0))
    assert np.all(np.diff(vals) <= 1e-12 * np.abs(vals[1:]))
    # Minimiser of the image subproblem (Eq. 4 over f >= 0) by L-BFGS-B
    fun = lambda f: psi(prob, A, D, f, z, 1.0)
    jac = lambda f: A.T @ (1 - prob.y / (A @ f + prob.r)) + D.T @ (D @ f - z)
    res = so.minimize(fun, np.ones(prob.J), jac=jac, method="L-BFGS-B",
                      bounds=[(0, None)] * prob.J, options=dict(ftol=1e-15, gtol=1e-12, maxiter=10000))
    assert vals[-1] <= res.fun + 1e-9 * abs(res.fun)
    np.testing.assert_allclose(g, res.x, atol=2e-4)


def test_em_surrogate_majorises_likelihood():
    """The EM surrogate plus constant touches L at g and lies above it elsewhere: checked through
    the monotone decrease of L under H -> 0 sweeps (MLEM) on a random problem."""
    prob, A = tiny_problem(9, ny=1, nx=1, Q=6, I=9)
    p0 = lambda f: np.sum(A @ f + prob.r - prob.y * np.log(A @ f + prob.r))
    f = np.ones(prob.J)
    s = A.T @ np.ones(prob.I)
    prev = p0(f)
    for _ in range(200):
        e = A.T @ (prob.y / (A @ f + prob.r))
        f = np.array([oracle.root(0.0, s[j], f[j] * e[j]) for j in range(prob.J)])
        cur = p0(f)
        assert cur <= prev + 1e-12 * abs(prev)
        prev = cur


# --- P8 / P10 / A10: special cases ---------------------------------------------------------

def test_identity_system_without_penalty_gives_clipped_data():
    ny, nx, Q = 2, 2, 3
    J = ny * nx * Q
    rng = np.random.default_rng(8)
    y = rng.poisson(2.0, J).astype(float)
    r = np.full(J, 0.5)
    prob = datagen.Problem(ny=ny, nx=nx, Q=Q, I=J, rowptr=np.arange(J + 1, dtype=np.int64),
                           col=np.arange(J, dtype=np.int32), val=np.ones(J), y=y, r=r,
                           x_true=np.zeros(J, np.float32), beta=0.0, rho=1.0, iters=0, sweeps=1)
    f, d, c, rep = oracle.admm(prob, 4000)
    np.testing.assert_allclose(f, np.maximum(y - r, 0), atol=1e-7)


def test_zero_counts_give_zero_image():
    prob, A = tiny_problem(1)
    prob.y = np.zeros(prob.I)
    assert oracle.plain_init(prob) == 0.0
    f, d, c, rep = oracle.admm(prob, 20)
    assert np.all(f == 0)
    assert rep[-1, 0] == pytest.approx(np.sum(prob.r))


def test_zero_image_is_a_fixed_point():
    """With the EM surrogate f = 0 never moves (every voxel has C = 0 and B = s > 0)."""
    prob, A = tiny_problem(2)
    f, d, c, rep = oracle.admm(prob, 10, f0=np.zeros(prob.J))
    assert np.all(f == 0)


def test_plain_init_matches_counts():
    prob, A = tiny_problem(3)
    kappa = oracle.plain_init(prob)
    assert kappa == pytest.approx(prob.y.sum() / A.sum(), rel=1e-14)


def test_q1_group_and_standard_tv_coincide():
    prob = datagen.make_problem(dict(ny=5, nx=4, Q=1, I=30, nnz_per_col=5, rects=2), seed=2)
    a = oracle.admm(prob, 30, grouping=0)
    b = oracle.admm(prob, 30, grouping=1)
    np.testing.assert_array_equal(a[0], b[0])


# --- P11 / P12: converged value by brute force and KKT ------------------------------------

def smoothed_objective(prob, A, D, eps, beta):
    S, Q = prob.ny * prob.nx, prob.Q
    # group index of every row of D: spatial bin s
    grp = np.repeat(np.arange(S), 4 * Q)

    def fun(f):
        p = A @ f + prob.r
        data = np.sum(p - prob.y + np.where(prob.y > 0, prob.y * np.log(np.where(prob.y > 0, prob.y, 1) / p), 0))
        g = D @ f
        nrm = np.sqrt(np.bincount(grp, g * g, minlength=S) + eps * eps)
        val = data + beta * nrm.sum()
        grad = A.T @ (1 - prob.y / p) + beta * (D.T @ (g / nrm[grp]))
        return val, grad
    return fun


@pytest.mark.parametrize("seed,shape", [(0, (2, 2, 2)), (1, (2, 3, 2)), (2, (1, 4, 3)), (3, (3, 3, 1))])
def test_converged_value_brackets_brute_force(seed, shape):
    ny, nx, Q = shape
    J = ny * nx * Q
    prob, A = tiny_problem(seed, ny=ny, nx=nx, Q=Q, I=max(6, J - 2), beta=0.5)
    D = explicit_D(ny, nx, Q)
    f, d, c, rep = oracle.admm(prob, 20000)
    phi_admm = oracle.objective(prob, f)[0]
    S = ny * nx
    eps = 1e-5
    fun = smoothed_objective(prob, A, D, eps, prob.beta)
    best = None
    for x0 in (np.ones(J), f + 1e-3, np.full(J, 3.0)):
        res = so.minimize(fun, x0, jac=True, method="L-BFGS-B", bounds=[(0, None)] * J,
                          options=dict(ftol=1e-16, gtol=1e-13, maxiter=50000, maxcor=30))
        best = res.fun if best is None else min(best, res.fun)
    # min Phi lies in [min Phi_eps - beta*S*eps, min Phi_eps]; ADMM must land there
    tol = 1e-9 * abs(best)
    assert phi_admm <= best + tol
    assert phi_admm >= best - prob.beta * S * eps - tol


@pytest.mark.parametrize("seed", [0, 4])
def test_kkt_at_convergence(seed):
    prob, A = tiny_problem(seed, ny=2, nx=3, Q=2, I=10, beta=0.3)
    D = explicit_D(prob.ny, prob.nx, prob.Q)
    lam = prob.rho
    f, d, c, rep = oracle.admm(prob, 30000)
    grad = A.T @ (1 - prob.y / (A @ f + prob.r)) + lam * (D.T @ c)
    tol = 1e-7
    pos = f > 1e-9
    assert np.all(np.abs(grad[pos]) <= tol)
    assert np.all(grad[~pos] >= -tol)
    assert np.linalg.norm(D @ f - d) <= tol
    Q = prob.Q
    for s in range(prob.ny * prob.nx):
        sl = slice(s * 4 * Q, (s + 1) * 4 * Q)
        assert lam * np.linalg.norm(c[sl]) <= prob.beta + tol
        nd = np.linalg.norm(d[sl])
        if nd > 1e-9:
            np.testing.assert_allclose(lam * c[sl], prob.beta * d[sl] / nd, atol=tol)
    # residuals reported by the oracle vanish
    assert rep[-1, 3] <= tol and rep[-1, 4] <= tol


def groups_of_rows(ny, nx, Q, grouping):
    """Group of every row (s, p, q) of D: the spatial bin s (spectral grouping)
    or the voxel (s, q) (standard TV), and the number of groups."""
    rho = np.arange(ny * nx * 4 * Q)
    s, q = rho // (4 * Q), rho % Q
    return (s, ny * nx) if grouping == 0 else (s * Q + q, ny * nx * Q)


def smoothed_objective_general(prob, A, D, eps, beta, grp, n_groups):
    def fun(f):
        p = A @ f + prob.r
        data = np.sum(p - prob.y + np.where(prob.y > 0, prob.y * np.log(np.where(prob.y > 0, prob.y, 1) / p), 0))
        g = D @ f
        nrm = np.sqrt(np.bincount(grp, g * g, minlength=n_groups) + eps * eps)
        return data + beta * nrm.sum(), A.T @ (1 - prob.y / p) + beta * (D.T @ (g / nrm[grp]))
    return fun


W4 = np.array([1.0, 0.7, 1.3, 0.9])


@pytest.mark.parametrize("seed,shape,grouping,weighted", [(5, (2, 2, 2), 1, False), (6, (2, 3, 2), 1, False),
                                                          (7, (2, 2, 3), 0, True), (8, (1, 3, 2), 1, True)])
def test_converged_value_brackets_brute_force_standard_tv_and_weights(seed, shape, grouping, weighted):
    """P11 for standard TV (groups of four differences per voxel) and for
    direction weights (w G f in the penalty and in the constraint)."""
    ny, nx, Q = shape
    J = ny * nx * Q
    prob, A = tiny_problem(seed, ny=ny, nx=nx, Q=Q, I=max(6, J - 2), beta=0.5)
    w4 = W4 if weighted else None
    wfull = np.broadcast_to(W4[None, :, None], (ny * nx, 4, Q)).ravel() if weighted else None
    D = explicit_D(ny, nx, Q, wfull)
    grp, n_groups = groups_of_rows(ny, nx, Q, grouping)
    f, d, c, rep = oracle.admm(prob, 20000, w=w4, grouping=grouping)
    phi_admm = oracle.objective(prob, f, w=w4, grouping=grouping)[0]
    eps = 1e-5
    fun = smoothed_objective_general(prob, A, D, eps, prob.beta, grp, n_groups)
    best = None
    for x0 in (np.ones(J), f + 1e-3, np.full(J, 3.0)):
        res = so.minimize(fun, x0, jac=True, method="L-BFGS-B", bounds=[(0, None)] * J,
                          options=dict(ftol=1e-16, gtol=1e-13, maxiter=50000, maxcor=30))
        best = res.fun if best is None else min(best, res.fun)
    tol = 1e-9 * abs(best)
    assert phi_admm <= best + tol
    assert phi_admm >= best - prob.beta * n_groups * eps - tol


@pytest.mark.parametrize("seed,grouping,weighted", [(9, 1, False), (10, 0, True), (11, 1, True)])
def test_kkt_at_convergence_standard_tv_and_weights(seed, grouping, weighted):
    """P12 for standard TV and direction weights: stationarity with D the
    weighted operator, d = D f, and per group lam ||c_g|| <= beta with
    lam c_g = beta d_g / ||d_g|| where d_g is not zero."""
    prob, A = tiny_problem(seed, ny=2, nx=3, Q=2, I=10, beta=0.3)
    ny, nx, Q = prob.ny, prob.nx, prob.Q
    w4 = W4 if weighted else None
    wfull = np.broadcast_to(W4[None, :, None], (ny * nx, 4, Q)).ravel() if weighted else None
    D = explicit_D(ny, nx, Q, wfull)
    lam = prob.rho
    f, d, c, rep = oracle.admm(prob, 30000, w=w4, grouping=grouping)
    grad = A.T @ (1 - prob.y / (A @ f + prob.r)) + lam * (D.T @ c)
    tol = 1e-7
    pos = f > 1e-9
    assert np.all(np.abs(grad[pos]) <= tol)
    assert np.all(grad[~pos] >= -tol)
    assert np.linalg.norm(D @ f - d) <= tol
    grp, n_groups = groups_of_rows(ny, nx, Q, grouping)
    for gi in range(n_groups):
        idx = grp == gi
        assert lam * np.linalg.norm(c[idx]) <= prob.beta + tol
        nd = np.linalg.norm(d[idx])
        if nd > 1e-9:
            np.testing.assert_allclose(lam * c[idx], prob.beta * d[idx] / nd, atol=tol)
    assert rep[-1, 3] <= tol and rep[-1, 4] <= tol


def test_report_matches_definitions():
    prob, A = tiny_problem(6, ny=2, nx=2, Q=3, I=9, beta=0.2)
    D = explicit_D(prob.ny, prob.nx, prob.Q)
    f0 = np.full(prob.J, oracle.plain_init(prob))
    f1, d1, c1, rep1 = oracle.admm(prob, 1, f0=f0)
    f2, d2, c2, rep2 = oracle.admm(prob, 1, f0=f1, d0=d1, c0=c1)
    p = A @ f2 + prob.r
    data = np.sum(p - prob.y + np.where(prob.y > 0, prob.y * np.log(np.where(prob.y > 0, prob.y, 1) / p), 0))
    tv = group_tv(prob.ny, prob.nx, prob.Q, f2)
    np.testing.assert_allclose(rep2[0, :3], [data + prob.beta * tv, data, tv], rtol=1e-13)
    np.testing.assert_allclose(rep2[0, 3], np.linalg.norm(D @ f2 - d2), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(rep2[0, 4], prob.rho * np.linalg.norm(D.T @ (d2 - d1)), rtol=1e-12, atol=1e-15)
    # dual update of Eq. 6
    np.testing.assert_allclose(c2, c1 + D @ f2 - d2, atol=1e-13)


def test_split_runs_equal_one_run_and_are_deterministic():
    prob = datagen.make_problem("small", seed=0)
    a = oracle.admm(prob, 6)
    b1 = oracle.admm(prob, 3)
    b = oracle.admm(prob, 3, f0=b1[0], d0=b1[1], c0=b1[2])
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    a2 = oracle.admm(prob, 6)
    for x, y in zip(a[:4], a2[:4]):
        np.testing.assert_array_equal(x, y)


def test_objective_decreases_on_small_workload():
    prob = datagen.make_problem("small", seed=1)
    f, d, c, rep = oracle.admm(prob, 50)
    assert rep[-1, 0] < rep[0, 0]
    assert np.all(f >= 0)
