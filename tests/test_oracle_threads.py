"""Determinism of the oracle across thread counts.

The oracle shares its loops over independent outputs (rows, columns, voxels,
groups) among OpenMP threads; every sum keeps the serial order and the
reductions over many outputs stay serial, so an ADMM run gives bitwise the
same image, split, dual and report at one thread and at many."""
import numpy as np
import pytest

import oracle
from paper_1601_08201_amd import datagen


@pytest.fixture
def threads():
    n0 = oracle.max_threads()
    yield max(4, n0)
    oracle.set_threads(n0)


@pytest.mark.parametrize("cfg,seed,kw", [("small", 0, {}), ("small", 5, {"grouping": 1}),
                                         ("teflon", 1, {"weights": True}),
                                         (dict(ny=5, nx=11, Q=7, I=300, nnz_per_col=6, rects=2),
                                          2, {"sweeps": 3})])
def test_admm_bitwise_equal_across_thread_counts(threads, cfg, seed, kw):
    prob = datagen.make_problem(cfg, seed)
    args = dict(grouping=kw.get("grouping", 0), sweeps=kw.get("sweeps", 1))
    if kw.get("weights"):
        args["w"] = prob.meta["weights"]
    runs = []
    for n in (1, threads):
        oracle.set_threads(n)
        runs.append(oracle.admm(prob, 25, report=True, **args))
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)


def test_projections_and_adjoint_bitwise_equal_across_thread_counts(threads):
    prob = datagen.make_problem("small", 7)
    rng = np.random.default_rng(7)
    f = rng.uniform(0, 2, prob.J)
    t = rng.normal(size=4 * prob.J)
    out = []
    for n in (1, threads):
        oracle.set_threads(n)
        out.append((oracle.forward(prob.rowptr, prob.col, prob.val, f, prob.r),
                    oracle.diff(prob.ny, prob.nx, prob.Q, f),
                    oracle.diff_adj(prob.ny, prob.nx, prob.Q, t),
                    oracle.objective(prob, f)))
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)
