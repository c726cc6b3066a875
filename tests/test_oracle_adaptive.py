"""Pins of the oracle's adaptive-penalty ADMM (residual balancing and the
residual stopping rule of Boyd et al. 2011, Sections 3.3 and 3.4.1), CPU only.

Residuals and tolerances are recomputed here from an explicitly assembled
difference operator, independently of the oracle's own loops.
"""
import numpy as np
import pytest

import oracle
from paper_1601_08201_amd import datagen
from test_oracle_pins import explicit_D


@pytest.fixture(scope="module")
def prob():
    return datagen.make_problem(dict(ny=6, nx=5, Q=4, I=256, nnz_per_col=12, rects=2, beta=0.2,
                                     rho=1.0), seed=3)


def test_tau_one_is_plain_admm(prob):
    """With tau = 1 and no stopping the adaptive run is plain ADMM, chunked."""
    f, d, c, lam, hist, k, conv = oracle.admm_adaptive(prob, 37, check=10, eps_abs=0.0, eps_rel=0.0,
                                                      mu=10.0, tau=1.0)
    f0, d0, c0, _ = oracle.admm(prob, 37, report=False)
    assert k == 37 and not conv and lam == prob.rho
    assert [int(h[0]) for h in hist] == [10, 20, 30, 37]
    np.testing.assert_array_equal(f, f0)
    np.testing.assert_array_equal(d, d0)
    np.testing.assert_array_equal(c, c0)


@pytest.mark.parametrize("grouping", [0, 1])
def test_rebalance_follows_residuals_and_keeps_unscaled_dual(prob, grouping):
    """One check after 10 iterations: the direction of the penalty change
    follows r and s recomputed from the states of iterations 9 and 10, the
    image and split are those of plain ADMM, and lam * c is unchanged."""
    D = explicit_D(prob.ny, prob.nx, prob.Q)
    _, d9, _, _ = oracle.admm(prob, 9, report=False, grouping=grouping)
    f10, d10, c10, _ = oracle.admm(prob, 10, report=False, grouping=grouping)
    r = np.linalg.norm(D @ f10 - d10)
    s = prob.rho * np.linalg.norm(D.T @ (d10 - d9))
    mu, tau = 1.5, 2.0
    f, d, c, lam, hist, k, _ = oracle.admm_adaptive(prob, 10, check=10, eps_abs=0.0, eps_rel=0.0,
                                                   mu=mu, tau=tau, grouping=grouping)
    assert hist[0, 1] == pytest.approx(r, rel=1e-12)
    assert hist[0, 2] == pytest.approx(s, rel=1e-12)
    want = prob.rho * (tau if r > mu * s else (1 / tau if s > mu * r else 1.0))
    assert lam == want and hist[0, 5] == want
    np.testing.assert_array_equal(f, f10)
    np.testing.assert_array_equal(d, d10)
    np.testing.assert_array_equal(lam * c, prob.rho * c10)


def test_stopping_rule_holds_when_the_run_stops(prob):
    eps_abs, eps_rel = 1e-4, 1e-3
    f, d, c, lam, hist, k, conv = oracle.admm_adaptive(prob, 3000, check=10, eps_abs=eps_abs,
                                                      eps_rel=eps_rel)
    assert conv and k < 3000 and k == int(hist[-1, 0])
    D = explicit_D(prob.ny, prob.nx, prob.Q)
    J = prob.ny * prob.nx * prob.Q
    gf = D @ f
    eps_pri = np.sqrt(4 * J) * eps_abs + eps_rel * max(np.linalg.norm(gf), np.linalg.norm(d))
    eps_dual = np.sqrt(J) * eps_abs + eps_rel * lam * np.linalg.norm(D.T @ c)
    assert hist[-1, 3] == pytest.approx(eps_pri, rel=1e-12)
    assert hist[-1, 4] == pytest.approx(eps_dual, rel=1e-12)
    assert np.linalg.norm(gf - d) == pytest.approx(hist[-1, 1], rel=1e-12)
    assert hist[-1, 1] <= eps_pri and hist[-1, 2] <= eps_dual
    # the check before did not meet both tolerances
    assert hist[-2, 1] > hist[-2, 3] or hist[-2, 2] > hist[-2, 4]


def test_adaptive_and_fixed_penalty_reach_the_same_minimiser():
    p = datagen.make_problem(dict(ny=4, nx=4, Q=3, I=96, nnz_per_col=10, rects=2, beta=0.3, rho=1.0),
                             seed=8)
    f_a, _, _, lam, hist, k, conv = oracle.admm_adaptive(p, 6000, check=10, eps_abs=1e-10,
                                                          eps_rel=1e-10)
    f_p, _, _, _ = oracle.admm(p, 6000, report=False)
    phi_a = oracle.objective(p, f_a)[0]
    phi_p = oracle.objective(p, f_p)[0]
    print("adaptive stopped after", k, "iterations, lam", lam, "objectives", phi_a, phi_p)
    assert phi_a == pytest.approx(phi_p, rel=1e-7)
    assert np.linalg.norm(f_a - f_p) <= 1e-3 * np.linalg.norm(f_p)
