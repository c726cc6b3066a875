"""Penalty changes and the adaptive iteration on the GPU against the FP64
oracle (residual balancing and the residual stopping rule of Boyd et al. 2011,
Sections 3.3 and 3.4.1).

The penalty decisions are integers decided by floating point: the cases below
were chosen so that every decision of the oracle clears its threshold by a
relative margin above 2e-3 (checked in the test), far above the rounding of
the FP32 residuals, so the GPU must take the same decisions at the same
iterations."""
import numpy as np
import pytest

import oracle
from paper_1601_08201_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_08201_amd import sgtv
    sgtv.lib()
    return sgtv


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def recon(sg, p, rho, grouping=0):
    R = sg.Reconstructor()
    R.set_system(p.I, p.ny, p.nx, p.Q, p.rowptr, p.col, p.val)
    if grouping:
        R.set_grouping(grouping)
    R.set_data(p.y, p.r, p.beta, rho, 1)
    return R


@pytest.mark.parametrize("grouping", [0, 1])
def test_penalty_change_keeps_unscaled_dual_and_matches_oracle(sg, grouping):
    p = datagen.make_problem("small", 4)
    R = recon(sg, p, 1.0, grouping)
    R.iterate(10)
    d0, c0 = R.split()
    R.set_penalty(0.25)
    assert R.penalty() == 0.25
    d1, c1 = R.split()
    assert rel_l2(d1, d0) <= 1e-6
    assert rel_l2(0.25 * c1.astype(np.float64), 1.0 * c0) <= 1e-4
    R.iterate(15)
    f, d, c, _ = oracle.admm(p, 10, grouping=grouping, report=False)
    f, d, c, _ = oracle.admm(p, 15, f0=f, d0=d, c0=c * 4.0, lam=0.25, grouping=grouping, report=False)
    err = rel_l2(R.image(), f)
    print("penalty change, grouping", grouping, "rel_l2", err, flush=True)
    assert err <= 1e-5
    R.close()


@pytest.mark.parametrize("seed,grouping,rho", [(0, 0, 1.0), (0, 1, 1.0), (1, 0, 0.01), (2, 0, 1.0)])
def test_adaptive_iteration_matches_oracle(sg, seed, grouping, rho):
    p = datagen.make_problem("small", seed)
    opt = dict(check=10, eps_abs=1e-4, eps_rel=1e-3, mu=10.0, tau=2.0)
    f_o, _, _, lam_o, hist, k_o, conv_o = oracle.admm_adaptive(p, 600, lam=rho, grouping=grouping, **opt)
    r, s, ep, ed = hist[:, 1], hist[:, 2], hist[:, 3], hist[:, 4]
    margin = min(np.min(np.abs(r - 10 * s) / (10 * s)), np.min(np.abs(s - 10 * r) / (10 * r)),
                 np.min(np.abs(r - ep) / ep), np.min(np.abs(s - ed) / ed))
    assert margin > 2e-3
    R = recon(sg, p, rho, grouping)
    out = R.iterate_adaptive(600, **opt)
    checks = out["checks"]
    print("seed", seed, "grouping", grouping, "iterations gpu/oracle", out["iterations"], k_o,
          "rho", R.penalty(), lam_o, flush=True)
    assert out["converged"] == conv_o and out["iterations"] == k_o
    assert [c["rho"] for c in checks] == list(hist[:, 5])
    for c, h in zip(checks, hist):
        assert c["iter"] == int(h[0])
        assert c["r_primal"] == pytest.approx(h[1], rel=1e-4)
        assert c["r_dual"] == pytest.approx(h[2], rel=1e-4)
        assert c["eps_primal"] == pytest.approx(h[3], rel=1e-5)
        assert c["eps_dual"] == pytest.approx(h[4], rel=1e-4)
    err = rel_l2(R.image(), f_o)
    print("  image rel_l2", err, flush=True)
    assert err <= 1e-5
    R.close()


def test_adaptive_argument_checks(sg):
    p = datagen.make_problem("small", 0)
    R = recon(sg, p, 1.0)
    with pytest.raises(sg.SgtvError):
        R.iterate_adaptive(10, check=0)
    with pytest.raises(sg.SgtvError):
        R.iterate_adaptive(10, tau=0.5)
    with pytest.raises(sg.SgtvError):
        R.iterate_adaptive(10, eps_abs=-1.0)
    with pytest.raises(sg.SgtvError):
        R.set_penalty(0.0)
    # tau = 1 and no stopping: plain iteration, bit for bit
    out = R.iterate_adaptive(25, check=10, eps_abs=0.0, eps_rel=0.0, tau=1.0)
    assert out["iterations"] == 25 and not out["converged"] and len(out["checks"]) == 3
    f_a = R.image()
    R.set_init(None)
    R.iterate(25)
    np.testing.assert_array_equal(f_a, R.image())
    R.close()
