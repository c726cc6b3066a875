"""Learned warm start end to end on the 64x64x64 scanner: the network trained
on plain reconstructions gives start images whose objective is below the
uniform start's (so the fallback is not taken), reaches a 1e-2 relative
objective gap in fewer iterations than the uniform start, and every run still
reaches the 1e-4 target (the iteration counts at 1e-4 are printed: on this
scanner the learned start needs more of them, see the design notes)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_learned_start_against_uniform_start():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_08201_amd import warmstart
    scanner = warmstart.make_scanner(1)
    xin, tgt, _ = warmstart.make_dataset(scanner, range(10000, 10512), iters=300)
    model, net, hist = warmstart.train(xin, tgt, epochs=40)
    print("training loss", hist[0], "->", hist[-1], flush=True)
    assert hist[-1] < 0.5 * hist[0]
    rc = warmstart.Reconstruction(scanner)
    R = rc.R
    tols = (1e-2, 1e-4)
    plain, learned = [], []
    for (_, y, r) in warmstart.draw_scans(scanner, range(20000, 20012)):
        rc.load(y, r)
        phi_star, _ = warmstart.converged_objective(R)
        R.set_init(None)
        phi_u = R.objective()["total"]
        it_p, _ = warmstart.iterations_to_targets(R, phi_star, tols)
        x0 = warmstart.predict(net, model, R.backprojection().reshape(1, 64, 64, 64)).reshape(-1)
        assert np.all(np.isfinite(x0)) and np.all(x0 >= 0)
        R.set_init_dual(x0)
        phi_n = R.objective()["total"]
        assert phi_n < phi_u            # no fallback needed
        it_l, _ = warmstart.iterations_to_targets(R, phi_star, tols)
        assert it_p[-1] is not None and it_l[-1] is not None
        plain.append(it_p)
        learned.append(it_l)
    plain, learned = np.array(plain, float), np.array(learned, float)
    print("median iterations to 1e-2 / 1e-4: plain", np.median(plain, 0), "learned", np.median(learned, 0),
          flush=True)
    assert np.median(learned[:, 0]) < np.median(plain[:, 0])
