"""Learned warm start end to end on the 64x64x64 scanner.

The network is trained on 1024 phantoms to map the image after 10 plain
iterations to a per-voxel correction factor towards the 300-iteration image.
On held-out phantoms the start it gives is taken (no fallback) and reaches the
1e-2 and 1e-4 relative objective gaps in fewer iterations, the 10 plain ones
included, than the uniform start.  A start made worse on purpose (output
scale 1000) is refused by the fallback, and the run then continues exactly as
the plain run.
"""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_08201_amd import warmstart
    scanner = warmstart.make_scanner(1)
    xin, tgt, _ = warmstart.make_dataset(scanner, range(10000, 11024), iters=300, input_iters=(10,))
    model, net, hist = warmstart.train(xin[10], tgt, mode="ratio", input_iters=10, epochs=40)
    print("training loss", hist[0], "->", hist[-1], flush=True)
    assert hist[-1] < hist[0]
    return scanner, model, net


def test_learned_start_against_uniform_start(trained):
    from paper_1601_08201_amd import warmstart
    scanner, model, net = trained
    shape = (scanner.ny, scanner.nx, scanner.Q)
    rc = warmstart.Reconstruction(scanner)
    R = rc.R
    tols = (1e-2, 1e-4)
    plain, learned = [], []
    for (_, y, r) in warmstart.draw_scans(scanner, range(20000, 20012)):
        rc.load(y, r)
        phi_star, _ = warmstart.converged_objective(R)
        R.set_init(None)
        it_p, _ = warmstart.iterations_to_targets(R, phi_star, tols)
        spent, fell_back = warmstart.warm_start(R, net, model, shape)
        assert spent == 10 and not fell_back
        assert np.all(R.image() >= 0)
        it_l, _ = warmstart.iterations_to_targets(R, phi_star, tols)
        assert it_p[-1] is not None and it_l[-1] is not None
        plain.append(it_p)
        learned.append([i + spent for i in it_l])
    plain, learned = np.array(plain, float), np.array(learned, float)
    print("median iterations to 1e-2 / 1e-4: plain", np.median(plain, 0), "learned", np.median(learned, 0),
          flush=True)
    assert np.median(learned[:, 0]) < np.median(plain[:, 0])
    assert np.median(learned[:, 1]) < np.median(plain[:, 1])


def test_fallback_refuses_a_worse_start(trained):
    from paper_1601_08201_amd import warmstart
    scanner, model, net = trained
    shape = (scanner.ny, scanner.nx, scanner.Q)
    bad = dataclasses.replace(model, c_out=model.c_out * 1000.0)
    rc = warmstart.Reconstruction(scanner)
    R = rc.R
    (_, y, r), = warmstart.draw_scans(scanner, [20100])
    rc.load(y, r)
    spent, fell_back = warmstart.warm_start(R, net, bad, shape)
    assert spent == 10 and fell_back
    R.iterate(20)
    f_fb = R.image()
    assert R.objective()["iter"] == 30
    R.set_init(None)
    R.iterate(10)
    R.iterate(20)
    np.testing.assert_array_equal(f_fb, R.image())
