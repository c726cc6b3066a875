"""Graph replay of the iteration against one-by-one launches (bitwise), with
the program's own eager work and synchronisations between replays."""
import numpy as np
import pytest

from paper_1601_08201_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_08201_amd import sgtv
    sgtv.lib()
    return sgtv


@pytest.mark.parametrize("n", [10, 7])
def test_graph_replays_match_eager(sg, n):
    prob = datagen.make_problem("small", 3)
    eager = sg.Reconstructor().set_graphs(False).set_problem(prob)
    graph = sg.Reconstructor().set_problem(prob)
    for rep in range(4):
        eager.iterate(n)
        graph.iterate(n)
        # eager work between replays: an objective (launches + sync) and copies
        r1, r2 = eager.objective(), graph.objective()
        assert r1 == r2
        for a, b in zip(eager.state()[:3], graph.state()[:3]):
            np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(eager.image(), graph.image())


def test_graphs_dropped_when_data_changes(sg):
    prob = datagen.make_problem("small", 4)
    R = sg.Reconstructor().set_problem(prob)
    R.iterate(6)
    a = R.image()
    R.set_data(prob.y, prob.r, prob.beta * 2, prob.rho, 1)
    R.iterate(6)
    E = sg.Reconstructor().set_graphs(False).set_problem(prob)
    E.set_data(prob.y, prob.r, prob.beta * 2, prob.rho, 1)
    E.iterate(6)
    np.testing.assert_array_equal(R.image(), E.image())
    assert not np.array_equal(a, R.image())
