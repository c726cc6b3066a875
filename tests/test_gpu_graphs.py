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


@pytest.mark.parametrize("first", [0, 3])
def test_prepare_captures_without_running(sg, first):
    """prepare(n) leaves the state as it is and the iterate(n) after it equals
    the run without prepare bitwise, from either buffer parity."""
    prob = datagen.make_problem("small", 5)
    plain = sg.Reconstructor().set_problem(prob)
    prep = sg.Reconstructor().set_problem(prob)
    plain.iterate(first)
    prep.iterate(first)
    before = prep.state()
    prep.prepare(12)
    prep.prepare(12)   # already cached: nothing to do
    for a, b in zip(before, prep.state()):
        np.testing.assert_array_equal(a, b)
    assert prep.objective()["iter"] == first
    for rep in range(3):
        plain.iterate(12)
        prep.iterate(12)
        assert plain.objective() == prep.objective()
        np.testing.assert_array_equal(plain.image(), prep.image())
    assert prep.objective()["iter"] == first + 36


def test_prepare_arguments(sg):
    prob = datagen.make_problem("small", 6)
    R = sg.Reconstructor()
    with pytest.raises(sg.SgtvError):
        R.prepare(5)   # no system yet
    R.set_problem(prob)
    with pytest.raises(sg.SgtvError):
        R.prepare(-1)
    R.prepare(0)
    R.prepare(1)
    R.set_graphs(False).prepare(8)   # graphs off: nothing to capture
    R.set_graphs(True)
    R.prepare(8)
    R.set_data(prob.y, prob.r, prob.beta, prob.rho, 1)   # drops the graph; the next call captures again
    R.iterate(8)
    E = sg.Reconstructor().set_graphs(False).set_problem(prob)
    E.iterate(8)
    np.testing.assert_array_equal(R.image(), E.image())
    R.close()
    E.close()
