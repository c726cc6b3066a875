"""Paper-scale scan (128 x 128 x 128, 1,048,576 measurements, 134M nonzeros):
FP32 parity after 200 iterations (automatic schedule, and the tuned schedule
the benchmark runs), after 1000 in the benchmark's configuration, and the error of the 16-bit-value paths
against the FP64 oracle on the exact FP32 matrix at iterations 50 and 200.

The FP64 oracle runs 200 iterations of the full problem once (about a minute
of host time); every GPU path is compared with that same run.
"""
import json

import numpy as np
import pytest

import oracle
from paper_1601_08201_amd import datagen

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def paper():
    prob = datagen.make_problem("paper", 1)
    print("paper-scale problem generated", flush=True)
    f50, d50, c50, _ = oracle.admm(prob, 50, report=False)
    print("oracle: 50 iterations done", flush=True)
    f200, d200, c200, _ = oracle.admm(prob, 150, f0=f50, d0=d50, c0=c50, report=False)
    print("oracle: 200 iterations done", flush=True)
    obj = {50: oracle.objective(prob, f50)[0], 200: oracle.objective(prob, f200)[0]}
    return prob, {50: f50, 200: f200}, obj, (d200, c200)


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available()
    from paper_1601_08201_amd import sgtv
    sgtv.lib()
    return sgtv


def gpu_images(sg, prob, storage, schedule=None):
    R = sg.Reconstructor()
    if schedule:
        R.set_schedule(format=0, **schedule)
    R.set_problem(prob, storage=storage)
    if schedule:
        got = R.schedule()
        assert all(got[k] == v for k, v in schedule.items()), got
    R.iterate(50)
    f50 = R.image()
    R.iterate(150)
    f200 = R.image()
    rep = R.objective()
    R.close()
    return {50: f50, 200: f200}, rep


@pytest.mark.parametrize("schedule", ["automatic", "tuned"])
def test_fp32_matches_oracle_after_200_iterations(sg, paper, schedule):
    """The automatic schedule (1024 rows per wave, 4 and 2 slabs) and the one
    the benchmark runs (the autotuner's cached schedule for this shape: 2048
    rows per wave, 8188-column blocks, 8 and 4 slabs)."""
    prob, f_or, obj, _ = paper
    sched = None
    if schedule == "tuned":
        from paper_1601_08201_amd import autotune
        sched = autotune.cached_schedule(prob)
        assert sched is not None
        print("tuned schedule", json.dumps(sched), flush=True)
    f_g, rep = gpu_images(sg, prob, "f32", sched)
    for k in (50, 200):
        err = rel_l2(f_g[k], f_or[k])
        print("fp32 (%s schedule) iteration %d: image rel L2 %.3e" % (schedule, k, err), flush=True)
        assert err <= 1e-5
    assert rep["total"] == pytest.approx(obj[200], rel=1e-6)


def test_fp32_long_run_in_the_benchmark_configuration(sg, paper):
    """1000 iterations with the tuned schedule against 1000 of the oracle
    (continued from its 200-iteration state): the image stays within the FP32
    tolerance and the objective within 1e-9."""
    from paper_1601_08201_amd import autotune
    prob, f_or, _, (d200, c200) = paper
    f_o, _, _, _ = oracle.admm(prob, 800, f0=f_or[200], d0=d200, c0=c200, report=False)
    print("oracle: 1000 iterations done", flush=True)
    R = sg.Reconstructor()
    R.set_schedule(format=0, **autotune.cached_schedule(prob))
    R.set_problem(prob)
    R.iterate(1000)
    f_g = R.image()
    R.close()
    err = rel_l2(f_g, f_o)
    phi_g, phi_o = oracle.objective(prob, f_g)[0], oracle.objective(prob, f_o)[0]
    print("1000 iterations: image rel L2 %.3e, objective rel %.3e" % (err, abs(phi_g - phi_o) / abs(phi_o)),
          flush=True)
    assert err <= 1e-5
    assert abs(phi_g - phi_o) <= 1e-9 * abs(phi_o)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_reduced_precision_error_against_fp64(sg, paper, storage):
    prob, f_or, obj, _ = paper
    f_g, rep = gpu_images(sg, prob, storage)
    out = {"storage": storage}
    for k in (50, 200):
        phi = oracle.objective(prob, f_g[k])[0]       # FP64 objective on the exact matrix
        out[k] = dict(image_rel_l2=rel_l2(f_g[k], f_or[k]),
                      rel_objective=abs(phi - obj[k]) / abs(obj[k]))
    print("reduced precision vs FP64 oracle (exact FP32 matrix): " + json.dumps(out), flush=True)
    assert np.all(np.isfinite(f_g[200])) and np.all(f_g[200] >= 0)
    assert out[200]["rel_objective"] <= 1e-4
