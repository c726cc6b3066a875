"""Row-block epilogues of the tiled products: the forward product computing the
ratio of the rows it completes and the back product the image update of the
voxels it completes give bit for bit the results of the separate ratio and
image-update launches (same sums in the same order), over many iterations (the
arrival counters return to zero after every launch), for every inner-loop
variant, value type, weighting, grouping, sweep count and ragged size, and
they stay within the FP32 tolerance of the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1601_08201_amd import datagen

pytestmark = pytest.mark.gpu

# several row blocks and uneven slabs on small problems
SLABS = dict(waves=4, fwd_rows_per_wave=64, fwd_block_cols=512, fwd_slabs=3,
             back_rows_per_wave=64, back_block_cols=256, back_slabs=4)

CASES = {
    "small, tuned schedule": dict(cfg="small", seed=1),
    "small, 3 and 4 slabs, variant 1": dict(cfg="small", seed=2, sched=dict(SLABS, variant=1)),
    "small, 3 and 4 slabs, variant 2": dict(cfg="small", seed=3, sched=dict(SLABS, variant=2)),
    "small, 3 and 4 slabs, variant 3": dict(cfg="small", seed=4, sched=dict(SLABS, variant=3)),
    "bf16 values, slabs": dict(cfg="small", seed=5, storage="bf16", sched=dict(SLABS, variant=1)),
    "f16 values, direction weights": dict(cfg="teflon", seed=6, storage="f16", w="dir"),
    "full weights, standard TV": dict(cfg=dict(ny=9, nx=13, Q=24, I=1501, nnz_per_col=8, rects=3), seed=7,
                                      w="full", grouping=1, sched=dict(SLABS, variant=1)),
    "ragged rows (I odd), 3 sweeps": dict(cfg=dict(ny=7, nx=11, Q=13, I=999, nnz_per_col=6, rects=2), seed=8,
                                          sweeps=3, sched=dict(SLABS, variant=2)),
    "Q = 1": dict(cfg=dict(ny=40, nx=23, Q=1, I=700, nnz_per_col=6, rects=3), seed=9,
                  sched=dict(SLABS, variant=1)),
}


def weights(prob, kind):
    if kind == "dir":
        return prob.meta["weights"]
    if kind == "full":
        return np.random.default_rng(3).uniform(0.5, 2.0, 4 * prob.J).astype(np.float32)
    return None


def run(sg, prob, c, epilogues, n):
    R = sg.Reconstructor()
    if c.get("sched"):
        R.set_schedule(format=0, **c["sched"])
    R.set_epilogues(epilogues)
    R.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, prob.val,
                 storage=c.get("storage", "f32"), w=weights(prob, c.get("w")))
    if c.get("grouping"):
        R.set_grouping(c["grouping"])
    R.set_data(prob.y, prob.r, prob.beta, prob.rho, c.get("sweeps", 1))
    R.iterate(n // 2)
    R.iterate(n - n // 2)
    out = dict(image=R.image(), objective=R.objective(), split=R.split(), epilogues=R.epilogues())
    R.close()
    return out


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_08201_amd import sgtv
    sgtv.lib()
    return sgtv


@pytest.mark.parametrize("name", list(CASES))
def test_epilogues_equal_separate_launches(sg, name):
    c = CASES[name]
    prob = datagen.make_problem(c["cfg"], c["seed"])
    on = run(sg, prob, c, True, 30)
    off = run(sg, prob, c, False, 30)
    assert on["epilogues"] and not off["epilogues"]
    print(name, "objective", on["objective"]["total"], flush=True)
    np.testing.assert_array_equal(on["image"], off["image"])
    assert on["objective"] == off["objective"]
    for a, b in zip(on["split"], off["split"]):
        np.testing.assert_array_equal(a, b)
    if c.get("storage", "f32") == "f32" and c.get("sweeps", 1) == 1:
        kw = {}
        if c.get("w"):
            kw["w"] = weights(prob, c["w"])
        if c.get("grouping"):
            kw["grouping"] = c["grouping"]
        f_o = oracle.admm(prob, 30, report=False, **kw)[0]
        err = np.linalg.norm(on["image"] - f_o) / np.linalg.norm(f_o)
        print(name, "rel_l2 vs oracle", err, flush=True)
        assert err <= 1e-5


def test_epilogues_on_the_paper_scale_scan(sg):
    """The 128 x 128 x 128 scan with its tuned schedule (2048 rows per wave,
    full-LDS tiles, 8 forward and 4 back slabs): 20 iterations with and
    without the epilogues, bit for bit."""
    prob = datagen.make_problem("paper", 1)
    from paper_1601_08201_amd import autotune
    tuned = autotune.cached_schedule(prob)
    assert tuned and tuned["fwd_rows_per_wave"] == 2048
    c = dict(sched=tuned)
    on = run(sg, prob, c, True, 20)
    off = run(sg, prob, c, False, 20)
    np.testing.assert_array_equal(on["image"], off["image"])
    assert on["objective"] == off["objective"]
