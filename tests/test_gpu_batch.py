"""Batched scans: every scan of a batch reproduces its own single-scan run bit
for bit (same schedule), matches the FP64 oracle, and the batched graph replays
agree with scan-after-scan launches."""
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


def scans():
    shapes = [(8, 8, 16, 0.1, 1.0), (12, 12, 24, 0.2, 1.0), (16, 16, 32, 0.1, 0.5),
              (5, 7, 9, 0.05, 2.0), (16, 16, 32, 0.1, 1.0), (20, 10, 40, 0.3, 1.0)]
    out = []
    for k, (ny, nx, Q, beta, rho) in enumerate(shapes):
        J = ny * nx * Q
        p = datagen.make_problem(dict(ny=ny, nx=nx, Q=Q, I=max(J // 2, 64), nnz_per_col=8, rects=3,
                                      beta=beta, rho=rho), seed=500 + k)
        out.append(p)
    return out


SCHED = dict(fwd_rows_per_wave=64, back_rows_per_wave=128, fwd_block_cols=2048, back_block_cols=1024)


def test_batch_matches_single_scans_and_oracle(sg):
    probs = scans()
    B = sg.Batch()
    for p in probs:
        B.add_scan(p, schedule=SCHED)
    assert len(B) == len(probs)
    B.iterate(20)
    B.iterate(10)
    for i, p in enumerate(probs):
        R = sg.Reconstructor()
        R.set_schedule(**SCHED)
        R.set_problem(p)
        R.iterate(30)
        np.testing.assert_array_equal(B.image(i), R.image())
        assert B.objective(i) == R.objective()
        f_o, _, _, _ = oracle.admm(p, 30, report=False)
        err = np.linalg.norm(B.image(i) - f_o) / np.linalg.norm(f_o)
        print("scan", i, p.ny, p.nx, p.Q, "rel_l2", err, flush=True)
        assert err <= 1e-5
        R.close()


def test_batched_graph_replays_equal_sequential(sg):
    probs = scans()
    A = sg.Batch()
    S = sg.Batch()
    for p in probs:
        A.add_scan(p, schedule=SCHED)
        S.add_scan(p, schedule=SCHED)
    for rep in range(3):
        A.iterate(6)
        S.iterate_sequential(6)
        for i in range(len(probs)):
            assert A.objective(i) == S.objective(i)
            np.testing.assert_array_equal(A.image(i), S.image(i))


def test_add_scan_after_iterating_is_refused(sg):
    probs = scans()
    B = sg.Batch()
    B.add_scan(probs[0])
    B.iterate(2)
    with pytest.raises(sg.SgtvError) as ei:
        B.add_scan(probs[1])
    assert ei.value.code == sg.SGTV_ESTATE
    assert len(B) == 1


def test_batch_prepare_both_modes(sg):
    """prepare(n) and prepare(n, sequential=True) capture without running; the
    iterations after them equal those of a batch that was not prepared."""
    import ctypes
    probs = scans()[:3]
    runs = []
    for prepared in (False, True):
        B = sg.Batch()
        for p in probs:
            B.add_scan(p, schedule=SCHED)
        if prepared:
            B.prepare(9)
            B.prepare(9, sequential=True)
            for i in range(len(probs)):
                assert B.objective(i)["iter"] == 0
        B.iterate(9)
        B.iterate_sequential(9)
        runs.append([B.image(i) for i in range(len(probs))])
        if prepared:
            with pytest.raises(sg.SgtvError):
                B.prepare(-1)
            assert sg.lib().sgtv_batch_prepare(B._b, 4, ctypes.c_int(2)) != 0
        B.close()
    for a, b in zip(*runs):
        np.testing.assert_array_equal(a, b)



@pytest.mark.parametrize("calls", [(30,), (7, 1, 22)])
def test_persistent_launch_equals_graph(sg, calls):
    """One cooperative launch with grid barriers gives bitwise the images and
    reports of the graph-replayed batched launches, also across calls of odd
    length (buffer parities)."""
    probs = scans()
    A, P = sg.Batch(), sg.Batch()
    for p in probs:
        A.add_scan(p, schedule=SCHED)
        P.add_scan(p, schedule=SCHED)
    P.set_launch("persistent")
    for n in calls:
        print("persistent launch of", n, "iterations", flush=True)
        A.iterate(n)
        P.iterate(n)
    mode, grid = P.launch()
    print("grid", grid, flush=True)
    assert mode == "persistent" and grid >= 1
    for i in range(len(probs)):
        np.testing.assert_array_equal(P.image(i), A.image(i))
        assert P.objective(i) == A.objective(i)


def test_persistent_launch_weights_and_groupings(sg):
    """The paper-shaped scan with pitch weights, both groupings and two betas
    in one persistent launch against the graph path and the oracle."""
    prob = datagen.make_problem("teflon", 1)
    w = prob.meta["weights"]
    pairs = [(0, 0.2), (1, 0.05), (0, 1.0), (1, 0.5)]
    A, P = sg.Batch(), sg.Batch()
    for g, b in pairs:
        A.add_scan(prob, w=w, grouping=g, beta=b)
        P.add_scan(prob, w=w, grouping=g, beta=b)
    P.set_launch("persistent")
    A.iterate(41)
    P.iterate(41)
    for i, (g, b) in enumerate(pairs):
        np.testing.assert_array_equal(P.image(i), A.image(i))
        f_o, _, _, _ = oracle.admm(prob, 41, beta=b, w=w, grouping=g, report=False)
        err = np.linalg.norm(P.image(i) - f_o) / np.linalg.norm(f_o)
        print("grouping", g, "beta", b, "rel_l2", err, flush=True)
        assert err <= 1e-5


def test_batch_of_mixed_tile_formats(sg):
    """Scans with 24-bit indices of 14 and of 13 column bits (1024 and 2048
    rows per wave) and with 32-bit indices in one batch: graph and persistent
    launches both reproduce every scan's single run bit for bit.  A tile that
    fills the whole 160 KiB of LDS (16 waves of 2048 rows, 8188-column
    blocks) runs in the graph launch; the persistent kernel, which keeps 16
    bytes of LDS of its own, refuses it."""
    probs = scans()[:3]
    full = [dict(fwd_rows_per_wave=1024, back_rows_per_wave=512, fwd_block_cols=4096, back_block_cols=16380),
            dict(fwd_rows_per_wave=2048, back_rows_per_wave=2048, fwd_block_cols=8188, back_block_cols=1000),
            dict(fwd_rows_per_wave=1024, back_rows_per_wave=1500, fwd_block_cols=16384, back_block_cols=8192)]
    fits = [dict(s) for s in full]
    fits[1]["fwd_block_cols"] = 4000
    for launch, scheds in (("graph", full), ("persistent", fits)):
        B = sg.Batch()
        for p, s in zip(probs, scheds):
            B.add_scan(p, schedule=s)
        B.set_launch(launch)
        B.iterate(25)
        for i, (p, s) in enumerate(zip(probs, scheds)):
            R = sg.Reconstructor()
            R.set_schedule(**s)
            R.set_problem(p)
            R.iterate(25)
            print(launch, "scan", i, R.schedule(), flush=True)
            np.testing.assert_array_equal(B.image(i), R.image())
            assert B.objective(i) == R.objective()
            R.close()
        B.close()
    B = sg.Batch()
    for p, s in zip(probs, full):
        B.add_scan(p, schedule=s)
    B.set_launch("persistent")
    with pytest.raises(sg.SgtvError) as ei:
        B.iterate(1)
    print("refused:", ei.value, flush=True)
    B.close()


@pytest.mark.parametrize("seed", range(4))
def test_random_batches_equal_single_scans(sg, seed):
    """Seeded random batches (3-6 scans of random shapes, groupings, betas
    and densities) under one random tile schedule: the graph launch, and the
    persistent launch where the schedule allows it (a multiple of 4 waves,
    room for its own LDS), reproduce every scan's single run bit for bit."""
    from paper_1601_08201_amd import autotune
    rng = np.random.default_rng(700 + seed)
    probs, setups = [], []
    for k in range(int(rng.integers(3, 7))):
        ny, nx, Q = int(rng.integers(3, 17)), int(rng.integers(3, 17)), int(rng.integers(1, 33))
        J = ny * nx * Q
        probs.append(datagen.make_problem(dict(ny=ny, nx=nx, Q=Q, I=int(rng.integers(64, max(65, J))),
                                               nnz_per_col=int(rng.integers(2, 13)), rects=2, beta=0.1),
                                          seed=1500 + 10 * seed + k))
        setups.append((int(rng.integers(0, 2)), float(rng.choice([0.05, 0.2, 1.0]))))
    while True:
        waves = int(rng.choice([4, 8, 16]))
        rw = int(rng.choice([64, 256, 1024, 2048]))
        cb = int(rng.choice([256, 4096, 8188, 16380]))
        if autotune.lds_bytes(waves, rw, cb) <= autotune.MAX_LDS:
            break
    sched = dict(waves=waves, fwd_rows_per_wave=rw, back_rows_per_wave=rw, fwd_block_cols=cb, back_block_cols=cb)
    persistent_ok = autotune.lds_bytes(waves, rw, cb) <= autotune.MAX_LDS - 16
    print("seed", seed, "scans", len(probs), "schedule", sched, "persistent", persistent_ok, flush=True)
    launches = ["graph"] + (["persistent"] if persistent_ok else [])
    for launch in launches:
        B = sg.Batch()
        for p, (g, b) in zip(probs, setups):
            B.add_scan(p, schedule=sched, grouping=g, beta=b)
        B.set_launch(launch)
        B.iterate(9)
        B.iterate(8)
        for i, (p, (g, b)) in enumerate(zip(probs, setups)):
            R = sg.Reconstructor()
            R.set_schedule(**sched)
            R.set_problem(p)
            if g:
                R.set_grouping(g)
            R.set_data(p.y, p.r, b, p.rho, p.sweeps)
            R.iterate(17)
            np.testing.assert_array_equal(B.image(i), R.image())
            assert B.objective(i) == R.objective()
            R.close()
        B.close()


def test_launch_mode_is_checked(sg):
    B = sg.Batch()
    assert B.launch() == ("graph", 0)
    with pytest.raises(sg.SgtvError):
        sg.sgtv_batch_set_launch(B._b, 7)
    B.set_launch("persistent")
    B.iterate(3)          # empty batch: nothing to run
    assert B.launch()[0] == "persistent"


def test_batch_from_saved_systems_equals_packed_batch(sg, tmp_path):
    """Scans added from system files (saved from a packed batch) iterate bit for
    bit like the packed batch; a file of another value type is refused."""
    probs = scans()
    A = sg.Batch()
    for p in probs:
        A.add_scan(p, schedule=SCHED)
    paths = []
    for i in range(len(probs)):
        paths.append(str(tmp_path / ("scan%d.sys" % i)))
        A.save_scan(i, paths[-1])
    B = sg.Batch()
    for path, p in zip(paths, probs):
        B.add_system_file(path, p)
    A.iterate(15)
    B.iterate(15)
    for i in range(len(probs)):
        np.testing.assert_array_equal(B.image(i), A.image(i))
        assert B.objective(i) == A.objective(i)
    R = sg.Reconstructor()
    R.set_system(probs[0].I, probs[0].ny, probs[0].nx, probs[0].Q, probs[0].rowptr, probs[0].col,
                 probs[0].val, storage="bf16")
    R.save_system(str(tmp_path / "bf16.sys"))
    with pytest.raises(RuntimeError):
        B.add_system_file(str(tmp_path / "bf16.sys"), probs[0])
    assert len(B) == len(probs)
    R.close()
    A.close()
    B.close()


def test_batch_of_the_64_scan_workload_matches_single_runs_and_oracle(sg):
    """The schedule the 64-scan benchmark batch uses (the batch rule over all
    64 shapes: 1024 rows per wave, automatic 16380-column blocks and slabs) on
    real scans of that workload: its three smallest scans (32 x 32 grids) and
    one 64 x 64 x 128 scan in one batch equal their single-scan runs with the
    same schedule bit for bit, and the two smallest the FP64 oracle at 1e-5."""
    from paper_1601_08201_amd import autotune
    shapes = datagen.batch_shapes(64, 300)
    sched = autotune.batch_schedule([(ny * nx * Q // 2, ny * nx * Q) for ny, nx, Q in shapes])
    assert sched["fwd_rows_per_wave"] == 1024
    order = sorted(range(len(shapes)), key=lambda k: shapes[k][0] * shapes[k][1] * shapes[k][2])
    picks = order[:3] + [next(k for k in order if shapes[k] == (64, 64, 128))]
    probs = [datagen.make_batch_scan(*shapes[k], seed=300 + k) for k in picks]
    B = sg.Batch()
    for p in probs:
        B.add_scan(p, schedule=sched)
    B.iterate(25)
    for i, p in enumerate(probs):
        R = sg.Reconstructor()
        R.set_schedule(format=0, **sched)
        R.set_problem(p)
        R.iterate(25)
        np.testing.assert_array_equal(B.image(i), R.image())
        assert B.objective(i) == R.objective()
        R.close()
        if i < 2:
            f_o = oracle.admm(p, 25, report=False)[0]
            err = np.linalg.norm(B.image(i) - f_o) / np.linalg.norm(f_o)
            print("scan", shapes[picks[i]], "rel_l2 vs oracle", err, flush=True)
            assert err <= 1e-5
    B.close()


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_batch_of_16_bit_scans_matches_single_scans(sg, storage):
    """Scans with 16-bit matrix values (per-column FP32 scale) in one batch
    equal their single-scan runs bit for bit (graph replays and eager
    launches), and the persistent launch refuses them with an error."""
    probs = scans()
    B = sg.Batch(storage=storage)
    for p in probs:
        B.add_scan(p, schedule=SCHED)
    B.iterate(12)
    B.iterate(8)
    for i, p in enumerate(probs):
        R = sg.Reconstructor()
        R.set_schedule(**SCHED)
        R.set_problem(p, storage=storage)
        R.iterate(20)
        np.testing.assert_array_equal(B.image(i), R.image())
        assert B.objective(i) == R.objective()
        R.close()
    with pytest.raises(RuntimeError):
        sg.sgtv_batch_set_storage(B._b, "f32")      # scans are already there
    B.set_launch("persistent")
    with pytest.raises(RuntimeError):
        B.iterate(2)
    B.close()
