"""GPU parity: the HIP library against the FP64 oracle on the same seeded inputs.

Tolerances: image relative L2 <= 1e-5 after a fixed iteration count on the
FP32 path (the acceptance bound of the method's GPU port); objective and data
terms compared to relative 1e-6; split variables d, c to relative L2 1e-4
(they are differences of nearly equal numbers in voxels where the group is
almost shrunk to zero).
"""
import numpy as np
import pytest

import oracle
from paper_1601_08201_amd import datagen

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def sg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1601_08201_amd import sgtv
    sgtv.lib()
    return sgtv


def run_gpu(sg, prob, n, storage="f32", w=None, grouping=0, sweeps=None, x0=None, schedule=None):
    R = sg.Reconstructor()
    if schedule:
        R.set_schedule(**schedule)
    R.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, prob.val, storage=storage, w=w)
    if grouping:
        R.set_grouping(grouping)
    R.set_data(prob.y, prob.r, prob.beta, prob.rho, prob.sweeps if sweeps is None else sweeps)
    if x0 is not None:
        R.set_init(x0)
    R.iterate(n)
    return R


def check_against_oracle(sg, prob, n, w=None, grouping=0, sweeps=None, x0=None, tol=IMG_TOL,
                         schedule=None):
    R = run_gpu(sg, prob, n, w=w, grouping=grouping, sweeps=sweeps, x0=x0, schedule=schedule)
    f_g = R.image()
    d_g, c_g = R.split()
    rep = R.objective()
    f_o, d_o, c_o, rep_o = oracle.admm(prob, n, f0=x0, w=w, grouping=grouping,
                                       sweeps=prob.sweeps if sweeps is None else sweeps)
    print("case", prob.ny, prob.nx, prob.Q, prob.I, "iters", n, "rel_l2", rel_l2(f_g, f_o), flush=True)
    assert np.all(f_g >= 0)
    assert rel_l2(f_g, f_o) <= tol
    assert rel_l2(d_g, d_o) <= 1e-4 or np.linalg.norm(d_g - d_o) <= 1e-5
    assert rel_l2(c_g, c_o) <= 1e-4
    obj_o = oracle.objective(prob, f_o, w=w, grouping=grouping)
    assert rep["total"] == pytest.approx(obj_o[0], rel=1e-6)
    assert rep["data"] == pytest.approx(obj_o[1], rel=1e-6, abs=1e-6)
    assert rep["tv"] == pytest.approx(obj_o[2], rel=1e-5)
    if n > 0:
        assert rep["r_primal"] == pytest.approx(rep_o[-1, 3], rel=1e-3, abs=1e-6)
        assert rep["r_dual"] == pytest.approx(rep_o[-1, 4], rel=1e-3, abs=1e-6)
    assert rep["iter"] == n
    R.close()


@pytest.mark.parametrize("seed", range(10))
def test_small_workload_50_iterations(sg, seed):
    prob = datagen.make_problem("small", seed)
    check_against_oracle(sg, prob, 50)


@pytest.mark.parametrize("Q", [1, 7, 33, 64, 129])
def test_spectral_sizes(sg, Q):
    prob = datagen.make_problem(dict(ny=5, nx=6, Q=Q, I=max(64, 3 * 30 * Q // 2), nnz_per_col=8,
                                     rects=3, beta=0.2, rho=1.0), seed=100 + Q)
    check_against_oracle(sg, prob, 20)


SCHEDULES = {
    "sell": dict(format=1),
    "tiles-small": dict(format=0, waves=4, fwd_rows_per_wave=64, fwd_block_cols=1024, fwd_slabs=3,
                        back_rows_per_wave=32, back_block_cols=512, back_slabs=2),
    "tiles-one-wave": dict(format=0, waves=1, fwd_rows_per_wave=100, fwd_block_cols=4092, fwd_slabs=1,
                           back_rows_per_wave=300, back_block_cols=12, back_slabs=5),
    # 16384-column blocks: the 32-bit index format of the simple loop
    "tiles-32bit-index": dict(format=0, waves=4, fwd_rows_per_wave=512, fwd_block_cols=16384, fwd_slabs=1,
                              back_rows_per_wave=1024, back_block_cols=16384, back_slabs=1),
    "tiles-pipelined": dict(format=0, waves=8, fwd_rows_per_wave=128, fwd_block_cols=2048, fwd_slabs=2,
                            back_rows_per_wave=256, back_block_cols=1024, back_slabs=2, variant=2),
    "tiles-prefetch": dict(format=0, waves=8, fwd_rows_per_wave=128, fwd_block_cols=2048, fwd_slabs=2,
                           back_rows_per_wave=256, back_block_cols=1024, back_slabs=2, variant=3),
    # 24-bit indices with 11-bit rows and 13-bit columns: 2048 rows per wave
    # and an 8188-column block (ragged 4-column tail), 1536 rows per wave over
    # two ragged row blocks
    "tiles-2048-rows": dict(format=0, waves=4, fwd_rows_per_wave=2048, fwd_block_cols=8188, fwd_slabs=1,
                            back_rows_per_wave=1536, back_block_cols=1000, back_slabs=2),
    # blocks too wide for 13-bit columns: the 32-bit format at 2048 rows per wave
    "tiles-2048-rows-32bit": dict(format=0, waves=2, fwd_rows_per_wave=2048, fwd_block_cols=16380,
                                  fwd_slabs=1, back_rows_per_wave=2048, back_block_cols=8192, back_slabs=2),
}


@pytest.mark.parametrize("name", sorted(SCHEDULES))
def test_schedules_agree_with_oracle(sg, name):
    prob = datagen.make_problem("small", 11)
    check_against_oracle(sg, prob, 30, schedule=SCHEDULES[name])


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_full_lds_tiles_of_2048_rows(sg, storage):
    """16 waves of 2048 rows with 8188-column blocks fill the 160 KiB of LDS
    (128 KiB of row sums, 32 KiB of block) on the 64^3 scanner (262144 voxels,
    131072 measurements); 16-bit values against the oracle on the quantised
    matrix."""
    prob = datagen.make_problem("warmstart", 3)
    sched = dict(format=0, waves=16, fwd_rows_per_wave=2048, fwd_block_cols=8188, fwd_slabs=4,
                 back_rows_per_wave=2048, back_block_cols=8188, back_slabs=2)
    if storage == "f32":
        check_against_oracle(sg, prob, 20, schedule=sched)
        return
    R = run_gpu(sg, prob, 20, storage=storage, schedule=sched)
    got = R.schedule()
    assert got["fwd_rows_per_wave"] == 2048 and got["back_block_cols"] == 8188
    import copy
    q = copy.copy(prob)
    q.val = oracle.quantise(prob.col, prob.val, prob.J, storage)[2]
    f_o = oracle.admm(q, 20, report=False)[0]
    err = rel_l2(R.image(), f_o)
    print("bf16 values, 2048-row tiles: rel_l2 vs oracle on the quantised matrix", err, flush=True)
    assert err <= IMG_TOL
    R.close()


def test_full_lds_tiles_standard_tv_weights_and_sweeps(sg):
    """The full-LDS 2048-row tiles with standard TV, per-direction weights and
    three surrogate sweeps per iteration on the 64^3 scanner."""
    prob = datagen.make_problem("warmstart", 4)
    sched = dict(format=0, waves=16, fwd_rows_per_wave=2048, fwd_block_cols=8188, fwd_slabs=4,
                 back_rows_per_wave=2048, back_block_cols=8188, back_slabs=2)
    w = np.array([1.0, 0.8, 1.25, 0.9], np.float32)
    check_against_oracle(sg, prob, 12, w=w, grouping=1, sweeps=3, schedule=sched)


def random_schedule(rng):
    """A tile schedule drawn at random within the limits of set_schedule and
    of the 160 KiB of LDS (both index formats, all three inner loops)."""
    from paper_1601_08201_amd import autotune
    while True:
        waves = int(rng.choice([1, 2, 4, 8, 16]))
        variant = int(rng.choice([1, 1, 2, 3]))
        side = []
        for _ in range(2):
            rw = int(rng.choice([64, 100, 256, 1024, 1536, 2048]))
            cb = int(rng.choice([12, 256, 1000, 4096, 8188, 16380, 16384]))
            side.append((rw, cb, int(rng.integers(1, 5))))
        if variant == 3 and any(cb > 16 * waves * 64 for _, cb, _ in side):
            continue   # the block prefetch of variant 3 holds at most 16 floats per thread
        if all(autotune.lds_bytes(waves, rw, cb, variant) <= autotune.MAX_LDS for rw, cb, _ in side):
            (fr, fc, fs), (br, bc, bs) = side
            return dict(format=0, waves=waves, variant=variant, fwd_rows_per_wave=fr, fwd_block_cols=fc,
                        fwd_slabs=fs, back_rows_per_wave=br, back_block_cols=bc, back_slabs=bs)


@pytest.mark.parametrize("seed", range(12))
def test_random_schedules_agree_with_oracle(sg, seed):
    """Seeded random problems (grid, spectral bins, measurements, density)
    under seeded random tile schedules, against the oracle."""
    rng = np.random.default_rng(900 + seed)
    ny, nx, Q = int(rng.integers(3, 21)), int(rng.integers(3, 21)), int(rng.integers(1, 41))
    J = ny * nx * Q
    cfg = dict(ny=ny, nx=nx, Q=Q, I=int(rng.integers(64, max(65, 3 * J // 2))), nnz_per_col=int(rng.integers(2, 17)),
               rects=int(rng.integers(1, 4)), beta=float(rng.choice([0.05, 0.2, 0.5])))
    sched = random_schedule(rng)
    print("seed", seed, "problem", cfg, "schedule", sched, flush=True)
    prob = datagen.make_problem(cfg, seed=1000 + seed)
    check_against_oracle(sg, prob, 15, schedule=sched)


@pytest.mark.parametrize("seed", range(6))
def test_random_schedules_16_bit_values(sg, seed):
    """Seeded random problems and schedules with BF16 or FP16 values: the GPU
    against the oracle given the same dequantised matrix."""
    import copy
    rng = np.random.default_rng(950 + seed)
    storage = ("bf16", "f16")[seed % 2]
    ny, nx, Q = int(rng.integers(3, 17)), int(rng.integers(3, 17)), int(rng.integers(1, 33))
    J = ny * nx * Q
    cfg = dict(ny=ny, nx=nx, Q=Q, I=int(rng.integers(64, max(65, J))), nnz_per_col=int(rng.integers(2, 13)),
               rects=2, beta=0.1)
    sched = random_schedule(rng)
    print("seed", seed, storage, "problem", cfg, "schedule", sched, flush=True)
    prob = datagen.make_problem(cfg, seed=1200 + seed)
    q = copy.copy(prob)
    q.val = oracle.quantise(prob.col, prob.val, prob.J, storage)[2]
    R = run_gpu(sg, prob, 15, storage=storage, schedule=sched)
    f_o = oracle.admm(q, 15, report=False)[0]
    err = rel_l2(R.image(), f_o)
    print("rel_l2 vs oracle on the quantised matrix", err, flush=True)
    assert err <= IMG_TOL
    R.close()


def test_non_square_grid_and_ragged_tails(sg):
    prob = datagen.make_problem(dict(ny=3, nx=11, Q=5, I=301, nnz_per_col=7, rects=3, beta=0.1),
                                seed=7)
    check_against_oracle(sg, prob, 30)


def test_empty_rows_and_columns(sg):
    prob = datagen.make_problem(dict(ny=4, nx=4, Q=8, I=200, nnz_per_col=6, rects=2, beta=0.1), seed=9)
    A = prob.csr().tolil()
    A[5, :] = 0
    A[17, :] = 0
    A[:, 3] = 0
    A[:, 64] = 0
    A = A.tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    prob.rowptr, prob.col, prob.val = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float32)
    check_against_oracle(sg, prob, 25)


def test_rows_with_many_entries(sg):
    prob = datagen.make_problem(dict(ny=4, nx=4, Q=16, I=40, nnz_per_col=12, rects=2, beta=0.1), seed=12)
    check_against_oracle(sg, prob, 25)


@pytest.mark.parametrize("sweeps", [1, 3])
def test_surrogate_sweeps(sg, sweeps):
    prob = datagen.make_problem("small", 3)
    check_against_oracle(sg, prob, 15, sweeps=sweeps)


def test_standard_tv_grouping(sg):
    prob = datagen.make_problem("small", 4)
    check_against_oracle(sg, prob, 30, grouping=1)


def test_direction_weights(sg):
    prob = datagen.make_problem(dict(ny=6, nx=5, Q=9, I=300, nnz_per_col=8, rects=3, beta=0.15), seed=21)
    check_against_oracle(sg, prob, 20, w=np.array([1.0, 1.0, 0.3, 0.3], np.float32))
    wfull = np.random.default_rng(3).uniform(0.5, 1.5, prob.J * 4).astype(np.float32)
    check_against_oracle(sg, prob, 20, w=wfull)


def test_explicit_start_image(sg):
    prob = datagen.make_problem("small", 5)
    x0 = np.random.default_rng(1).uniform(0, 3, prob.J).astype(np.float32)
    check_against_oracle(sg, prob, 20, x0=x0)


def test_split_calls_equal_one_call_bitwise(sg):
    prob = datagen.make_problem("small", 6)
    a = run_gpu(sg, prob, 50)
    b = run_gpu(sg, prob, 25)
    b.iterate(25)
    np.testing.assert_array_equal(a.image(), b.image())
    for x, y in zip(a.state()[:3], b.state()[:3]):
        np.testing.assert_array_equal(x, y)


def test_checkpoint_resume_bitwise(sg):
    prob = datagen.make_problem("small", 7)
    a = run_gpu(sg, prob, 40)
    b = run_gpu(sg, prob, 15)
    f, v, al, k = b.state()
    c = run_gpu(sg, prob, 0)
    c.set_state(f, v, al, k)
    c.iterate(25)
    np.testing.assert_array_equal(a.image(), c.image())
    assert c.objective()["iter"] == 40


def test_run_twice_bitwise(sg):
    prob = datagen.make_problem("small", 8)
    a = run_gpu(sg, prob, 30).image()
    b = run_gpu(sg, prob, 30).image()
    np.testing.assert_array_equal(a, b)


def test_device_tensors_in_and_out(sg):
    import torch
    prob = datagen.make_problem("small", 2)
    R = sg.Reconstructor(stream=torch.cuda.current_stream().cuda_stream)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    R.set_system(prob.I, prob.ny, prob.nx, prob.Q, dev(prob.rowptr), dev(prob.col), dev(prob.val))
    R.set_data(dev(prob.y), dev(prob.r), prob.beta, prob.rho, 1)
    R.iterate(10)
    out = torch.empty(prob.J, dtype=torch.float32, device="cuda")
    R.image(out)
    torch.cuda.synchronize()
    ref = run_gpu(sg, prob, 10).image()
    np.testing.assert_array_equal(out.cpu().numpy(), ref)


def test_zero_counts_stay_zero(sg):
    prob = datagen.make_problem("small", 1)
    prob.y = np.zeros_like(prob.y)
    R = run_gpu(sg, prob, 10)
    assert np.all(R.image() == 0)
    rep = R.objective()
    assert rep["total"] == pytest.approx(float(np.sum(prob.r.astype(np.float64))), rel=1e-6)


def test_backprojection_normalised(sg):
    prob = datagen.make_problem("small", 0)
    R = run_gpu(sg, prob, 0)
    x = R.backprojection()
    e = oracle.back(prob.rowptr, prob.col, prob.val, prob.y, prob.J)
    s = oracle.back(prob.rowptr, prob.col, prob.val, np.ones(prob.I), prob.J)
    ref = np.where(s > 0, e / np.where(s > 0, s, 1), 0)
    assert rel_l2(x, ref) <= 1e-6


def test_invalid_inputs_leave_state_unchanged(sg):
    prob = datagen.make_problem("small", 0)
    R = run_gpu(sg, prob, 5)
    before = R.state()
    bad_col = prob.col.copy()
    bad_col[3] = prob.J
    with pytest.raises(sg.SgtvError) as ei:
        R.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, bad_col, prob.val)
    assert ei.value.code == sg.SGTV_ESHAPE
    bad_val = prob.val.copy()
    bad_val[0] = -1.0
    with pytest.raises(sg.SgtvError) as ei:
        R.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, bad_val)
    assert ei.value.code == sg.SGTV_EINVAL
    bad_val[0] = np.nan
    with pytest.raises(sg.SgtvError):
        R.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, bad_val)
    y = prob.y.copy()
    y[2] = np.inf
    with pytest.raises(sg.SgtvError):
        R.set_data(y, prob.r, prob.beta, prob.rho)
    with pytest.raises(sg.SgtvError):
        R.set_data(prob.y, np.zeros_like(prob.r), prob.beta, prob.rho)
    with pytest.raises(sg.SgtvError):
        R.set_data(prob.y, prob.r, -1.0, prob.rho)
    with pytest.raises(sg.SgtvError):
        R.set_data(prob.y, prob.r, prob.beta, 0.0)
    x0 = np.ones(prob.J, np.float32)
    x0[1] = -0.5
    with pytest.raises(sg.SgtvError):
        R.set_init(x0)
    after = R.state()
    for a, b in zip(before[:3], after[:3]):
        np.testing.assert_array_equal(a, b)
    assert before[3] == after[3]
    R2 = sg.Reconstructor()
    with pytest.raises(sg.SgtvError) as ei:
        R2.iterate(1)
    assert ei.value.code == sg.SGTV_ESTATE


def test_paper_scale_first_iterations_and_properties(sg):
    """128x128x128 scan, 1,048,576 measurements, 64 entries per column: full-size parity
    after 2 iterations, then 200 iterations stay finite, nonnegative and lower the objective."""
    prob = datagen.make_problem("paper", 1)
    print("paper-scale problem generated", flush=True)
    R = run_gpu(sg, prob, 2)
    f_g = R.image()
    f_o, _, _, rep_o = oracle.admm(prob, 2, report=False)
    err = rel_l2(f_g, f_o)
    print("paper-scale rel_l2 after 2 iterations", err, flush=True)
    assert err <= IMG_TOL
    first = R.objective()["total"]
    R.iterate(198)
    rep = R.objective()
    f = R.image()
    assert np.all(np.isfinite(f)) and np.all(f >= 0)
    assert rep["total"] < first
    assert rep["iter"] == 200


@pytest.mark.parametrize("storage", ["bf16", "f16"])
@pytest.mark.parametrize("fmt", [0, 1])
def test_reduced_precision_matches_oracle_on_quantised_matrix(sg, storage, fmt):
    """16-bit values with per-column scales: the GPU multiplies with
    sigma_j * decode(code); the oracle given that same dequantised matrix must
    agree to the FP32 tolerance."""
    import copy
    prob = datagen.make_problem("small", 12)
    scale, codes, deq = oracle.quantise(prob.col, prob.val, prob.J, storage)
    q = copy.copy(prob)
    q.val = deq
    R = run_gpu(sg, prob, 50, storage=storage, schedule=dict(format=fmt))
    f_g = R.image()
    rep = R.objective()
    f_o, _, _, _ = oracle.admm(q, 50, report=False)
    err = rel_l2(f_g, f_o)
    print("storage", storage, "format", fmt, "rel_l2 vs oracle on quantised matrix", err, flush=True)
    assert err <= IMG_TOL
    # objective reported by the GPU is that of the quantised system
    assert rep["total"] == pytest.approx(oracle.objective(q, f_o)[0], rel=1e-6)
    # and against the exact matrix the image stays close
    f_x, _, _, _ = oracle.admm(prob, 50, report=False)
    phi_g = oracle.objective(prob, f_g)[0]
    phi_x = oracle.objective(prob, f_x)[0]
    print("storage", storage, "rel objective vs exact-matrix oracle", abs(phi_g - phi_x) / phi_x, flush=True)
    assert abs(phi_g - phi_x) / phi_x <= 1e-3


def consistent_split(prob, x0, grouping=0):
    """d = D x0 and c = (beta/rho) d_g/||d_g|| per group (0 where d_g = 0)."""
    thr = prob.beta / prob.rho
    d = oracle.diff(prob.ny, prob.nx, prob.Q, x0).reshape(prob.ny * prob.nx, 4, prob.Q)
    if grouping == 0:
        n = np.sqrt((d ** 2).sum(axis=(1, 2)))[:, None, None]
    else:
        n = np.sqrt((d ** 2).sum(axis=1))[:, None, :]
    c = np.where(n > 0, thr * d / np.where(n > 0, n, 1), 0.0)
    return d.ravel(), c.ravel()


@pytest.mark.parametrize("grouping", [0, 1])
def test_dual_consistent_start_matches_oracle(sg, grouping):
    prob = datagen.make_problem("small", 13)
    x0 = np.random.default_rng(2).uniform(0, 3, prob.J).astype(np.float32)
    R = sg.Reconstructor()
    if grouping:
        R.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, prob.val)
        R.set_grouping(grouping)
        R.set_data(prob.y, prob.r, prob.beta, prob.rho, 1)
    else:
        R.set_problem(prob)
    R.set_init_dual(x0)
    d_g, c_g = R.split()
    d0, c0 = consistent_split(prob, x0.astype(np.float64), grouping)
    assert rel_l2(d_g, d0) <= 1e-6
    # c = v - a v is formed in FP32 from the stored (v, a): cancellation of
    # order eps * ||d_g|| / (beta / rho)
    assert rel_l2(c_g, c0) <= 1e-4
    R.iterate(20)
    f_o, _, _, _ = oracle.admm(prob, 20, f0=x0, d0=d0, c0=c0, grouping=grouping, report=False)
    assert rel_l2(R.image(), f_o) <= IMG_TOL


def test_dual_consistent_start_is_near_fixed_point(sg):
    """Started at a converged image with its consistent split, one iteration
    barely moves it; with d = c = 0 the same image moves away."""
    prob = datagen.make_problem("small", 14)
    R = sg.Reconstructor().set_problem(prob)
    R.iterate(3000)
    f_star = R.image()
    phi_star = R.objective()["total"]
    R.set_init_dual(f_star)
    R.iterate(1)
    moved_dual = rel_l2(R.image(), f_star)
    phi_dual = R.objective()["total"]
    R.set_init(f_star)
    R.iterate(1)
    moved_zero = rel_l2(R.image(), f_star)
    print("moved: consistent", moved_dual, "zero", moved_zero, flush=True)
    assert moved_dual < 0.1 * moved_zero
    assert abs(phi_dual - phi_star) <= 1e-5 * phi_star


@pytest.mark.parametrize("cfg,storage", [("small", "f32"), ("warmstart", "f32"), ("warmstart", "bf16")])
def test_workspace_estimate_and_device_bytes(sg, cfg, storage):
    prob = datagen.make_problem(cfg, 2)
    est = sg.sgtv_workspace_bytes(prob.I, prob.J, prob.nnz, storage)
    R = sg.Reconstructor()
    R.set_problem(prob, storage=storage)
    held = R.device_bytes()
    print("workspace", cfg, storage, "estimate", est, "held", held, flush=True)
    assert held > 0
    if cfg != "small":     # the fixed 1 MiB of scratch dominates tiny systems
        assert abs(est - held) <= 0.25 * held
    assert sg.sgtv_workspace_bytes(-1, 1, 1) == -1
    R.close()


def test_tiles_with_and_without_row_balancing(sg):
    """24-bit lists deal each tile's rows to the waves by their entry counts
    unless the per-row-block counts (slabs x rows x column blocks) pass 2^24;
    then the rows keep their contiguous order.  With 16 x 64 rows per row block
    and 12-column blocks the forward product (262144 columns, 21846 blocks)
    takes the contiguous order and the back product (32768 columns, 2731
    blocks) the dealt one; both must match the oracle."""
    for rows, blocks in ((16 * 64, 21846), (16 * 64, 2731)):
        assert (rows * blocks > 1 << 24) == (blocks == 21846)
    prob = datagen.make_problem(dict(ny=32, nx=32, Q=256, I=32768, nnz_per_col=8, rects=3, beta=0.1),
                                seed=31)
    assert prob.J == 262144 and -(-prob.J // 12) == 21846
    sched = dict(format=0, waves=16, fwd_rows_per_wave=64, fwd_block_cols=12, fwd_slabs=1,
                 back_rows_per_wave=64, back_block_cols=12, back_slabs=1)
    check_against_oracle(sg, prob, 20, schedule=sched)


FUSED_CASES = {
    "small": dict(cfg="small", seed=1),
    "teflon weights": dict(cfg="teflon", seed=1, w="dir"),
    "teflon standard TV": dict(cfg="teflon", seed=2, w="dir", grouping=1),
    "full weights": dict(cfg=dict(ny=9, nx=13, Q=24, I=1500, nnz_per_col=8, rects=3), seed=4, w="full"),
    "Q=1": dict(cfg=dict(ny=40, nx=23, Q=1, I=700, nnz_per_col=6, rects=3), seed=5),
    "Q=129": dict(cfg=dict(ny=6, nx=11, Q=129, I=4000, nnz_per_col=8, rects=2), seed=6),
    "one row": dict(cfg=dict(ny=1, nx=37, Q=16, I=300, nnz_per_col=6, rects=1), seed=7),
    "3 sweeps": dict(cfg="small", seed=8, sweeps=3),
    "bf16 values": dict(cfg="small", seed=9, storage="bf16"),
}


@pytest.mark.parametrize("name", list(FUSED_CASES))
def test_fused_update_equals_two_launches(sg, name):
    """The image and split update in one pass give the images, splits and
    reports of the two separate launches bit for bit (tile edges, partial
    tiles, grid borders, weights, both groupings, several sweeps, 16-bit
    values), and the fused pass is the one in use."""
    c = FUSED_CASES[name]
    prob = datagen.make_problem(c["cfg"], c["seed"])
    w = None
    if c.get("w") == "dir":
        w = prob.meta["weights"]
    elif c.get("w") == "full":
        w = np.random.default_rng(3).uniform(0.5, 2.0, 4 * prob.J).astype(np.float32)
    out = []
    for fused in (True, False):
        R = sg.Reconstructor()
        R.set_fused_update(fused)
        R.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, prob.val,
                     storage=c.get("storage", "f32"), w=w)
        if c.get("grouping"):
            R.set_grouping(c["grouping"])
        R.set_data(prob.y, prob.r, prob.beta, prob.rho, c.get("sweeps", 1))
        active, tx, ty = R.fused_update()
        print(name, "fused" if fused else "two launches", "active", active, "tile", tx, ty, flush=True)
        assert active == fused and tx > 0 and ty > 0
        R.iterate(17)
        R.iterate(4)
        out.append((R.image(), *R.split(), R.objective()))
        R.close()
    for a, b in zip(out[0][:3], out[1][:3]):
        np.testing.assert_array_equal(a, b)
    assert out[0][3] == out[1][3]


def test_caller_owned_workspace(sg):
    """Two-phase set-up: the exact size from sgtv_plan_system, a torch tensor
    as the workspace, no device memory of the library's own afterwards, and
    the same iterations (bit for bit) as a context that allocates itself;
    every call that needs temporaries works inside the workspace."""
    import torch
    prob = datagen.make_problem("small", 3)
    ref = run_gpu(sg, prob, 0)
    R = sg.Reconstructor()
    with pytest.raises(sg.SgtvError) as ei:
        R.commit_system(torch.empty(1024, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == sg.SGTV_ESTATE
    nbytes = R.plan_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, prob.val)
    print("planned workspace", nbytes, "bytes; library-allocated context holds", ref.device_bytes(), flush=True)
    assert nbytes > 0
    small = torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(sg.SgtvError) as ei:
        R.commit_system(small)
    assert ei.value.code == sg.SGTV_ENOMEM
    ws = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(sg.SgtvError) as ei:
        sg.sgtv_commit_system(R._ctx, ws.data_ptr() + 4, nbytes)
    assert ei.value.code == sg.SGTV_EINVAL
    R.commit_system(ws, nbytes)
    R.set_data(prob.y, prob.r, prob.beta, prob.rho, 1)
    assert R.device_bytes() == 0
    for Rx in (R, ref):
        Rx.iterate(30)
    np.testing.assert_array_equal(R.image(), ref.image())
    assert R.objective() == ref.objective()
    f_o, _, _, _ = oracle.admm(prob, 30, report=False)
    assert rel_l2(R.image(), f_o) <= IMG_TOL
    # temporaries and state changes inside the workspace
    d1, c1 = R.split()
    d2, c2 = ref.split()
    np.testing.assert_array_equal(d1, d2)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_array_equal(R.backprojection(), ref.backprojection())
    st = R.state()
    R.iterate(5)
    R.set_state(*st)
    R.iterate(5)
    ref.iterate(5)
    np.testing.assert_array_equal(R.image(), ref.image())
    for Rx in (R, ref):
        Rx.set_grouping(1)
        Rx.set_init_dual(ref.image())
        Rx.iterate(7)
    np.testing.assert_array_equal(R.image(), ref.image())
    for Rx in (R, ref):
        Rx.set_data(prob.y * np.float32(2), prob.r, prob.beta, prob.rho, 1)
        Rx.set_init(np.full(prob.J, 0.5, np.float32))
        Rx.iterate(9)
    np.testing.assert_array_equal(R.image(), ref.image())
    assert R.device_bytes() == 0
    R.close()
    ref.close()
    del ws


def test_workspace_of_the_paper_scale_scan(sg):
    """The planned size of the paper-scale scan, its set-up in a torch tensor
    and two iterations equal to a library-allocated context."""
    import torch
    prob = datagen.make_problem("paper", 1)
    R = sg.Reconstructor()
    nbytes = R.plan_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, prob.val)
    est = sg.sgtv_workspace_bytes(prob.I, prob.J, prob.nnz, "f32")
    print("paper scan workspace", nbytes, "estimate", est, flush=True)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    R.commit_system(ws)
    R.set_data(prob.y, prob.r, prob.beta, prob.rho, 1)
    R.iterate(2)
    ref = run_gpu(sg, prob, 2)
    np.testing.assert_array_equal(R.image(), ref.image())
    assert R.device_bytes() == 0 and ref.device_bytes() > 0.8 * nbytes
    R.close()
    ref.close()


def _degenerate(kind):
    import dataclasses
    if kind == "no entries":
        p = datagen.make_problem("small", 41)
        return dataclasses.replace(p, rowptr=np.zeros(p.I + 1, np.int64), col=np.zeros(0, np.int32),
                                   val=np.zeros(0, np.float32))
    if kind == "one measurement":
        p = datagen.make_problem(dict(ny=6, nx=5, Q=8, I=1, nnz_per_col=1, rects=2), 42)
        return p
    if kind == "one voxel":
        return datagen.make_problem(dict(ny=1, nx=1, Q=1, I=50, nnz_per_col=7, rects=1), 43)
    if kind == "one spatial bin":
        return datagen.make_problem(dict(ny=1, nx=1, Q=40, I=300, nnz_per_col=5, rects=1), 44)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["no entries", "one measurement", "one voxel", "one spatial bin"])
@pytest.mark.parametrize("fmt", [0, 1])
def test_degenerate_systems(sg, kind, fmt):
    """A matrix without entries (the image stays at the zero start: the uniform
    start is 0 when A^T 1 = 0, the EM step keeps 0), a single measurement, a
    single voxel and a single spatial bin (no neighbours: the penalty
    vanishes), in both formats, against the oracle."""
    prob = _degenerate(kind)
    check_against_oracle(sg, prob, 15, schedule=dict(format=fmt))
