"""Host-side schedule rules (no GPU): candidate ranking limits, the slab rule
and the batch rule."""
from paper_1601_08201_amd import autotune


def test_candidates_fit_lds_and_slabs():
    fwd, back = autotune.candidates(1 << 20, 1 << 21)
    assert fwd and back
    for rw, cb, ns in fwd + back:
        assert autotune.lds_bytes(16, rw, cb) <= autotune.MAX_LDS
        assert ns in (1, 2, 4, 8)


def test_auto_slabs_keep_slab_at_most_2mib():
    for n in (1, 100, 4096, 1 << 19, (1 << 19) + 1, 1 << 21, 3 << 20, 1 << 22, 10 ** 8):
        ns = autotune._auto_slabs(n)
        assert 1 <= ns <= 8 and ns & (ns - 1) == 0
        if ns < 8:
            assert n * 4 / ns <= 2 ** 21 or -(-n // 16380) == ns


def test_batch_schedule_prefers_long_tiles_for_big_batches():
    big = [(ny * nx * q // 2, ny * nx * q) for ny, nx, q in [(128, 128, 128)] * 32 + [(64, 64, 96)] * 32]
    assert autotune.batch_schedule(big) == dict(fwd_rows_per_wave=1024, back_rows_per_wave=1024)
    # a handful of tiny scans cannot fill the GPU with long tiles
    tiny = [(8192, 19926)] * 16
    assert autotune.batch_schedule(tiny) == dict(fwd_rows_per_wave=64, back_rows_per_wave=64)
    # in between, the tile count over the batch decides
    mid = [(1 << 18, 1 << 19)] * 8
    s = autotune.batch_schedule(mid, min_tiles=256)
    rw = s["fwd_rows_per_wave"]
    tiles = lambda r: sum(-(-I // (16 * r)) * autotune._auto_slabs(J) for I, J in mid)
    assert tiles(rw) >= 256 and (rw == 1024 or tiles(2 * rw) < 256 or
                                 sum(-(-J // (32 * rw)) * autotune._auto_slabs(I) for I, J in mid) < 256)


def test_batch_tuner_candidates_and_cache_key(tmp_path):
    """The batch tuner times the rule's tile height and the two next shorter
    ones; its cache key depends on every scan's shape and entry count and on
    their order, and a cached entry is returned for the same batch only."""
    import json
    from types import SimpleNamespace as NS
    from paper_1601_08201_amd import autotune
    sizes = [(32768, 65536)] * 64
    cands = autotune.batch_candidates(sizes)
    rule = autotune.batch_schedule(sizes)["fwd_rows_per_wave"]
    assert [c["fwd_rows_per_wave"] for c in cands] == [r for r in (rule, rule // 2, rule // 4) if r >= 64]
    assert all(c["fwd_rows_per_wave"] == c["back_rows_per_wave"] for c in cands)
    a = [NS(I=100, ny=4, nx=5, Q=6, nnz=1000), NS(I=200, ny=8, nx=5, Q=6, nnz=2000)]
    b = list(reversed(a))
    c = [a[0], NS(I=200, ny=8, nx=5, Q=6, nnz=2001)]
    keys = {autotune.batch_key(x) for x in (a, b, c)}
    assert len(keys) == 3
    path = str(tmp_path / "cache.json")
    with open(path, "w") as fh:
        json.dump({autotune.batch_key(a): {"schedule": {"fwd_rows_per_wave": 512, "back_rows_per_wave": 512}}}, fh)
    assert autotune.cached_batch_schedule(a, path) == {"fwd_rows_per_wave": 512, "back_rows_per_wave": 512}
    assert autotune.cached_batch_schedule(b, path) is None


def test_schedule_cache_keys_by_value_type(tmp_path):
    """16-bit value types look up an entry of their own and fall back to the
    FP32 entry of the same shape."""
    import json
    from types import SimpleNamespace as NS
    from paper_1601_08201_amd import autotune
    p = NS(I=1000, ny=4, nx=5, Q=6, nnz=777)
    k32 = autotune.shape_key(p.I, p.ny, p.nx, p.Q, p.nnz)
    kb = autotune.shape_key(p.I, p.ny, p.nx, p.Q, p.nnz, "bf16")
    assert kb != k32 and kb.startswith(k32)
    path = str(tmp_path / "cache.json")
    with open(path, "w") as fh:
        json.dump({k32: {"schedule": {"fwd_rows_per_wave": 2048}}, kb: {"schedule": {"fwd_rows_per_wave": 1024}}}, fh)
    assert autotune.cached_schedule(p, path) == {"fwd_rows_per_wave": 2048}
    assert autotune.cached_schedule(p, path, storage="bf16") == {"fwd_rows_per_wave": 1024}
    assert autotune.cached_schedule(p, path, storage="f16") == {"fwd_rows_per_wave": 2048}


def test_tuner_picks_the_fastest_iteration_among_finalists(tmp_path, monkeypatch):
    """The tuner times every candidate's products, pairs the two fastest
    forward and the two fastest back parameters, and keeps the pairing whose
    whole iteration is fastest (which need not be the fastest products); the
    result is cached under the shape and value type."""
    import json
    import sys
    import types
    from types import SimpleNamespace as NS
    from paper_1601_08201_amd import autotune
    prob = NS(I=1 << 20, J=1 << 21, ny=128, nx=128, Q=128, nnz=1 << 27)
    fwd_us = {}   # forward product time by (rows, block, slabs): prefer many rows
    back_us = {}

    def fake_products(p, sched, reps, warmup=10, storage="f32"):
        f = (sched["fwd_rows_per_wave"], sched["fwd_block_cols"], sched["fwd_slabs"])
        b = (sched["back_rows_per_wave"], sched["back_block_cols"], sched["back_slabs"])
        fwd_us[f] = 300.0 - f[0] / 16.0 - f[1] / 1000.0
        back_us[b] = 300.0 - b[0] / 16.0 - b[1] / 1000.0
        return fwd_us[f], back_us[b]

    def fake_iteration(p, sched, reps, warmup=10, storage="f32"):
        # the iteration also pays per slab (ratio and image update partial sums)
        return (fwd_us[(sched["fwd_rows_per_wave"], sched["fwd_block_cols"], sched["fwd_slabs"])]
                + back_us[(sched["back_rows_per_wave"], sched["back_block_cols"], sched["back_slabs"])]
                + 5.0 * (sched["fwd_slabs"] + sched["back_slabs"])) / 1e3

    monkeypatch.setattr(autotune, "_time_schedule", fake_products)
    monkeypatch.setattr(autotune, "_time_iteration", fake_iteration)
    monkeypatch.setitem(sys.modules, "torch", types.SimpleNamespace(cuda=types.SimpleNamespace(init=lambda: None)))
    path = str(tmp_path / "cache.json")
    best, report = autotune.tune(prob, max_candidates=8, cache_path=path, storage="bf16")
    timed = [r for r in report if "iteration_ms" in r]
    assert len(timed) == 4                     # two forward x two back finalists
    fastest = min(timed, key=lambda r: r["iteration_ms"])
    assert best == fastest["schedule"]
    top_f = sorted(fwd_us.values())[:2]
    assert fwd_us[(best["fwd_rows_per_wave"], best["fwd_block_cols"], best["fwd_slabs"])] in top_f
    rec = json.load(open(path))[autotune.shape_key(prob.I, prob.ny, prob.nx, prob.Q, prob.nnz, "bf16")]
    assert rec["schedule"] == best and rec["iteration_ms"] == fastest["iteration_ms"]
