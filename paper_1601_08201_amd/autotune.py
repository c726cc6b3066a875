"""Autotuner for the launch schedule of the tiled sparse products.

For one system the tuner builds the tiled matrices under a list of candidate
schedules (rows per wave, column-block width, number of slabs, inner-loop
variant), times the forward and the back product with HIP events on the
device, and keeps the fastest forward and the fastest back parameters
independently (the two products share no data layout).  Results are cached
per problem shape in a JSON file so a batch of scans tunes every distinct
shape once.
"""
from __future__ import annotations

import json
import os
import time

from . import sgtv

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "schedules.json")
MAX_LDS = 163840


def idx24_fits(rw, cb):
    """Whether the simple loop stores this tile's indices in 24 bits: row in
    10 bits and column in 14 up to 1024 rows per wave, 11 and 13 up to 2048."""
    return 64 <= rw <= 2048 and cb % 4 == 0 and cb <= (1 << (14 if rw <= 1024 else 13)) - 4


def lds_bytes(waves, rw, cb, variant=1):
    """LDS of one workgroup: the row sums (a spare row per wave with 32-bit
    indices), the column block and the zero slot of the 24-bit format."""
    i24 = variant == 1 and idx24_fits(rw, cb)
    a = waves * (rw + (0 if i24 else 1)) * 4
    a = (a + 15) // 16 * 16
    return a + cb * 4 + (16 if i24 else 0)


def shape_key(I, ny, nx, Q, nnz, storage="f32"):
    """Cache key of a problem shape; 16-bit value types have entries of their
    own (their products and image update weigh differently)."""
    key = "I%d_g%dx%dx%d_nnz%d" % (I, ny, nx, Q, nnz)
    return key if storage == "f32" else key + "_" + storage


def candidates(I, J, waves=16, per_side=10):
    """Ranked candidate (rows per wave, block columns, slabs) for the forward
    product (rows = measurements) and the back product (rows = voxels)."""
    import math

    def side(n_rows, n_cols):
        out = []
        for rw in (64, 128, 256, 512, 1024, 2048):
            for cb in (4096, 8188, 16380):
                cb_eff = min(cb, max(4, 1 << (max(n_cols, 4) - 1).bit_length()))
                if lds_bytes(waves, rw, cb_eff) > MAX_LDS:
                    continue
                n_cb = -(-n_cols // cb_eff)
                for ns in (1, 2, 4, 8):
                    if ns > n_cb:
                        continue
                    tiles = -(-n_rows // (waves * rw)) * ns
                    slab = n_cols * 4 / ns
                    entries = rw * cb_eff * 1.0   # list length scales with this (fixed density)
                    # heuristic rank: ~256-512 workgroups, ~2 MiB slabs, long lists
                    score = (abs(math.log2(max(tiles, 1) / 384.0)) + 0.5 * abs(math.log2(slab / 2 ** 21))
                             - 0.25 * math.log2(entries / 2 ** 24))
                    out.append((score, (rw, cb_eff, ns)))
        out.sort()
        seen, ranked = set(), []
        for _, c in out:
            if c not in seen:
                seen.add(c)
                ranked.append(c)
        return ranked[:per_side]
    return side(I, J), side(J, I)


def _auto_slabs(n_cols):
    """Slab count of the automatic schedule (slab of the gathered vector <= 2 MiB)."""
    cb = min(16380, max(4, 1 << (max(n_cols, 4) - 1).bit_length()))
    n_cb = -(-n_cols // cb)
    want = 1 << max(0, (-(-(n_cols * 4) // 2 ** 21) - 1).bit_length())
    return max(1, min(want, 8, n_cb))


def batch_schedule(sizes, waves=16, min_tiles=1024):
    """One schedule for every scan of a batch, sizes = [(I, J), ...]: the
    largest rows per wave (up to 1024) whose forward and back tiles over the
    whole batch still number at least min_tiles.  A single scan must fill the
    GPU by itself and so takes short tiles; in a batch the scans fill it
    together, and longer tiles stage each gathered block for more entries."""
    rw = 1024
    while rw > 64:
        tf = sum(-(-I // (waves * rw)) * _auto_slabs(J) for I, J in sizes)
        tb = sum(-(-J // (waves * rw)) * _auto_slabs(I) for I, J in sizes)
        if min(tf, tb) >= min_tiles:
            break
        rw //= 2
    return dict(fwd_rows_per_wave=rw, back_rows_per_wave=rw)


def batch_key(probs):
    """Cache key of a batch: its scans' shapes and entry counts, in order."""
    import hashlib
    desc = ";".join(shape_key(p.I, p.ny, p.nx, p.Q, p.nnz) for p in probs)
    return "batch%d_%s" % (len(probs), hashlib.sha1(desc.encode()).hexdigest()[:16])


def batch_candidates(sizes, waves=16):
    """Schedules the batch tuner times: the rule's choice and the two next
    shorter tile heights (column blocks and slabs automatic per scan)."""
    rule = batch_schedule(sizes, waves)["fwd_rows_per_wave"]
    out = []
    for rw in (rule, rule // 2, rule // 4):
        if rw >= 64:
            out.append(dict(fwd_rows_per_wave=rw, back_rows_per_wave=rw))
    return out


def tune_batch(probs, reps=5, threads=8, log=None, cache_path=CACHE_PATH, stream=None):
    """Time the batch (graph replay of `reps` iterations after 2 warm-up
    iterations) under each candidate schedule and keep the fastest; the result
    is cached under batch_key(probs)."""
    import concurrent.futures as cf
    import torch
    sizes = [(p.I, p.J) for p in probs]
    report = []
    t0 = time.time()
    for sched in batch_candidates(sizes):
        B = sgtv.Batch(stream=stream)
        tb = time.time()
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda p: B.add_scan(p, sched), probs))
        build = time.time() - tb
        B.iterate(2)
        B.prepare(reps)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st = torch.cuda.current_stream()
        a.record(st)
        B.iterate(reps)
        b.record(st)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        B.close()
        report.append(dict(schedule=sched, ms_per_iteration=ms, build_seconds=build))
        if log:
            log("batch autotune %s: %.3f ms per iteration (built in %.1fs)" % (json.dumps(sched), ms, build))
    best = min(report, key=lambda r: r["ms_per_iteration"])
    if cache_path:
        cache = load_cache(cache_path)
        cache[batch_key(probs)] = dict(schedule=best["schedule"], ms_per_iteration=best["ms_per_iteration"],
                                       candidates=report, seconds=time.time() - t0)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best["schedule"], report


def cached_batch_schedule(probs, path=CACHE_PATH):
    """The timed schedule of this batch, or None (then the batch rule applies)."""
    rec = load_cache(path).get(batch_key(probs))
    return rec["schedule"] if rec else None


def _time_schedule(prob, sched, reps, warmup=10, storage="f32"):
    """Average forward and back product times (us) over `reps` iterations
    after `warmup` iterations, HIP events around every launch."""
    R = sgtv.Reconstructor()
    R.set_schedule(format=0, **sched)
    R.set_problem(prob, storage=storage)
    R.set_graphs(False)
    R.iterate(warmup)
    R.set_profiling(True)
    R.iterate(reps)
    t = R.kernel_times()
    R.close()
    return t["forward"][0] / t["forward"][1] * 1e3, t["back"][0] / t["back"][1] * 1e3


def _time_iteration(prob, sched, reps, warmup=10, storage="f32"):
    """Milliseconds per ADMM iteration (graph replay of `reps` iterations
    after `warmup`): the products and the ratio and update kernels, whose
    partial-sum reads grow with the slab counts."""
    import torch
    R = sgtv.Reconstructor()
    R.set_schedule(format=0, **sched)
    R.set_problem(prob, storage=storage)
    R.iterate(warmup)
    R.prepare(reps)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    R.iterate(reps)
    b.record()
    torch.cuda.synchronize()
    R.close()
    return a.elapsed_time(b) / reps


def tune(prob, reps=20, max_candidates=10, variants=(1,), log=None, cache_path=CACHE_PATH, finalists=2,
         iter_reps=100, storage="f32"):
    """Time candidate schedules on the device; return (schedule dict, report).

    Every candidate's forward and back products are timed; the `finalists`
    fastest parameters of each product are then combined and the whole
    iteration of every combination is timed, and the fastest iteration wins
    (more slabs make the products faster but give the ratio and image update
    more partial sums to add)."""
    import torch
    torch.cuda.init()   # before the library's first HIP call (the iteration timing uses torch events)
    I, J = prob.I, prob.J
    fw, bk = candidates(I, J, per_side=max_candidates)
    # pair forward and back candidates so each build measures both products
    n = max(len(fw), len(bk))
    pairs = [(fw[k % len(fw)], bk[k % len(bk)]) for k in range(n)][:max_candidates]
    timed_f, timed_b = [], []
    report = []
    t0 = time.time()
    for (f, b) in pairs:
        for v in variants:
            sched = dict(waves=16, variant=v, fwd_rows_per_wave=f[0], fwd_block_cols=f[1], fwd_slabs=f[2],
                         back_rows_per_wave=b[0], back_block_cols=b[1], back_slabs=b[2])
            try:
                tf, tb = _time_schedule(prob, sched, reps, storage=storage)
            except sgtv.SgtvError as e:
                report.append(dict(schedule=sched, error=str(e)))
                continue
            report.append(dict(schedule=sched, forward_us=tf, back_us=tb))
            if log:
                log("autotune %s: forward %.1f us, back %.1f us" % (json.dumps(sched), tf, tb))
            timed_f.append((tf, f, v))
            timed_b.append((tb, b, v))
    if not timed_f:
        return {}, report
    # finalists of each product (distinct parameters, fastest first), combined
    def top(timed):
        out, seen = [], set()
        for t in sorted(timed, key=lambda e: e[0]):
            if (t[1], t[2]) not in seen:
                seen.add((t[1], t[2]))
                out.append(t)
        return out[:finalists]
    best = None
    for ff in top(timed_f):
        for bb in top(timed_b):
            # one variant per launch family: take the forward product's
            sched = dict(waves=16, variant=ff[2],
                         fwd_rows_per_wave=ff[1][0], fwd_block_cols=ff[1][1], fwd_slabs=ff[1][2],
                         back_rows_per_wave=bb[1][0], back_block_cols=bb[1][1], back_slabs=bb[1][2])
            ms = _time_iteration(prob, sched, iter_reps, storage=storage)
            report.append(dict(schedule=sched, iteration_ms=ms))
            if log:
                log("autotune %s: %.4f ms per iteration" % (json.dumps(sched), ms))
            if best is None or ms < best[0]:
                best = (ms, sched, ff[0], bb[0])
    if cache_path:
        cache = load_cache(cache_path)
        cache[shape_key(I, prob.ny, prob.nx, prob.Q, prob.nnz, storage)] = dict(
            schedule=best[1], forward_us=best[2], back_us=best[3], iteration_ms=best[0],
            seconds=time.time() - t0, candidates=len(report))
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return best[1], report


def load_cache(path=CACHE_PATH):
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def cached_schedule(prob, path=CACHE_PATH, storage="f32"):
    """The tuned schedule for this problem's shape, or None (automatic)."""
    cache = load_cache(path)
    key = shape_key(prob.I, prob.ny, prob.nx, prob.Q, prob.nnz)
    # 16-bit values: their own entry, else the FP32 one
    rec = cache.get(shape_key(prob.I, prob.ny, prob.nx, prob.Q, prob.nnz, storage)) or cache.get(key)
    return rec["schedule"] if rec else None


def _batch_scan(ny, nx, Q, seed):
    from . import datagen
    return datagen.make_batch_scan(ny, nx, Q, seed=seed)


def _main():
    import argparse
    import sys

    from . import datagen
    ap = argparse.ArgumentParser(description="tune the tiled-product schedules of standard workloads")
    ap.add_argument("--workloads", default="paper,warmstart,batch")
    ap.add_argument("--out", default=CACHE_PATH)
    ap.add_argument("--candidates", type=int, default=8)
    ap.add_argument("--storage", default="f32", help="value types to tune for, comma-separated (f32, bf16, f16)")
    ap.add_argument("--batch-scans", type=int, default=64)
    ap.add_argument("--tune-batch", action="store_true",
                    help="time the schedules of the whole batch workload (its scans, seeds 300 + k) instead")
    args = ap.parse_args()
    log = lambda m: print("[autotune] " + m, file=sys.stderr, flush=True)
    if args.tune_batch:
        import multiprocessing as mp
        shapes = datagen.batch_shapes(args.batch_scans, 300)
        with mp.get_context("fork").Pool(min(16, len(shapes))) as pool:
            probs = pool.starmap(_batch_scan, [(ny, nx, Q, 300 + k) for k, (ny, nx, Q) in enumerate(shapes)])
        log("generated %d scans" % len(probs))
        best, _ = tune_batch(probs, log=log, cache_path=args.out)
        log("batch of %d scans: best %s" % (len(probs), json.dumps(best)))
        return
    probs = []
    for w in args.workloads.split(","):
        if w in ("paper", "warmstart", "small"):
            probs.append(datagen.make_problem(w, 1))
        elif w == "batch":
            seen = set()
            for (ny, nx, Q) in datagen.batch_shapes(args.batch_scans, 300):
                if (ny, nx, Q) not in seen:
                    seen.add((ny, nx, Q))
                    probs.append(datagen.make_batch_scan(ny, nx, Q, seed=900))
    for p in probs:
        t0 = time.time()
        for st in args.storage.split(","):
            best, rep = tune(p, max_candidates=args.candidates, log=log, cache_path=args.out, storage=st)
            log("shape %dx%dx%d I=%d %s: best %s (%.1fs)" % (p.ny, p.nx, p.Q, p.I, st, json.dumps(best),
                                                             time.time() - t0))


if __name__ == "__main__":
    _main()
