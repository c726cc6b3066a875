#!/usr/bin/env python3
"""Throughput of the ADMM iteration for spectrally grouped TV reconstruction.

One step = one ADMM iteration (forward projection and ratio, backprojection
with the per-voxel image update, group shrink and dual update) on the
paper-scale synthetic scan: 128 x 128 spatial x 128 spectral bins
(2,097,152 unknowns), 1,048,576 measurements, 64 system-matrix entries per
column (134,217,728 nonzeros).  Inputs are seeded synthetic data resident in
HBM before timing starts.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 200] [--warmup 10] [--storage f32|bf16|f16]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(prob, value_bytes, fmt, fused=False, epilogues=False, full_weights=False):
    """Bytes each kernel must move per launch: every array it needs, touched once.

    Tiled format: forward = A (values + indices), x, p out; ratio = p, y, r,
    ratio out; back = A, ratio, e out; image update = e, g, v, a, sens, g out
    (and H with full weights; with weights constant per direction H0 comes
    from a 16-entry table); split = f, v, a in and v, a out; the image and
    split update in one pass (fused) = e, g, sens, g out, v and a in and out
    (48 J + 8 S bytes).  With the row-block epilogues the forward launch
    includes the ratio (A, x, y, r in, ratio out) and the back launch the
    image update (A, ratio, g, v, a, sens in, g out): the partial sums between
    them are not part of the count.  The sliced-ELL kernels fuse the ratio
    into the forward pass and the image update into the back pass.
    """
    I, J, nnz = prob.I, prob.J, prob.nnz
    S = prob.ny * prob.nx
    a = nnz * (value_bytes + 4)
    h = 4 * J if full_weights else 0
    out = {"split_update": 4 * J + 16 * J + 4 * S + 16 * J + 4 * S}
    if fmt == "tiled":
        out["forward"] = a + 4 * J + 4 * I
        out["ratio"] = 16 * I
        out["back"] = a + 4 * I + 4 * J
        out["image_update"] = 4 * J + 4 * J + 16 * J + 4 * S + 4 * J + h + 4 * J
        if epilogues:
            del out["ratio"], out["image_update"]
            out["forward"] = a + 4 * J + 12 * I
            out["back"] = a + 4 * I + 4 * J + 16 * J + 4 * S + 4 * J + h + 4 * J
        if fused:
            out.pop("split_update")
            out.pop("image_update", None)
            out["back"] = a + 4 * I + 4 * J
            out["update_fused"] = 4 * J + 4 * J + 4 * J + 4 * J + 32 * J + 8 * S
    else:
        out["forward"] = a + 4 * (I + 1) + 4 * J + 12 * I
        out["back"] = a + 4 * (J + 1) + 4 * I + 32 * J + 4 * S
    return out


PRODUCT_SOURCES = ("sgtv_tiled.hip", "sgtv_device.h", "sgtv_kernels.h")


def _code_only(src):
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_fingerprint(schedule=None):
    """SHA-256 of what decides the bytes the products stream: the product
    kernels' sources (sgtv_tiled.hip, sgtv_device.h, sgtv_kernels.h), the host
    builder of the tiled format in sgtv_api.hip (automatic schedule, packing,
    upload) and the schedule in use, with comments and white space removed: a
    counter summary stays valid across edits of comments only."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1601_08201_amd", "csrc")
    for f in PRODUCT_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            h.update(_code_only(fh.read()).encode())
    with open(os.path.join(csrc, "sgtv_api.hip")) as fh:
        api = fh.read()
    a, b = api.find("TileParams choose_tiles("), api.find("struct System {")
    if a >= 0 and b > a:
        h.update(_code_only(api[a:b]).encode())
    if schedule is not None:
        h.update(json.dumps(schedule, sort_keys=True).encode())
    return h.hexdigest()


PRODUCT_PROFILE = os.path.join("profiles", "tiled_product_fp32_paper_scan.md")


def measured_traffic(kernel, storage, fmt, config, schedule=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when there is none for this workload or the kernels, the builder or the
    schedule changed since it was taken."""
    import re
    if storage != "f32" or fmt != "tiled" or config != "paper" or kernel not in ("forward", "back"):
        return None
    path = os.path.join(ROOT, PRODUCT_PROFILE)
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if kernel_fingerprint(schedule) != rec.get("kernel_source_sha256"):
        return None
    return rec["traffic_bytes_per_launch"].get(kernel)


def host_threads():
    """Threads the oracle may use on this host: the CPUs this process may run
    on, capped by OMP_NUM_THREADS when it is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_problem(prob):
    """The scan with FP64 arrays (widened once, outside any timing)."""
    import numpy as np

    class P:
        pass
    p = P()
    p.__dict__.update(dict(ny=prob.ny, nx=prob.nx, Q=prob.Q, I=prob.I, J=prob.J, rowptr=prob.rowptr,
                           col=prob.col, val=prob.val.astype(np.float64), y=prob.y.astype(np.float64),
                           r=prob.r.astype(np.float64), beta=prob.beta, rho=prob.rho, sweeps=prob.sweeps))
    return p


def oracle_run(p, iters, threads, **kw):
    """The FP64 oracle from the uniform start on `threads` threads: (image, iterations per
    second of the iteration loop alone, loop seconds)."""
    import numpy as np
    import oracle
    oracle.set_threads(threads)
    f0 = np.full(p.J, oracle.plain_init(p), np.float64)
    f, _, _, _ = oracle.admm(p, iters, f0=f0, report=False, **kw)
    sec = oracle.last_loop_seconds()
    return f, iters / sec, sec


def oracle_error(p, f_gpu, f_or, **kw):
    """Image relative L2 error and relative objective error of a GPU image against the
    oracle's image after the same iterations, both objectives from the oracle (FP64)."""
    import numpy as np
    import oracle
    g = f_gpu.astype(np.float64)
    rel_l2 = float(np.linalg.norm(g - f_or) / max(np.linalg.norm(f_or), 1e-300))
    phi_g = oracle.objective(p, g, **kw)[0]
    phi_o = oracle.objective(p, f_or, **kw)[0]
    return {"image_rel_l2": rel_l2, "objective_rel": abs(phi_g - phi_o) / abs(phi_o)}


def _gen_batch_scan(args):
    from paper_1601_08201_amd import datagen
    ny, nx, Q, seed = args
    return datagen.make_batch_scan(ny, nx, Q, seed=seed)


def system_file_times(R, prob, stream):
    """Save the packed system and load it into a second context: the set-up
    of a fixed scanner after the first time."""
    import shutil
    import tempfile
    from paper_1601_08201_amd import sgtv
    tmp = tempfile.mkdtemp(prefix="sgtv_system_")
    try:
        if shutil.disk_usage(tmp).free < 1.5 * (16 * prob.nnz + 64 * prob.J):
            log("system file skipped: not enough space in " + tmp)
            return {}
        path = os.path.join(tmp, "system.sys")
        t0 = time.time()
        R.save_system(path)
        t_save = time.time() - t0
        R2 = sgtv.Reconstructor(device=0, stream=stream.cuda_stream)
        t0 = time.time()
        R2.load_system(path)
        t_load = time.time() - t0
        R2.close()
        size = os.path.getsize(path)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    log("system file: %.2f GB saved in %.2fs, loaded in %.3fs" % (size / 1e9, t_save, t_load))
    return {"save_s": t_save, "load_system_s": t_load, "file_bytes": size}


def batch_from_files(B, probs, index, stream, setup):
    """Save every scan's packed system to a file, then build the batch again
    from the files (the set-up of a fixed set of scanners after the first
    time); returns the rebuilt batch, which iterates bit for bit like the
    packed one, and the set-up times."""
    import shutil
    import tempfile
    from paper_1601_08201_amd import sgtv
    tmp = tempfile.mkdtemp(prefix="sgtv_systems_")
    need = sum(16 * p.nnz + 64 * p.J for p in probs)
    free = shutil.disk_usage(tmp).free
    if free < 1.5 * need:
        log("system files skipped: %.1f GB free in %s, %.1f GB needed" % (free / 1e9, tmp, need / 1e9))
        shutil.rmtree(tmp, ignore_errors=True)
        return B, setup
    try:
        paths = [os.path.join(tmp, "scan%03d.sys" % k) for k in range(len(probs))]
        t0 = time.time()
        for k, path in enumerate(paths):
            B.save_scan(index[k], path)
        t_save = time.time() - t0
        size = sum(os.path.getsize(x) for x in paths)
        B.close()
        B = sgtv.Batch(stream=stream.cuda_stream)
        t0 = time.time()
        for path, p in zip(paths, probs):
            B.add_system_file(path, p)
        t_load = time.time() - t0
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    log("system files: saved %.1f GB in %.1fs, batch rebuilt from them in %.2fs" % (size / 1e9, t_save, t_load))
    return B, dict(setup, from_files_s=t_load, save_s=t_save, file_bytes=size)


def batch_main(args):
    """Batch of uneven scans: batched launches (one graph per call, the batch
    schedule) against the same scans iterated one after another, each with its
    own single-scan schedule."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import torch
    from paper_1601_08201_amd import autotune, datagen, sgtv

    torch.cuda.set_device(0)
    shapes = datagen.batch_shapes(args.batch_scans, 300)
    t0 = time.time()
    with mp.get_context("fork").Pool(min(16, len(shapes))) as pool:
        probs = pool.map(_gen_batch_scan, [(ny, nx, Q, 300 + k) for k, (ny, nx, Q) in enumerate(shapes)])
    nnz = sum(p.nnz for p in probs)
    unknowns = sum(p.J for p in probs)
    log("generated %d scans: %d unknowns, %d nonzeros in %.1fs" % (len(probs), unknowns, nnz, time.time() - t0))
    stream = torch.cuda.current_stream()
    B = sgtv.Batch(stream=stream.cuda_stream)
    t0 = time.time()
    sched = autotune.cached_batch_schedule(probs)
    sched_source = "timed by the batch autotuner (cache)" if sched else "batch rule"
    if not sched:
        sched = autotune.batch_schedule([(p.I, p.J) for p in probs])
    with cf.ThreadPoolExecutor(8) as ex:
        index = list(ex.map(lambda p: B.add_scan(p, sched), probs))
    t_pack = time.time() - t0
    log("batch built in %.1fs (schedule %s, %s)" % (t_pack, sched, sched_source))
    setup = {"pack_s": t_pack, "from_files_s": None}
    if not args.no_system_files:
        B, setup = batch_from_files(B, probs, index, stream, setup)
        index = list(range(len(probs)))
    B.iterate(args.warmup)
    B.prepare(args.steps)   # graph capture outside the timed region
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    a, b = ev(), ev()
    a.record(stream)
    B.iterate(args.steps)
    b.record(stream)
    torch.cuda.synchronize()
    ms_batched = a.elapsed_time(b)
    # the same batch continued in one cooperative launch per call (persistent kernel)
    B.set_launch("persistent")
    B.iterate(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.iterate(args.steps)
    torch.cuda.synchronize()
    ms_persistent = 1e3 * (time.perf_counter() - t0)
    B.phase_times()
    B.iterate(args.steps)   # again, for the phase clocks of the persistent kernel
    ph, ph_it = B.phase_times()
    phases = {k: v / max(ph_it, 1) for k, v in zip(("forward+split", "ratio", "back", "image_update",
                                                     "last_split"), ph.tolist())}
    log("persistent phases, ms per iteration: " + json.dumps(phases))
    B.set_launch("graph")
    log("batched: graph %.3f ms/iter, persistent %.3f ms/iter (grid %d)"
        % (ms_batched / args.steps, ms_persistent / args.steps, B.launch()[1]))
    # error against the FP64 oracle of the two smallest scans after the same iterations
    err = []
    if not args.no_cpu_baseline:
        nth = host_threads()
        for k in sorted(range(len(probs)), key=lambda k: probs[k].nnz)[:2]:
            p = oracle_problem(probs[k])
            n_done = int(B.objective(index[k])["iter"])   # iterations the scan has run
            f_or, _, _ = oracle_run(p, n_done, nth)
            e = oracle_error(p, B.image(index[k]), f_or)
            err.append(dict(e, scan="%dx%dx%d" % (p.ny, p.nx, p.Q), iterations=n_done))
            log("scan %s after %d iterations vs the FP64 oracle: %s" % (err[-1]["scan"], n_done, json.dumps(e)))
    B.close()
    # the same scans one after another, each with its own single-scan schedule
    # (tuned when cached): a scan launched alone has to fill the GPU by itself
    Bs = sgtv.Batch(stream=stream.cuda_stream)
    t0 = time.time()
    scheds = [autotune.cached_schedule(p) for p in probs]
    with cf.ThreadPoolExecutor(8) as ex:
        list(ex.map(lambda ps: Bs.add_scan(ps[0], ps[1]), zip(probs, scheds)))
    log("sequential reference built in %.1fs (%d scans with tuned schedules)"
        % (time.time() - t0, sum(x is not None for x in scheds)))
    Bs.iterate_sequential(args.warmup)
    Bs.prepare(args.steps, sequential=True)
    torch.cuda.synchronize()
    a.record(stream)
    Bs.iterate_sequential(args.steps)
    b.record(stream)
    torch.cuda.synchronize()
    ms_seq = a.elapsed_time(b)
    Bs.close()
    alg = sum(sum(algorithmic_bytes(p, 4, "tiled").values()) for p in probs)
    scan_its = len(probs) * args.steps
    out = {
        "metric": "aggregate scan-iterations/s, batched launch vs sequential launches",
        "value": scan_its / (ms_batched * 1e-3),
        "unit": "scan-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_batched / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded phantoms, random coded-mask system matrices, Poisson counts)",
        "config": {"workload": "batch of %d scans, side in {32,48,64,96,128}, Q in {64,96,128}, "
                               "I = J/2, 32 nnz/col; %d unknowns, %d nonzeros" % (len(probs), unknowns, nnz),
                   "global_batch": len(probs), "parallelism": "single GPU"},
        "sequential": {"value": scan_its / (ms_seq * 1e-3), "ms_per_step": ms_seq / args.steps},
        "persistent": {"value": scan_its / (ms_persistent * 1e-3), "ms_per_step": ms_persistent / args.steps,
                       "note": "one cooperative launch per call with grid barriers; host clock around the "
                               "call, which waits for the launch",
                       "phase_ms_per_iteration": phases},
        "speedup_vs_sequential": ms_seq / ms_batched,
        "schedule": dict(sched, source=sched_source),
        "setup": dict(setup, note="pack_s: the systems packed on the host (8 scans at a time); "
                                  "from_files_s: the same batch built from the saved packed systems"),
        "batch_iteration_alg_GBs": alg * args.steps / (ms_batched * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "kernel": "whole batched iteration",
                     "achieved": alg * args.steps / (ms_batched * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg * args.steps / (ms_batched * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None},
        "cpu_baseline": None,
        "oracle_error": err or None,
    }
    print(json.dumps(out), flush=True)


def sweep_main(args):
    """The beta sweep of both regularisers on the paper-shaped problem as one
    batch (one batched launch per kernel and iteration), against the same
    scans launched one after another; the images after warmup + steps
    iterations are scored against the phantom."""
    import numpy as np
    import torch
    from paper_1601_08201_amd import datagen, sgtv, study

    torch.cuda.set_device(0)
    prob = datagen.make_problem("teflon", args.seed)
    w = prob.meta["weights"]
    betas = [float(b) for b in args.betas.split(",")]
    pairs = [(g, b) for g in (0, 1) for b in betas]
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def run(sequential, persistent=False):
        B = sgtv.Batch(stream=stream.cuda_stream)
        for g, b in pairs:
            B.add_scan(prob, w=w, grouping=g, beta=b)
        if persistent:
            B.set_launch("persistent")
        it = B.iterate_sequential if sequential else B.iterate
        it(args.warmup)
        B.prepare(args.steps, sequential=sequential)   # graph capture outside the timed region
        torch.cuda.synchronize()
        a, e = ev(), ev()
        a.record(stream)
        it(args.steps)
        e.record(stream)
        torch.cuda.synchronize()
        return B, a.elapsed_time(e)

    B, ms_batched = run(False)
    Bs, ms_seq = run(True)
    Bp, ms_pers = run(False, persistent=True)
    ph, ph_it = Bp.phase_times()
    phases = {k: v / max(ph_it, 1) for k, v in zip(("forward+split", "ratio", "back", "image_update",
                                                     "last_split"), ph.tolist())}
    log("sweep persistent phases, ms per iteration: " + json.dumps(phases))
    same_p = all(np.array_equal(B.image(i), Bp.image(i)) for i in range(len(pairs)))
    log("sweep persistent launch: %.4f ms/iter (graph %.4f), images equal: %s"
        % (ms_pers / args.steps, ms_batched / args.steps, same_p))
    Bp.close()
    S, Q = prob.ny * prob.nx, prob.Q
    res = []
    same = True
    for i, (g, b) in enumerate(pairs):
        x = B.image(i)
        same = same and bool(np.array_equal(x, Bs.image(i)))
        res.append(dict(grouping=g, beta=b, spatial_error=study.spatial_error(x, prob.x_true, S, Q),
                        spectral_error=study.spectral_error(x, prob.x_true, S, Q)))
    best = study.select(res)
    n_total = args.warmup + args.steps
    err = []
    if not args.no_cpu_baseline:
        p = oracle_problem(prob)
        nth = host_threads()
        for i in (0, len(pairs) - 1):
            g, b = pairs[i]
            assert int(B.objective(i)["iter"]) == n_total
            f_or, _, _ = oracle_run(p, n_total, nth, w=w, grouping=g, beta=b)
            e = oracle_error(p, B.image(i), f_or, w=w, grouping=g, beta=b)
            err.append(dict(e, grouping=study.GROUPINGS[g], beta=b, iterations=n_total))
            log("scan %s beta %g after %d iterations vs the FP64 oracle: %s"
                % (study.GROUPINGS[g], b, n_total, json.dumps(e)))
    log("sweep of %d scans: batched %.3f ms/iter, sequential %.3f ms/iter, images equal: %s"
        % (len(pairs), ms_batched / args.steps, ms_seq / args.steps, same))
    for r in res:
        log("  %-18s beta %-6g spatial error %.4f  spectral error %.5f"
            % (study.GROUPINGS[r["grouping"]], r["beta"], r["spatial_error"], r["spectral_error"]))
    alg = len(pairs) * sum(algorithmic_bytes(prob, 4, "tiled").values())
    scan_its = len(pairs) * args.steps
    cpu = None
    if not args.no_cpu_baseline:
        n_cpu = args.cpu_iters
        p = oracle_problem(prob)
        nth = host_threads()
        _, rate1, sec1 = oracle_run(p, n_cpu, 1, beta=betas[0], w=w, grouping=0)
        _, rate, sec = oracle_run(p, n_cpu, nth, beta=betas[0], w=w, grouping=0)
        cpu = {"value": rate, "unit": "scan-iters/s", "cores": nth, "kind": "oracle",
               "sample": "one scan of the sweep, %d iterations (FP64 C oracle, %d OpenMP threads), loop %.1fs"
                         % (n_cpu, nth, sec),
               "single_thread": {"value": rate1, "unit": "scan-iters/s", "cores": 1,
                                 "sample": "the same, one thread, loop %.1fs" % sec1},
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    out = {
        "metric": "beta-sweep scan-iterations/s (both regularisers, one batch)",
        "value": scan_its / (ms_batched * 1e-3),
        "unit": "scan-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_batched / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded phantom scaled to ~26 mean counts, random coded-mask system matrix, Poisson counts)",
        "config": {"workload": "paper-shaped scan 9x41x54, I=8192, 24 nnz/col, weights from 5 mm x 1.5 mm pitch; "
                               "%d betas x 2 regularisers = %d scans, images after %d iterations"
                               % (len(betas), len(pairs), n_total),
                   "global_batch": len(pairs), "parallelism": "single GPU"},
        "sequential": {"value": scan_its / (ms_seq * 1e-3), "ms_per_step": ms_seq / args.steps,
                       "images_bitwise_equal": same},
        "persistent": {"value": scan_its / (ms_pers * 1e-3), "ms_per_step": ms_pers / args.steps,
                       "images_bitwise_equal": same_p, "phase_ms_per_iteration": phases},
        "speedup_vs_sequential": ms_seq / ms_batched,
        "selected": {study.GROUPINGS[g]: {"beta": r["beta"], "spatial_error": r["spatial_error"],
                                          "spectral_error": r["spectral_error"]} for g, r in best.items()},
        "sweep": [[r["grouping"], r["beta"], r["spatial_error"], r["spectral_error"]] for r in res],
        "roofline": {"bound": "hbm", "kernel": "whole batched iteration",
                     "achieved": alg * args.steps / (ms_batched * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg * args.steps / (ms_batched * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None},
        "cpu_baseline": cpu,
        "oracle_error": err or None,
    }
    print(json.dumps(out), flush=True)
    B.close()
    Bs.close()


def adaptive_main(args):
    """Fixed penalty against residual balancing on the paper-scale scan: both
    run until the residual stopping rule holds (checked every 10 iterations)."""
    import torch
    from paper_1601_08201_amd import autotune, datagen, sgtv

    torch.cuda.set_device(0)
    prob = datagen.make_problem("paper", args.seed)
    stream = torch.cuda.current_stream()
    R = sgtv.Reconstructor(stream=stream.cuda_stream)
    tuned = autotune.cached_schedule(prob)
    if tuned:
        R.set_schedule(**tuned)
    R.set_problem(prob)
    opt = dict(check=10, eps_abs=args.eps_abs, eps_rel=args.eps_rel, mu=10.0)
    R.set_init(None)
    R.iterate_adaptive(20, tau=1.0, eps_abs=0.0, eps_rel=0.0, check=10, mu=10.0)   # warm-up, graphs
    res = {}
    for name, tau in (("fixed", 1.0), ("adaptive", 2.0)):
        R.set_penalty(prob.rho)
        R.set_init(None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = R.iterate_adaptive(args.max_iters, tau=tau, **opt)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        rep = R.objective()
        res[name] = {"iterations": out["iterations"], "converged": out["converged"], "seconds": sec,
                     "rho_final": R.penalty(), "objective": rep["total"],
                     "rho_changes": sum(1 for a, b in zip([prob.rho] + [c["rho"] for c in out["checks"]],
                                                         [c["rho"] for c in out["checks"]]) if a != b)}
        log("%-8s %5d iterations, converged %s, %.3f s, rho %g, objective %.6f"
            % (name, out["iterations"], out["converged"], sec, R.penalty(), rep["total"]))
    out = {
        "metric": "time to the residual stopping rule, fixed vs adaptive penalty (paper-scale scan)",
        "value": res["fixed"]["seconds"] / res["adaptive"]["seconds"],
        "unit": "x speedup (fixed / adaptive)",
        "n_gpus": 1, "steps": res["adaptive"]["iterations"], "warmup": 20,
        "ms_per_step": 1e3 * res["adaptive"]["seconds"] / max(res["adaptive"]["iterations"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded phantom, random coded-mask system matrix, Poisson counts)",
        "config": {"workload": "paper-scale scan 128x128x128, I=1048576, 64 nnz/col; stop when r <= eps_pri and "
                               "s <= eps_dual (eps_abs %g, eps_rel %g, checked every 10), mu 10, tau 2"
                               % (args.eps_abs, args.eps_rel),
                   "global_batch": 1, "parallelism": "single GPU"},
        "runs": res,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    R.close()


def warmstart_main(args):
    """Learned warm start against the plain uniform start on held-out phantoms of
    a fixed 64x64x64 scanner: iterations and wall time until the objective is
    within 1e-2, 1e-3, 1e-4 (relative) of the plain converged objective.  Two
    networks: the default one sees the image after 10 plain iterations and
    predicts a per-voxel correction factor; the other sees the normalised
    backprojection and predicts the image."""
    import numpy as np
    import torch
    from paper_1601_08201_amd import autotune, warmstart

    torch.cuda.set_device(0)
    t0 = time.time()
    scanner = warmstart.make_scanner(1)
    shape = (scanner.ny, scanner.nx, scanner.Q)
    tuned = autotune.cached_schedule(datagen_problem_like(scanner))
    recon = warmstart.Reconstruction(scanner, schedule=tuned)
    k_in = args.input_iters
    xin, tgt, _ = warmstart.make_dataset(scanner, range(10000, 10000 + args.train_scans), iters=300,
                                         input_iters=(0, k_in), log=log, recon=recon)
    log("training set: %d scans in %.1fs" % (args.train_scans, time.time() - t0))
    variants = {"learned": (k_in, "ratio"), "learned_backprojection": (0, "direct")}
    nets, train_info = {}, {}
    for name, (k, mode) in variants.items():
        t1 = time.time()
        model, net, hist = warmstart.train(xin[k], tgt, mode=mode, input_iters=k, epochs=args.epochs, log=log)
        nets[name] = (model, net)
        const = warmstart.constant_loss(xin[k], tgt, mode)
        train_info[name] = {"seconds": time.time() - t1, "loss_first_last": [hist[0], hist[-1]],
                            "loss_of_constant_prediction": const,
                            "input": "plain image after %d iterations" % k if k else "normalised backprojection",
                            "output": mode, "start_floor": model.floor}
        log("%s: trained %d epochs in %.1fs, loss %.5f -> %.5f (constant prediction %.5f)"
            % (name, args.epochs, train_info[name]["seconds"], hist[0], hist[-1], const))
    del xin, tgt
    scans = warmstart.draw_scans(scanner, range(20000, 20000 + args.eval_scans))
    R = recon.R
    tols = (1e-2, 1e-3, 1e-4)
    recs = {"plain": [], "restart_without_network": []}
    recs.update({name: [] for name in variants})
    fallbacks = {name: 0 for name in variants}
    for n, (_, y, r) in enumerate(scans):
        recon.load(y, r)
        phi_star, _ = warmstart.converged_objective(R)
        torch.cuda.synchronize()
        # plain: uniform start (its setup is inside the timed region too)
        t = time.perf_counter()
        R.set_init(None)
        setup = time.perf_counter() - t
        it, sec = warmstart.iterations_to_targets(R, phi_star, tols)
        recs["plain"].append((it, [setup + s_ if s_ is not None else None for s_ in sec]))
        # ablation: the same restart (k_in plain iterations, consistent split and
        # dual) from the plain image itself, no network
        t = time.perf_counter()
        spent = warmstart.restart_without_network(R, k_in)
        setup = time.perf_counter() - t
        it, sec = warmstart.iterations_to_targets(R, phi_star, tols)
        recs["restart_without_network"].append(([None if i is None else i + spent for i in it],
                                                [setup + s_ if s_ is not None else None for s_ in sec]))
        for name, (model, net) in nets.items():
            # plain iterations, network, fallback test, restart with consistent split and dual
            t = time.perf_counter()
            spent, fell_back = warmstart.warm_start(R, net, model, shape)
            setup = time.perf_counter() - t
            fallbacks[name] += fell_back
            it, sec = warmstart.iterations_to_targets(R, phi_star, tols)
            recs[name].append(([None if i is None else i + spent for i in it],
                               [setup + s_ if s_ is not None else None for s_ in sec]))
        if (n + 1) % 25 == 0:
            log("eval %d / %d" % (n + 1, args.eval_scans))

    def quart(vals):
        v = np.array([np.nan if x is None else x for x in vals], np.float64)
        return [float(np.nanpercentile(v, 25)), float(np.nanmedian(v)), float(np.nanpercentile(v, 75))]

    summary = {}
    for name, rr in recs.items():
        summary[name] = {}
        for i, tol in enumerate(tols):
            summary[name]["%g" % tol] = {"iterations_q25_q50_q75": quart([x[0][i] for x in rr]),
                                         "ms_q25_q50_q75": [1e3 * v for v in quart([x[1][i] for x in rr])],
                                         "reached": int(sum(x[0][i] is not None for x in rr))}
        log("%-24s median iterations to 1e-2/1e-3/1e-4: %s" % (
            name, [summary[name]["%g" % t]["iterations_q25_q50_q75"][1] for t in tols]))
    med_plain = summary["plain"]["0.0001"]["ms_q25_q50_q75"][1]
    med_learn = summary["learned"]["0.0001"]["ms_q25_q50_q75"][1]
    med_restart = summary["restart_without_network"]["0.0001"]["ms_q25_q50_q75"][1]
    # paired per-scan comparison of the network leg with its ablation at 1e-4
    pairs_it = [(a[0][-1], b[0][-1]) for a, b in zip(recs["learned"], recs["restart_without_network"])
                if a[0][-1] is not None and b[0][-1] is not None]
    network_vs_ablation = {
        "median_iterations_learned": float(np.median([a for a, _ in pairs_it])) if pairs_it else None,
        "median_iterations_restart_without_network": float(np.median([b for _, b in pairs_it])) if pairs_it else None,
        "scans_where_network_fewer_iterations": int(sum(a < b for a, b in pairs_it)),
        "scans_where_network_more_iterations": int(sum(a > b for a, b in pairs_it)),
        "median_ms_ratio_restart_over_learned": med_restart / med_learn,
    }
    log("network vs restart without network at 1e-4: " + json.dumps(network_vs_ablation))
    # error against the FP64 oracle: the plain reconstruction of two held-out
    # scans after 100 iterations
    err = []
    if not args.no_cpu_baseline:
        nth = host_threads()
        for n, (_, y, r) in enumerate(scans[:2]):
            class Scan:
                pass
            sc = Scan()
            sc.__dict__.update(dict(ny=scanner.ny, nx=scanner.nx, Q=scanner.Q, I=scanner.I, J=scanner.J,
                                    rowptr=scanner.rowptr, col=scanner.col, val=scanner.val, y=y, r=r,
                                    beta=scanner.beta, rho=scanner.rho, sweeps=1))
            p = oracle_problem(sc)
            recon.load(y, r)
            f_gpu = recon.plain(100)
            f_or, _, _ = oracle_run(p, 100, nth)
            err.append(dict(oracle_error(p, f_gpu, f_or), scan=20000 + n, iterations=100))
        log("plain reconstructions vs the FP64 oracle: " + json.dumps(err))
    out = {
        "metric": "time to 1e-4 rel obj, learned vs plain (64x64x64 scanner, held-out phantoms)",
        "value": med_plain / med_learn,
        "unit": "x speedup of median wall time (plain / learned)",
        "n_gpus": 1, "steps": args.eval_scans, "warmup": 0,
        "ms_per_step": med_learn,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 ADMM, bf16 MFMA network",
        "data": "synthetic (fixed random coded-mask scanner, seeded phantoms with 6-16 rectangles, Poisson counts)",
        "config": {"workload": "warm start 64x64x64, I=131072, 32 nnz/col; %d training scans (300-iteration targets), "
                               "%d epochs, %d held-out scans; network input: image after %d plain iterations"
                               % (args.train_scans, args.epochs, args.eval_scans, k_in),
                   "global_batch": 32, "parallelism": "single GPU"},
        "by_tolerance": summary,
        "network_vs_restart_without_network": network_vs_ablation,
        "fallbacks": fallbacks,
        "training": train_info,
        "cpu_baseline": None,
        "oracle_error": err or None,
    }
    print(json.dumps(out), flush=True)


def datagen_problem_like(s):
    class P:
        pass
    p = P()
    p.I, p.ny, p.nx, p.Q, p.nnz = s.I, s.ny, s.nx, s.Q, int(s.col.shape[0])
    return p


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--config", default="paper")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--format", default="tiled", choices=["tiled", "sell"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--epilogues", action="store_true",
                    help="the ratio and the image update as row-block epilogues of the two products")
    ap.add_argument("--no-system-files", action="store_true",
                    help="batch workload: skip saving the packed systems and rebuilding the batch from them")
    ap.add_argument("--workload", default="scan", choices=["scan", "batch", "warmstart", "sweep", "adaptive"],
                    help="scan: the paper-scale scan (default); batch: 64 uneven scans; "
                         "warmstart: learned start vs plain start; sweep: beta sweep of both "
                         "regularisers on the paper-shaped scan in one batch; adaptive: fixed vs "
                         "adaptive penalty to the residual stopping rule")
    ap.add_argument("--eps-abs", type=float, default=1e-5)
    ap.add_argument("--eps-rel", type=float, default=1e-3)
    ap.add_argument("--max-iters", type=int, default=4000)
    ap.add_argument("--betas", default="0.01,0.02,0.05,0.1,0.2,0.5,1,2")
    ap.add_argument("--train-scans", type=int, default=2000)
    ap.add_argument("--eval-scans", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--input-iters", type=int, default=10,
                    help="warmstart: plain iterations whose image the network sees")
    ap.add_argument("--batch-scans", type=int, default=64)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the reconstruction of one scan is not sharded across "
              "GPUs in this library (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1601_08201_amd import datagen, sgtv

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "batch":
        if args.steps == 200:
            args.steps = 100
        return batch_main(args)
    if args.workload == "warmstart":
        return warmstart_main(args)
    if args.workload == "adaptive":
        return adaptive_main(args)
    if args.workload == "sweep":
        if args.steps == 200:
            args.steps = 1000
        if args.warmup == 10:
            args.warmup = 50
        if args.cpu_iters == 40:
            args.cpu_iters = 4000
        return sweep_main(args)

    t0 = time.time()
    prob = datagen.make_problem(args.config, args.seed)
    log("generated %s scan: %dx%dx%d, I=%d, nnz=%d, mean(y)=%.3f in %.1fs" % (
        args.config, prob.ny, prob.nx, prob.Q, prob.I, prob.nnz, float(prob.y.mean()), time.time() - t0))

    stream = torch.cuda.current_stream()
    R = sgtv.Reconstructor(device=0, stream=stream.cuda_stream)
    from paper_1601_08201_amd import autotune
    tuned = autotune.cached_schedule(prob, storage=args.storage) if args.format == "tiled" else None
    if tuned:
        R.set_schedule(format=0, **tuned)
        log("tuned schedule from the autotuner cache: " + json.dumps(tuned))
    else:
        R.set_schedule(format=0 if args.format == "tiled" else 1)
    if args.epilogues:
        R.set_epilogues(True)
    t0 = time.time()
    R.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, prob.val, storage=args.storage)
    setup = {"set_system_s": time.time() - t0}
    R.set_data(prob.y, prob.r, prob.beta, prob.rho, prob.sweeps)
    log("system set in %.2fs, data in %.2fs" % (setup["set_system_s"], time.time() - t0 - setup["set_system_s"]))
    if not args.no_system_files:
        setup.update(system_file_times(R, prob, stream))

    R.iterate(args.warmup)
    R.prepare(args.steps)   # graph capture outside the timed region
    torch.cuda.synchronize()
    log("warmup done")

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    R.iterate(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    ms_per_step = ms / max(args.steps, 1)
    rep = R.objective()
    log("timed %d iterations: %.3f ms/iter, objective %.6f" % (args.steps, ms_per_step, rep["total"]))

    # per-kernel durations with HIP events on the library stream (same launches, second pass)
    R.set_profiling(True)
    R.iterate(args.steps)
    times = R.kernel_times()
    R.set_profiling(False)
    vb = {"f32": 4, "bf16": 2, "f16": 2}[args.storage]
    fused = R.fused_update()[0]
    alg = algorithmic_bytes(prob, vb, args.format, fused=fused, epilogues=args.format == "tiled" and R.epilogues())
    if fused:
        times["update_fused"] = times.pop("image_update")
    kern = {}
    for name, (tot, cnt) in times.items():
        if cnt and name in alg:
            avg_ms = tot / cnt
            kern[name] = {"avg_us": avg_ms * 1e3, "launches": cnt, "alg_bytes": alg[name],
                          "gbs": alg[name] / (avg_ms * 1e-3) / 1e9}
    dom = max(kern, key=lambda k: kern[k]["avg_us"])
    achieved = kern[dom]["gbs"]
    log("kernels: " + json.dumps(kern))
    log("schedule: " + json.dumps(R.schedule()) + ", fused image and split update (tile): "
        + json.dumps(R.fused_update()) + ", row-block epilogues: " + json.dumps(R.epilogues()))
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    iter_bytes = sum(alg.values())

    # the same iterations handed over through host memory: counts and
    # background from host arrays, the image back to a host array (set_data
    # drops the captured graphs, so the iterations' graph is captured again
    # inside this region, as it would be for a caller doing the same)
    torch.cuda.synchronize()
    t_h = time.perf_counter()
    R.set_data(prob.y, prob.r, prob.beta, prob.rho, prob.sweeps)
    R.iterate(args.steps)
    R.image()
    host_s = time.perf_counter() - t_h
    host_leg = {"value": args.steps / host_s, "unit": "iters/s", "seconds": host_s,
                "note": "set_data from host arrays (y, r: %.1f MB), %d iterations, the image to a host array "
                        "(%.1f MB), wall clock; the iteration graph is captured again after set_data"
                        % (8e-6 * prob.I, args.steps, 4e-6 * prob.J)}
    log("host-memory handover: %.1f iters/s (%.3f s for %d iterations)" % (host_leg["value"], host_s, args.steps))

    cpu = None
    err = None
    if not args.no_cpu_baseline:
        # the FP64 oracle on the host: one thread, then every thread of this
        # host; its image after cpu_iters iterations is the reference of the
        # GPU's image after as many iterations from the same uniform start
        p = oracle_problem(prob)
        nth = host_threads()
        n1 = max(1, args.cpu_iters // 4)
        log("cpu baseline: %d oracle iterations on 1 thread, %d on %d threads ..." % (n1, args.cpu_iters, nth))
        _, rate1, sec1 = oracle_run(p, n1, 1)
        f_or, rate, secs = oracle_run(p, args.cpu_iters, nth)
        cpu = {"value": rate, "unit": "iters/s", "cores": nth, "kind": "oracle",
               "sample": "%d ADMM iterations of the same %dx%dx%d scan (FP64 C oracle, %d OpenMP threads), "
                         "iteration loop %.1fs" % (args.cpu_iters, prob.ny, prob.nx, prob.Q, nth, secs),
               "single_thread": {"value": rate1, "unit": "iters/s", "cores": 1,
                                 "sample": "%d iterations, loop %.1fs" % (n1, sec1)},
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        log("cpu baseline %.4f iters/s on %d threads, %.4f on one (%s)" % (rate, nth, rate1, cpu["cpu_model"]))
        R.set_init(None)
        R.iterate(args.cpu_iters)
        err = dict(oracle_error(p, R.image(), f_or), iterations=args.cpu_iters)
        log("GPU image after %d iterations vs the FP64 oracle: %s" % (args.cpu_iters, json.dumps(err)))

    out = {
        "metric": "ADMM iters/s + HBM GB/s at 128^2x128; time to 1e-4 rel obj, learned vs plain",
        "value": 1e3 / ms_per_step,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16-values/f32-accum", "f16": "f16-values/f32-accum"}[args.storage],
        "data": "synthetic (seeded phantom, random coded-mask system matrix, Poisson counts)",
        "config": {"workload": "%s scan %dx%dx%d, I=%d, %d nnz/col, nnz=%d, beta=%g, rho=%g, %s values, %s format"
                               % (args.config, prob.ny, prob.nx, prob.Q, prob.I, prob.nnz // prob.J,
                                  prob.nnz, prob.beta, prob.rho, args.storage, args.format),
                   "global_batch": 1, "parallelism": "single GPU"},
        "iteration_alg_GBs": iter_bytes * 1e3 / ms_per_step / 1e9,
        "kernels": kern,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, args.storage, args.format, args.config, R.schedule()),
                     "traffic_unit": "bytes per launch",
                     "traffic_source": "HBM counters (FETCH_SIZE, WRITE_SIZE, calibrated) in " + PRODUCT_PROFILE
                                       + ", valid for the current kernels, builder and schedule"},
        "cpu_baseline": cpu,
        "oracle_error": err,
        "host_memory_handover": host_leg,
        "setup": dict(setup, note="set_system_s: packing on the host and upload; load_system_s: the same "
                                  "packed system read back from a file into a new context"),
    }
    print(json.dumps(out), flush=True)
    R.close()


if __name__ == "__main__":
    main()
