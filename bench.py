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


def algorithmic_bytes(prob, value_bytes, fmt):
    """Bytes each kernel must move per launch: every array it needs, touched once.

    Tiled format: forward = A (values + indices), x, p out; ratio = p, y, r,
    ratio out; back = A, ratio, e out; image update = e, g, v, a, sens, H,
    g out; split = f, v, a in and v, a out.  The sliced-ELL kernels fuse the
    ratio into the forward pass and the image update into the back pass.
    """
    I, J, nnz = prob.I, prob.J, prob.nnz
    S = prob.ny * prob.nx
    a = nnz * (value_bytes + 4)
    out = {"split_update": 4 * J + 16 * J + 4 * S + 16 * J + 4 * S}
    if fmt == "tiled":
        out["forward"] = a + 4 * J + 4 * I
        out["ratio"] = 16 * I
        out["back"] = a + 4 * I + 4 * J
        out["image_update"] = 4 * J + 4 * J + 16 * J + 4 * S + 4 * J + 4 * J + 4 * J
    else:
        out["forward"] = a + 4 * (I + 1) + 4 * J + 12 * I
        out["back"] = a + 4 * (J + 1) + 4 * I + 32 * J + 4 * S
    return out


def measured_traffic(kernel, storage, fmt, config):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when there is none for this workload or the kernel sources changed since."""
    import hashlib
    import re
    if storage != "f32" or fmt != "tiled" or config != "paper" or kernel not in ("forward", "back"):
        return None
    path = os.path.join(ROOT, "profiles", "tiled_product_fp32_paper_scan.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    h = hashlib.sha256()
    for f in ("sgtv_tiled.hip", "sgtv_device.h", "sgtv_kernels.h"):
        with open(os.path.join(ROOT, "paper_1601_08201_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec.get("kernel_source_sha256"):
        return None
    return rec["traffic_bytes_per_launch"].get(kernel)


def cpu_baseline(prob, iters):
    import numpy as np
    import oracle
    rp = prob.rowptr
    col = prob.col
    val = prob.val.astype(np.float64)
    y = prob.y.astype(np.float64)
    r = prob.r.astype(np.float64)

    class P:
        pass
    p = P()
    p.__dict__.update(dict(ny=prob.ny, nx=prob.nx, Q=prob.Q, I=prob.I, rowptr=rp, col=col, val=val,
                           y=y, r=r, beta=prob.beta, rho=prob.rho, sweeps=prob.sweeps))
    f0 = np.full(prob.J, oracle.plain_init(p), np.float64)
    t0 = time.perf_counter()
    oracle.admm(p, iters, f0=f0, report=False)
    dt = time.perf_counter() - t0
    return iters / dt, dt


def _gen_batch_scan(args):
    from paper_1601_08201_amd import datagen
    ny, nx, Q, seed = args
    return datagen.make_batch_scan(ny, nx, Q, seed=seed)


def batch_main(args):
    """Batch of uneven scans: batched launches (one graph per call) against the
    same scans iterated one after another."""
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
    tuned = 0
    scheds = []
    for p in probs:
        sch = autotune.cached_schedule(p)
        tuned += sch is not None
        scheds.append(sch)
    with cf.ThreadPoolExecutor(8) as ex:
        list(ex.map(lambda ps: B.add_scan(ps[0], ps[1]), zip(probs, scheds)))
    log("batch built in %.1fs (%d scans with tuned schedules)" % (time.time() - t0, tuned))
    B.iterate(args.warmup)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    a, b = ev(), ev()
    a.record(stream)
    B.iterate(args.steps)
    b.record(stream)
    torch.cuda.synchronize()
    ms_batched = a.elapsed_time(b)
    B.iterate_sequential(args.warmup)
    torch.cuda.synchronize()
    a.record(stream)
    B.iterate_sequential(args.steps)
    b.record(stream)
    torch.cuda.synchronize()
    ms_seq = a.elapsed_time(b)
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
        "speedup_vs_sequential": ms_seq / ms_batched,
        "batch_iteration_alg_GBs": alg * args.steps / (ms_batched * 1e-3) / 1e9,
        "roofline": {"bound": "hbm", "kernel": "whole batched iteration",
                     "achieved": alg * args.steps / (ms_batched * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg * args.steps / (ms_batched * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    B.close()


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
    ap.add_argument("--workload", default="scan", choices=["scan", "batch"],
                    help="scan: the paper-scale scan (default); batch: 64 uneven scans")
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

    t0 = time.time()
    prob = datagen.make_problem(args.config, args.seed)
    log("generated %s scan: %dx%dx%d, I=%d, nnz=%d, mean(y)=%.3f in %.1fs" % (
        args.config, prob.ny, prob.nx, prob.Q, prob.I, prob.nnz, float(prob.y.mean()), time.time() - t0))

    stream = torch.cuda.current_stream()
    R = sgtv.Reconstructor(device=0, stream=stream.cuda_stream)
    from paper_1601_08201_amd import autotune
    tuned = autotune.cached_schedule(prob) if args.format == "tiled" else None
    if tuned:
        R.set_schedule(format=0, **tuned)
        log("tuned schedule from the autotuner cache: " + json.dumps(tuned))
    else:
        R.set_schedule(format=0 if args.format == "tiled" else 1)
    t0 = time.time()
    R.set_problem(prob, storage=args.storage)
    log("system and data set in %.1fs" % (time.time() - t0))

    R.iterate(args.warmup)
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
    alg = algorithmic_bytes(prob, vb, args.format)
    kern = {}
    for name, (tot, cnt) in times.items():
        if cnt and name in alg:
            avg_ms = tot / cnt
            kern[name] = {"avg_us": avg_ms * 1e3, "launches": cnt, "alg_bytes": alg[name],
                          "gbs": alg[name] / (avg_ms * 1e-3) / 1e9}
    dom = max(kern, key=lambda k: kern[k]["avg_us"])
    achieved = kern[dom]["gbs"]
    log("kernels: " + json.dumps(kern))
    log("schedule: " + json.dumps(R.schedule()))
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    iter_bytes = sum(alg.values())

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: %d oracle iterations on the host ..." % args.cpu_iters)
        rate, secs = cpu_baseline(prob, args.cpu_iters)
        cpu = {"value": rate, "unit": "iters/s", "cores": 1, "kind": "oracle",
               "sample": "%d ADMM iterations of the same %dx%dx%d scan (FP64, serial C), %.1fs"
                         % (args.cpu_iters, prob.ny, prob.nx, prob.Q, secs)}
        log("cpu baseline %.4f iters/s" % rate)

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
                     "traffic": measured_traffic(dom, args.storage, args.format, args.config),
                     "traffic_unit": "bytes per launch"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    R.close()


if __name__ == "__main__":
    main()
