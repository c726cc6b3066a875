"""Learned warm start for the plain reconstruction.

A fixed scanner (one system matrix) sees many phantoms.  For each training
phantom the plain method (uniform start, 300 ADMM iterations) gives the
target image.  The network sees an early image of the same run, scaled by
its mean: by default the image f_k after k = 10 plain iterations, from which
it predicts a per-voxel correction factor (start image x0 = f_k * factor,
mode "ratio"); with k = 0 it sees the normalised backprojection A^T y / A^T 1
and predicts the image itself (mode "direct").  ADMM then restarts from x0
with the split and dual that make x0 consistent (sgtv_set_init_dual), unless
x0's objective is worse than that of the uniform start, in which case the
plain run continues unchanged (fallback).  (A start can converge faster than
the plain image it came from while its objective is higher: the objective is
only a guard against unusable network output.)

Every reconstruction and network step runs in the library (sgtv / wsnet
entry points); NumPy and torch hold arrays and prepare the training targets.
"""
from __future__ import annotations

import math
import multiprocessing as mp
import time
from dataclasses import dataclass

import numpy as np

from . import datagen, sgtv

_SYSTEM = None     # (rowptr, col, val, ny, nx, Q, I) shared with forked workers


@dataclass
class Scanner:
    ny: int
    nx: int
    Q: int
    I: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    beta: float
    rho: float

    @property
    def J(self):
        return self.ny * self.nx * self.Q


def make_scanner(seed=1, cfg="warmstart"):
    p = datagen.make_problem(cfg, seed)
    return Scanner(p.ny, p.nx, p.Q, p.I, p.rowptr, p.col, p.val, p.beta, p.rho)


def _draw(seed):
    rowptr, col, val, ny, nx, Q, I = _SYSTEM
    x, y, r = datagen.make_scan_for_system(rowptr, col, val, ny, nx, Q, I, seed, rects=(6, 16))
    return x, y, r


def draw_scans(scanner, seeds, workers=16):
    """Phantoms and counts for the fixed scanner (parallel over seeds)."""
    global _SYSTEM
    _SYSTEM = (scanner.rowptr, scanner.col, scanner.val, scanner.ny, scanner.nx, scanner.Q, scanner.I)
    if workers <= 1 or len(seeds) < 4:
        return [_draw(s) for s in seeds]
    with mp.get_context("fork").Pool(min(workers, len(seeds))) as pool:
        return pool.map(_draw, list(seeds), chunksize=8)


class Reconstruction:
    """One reconstructor holding the scanner; data swapped per scan."""

    def __init__(self, scanner, device=0, stream=None, schedule=None):
        self.s = scanner
        self.R = sgtv.Reconstructor(device, stream)
        if schedule:
            self.R.set_schedule(format=0, **schedule)
        self.R.set_system(scanner.I, scanner.ny, scanner.nx, scanner.Q, scanner.rowptr, scanner.col,
                          scanner.val)

    def load(self, y, r):
        self.R.set_data(y, r, self.s.beta, self.s.rho, 1)
        return self

    def plain(self, iters):
        """Uniform start, `iters` iterations; returns the image."""
        self.R.set_init(None)
        self.R.iterate(iters)
        return self.R.image()

    def backprojection(self):
        return self.R.backprojection()


def make_dataset(scanner, seeds, iters=300, input_iters=(10,), log=None, recon=None):
    """Network inputs and targets as float32 [N, ny, nx, Q]: for each k in
    `input_iters` the plain image after k iterations (k = 0: the normalised
    backprojection), and the plain image after `iters` iterations.  Returns
    ({k: inputs}, targets, scans)."""
    scans = draw_scans(scanner, seeds)
    rc = recon or Reconstruction(scanner)
    R = rc.R
    N = len(seeds)
    shp = (N, scanner.ny, scanner.nx, scanner.Q)
    ks = sorted(set(int(k) for k in input_iters))
    if ks and ks[-1] > iters:
        raise ValueError("input iterations exceed the target's")
    xin = {k: np.empty(shp, np.float32) for k in ks}
    tgt = np.empty(shp, np.float32)
    t0 = time.time()
    for n, (_, y, r) in enumerate(scans):
        rc.load(y, r)
        R.set_init(None)
        done = 0
        for k in ks:
            if k == 0:
                xin[0][n] = R.backprojection().reshape(shp[1:])
                continue
            R.iterate(k - done)
            done = k
            xin[k][n] = R.image().reshape(shp[1:])
        R.iterate(iters - done)
        tgt[n] = R.image().reshape(shp[1:])
        if log and (n + 1) % 250 == 0:
            log("dataset: %d / %d scans reconstructed (%.1fs)" % (n + 1, N, time.time() - t0))
    return xin, tgt, scans


RATIO_CLIP = 20.0      # training targets of the correction factor are clipped to [0, RATIO_CLIP]
RATIO_EPS = 1e-3       # ... and computed as target / (input + RATIO_EPS * mean(input))


@dataclass
class Model:
    """Trained parameters, the output scale c_out, the output mode and the
    number of plain iterations whose image the network sees.  The network sees
    each input image divided by its own mean m (counts, backprojection and
    image all scale with the object's intensity, so only the shape is learned);
    mode "ratio": x0 = c_out * net * f_k, mode "direct": x0 = c_out * net * m;
    every voxel of x0 at least floor * c_out * m (wsnet_start)."""
    params: np.ndarray
    c_out: float
    mode: str = "ratio"
    input_iters: int = 10
    layers: int = 6
    floor: float = 0.0


def image_means(x):
    m = x.reshape(x.shape[0], -1).mean(axis=1).astype(np.float32)
    return np.where(m > 0, m, np.float32(1.0))


def training_targets(xin, tgt, mode):
    """Scaled network targets and c_out for the given output mode."""
    m = image_means(xin)[:, None, None, None]
    if mode == "ratio":
        t = np.clip(tgt / (xin + np.float32(RATIO_EPS) * m), 0.0, RATIO_CLIP).astype(np.float32)
    elif mode == "direct":
        t = (tgt / m).astype(np.float32)
    else:
        raise ValueError("mode must be 'ratio' or 'direct'")
    c_out = float(t.mean())
    t /= np.float32(c_out)
    return t, c_out


def train(xin, tgt, mode="ratio", input_iters=10, epochs=40, batch=32, lr=1e-3, lr_min=1e-5, seed=0,
          log=None, device=0, layers=6, floor=None):
    """Adam on the mean squared error of the scaled targets; cosine learning
    rate.  floor (default: 0.2 for mode "direct", 0 for "ratio"): the start
    images' floor as a fraction of the predicted mean level.  A direct
    prediction from the backprojection leaves voxels near zero that the
    multiplicative image update is slow to raise."""
    import torch
    dev = torch.device("cuda", device)
    m = image_means(xin)[:, None, None, None]
    t, c_out = training_targets(xin, tgt, mode)
    X = torch.from_numpy(xin / m).to(dev)
    T = torch.from_numpy(t).to(dev)
    del t
    N = X.shape[0]
    H, W, C = X.shape[1:]
    net = sgtv.WarmStartNet(device=device, stream=torch.cuda.current_stream(dev).cuda_stream,
                            layers=layers, height=H, width=W, channels=C, max_batch=batch)
    net.set_params(sgtv.init_params(layers, C, seed))
    rng = np.random.default_rng(seed)
    steps = epochs * (N // batch)
    step = 0
    history = []
    t0 = time.time()
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(N)).to(dev)
        for b in range(N // batch):
            idx = order[b * batch:(b + 1) * batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / max(steps, 1)))
            net.train_step(xb, tb, lr=cur)      # no wait for the device: the losses add up there
            step += 1
        tot, _ = net.loss_sum(reset=True)
        history.append(tot / max(N // batch, 1))
        if log and (ep + 1) % 5 == 0:
            log("train: epoch %d / %d, loss %.5f (%.1fs)" % (ep + 1, epochs, history[-1], time.time() - t0))
    if floor is None:
        floor = 0.2 if mode == "direct" else 0.0
    model = Model(net.params(), c_out, mode, int(input_iters), int(layers), float(floor))
    return model, net, history


def predict(net, model, f):
    """Start images for a batch of network inputs f (float32 NHWC, host array
    or device tensor): the plain images after model.input_iters iterations, or
    normalised backprojections."""
    return net.start(f, model.mode, model.c_out, floor=model.floor)


def warm_start(R, net, model, shape):
    """Initialise reconstructor R (data set) from the network: plain start,
    model.input_iters plain iterations (none: the backprojection is the input),
    then the network's start image with a consistent split and dual, unless
    its objective is worse than the uniform start's (fallback: the plain run
    continues).  shape = (ny, nx, Q).  Returns (plain iterations spent,
    fell back)."""
    import torch
    k = int(model.input_iters)
    buf = torch.empty(int(np.prod(shape)), dtype=torch.float32, device="cuda")
    R.set_init(None)
    phi_ref = R.objective()["total"]
    if k > 0:
        R.iterate(k)
        saved = R.state()
        R.image(out=buf)
    else:
        R.backprojection(out=buf)
    x0 = predict(net, model, buf.view(1, *shape))
    R.set_init_dual(x0.view(-1))
    phi = R.objective()["total"]
    if math.isfinite(phi) and phi <= phi_ref:
        return k, False
    if k > 0:
        R.set_state(*saved)
    else:
        R.set_init(None)
    return k, True


def restart_without_network(R, k):
    """The ablation of the learned start: from the uniform start, k plain
    iterations, then a restart from that image with the consistent split and
    dual (sgtv_set_init_dual), as warm_start does with the network's image.
    Returns the plain iterations spent."""
    R.set_init(None)
    R.iterate(k)
    R.set_init_dual(R.image())
    return k


def constant_loss(xin, tgt, mode):
    """Mean squared error of the constant prediction 1 against the scaled
    training targets (the loss of a network that learned nothing but the mean)."""
    t, _ = training_targets(xin, tgt, mode)
    return float(np.mean((t.astype(np.float64) - 1.0) ** 2))


def iterations_to_target(R, phi_star, tol=1e-4, check=5, cap=3000):
    """Iterate (already initialised) until objective <= phi_star (1 + tol),
    checking every `check` iterations; returns (iterations, reached)."""
    k = 0
    while k < cap:
        R.iterate(check)
        k += check
        if R.objective()["total"] <= phi_star * (1 + tol):
            return k, True
    return k, False


def iterations_to_targets(R, phi_star, tols=(1e-2, 1e-3, 1e-4), check=5, cap=3000):
    """Like iterations_to_target for several tolerances in one run: returns the
    first checked iteration count at which each one is met (None if not met)
    and the wall time (seconds, host clock around the launches) at each."""
    out = [None] * len(tols)
    secs = [None] * len(tols)
    t0 = time.perf_counter()
    k = 0
    phi = R.objective()["total"]
    for i, t in enumerate(tols):
        if phi <= phi_star * (1 + t):
            out[i], secs[i] = 0, time.perf_counter() - t0
    while k < cap and out[-1] is None:
        R.iterate(check)
        k += check
        phi = R.objective()["total"]
        for i, t in enumerate(tols):
            if out[i] is None and phi <= phi_star * (1 + t):
                out[i], secs[i] = k, time.perf_counter() - t0
    return out, secs


def converged_objective(R, chunk=50, cap=3000, rel=1e-10):
    """min objective of a plain run stopped when it changes by < rel over `chunk` iterations."""
    R.set_init(None)
    best = R.objective()["total"]
    prev = best
    k = 0
    while k < cap:
        R.iterate(chunk)
        k += chunk
        cur = R.objective()["total"]
        best = min(best, cur)
        if abs(prev - cur) <= rel * abs(cur):
            break
        prev = cur
    return best, k
