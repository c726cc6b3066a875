"""Learned warm start for the plain reconstruction.

A fixed scanner (one system matrix) sees many phantoms.  For each training
phantom the plain method (uniform start, 300 ADMM iterations) gives the
target image; the network learns to map the normalised backprojection
A^T y / A^T 1 to that image.  At inference the network's output starts ADMM
(d = c = 0) unless its objective is worse than the uniform start's, in which
case the uniform start is used (fallback).

Every reconstruction and network step runs in the library (sgtv / wsnet
entry points); NumPy and torch only hold arrays.
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


def make_dataset(scanner, seeds, iters=300, log=None, recon=None):
    """(inputs, targets) as float32 [N, ny, nx, Q]: normalised backprojections
    and plain reconstructions after `iters` iterations."""
    scans = draw_scans(scanner, seeds)
    rc = recon or Reconstruction(scanner)
    N = len(seeds)
    shp = (N, scanner.ny, scanner.nx, scanner.Q)
    xin = np.empty(shp, np.float32)
    tgt = np.empty(shp, np.float32)
    t0 = time.time()
    for k, (_, y, r) in enumerate(scans):
        rc.load(y, r)
        xin[k] = rc.backprojection().reshape(shp[1:])
        tgt[k] = rc.plain(iters).reshape(shp[1:])
        if log and (k + 1) % 250 == 0:
            log("dataset: %d / %d scans reconstructed (%.1fs)" % (k + 1, N, time.time() - t0))
    return xin, tgt, scans


@dataclass
class Model:
    """Trained parameters and the output scale: the network sees each input
    image divided by its own mean m and its output is multiplied by c_out * m
    (the counts, the backprojection and the image all scale with the object's
    intensity, so the network only has to learn the shape)."""
    params: np.ndarray
    c_out: float
    layers: int = 6


def image_means(x):
    m = x.reshape(x.shape[0], -1).mean(axis=1).astype(np.float32)
    return np.where(m > 0, m, np.float32(1.0))


def train(xin, tgt, epochs=40, batch=32, lr=1e-3, lr_min=1e-5, seed=0, log=None, device=0):
    """Adam on the mean squared error of the scaled images; cosine learning rate."""
    import torch
    dev = torch.device("cuda", device)
    m = image_means(xin)[:, None, None, None]
    c_out = float((tgt / m).mean())
    X = torch.from_numpy(xin / m).to(dev)
    T = torch.from_numpy(tgt / (m * np.float32(c_out))).to(dev)
    N = X.shape[0]
    H, W, C = X.shape[1:]
    net = sgtv.WarmStartNet(device=device, stream=torch.cuda.current_stream(dev).cuda_stream,
                            layers=6, height=H, width=W, channels=C, max_batch=batch)
    net.set_params(sgtv.init_params(6, C, seed))
    rng = np.random.default_rng(seed)
    steps = epochs * (N // batch)
    step = 0
    history = []
    t0 = time.time()
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(N)).to(dev)
        tot = 0.0
        for b in range(N // batch):
            idx = order[b * batch:(b + 1) * batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            loss = net.backward(xb, tb)
            cur = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / max(steps, 1)))
            net.adam_step(lr=cur)
            tot += loss
            step += 1
        history.append(tot / max(N // batch, 1))
        if log and (ep + 1) % 5 == 0:
            log("train: epoch %d / %d, loss %.5f (%.1fs)" % (ep + 1, epochs, history[-1], time.time() - t0))
    model = Model(net.params(), c_out)
    return model, net, history


def predict(net, model, xin):
    """Start images for a batch of normalised backprojections (float32 NHWC)."""
    m = image_means(xin)[:, None, None, None]
    out = net.forward(np.ascontiguousarray(xin / m, np.float32))
    return out * (m * np.float32(model.c_out))


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
