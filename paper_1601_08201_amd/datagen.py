"""Seeded synthetic inputs shaped like the paper's coherent-scatter scans.

This module only draws inputs: a hyperspectral phantom, a random nonnegative
coded-mask system matrix, and Poisson counts drawn from the measurement model
of Eq. 1 (Section II).  It holds none of the reconstruction's arithmetic and
is shared by the FP64 oracle, the GPU tests and the benchmark.

Recipe (draw order is part of the definition, PCG64(seed)):

1. Phantom: for each of R rectangles in turn draw height h ~ U{2..ceil(ny/2)},
   width w ~ U{2..ceil(nx/2)}, a top-left corner uniform over the positions
   where it fits, then mu ~ U[0, Q-1], sigma ~ U[1, 4], amp ~ U[1, 10].  The
   rectangle's hyper-voxels get the Gaussian momentum-transfer profile
   amp*exp(-(q-mu)^2/(2 sigma^2)); later rectangles overwrite earlier ones;
   the background is zero.
2. System matrix: for every column (hyper-voxel) draw `nnz_per_col` distinct
   rows uniformly (duplicates redrawn), values U(0,1) times a Bernoulli(0.5)
   coded-mask factor; a column whose values are all zero is redrawn.  Zero
   values stay structural, so nnz = nnz_per_col * J exactly.
3. Data: y ~ Poisson(A x_true + b) with b = float32(0.1), stored as float32.

Voxel order is j = (iy*nx + ix)*Q + q (spectral bin fastest).  Arrays are
float32 / int32 (row pointer int64), the exact values both sides consume.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

BACKGROUND = np.float32(0.1)

# Workloads: the small parity case and the paper-scale single scan, the
# reduced-precision study on the same scan, the batched-scan mix and the
# learned warm-start scanner.
CONFIGS = {
    "small": dict(ny=16, nx=16, Q=32, I=4096, nnz_per_col=16, rects=4,
                  beta=0.1, rho=1.0, iters=50, sweeps=1),
    "paper": dict(ny=128, nx=128, Q=128, I=1048576, nnz_per_col=64, rects=12,
                  beta=0.05, rho=1.0, iters=200, sweeps=1),
    "warmstart": dict(ny=64, nx=64, Q=64, I=131072, nnz_per_col=32, rects=(6, 16),
                      beta=0.1, rho=1.0, iters=300, sweeps=1),
    # the shape of the paper's experiment (Section IV): a 205 mm x 13.5 mm region
    # sampled every 5 mm along z (x here) and 1.5 mm along y, 54 momentum-transfer
    # bins, a 128-pixel x 64-channel detector, about 26 detected photons per
    # measurement; difference weights follow the voxel pitches
    "teflon": dict(ny=9, nx=41, Q=54, I=8192, nnz_per_col=24, rects=2, beta=0.5, rho=1.0,
                   iters=300, sweeps=1, mean_count=26.0, pitch=(5.0, 1.5)),
}


def direction_weights(pitch_x, pitch_y):
    """Weights of the +x, -x, +y, -y differences for voxel pitches (any unit):
    each difference is divided by its pitch, scaled so the finer direction has
    weight one."""
    fine = min(pitch_x, pitch_y)
    return np.array([fine / pitch_x, fine / pitch_x, fine / pitch_y, fine / pitch_y], np.float32)


@dataclass
class Problem:
    ny: int
    nx: int
    Q: int
    I: int
    rowptr: np.ndarray          # int64 [I+1]
    col: np.ndarray             # int32 [nnz]
    val: np.ndarray             # float32 [nnz]
    y: np.ndarray               # float32 [I]
    r: np.ndarray               # float32 [I]
    x_true: np.ndarray          # float32 [J]
    beta: float = 0.1
    rho: float = 1.0
    iters: int = 50
    sweeps: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def J(self) -> int:
        return self.ny * self.nx * self.Q

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.I, self.J))


def make_phantom(rng: np.random.Generator, ny: int, nx: int, Q: int, n_rect: int) -> np.ndarray:
    """Piecewise-constant-in-space phantom with Gaussian spectra, float32 [J]."""
    x = np.zeros((ny, nx, Q), dtype=np.float64)
    q = np.arange(Q, dtype=np.float64)
    for _ in range(n_rect):
        h = int(rng.integers(min(2, ny), max(min(2, ny), math.ceil(ny / 2)) + 1))
        w = int(rng.integers(min(2, nx), max(min(2, nx), math.ceil(nx / 2)) + 1))
        h, w = min(h, ny), min(w, nx)
        y0 = int(rng.integers(0, ny - h + 1))
        x0 = int(rng.integers(0, nx - w + 1))
        mu = rng.uniform(0.0, max(Q - 1, 0))
        sigma = rng.uniform(1.0, 4.0)
        amp = rng.uniform(1.0, 10.0)
        x[y0:y0 + h, x0:x0 + w, :] = amp * np.exp(-(q - mu) ** 2 / (2.0 * sigma * sigma))
    return x.reshape(-1).astype(np.float32)


def make_system(rng: np.random.Generator, I: int, J: int, nnz_per_col: int):
    """Random coded-mask system matrix, returned as sorted CSR (rowptr int64, col int32, val f32)."""
    k = int(nnz_per_col)
    if k > I:
        raise ValueError("nnz_per_col exceeds the number of measurements")
    if k == 0 or J == 0:
        return np.zeros(I + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32)
    if 4 * k > I:
        rows = np.stack([rng.choice(I, size=k, replace=False) for _ in range(J)])
        rows.sort(axis=1)
    else:
        rows = rng.integers(0, I, (J, k), dtype=np.int64)
        rows.sort(axis=1)
        while True:
            bad = np.flatnonzero((rows[:, 1:] == rows[:, :-1]).any(axis=1))
            if bad.size == 0:
                break
            redraw = rng.integers(0, I, (bad.size, k), dtype=np.int64)
            redraw.sort(axis=1)
            rows[bad] = redraw
    vals = rng.random((J, k)) * (rng.random((J, k)) < 0.5)
    while True:
        bad = np.flatnonzero(~(vals > 0).any(axis=1))
        if bad.size == 0:
            break
        vals[bad] = rng.random((bad.size, k)) * (rng.random((bad.size, k)) < 0.5)
    vals = vals.astype(np.float32)
    csc = sp.csc_matrix((vals.ravel(), rows.ravel().astype(np.int32),
                         np.arange(0, J * k + 1, k, dtype=np.int64)), shape=(I, J))
    csr = csc.tocsr()
    if not csr.has_sorted_indices:
        csr.sort_indices()
    return csr.indptr.astype(np.int64), csr.indices.astype(np.int32), csr.data.astype(np.float32)


def draw_counts(rng: np.random.Generator, rowptr, col, val, x_true, I: int, b=BACKGROUND):
    """y ~ Poisson(A x_true + b) (Eq. 1), float32; r = b everywhere."""
    J = x_true.shape[0]
    A = sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(I, J))
    mean = A @ x_true.astype(np.float64) + float(b)
    y = rng.poisson(mean).astype(np.float32)
    r = np.full(I, b, dtype=np.float32)
    return y, r


def make_problem(cfg, seed: int) -> Problem:
    """One scan: phantom, then system matrix, then counts, all from PCG64(seed)."""
    c = dict(CONFIGS[cfg]) if isinstance(cfg, str) else dict(cfg)
    rng = np.random.Generator(np.random.PCG64(seed))
    ny, nx, Q, I = int(c["ny"]), int(c["nx"]), int(c["Q"]), int(c["I"])
    rects = c.get("rects", 4)
    if isinstance(rects, tuple):
        rects = int(rng.integers(rects[0], rects[1] + 1))
    x_true = make_phantom(rng, ny, nx, Q, int(rects))
    rowptr, col, val = make_system(rng, I, ny * nx * Q, int(c["nnz_per_col"]))
    if c.get("mean_count"):
        # scale the object so that the expected counts average mean_count (no draws)
        A = sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(I, ny * nx * Q))
        mean = float((A @ x_true.astype(np.float64)).mean())
        if mean > 0:
            x_true = (x_true.astype(np.float64) * ((c["mean_count"] - float(BACKGROUND)) / mean)).astype(np.float32)
    y, r = draw_counts(rng, rowptr, col, val, x_true, I)
    return Problem(ny=ny, nx=nx, Q=Q, I=I, rowptr=rowptr, col=col, val=val, y=y, r=r,
                   x_true=x_true, beta=float(c.get("beta", 0.1)), rho=float(c.get("rho", 1.0)),
                   iters=int(c.get("iters", 50)), sweeps=int(c.get("sweeps", 1)),
                   meta=dict(cfg=cfg if isinstance(cfg, str) else "custom", seed=seed,
                             rects=int(rects),
                             weights=(direction_weights(*c["pitch"]) if c.get("pitch") else None)))


def make_scan_for_system(rowptr, col, val, ny: int, nx: int, Q: int, I: int, seed: int,
                         rects=(6, 16)):
    """A new phantom and its counts for a fixed scanner (system matrix held fixed).

    Draw order: number of rectangles, phantom, counts.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(rects[0], rects[1] + 1)) if isinstance(rects, tuple) else int(rects)
    x_true = make_phantom(rng, ny, nx, Q, n)
    y, r = draw_counts(rng, rowptr, col, val, x_true, I)
    return x_true, y, r


def batch_shapes(n_scans: int, seed: int):
    """Grid shapes of a batch of uneven scans: side in {32,48,64,96,128}, Q in {64,96,128}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.choice(np.array([32, 48, 64, 96, 128]), size=n_scans)
    qs = rng.choice(np.array([64, 96, 128]), size=n_scans)
    return [(int(s), int(s), int(q)) for s, q in zip(sides, qs)]


def make_batch_scan(ny: int, nx: int, Q: int, seed: int, nnz_per_col: int = 32,
                    rects: int = 4, beta: float = 0.1, rho: float = 1.0, iters: int = 100):
    """One scan of a batch: I = J/2 measurements, otherwise the single-scan recipe."""
    J = ny * nx * Q
    return make_problem(dict(ny=ny, nx=nx, Q=Q, I=max(J // 2, 1), nnz_per_col=nnz_per_col,
                             rects=rects, beta=beta, rho=rho, iters=iters, sweeps=1), seed)
