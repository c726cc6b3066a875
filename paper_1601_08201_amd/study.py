"""Regularisation-strength sweeps and the group-versus-standard comparison.

Section IV picks, for each regulariser, the strength beta whose image has the
most accurate spatial distribution, and then compares the two regularisers'
images.  Here the scans are synthetic, so the ground truth is known: every
(beta, grouping) pair of a sweep is one scan of a single batch (all
reconstructions advance together, one batched launch per kernel and
iteration), and each image is scored against the phantom.

Scores (host-side bookkeeping, no reconstruction arithmetic):
- spatial error: relative L2 distance between the spatial maps sum_q f[s, q]
  of the image and of the phantom;
- spectral error: over spatial bins where the phantom is nonzero, the mean of
  1 - cos(angle) between the image's and the phantom's spectra.
"""
from __future__ import annotations

import numpy as np

from . import sgtv

GROUPINGS = {0: "spectral group TV", 1: "standard TV"}


def spatial_map(f, S, Q):
    return np.asarray(f, np.float64).reshape(S, Q).sum(axis=1)


def spatial_error(f, x_true, S, Q):
    m, t = spatial_map(f, S, Q), spatial_map(x_true, S, Q)
    nt = np.linalg.norm(t)
    return float(np.linalg.norm(m - t) / nt) if nt > 0 else float(np.linalg.norm(m))


def spectral_error(f, x_true, S, Q):
    F = np.asarray(f, np.float64).reshape(S, Q)
    T = np.asarray(x_true, np.float64).reshape(S, Q)
    obj = T.sum(axis=1) > 0
    if not obj.any():
        return 0.0
    F, T = F[obj], T[obj]
    nf, nt = np.linalg.norm(F, axis=1), np.linalg.norm(T, axis=1)
    cos = np.where(nf > 0, (F * T).sum(axis=1) / np.maximum(nf * nt, 1e-300), 0.0)
    return float(np.mean(1.0 - cos))


def sweep(prob, betas, iters, groupings=(0, 1), w=None, schedule=None, device=0, stream=None,
          batch=None):
    """Reconstruct `prob` for every (grouping, beta) pair in one batch and
    score each image.  Returns a list of dicts (grouping, beta, image,
    objective, spatial_error, spectral_error) in (grouping, beta) order."""
    B = batch or sgtv.Batch(device, stream)
    pairs = [(g, float(b)) for g in groupings for b in betas]
    for g, b in pairs:
        B.add_scan(prob, schedule=schedule, w=w, grouping=g, beta=b)
    B.iterate(int(iters))
    S, Q = prob.ny * prob.nx, prob.Q
    out = []
    for i, (g, b) in enumerate(pairs):
        x = B.image(i)
        out.append(dict(grouping=g, beta=b, image=x, objective=B.objective(i)["total"],
                        spatial_error=spatial_error(x, prob.x_true, S, Q),
                        spectral_error=spectral_error(x, prob.x_true, S, Q)))
    return out


def select(results):
    """Per grouping, the result with the smallest spatial error (the paper's
    selection rule)."""
    best = {}
    for r in results:
        g = r["grouping"]
        if g not in best or r["spatial_error"] < best[g]["spatial_error"]:
            best[g] = r
    return best
