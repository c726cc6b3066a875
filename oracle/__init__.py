"""FP64 CPU oracle (ctypes wrapper around the plain C in this folder).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and by
the benchmark's CPU-baseline leg.  The GPU library never imports, links or
calls anything here, and this folder imports nothing from the GPU package.

Every function takes float32/float64 NumPy arrays, widens them exactly to
float64 and runs the plain C routines of sgtv_oracle.c (and wsnet_oracle.c
for the warm-start network).  Layout conventions are those of the C file:
voxel j = (iy*nx + ix)*Q + q, stacked differences [s][p][q] with
p = +x, -x, +y, -y.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_SOURCES = ["sgtv_oracle.c", "wsnet_oracle.c"]
_lib = None

NDIR = 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math, no contraction); OpenMP
    shares the loops over independent outputs among threads."""
    os.makedirs(_BUILD, exist_ok=True)
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-Wall", "-o", tmp] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = ctypes.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double


def _declare(lib):
    sig = {
        "or_forward": (None, [_I64, _P, _P, _P, _P, _P, _P]),
        "or_back": (None, [_I64, _I64, _P, _P, _P, _P, _P]),
        "or_diff": (None, [_I, _I, _I, _P, _P, _P]),
        "or_diff_adj": (None, [_I, _I, _I, _P, _P, _P]),
        "or_curv": (None, [_I, _I, _I, _P, _D, _P]),
        "or_root": (_D, [_D, _D, _D]),
        "or_shrink": (None, [_I, _I, _I, _I, _D, _P, _P]),
        "or_group_norm_sum": (_D, [_I, _I, _I, _I, _P]),
        "or_data_term": (_D, [_I64, _P, _P]),
        "or_admm_flat": (_I, [_I64, _I, _I, _I, _P, _P, _P, _P, _P, _P, _D, _D, _I, _I, _I,
                              _P, _P, _P, _P]),
        "or_admm_adaptive_flat": (_I, [_I64, _I, _I, _I, _P, _P, _P, _P, _P, _P, _D, _D, _I, _I, _I, _I,
                                       _D, _D, _D, _D, _P, _P, _P, _P, _I, _P, _P, _P]),
        "or_objective_flat": (None, [_I64, _I, _I, _I, _P, _P, _P, _P, _P, _P, _D, _I, _P, _P]),
        "or_image_sweep_flat": (None, [_I64, _I, _I, _I, _P, _P, _P, _P, _P, _P, _D, _P, _P]),
        "or_plain_init_flat": (_D, [_I64, _I, _I, _I, _P, _P, _P, _P]),
        "or_quantise": (None, [_I64, _I64, _P, _P, _I, _P, _P, _P]),
        "wn_conv_fwd": (None, [_I, _I, _I, _I, _I, _P, _P, _P, _P]),
        "wn_conv_bwd_data": (None, [_I, _I, _I, _I, _I, _P, _P, _P]),
        "wn_conv_bwd_weight": (None, [_I, _I, _I, _I, _I, _P, _P, _P, _P]),
        "wn_forward": (None, [_I, _I, _I, _I, _I, _P, _P, _P, _P, _P]),
        "wn_loss_grad": (_D, [_I, _I, _I, _I, _I, _P, _P, _P, _P]),
        "wn_adam": (None, [_I64, _P, _P, _P, _P, _I64, _D, _D, _D, _D]),
        "or_set_threads": (None, [_I]),
        "or_max_threads": (_I, []),
        "or_last_loop_seconds": (_D, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


def set_threads(n):
    """Threads of the loops over independent outputs (results do not depend on it)."""
    _load().or_set_threads(int(n))


def max_threads():
    return int(_load().or_max_threads())


def last_loop_seconds():
    """Wall time of the iteration loop of the last admm() call (set-up excluded)."""
    return float(_load().or_last_loop_seconds())


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _csr(rowptr, col, val):
    return (np.ascontiguousarray(rowptr, dtype=np.int64),
            np.ascontiguousarray(col, dtype=np.int32), _f64(val))


def _weights(w, ny, nx, Q):
    """None -> all ones; 4 values -> one per direction; else the full [s][p][q] array."""
    if w is None:
        return None
    w = np.asarray(w, dtype=np.float64).ravel()
    if w.size == NDIR:
        return np.ascontiguousarray(np.broadcast_to(w[None, :, None], (ny * nx, NDIR, Q)).ravel())
    if w.size != ny * nx * Q * NDIR:
        raise ValueError("weights must have 4 or 4*J entries")
    return np.ascontiguousarray(w)


def forward(rowptr, col, val, f, r=None):
    """p = A f + r (Eq. 1 mean)."""
    lib = _load()
    rp, c, v = _csr(rowptr, col, val)
    I = rp.shape[0] - 1
    f = _f64(f)
    rr = _f64(r) if r is not None else None
    p = np.empty(I, np.float64)
    lib.or_forward(I, _ptr(rp), _ptr(c), _ptr(v), _ptr(f), _ptr(rr), _ptr(p))
    return p


def back(rowptr, col, val, t, J):
    """e = A^T t."""
    lib = _load()
    rp, c, v = _csr(rowptr, col, val)
    I = rp.shape[0] - 1
    t = _f64(t)
    e = np.empty(J, np.float64)
    lib.or_back(I, J, _ptr(rp), _ptr(c), _ptr(v), _ptr(t), _ptr(e))
    return e


def diff(ny, nx, Q, f, w=None):
    """Stacked weighted differences D f, shape [S, 4, Q] flattened."""
    lib = _load()
    f = _f64(f)
    ww = _weights(w, ny, nx, Q)
    g = np.empty(ny * nx * Q * NDIR, np.float64)
    lib.or_diff(ny, nx, Q, _ptr(ww), _ptr(f), _ptr(g))
    return g


def diff_adj(ny, nx, Q, t, w=None):
    """D^T t for t laid out [S, 4, Q]."""
    lib = _load()
    t = _f64(t)
    ww = _weights(w, ny, nx, Q)
    out = np.empty(ny * nx * Q, np.float64)
    lib.or_diff_adj(ny, nx, Q, _ptr(ww), _ptr(t), _ptr(out))
    return out


def curvature(ny, nx, Q, lam, w=None):
    """De Pierro curvature H = lam |D|^T |D| 1."""
    lib = _load()
    ww = _weights(w, ny, nx, Q)
    H = np.empty(ny * nx * Q, np.float64)
    lib.or_curv(ny, nx, Q, _ptr(ww), float(lam), _ptr(H))
    return H


def root(H, B, C):
    """Nonnegative root of H t^2 + B t - C = 0 (scalar)."""
    return _load().or_root(float(H), float(B), float(C))


def shrink(ny, nx, Q, thr, v, grouping=0):
    """Block soft-threshold of v ([S,4,Q]) with threshold thr = beta/lam."""
    lib = _load()
    v = _f64(v)
    d = np.empty_like(v)
    lib.or_shrink(ny, nx, Q, int(grouping), float(thr), _ptr(v), _ptr(d))
    return d


def group_norm_sum(ny, nx, Q, g, grouping=0):
    return _load().or_group_norm_sum(ny, nx, Q, int(grouping), _ptr(_f64(g)))


def data_term(p, y):
    p, y = _f64(p), _f64(y)
    return _load().or_data_term(p.shape[0], _ptr(p), _ptr(y))


def objective(prob, f, w=None, grouping=0, beta=None):
    """(total, data, tv) of f for a datagen.Problem-like object."""
    lib = _load()
    rp, c, v = _csr(prob.rowptr, prob.col, prob.val)
    y, r, f = _f64(prob.y), _f64(prob.r), _f64(f)
    ww = _weights(w, prob.ny, prob.nx, prob.Q)
    out = np.empty(3, np.float64)
    b = prob.beta if beta is None else beta
    lib.or_objective_flat(prob.I, prob.ny, prob.nx, prob.Q, _ptr(rp), _ptr(c), _ptr(v),
                          _ptr(y), _ptr(r), _ptr(ww), float(b), int(grouping), _ptr(f), _ptr(out))
    return out


def image_sweep(prob, g, z, lam=None, w=None):
    """One optimisation-transfer pass of the image update from g with z = d - c."""
    lib = _load()
    rp, c, v = _csr(prob.rowptr, prob.col, prob.val)
    y, r = _f64(prob.y), _f64(prob.r)
    ww = _weights(w, prob.ny, prob.nx, prob.Q)
    g = _f64(g).copy()
    z = _f64(z)
    lib.or_image_sweep_flat(prob.I, prob.ny, prob.nx, prob.Q, _ptr(rp), _ptr(c), _ptr(v),
                            _ptr(y), _ptr(r), _ptr(ww), float(prob.rho if lam is None else lam),
                            _ptr(z), _ptr(g))
    return g


def plain_init(prob):
    """kappa = sum(y) / sum(A^T 1): the uniform start matched to the total counts."""
    lib = _load()
    rp, c, v = _csr(prob.rowptr, prob.col, prob.val)
    y = _f64(prob.y)
    return lib.or_plain_init_flat(prob.I, prob.ny, prob.nx, prob.Q, _ptr(rp), _ptr(c), _ptr(v),
                                  _ptr(y))


def quantise(col, val, J, kind):
    """Per-column scaled 16-bit codes of the matrix values (kind 'bf16' or 'f16').

    Returns (scale float32[J], codes uint16[nnz], dequantised float64[nnz]).
    """
    lib = _load()
    k = {"bf16": 1, "f16": 2}[kind]
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float32)
    scale = np.empty(J, np.float32)
    codes = np.empty(col.shape[0], np.uint16)
    deq = np.empty(col.shape[0], np.float64)
    lib.or_quantise(col.shape[0], J, _ptr(col), _ptr(val), k, _ptr(scale), _ptr(codes), _ptr(deq))
    return scale, codes, deq


def admm(prob, n_iter, f0=None, d0=None, c0=None, sweeps=None, beta=None, lam=None, w=None,
         grouping=0, report=True):
    """Run ADMM (Eqs. 4-6) from (f0, d0, c0); defaults: f0 = kappa*1, d0 = c0 = 0.

    Returns (f, d, c, rep) with rep[k] = (objective, data, tv, r_primal, r_dual)
    after iteration k+1.
    """
    lib = _load()
    J = prob.ny * prob.nx * prob.Q
    rp, c, v = _csr(prob.rowptr, prob.col, prob.val)
    y, r = _f64(prob.y), _f64(prob.r)
    ww = _weights(w, prob.ny, prob.nx, prob.Q)
    f = _f64(f0).copy() if f0 is not None else np.full(J, plain_init(prob), np.float64)
    d = _f64(d0).copy() if d0 is not None else np.zeros(J * NDIR, np.float64)
    cc = _f64(c0).copy() if c0 is not None else np.zeros(J * NDIR, np.float64)
    rep = np.zeros((max(n_iter, 1), 5), np.float64) if report else None
    st = lib.or_admm_flat(prob.I, prob.ny, prob.nx, prob.Q, _ptr(rp), _ptr(c), _ptr(v),
                          _ptr(y), _ptr(r), _ptr(ww),
                          float(prob.beta if beta is None else beta),
                          float(prob.rho if lam is None else lam), int(grouping), int(n_iter),
                          int(prob.sweeps if sweeps is None else sweeps),
                          _ptr(f), _ptr(d), _ptr(cc), _ptr(rep))
    if st != 0:
        raise MemoryError("oracle allocation failed")
    return f, d, cc, (rep[:n_iter] if report else None)


def admm_adaptive(prob, max_iter, check=10, eps_abs=1e-4, eps_rel=1e-3, mu=10.0, tau=2.0,
                  f0=None, d0=None, c0=None, sweeps=None, beta=None, lam=None, w=None, grouping=0):
    """ADMM with residual balancing and the residual stopping rule (Boyd et al.
    2011, Sections 3.3, 3.4.1).  Returns (f, d, c, lam, hist, iterations,
    converged), hist[m] = (iterations, r, s, eps_pri, eps_dual, lam after check m)."""
    lib = _load()
    J = prob.ny * prob.nx * prob.Q
    rp, c, v = _csr(prob.rowptr, prob.col, prob.val)
    y, r = _f64(prob.y), _f64(prob.r)
    ww = _weights(w, prob.ny, prob.nx, prob.Q)
    f = _f64(f0).copy() if f0 is not None else np.full(J, plain_init(prob), np.float64)
    d = _f64(d0).copy() if d0 is not None else np.zeros(J * NDIR, np.float64)
    cc = _f64(c0).copy() if c0 is not None else np.zeros(J * NDIR, np.float64)
    max_checks = max_iter // max(check, 1) + 2
    hist = np.zeros((max_checks, 6), np.float64)
    n_checks, lam_out, conv = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
    k = lib.or_admm_adaptive_flat(prob.I, prob.ny, prob.nx, prob.Q, _ptr(rp), _ptr(c), _ptr(v),
                                  _ptr(y), _ptr(r), _ptr(ww), float(prob.beta if beta is None else beta),
                                  float(prob.rho if lam is None else lam), int(grouping), int(max_iter),
                                  int(prob.sweeps if sweeps is None else sweeps), int(check), float(eps_abs),
                                  float(eps_rel), float(mu), float(tau), _ptr(f), _ptr(d), _ptr(cc),
                                  _ptr(hist), max_checks, ctypes.byref(n_checks), ctypes.byref(lam_out),
                                  ctypes.byref(conv))
    if k < 0:
        raise MemoryError("oracle allocation failed")
    return f, d, cc, lam_out.value, hist[:n_checks.value], k, bool(conv.value)


# ---- warm-start network (NHWC images, weights [co][ky][kx][ci]) ---------------------------

def wn_n_params(C, L=6):
    return L * (C * 9 * C + C)


def wn_conv_fwd(x, w, b=None):
    """x [B,H,W,Ci], w [Co,3,3,Ci], b [Co] -> z [B,H,W,Co] (zero padding 1)."""
    lib = _load()
    x, w = _f64(x), _f64(w)
    B, H, W, Ci = x.shape
    Co = w.shape[0]
    z = np.empty((B, H, W, Co), np.float64)
    bb = _f64(b) if b is not None else None
    lib.wn_conv_fwd(B, H, W, Ci, Co, _ptr(x), _ptr(w), _ptr(bb), _ptr(z))
    return z


def wn_conv_bwd_data(dz, w, Ci):
    lib = _load()
    dz, w = _f64(dz), _f64(w)
    B, H, W, Co = dz.shape
    dx = np.empty((B, H, W, Ci), np.float64)
    lib.wn_conv_bwd_data(B, H, W, Ci, Co, _ptr(dz), _ptr(w), _ptr(dx))
    return dx


def wn_conv_bwd_weight(x, dz):
    lib = _load()
    x, dz = _f64(x), _f64(dz)
    B, H, W, Ci = x.shape
    Co = dz.shape[3]
    dw = np.empty((Co, 3, 3, Ci), np.float64)
    db = np.empty(Co, np.float64)
    lib.wn_conv_bwd_weight(B, H, W, Ci, Co, _ptr(x), _ptr(dz), _ptr(dw), _ptr(db))
    return dw, db


def wn_forward(params, x_in, L=6):
    lib = _load()
    x_in = _f64(x_in)
    B, H, W, C = x_in.shape
    p = _f64(params)
    out = np.empty_like(x_in)
    lib.wn_forward(L, B, H, W, C, _ptr(p), _ptr(x_in), _ptr(out), None, None)
    return out


def wn_loss_grad(params, x_in, target, L=6):
    lib = _load()
    x_in, t, p = _f64(x_in), _f64(target), _f64(params)
    B, H, W, C = x_in.shape
    g = np.empty_like(p)
    loss = lib.wn_loss_grad(L, B, H, W, C, _ptr(p), _ptr(x_in), _ptr(t), _ptr(g))
    return loss, g


def wn_adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays; t is the 1-based step."""
    lib = _load()
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib.wn_adam(params.size, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), float(lr),
                float(b1), float(b2), float(eps))
