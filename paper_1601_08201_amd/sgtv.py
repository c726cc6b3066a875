"""Python binding of libsgtv.so (ctypes): argument marshalling only.

The functions below carry the names of the C entry points declared in
include/sgtv.h and forward their arguments unchanged; every step of the
reconstruction runs in the library's HIP kernels.  NumPy arrays are passed as
host memory, torch CUDA tensors as device memory (PyTorch provides device
memory and streams, nothing else).  If the library has not been built the
first call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH

SGTV_OK, SGTV_EINVAL, SGTV_ESHAPE, SGTV_ESTATE, SGTV_EDEVICE, SGTV_ENOMEM = 0, -1, -2, -3, -4, -5
SGTV_NOALLOC_MAX_VOXELS = 4194304   # largest J of sgtv_backprojection_noalloc
SGTV_F32, SGTV_BF16, SGTV_F16 = 0, 1, 2
SGTV_HOST, SGTV_DEVICE = 0, 1
WSNET_START_RATIO, WSNET_START_DIRECT = 0, 1
SGTV_GROUP_SPECTRAL, SGTV_GROUP_STANDARD = 0, 1

STORAGE = {"f32": SGTV_F32, "bf16": SGTV_BF16, "f16": SGTV_F16}


class SgtvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sgtv error %d: %s" % (code, msg))
        self.code = code


class Adaptive(ctypes.Structure):
    _fields_ = [("check", ctypes.c_int32), ("eps_abs", ctypes.c_double), ("eps_rel", ctypes.c_double),
                ("mu", ctypes.c_double), ("tau", ctypes.c_double)]


class Check(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int64), ("r_primal", ctypes.c_double), ("r_dual", ctypes.c_double),
                ("eps_primal", ctypes.c_double), ("eps_dual", ctypes.c_double), ("rho", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Report(ctypes.Structure):
    _fields_ = [("total", ctypes.c_double), ("data", ctypes.c_double), ("tv", ctypes.c_double),
                ("r_primal", ctypes.c_double), ("r_dual", ctypes.c_double), ("iter", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Schedule(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("fwd_rows_per_wave", ctypes.c_int32), ("fwd_block_cols", ctypes.c_int32),
                ("fwd_slabs", ctypes.c_int32), ("back_rows_per_wave", ctypes.c_int32),
                ("back_block_cols", ctypes.c_int32), ("back_slabs", ctypes.c_int32),
                ("variant", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SGTV_FORMAT_TILED, SGTV_FORMAT_SELL = 0, 1

_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_I = ctypes.c_int
_D = ctypes.c_double


def lib():
    """Load libsgtv.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsgtv.so is not built: run python -m paper_1601_08201_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "sgtv_create": (_I, [ctypes.POINTER(_P), _I, _P]),
            "sgtv_destroy": (None, [_P]),
            "sgtv_last_error": (ctypes.c_char_p, []),
            "sgtv_version": (ctypes.c_char_p, []),
            "sgtv_set_system": (_I, [_P, _I64, _I32, _I32, _I32, _P, _P, _P, _I64, _I, _P, _I64, _I]),
            "sgtv_plan_system": (_I, [_P, _I64, _I32, _I32, _I32, _P, _P, _P, _I64, _I, _P, _I64, _I,
                                      ctypes.POINTER(_I64)]),
            "sgtv_commit_system": (_I, [_P, _P, _I64]),
            "sgtv_save_system": (_I, [_P, ctypes.c_char_p]),
            "sgtv_load_system": (_I, [_P, ctypes.c_char_p]),
            "sgtv_set_data": (_I, [_P, _P, _P, _D, _D, _I, _I]),
            "sgtv_set_grouping": (_I, [_P, _I]),
            "sgtv_set_init": (_I, [_P, _P, _I]),
            "sgtv_set_init_dual": (_I, [_P, _P, _I]),
            "sgtv_iterate": (_I, [_P, _I]),
            "sgtv_prepare": (_I, [_P, _I]),
            "sgtv_objective": (_I, [_P, ctypes.POINTER(Report)]),
            "sgtv_get_image": (_I, [_P, _P, _I]),
            "sgtv_get_split": (_I, [_P, _P, _P, _I]),
            "sgtv_state_sizes": (_I, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
            "sgtv_get_state": (_I, [_P, _P, _P, _P, ctypes.POINTER(_I64), _I]),
            "sgtv_set_state": (_I, [_P, _P, _P, _P, _I64, _I]),
            "sgtv_backprojection": (_I, [_P, _P, _I]),
            "sgtv_backprojection_noalloc": (_I, [_P, _P, _I]),
            "sgtv_set_fused_update": (_I, [_P, _I]),
            "sgtv_set_epilogues": (_I, [_P, _I]),
            "sgtv_get_epilogues": (_I, [_P, ctypes.POINTER(_I)]),
            "sgtv_get_fused_update": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
            "sgtv_set_profiling": (_I, [_P, _I]),
            "sgtv_set_graphs": (_I, [_P, _I]),
            "sgtv_batch_create": (_I, [ctypes.POINTER(_P), _I, _P]),
            "sgtv_batch_destroy": (None, [_P]),
            "sgtv_batch_add_scan": (_I, [_P, _I64, _I32, _I32, _I32, _P, _P, _P, _I64, _P, _I64, _P, _P,
                                         _D, _D, _I, ctypes.POINTER(Schedule), _I, ctypes.POINTER(_I32)]),
            "sgtv_batch_add_system_file": (_I, [_P, ctypes.c_char_p, _P, _P, _D, _D, _I, _I,
                                                ctypes.POINTER(_I32)]),
            "sgtv_batch_save_scan": (_I, [_P, _I32, ctypes.c_char_p]),
            "sgtv_batch_set_storage": (_I, [_P, _I]),
            "sgtv_batch_size": (_I, [_P, ctypes.POINTER(_I32)]),
            "sgtv_batch_iterate": (_I, [_P, _I]),
            "sgtv_batch_prepare": (_I, [_P, _I, _I]),
            "sgtv_batch_iterate_sequential": (_I, [_P, _I]),
            "sgtv_batch_set_launch": (_I, [_P, _I]),
            "sgtv_batch_get_launch": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I32)]),
            "sgtv_batch_phase_times": (_I, [_P, _P, ctypes.POINTER(_I64)]),
            "sgtv_batch_objective": (_I, [_P, _I32, ctypes.POINTER(Report)]),
            "sgtv_batch_get_image": (_I, [_P, _I32, _P, _I]),
            "wsnet_create": (_I, [ctypes.POINTER(_P), _I, _P, _I32, _I32, _I32, _I32, _I32]),
            "wsnet_destroy": (None, [_P]),
            "wsnet_param_count": (_I64, [_I32, _I32]),
            "wsnet_set_params": (_I, [_P, _P, _I64, _I]),
            "wsnet_get_params": (_I, [_P, _P, _I64, _I]),
            "wsnet_forward": (_I, [_P, _P, _I32, _P, _I]),
            "wsnet_start": (_I, [_P, _P, _I32, _I, _D, _D, _P, _I]),
            "wsnet_backward": (_I, [_P, _P, _P, _I32, ctypes.POINTER(_D), _P, _I]),
            "wsnet_adam_step": (_I, [_P, _D, _D, _D, _D]),
            "wsnet_train_step": (_I, [_P, _P, _P, _I32, _D, _D, _D, _D, _I]),
            "wsnet_loss_sum": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I64), _I]),
            "wsnet_reset_adam": (_I, [_P]),
            "sgtv_set_schedule": (_I, [_P, ctypes.POINTER(Schedule)]),
            "sgtv_set_penalty": (_I, [_P, _D]),
            "sgtv_workspace_bytes": (_I64, [_I64, _I64, _I64, _I]),
            "sgtv_device_bytes": (_I, [_P, ctypes.POINTER(_I64)]),
            "wsnet_save": (_I, [_P, ctypes.c_char_p]),
            "wsnet_load": (_I, [_P, ctypes.c_char_p]),
            "sgtv_get_penalty": (_I, [_P, ctypes.POINTER(_D)]),
            "sgtv_iterate_adaptive": (_I, [_P, _I64, ctypes.POINTER(Adaptive), ctypes.POINTER(Check), _I32,
                                           ctypes.POINTER(_I32), ctypes.POINTER(_I64), ctypes.POINTER(_I)]),
            "sgtv_get_schedule": (_I, [_P, ctypes.POINTER(Schedule)]),
            "sgtv_kernel_times": (_I, [_P, _P, _P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != SGTV_OK:
        raise SgtvError(code, lib().sgtv_last_error().decode(errors="replace"))


def _is_torch_cuda(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def _arg(a, dtype):
    """(pointer, mem_kind, keepalive) for a NumPy array or torch CUDA tensor."""
    if a is None:
        return None, SGTV_HOST, None
    if _is_torch_cuda(a):
        import torch
        tdt = {np.float32: torch.float32, np.int32: torch.int32, np.int64: torch.int64}[dtype]
        if a.dtype != tdt or not a.is_contiguous():
            a = a.to(tdt).contiguous()
        return ctypes.c_void_p(a.data_ptr()), SGTV_DEVICE, a
    arr = np.ascontiguousarray(np.asarray(a), dtype=dtype)
    return arr.ctypes.data_as(ctypes.c_void_p), SGTV_HOST, arr


def _kind(*items):
    kinds = {k for (_, k, keep) in items if keep is not None}
    if len(kinds) > 1:
        raise ValueError("mix of host arrays and device tensors in one call")
    return kinds.pop() if kinds else SGTV_HOST


# ---- thin wrappers with the C names ---------------------------------------------------

def sgtv_create(device=0, stream=None):
    h = ctypes.c_void_p()
    _check(lib().sgtv_create(ctypes.byref(h), int(device), stream))
    return h


def sgtv_destroy(ctx):
    lib().sgtv_destroy(ctx)


def sgtv_last_error():
    return lib().sgtv_last_error().decode(errors="replace")


def sgtv_version():
    return lib().sgtv_version().decode()


def sgtv_set_system(ctx, I, ny, nx, Q, row_ptr, col_idx, val, storage="f32", w=None):
    a = _arg(row_ptr, np.int64)
    b = _arg(col_idx, np.int32)
    c = _arg(val, np.float32)
    wa = _arg(w, np.float32)
    mk = _kind(a, b, c, wa)
    nnz = int(b[2].shape[0]) if b[2] is not None else 0
    wlen = 0 if w is None else int(np.prod(wa[2].shape))
    _check(lib().sgtv_set_system(ctx, int(I), int(ny), int(nx), int(Q), a[0], b[0], c[0], nnz,
                                 STORAGE.get(storage, storage), wa[0], wlen, mk))


def sgtv_plan_system(ctx, I, ny, nx, Q, row_ptr, col_idx, val, storage="f32", w=None):
    """Pack the system on the host; returns the exact device bytes of the
    workspace that sgtv_commit_system needs."""
    a = _arg(row_ptr, np.int64)
    b = _arg(col_idx, np.int32)
    c = _arg(val, np.float32)
    wa = _arg(w, np.float32)
    mk = _kind(a, b, c, wa)
    nnz = int(b[2].shape[0]) if b[2] is not None else 0
    wlen = 0 if w is None else int(np.prod(wa[2].shape))
    n = _I64()
    _check(lib().sgtv_plan_system(ctx, int(I), int(ny), int(nx), int(Q), a[0], b[0], c[0], nnz,
                                  STORAGE.get(storage, storage), wa[0], wlen, mk, ctypes.byref(n)))
    return n.value


def sgtv_commit_system(ctx, workspace, nbytes=None):
    """Put the planned system into a caller-owned device buffer: a torch
    tensor on the context's GPU (its bytes are used) or a raw device pointer
    with nbytes."""
    if hasattr(workspace, "data_ptr"):
        ptr = workspace.data_ptr()
        size = workspace.numel() * workspace.element_size() if nbytes is None else int(nbytes)
    else:
        ptr, size = int(workspace), int(nbytes)
    _check(lib().sgtv_commit_system(ctx, ctypes.c_void_p(ptr), size))


def sgtv_save_system(ctx, path):
    """Write the context's packed system to a file."""
    _check(lib().sgtv_save_system(ctx, os.fsencode(path)))


def sgtv_load_system(ctx, path):
    """Install a packed system from a file that sgtv_save_system wrote."""
    _check(lib().sgtv_load_system(ctx, os.fsencode(path)))


def sgtv_set_data(ctx, y, r, beta, rho, sweeps=1):
    a, b = _arg(y, np.float32), _arg(r, np.float32)
    _check(lib().sgtv_set_data(ctx, a[0], b[0], float(beta), float(rho), int(sweeps), _kind(a, b)))


def sgtv_set_grouping(ctx, grouping):
    _check(lib().sgtv_set_grouping(ctx, int(grouping)))


def sgtv_set_init(ctx, x0=None):
    a = _arg(x0, np.float32)
    _check(lib().sgtv_set_init(ctx, a[0], _kind(a)))


def sgtv_set_init_dual(ctx, x0):
    a = _arg(x0, np.float32)
    _check(lib().sgtv_set_init_dual(ctx, a[0], _kind(a)))


def sgtv_iterate(ctx, n_iters):
    _check(lib().sgtv_iterate(ctx, int(n_iters)))


def sgtv_prepare(ctx, n_iters):
    _check(lib().sgtv_prepare(ctx, int(n_iters)))


def sgtv_objective(ctx):
    rep = Report()
    _check(lib().sgtv_objective(ctx, ctypes.byref(rep)))
    return rep.as_dict()


def sgtv_state_sizes(ctx):
    a, b, c = _I64(), _I64(), _I64()
    _check(lib().sgtv_state_sizes(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def _out(n, like=None):
    if like is not None:
        return like
    return np.empty(n, np.float32)


def _out_arg(out):
    if _is_torch_cuda(out):
        return ctypes.c_void_p(out.data_ptr()), SGTV_DEVICE
    return out.ctypes.data_as(ctypes.c_void_p), SGTV_HOST


def sgtv_get_image(ctx, out=None):
    n_img, _, _ = sgtv_state_sizes(ctx)
    out = _out(n_img, out)
    p, mk = _out_arg(out)
    _check(lib().sgtv_get_image(ctx, p, mk))
    return out


def sgtv_get_split(ctx):
    _, n_split, _ = sgtv_state_sizes(ctx)
    d, c = np.empty(n_split, np.float32), np.empty(n_split, np.float32)
    _check(lib().sgtv_get_split(ctx, d.ctypes.data_as(_P), c.ctypes.data_as(_P), SGTV_HOST))
    return d, c


def sgtv_workspace_bytes(I, J, nnz, storage="f32"):
    return int(lib().sgtv_workspace_bytes(int(I), int(J), int(nnz), STORAGE[storage]
                                          if isinstance(storage, str) else int(storage)))


def sgtv_device_bytes(ctx):
    b = _I64()
    _check(lib().sgtv_device_bytes(ctx, ctypes.byref(b)))
    return b.value


def sgtv_set_penalty(ctx, rho):
    _check(lib().sgtv_set_penalty(ctx, float(rho)))


def sgtv_get_penalty(ctx):
    r = _D()
    _check(lib().sgtv_get_penalty(ctx, ctypes.byref(r)))
    return r.value


def sgtv_iterate_adaptive(ctx, max_iters, check=10, eps_abs=1e-4, eps_rel=1e-3, mu=10.0, tau=2.0):
    opt = Adaptive(int(check), float(eps_abs), float(eps_rel), float(mu), float(tau))
    cap = int(max_iters) // max(int(check), 1) + 2
    arr = (Check * cap)()
    n, k, conv = _I32(), _I64(), _I()
    _check(lib().sgtv_iterate_adaptive(ctx, int(max_iters), ctypes.byref(opt), arr, cap, ctypes.byref(n),
                                       ctypes.byref(k), ctypes.byref(conv)))
    return {"iterations": k.value, "converged": bool(conv.value),
            "checks": [arr[i].as_dict() for i in range(min(n.value, cap))]}


def sgtv_get_state(ctx):
    n_img, n_split, n_gr = sgtv_state_sizes(ctx)
    f, v, a = np.empty(n_img, np.float32), np.empty(n_split, np.float32), np.empty(n_gr, np.float32)
    k = _I64()
    _check(lib().sgtv_get_state(ctx, f.ctypes.data_as(_P), v.ctypes.data_as(_P), a.ctypes.data_as(_P),
                                ctypes.byref(k), SGTV_HOST))
    return f, v, a, k.value


def sgtv_set_state(ctx, f, v, a, k):
    fa, va, aa = _arg(f, np.float32), _arg(v, np.float32), _arg(a, np.float32)
    _check(lib().sgtv_set_state(ctx, fa[0], va[0], aa[0], int(k), _kind(fa, va, aa)))


def sgtv_backprojection(ctx, out=None):
    n_img, _, _ = sgtv_state_sizes(ctx)
    out = _out(n_img, out)
    p, mk = _out_arg(out)
    _check(lib().sgtv_backprojection(ctx, p, mk))
    return out


def sgtv_backprojection_noalloc(ctx, out=None):
    """As sgtv_backprojection, with no device allocation inside the call (the
    library's static device buffer holds the intermediates)."""
    n_img, _, _ = sgtv_state_sizes(ctx)
    out = _out(n_img, out)
    p, mk = _out_arg(out)
    _check(lib().sgtv_backprojection_noalloc(ctx, p, mk))
    return out


def sgtv_set_epilogues(ctx, enable=True):
    _check(lib().sgtv_set_epilogues(ctx, 1 if enable else 0))


def sgtv_get_epilogues(ctx):
    e = _I()
    _check(lib().sgtv_get_epilogues(ctx, ctypes.byref(e)))
    return bool(e.value)


def sgtv_set_fused_update(ctx, enable=True):
    _check(lib().sgtv_set_fused_update(ctx, 1 if enable else 0))


def sgtv_get_fused_update(ctx):
    """(in use, tile bins in x, tile bins in y)"""
    a, tx, ty = _I(), _I32(), _I32()
    _check(lib().sgtv_get_fused_update(ctx, ctypes.byref(a), ctypes.byref(tx), ctypes.byref(ty)))
    return bool(a.value), tx.value, ty.value


def sgtv_set_schedule(ctx, **fields):
    """Schedule for the next set_system; unnamed fields are automatic (0)."""
    sch = Schedule(**{k: int(v) for k, v in fields.items()})
    _check(lib().sgtv_set_schedule(ctx, ctypes.byref(sch)))


def sgtv_get_schedule(ctx):
    sch = Schedule()
    _check(lib().sgtv_get_schedule(ctx, ctypes.byref(sch)))
    return sch.as_dict()


def sgtv_set_graphs(ctx, enable):
    _check(lib().sgtv_set_graphs(ctx, int(bool(enable))))


def sgtv_set_profiling(ctx, enable):
    _check(lib().sgtv_set_profiling(ctx, int(bool(enable))))


KERNEL_CLASSES = ("forward", "back", "split_update", "ratio", "image_update")


def sgtv_kernel_times(ctx):
    """{class: (total_ms, launches)} accumulated since the last call."""
    ms = (ctypes.c_double * 5)()
    cnt = (ctypes.c_int64 * 5)()
    _check(lib().sgtv_kernel_times(ctx, ctypes.cast(ms, _P), ctypes.cast(cnt, _P)))
    return {KERNEL_CLASSES[i]: (ms[i], cnt[i]) for i in range(5)}


class Reconstructor:
    """Owning handle around one library context (one scan)."""

    def __init__(self, device=0, stream=None):
        self._ctx = sgtv_create(device, stream)

    def close(self):
        if self._ctx is not None:
            sgtv_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._ctx

    def set_system(self, I, ny, nx, Q, row_ptr, col_idx, val, storage="f32", w=None):
        sgtv_set_system(self._ctx, I, ny, nx, Q, row_ptr, col_idx, val, storage, w)
        return self

    def set_problem(self, prob, storage="f32", w=None, sweeps=None):
        """Convenience: set system and data of a datagen.Problem."""
        self.set_system(prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col, prob.val,
                        storage=storage, w=w)
        self.set_data(prob.y, prob.r, prob.beta, prob.rho, prob.sweeps if sweeps is None else sweeps)
        return self

    def set_data(self, y, r, beta, rho, sweeps=1):
        sgtv_set_data(self._ctx, y, r, beta, rho, sweeps)
        return self

    def set_grouping(self, grouping):
        sgtv_set_grouping(self._ctx, grouping)
        return self

    def set_init(self, x0=None):
        sgtv_set_init(self._ctx, x0)
        return self

    def set_init_dual(self, x0):
        sgtv_set_init_dual(self._ctx, x0)
        return self

    def iterate(self, n):
        sgtv_iterate(self._ctx, n)
        return self

    def prepare(self, n):
        """Capture the graph of iterate(n) now, without running it."""
        sgtv_prepare(self._ctx, n)
        return self

    def objective(self):
        return sgtv_objective(self._ctx)

    def image(self, out=None):
        return sgtv_get_image(self._ctx, out)

    def split(self):
        return sgtv_get_split(self._ctx)

    def state(self):
        return sgtv_get_state(self._ctx)

    def set_penalty(self, rho):
        sgtv_set_penalty(self._ctx, rho)
        return self

    def device_bytes(self):
        return sgtv_device_bytes(self._ctx)

    def penalty(self):
        return sgtv_get_penalty(self._ctx)

    def iterate_adaptive(self, max_iters, check=10, eps_abs=1e-4, eps_rel=1e-3, mu=10.0, tau=2.0):
        """Residual balancing and the residual stopping rule; returns
        {"iterations", "converged", "checks": [...]}."""
        return sgtv_iterate_adaptive(self._ctx, max_iters, check, eps_abs, eps_rel, mu, tau)

    def set_state(self, f, v, a, k):
        sgtv_set_state(self._ctx, f, v, a, k)
        return self

    def backprojection(self, out=None):
        return sgtv_backprojection(self._ctx, out)

    def set_schedule(self, **fields):
        sgtv_set_schedule(self._ctx, **fields)
        return self

    def plan_system(self, I, ny, nx, Q, row_ptr, col_idx, val, storage="f32", w=None):
        return sgtv_plan_system(self._ctx, I, ny, nx, Q, row_ptr, col_idx, val, storage, w)

    def commit_system(self, workspace, nbytes=None):
        sgtv_commit_system(self._ctx, workspace, nbytes)
        return self

    def save_system(self, path):
        sgtv_save_system(self._ctx, path)
        return self

    def load_system(self, path):
        sgtv_load_system(self._ctx, path)
        return self

    def set_fused_update(self, enable=True):
        sgtv_set_fused_update(self._ctx, enable)
        return self

    def fused_update(self):
        return sgtv_get_fused_update(self._ctx)

    def set_epilogues(self, enable=True):
        sgtv_set_epilogues(self._ctx, enable)
        return self

    def epilogues(self):
        return sgtv_get_epilogues(self._ctx)

    def schedule(self):
        return sgtv_get_schedule(self._ctx)

    def set_graphs(self, enable=True):
        sgtv_set_graphs(self._ctx, enable)
        return self

    def set_profiling(self, enable=True):
        sgtv_set_profiling(self._ctx, enable)
        return self

    def kernel_times(self):
        return sgtv_kernel_times(self._ctx)


# ---- batches -----------------------------------------------------------------------------

def sgtv_batch_create(device=0, stream=None):
    h = ctypes.c_void_p()
    _check(lib().sgtv_batch_create(ctypes.byref(h), int(device), stream))
    return h


def sgtv_batch_destroy(b):
    lib().sgtv_batch_destroy(b)


def sgtv_batch_add_scan(b, I, ny, nx, Q, row_ptr, col_idx, val, y, r, beta, rho, schedule=None,
                        w=None, grouping=0):
    a = _arg(row_ptr, np.int64)
    c = _arg(col_idx, np.int32)
    v = _arg(val, np.float32)
    ya, ra = _arg(y, np.float32), _arg(r, np.float32)
    wa = _arg(w, np.float32)
    mk = _kind(a, c, v, ya, ra, wa)
    wlen = 0 if w is None else int(np.prod(wa[2].shape))
    sch = ctypes.byref(Schedule(**{k: int(x) for k, x in schedule.items()})) if schedule else None
    idx = _I32()
    _check(lib().sgtv_batch_add_scan(b, int(I), int(ny), int(nx), int(Q), a[0], c[0], v[0],
                                     int(c[2].shape[0]), wa[0], wlen, ya[0], ra[0], float(beta), float(rho),
                                     int(grouping), sch, mk, ctypes.byref(idx)))
    return idx.value


def sgtv_batch_add_system_file(b, path, y, r, beta, rho, grouping=0):
    ya, ra = _arg(y, np.float32), _arg(r, np.float32)
    idx = _I32()
    _check(lib().sgtv_batch_add_system_file(b, os.fsencode(path), ya[0], ra[0], float(beta), float(rho),
                                            int(grouping), _kind(ya, ra), ctypes.byref(idx)))
    return idx.value


def sgtv_batch_set_storage(b, storage="f32"):
    _check(lib().sgtv_batch_set_storage(b, STORAGE.get(storage, storage)))


def sgtv_batch_save_scan(b, scan, path):
    _check(lib().sgtv_batch_save_scan(b, int(scan), os.fsencode(path)))


def sgtv_batch_size(b):
    n = _I32()
    _check(lib().sgtv_batch_size(b, ctypes.byref(n)))
    return n.value


def sgtv_batch_iterate(b, n_iters):
    _check(lib().sgtv_batch_iterate(b, int(n_iters)))


def sgtv_batch_prepare(b, n_iters, sequential=False):
    _check(lib().sgtv_batch_prepare(b, int(n_iters), int(bool(sequential))))


def sgtv_batch_iterate_sequential(b, n_iters):
    _check(lib().sgtv_batch_iterate_sequential(b, int(n_iters)))


BATCH_LAUNCH = {"graph": 0, "persistent": 1}


def sgtv_batch_set_launch(b, mode):
    """mode: "graph" (five batched launches per iteration in a HIP graph) or
    "persistent" (one cooperative launch with grid barriers)."""
    _check(lib().sgtv_batch_set_launch(b, BATCH_LAUNCH[mode] if isinstance(mode, str) else int(mode)))


def sgtv_batch_phase_times(b):
    """Milliseconds per phase of the persistent launches since the last call
    (forward + split, ratio, back, image update, final split) and the
    iterations they cover."""
    ms = np.zeros(5, np.float64)
    it = _I64()
    _check(lib().sgtv_batch_phase_times(b, ms.ctypes.data_as(_P), ctypes.byref(it)))
    return ms, it.value


def sgtv_batch_get_launch(b):
    m, g = _I(), _I32()
    _check(lib().sgtv_batch_get_launch(b, ctypes.byref(m), ctypes.byref(g)))
    return {v: k for k, v in BATCH_LAUNCH.items()}[m.value], g.value


def sgtv_batch_objective(b, scan):
    rep = Report()
    _check(lib().sgtv_batch_objective(b, int(scan), ctypes.byref(rep)))
    return rep.as_dict()


def sgtv_batch_get_image(b, scan, n, out=None):
    out = _out(n, out)
    p, mk = _out_arg(out)
    _check(lib().sgtv_batch_get_image(b, int(scan), p, mk))
    return out


class Batch:
    """Owning handle around a batch of scans iterated together."""

    def __init__(self, device=0, stream=None, storage="f32"):
        self._b = sgtv_batch_create(device, stream)
        self._J = {}     # batch index -> unknowns (add_scan may run on several threads)
        if storage != "f32":
            sgtv_batch_set_storage(self._b, storage)

    def close(self):
        if self._b is not None:
            sgtv_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_scan(self, prob, schedule=None, w=None, grouping=0, beta=None):
        i = sgtv_batch_add_scan(self._b, prob.I, prob.ny, prob.nx, prob.Q, prob.rowptr, prob.col,
                                prob.val, prob.y, prob.r, prob.beta if beta is None else beta, prob.rho,
                                schedule, w, grouping)
        self._J[i] = prob.ny * prob.nx * prob.Q
        return i

    def add_system_file(self, path, prob, grouping=0, beta=None):
        """Add a scan whose system a file holds (save_scan or
        Reconstructor.save_system); data, beta and rho from prob."""
        i = sgtv_batch_add_system_file(self._b, path, prob.y, prob.r, prob.beta if beta is None else beta,
                                       prob.rho, grouping)
        self._J[i] = prob.ny * prob.nx * prob.Q
        return i

    def save_scan(self, scan, path):
        sgtv_batch_save_scan(self._b, scan, path)
        return self

    def __len__(self):
        return sgtv_batch_size(self._b)

    def iterate(self, n):
        sgtv_batch_iterate(self._b, n)
        return self

    def prepare(self, n, sequential=False):
        """Capture now, without running them, the graphs of iterate(n)
        (sequential=False) or of iterate_sequential(n) (sequential=True)."""
        sgtv_batch_prepare(self._b, n, sequential)
        return self

    def iterate_sequential(self, n):
        sgtv_batch_iterate_sequential(self._b, n)
        return self

    def set_launch(self, mode):
        sgtv_batch_set_launch(self._b, mode)
        return self

    def launch(self):
        """(mode, grid of the last persistent launch)"""
        return sgtv_batch_get_launch(self._b)

    def phase_times(self):
        return sgtv_batch_phase_times(self._b)

    def objective(self, scan):
        return sgtv_batch_objective(self._b, scan)

    def image(self, scan, out=None):
        return sgtv_batch_get_image(self._b, scan, self._J[scan], out)


# ---- warm-start network ------------------------------------------------------------------

def wsnet_create(device=0, stream=None, layers=6, height=64, width=64, channels=64, max_batch=32):
    h = ctypes.c_void_p()
    _check(lib().wsnet_create(ctypes.byref(h), int(device), stream, int(layers), int(height),
                              int(width), int(channels), int(max_batch)))
    return h


def wsnet_destroy(net):
    lib().wsnet_destroy(net)


def wsnet_param_count(layers, channels):
    return int(lib().wsnet_param_count(int(layers), int(channels)))


def wsnet_set_params(net, params):
    a = _arg(params, np.float32)
    _check(lib().wsnet_set_params(net, a[0], int(np.prod(a[2].shape)), _kind(a)))


def wsnet_get_params(net, n):
    out = np.empty(n, np.float32)
    _check(lib().wsnet_get_params(net, out.ctypes.data_as(_P), n, SGTV_HOST))
    return out


def wsnet_forward(net, x_in, batch, out):
    a = _arg(x_in, np.float32)
    p, mk = _out_arg(out)
    if mk != _kind(a):
        raise ValueError("x_in and out must both be host arrays or both device tensors")
    _check(lib().wsnet_forward(net, a[0], int(batch), p, mk))
    return out


def wsnet_start(net, f, batch, mode, c_out, out, floor=0.0):
    a = _arg(f, np.float32)
    p, mk = _out_arg(out)
    if mk != _kind(a):
        raise ValueError("f and out must both be host arrays or both device tensors")
    _check(lib().wsnet_start(net, a[0], int(batch), int(mode), float(c_out), float(floor), p, mk))
    return out


def wsnet_backward(net, x_in, target, batch, grad=None):
    a, t = _arg(x_in, np.float32), _arg(target, np.float32)
    mk = _kind(a, t)
    loss = ctypes.c_double()
    gp = None
    if grad is not None:
        gp, gmk = _out_arg(grad)
        if gmk != mk:
            raise ValueError("grad must live where the inputs live")
    _check(lib().wsnet_backward(net, a[0], t[0], int(batch), ctypes.byref(loss), gp, mk))
    return loss.value


def wsnet_adam_step(net, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().wsnet_adam_step(net, float(lr), float(beta1), float(beta2), float(eps)))


def wsnet_train_step(net, x_in, target, batch, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    a, t = _arg(x_in, np.float32), _arg(target, np.float32)
    _check(lib().wsnet_train_step(net, a[0], t[0], int(batch), float(lr), float(beta1), float(beta2),
                                  float(eps), _kind(a, t)))


def wsnet_loss_sum(net, reset=True):
    s, n = ctypes.c_double(), _I64()
    _check(lib().wsnet_loss_sum(net, ctypes.byref(s), ctypes.byref(n), 1 if reset else 0))
    return s.value, n.value


def wsnet_reset_adam(net):
    _check(lib().wsnet_reset_adam(net))


class WarmStartNet:
    """Owning handle of the warm-start network (images NHWC, 64 channels)."""

    def __init__(self, device=0, stream=None, layers=6, height=64, width=64, channels=64, max_batch=32):
        self.shape = (height, width, channels)
        self.layers = layers
        self.max_batch = max_batch
        self.n_params = wsnet_param_count(layers, channels)
        self._n = wsnet_create(device, stream, layers, height, width, channels, max_batch)

    def close(self):
        if self._n is not None:
            wsnet_destroy(self._n)
            self._n = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        wsnet_set_params(self._n, params)
        return self

    def params(self):
        return wsnet_get_params(self._n, self.n_params)

    def forward(self, x_in, out=None):
        b = x_in.shape[0]
        if out is None:
            out = np.empty((b,) + self.shape, np.float32) if not _is_torch_cuda(x_in) else x_in.new_empty(x_in.shape)
        return wsnet_forward(self._n, x_in, b, out)

    def save(self, path):
        _check(lib().wsnet_save(self._n, os.fsencode(path)))
        return self

    def load(self, path):
        _check(lib().wsnet_load(self._n, os.fsencode(path)))
        return self

    def start(self, f, mode="ratio", c_out=1.0, out=None, floor=0.0):
        """Start images x0 from images f (see wsnet_start): mode "ratio" gives
        c_out * net(f / mean f) * f, "direct" c_out * net(f / mean f) * mean f;
        floor > 0 raises every voxel to at least floor * c_out * mean f."""
        b = f.shape[0]
        if out is None:
            out = np.empty((b,) + self.shape, np.float32) if not _is_torch_cuda(f) else f.new_empty(f.shape)
        m = {"ratio": WSNET_START_RATIO, "direct": WSNET_START_DIRECT}[mode]
        return wsnet_start(self._n, f, b, m, c_out, out, floor)

    def backward(self, x_in, target, grad=None):
        return wsnet_backward(self._n, x_in, target, x_in.shape[0], grad)

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        wsnet_adam_step(self._n, lr, beta1, beta2, eps)
        return self

    def train_step(self, x_in, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """backward + adam_step without waiting for the device; the loss goes
        to a running sum (loss_sum)."""
        wsnet_train_step(self._n, x_in, target, x_in.shape[0], lr, beta1, beta2, eps)
        return self

    def loss_sum(self, reset=True):
        """(sum of the train_step losses, number of steps) since the last reset."""
        return wsnet_loss_sum(self._n, reset)

    def reset_adam(self):
        wsnet_reset_adam(self._n)
        return self


def init_params(layers=6, channels=64, seed=0):
    """He-style random initial parameters (float32), biases zero."""
    rng = np.random.default_rng(seed)
    per = channels * 9 * channels
    out = []
    for _ in range(layers):
        out.append(rng.normal(scale=np.sqrt(2.0 / (9 * channels)), size=per).astype(np.float32))
        out.append(np.zeros(channels, np.float32))
    return np.concatenate(out)
