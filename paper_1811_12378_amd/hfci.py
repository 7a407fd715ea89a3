"""Thin ctypes binding of libhfci (include/hfci.h).

Every function here only marshals arguments and calls the C ABI of the same
name; all arithmetic runs in the library's HIP kernels.  torch tensors are used
for device memory only (their data_ptr() crosses the boundary).  If the built
library is missing the import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfci.so")

HFCI_OK, HFCI_W_NOCONV = 0, 1
HFCI_F32, HFCI_F64 = 32, 64
HFCI_PRECOND_NONE, HFCI_PRECOND_FCI, HFCI_PRECOND_LEARNED = 0, 1, 2

STATUS_NAMES = {0: "HFCI_OK", 1: "HFCI_W_NOCONV", -1: "HFCI_E_ARG", -2: "HFCI_E_HIP", -3: "HFCI_E_OOM",
                -4: "HFCI_E_CONTOUR", -5: "HFCI_E_NUMERIC", -6: "HFCI_E_STATE"}

# every symbol include/hfci.h declares
EXPORTED = ["hfci_default_opts", "hfci_last_error", "hfci_version", "hfci_ctx_create", "hfci_ctx_destroy",
            "hfci_op_create", "hfci_op_destroy", "hfci_op_info", "hfci_apply", "hfci_contour_create",
            "hfci_contour_destroy", "hfci_contour_get", "hfci_shifted_solve", "hfci_fci_apply", "hfci_solve",
            "hfci_ctx_profile", "hfci_ctx_profile_read", "hfci_net_create", "hfci_net_destroy",
            "hfci_net_param_count", "hfci_net_get_params", "hfci_net_set_params", "hfci_net_get_grads",
            "hfci_net_eval", "hfci_net_train_step", "hfci_net_train", "hfci_net_apply", "hfci_op_medium_channel",
            "hfci_net_save", "hfci_net_load", "hfci_op_set_tune", "hfci_op_get_tune", "hfci_op_autotune",
            "hfci_shifted_solve_batch", "hfci_solve_batch", "hfci_op_case_two", "hfci_contour_q",
            "hfci_op_create_spectral", "hfci_shifted_solve_noalloc", "hfci_contour_params",
            "hfci_contour_rule"]
PROF_CLASSES = ["fp_stage", "fp_stage_first", "apply", "fp_stage_last", "fp_stage_init", "fp_stage_triple"]


class HfciError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class KernelProf(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong), ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_size_t), ("precision", ctypes.c_int), ("restart", ctypes.c_int),
                ("max_it", ctypes.c_int), ("tol", ctypes.c_double), ("fp_steps", ctypes.c_int),
                ("fp_reduce", ctypes.c_double), ("fp_max_steps", ctypes.c_int), ("k_in", ctypes.c_int),
                ("precond", ctypes.c_int), ("pole_batch", ctypes.c_int), ("verbose", ctypes.c_int),
                ("net", ctypes.c_void_p), ("learned_tau", ctypes.c_double), ("learned_patience", ctypes.c_int),
                ("harvest_cap", ctypes.c_int),
                ("harvest_v", ctypes.c_void_p), ("harvest_z", ctypes.c_void_p), ("graphs", ctypes.c_int),
                ("inner_precond", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("size", ctypes.c_size_t), ("its", ctypes.c_int), ("restarts", ctypes.c_int),
                ("matvecs", ctypes.c_longlong), ("fp_steps", ctypes.c_longlong),
                ("final_relres", ctypes.c_double), ("time_fci_ms", ctypes.c_double),
                ("time_arnoldi_ms", ctypes.c_double), ("time_total_ms", ctypes.c_double),
                ("harvested", ctypes.c_int), ("learned_accepted", ctypes.c_int), ("learned_fallbacks", ctypes.c_int),
                ("time_net_ms", ctypes.c_double), ("net_rho_mean", ctypes.c_double),
                ("fci_rho_mean", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "size"}


class NetDesc(ctypes.Structure):
    _fields_ = [("size", ctypes.c_size_t), ("seed", ctypes.c_ulonglong)]


class TrainDesc(ctypes.Structure):
    _fields_ = [("size", ctypes.c_size_t), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("npairs", ctypes.c_int), ("v", ctypes.c_void_p), ("e", ctypes.c_void_p),
                ("kch", ctypes.c_void_p), ("nmedia", ctypes.c_int), ("medium_of_pair", ctypes.c_void_p),
                ("crop", ctypes.c_int),
                ("steps", ctypes.c_int), ("lr", ctypes.c_float), ("lr_min", ctypes.c_float),
                ("phase_aug", ctypes.c_int), ("seed", ctypes.c_ulonglong), ("log_every", ctypes.c_int),
                ("verbose", ctypes.c_int), ("loss_curve", ctypes.c_void_p), ("loss_curve_cap", ctypes.c_int),
                ("loss_kind", ctypes.c_int)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhfci.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhfci.so not found at %s: build it with `python -m paper_1811_12378_amd.build`"
                          % path)
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "hfci_default_opts": (None, [P(SolveOpts)]),
        "hfci_last_error": (ctypes.c_char_p, []),
        "hfci_version": (ctypes.c_char_p, []),
        "hfci_ctx_create": (ip, [ip, vp, P(vp)]),
        "hfci_ctx_destroy": (None, [vp]),
        "hfci_op_create": (ip, [vp, ip, ip, ip, dp, vp, dp, ip, dp, P(vp)]),
        "hfci_op_destroy": (None, [vp]),
        "hfci_op_case_two": (ip, [vp, P(vp)]),
        "hfci_op_create_spectral": (ip, [vp, ip, ip, ip, dp, vp, dp, ip, dp, P(vp)]),
        "hfci_op_info": (ip, [vp, P(dp)]),
        "hfci_apply": (ip, [vp, c128, ip, ip, vp, vp]),
        "hfci_contour_create": (ip, [vp, ip, dp, dp, ip, vp, vp, vp, P(vp)]),
        "hfci_contour_destroy": (None, [vp]),
        "hfci_contour_get": (ip, [vp, vp, vp, vp, vp, vp]),
        "hfci_contour_q": (ip, [vp, P(ip)]),
        "hfci_contour_params": (ip, [vp, P(ip), P(dp), P(dp)]),
        "hfci_contour_rule": (ip, [dp, dp, dp, dp, ip, dp, ip, ip, dp, P(ip), P(dp), P(ip)]),
        "hfci_shifted_solve": (ip, [vp, vp, ip, ip, vp, vp, ip, dp, ip, vp]),
        "hfci_shifted_solve_noalloc": (ip, [vp, vp, ip, ip, vp, vp, ip, dp, ip, vp]),
        "hfci_fci_apply": (ip, [vp, vp, P(SolveOpts), ip, vp, vp, P(Stats)]),
        "hfci_solve": (ip, [vp, vp, P(SolveOpts), ip, vp, vp, P(Stats)]),
        "hfci_ctx_profile": (ip, [vp, ip]),
        "hfci_net_create": (ip, [vp, P(NetDesc), P(vp)]),
        "hfci_net_destroy": (None, [vp]),
        "hfci_net_param_count": (ctypes.c_longlong, [vp]),
        "hfci_net_get_params": (ip, [vp, vp]),
        "hfci_net_set_params": (ip, [vp, vp]),
        "hfci_net_get_grads": (ip, [vp, vp]),
        "hfci_net_eval": (ip, [vp, ip, ip, ip, vp, vp]),
        "hfci_net_train_step": (ip, [vp, ip, ip, ip, vp, vp, ctypes.c_float, ip, ip, P(dp)]),
        "hfci_net_train": (ip, [vp, P(TrainDesc), P(dp)]),
        "hfci_net_apply": (ip, [vp, vp, ip, vp, vp]),
        "hfci_op_medium_channel": (ip, [vp, vp]),
        "hfci_net_save": (ip, [vp, ctypes.c_char_p]),
        "hfci_net_load": (ip, [vp, ctypes.c_char_p]),
        "hfci_ctx_profile_read": (ip, [vp, P(KernelProf)]),
        "hfci_op_set_tune": (ip, [vp, ip, vp]),
        "hfci_op_get_tune": (ip, [vp, ip, vp]),
        "hfci_op_autotune": (ip, [vp, ip, ip, vp, vp, ip, vp]),
        "hfci_shifted_solve_batch": (ip, [ip, vp, vp, ip, vp, vp, ip, dp, ip, vp]),
        "hfci_solve_batch": (ip, [ip, vp, vp, P(SolveOpts), vp, vp, P(Stats)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status < 0:
        raise HfciError(status, load_library().hfci_last_error().decode())
    return status


def _sync():
    import torch
    torch.cuda.synchronize()


def _ptr(t, dtype=None, what="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (what, dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _check_grid(op, t, what, lead=1):
    """Raise ValueError unless t is `lead` leading batch dimensions followed by the
    operator's grid shape (op.shape: [nz, ny, nx], or [2, nz, ny, nx] for case two).
    The library derives every vector length from op.n and the batch count alone, so a
    wrongly shaped tensor must never reach it."""
    shp = tuple(op.shape)
    if t.dim() != lead + len(shp) or tuple(t.shape[lead:]) != shp:
        raise ValueError("%s has shape %s; expected %d batch dimension(s) followed by %s"
                         % (what, tuple(t.shape), lead, list(shp)))


def _check_like(t, ref, what):
    """t must match ref in shape, dtype and device (an initial guess against its f)."""
    if tuple(t.shape) != tuple(ref.shape) or t.dtype != ref.dtype or t.device != ref.device:
        raise ValueError("%s must match f: shape %s dtype %s device %s, got %s %s %s"
                         % (what, tuple(ref.shape), ref.dtype, ref.device, tuple(t.shape), t.dtype, t.device))


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load_library().hfci_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


_live_contexts = weakref.WeakSet()


class _Handle:
    """Owner of one library handle; released by close(), __del__ or interpreter exit."""

    _destroy = None

    def close(self):
        if getattr(self, "h", None):
            getattr(load_library(), self._destroy)(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the atexit hook has already released every handle
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass


class Context(_Handle):
    """hfci_ctx_create / hfci_ctx_destroy.  Closing a context first closes the
    operators and contours created from it."""

    _destroy = "hfci_ctx_destroy"

    def __init__(self, device: int = 0):
        self.h = ctypes.c_void_p()
        self._children = weakref.WeakSet()
        _check(load_library().hfci_ctx_create(device, None, ctypes.byref(self.h)))
        self.device = device
        _live_contexts.add(self)

    def _adopt(self, child):
        self._children.add(child)

    def profile(self, enable: bool = True, every: int = 1):
        """hfci_ctx_profile: start (counters reset; every k-th launch of each class timed)
        or stop kernel timing."""
        _check(load_library().hfci_ctx_profile(self.h, int(every) if enable else 0))

    def profile_read(self):
        """hfci_ctx_profile_read -> {class: {launches, total_ms, alg_bytes}}."""
        out = (KernelProf * len(PROF_CLASSES))()
        _check(load_library().hfci_ctx_profile_read(self.h, out))
        return {name: {"launches": out[k].launches, "total_ms": out[k].total_ms, "alg_bytes": out[k].alg_bytes}
                for k, name in enumerate(PROF_CLASSES)}

    def close(self):
        kids = list(self._children)
        for k in kids:  # contours before operators
            if isinstance(k, Contour):
                k.close()
        for k in kids:
            k.close()
        super().close()


@atexit.register
def _close_all():
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


class Operator(_Handle):
    """hfci_op_create: c is a float64 CUDA tensor [nz, ny, nx] (x fastest)."""

    _destroy = "hfci_op_destroy"

    def __init__(self, ctx: Context, c, h: float, omega: float, damp_cells: int, damp_rho2: float):
        import torch
        self.h = ctypes.c_void_p()
        if c.dim() != 3:
            raise ValueError("c must be [nz, ny, nx]")
        self.ctx = ctx
        self.shape = tuple(c.shape)
        nz, ny, nx = self.shape
        _sync()
        _check(load_library().hfci_op_create(ctx.h, nx, ny, nz, h, _ptr(c, torch.float64, "c"), omega,
                                             damp_cells, damp_rho2, ctypes.byref(self.h)))
        self.n = nx * ny * nz
        ctx._adopt(self)

    def info(self):
        out = (ctypes.c_double * 7)()
        _check(load_library().hfci_op_info(self.h, out))
        keys = ["s", "s_h2", "b1", "b2", "rho2", "kappa_min", "kappa_max"]
        return dict(zip(keys, list(out)))

    def set_tune(self, prec: int, kern: int, ty: int, pd: int, cz: int = 0, fuse: int = 0, sg: int = 1):
        """hfci_op_set_tune: stencil launch shape (kernel, 64 x ty tile, prefetch depth pd, z-chunk cz,
        two fixed-point factors per pass, systems taken sg at a time tile by tile)."""
        t = (ctypes.c_int * 6)(kern, ty, pd, cz, fuse, sg)
        _check(load_library().hfci_op_set_tune(self.h, prec, ctypes.cast(t, ctypes.c_void_p)))

    def autotune(self, prec: int, nsys: int = 2):
        """hfci_op_autotune: pick the fastest stencil launch shape; returns (best, [(shape, ms), ...])."""
        best = (ctypes.c_int * 6)()
        cap = 128
        tm = (ctypes.c_double * (7 * cap))()
        cnt = ctypes.c_int()
        _check(load_library().hfci_op_autotune(self.h, prec, nsys, ctypes.cast(best, ctypes.c_void_p),
                                               ctypes.cast(tm, ctypes.c_void_p), cap,
                                               ctypes.cast(ctypes.byref(cnt), ctypes.c_void_p)))
        rows = [(tuple(int(v) for v in tm[7 * k:7 * k + 6]), float(tm[7 * k + 6])) for k in range(min(cnt.value, cap))]
        return tuple(best), rows

    def get_tune(self, prec: int):
        t = (ctypes.c_int * 6)()
        _check(load_library().hfci_op_get_tune(self.h, prec, ctypes.cast(t, ctypes.c_void_p)))
        return tuple(t)

    def case_two(self):
        """hfci_op_case_two: the double-size operator B = iC - I of eq. mat-2x2 on this A."""
        return CaseTwoOperator(self)


class SpectralOperator(Operator):
    """hfci_op_create_spectral: the Fourier-spectral Laplacian of Sec. 7.1 on a periodic grid."""

    def __init__(self, ctx: Context, c, h: float, omega: float, damp_cells: int, damp_rho2: float):
        import torch
        self.h = ctypes.c_void_p()
        if c.dim() != 3:
            raise ValueError("c must be [nz, ny, nx]")
        self.ctx = ctx
        self.shape = tuple(c.shape)
        nz, ny, nx = self.shape
        _sync()
        _check(load_library().hfci_op_create_spectral(ctx.h, nx, ny, nz, h, _ptr(c, torch.float64, "c"), omega,
                                                      damp_cells, damp_rho2, ctypes.byref(self.h)))
        self.n = nx * ny * nz
        ctx._adopt(self)


class CaseTwoOperator(_Handle):
    """hfci_op_case_two: B = iC - I (eq. mat-2x2); vectors have shape [2, nz, ny, nx] (x1 then x2)."""

    _destroy = "hfci_op_destroy"

    def __init__(self, base: Operator):
        self.h = ctypes.c_void_p()
        self.ctx = base.ctx
        self.base = base
        self.shape = (2,) + tuple(base.shape)
        self.n = 2 * base.n
        _check(load_library().hfci_op_case_two(base.h, ctypes.byref(self.h)))
        base.ctx._adopt(self)

    def info(self):
        out = (ctypes.c_double * 7)()
        _check(load_library().hfci_op_info(self.h, out))
        keys = ["s", "s_h2", "b1", "b2", "rho2", "kappa_min", "kappa_max"]
        return dict(zip(keys, list(out)))


class Net(_Handle):
    """hfci_net_create: the learned preconditioner (3-level 3D U-Net, BF16 on the matrix cores)."""

    _destroy = "hfci_net_destroy"

    def __init__(self, ctx: Context, seed: int = 1234):
        self.h = ctypes.c_void_p()
        d = NetDesc(ctypes.sizeof(NetDesc), seed)
        _check(load_library().hfci_net_create(ctx.h, ctypes.byref(d), ctypes.byref(self.h)))
        self.ctx = ctx
        self.nparam = int(load_library().hfci_net_param_count(self.h))
        ctx._adopt(self)

    def get_params(self):
        out = np.empty(self.nparam, dtype=np.float32)
        _check(load_library().hfci_net_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.nparam
        _check(load_library().hfci_net_set_params(self.h, flat.ctypes.data))

    def get_grads(self):
        out = np.empty(self.nparam, dtype=np.float32)
        _check(load_library().hfci_net_get_grads(self.h, out.ctypes.data))
        return out

    def eval(self, x16):
        """hfci_net_eval: x16 bf16 CUDA tensor [nz, ny, nx, 16] -> float32 [nz, ny, nx, 2]."""
        import torch
        nz, ny, nx, c = x16.shape
        out = torch.empty((nz, ny, nx, 2), dtype=torch.float32, device=x16.device)
        _sync()
        _check(load_library().hfci_net_eval(self.h, nx, ny, nz, _ptr(x16, torch.bfloat16, "x16"), _ptr(out)))
        return out

    def train_step(self, x16, target, lr: float = 1e-3, update: bool = True, loss_kind: int = 0):
        import torch
        nz, ny, nx, _ = x16.shape
        loss = ctypes.c_double()
        _sync()
        _check(load_library().hfci_net_train_step(self.h, nx, ny, nz, _ptr(x16, torch.bfloat16, "x16"),
                                                  _ptr(target, torch.float32, "target"), lr, 1 if update else 0,
                                                  loss_kind, ctypes.byref(loss)))
        return loss.value

    def train(self, v, e, kch, medium_of_pair, crop: int, steps: int, lr: float = 1e-3, lr_min: float = 1e-5,
              phase_aug: bool = True, seed: int = 0, log_every: int = 0, verbose: bool = False,
              loss_kind: int = 1):
        """hfci_net_train: v, e complex64 [P, nz, ny, nx]; kch float32 [M, nz, ny, nx]."""
        import torch
        P, nz, ny, nx = v.shape
        mop = np.ascontiguousarray(medium_of_pair, dtype=np.int32)
        ncurve = (steps // log_every + 2) if log_every > 0 else 0
        curve = np.zeros(max(ncurve, 1))
        if kch.dim() != 4 or tuple(kch.shape[1:]) != (nz, ny, nx) or tuple(e.shape) != tuple(v.shape):
            raise ValueError("v, e [P, nz, ny, nx] and kch [M, nz, ny, nx] must share the grid")
        d = TrainDesc(ctypes.sizeof(TrainDesc), nx, ny, nz, P, _ptr(v, torch.complex64, "v"),
                      _ptr(e, torch.complex64, "e"), _ptr(kch, torch.float32, "kch"), kch.shape[0],
                      mop.ctypes.data, crop, steps,
                      lr, lr_min, 1 if phase_aug else 0, seed, log_every, 1 if verbose else 0,
                      curve.ctypes.data, ncurve, loss_kind)
        final = ctypes.c_double()
        _sync()
        _check(load_library().hfci_net_train(self.h, ctypes.byref(d), ctypes.byref(final)))
        return final.value, curve[:ncurve]

    def apply(self, op, r):
        """hfci_net_apply: complex128 [nvec, nz, ny, nx] -> z of the same shape."""
        import torch
        _check_grid(op, r, "r")
        z = torch.empty_like(r)
        nvec = r.shape[0]
        _sync()
        _check(load_library().hfci_net_apply(self.h, op.h, nvec, _ptr(r, torch.complex128, "r"), _ptr(z)))
        return z

    def save(self, path: str):
        _check(load_library().hfci_net_save(self.h, path.encode()))

    def load(self, path: str):
        _check(load_library().hfci_net_load(self.h, path.encode()))


def medium_channel(op):
    """hfci_op_medium_channel: omega^2 h^2 / c^2 as a float32 CUDA tensor [nz, ny, nx]."""
    import torch
    out = torch.empty(op.shape, dtype=torch.float32, device="cuda")
    _sync()
    _check(load_library().hfci_op_medium_channel(op.h, _ptr(out)))
    return out


def _prec_of(t):
    import torch
    if t.dtype == torch.complex128:
        return HFCI_F64
    if t.dtype == torch.complex64:
        return HFCI_F32
    raise TypeError("complex64 or complex128 expected, got %s" % t.dtype)


def apply(op, x, shift: complex = 0.0, out=None):
    """hfci_apply: (A - shift I) x for x of shape [..., nz, ny, nx] (batch = leading dims); for a
    case-two operator (B - shift I) x with x of shape [..., 2, nz, ny, nx]."""
    import torch
    prec = _prec_of(x)
    k = len(op.shape)
    if tuple(x.shape[-k:]) != op.shape:
        raise ValueError("x shape %s != operator %s" % (tuple(x.shape[-k:]), op.shape))
    nvec = x.numel() // op.n
    if out is None:
        out = torch.empty_like(x)
    _sync()
    _check(load_library().hfci_apply(op.h, c128(shift.real, shift.imag), prec, nvec, _ptr(x, None, "x"),
                                     _ptr(out, x.dtype, "out")))
    return out


class Contour(_Handle):
    """hfci_contour_create: poles/weights/delta default to eq. quad-points and the delta search."""

    _destroy = "hfci_contour_destroy"

    def __init__(self, op: Operator, J: int, t: float = 1.0, eps: float = 0.5, q: int = 8,
                 z=None, sigma=None, delta=None):
        self.h = ctypes.c_void_p()
        self.op = op
        self.J = J
        self.q = q
        zp = sp = dp = None
        if z is not None:
            za = (c128 * J)(*[c128(complex(v).real, complex(v).imag) for v in z])
            sa = (c128 * J)(*[c128(complex(v).real, complex(v).imag) for v in sigma])
            zp, sp = ctypes.cast(za, ctypes.c_void_p), ctypes.cast(sa, ctypes.c_void_p)
            self._keep = (za, sa)
        if delta is not None:
            da = (ctypes.c_double * J)(*[float(v) for v in delta])
            dp = ctypes.cast(da, ctypes.c_void_p)
            self._keepd = da
        _check(load_library().hfci_contour_create(op.h, J, t, eps, q, zp, sp, dp, ctypes.byref(self.h)))
        op.ctx._adopt(self)
        if q == 0:  # chosen by the library (Sec. 4.2)
            qv = ctypes.c_int()
            _check(load_library().hfci_contour_q(self.h, ctypes.byref(qv)))
            self.q = qv.value
        if J == 0 or eps == 0:  # chosen by the library's rule
            self.J = self.params()["J"]

    def params(self):
        """hfci_contour_params: {"J", "t", "eps"} (the chosen values for J = 0 or eps = 0)."""
        Jv, tv, ev = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        _check(load_library().hfci_contour_params(self.h, ctypes.byref(Jv), ctypes.byref(tv), ctypes.byref(ev)))
        return {"J": Jv.value, "t": tv.value, "eps": ev.value}

    def get(self):
        J = self.J
        z, s, z0 = (c128 * J)(), (c128 * J)(), (c128 * J)()
        d, nu = (ctypes.c_double * J)(), (ctypes.c_double * J)()
        _check(load_library().hfci_contour_get(self.h, z, s, d, z0, nu))
        cz = lambda a: np.array([complex(v.re, v.im) for v in a])
        return {"z": cz(z), "sigma": cz(s), "delta": np.array(d[:]), "z0": cz(z0), "nu": np.array(nu[:])}


def contour_rule(b1: float, b2: float, rho2: float, npoints: float, J: int = 0, t: float = 1.0, q: int = 0,
                 per_pass: int = 2, fp_reduce: float = 5.0):
    """hfci_contour_rule (host arithmetic only): (J, eps, q) for the spectrum box [b1, b2] x [-rho2, 0]
    of an operator on npoints grid points (per_pass = 2 for finite differences, 1 spectral)."""
    Jv, ev, qv = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
    _check(load_library().hfci_contour_rule(b1, b2, rho2, float(npoints), J, t, q, per_pass, fp_reduce,
                                            ctypes.byref(Jv), ctypes.byref(ev), ctypes.byref(qv)))
    return Jv.value, ev.value, qv.value


def shifted_solve(op, c: Contour, f, steps: int = 0, reduce: float = 5.0, max_steps: int = 200):
    """hfci_shifted_solve: f [nrhs, *op.shape] -> (y [J, nrhs, *op.shape], steps taken [J, nrhs])."""
    import torch
    prec = _prec_of(f)
    _check_grid(op, f, "f")
    nrhs = f.shape[0]
    y = torch.empty((c.J,) + tuple(f.shape), dtype=f.dtype, device=f.device)
    st = (ctypes.c_int * (c.J * nrhs))()
    _sync()
    _check(load_library().hfci_shifted_solve(op.h, c.h, prec, nrhs, _ptr(f, None, "f"), _ptr(y), steps, reduce,
                                             max_steps, ctypes.cast(st, ctypes.c_void_p)))
    return y, np.array(st[:]).reshape(c.J, nrhs)


def shifted_solve_noalloc(op, c: Contour, f, y, steps: int = 0, reduce: float = 5.0, max_steps: int = 200):
    """hfci_shifted_solve_noalloc: as shifted_solve, into a caller-provided y [J, nrhs, *op.shape]
    of f's dtype, with every other buffer in the library's static scratch array (no device
    allocation, by the library or here).  Returns the steps taken [J, nrhs]."""
    prec = _prec_of(f)
    _check_grid(op, f, "f")
    nrhs = f.shape[0]
    if tuple(y.shape) != (c.J,) + tuple(f.shape) or y.dtype != f.dtype or y.device != f.device:
        raise ValueError("y must be [J, nrhs, *grid] with f's dtype and device")
    st = (ctypes.c_int * (c.J * nrhs))()
    _sync()
    _check(load_library().hfci_shifted_solve_noalloc(op.h, c.h, prec, nrhs, _ptr(f, None, "f"), _ptr(y, None, "y"),
                                                     steps, reduce, max_steps, ctypes.cast(st, ctypes.c_void_p)))
    return np.array(st[:]).reshape(c.J, nrhs)


def fci_apply(op: Operator, c: Contour, f, opts: SolveOpts | None = None):
    """hfci_fci_apply (Algorithm 1): f complex128 [nrhs, nz, ny, nx] -> out, stats."""
    import torch
    _check_grid(op, f, "f")
    if f.dtype != torch.complex128:
        raise TypeError("f must be complex128, got %s" % f.dtype)
    opts = opts or default_opts()
    out = torch.empty_like(f)
    st = Stats()
    st.size = ctypes.sizeof(Stats)
    _sync()
    _check(load_library().hfci_fci_apply(op.h, c.h, ctypes.byref(opts), f.shape[0],
                                         _ptr(f, torch.complex128, "f"), _ptr(out), ctypes.byref(st)))
    return out, st.as_dict()


def solve(op: Operator, c: Contour | None, f, u0=None, opts: SolveOpts | None = None):
    """hfci_solve: physical f complex128 [nrhs, nz, ny, nx] -> (u, stats, status)."""
    import torch
    _check_grid(op, f, "f")
    if f.dtype != torch.complex128:
        raise TypeError("f must be complex128, got %s" % f.dtype)
    if u0 is not None:
        _check_like(u0, f, "u0")
    opts = opts or default_opts()
    u = torch.zeros_like(f) if u0 is None else u0.clone()
    st = Stats()
    st.size = ctypes.sizeof(Stats)
    _sync()
    status = _check(load_library().hfci_solve(op.h, c.h if c is not None else None, ctypes.byref(opts),
                                              f.shape[0], _ptr(f, torch.complex128, "f"), _ptr(u),
                                              ctypes.byref(st)))
    d = st.as_dict()
    d["status"] = STATUS_NAMES[status]
    return u, d


def _ptr_array(ts, dtype=None, what="vector"):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t, dtype, what)
    return arr


def shifted_solve_batch(ops, contours, fs, steps: int = 0, reduce: float = 5.0, max_steps: int = 200):
    """hfci_shifted_solve_batch: fs[i] [nz_i, ny_i, nx_i] (one rhs per instance, complex64 or complex128)
    -> ([y_i [J_i, nz_i, ny_i, nx_i]], [steps_i [J_i]])."""
    import torch
    if not (len(ops) == len(contours) == len(fs)) or not ops:
        raise ValueError("ops, contours and fs must be non-empty lists of one length")
    prec = _prec_of(fs[0])
    for i, (o, f) in enumerate(zip(ops, fs)):
        _check_grid(o, f, "fs[%d]" % i, lead=0)
        if f.dtype != fs[0].dtype:
            raise TypeError("fs[%d] has dtype %s; every right-hand side must be %s" % (i, f.dtype, fs[0].dtype))
    ys = [torch.empty((c.J,) + tuple(f.shape), dtype=f.dtype, device=f.device) for c, f in zip(contours, fs)]
    nsys = sum(c.J for c in contours)
    st = (ctypes.c_int * nsys)()
    oh = (ctypes.c_void_p * len(ops))(*[o.h.value for o in ops])
    ch = (ctypes.c_void_p * len(ops))(*[c.h.value for c in contours])
    _sync()
    _check(load_library().hfci_shifted_solve_batch(len(ops), ctypes.cast(oh, ctypes.c_void_p),
                                                   ctypes.cast(ch, ctypes.c_void_p), prec,
                                                   ctypes.cast(_ptr_array(fs, None, "f"), ctypes.c_void_p),
                                                   ctypes.cast(_ptr_array(ys), ctypes.c_void_p), steps, reduce,
                                                   max_steps, ctypes.cast(st, ctypes.c_void_p)))
    out, k = [], 0
    for c in contours:
        out.append(np.array(st[k:k + c.J]))
        k += c.J
    return ys, out


def solve_batch(ops, contours, fs, opts: SolveOpts | None = None, u0s=None):
    """hfci_solve_batch: physical fs[i] complex128 [nz_i, ny_i, nx_i] -> ([u_i], [stats_i], status)."""
    import torch
    n = len(ops)
    if n == 0 or len(fs) != n or (contours is not None and len(contours) != n) or \
            (u0s is not None and len(u0s) != n):
        raise ValueError("ops, contours, fs (and u0s) must be non-empty lists of one length")
    for i, (o, f) in enumerate(zip(ops, fs)):
        _check_grid(o, f, "fs[%d]" % i, lead=0)
        if f.dtype != torch.complex128:
            raise TypeError("fs[%d] must be complex128, got %s" % (i, f.dtype))
        if u0s is not None:
            _check_like(u0s[i], f, "u0s[%d]" % i)
    opts = opts or default_opts()
    us = [torch.zeros_like(f) if u0s is None else u0s[i].clone() for i, f in enumerate(fs)]
    sts = (Stats * n)()
    for k in range(n):
        sts[k].size = ctypes.sizeof(Stats)
    oh = (ctypes.c_void_p * n)(*[o.h.value for o in ops])
    ch = (ctypes.c_void_p * n)(*[c.h.value for c in contours]) if contours is not None else None
    _sync()
    status = _check(load_library().hfci_solve_batch(
        n, ctypes.cast(oh, ctypes.c_void_p), ctypes.cast(ch, ctypes.c_void_p) if ch is not None else None,
        ctypes.byref(opts), ctypes.cast(_ptr_array(fs, torch.complex128, "f"), ctypes.c_void_p),
        ctypes.cast(_ptr_array(us), ctypes.c_void_p), sts))
    return us, [sts[k].as_dict() for k in range(n)], STATUS_NAMES[status]
