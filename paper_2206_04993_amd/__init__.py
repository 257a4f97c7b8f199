"""Python binding of the MI355X streaming SGEP library (libsgep.so).

Argument marshalling only: every function forwards to the C ABI of
``include/sgep.h`` with the same name; all arithmetic of an iteration runs in
the library's HIP kernels.  Device arrays are passed as ``torch`` tensors (or
raw integer device addresses); host arrays of player vectors are numpy
``(d, k)`` arrays whose column i is player i.

The library must have been built (``python -m paper_2206_04993_amd.build``);
importing the binding without it raises ``ImportError`` -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsgep.so")

SGEP_OK = 0
SGEP_EINVAL = -1
SGEP_ESHAPE = -2
SGEP_ENOMEM = -3
SGEP_EDEVICE = -4
SGEP_ENONFINITE = -5
SGEP_EUNSUPPORTED = -6
SGEP_EPOISONED = -7
SGEP_ELABEL = -8

SGEP_VEC_BNORM, SGEP_VEC_CANONICAL = 1, 2  # flags of sgep_vectors

SGEP_KIND_CCA, SGEP_KIND_GENERAL, SGEP_KIND_LDA, SGEP_KIND_ICA = 0, 1, 2, 3
SGEP_F64, SGEP_F32, SGEP_BF16, SGEP_FP8_E4M3 = 0, 1, 2, 3
SGEP_SGD, SGEP_ADAM = 0, 1
SGEP_SCHED_CONST, SGEP_SCHED_INV, SGEP_SCHED_WARMUP_HARMONIC = 0, 1, 2

# every symbol include/sgep.h declares
EXPORTS = (
    "sgep_init", "sgep_init_ex", "sgep_step", "sgep_step_lda", "sgep_kernels_per_step",
    "sgep_step_kernel_name",
    "sgep_step_profiled", "sgep_sync", "sgep_eigvals", "sgep_vectors", "sgep_vectors_noalloc",
    "sgep_auxiliary",
    "sgep_step_count", "sgep_means", "sgep_state_size", "sgep_get_state", "sgep_set_state",
    "sgep_destroy",
    "sgep_status_string", "sgep_version",
    "sgep_batch_init", "sgep_batch_instance", "sgep_batch_step", "sgep_batch_launches",
    "sgep_batch_step_profiled", "sgep_batch_plan", "sgep_batch_set_plan", "sgep_batch_tune",
    "sgep_batch_sync", "sgep_batch_destroy",
)


class sgep_config(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("k", ctypes.c_int32),
        ("optimizer", ctypes.c_int32), ("schedule", ctypes.c_int32),
        ("n_classes", ctypes.c_int32),
        ("dx", ctypes.c_int64), ("dy", ctypes.c_int64), ("b_max", ctypes.c_int64),
        ("eta0", ctypes.c_double), ("eta_T", ctypes.c_double), ("t0", ctypes.c_double),
        ("t_c", ctypes.c_double), ("T", ctypes.c_double), ("gamma", ctypes.c_double),
        ("rho", ctypes.c_double), ("eps_reg", ctypes.c_double),
        ("adam_b1", ctypes.c_double), ("adam_b2", ctypes.c_double),
        ("adam_eps", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("smooth", ctypes.c_int32), ("center", ctypes.c_int32), ("nu", ctypes.c_double),
    ]


def make_config(kind: int, dtype: int, k: int, dx: int, dy: int, b_max: int, *,
                optimizer: int = SGEP_SGD, schedule: int = SGEP_SCHED_CONST,
                eta0: float = 0.1, eta_T: float = 0.0, t0: float = 1.0, t_c: float = 1.0,
                T: float = 1.0, gamma: float = 1.0, rho: float = 1e-6, eps_reg: float = 0.0,
                adam_b1: float = 0.9, adam_b2: float = 0.999, adam_eps: float = 1e-8,
                n_classes: int = 0, seed: int = 0, smooth: int = 0,
                nu: float = 0.0, center: int = 0) -> sgep_config:
    """smooth = 1 selects Alg. 3 (smooth estimate between rho and nu);
    center = 1 centres the views by running means."""
    return sgep_config(kind, dtype, k, optimizer, schedule, n_classes, dx, dy, b_max, eta0,
                       eta_T, t0, t_c, T, gamma, rho, eps_reg, adam_b1, adam_b2, adam_eps, seed,
                       smooth, center, nu)


class sgep_init_aux(ctypes.Structure):
    _fields_ = [
        ("x_col_scale", ctypes.POINTER(ctypes.c_float)),
        ("y_col_scale", ctypes.POINTER(ctypes.c_float)),
        ("class_means", ctypes.POINTER(ctypes.c_double)),
        ("class_priors", ctypes.POINTER(ctypes.c_double)),
    ]


class SgepError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {sgep_status_string(status)} ({status})")


_lib = None


def load() -> ctypes.CDLL:
    """Load libsgep.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2206_04993_amd.build`")
    # torch ships its own HIP runtime under the same soname as ROCm's
    # (libamdhip64.so.7); loading torch first makes the library bind to that
    # one runtime, so torch's streams, events and allocations are valid here.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    lib.sgep_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(sgep_config), dp, vp]
    lib.sgep_init_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(sgep_config), dp,
                                 ctypes.POINTER(sgep_init_aux), vp]
    lib.sgep_step.argtypes = [vp, vp, i64, vp, i64, i64]
    lib.sgep_step_lda.argtypes = [vp, vp, i64, vp, i64]
    lib.sgep_kernels_per_step.argtypes = [vp, ctypes.POINTER(i32)]
    lib.sgep_step_kernel_name.argtypes = [vp, i32]
    lib.sgep_step_kernel_name.restype = ctypes.c_char_p
    lib.sgep_step_profiled.argtypes = [vp, vp, i64, vp, i64, vp, i64, ctypes.POINTER(vp), i32]
    lib.sgep_sync.argtypes = [vp]
    lib.sgep_eigvals.argtypes = [vp, dp]
    lib.sgep_vectors.argtypes = [vp, i32, dp]
    lib.sgep_vectors_noalloc.argtypes = [vp, i32, dp]
    lib.sgep_auxiliary.argtypes = [vp, dp]
    lib.sgep_step_count.argtypes = [vp, ctypes.POINTER(i64)]
    lib.sgep_means.argtypes = [vp, dp]
    lib.sgep_state_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.sgep_get_state.argtypes = [vp, vp, ctypes.c_size_t]
    lib.sgep_set_state.argtypes = [vp, vp, ctypes.c_size_t]
    lib.sgep_destroy.argtypes = [vp]
    lib.sgep_status_string.argtypes = [i32]
    lib.sgep_status_string.restype = ctypes.c_char_p
    lib.sgep_version.argtypes = []
    pi32, pi64 = ctypes.POINTER(i32), ctypes.POINTER(i64)
    lib.sgep_batch_init.argtypes = [ctypes.POINTER(vp), i32, pi64, pi64, ctypes.POINTER(sgep_config),
                                    ctypes.POINTER(dp), vp]
    lib.sgep_batch_instance.argtypes = [vp, i32, ctypes.POINTER(vp)]
    lib.sgep_batch_step.argtypes = [vp, vp, vp, i64]
    lib.sgep_batch_launches.argtypes = [vp, pi32, pi32, i32]
    lib.sgep_batch_step_profiled.argtypes = [vp, vp, vp, i64, ctypes.POINTER(vp), i32]
    lib.sgep_batch_plan.argtypes = [vp, pi32, pi32]
    lib.sgep_batch_set_plan.argtypes = [vp, i32, pi32]
    lib.sgep_batch_tune.argtypes = [vp, vp, vp, i64, i32, dp]
    lib.sgep_batch_sync.argtypes = [vp]
    lib.sgep_batch_destroy.argtypes = [vp]
    for name in EXPORTS:
        fn = getattr(lib, name)
        if name not in ("sgep_status_string", "sgep_step_kernel_name"):
            fn.restype = i32
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != SGEP_OK:
        raise SgepError(rc, where)


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def sgep_status_string(status: int) -> str:
    try:
        return load().sgep_status_string(status).decode()
    except ImportError:
        return f"status {status}"


def sgep_version() -> int:
    return int(load().sgep_version())


def sgep_init(cfg: sgep_config, V0: np.ndarray, stream=None) -> ctypes.c_void_p:
    """Create a solver.  V0: (d, k) host array of starting points."""
    lib = load()
    V0c = np.ascontiguousarray(np.asarray(V0, dtype=np.float64).T)  # column-major d x k
    h = ctypes.c_void_p()
    rc = lib.sgep_init(ctypes.byref(h), ctypes.byref(cfg),
                       V0c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream))
    _check(rc, "sgep_init")
    return h


def sgep_init_ex(cfg: sgep_config, V0: np.ndarray, stream=None, *, x_col_scale=None,
                 y_col_scale=None, class_means=None, class_priors=None) -> ctypes.c_void_p:
    """Create a solver with the problem data FP8 (column scales) or LDA (class
    means, n_classes x d, and priors) configurations need; host numpy arrays."""
    lib = load()
    V0c = np.ascontiguousarray(np.asarray(V0, dtype=np.float64).T)
    keep = []

    def f32p(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float32)
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def f64p(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    aux = sgep_init_aux(f32p(x_col_scale), f32p(y_col_scale), f64p(class_means),
                        f64p(class_priors))
    h = ctypes.c_void_p()
    rc = lib.sgep_init_ex(ctypes.byref(h), ctypes.byref(cfg),
                          V0c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          ctypes.byref(aux), _stream(stream))
    _check(rc, "sgep_init_ex")
    return h


def sgep_step(h, X, ldx: int, Y, ldy: int, b: int) -> None:
    """Enqueue one iteration on the minibatch views X (b x dx) and Y (b x dy)."""
    _check(load().sgep_step(h, _ptr(X), ldx, _ptr(Y), ldy, b), "sgep_step")


def sgep_step_lda(h, X, ldx: int, labels, b: int) -> None:
    """Enqueue one LDA iteration on X (b x d) with int32 device labels (b)."""
    _check(load().sgep_step_lda(h, _ptr(X), ldx, _ptr(labels), b), "sgep_step_lda")


def sgep_kernels_per_step(h) -> int:
    n = ctypes.c_int32()
    _check(load().sgep_kernels_per_step(h, ctypes.byref(n)), "sgep_kernels_per_step")
    return int(n.value)


def sgep_step_kernel_name(h, i: int) -> str:
    """Short name of kernel i of one iteration, in launch order."""
    n = load().sgep_step_kernel_name(h, i)
    if n is None:
        raise ValueError(f"sgep_step_kernel_name: no kernel {i}")
    return n.decode()


def sgep_step_profiled(h, X, ldx: int, Y, ldy: int, labels, b: int, events) -> None:
    """One iteration with caller-owned hipEvent_t handles (ints), a start/end
    pair per kernel in launch order (2 * sgep_kernels_per_step of them)."""
    ev = (ctypes.c_void_p * len(events))(*[int(e) for e in events])
    _check(load().sgep_step_profiled(h, _ptr(X), ldx, _ptr(Y), ldy, _ptr(labels), b, ev,
                                     len(events)), "sgep_step_profiled")


def sgep_sync(h) -> None:
    _check(load().sgep_sync(h), "sgep_sync")


def sgep_eigvals(h, k: int) -> np.ndarray:
    out = np.zeros(k)
    _check(load().sgep_eigvals(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "sgep_eigvals")
    return out


def sgep_vectors(h, d: int, k: int, flags: int = 0) -> np.ndarray:
    """Players as a (d, k) array; flags: an OR of SGEP_VEC_BNORM and
    SGEP_VEC_CANONICAL."""
    out = np.zeros((k, d))
    _check(load().sgep_vectors(h, int(flags),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "sgep_vectors")
    return out.T.copy()


def sgep_vectors_noalloc(h, d: int, k: int, flags: int = 0) -> np.ndarray:
    """sgep_vectors through the entry point that allocates no device memory."""
    out = np.zeros((k, d))
    _check(load().sgep_vectors_noalloc(h, int(flags),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "sgep_vectors_noalloc")
    return out.T.copy()


def sgep_auxiliary(h, d: int, k: int) -> np.ndarray:
    out = np.zeros((k, d))
    _check(load().sgep_auxiliary(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "sgep_auxiliary")
    return out.T.copy()


def sgep_means(h, n: int) -> np.ndarray:
    """Running means of the views (centring): n = dx + dy (GENERAL: 2 dx)."""
    out = np.zeros(n)
    _check(load().sgep_means(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "sgep_means")
    return out


def sgep_step_count(h) -> int:
    t = ctypes.c_int64()
    _check(load().sgep_step_count(h, ctypes.byref(t)), "sgep_step_count")
    return int(t.value)


def sgep_state_size(h) -> int:
    n = ctypes.c_size_t()
    _check(load().sgep_state_size(h, ctypes.byref(n)), "sgep_state_size")
    return int(n.value)


def sgep_get_state(h) -> bytes:
    n = sgep_state_size(h)
    buf = ctypes.create_string_buffer(n)
    _check(load().sgep_get_state(h, buf, n), "sgep_get_state")
    return buf.raw


def sgep_set_state(h, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(load().sgep_set_state(h, buf, len(blob)), "sgep_set_state")


def sgep_destroy(h) -> None:
    _check(load().sgep_destroy(h), "sgep_destroy")


def sgep_batch_init(d, ld, cfg: sgep_config, V0s, stream=None) -> ctypes.c_void_p:
    """Create n instances of widths d (host ints) with row leading dimensions
    ld; V0s: n host arrays (d_i, k) of starting points."""
    lib = load()
    n = len(d)
    d64 = (ctypes.c_int64 * n)(*[int(x) for x in d])
    ld64 = (ctypes.c_int64 * n)(*[int(x) for x in ld])
    cols = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).T) for v in V0s]
    ptrs = (ctypes.POINTER(ctypes.c_double) * n)(
        *[c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for c in cols])
    bt = ctypes.c_void_p()
    _check(lib.sgep_batch_init(ctypes.byref(bt), n, d64, ld64, ctypes.byref(cfg), ptrs,
                               _stream(stream)), "sgep_batch_init")
    return bt


def sgep_batch_instance(bt, i: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().sgep_batch_instance(bt, int(i), ctypes.byref(h)), "sgep_batch_instance")
    return h


def sgep_batch_step(bt, X_ptrs, Y_ptrs, b: int) -> None:
    """X_ptrs, Y_ptrs: int64 device tensors holding the n device pointers."""
    _check(load().sgep_batch_step(bt, _ptr(X_ptrs), _ptr(Y_ptrs), b), "sgep_batch_step")


def sgep_batch_launches(bt) -> list:
    lib = load()
    n = ctypes.c_int32()
    _check(lib.sgep_batch_launches(bt, ctypes.byref(n), None, 0), "sgep_batch_launches")
    kinds = (ctypes.c_int32 * max(1, n.value))()
    _check(lib.sgep_batch_launches(bt, ctypes.byref(n), kinds, n.value), "sgep_batch_launches")
    return [int(kinds[i]) for i in range(n.value)]


def sgep_batch_step_profiled(bt, X_ptrs, Y_ptrs, b: int, events) -> None:
    ev = (ctypes.c_void_p * len(events))(*[int(e) for e in events])
    _check(load().sgep_batch_step_profiled(bt, _ptr(X_ptrs), _ptr(Y_ptrs), b, ev, len(events)),
           "sgep_batch_step_profiled")


def sgep_batch_plan(bt):
    g = ctypes.c_int32()
    mb = (ctypes.c_int32 * 3)()
    _check(load().sgep_batch_plan(bt, ctypes.byref(g), mb), "sgep_batch_plan")
    return int(g.value), [int(mb[i]) for i in range(3)]


def sgep_batch_set_plan(bt, groups: int, mb_bucket) -> None:
    mb = (ctypes.c_int32 * 3)(*[int(x) for x in mb_bucket])
    _check(load().sgep_batch_set_plan(bt, int(groups), mb), "sgep_batch_set_plan")


def sgep_batch_tune(bt, X_ptrs, Y_ptrs, b: int, reps: int = 3) -> float:
    us = ctypes.c_double()
    _check(load().sgep_batch_tune(bt, _ptr(X_ptrs), _ptr(Y_ptrs), b, int(reps),
                                  ctypes.byref(us)), "sgep_batch_tune")
    return float(us.value)


def sgep_batch_sync(bt) -> None:
    _check(load().sgep_batch_sync(bt), "sgep_batch_sync")


def sgep_batch_destroy(bt) -> None:
    _check(load().sgep_batch_destroy(bt), "sgep_batch_destroy")


class Solver:
    """Owning convenience wrapper around one handle (same calls, fewer args)."""

    def __init__(self, cfg: sgep_config, V0: np.ndarray, stream=None, **aux):
        self.cfg = cfg
        self.d = cfg.dx + cfg.dy if cfg.kind == SGEP_KIND_CCA else cfg.dx
        self.k = cfg.k
        self.h = sgep_init_ex(cfg, V0, stream, **aux) if aux else sgep_init(cfg, V0, stream)

    def step(self, X, Y, b: Optional[int] = None, ldx: Optional[int] = None,
             ldy: Optional[int] = None):
        """One iteration; for LDA, Y is the int32 label vector; for ICA, Y is
        None."""
        b = X.shape[0] if b is None else b
        ldx = X.stride(0) if ldx is None else ldx
        if self.cfg.kind == SGEP_KIND_LDA:
            sgep_step_lda(self.h, X, ldx, Y, b)
            return
        if self.cfg.kind == SGEP_KIND_ICA:
            sgep_step(self.h, X, ldx, None, 0, b)
            return
        ldy = Y.stride(0) if ldy is None else ldy
        sgep_step(self.h, X, ldx, Y, ldy, b)

    def kernels_per_step(self):
        return sgep_kernels_per_step(self.h)

    def kernel_names(self):
        """Short names of the kernels of one iteration, in launch order."""
        return tuple(sgep_step_kernel_name(self.h, i) for i in range(self.kernels_per_step()))

    def sync(self):
        sgep_sync(self.h)

    def eigvals(self):
        return sgep_eigvals(self.h, self.k)

    def vectors(self, flags: int = 0):
        return sgep_vectors(self.h, self.d, self.k, flags)

    def auxiliary(self):
        return sgep_auxiliary(self.h, self.d, self.k)

    def step_count(self):
        return sgep_step_count(self.h)

    def means(self):
        """(mu_x, mu_y): the running means of the views (centring only)."""
        c = self.cfg
        dy = c.dy if c.kind == SGEP_KIND_CCA else c.dx
        m = sgep_means(self.h, c.dx + dy)
        return m[:c.dx], m[c.dx:]

    def get_state(self):
        return sgep_get_state(self.h)

    def set_state(self, blob):
        sgep_set_state(self.h, blob)

    def close(self):
        if self.h is not None:
            sgep_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Owning wrapper around a batch of GENERAL instances.  Minibatches are
    given as lists of device tensors (or one int64 device tensor of
    pointers per view)."""

    def __init__(self, d, cfg: sgep_config, V0s, ld=None, stream=None):
        self.d = [int(x) for x in d]
        self.ld = list(self.d) if ld is None else [int(x) for x in ld]
        self.k = cfg.k
        self.cfg = cfg
        self.bt = sgep_batch_init(self.d, self.ld, cfg, V0s, stream)

    @staticmethod
    def pointers(tensors, device):
        """int64 device tensor of the data pointers of `tensors`."""
        import torch
        return torch.tensor([t.data_ptr() for t in tensors], dtype=torch.int64, device=device)

    def step(self, Xp, Yp, b: int):
        sgep_batch_step(self.bt, Xp, Yp, b)

    def launches(self):
        return sgep_batch_launches(self.bt)

    def plan(self):
        return sgep_batch_plan(self.bt)

    def set_plan(self, groups, mb_bucket):
        sgep_batch_set_plan(self.bt, groups, mb_bucket)

    def tune(self, Xp, Yp, b: int, reps: int = 3):
        return sgep_batch_tune(self.bt, Xp, Yp, b, reps)

    def sync(self):
        sgep_batch_sync(self.bt)

    def instance(self, i):
        return sgep_batch_instance(self.bt, i)

    def vectors(self, i, flags: int = 0):
        return sgep_vectors(self.instance(i), self.d[i], self.k, flags)

    def auxiliary(self, i):
        return sgep_auxiliary(self.instance(i), self.d[i], self.k)

    def eigvals(self, i):
        return sgep_eigvals(self.instance(i), self.k)

    def step_count(self, i):
        return sgep_step_count(self.instance(i))

    def close(self):
        if self.bt is not None:
            sgep_batch_destroy(self.bt)
            self.bt = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
