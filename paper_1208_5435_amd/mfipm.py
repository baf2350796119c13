"""Python binding of the HIP mfIPM library (ctypes).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  The
binding fails loudly when the built library is missing; there is no CPU path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmfipm.so")

OP_DENSE = 0
OP_PDCT = 1
OP_WHT = 2
OP_PDST = 3
TRANSFORMS = {"dct": OP_PDCT, "wht": OP_WHT, "dst": OP_PDST}

STATUS = {0: "CONVERGED", 1: "MAXITER", 2: "PCG_BREAKDOWN", 3: "NONFINITE", 4: "STEP_UNDERFLOW",
          5: "ABORTED", 6: "INPUT_CHECK", 7: "PCG_MAXITER"}
ERRORS = {-1: "INVALID_ARG", -2: "HIP_ERROR", -3: "WORKSPACE_TOO_SMALL", -4: "NO_STATE",
          -5: "DEVICE_CHECK", -6: "TOO_LARGE"}

# every symbol declared in include/mfipm.h
EXPORTS = ("mfipm_params_default", "mfipm_create", "mfipm_set_params", "mfipm_destroy",
           "mfipm_workspace_size", "mfipm_solve", "mfipm_solve_noalloc", "mfipm_solve_batched",
           "mfipm_backward", "mfipm_set_launch", "mfipm_last_kernel_ms", "mfipm_status_string")


class Params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiters", ctypes.c_int32),
                ("tolpcg", ctypes.c_double), ("mxiterpcg", ctypes.c_int32),
                ("sigma1", ctypes.c_double), ("sigma2", ctypes.c_double), ("sigma3", ctypes.c_double),
                ("alpha_bar", ctypes.c_double), ("alpha_tilde", ctypes.c_double),
                ("eta", ctypes.c_double), ("rho", ctypes.c_double),
                ("z0", ctypes.c_double), ("s0", ctypes.c_double),
                ("tolpcg_adj", ctypes.c_double), ("mxiterpcg_adj", ctypes.c_int32),
                ("step_min", ctypes.c_double), ("reduced", ctypes.c_int32),
                ("direct", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("ipm_iters", ctypes.c_int32),
                ("pcg_iters", ctypes.c_int32), ("correctors", ctypes.c_int32),
                ("nmat", ctypes.c_int64), ("rel_gap", ctypes.c_double), ("mu", ctypes.c_double),
                ("primal_obj", ctypes.c_double), ("dual_obj", ctypes.c_double),
                ("rho", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class Operator(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("rows", ctypes.c_void_p)]


_lib = None
_live = weakref.WeakSet()  # open Solver handles, closed at interpreter exit


@atexit.register
def _close_all():
    """Releases every open handle while the HIP runtime is still up (before
    module teardown), after the device has finished its work."""
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass


def load_library(path: str | None = None):
    """Loads libmfipm.so (built by paper_1208_5435_amd.build); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} (run python -m paper_1208_5435_amd.build)")
    lib = ctypes.CDLL(p)
    P, I = ctypes.POINTER(Params), ctypes.POINTER(Info)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    pi64 = ctypes.POINTER(ctypes.c_int64)
    pdbl = ctypes.POINTER(ctypes.c_double)
    lib.mfipm_params_default.argtypes = [P]
    lib.mfipm_create.argtypes = [ctypes.POINTER(vp), P, vp]
    lib.mfipm_set_params.argtypes = [vp, P]
    lib.mfipm_destroy.argtypes = [vp]
    lib.mfipm_workspace_size.argtypes = [vp, i32, i64, i64, i32, ctypes.POINTER(sz)]
    lib.mfipm_solve.argtypes = [vp, ctypes.POINTER(Operator), vp, dbl, vp, vp, vp, sz, I]
    lib.mfipm_solve_noalloc.argtypes = [vp, ctypes.POINTER(Operator), vp, dbl, vp, vp, I]
    lib.mfipm_solve_batched.argtypes = [vp, i32, pi64, pi64, pi64, i32, vp, vp, i32, vp, pdbl, vp, vp, vp,
                                        sz, I]
    lib.mfipm_backward.argtypes = [vp, i32, pi64, pi64, pi64, i32, vp, vp, i32, vp, vp, vp, vp, vp, sz, I]
    lib.mfipm_set_launch.argtypes = [vp, i32, i32, i32]
    lib.mfipm_last_kernel_ms.argtypes = [vp]
    lib.mfipm_last_kernel_ms.restype = dbl
    lib.mfipm_status_string.argtypes = [i32]
    lib.mfipm_status_string.restype = ctypes.c_char_p
    for name in ("mfipm_params_default", "mfipm_create", "mfipm_set_params", "mfipm_destroy",
                 "mfipm_workspace_size", "mfipm_solve", "mfipm_solve_noalloc", "mfipm_solve_batched",
                 "mfipm_backward", "mfipm_set_launch"):
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def default_params() -> Params:
    p = Params()
    rc = load_library().mfipm_params_default(ctypes.byref(p))
    if rc:
        raise RuntimeError(f"mfipm_params_default: {rc}")
    return p


class MfipmError(RuntimeError):
    def __init__(self, where, code):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({code})")
        self.code = code


def _check(where, rc):
    if rc != 0:
        raise MfipmError(where, rc)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclass
class Result:
    x: object            # torch tensor(s) on the device
    state: object        # (sum n) * 4 doubles
    infos: list          # list of dicts
    kernel_ms: float


class Solver:
    """A library handle bound to one device and the current torch stream."""

    def __init__(self, params: dict | None = None, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the mfIPM library needs a HIP device")
        self.torch = torch
        self.device = (torch.device("cuda", torch.cuda.current_device()) if device is None
                       else torch.device(device))
        self.lib = load_library()
        prm = default_params()
        for k, v in (params or {}).items():
            setattr(prm, k, v)
        self.params = prm
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check("mfipm_create", self.lib.mfipm_create(ctypes.byref(h), ctypes.byref(prm),
                                                         ctypes.c_void_p(self.stream.cuda_stream)))
        self.h = h
        _live.add(self)
        self._ws = None
        self._explicit = None  # launch shape fixed by the caller
        self.arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        self.num_cu = torch.cuda.get_device_properties(self.device).multi_processor_count

    def close(self):
        """Waits for the handle's stream, then releases the handle."""
        if getattr(self, "h", None):
            self.stream.synchronize()
            self.lib.mfipm_destroy(self.h)
            self.h = None
            self._ws = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the runtime may already be gone (and module
        # globals cleared); the exit handler above has closed every handle.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw):
        for k, v in kw.items():
            setattr(self.params, k, v)
        _check("mfipm_set_params", self.lib.mfipm_set_params(self.h, ctypes.byref(self.params)))

    def set_launch(self, workgroups=0, team_size=0, tile=0):
        """Fixes the launch shape for later calls; (0, 0, 0) returns to the
        tuned table (or the library's own choice when nothing is tuned)."""
        shape = (int(workgroups), int(team_size), int(tile))
        self._explicit = None if shape == (0, 0, 0) else shape
        _check("mfipm_set_launch", self.lib.mfipm_set_launch(self.h, *shape))

    def tune_key(self, op_kind, n_max, m_max, batch, shared, backward=False):
        from . import autotune
        # the DST rows run on the DCT kernel: they share its tuned shapes
        kind = OP_PDCT if op_kind == OP_PDST else op_kind
        return autotune.make_key(self.arch, kind, n_max, m_max, batch, shared, backward)

    def _apply_shape(self, op_kind, n_max, m_max, batch, shared, backward=False):
        from . import autotune
        shape = self._explicit
        if shape is None:
            shape = autotune.lookup(self.tune_key(op_kind, n_max, m_max, batch, shared, backward)) \
                or (0, 0, 0)
        _check("mfipm_set_launch", self.lib.mfipm_set_launch(self.h, *shape))
        return shape

    def last_kernel_ms(self) -> float:
        return float(self.lib.mfipm_last_kernel_ms(self.h))

    def workspace(self, op_kind, max_n, max_m, batch):
        nbytes = ctypes.c_size_t()
        _check("mfipm_workspace_size", self.lib.mfipm_workspace_size(self.h, op_kind, max_n, max_m, batch,
                                                                       ctypes.byref(nbytes)))
        if self._ws is None or self._ws.numel() < nbytes.value:
            self._ws = self.torch.empty(nbytes.value, dtype=self.torch.uint8, device=self.device)
        return self._ws, nbytes.value

    # -- single instance ------------------------------------------------------
    def solve(self, b, tau, A=None, rows=None, n=None, want_state=True, transform="dct") -> Result:
        """Solves min tau||x||_1 + 1/2||Ax-b||^2 with a dense A (m x n, float64,
        contiguous) or rows of a fast transform of length n (rows: int32 sorted
        distinct; transform "dct", "dst" or "wht")."""
        torch = self.torch
        b = _dev(b, self.device, torch.float64)
        if A is not None:
            A = _dev(A, self.device, torch.float64)
            m, n = A.shape
            op = Operator(OP_DENSE, m, n, A.data_ptr(), n, None)
            kind = OP_DENSE
        else:
            rows = _dev(rows, self.device, torch.int32)
            m = rows.shape[0]
            kind = _transform(transform)
            op = Operator(kind, m, int(n), None, 0, rows.data_ptr())
        if b.shape[0] != m:
            raise ValueError("b has the wrong length")
        x = torch.empty(int(op.n), dtype=torch.float64, device=self.device)
        state = torch.empty(4 * int(op.n), dtype=torch.float64, device=self.device) if want_state else None
        self._apply_shape(kind, int(op.n), m, 1, True)
        ws, nb = self.workspace(kind, int(op.n), m, 1)
        info = Info()
        rc = self.lib.mfipm_solve(self.h, ctypes.byref(op), _ptr(b), float(tau), _ptr(x), _ptr(state),
                                  _ptr(ws), nb, ctypes.byref(info))
        _check("mfipm_solve", rc)
        return Result(x=x, state=state, infos=[info.as_dict()], kernel_ms=self.last_kernel_ms())

    def solve_noalloc(self, b, tau, x, state=None, A=None, rows=None, n=None, transform="dct") -> dict:
        """mfipm_solve_noalloc: like `solve`, but the library uses its static
        per-device scratch instead of a workspace and allocates nothing; the
        caller passes device tensors for b, x (n) and optionally state (4n).
        Returns the report."""
        if A is not None:
            m, nn = A.shape
            op = Operator(OP_DENSE, m, nn, A.data_ptr(), nn, None)
        else:
            op = Operator(_transform(transform), rows.shape[0], int(n), None, 0, rows.data_ptr())
        if b.shape[0] != op.m or x.shape[0] != op.n or (state is not None and state.shape[0] != 4 * op.n):
            raise ValueError("b, x or state has the wrong length")
        for t in (b, x, state, A, rows):
            if t is not None and (t.device != self.device or not t.is_contiguous()):
                raise ValueError("tensors must be contiguous and on the solver's device")
        self._apply_shape(op.op, int(op.n), int(op.m), 1, True)
        info = Info()
        with self.torch.cuda.device(self.device):
            rc = self.lib.mfipm_solve_noalloc(self.h, ctypes.byref(op), _ptr(b), float(tau), _ptr(x), _ptr(state),
                                              ctypes.byref(info))
        _check("mfipm_solve_noalloc", rc)
        return info.as_dict()

    # -- batches ----------------------------------------------------------------
    def solve_batched(self, b_packed, tau, n_off, m_off, A_packed=None, a_off=None, rows=None,
                      shared_op=False, want_state=True, transform="dct") -> Result:
        torch = self.torch
        batch = len(n_off) - 1
        n_off = np.ascontiguousarray(n_off, dtype=np.int64)
        m_off = np.ascontiguousarray(m_off, dtype=np.int64)
        tau = np.ascontiguousarray(tau, dtype=np.float64)
        kind = OP_DENSE if A_packed is not None else _transform(transform)
        if kind == OP_DENSE and not shared_op:
            a_off = np.ascontiguousarray(a_off, dtype=np.int64)
        else:
            a_off = np.zeros(batch + 1, dtype=np.int64) if a_off is None else np.ascontiguousarray(a_off, np.int64)
        b_packed = _dev(b_packed, self.device, torch.float64)
        A_packed = _dev(A_packed, self.device, torch.float64) if A_packed is not None else None
        rows = _dev(rows, self.device, torch.int32) if rows is not None else None
        N = int(n_off[-1])
        x = torch.empty(N, dtype=torch.float64, device=self.device)
        state = torch.empty(4 * N, dtype=torch.float64, device=self.device) if want_state else None
        nmax, mmax = _max_sizes(n_off, m_off)
        self._apply_shape(kind, nmax, mmax, batch, shared_op)
        ws, nb = self.workspace(kind, nmax, mmax, batch)
        infos = (Info * batch)()
        rc = self.lib.mfipm_solve_batched(
            self.h, batch, n_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            m_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            a_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), kind, _ptr(A_packed), _ptr(rows),
            1 if shared_op else 0, _ptr(b_packed), tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            _ptr(x), _ptr(state), _ptr(ws), nb, infos)
        _check("mfipm_solve_batched", rc)
        return Result(x=x, state=state, infos=[i.as_dict() for i in infos], kernel_ms=self.last_kernel_ms())

    def backward(self, state, grad_x, n_off, m_off, A_packed=None, a_off=None, rows=None, shared_op=False,
                 transform="dct"):
        """Adjoint at `state`: returns (grad_b packed, grad_tau per instance, infos)."""
        torch = self.torch
        batch = len(n_off) - 1
        n_off = np.ascontiguousarray(n_off, dtype=np.int64)
        m_off = np.ascontiguousarray(m_off, dtype=np.int64)
        kind = OP_DENSE if A_packed is not None else _transform(transform)
        if kind == OP_DENSE and not shared_op:
            a_off = np.ascontiguousarray(a_off, dtype=np.int64)
        else:
            a_off = np.zeros(batch + 1, dtype=np.int64) if a_off is None else np.ascontiguousarray(a_off, np.int64)
        grad_x = _dev(grad_x, self.device, torch.float64)
        A_packed = _dev(A_packed, self.device, torch.float64) if A_packed is not None else None
        rows = _dev(rows, self.device, torch.int32) if rows is not None else None
        grad_b = torch.empty(int(m_off[-1]), dtype=torch.float64, device=self.device)
        grad_tau = torch.empty(batch, dtype=torch.float64, device=self.device)
        nmax, mmax = _max_sizes(n_off, m_off)
        self._apply_shape(kind, nmax, mmax, batch, shared_op, backward=True)
        ws, nb = self.workspace(kind, nmax, mmax, batch)
        infos = (Info * batch)()
        rc = self.lib.mfipm_backward(
            self.h, batch, n_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            m_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            a_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), kind, _ptr(A_packed), _ptr(rows),
            1 if shared_op else 0, _ptr(state), _ptr(grad_x), _ptr(grad_b), _ptr(grad_tau), _ptr(ws), nb, infos)
        _check("mfipm_backward", rc)
        return grad_b, grad_tau, [i.as_dict() for i in infos]


def _max_sizes(n_off, m_off):
    """Largest n and m of a batch (1, 1 for an empty one, which the library
    then rejects)."""
    ns = np.diff(n_off)
    ms = np.diff(m_off)
    return (int(ns.max()) if ns.size else 1), (int(ms.max()) if ms.size else 1)


def _transform(name):
    try:
        return TRANSFORMS[name]
    except KeyError:
        raise ValueError(f"unknown transform {name!r}; expected one of {sorted(TRANSFORMS)}") from None


def _dev(t, device, dtype):
    import torch
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    t = t.to(device=device, dtype=dtype)
    return t.contiguous()
