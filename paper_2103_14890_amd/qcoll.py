"""ctypes binding of libqcoll.so (argument marshalling only).

Every step of the collision operator runs in the HIP library; this module
only passes device pointers, sizes and a stream. PyTorch tensors are used as
device buffers. There is no fallback: if the library is not built, importing
the binding raises.
"""

from __future__ import annotations

import ctypes
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqcoll.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "qcoll.h")

MAXWELL, HARD_SPHERE = 0, 1
FP32, MIX_FX16 = 1, 4
EXPLICIT_EULER, IMEX_EULER_PENALIZED = 0, 1
CONSERVE, R_LITERAL, HOST_ONLY = 0x1, 0x2, 0x100
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4

_KERNELS = {"maxwell": MAXWELL, "hard_sphere": HARD_SPHERE}
_PRECISIONS = {"fp32": FP32, "fx16": MIX_FX16}
_SCHEMES = {"explicit": EXPLICIT_EULER, "imex": IMEX_EULER_PENALIZED}


class QcollError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2103_14890_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.qcoll_plan.argtypes = [ctypes.POINTER(vp), c_int, c_int, dbl, c_int, dbl, c_int, c_int, c_int,
                               ctypes.c_uint]
    lib.qcoll_plan.restype = c_int
    lib.qcoll_eval.argtypes = [vp, vp, vp, i64, vp]
    lib.qcoll_eval.restype = c_int
    lib.qcoll_step.argtypes = [vp, vp, i64, dbl, dbl, c_int, vp, vp]
    lib.qcoll_step.restype = c_int
    lib.qcoll_plan_info.argtypes = [vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(dbl),
                                    ctypes.POINTER(i64)]
    lib.qcoll_plan_info.restype = c_int
    lib.qcoll_plan_table.argtypes = [vp, c_int, c_int, ctypes.POINTER(dbl), i64]
    lib.qcoll_plan_table.restype = c_int
    lib.qcoll_plan_destroy.argtypes = [vp]
    lib.qcoll_plan_destroy.restype = None
    lib.qcoll_strerror.argtypes = [c_int]
    lib.qcoll_strerror.restype = ctypes.c_char_p
    return lib


LIB = _load()


def strerror(code: int) -> str:
    return LIB.qcoll_strerror(int(code)).decode()


def header_symbols() -> list[str]:
    """Names of the functions declared in include/qcoll.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(qcoll_\w+)\s*\(", text)))


def _check(code: int, what: str) -> int:
    if code < 0:
        raise QcollError(code, what)
    return code


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Plan of Q_h for one velocity grid and kernel (see include/qcoll.h)."""

    def __init__(self, d: int, N: int, L: float, kernel: str = "hard_sphere", M: int = 8, b: float = 0.0,
                 K_r: int = 0, precision: str = "fx16", conserve: bool = False, r_literal: bool = False,
                 host_only: bool = False):
        flags = (CONSERVE if conserve else 0) | (R_LITERAL if r_literal else 0) | (HOST_ONLY if host_only else 0)
        h = ctypes.c_void_p()
        _check(LIB.qcoll_plan(ctypes.byref(h), d, N, float(L), _KERNELS[kernel], float(b), M, K_r,
                              _PRECISIONS[precision], flags), "qcoll_plan")
        self._h = h
        self.d, self.N, self.L, self.kernel, self.M = d, N, float(L), kernel, M
        self.precision, self.conserve = precision, conserve

    @property
    def n(self) -> int:
        return self.N ** self.d

    def info(self) -> dict:
        t, k = ctypes.c_int(), ctypes.c_int()
        r, nb = ctypes.c_double(), ctypes.c_int64()
        _check(LIB.qcoll_plan_info(self._h, ctypes.byref(t), ctypes.byref(k), ctypes.byref(r), ctypes.byref(nb)),
               "qcoll_plan_info")
        return {"transforms": t.value, "K_r": k.value, "R": r.value, "device_bytes": nb.value}

    def table(self, which: int, index: int = 0, size: int | None = None):
        import numpy as np
        cap = size if size is not None else max(self.n, 64)
        out = np.zeros(cap, dtype=np.float64)
        cnt = _check(LIB.qcoll_plan_table(self._h, which, index, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          cap), "qcoll_plan_table")
        return out[:cnt].copy()

    def eval(self, f, q=None, stream=None):
        """Q_h(f) for a [cells, N, .., N] float32 device tensor."""
        import torch
        cells = f.shape[0]
        if q is None:
            q = torch.empty(f.shape, dtype=torch.float64 if self.conserve else torch.float32, device=f.device)
        _check(LIB.qcoll_eval(self._h, _dev_ptr(f, torch.float32, "f"),
                              _dev_ptr(q, torch.float64 if self.conserve else torch.float32, "Q"),
                              cells, _stream_ptr(stream)), "qcoll_eval")
        return q

    def step(self, f, dt: float, eps: float = 1.0, scheme: str = "explicit", status=None, stream=None):
        """One homogeneous step of f (in place)."""
        import torch
        st = ctypes.c_void_p(0) if status is None else _dev_ptr(status, torch.int32, "status")
        _check(LIB.qcoll_step(self._h, _dev_ptr(f, torch.float32, "f"), f.shape[0], float(dt), float(eps),
                              _SCHEMES[scheme], st, _stream_ptr(stream)), "qcoll_step")
        return f

    def close(self):
        if getattr(self, "_h", None):
            LIB.qcoll_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
