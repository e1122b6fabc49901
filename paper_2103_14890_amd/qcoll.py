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
# launch shapes chosen by the autotuner on the batch workloads (see tune.py)
DEFAULT_TUNING = os.path.join(_PKG, "tuning_gfx950.json")

MAXWELL, HARD_SPHERE, VHS = 0, 1, 2
FP32, MIX_FX16 = 1, 4
EXPLICIT_EULER, IMEX_EULER_PENALIZED, IMEX_ARS222, IMEX_BPR343 = 0, 1, 2, 3
CONSERVE, R_LITERAL, GALERKIN, CLASSICAL, SEPARABLE_MODES, HOST_ONLY = 0x1, 0x2, 0x4, 0x8, 0x10, 0x100
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ETOOLARGE = 0, -1, -2, -3, -4, -5
NOALLOC_SCRATCH_BYTES = 64 << 20

_KERNELS = {"maxwell": MAXWELL, "hard_sphere": HARD_SPHERE, "vhs": VHS}
_PRECISIONS = {"fp32": FP32, "fx16": MIX_FX16}
_SCHEMES = {"explicit": EXPLICIT_EULER, "imex": IMEX_EULER_PENALIZED}
_RK_SCHEMES = {"ars222": IMEX_ARS222, "bpr343": IMEX_BPR343}


class QcollError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2103_14890_amd.build`")
    # The device buffers and streams passed in come from PyTorch's HIP runtime,
    # so the library must bind to that same runtime instance: load torch (and
    # with it its libamdhip64) first, so that libqcoll's libamdhip64.so.7
    # dependency resolves to the copy already in the process instead of
    # bringing a second HIP/HSA runtime along.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.qcoll_plan.argtypes = [ctypes.POINTER(vp), c_int, c_int, dbl, c_int, dbl, c_int, c_int, c_int,
                               ctypes.c_uint]
    lib.qcoll_plan.restype = c_int
    lib.qcoll_plan_vhs.argtypes = [ctypes.POINTER(vp), c_int, dbl, dbl, dbl, c_int, c_int, c_int, ctypes.c_uint]
    lib.qcoll_plan_vhs.restype = c_int
    lib.qcoll_eval.argtypes = [vp, vp, vp, i64, vp]
    lib.qcoll_eval.restype = c_int
    lib.qcoll_step.argtypes = [vp, vp, i64, dbl, dbl, c_int, vp, vp]
    lib.qcoll_step.restype = c_int
    lib.qcoll_scratch_bytes.argtypes = [vp]
    lib.qcoll_scratch_bytes.restype = i64
    lib.qcoll_eval_ws.argtypes = [vp, vp, vp, i64, vp, i64, vp]
    lib.qcoll_eval_ws.restype = c_int
    lib.qcoll_step_ws.argtypes = [vp, vp, i64, dbl, dbl, c_int, vp, vp, i64, vp]
    lib.qcoll_step_ws.restype = c_int
    lib.qcoll_step_rk_work_bytes.argtypes = [vp, c_int, i64]
    lib.qcoll_step_rk_work_bytes.restype = i64
    lib.qcoll_step_rk.argtypes = [vp, vp, i64, dbl, dbl, c_int, vp, i64, vp, vp]
    lib.qcoll_step_rk.restype = c_int
    lib.qcoll_step_rk_noalloc.argtypes = [vp, vp, i64, dbl, dbl, c_int, vp, vp]
    lib.qcoll_step_rk_noalloc.restype = c_int
    lib.qcoll_galerkin_work_bytes.argtypes = [vp, i64]
    lib.qcoll_galerkin_work_bytes.restype = i64
    lib.qcoll_eval_galerkin.argtypes = [vp, vp, vp, i64, vp, i64, vp]
    lib.qcoll_eval_galerkin.restype = c_int
    lib.qcoll_plan_info.argtypes = [vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(dbl),
                                    ctypes.POINTER(i64)]
    lib.qcoll_plan_info.restype = c_int
    lib.qcoll_plan_table.argtypes = [vp, c_int, c_int, ctypes.POINTER(dbl), i64]
    lib.qcoll_plan_table.restype = c_int
    lib.qcoll_eval_multi.argtypes = [ctypes.POINTER(vp), c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                     ctypes.POINTER(i64), vp]
    lib.qcoll_eval_multi.restype = c_int
    lib.qcoll_step_multi.argtypes = [ctypes.POINTER(vp), c_int, ctypes.POINTER(vp), ctypes.POINTER(i64), dbl, dbl,
                                     c_int, ctypes.POINTER(vp), vp]
    lib.qcoll_step_multi.restype = c_int
    lib.qcoll_plan_set_launch.argtypes = [vp, c_int, i64]
    lib.qcoll_plan_set_launch.restype = c_int
    lib.qcoll_plan_get_launch.argtypes = [vp, ctypes.POINTER(c_int), ctypes.POINTER(i64)]
    lib.qcoll_plan_get_launch.restype = c_int
    lib.qcoll_plan_set_tile.argtypes = [vp, c_int]
    lib.qcoll_plan_set_tile.restype = c_int
    lib.qcoll_plan_get_tile.argtypes = [vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    lib.qcoll_plan_get_tile.restype = c_int
    lib.qcoll_plan_set_split.argtypes = [vp, c_int]
    lib.qcoll_plan_set_split.restype = c_int
    lib.qcoll_plan_get_split.argtypes = [vp, ctypes.POINTER(c_int)]
    lib.qcoll_plan_get_split.restype = c_int
    lib.qcoll_plan_autotune.argtypes = [vp, vp, vp, i64, c_int, vp]
    lib.qcoll_plan_autotune.restype = c_int
    lib.qcoll_plan_destroy.argtypes = [vp]
    lib.qcoll_plan_destroy.restype = None
    lib.qcoll_strerror.argtypes = [c_int]
    lib.qcoll_strerror.restype = ctypes.c_char_p
    pi64, pdbl = ctypes.POINTER(i64), ctypes.POINTER(dbl)
    lib.qcoll_transport_plan.argtypes = [ctypes.POINTER(vp), i64, pi64, pdbl, pi64, pdbl, pi64, pdbl, c_int, c_int,
                                         dbl, ctypes.c_uint]
    lib.qcoll_transport_plan.restype = c_int
    lib.qcoll_transport_work_bytes.argtypes = [vp]
    lib.qcoll_transport_work_bytes.restype = i64
    lib.qcoll_transport_rhs.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.qcoll_transport_rhs.restype = c_int
    lib.qcoll_transport_step.argtypes = [vp, vp, vp, dbl, vp, i64, vp]
    lib.qcoll_transport_step.restype = c_int
    lib.qcoll_transport_table.argtypes = [vp, c_int, i64, pdbl, i64]
    lib.qcoll_transport_table.restype = c_int
    lib.qcoll_transport_destroy.argtypes = [vp]
    lib.qcoll_transport_destroy.restype = None
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


def _alloc(shape, dtype, like, stream):
    """A device buffer for a call queued on `stream`. Buffers come from the
    caching allocator of the current stream; when the call runs on another
    stream the buffer is recorded on it, so that its memory is not handed out
    again before that stream's work on it has completed."""
    import torch
    t = torch.empty(shape, dtype=dtype, device=like.device)
    if stream is not None and stream != torch.cuda.current_stream(like.device):
        t.record_stream(stream)
    return t


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
                 host_only: bool = False, galerkin: bool = False, gamma: float = 1.0, classical: bool = False,
                 separable_modes: bool = False):
        flags = ((CONSERVE if conserve else 0) | (R_LITERAL if r_literal else 0) | (HOST_ONLY if host_only else 0)
                 | (GALERKIN if galerkin else 0) | (CLASSICAL if classical else 0)
                 | (SEPARABLE_MODES if separable_modes else 0))
        h = ctypes.c_void_p()
        if kernel == "vhs":
            if d != 2:
                raise ValueError("variable hard spheres are 2D")
            _check(LIB.qcoll_plan_vhs(ctypes.byref(h), N, float(L), float(gamma), float(b), M, K_r,
                                      _PRECISIONS[precision], flags), "qcoll_plan_vhs")
        else:
            _check(LIB.qcoll_plan(ctypes.byref(h), d, N, float(L), _KERNELS[kernel], float(b), M, K_r,
                                  _PRECISIONS[precision], flags), "qcoll_plan")
        self.gamma, self.classical = float(gamma), classical
        self._h = h
        self.d, self.N, self.L, self.kernel, self.M = d, N, float(L), kernel, M
        self.precision, self.conserve, self.galerkin = precision, conserve, galerkin

    def step_rk(self, f, dt: float, eps: float = 1.0, scheme: str = "ars222", status=None, work=None,
                stream=None):
        """One multi-stage penalised IMEX step of f in place (qcoll_step_rk);
        work is a float32 device tensor of at least work_bytes() bytes (allocated
        here when not given)."""
        import torch
        code = _RK_SCHEMES[scheme]
        need = int(LIB.qcoll_step_rk_work_bytes(self._h, code, f.shape[0]))
        if work is None:
            work = _alloc(max(need // 4, 1), torch.float32, f, stream)
        st = ctypes.c_void_p(0) if status is None else _dev_ptr(status, torch.int32, "status")
        _check(LIB.qcoll_step_rk(self._h, _dev_ptr(f, torch.float32, "f"), f.shape[0], float(dt), float(eps), code,
                                 _dev_ptr(work, torch.float32, "work"), work.numel() * 4, st,
                                 _stream_ptr(stream)), "qcoll_step_rk")
        return f

    def step_rk_noalloc(self, f, dt: float, eps: float = 1.0, scheme: str = "ars222", status=None, stream=None):
        """qcoll_step_rk_noalloc: the same step with the library's fixed device
        scratch as the work buffer (nothing allocated)."""
        import torch
        st = ctypes.c_void_p(0) if status is None else _dev_ptr(status, torch.int32, "status")
        _check(LIB.qcoll_step_rk_noalloc(self._h, _dev_ptr(f, torch.float32, "f"), f.shape[0], float(dt),
                                         float(eps), _RK_SCHEMES[scheme], st, _stream_ptr(stream)),
               "qcoll_step_rk_noalloc")
        return f

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
        grid = (3 * self.N // 2) ** self.d if self.galerkin else self.n   # Galerkin tables live on the 3N/2 grid
        cap = size if size is not None else max(grid, 64)
        out = np.zeros(cap, dtype=np.float64)
        cnt = _check(LIB.qcoll_plan_table(self._h, which, index, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          cap), "qcoll_plan_table")
        return out[:cnt].copy()

    def eval(self, f, q=None, stream=None):
        """Q_h(f) for a [cells, N, .., N] float32 device tensor."""
        import torch
        cells = f.shape[0]
        if q is None:
            q = _alloc(f.shape, torch.float64 if self.conserve else torch.float32, f, stream)
        _check(LIB.qcoll_eval(self._h, _dev_ptr(f, torch.float32, "f"),
                              _dev_ptr(q, torch.float64 if self.conserve else torch.float32, "Q"),
                              cells, _stream_ptr(stream)), "qcoll_eval")
        return q

    def scratch_bytes(self) -> int:
        """Bytes of one workgroup's scratch of a 3D plan (0 for 2D plans)."""
        return _check(int(LIB.qcoll_scratch_bytes(self._h)), "qcoll_scratch_bytes")

    def eval_ws(self, f, work, q=None, stream=None):
        """Q_h(f) with the caller's workspace (qcoll_eval_ws): calls on one 3D plan
        with distinct workspaces may run concurrently."""
        import torch
        if q is None:
            q = _alloc(f.shape, torch.float64 if self.conserve else torch.float32, f, stream)
        _check(LIB.qcoll_eval_ws(self._h, _dev_ptr(f, torch.float32, "f"),
                                 _dev_ptr(q, torch.float64 if self.conserve else torch.float32, "Q"), f.shape[0],
                                 _dev_ptr(work, work.dtype, "work"), work.numel() * work.element_size(),
                                 _stream_ptr(stream)), "qcoll_eval_ws")
        return q

    def step_ws(self, f, dt: float, work, eps: float = 1.0, scheme: str = "explicit", status=None, stream=None):
        """One homogeneous step of f in place with the caller's workspace (qcoll_step_ws)."""
        import torch
        st = ctypes.c_void_p(0) if status is None else _dev_ptr(status, torch.int32, "status")
        _check(LIB.qcoll_step_ws(self._h, _dev_ptr(f, torch.float32, "f"), f.shape[0], float(dt), float(eps),
                                 _SCHEMES[scheme], st, _dev_ptr(work, work.dtype, "work"),
                                 work.numel() * work.element_size(), _stream_ptr(stream)), "qcoll_step_ws")
        return f

    def galerkin_work_bytes(self, cells: int) -> int:
        return _check(int(LIB.qcoll_galerkin_work_bytes(self._h, int(cells))), "qcoll_galerkin_work_bytes")

    def eval_galerkin(self, f, q=None, work=None, stream=None):
        """Dealiased Q_h(f) of a Galerkin plan (qcoll_eval_galerkin); work is a
        device tensor of at least galerkin_work_bytes() bytes (allocated here
        when not given)."""
        import torch
        cells = f.shape[0]
        if q is None:
            q = _alloc(f.shape, torch.float64 if self.conserve else torch.float32, f, stream)
        need = self.galerkin_work_bytes(cells)
        if work is None:
            work = _alloc(max(need // 8, 1), torch.float64, f, stream)
        _check(LIB.qcoll_eval_galerkin(self._h, _dev_ptr(f, torch.float32, "f"),
                                       _dev_ptr(q, torch.float64 if self.conserve else torch.float32, "Q"), cells,
                                       _dev_ptr(work, work.dtype, "work"), work.numel() * work.element_size(),
                                       _stream_ptr(stream)), "qcoll_eval_galerkin")
        return q

    def step(self, f, dt: float, eps: float = 1.0, scheme: str = "explicit", status=None, stream=None):
        """One homogeneous step of f (in place)."""
        import torch
        st = ctypes.c_void_p(0) if status is None else _dev_ptr(status, torch.int32, "status")
        _check(LIB.qcoll_step(self._h, _dev_ptr(f, torch.float32, "f"), f.shape[0], float(dt), float(eps),
                              _SCHEMES[scheme], st, _stream_ptr(stream)), "qcoll_step")
        return f

    @property
    def key(self) -> str:
        """Identity of the plan's workload shape for the autotuning cache."""
        return (f"d{self.d}_N{self.N}_{self.kernel}_M{self.M}_{self.precision}_{'c' if self.conserve else 'n'}"
                + ("_galerkin" if self.galerkin else "") + ("_classical" if self.classical else "")
                + (f"_g{self.gamma}" if self.kernel == "vhs" else ""))

    def launch(self) -> tuple[int, int]:
        w, b = ctypes.c_int(), ctypes.c_int64()
        _check(LIB.qcoll_plan_get_launch(self._h, ctypes.byref(w), ctypes.byref(b)), "qcoll_plan_get_launch")
        return w.value, b.value

    def set_launch(self, waves_per_block: int, max_blocks: int) -> None:
        _check(LIB.qcoll_plan_set_launch(self._h, int(waves_per_block), int(max_blocks)), "qcoll_plan_set_launch")

    def tile(self) -> tuple[int, int]:
        """(selected tile family, alternate one or 0)."""
        t, a = ctypes.c_int(), ctypes.c_int()
        _check(LIB.qcoll_plan_get_tile(self._h, ctypes.byref(t), ctypes.byref(a)), "qcoll_plan_get_tile")
        return t.value, a.value

    def set_tile(self, tile: int) -> None:
        _check(LIB.qcoll_plan_set_tile(self._h, int(tile)), "qcoll_plan_set_tile")

    def split(self) -> int:
        """Transform split factor (see qcoll_plan_set_split)."""
        s = ctypes.c_int()
        _check(LIB.qcoll_plan_get_split(self._h, ctypes.byref(s)), "qcoll_plan_get_split")
        return s.value

    def set_split(self, split: int) -> None:
        _check(LIB.qcoll_plan_set_split(self._h, int(split)), "qcoll_plan_set_split")

    def shape(self) -> dict:
        """The launch shape the autotuner chooses among."""
        w, b = self.launch()
        return {"tile": self.tile()[0], "waves_per_block": w, "max_blocks": b}

    def apply_shape(self, shape: dict) -> None:
        if "tile" in shape:
            self.set_tile(shape["tile"])
        self.set_launch(shape["waves_per_block"], shape["max_blocks"])

    def autotune(self, f, reps: int = 3, cache: str | None = None, stream=None) -> dict:
        """Pick the fastest launch shape on f (see qcoll_plan_autotune) and store it
        in the JSON cache (path `cache`, or $QCOLL_TUNE_CACHE) under the plan key."""
        import torch
        q = _alloc(f.shape, torch.float64 if self.conserve else torch.float32, f, stream)
        _check(LIB.qcoll_plan_autotune(self._h, _dev_ptr(f, torch.float32, "f"), ctypes.c_void_p(q.data_ptr()),
                                       f.shape[0], int(reps), _stream_ptr(stream)), "qcoll_plan_autotune")
        best = self.shape()
        path = cache or os.environ.get("QCOLL_TUNE_CACHE")
        if path:
            import json
            data = json.load(open(path)) if os.path.exists(path) else {}
            data[self.key] = best
            tmp = path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(data, fh, indent=1, sort_keys=True)
            os.replace(tmp, path)
        return best

    def load_tuning(self, cache: str | None = None) -> bool:
        """Apply a cached launch shape for this plan's key, if any (cache path,
        else $QCOLL_TUNE_CACHE, else the shapes shipped with the package)."""
        import json
        path = cache or os.environ.get("QCOLL_TUNE_CACHE") or DEFAULT_TUNING
        if not path or not os.path.exists(path):
            return False
        ent = json.load(open(path)).get(self.key)
        if not ent:
            return False
        self.apply_shape(ent)
        return True

    def close(self):
        if getattr(self, "_h", None):
            LIB.qcoll_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_array(items):
    arr = (ctypes.c_void_p * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def eval_multi(plans, fs, qs, stream=None):
    """One launch over several plans (qcoll_eval_multi); fs, qs device tensors."""
    import torch
    n = len(plans)
    pl = _ptr_array([p._h.value for p in plans])
    fp = _ptr_array([_dev_ptr(f, torch.float32, "f").value for f in fs])
    qp = _ptr_array([_dev_ptr(q, torch.float64 if p.conserve else torch.float32, "Q").value
                     for p, q in zip(plans, qs)])
    cells = (ctypes.c_int64 * n)(*[f.shape[0] for f in fs])
    _check(LIB.qcoll_eval_multi(pl, n, fp, qp, cells, _stream_ptr(stream)), "qcoll_eval_multi")
    return qs


def step_multi(plans, fs, dt: float, eps: float = 1.0, scheme: str = "explicit", statuses=None, stream=None):
    """One stage update over several plans in one launch (qcoll_step_multi)."""
    import torch
    n = len(plans)
    pl = _ptr_array([p._h.value for p in plans])
    fp = _ptr_array([_dev_ptr(f, torch.float32, "f").value for f in fs])
    cells = (ctypes.c_int64 * n)(*[f.shape[0] for f in fs])
    st = None
    if statuses is not None:
        st = _ptr_array([0 if s is None else _dev_ptr(s, torch.int32, "status").value for s in statuses])
    _check(LIB.qcoll_step_multi(pl, n, fp, cells, float(dt), float(eps), _SCHEMES[scheme], st,
                                _stream_ptr(stream)), "qcoll_step_multi")
    return fs


class TransportPlan:
    """CWENO + Rusanov transport on a polygonal mesh (qcoll_transport_*): mesh is
    any object with the arrays cell_ptr, verts, nbr, shift, twin and gen."""

    def __init__(self, mesh, degree: int, N: int, L: float, host_only: bool = False):
        import numpy as np
        self._keep = [np.ascontiguousarray(a, dtype=t) for a, t in (
            (mesh.cell_ptr, np.int64), (mesh.verts, np.float64), (mesh.nbr, np.int64),
            (mesh.shift, np.float64), (mesh.twin, np.int64), (mesh.gen, np.float64))]
        cp, vt, nb, sh, tw, gn = self._keep
        P64, PD = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
        h = ctypes.c_void_p()
        _check(LIB.qcoll_transport_plan(ctypes.byref(h), len(gn), cp.ctypes.data_as(P64), vt.ctypes.data_as(PD),
                                        nb.ctypes.data_as(P64), sh.ctypes.data_as(PD), tw.ctypes.data_as(P64),
                                        gn.ctypes.data_as(PD), int(degree), int(N), float(L),
                                        HOST_ONLY if host_only else 0), "qcoll_transport_plan")
        self._h = h
        self.cells, self.degree, self.N, self.L = len(gn), degree, N, float(L)

    def work_bytes(self) -> int:
        return _check(int(LIB.qcoll_transport_work_bytes(self._h)), "qcoll_transport_work_bytes")

    def _work(self, work, like, stream):
        import torch
        if work is None:
            work = _alloc(max(self.work_bytes() // 4, 1), torch.float32, like, stream)
        return work

    def rhs(self, f, R=None, work=None, stream=None):
        """R = -(1/|P_i|) sum of the face fluxes, f and R float32 [cells, N, N]."""
        import torch
        if R is None:
            R = _alloc(f.shape, torch.float32, f, stream)
        work = self._work(work, f, stream)
        _check(LIB.qcoll_transport_rhs(self._h, _dev_ptr(f, torch.float32, "f"), _dev_ptr(R, torch.float32, "R"),
                                       _dev_ptr(work, work.dtype, "work"), work.numel() * work.element_size(),
                                       _stream_ptr(stream)), "qcoll_transport_rhs")
        return R

    def step(self, f, dt: float, out=None, work=None, stream=None):
        """out = f + dt R(f) (explicit Euler transport step)."""
        import torch
        if out is None:
            out = _alloc(f.shape, torch.float32, f, stream)
        work = self._work(work, f, stream)
        _check(LIB.qcoll_transport_step(self._h, _dev_ptr(f, torch.float32, "f"), _dev_ptr(out, torch.float32, "out"),
                                        float(dt), _dev_ptr(work, work.dtype, "work"),
                                        work.numel() * work.element_size(), _stream_ptr(stream)),
               "qcoll_transport_step")
        return out

    def table(self, which: int, cell: int, size: int = 256):
        import numpy as np
        out = np.zeros(size, dtype=np.float64)
        cnt = _check(LIB.qcoll_transport_table(self._h, which, int(cell),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), size),
                     "qcoll_transport_table")
        return out[:cnt].copy()

    def close(self):
        if getattr(self, "_h", None):
            LIB.qcoll_transport_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
