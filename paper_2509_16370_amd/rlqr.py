"""Thin Python binding of the rlqr C ABI (include/rlqr.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
librlqr.so. torch tensors provide device memory and the stream. The functions
rlqr_create, rlqr_create_tuned, rlqr_get_tuning, rlqr_factor, rlqr_factor_rhs,
rlqr_solve, rlqr_solve_multi, rlqr_pivot_inertia, rlqr_precision_path,
rlqr_residual, rlqr_residual_noalloc and rlqr_destroy carry the C names; `Solver` wraps one handle. The cross-stage
calls of include/rlqr_xs.h (rlqr_xs_*) are wrapped by `CrossStage`, the
general-SPD calls of include/rlqr_spd.h (rlqr_spd_*) by `SpdRegularized`.

If librlqr.so is missing this module raises at import: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librlqr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "(the solver has no CPU fallback)")

# torch first: its HIP runtime is loaded under the name libamdhip64.so, which
# does not match the SONAME (libamdhip64.so.7) of a runtime loaded earlier
# through this library's dependency, so the opposite order puts two HIP
# runtimes in the process (device pointers of one are foreign to the other).
# Loaded in this order, the library binds to torch's runtime.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

RLQR_OK, RLQR_E_INVALID, RLQR_E_NOMEM, RLQR_E_HIP, RLQR_E_STATE, RLQR_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
RLQR_SEQ_FP64, RLQR_SEQ_MIXED, RLQR_SCAN_FP32, RLQR_SCAN_BF16 = 0, 1, 2, 3
INST_OK, INST_NOT_PD, INST_SINGULAR, INST_NOT_CONVERGED, INST_NONFINITE = 0, 1, 2, 3, 4
PATH_FP32, PATH_FP64, PATH_FP64_GUARD, PATH_FP64_REDO = 0, 1, 2, 3
ARRAYS = ("Q", "M", "R", "A", "B", "q", "r", "c", "x", "u", "y", "res")
MODES = {"fp64": RLQR_SEQ_FP64, "mixed": RLQR_SEQ_MIXED, "scan": RLQR_SCAN_FP32, "scan_bf16": RLQR_SCAN_BF16}

_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)


class _Shape(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("N", _i32p), ("nx", _i32p), ("nu", _i32p)]


class _Lhs(ctypes.Structure):
    _fields_ = [(k, _vp) for k in ("Q", "M", "R", "A", "B", "delta", "delta_diag")]


class _Rhs(ctypes.Structure):
    _fields_ = [(k, _vp) for k in ("q", "r", "c")]


class _Sol(ctypes.Structure):
    _fields_ = [(k, _vp) for k in ("x", "u", "y")]


class _Tuning(ctypes.Structure):
    _fields_ = [("scan_chunk", ctypes.c_int32), ("inst_chunk", _i32p), ("inst_fp64", _i32p),
                ("max_rhs", ctypes.c_int32), ("scan_carry_pc", ctypes.c_int32), ("mw_waves", ctypes.c_int32)]


_lib.rlqr_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_Shape), ctypes.c_int,
                             ctypes.POINTER(ctypes.c_size_t)]
_lib.rlqr_create_tuned.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_Shape), ctypes.c_int,
                                   ctypes.POINTER(_Tuning), ctypes.POINTER(ctypes.c_size_t)]
_lib.rlqr_get_tuning.argtypes = [_vp, ctypes.POINTER(_Tuning)]
_lib.rlqr_graph_capture.argtypes = [_vp, ctypes.POINTER(_Lhs), ctypes.POINTER(_Rhs), ctypes.POINTER(_Sol),
                                    ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp]
_lib.rlqr_graph_launch.argtypes = [_vp, _vp]
_lib.rlqr_layout_offsets.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
_lib.rlqr_factor.argtypes = [_vp, ctypes.POINTER(_Lhs), _vp]
_lib.rlqr_factor_rhs.argtypes = [_vp, ctypes.POINTER(_Lhs), ctypes.POINTER(_Rhs), _vp]
_lib.rlqr_solve.argtypes = [_vp, ctypes.POINTER(_Rhs), ctypes.POINTER(_Sol), ctypes.c_double,
                            ctypes.c_int32, _vp, _vp, _vp]
_lib.rlqr_solve_multi.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(_Rhs), ctypes.POINTER(_Sol), ctypes.c_double,
                                  ctypes.c_int32, _vp, _vp, _vp]
_lib.rlqr_pivot_inertia.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.rlqr_precision_path.argtypes = [_vp, _vp, _vp]
_lib.rlqr_set_skip.argtypes = [_vp, _vp]
_lib.rlqr_residual.argtypes = [_vp, ctypes.POINTER(_Rhs), ctypes.POINTER(_Sol), _vp, _vp, _vp]
_lib.rlqr_residual_noalloc.argtypes = [ctypes.POINTER(_Shape), ctypes.POINTER(_Lhs), ctypes.POINTER(_Rhs),
                                       ctypes.POINTER(_Sol), _vp, _vp, _vp]
_lib.rlqr_destroy.argtypes = [_vp]
_lib.rlqr_destroy.restype = None
_lib.rlqr_status_string.argtypes = [ctypes.c_int]
_lib.rlqr_status_string.restype = ctypes.c_char_p
for _f in ("rlqr_create", "rlqr_create_tuned", "rlqr_get_tuning", "rlqr_layout_offsets", "rlqr_factor",
           "rlqr_factor_rhs", "rlqr_solve", "rlqr_solve_multi", "rlqr_pivot_inertia", "rlqr_residual", "rlqr_graph_capture", "rlqr_graph_launch",
           "rlqr_set_skip", "rlqr_precision_path", "rlqr_residual_noalloc"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("rlqr_create", "rlqr_create_tuned", "rlqr_get_tuning", "rlqr_layout_offsets", "rlqr_factor",
            "rlqr_factor_rhs", "rlqr_solve", "rlqr_solve_multi", "rlqr_pivot_inertia", "rlqr_residual", "rlqr_graph_capture", "rlqr_graph_launch",
            "rlqr_set_skip", "rlqr_precision_path", "rlqr_residual_noalloc",
            "rlqr_destroy", "rlqr_status_string")


class RlqrError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {_lib.rlqr_status_string(code).decode()} ({code})")
        self.code = code


def _check(code: int, where: str):
    if code != RLQR_OK:
        raise RlqrError(code, where)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


# ------------------------------------------------------------- C-named calls

def _shape(N, nx, nu):
    arrs = [np.ascontiguousarray(a, dtype=np.int32) for a in (N, nx, nu)]
    shape = _Shape(len(arrs[0]), *(a.ctypes.data_as(_i32p) for a in arrs))
    return shape, arrs  # keep the arrays alive for the call


def rlqr_create(N: Sequence[int], nx: Sequence[int], nu: Sequence[int], mode: int):
    """Returns (handle, workspace_bytes)."""
    shape, _keep = _shape(N, nx, nu)
    h = _vp()
    ws = ctypes.c_size_t(0)
    _check(_lib.rlqr_create(ctypes.byref(h), ctypes.byref(shape), int(mode), ctypes.byref(ws)), "rlqr_create")
    return h, int(ws.value)


def rlqr_create_tuned(N, nx, nu, mode: int, scan_chunk: int = 0, inst_chunk=None, inst_fp64=None, max_rhs: int = 0,
                      scan_carry_pc: bool = False, mw_waves: int = 0):
    """Returns (handle, workspace_bytes). inst_chunk / inst_fp64: optional per-instance arrays."""
    shape, _keep = _shape(N, nx, nu)
    h = _vp()
    ws = ctypes.c_size_t(0)
    ic = None if inst_chunk is None else np.ascontiguousarray(inst_chunk, dtype=np.int32)
    i64 = None if inst_fp64 is None else np.ascontiguousarray(inst_fp64, dtype=np.int32)
    t = _Tuning(int(scan_chunk), ic.ctypes.data_as(_i32p) if ic is not None else None,
                i64.ctypes.data_as(_i32p) if i64 is not None else None, int(max_rhs), int(bool(scan_carry_pc)),
                int(mw_waves))
    _check(_lib.rlqr_create_tuned(ctypes.byref(h), ctypes.byref(shape), int(mode), ctypes.byref(t),
                                  ctypes.byref(ws)), "rlqr_create_tuned")
    return h, int(ws.value)


def rlqr_get_tuning(h) -> Dict[str, int]:
    t = _Tuning(0)
    _check(_lib.rlqr_get_tuning(h, ctypes.byref(t)), "rlqr_get_tuning")
    return {"scan_chunk": int(t.scan_chunk), "max_rhs": int(t.max_rhs), "scan_carry_pc": int(t.scan_carry_pc),
            "mw_waves": int(t.mw_waves)}


def rlqr_layout_offsets(h, array: int, batch: int) -> np.ndarray:
    off = np.zeros(batch + 1, dtype=np.int64)
    _check(_lib.rlqr_layout_offsets(h, int(array), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
           "rlqr_layout_offsets")
    return off


def rlqr_factor(h, Q, M, R, A, B, delta, stream=None, delta_diag=None):
    lhs = _Lhs(*[_ptr(t) for t in (Q, M, R, A, B, delta, delta_diag)])
    _check(_lib.rlqr_factor(h, ctypes.byref(lhs), _stream(stream)), "rlqr_factor")


def rlqr_factor_rhs(h, Q, M, R, A, B, delta, q, r, c, stream=None, delta_diag=None):
    lhs = _Lhs(*[_ptr(t) for t in (Q, M, R, A, B, delta, delta_diag)])
    rhs = _Rhs(_ptr(q), _ptr(r), _ptr(c))
    _check(_lib.rlqr_factor_rhs(h, ctypes.byref(lhs), ctypes.byref(rhs), _stream(stream)), "rlqr_factor_rhs")


def rlqr_solve(h, q, r, c, x, u, y, rel_tol, max_refine, inst_status=None, inst_relres=None, stream=None):
    rhs = _Rhs(_ptr(q), _ptr(r), _ptr(c))
    sol = _Sol(_ptr(x), _ptr(u), _ptr(y))
    _check(_lib.rlqr_solve(h, ctypes.byref(rhs), ctypes.byref(sol), float(rel_tol), int(max_refine),
                           _ptr(inst_status), _ptr(inst_relres), _stream(stream)), "rlqr_solve")


def rlqr_solve_multi(h, nrhs, q, r, c, x, u, y, rel_tol, max_refine, inst_status=None, inst_relres=None,
                     stream=None):
    rhs = _Rhs(_ptr(q), _ptr(r), _ptr(c))
    sol = _Sol(_ptr(x), _ptr(u), _ptr(y))
    _check(_lib.rlqr_solve_multi(h, int(nrhs), ctypes.byref(rhs), ctypes.byref(sol), float(rel_tol),
                                 int(max_refine), _ptr(inst_status), _ptr(inst_relres), _stream(stream)),
           "rlqr_solve_multi")


def rlqr_set_skip(h, skip=None):
    _check(_lib.rlqr_set_skip(h, _ptr(skip)), "rlqr_set_skip")


def rlqr_pivot_inertia(h, verdict=None, first_bad=None, inertia=None, stream=None):
    _check(_lib.rlqr_pivot_inertia(h, _ptr(verdict), _ptr(first_bad), _ptr(inertia), _stream(stream)),
           "rlqr_pivot_inertia")


def rlqr_precision_path(h, path, stream=None):
    _check(_lib.rlqr_precision_path(h, _ptr(path), _stream(stream)), "rlqr_precision_path")


def rlqr_residual(h, q, r, c, x, u, y, res=None, inst_relres=None, stream=None):
    rhs = _Rhs(_ptr(q), _ptr(r), _ptr(c))
    sol = _Sol(_ptr(x), _ptr(u), _ptr(y))
    _check(_lib.rlqr_residual(h, ctypes.byref(rhs), ctypes.byref(sol), _ptr(res), _ptr(inst_relres),
                              _stream(stream)), "rlqr_residual")


def rlqr_residual_noalloc(N, nx, nu, Q, M, R, A, B, delta, q, r, c, x, u, y, res=None, inst_relres=None,
                          stream=None, delta_diag=None):
    """rlqr_residual without a handle (no device allocation; see include/rlqr.h)."""
    shape, _keep = _shape(N, nx, nu)
    lhs = _Lhs(_ptr(Q), _ptr(M), _ptr(R), _ptr(A), _ptr(B), _ptr(delta), _ptr(delta_diag))
    rhs = _Rhs(_ptr(q), _ptr(r), _ptr(c))
    sol = _Sol(_ptr(x), _ptr(u), _ptr(y))
    _check(_lib.rlqr_residual_noalloc(ctypes.byref(shape), ctypes.byref(lhs), ctypes.byref(rhs), ctypes.byref(sol),
                                      _ptr(res), _ptr(inst_relres), _stream(stream)), "rlqr_residual_noalloc")


def rlqr_graph_capture(h, Q, M, R, A, B, delta, q, r, c, x, u, y, rel_tol, max_refine,
                       inst_status=None, inst_relres=None, stream=None, delta_diag=None):
    lhs = _Lhs(*[_ptr(t) for t in (Q, M, R, A, B, delta, delta_diag)])
    rhs = _Rhs(_ptr(q), _ptr(r), _ptr(c))
    sol = _Sol(_ptr(x), _ptr(u), _ptr(y))
    _check(_lib.rlqr_graph_capture(h, ctypes.byref(lhs), ctypes.byref(rhs), ctypes.byref(sol), float(rel_tol),
                                   int(max_refine), _ptr(inst_status), _ptr(inst_relres), _stream(stream)),
           "rlqr_graph_capture")


def rlqr_graph_launch(h, stream=None):
    _check(_lib.rlqr_graph_launch(h, _stream(stream)), "rlqr_graph_launch")


def rlqr_destroy(h):
    _lib.rlqr_destroy(h)


# ------------------------------------------------------------- convenience

class Solver:
    """One handle over a fixed batch of shapes; tensors are torch CUDA float64."""

    def __init__(self, N, nx, nu, mode: str = "fp64", device: str = "cuda:0", scan_chunk: int = 0,
                 inst_chunk=None, inst_fp64=None, max_rhs: int = 0, scan_carry_pc: bool = False, mw_waves: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.N = np.asarray(N, dtype=np.int32)
        self.nx = np.asarray(nx, dtype=np.int32)
        self.nu = np.asarray(nu, dtype=np.int32)
        self.batch = int(self.N.shape[0])
        self.mode = mode
        with torch.cuda.device(self.device):
            self.handle, self.workspace_bytes = rlqr_create_tuned(self.N, self.nx, self.nu, MODES[mode],
                                                                  scan_chunk, inst_chunk, inst_fp64, max_rhs,
                                                                  scan_carry_pc, mw_waves)
        self.tuning = rlqr_get_tuning(self.handle)
        self.offsets = {name: rlqr_layout_offsets(self.handle, i, self.batch) for i, name in enumerate(ARRAYS)}
        self._lhs = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            try:
                _lib.rlqr_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None

    def size(self, name: str) -> int:
        return int(self.offsets[name][-1])

    def empty(self, name: str):
        return self.torch.empty(max(self.size(name), 1), dtype=self.torch.float64, device=self.device)

    def factor(self, lhs: Dict[str, "torch.Tensor"], rhs: Optional[Dict[str, "torch.Tensor"]] = None, stream=None):
        """rlqr_factor, or rlqr_factor_rhs when the next solve's rhs is given."""
        for k in ("Q", "M", "R", "A", "B"):
            t = lhs[k]
            assert t.dtype == self.torch.float64 and t.is_cuda and t.is_contiguous() and t.numel() >= self.size(k), k
        assert lhs["delta"].numel() >= self.batch and lhs["delta"].dtype == self.torch.float64
        dd = lhs.get("delta_diag")
        if dd is not None:  # per-stage diagonal Delta_i, laid out like x
            assert dd.dtype == self.torch.float64 and dd.is_cuda and dd.is_contiguous() and \
                dd.numel() >= self.size("x")
        self._lhs = lhs  # the library re-reads the lhs during refinement: keep it alive
        args = [lhs[k] for k in ("Q", "M", "R", "A", "B", "delta")]
        if rhs is None:
            rlqr_factor(self.handle, *args, stream=stream, delta_diag=dd)
            return
        for k in ("q", "r", "c"):
            t = rhs[k]
            assert t.dtype == self.torch.float64 and t.is_cuda and t.is_contiguous() and t.numel() >= self.size(k), k
        self._rhs = rhs
        rlqr_factor_rhs(self.handle, *args, rhs["q"], rhs["r"], rhs["c"], stream=stream, delta_diag=dd)

    def solve(self, rhs, out=None, rel_tol: float = 1e-8, max_refine: int = 0, stream=None):
        torch = self.torch
        for k in ("q", "r", "c"):
            t = rhs[k]
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and t.numel() >= self.size(k), k
        if out is None:
            out = {k: self.empty(k) for k in ("x", "u", "y")}
        status = torch.empty(max(self.batch, 1), dtype=torch.int32, device=self.device)
        relres = torch.empty(max(self.batch, 1), dtype=torch.float64, device=self.device)
        rlqr_solve(self.handle, rhs["q"], rhs["r"], rhs["c"], out["x"], out["u"], out["y"],
                   rel_tol, max_refine, status, relres, stream=stream)
        return out, status, relres

    def solve_multi(self, nrhs: int, rhs, out=None, rel_tol: float = 1e-8, max_refine: int = 0, stream=None):
        """rlqr_solve_multi: rhs[k] holds nrhs stacked vectors of the batch length of k."""
        torch = self.torch
        for k in ("q", "r", "c"):
            t = rhs[k]
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and \
                t.numel() >= nrhs * self.size(k), k
        if out is None:
            out = {k: torch.empty(max(nrhs * self.size(k), 1), dtype=torch.float64, device=self.device)
                   for k in ("x", "u", "y")}
        status = torch.empty(max(nrhs * self.batch, 1), dtype=torch.int32, device=self.device)
        relres = torch.empty(max(nrhs * self.batch, 1), dtype=torch.float64, device=self.device)
        rlqr_solve_multi(self.handle, nrhs, rhs["q"], rhs["r"], rhs["c"], out["x"], out["u"], out["y"],
                         rel_tol, max_refine, status, relres, stream=stream)
        return out, status, relres

    def capture(self, lhs, rhs, out, rel_tol: float = 1e-8, max_refine: int = 0, stream=None):
        """Capture factor + solve on `stream` (a torch.cuda.Stream, not the default
        stream) into the handle's graph; returns (status, relres) tensors that each
        replay refreshes."""
        torch = self.torch
        self._lhs = lhs
        self._graph_args = (lhs, rhs, out)
        status = torch.empty(max(self.batch, 1), dtype=torch.int32, device=self.device)
        relres = torch.empty(max(self.batch, 1), dtype=torch.float64, device=self.device)
        self._graph_out = (status, relres)
        rlqr_graph_capture(self.handle, *(lhs[k] for k in ("Q", "M", "R", "A", "B", "delta")),
                           rhs["q"], rhs["r"], rhs["c"], out["x"], out["u"], out["y"], rel_tol, max_refine,
                           status, relres, stream=stream, delta_diag=lhs.get("delta_diag"))
        return status, relres

    def replay(self, stream=None):
        rlqr_graph_launch(self.handle, stream=stream)

    def set_skip(self, skip=None):
        """rlqr_set_skip: int32 device tensor [B] (nonzero = leave out), or None."""
        if skip is not None:
            assert skip.dtype == self.torch.int32 and skip.is_cuda and skip.numel() >= self.batch
        self._skip = skip  # read by later calls: keep it alive
        rlqr_set_skip(self.handle, skip)

    def pivot_inertia(self, stream=None):
        torch = self.torch
        verdict = torch.empty(max(self.batch, 1), dtype=torch.int32, device=self.device)
        first_bad = torch.empty(max(self.batch, 1), dtype=torch.int32, device=self.device)
        inertia = torch.empty(max(3 * self.batch, 1), dtype=torch.int64, device=self.device)
        rlqr_pivot_inertia(self.handle, verdict, first_bad, inertia, stream=stream)
        return verdict, first_bad, inertia.view(-1, 3) if self.batch else inertia

    def precision_path(self, stream=None):
        """rlqr_precision_path: int32 device tensor [B] of PATH_* values."""
        path = self.torch.empty(max(self.batch, 1), dtype=self.torch.int32, device=self.device)
        rlqr_precision_path(self.handle, path, stream=stream)
        return path

    def residual(self, rhs, sol, stream=None):
        torch = self.torch
        res = self.empty("res")
        relres = torch.empty(max(self.batch, 1), dtype=torch.float64, device=self.device)
        rlqr_residual(self.handle, rhs["q"], rhs["r"], rhs["c"], sol["x"], sol["u"], sol["y"],
                      res, relres, stream=stream)
        return res, relres


def to_device(packed, device="cuda:0"):
    """Copy a workloads.Packed batch to device tensors (lhs, rhs dicts)."""
    import torch
    dev = torch.device(device)

    def t(a):  # never hand the library a NULL pointer for an empty array
        a = np.ascontiguousarray(a, dtype=np.float64)
        return torch.from_numpy(a if a.size else np.zeros(1)).to(dev)
    lhs = {k: t(packed.arrays[k]) for k in ("Q", "M", "R", "A", "B")}
    lhs["delta"] = t(packed.delta)
    if "delta_diag" in packed.arrays:
        lhs["delta_diag"] = t(packed.arrays["delta_diag"])
    if "delta_full" in packed.arrays:  # full SPD Delta_i (SpdRegularized), laid out like Q
        lhs["delta_full"] = t(packed.arrays["delta_full"])
    rhs = {k: t(packed.arrays[k]) for k in ("q", "r", "c")}
    return lhs, rhs


# ------------------------------------------------------------- general SPD Delta_i (include/rlqr_spd.h)

_lib.rlqr_spd_create.argtypes = [ctypes.POINTER(_vp), _vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.rlqr_spd_factor.argtypes = [_vp, ctypes.POINTER(_Lhs), _vp, _vp]
_lib.rlqr_spd_solve.argtypes = [_vp, ctypes.POINTER(_Rhs), ctypes.POINTER(_Sol), ctypes.c_double, ctypes.c_int32,
                                _vp, _vp, _vp]
_lib.rlqr_spd_residual.argtypes = [_vp, ctypes.POINTER(_Rhs), ctypes.POINTER(_Sol), _vp, _vp, _vp]
_lib.rlqr_spd_destroy.argtypes = [_vp]
_lib.rlqr_spd_destroy.restype = None
for _f in ("rlqr_spd_create", "rlqr_spd_factor", "rlqr_spd_solve", "rlqr_spd_residual"):
    getattr(_lib, _f).restype = ctypes.c_int
SPD_EXPORTED = ("rlqr_spd_create", "rlqr_spd_factor", "rlqr_spd_solve", "rlqr_spd_residual", "rlqr_spd_destroy")


class SpdRegularized:
    """rlqr_spd context over a Solver's handle: every Delta_i a full SPD
    matrix (laid out like Q), solved through the handle's mode."""

    def __init__(self, solver: "Solver"):
        self.solver = solver
        self.torch = solver.torch
        ctx = _vp()
        ws = ctypes.c_size_t(0)
        with self.torch.cuda.device(solver.device):
            _check(_lib.rlqr_spd_create(ctypes.byref(ctx), solver.handle, ctypes.byref(ws)), "rlqr_spd_create")
        self.ctx, self.workspace_bytes = ctx, int(ws.value)
        self._keep = None

    def __del__(self):
        x = getattr(self, "ctx", None)
        if x is not None and x.value and _lib is not None:
            try:
                _lib.rlqr_spd_destroy(x)
            except Exception:  # interpreter shutdown
                pass
            self.ctx = None

    def factor(self, lhs, Delta, stream=None):
        self._keep = (lhs, Delta)  # re-read by solve and residual
        L = _Lhs(*[_ptr(lhs.get(k)) for k in ("Q", "M", "R", "A", "B")], None, None)
        _check(_lib.rlqr_spd_factor(self.ctx, ctypes.byref(L), _ptr(Delta), _stream(stream)), "rlqr_spd_factor")

    def solve(self, rhs, out=None, rel_tol: float = 1e-8, max_refine: int = 3, stream=None):
        torch = self.torch
        s = self.solver
        if out is None:
            out = {k: s.empty(k) for k in ("x", "u", "y")}
        status = torch.empty(max(s.batch, 1), dtype=torch.int32, device=s.device)
        relres = torch.empty(max(s.batch, 1), dtype=torch.float64, device=s.device)
        R = _Rhs(_ptr(rhs["q"]), _ptr(rhs["r"]), _ptr(rhs["c"]))
        S = _Sol(_ptr(out["x"]), _ptr(out["u"]), _ptr(out["y"]))
        _check(_lib.rlqr_spd_solve(self.ctx, ctypes.byref(R), ctypes.byref(S), float(rel_tol), int(max_refine),
                                   _ptr(status), _ptr(relres), _stream(stream)), "rlqr_spd_solve")
        return out, status, relres

    def residual(self, rhs, sol, stream=None):
        torch = self.torch
        s = self.solver
        res = s.empty("res")
        relres = torch.empty(max(s.batch, 1), dtype=torch.float64, device=s.device)
        R = _Rhs(_ptr(rhs["q"]), _ptr(rhs["r"]), _ptr(rhs["c"]))
        S = _Sol(_ptr(sol["x"]), _ptr(sol["u"]), _ptr(sol["y"]))
        _check(_lib.rlqr_spd_residual(self.ctx, ctypes.byref(R), ctypes.byref(S), _ptr(res), _ptr(relres),
                                      _stream(stream)), "rlqr_spd_residual")
        return res, relres


# ------------------------------------------------------------- cross-stage variables (include/rlqr_xs.h)

RLQR_XS_MAX_P = 8


class _XsLhs(ctypes.Structure):
    _fields_ = [(k, _vp) for k in ("Jq", "Jr", "Jc", "H")]


_lib.rlqr_xs_create.argtypes = [ctypes.POINTER(_vp), _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
_lib.rlqr_xs_factor.argtypes = [_vp, ctypes.POINTER(_Lhs), ctypes.POINTER(_XsLhs), ctypes.c_double, ctypes.c_int32,
                                _vp]
_lib.rlqr_xs_solve.argtypes = [_vp, ctypes.POINTER(_Rhs), _vp, ctypes.POINTER(_Sol), _vp, ctypes.c_double,
                               ctypes.c_int32, _vp, _vp, _vp]
_lib.rlqr_xs_inertia.argtypes = [_vp, _vp, _vp, _vp]
_lib.rlqr_xs_destroy.argtypes = [_vp]
_lib.rlqr_xs_destroy.restype = None
for _f in ("rlqr_xs_create", "rlqr_xs_factor", "rlqr_xs_solve", "rlqr_xs_inertia"):
    getattr(_lib, _f).restype = ctypes.c_int
XS_EXPORTED = ("rlqr_xs_create", "rlqr_xs_factor", "rlqr_xs_solve", "rlqr_xs_inertia", "rlqr_xs_destroy")

# ------------------------------------------------------------- stagewise equality rows (include/rlqr_eq.h)

class _EqData(ctypes.Structure):
    _fields_ = [(k, _vp) for k in ("E", "r", "eta")]


_lib.rlqr_eq_create.argtypes = [ctypes.POINTER(_vp), _vp, _i32p, ctypes.POINTER(ctypes.c_size_t)]
_lib.rlqr_eq_create.restype = ctypes.c_int
_lib.rlqr_eq_offsets.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
_lib.rlqr_eq_offsets.restype = ctypes.c_int
_lib.rlqr_eq_reduce.argtypes = [_vp, ctypes.POINTER(_Lhs), ctypes.POINTER(_Rhs), ctypes.POINTER(_EqData)] + [_vp] * 5 + [_vp]
_lib.rlqr_eq_reduce.restype = ctypes.c_int
_lib.rlqr_eq_recover.argtypes = [_vp, ctypes.POINTER(_EqData), ctypes.POINTER(_Sol), _vp, _vp]
_lib.rlqr_eq_recover.restype = ctypes.c_int
_lib.rlqr_eq_destroy.argtypes = [_vp]
_lib.rlqr_eq_destroy.restype = None
EQ_EXPORTED = ("rlqr_eq_create", "rlqr_eq_offsets", "rlqr_eq_reduce", "rlqr_eq_recover", "rlqr_eq_destroy")
RLQR_EQ_ARR_E, RLQR_EQ_ARR_V = 0, 1


class StageEquality:
    """rlqr_eq context over a Solver's batch: ne[b] equality rows per stage.
    reduce() gives the reduced lhs / rhs dicts for the Solver, recover() the
    equality multipliers w."""

    def __init__(self, solver: "Solver", ne):
        self.solver = solver
        self.torch = solver.torch
        self.ne = np.ascontiguousarray(ne, dtype=np.int32)
        assert self.ne.shape[0] == solver.batch
        ctx = _vp()
        ws = ctypes.c_size_t(0)
        with self.torch.cuda.device(solver.device):
            _check(_lib.rlqr_eq_create(ctypes.byref(ctx), solver.handle, self.ne.ctypes.data_as(_i32p),
                                       ctypes.byref(ws)), "rlqr_eq_create")
        self.ctx, self.workspace_bytes = ctx, int(ws.value)
        self.offsets = {}
        for name, arr in (("E", RLQR_EQ_ARR_E), ("v", RLQR_EQ_ARR_V)):
            off = np.zeros(solver.batch + 1, dtype=np.int64)
            _check(_lib.rlqr_eq_offsets(self.ctx, arr, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
                   "rlqr_eq_offsets")
            self.offsets[name] = off

    def __del__(self):
        x = getattr(self, "ctx", None)
        if x is not None and x.value and _lib is not None:
            try:
                _lib.rlqr_eq_destroy(x)
            except Exception:  # interpreter shutdown
                pass
            self.ctx = None

    def reduce(self, lhs, rhs, eq, out=None, stream=None):
        """eq: dict of device tensors E, r, eta. Returns (lhs', rhs') with the
        reduced Q, M, R, q, r (new tensors unless `out` is given; `out` may
        be lhs / rhs themselves: in place) and A, B, c, delta(, delta_diag)
        shared with the inputs."""
        if out is None:
            out = {k: self.torch.empty_like(lhs[k]) for k in ("Q", "M", "R")}
            out.update({k: self.torch.empty_like(rhs[k]) for k in ("q", "r")})
        L = _Lhs(*[_ptr(lhs.get(k)) for k in ("Q", "M", "R", "A", "B", "delta", "delta_diag")])
        Rh = _Rhs(_ptr(rhs["q"]), _ptr(rhs["r"]), _ptr(rhs["c"]))
        D = _EqData(_ptr(eq["E"]), _ptr(eq["r"]), _ptr(eq["eta"]))
        _check(_lib.rlqr_eq_reduce(self.ctx, ctypes.byref(L), ctypes.byref(Rh), ctypes.byref(D),
                                   *[_ptr(out[k]) for k in ("Q", "M", "R", "q", "r")], _stream(stream)),
               "rlqr_eq_reduce")
        lhs2 = dict(lhs)
        lhs2.update({k: out[k] for k in ("Q", "M", "R")})
        rhs2 = dict(rhs)
        rhs2.update({k: out[k] for k in ("q", "r")})
        return lhs2, rhs2

    def recover(self, eq, sol, w=None, stream=None):
        if w is None:
            w = self.torch.empty(max(int(self.offsets["v"][-1]), 1), dtype=self.torch.float64,
                                 device=self.solver.device)
        D = _EqData(_ptr(eq["E"]), _ptr(eq["r"]), _ptr(eq["eta"]))
        S = _Sol(_ptr(sol["x"]), _ptr(sol["u"]), _ptr(sol["y"]))
        _check(_lib.rlqr_eq_recover(self.ctx, ctypes.byref(D), ctypes.byref(S), _ptr(w), _stream(stream)),
               "rlqr_eq_recover")
        return w


def rlqr_xs_create(h, p: int):
    """Returns (context, workspace_bytes)."""
    x = _vp()
    ws = ctypes.c_size_t(0)
    _check(_lib.rlqr_xs_create(ctypes.byref(x), h, int(p), ctypes.byref(ws)), "rlqr_xs_create")
    return x, int(ws.value)


def rlqr_xs_factor(x, Q, M, R, A, B, delta, Jq, Jr, Jc, H, rel_tol, max_refine, stream=None, delta_diag=None):
    lhs = _Lhs(*[_ptr(t) for t in (Q, M, R, A, B, delta, delta_diag)])
    xl = _XsLhs(_ptr(Jq), _ptr(Jr), _ptr(Jc), _ptr(H))
    _check(_lib.rlqr_xs_factor(x, ctypes.byref(lhs), ctypes.byref(xl), float(rel_tol), int(max_refine),
                               _stream(stream)), "rlqr_xs_factor")


def rlqr_xs_solve(x, q, r, c, rtheta, dx, du, dy, dtheta, rel_tol, max_refine, inst_status=None,
                  inst_relres=None, stream=None):
    rhs = _Rhs(_ptr(q), _ptr(r), _ptr(c))
    sol = _Sol(_ptr(dx), _ptr(du), _ptr(dy))
    _check(_lib.rlqr_xs_solve(x, ctypes.byref(rhs), _ptr(rtheta), ctypes.byref(sol), _ptr(dtheta), float(rel_tol),
                              int(max_refine), _ptr(inst_status), _ptr(inst_relres), _stream(stream)),
           "rlqr_xs_solve")


def rlqr_xs_inertia(x, verdict=None, inertia=None, stream=None):
    _check(_lib.rlqr_xs_inertia(x, _ptr(verdict), _ptr(inertia), _stream(stream)), "rlqr_xs_inertia")


def rlqr_xs_destroy(x):
    _lib.rlqr_xs_destroy(x)


class CrossStage:
    """rlqr_xs context over a Solver's handle: p cross-stage variables. A
    Solver created with max_rhs >= p solves the p columns of J together."""

    def __init__(self, solver: "Solver", p: int):
        self.solver = solver
        self.torch = solver.torch
        self.p = int(p)
        with self.torch.cuda.device(solver.device):
            self.ctx, self.workspace_bytes = rlqr_xs_create(solver.handle, self.p)

    def __del__(self):
        x = getattr(self, "ctx", None)
        if x is not None and x.value and _lib is not None:
            try:
                _lib.rlqr_xs_destroy(x)
            except Exception:  # interpreter shutdown
                pass
            self.ctx = None

    def factor(self, lhs, J, H, rel_tol: float = 1e-8, max_refine: int = 3, stream=None):
        """J: dict Jq, Jr, Jc of p stacked columns; H: (B*p*p) float64."""
        s, torch = self.solver, self.torch
        for k, base in (("Jq", "q"), ("Jr", "r"), ("Jc", "c")):
            t = J[k]
            assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous() and \
                t.numel() >= self.p * s.size(base), k
        assert H.dtype == torch.float64 and H.is_contiguous() and H.numel() >= s.batch * self.p * self.p
        s._lhs = lhs
        self._keep = (lhs, J, H)  # re-read by every solve
        rlqr_xs_factor(self.ctx, *(lhs[k] for k in ("Q", "M", "R", "A", "B", "delta")), J["Jq"], J["Jr"], J["Jc"],
                       H, rel_tol, max_refine, stream=stream, delta_diag=lhs.get("delta_diag"))

    def solve(self, rhs, rtheta, out=None, rel_tol: float = 1e-8, max_refine: int = 3, stream=None):
        s, torch = self.solver, self.torch
        if out is None:
            out = {k: s.empty(k) for k in ("x", "u", "y")}
            out["theta"] = torch.empty(max(s.batch * self.p, 1), dtype=torch.float64, device=s.device)
        status = torch.empty(max(s.batch, 1), dtype=torch.int32, device=s.device)
        relres = torch.empty(max(s.batch, 1), dtype=torch.float64, device=s.device)
        rlqr_xs_solve(self.ctx, rhs["q"], rhs["r"], rhs["c"], rtheta, out["x"], out["u"], out["y"], out["theta"],
                      rel_tol, max_refine, status, relres, stream=stream)
        return out, status, relres

    def inertia(self, stream=None):
        s, torch = self.solver, self.torch
        verdict = torch.empty(max(s.batch, 1), dtype=torch.int32, device=s.device)
        inertia = torch.empty(max(3 * s.batch, 1), dtype=torch.int64, device=s.device)
        rlqr_xs_inertia(self.ctx, verdict, inertia, stream=stream)
        return verdict, inertia.view(-1, 3) if s.batch else inertia


# ------------------------------------------------------------- interior-point driver (include/ripm.h)

_dp = ctypes.POINTER(ctypes.c_double)


class _IpmProblem(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("N", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("dt", ctypes.c_double), ("wx", ctypes.c_double), ("wu", ctypes.c_double),
                ("wN", ctypes.c_double), ("xmax", ctypes.c_double), ("umax", ctypes.c_double),
                ("A", _dp), ("B", _dp), ("a", _dp), ("eta", ctypes.c_double), ("tol", ctypes.c_double),
                ("lqr_mode", ctypes.c_int32), ("ne", ctypes.c_int32), ("Eu", _dp)]


_lib.ripm_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_IpmProblem), ctypes.POINTER(ctypes.c_size_t)]
_lib.ripm_start.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
_lib.ripm_iterate.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), _vp]
_lib.ripm_solve.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp]
_lib.ripm_solution.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.ripm_destroy.argtypes = [_vp]
_lib.ripm_destroy.restype = None
for _f in ("ripm_create", "ripm_start", "ripm_iterate", "ripm_solve", "ripm_solution"):
    getattr(_lib, _f).restype = ctypes.c_int
IPM_EXPORTED = ("ripm_create", "ripm_start", "ripm_iterate", "ripm_solve", "ripm_solution", "ripm_destroy")

IPM_ETA = 1.0e3


class IPM:
    """Batched regularized interior-point driver over a workloads.TrajectorySet.
    eq: optional stagewise equality rows (E_u (ne, m), b (batch, N, ne)), E_u u_i = b_i."""

    def __init__(self, ts, lqr: str = "fp64", eta: float = IPM_ETA, tol: float = 1e-6, device: str = "cuda:0",
                 eq=None):
        import torch
        self.torch = torch
        self.ts = ts
        self.device = torch.device(device)
        self.N, self.n, self.m = ts.N, ts.n, ts.m
        self.ng = 2 + 2 * ts.m
        self.batch = ts.batch
        self._model = [np.ascontiguousarray(v, dtype=np.float64) for v in (ts.A, ts.B, ts.a)]
        self.ne = 0
        self._Eu = None
        if eq is not None:
            self._Eu = np.ascontiguousarray(np.atleast_2d(eq[0]), dtype=np.float64)
            self.ne = int(self._Eu.shape[0])
            assert self._Eu.shape == (self.ne, ts.m)
        p = _IpmProblem(self.batch, ts.N, ts.n, ts.m, ts.dt, ts.wx, ts.wu, ts.wN, ts.xmax, ts.umax,
                        *(v.ctypes.data_as(_dp) for v in self._model), float(eta), float(tol), MODES[lqr],
                        self.ne, None if self._Eu is None else self._Eu.ctypes.data_as(_dp))
        self.handle = _vp()
        ws = ctypes.c_size_t(0)
        with torch.cuda.device(self.device):
            _check(_lib.ripm_create(ctypes.byref(self.handle), ctypes.byref(p), ctypes.byref(ws)), "ripm_create")
        self.workspace_bytes = int(ws.value)
        self.x0 = torch.from_numpy(np.ascontiguousarray(ts.x0, dtype=np.float64)).to(self.device)
        self.goal = torch.from_numpy(np.ascontiguousarray(ts.goal, dtype=np.float64)).to(self.device)
        self.eb = None
        if eq is not None:
            eb = np.ascontiguousarray(np.broadcast_to(eq[1], (self.batch, ts.N, self.ne)), dtype=np.float64)
            self.eb = torch.from_numpy(eb).to(self.device)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            try:
                _lib.ripm_destroy(h)
            except Exception:
                pass
            self.handle = None

    def warm_size(self) -> int:
        N, n, m, ng = self.N, self.n, self.m, self.ng
        return (N + 1) * n * 2 + N * m + (N + 1) * ng

    def start(self, warm=None, stream=None):
        """warm: None (cold) or a float64 device tensor [batch, warm_size()] of x, u, y, log z."""
        if warm is not None:
            assert warm.dtype == self.torch.float64 and warm.is_cuda and warm.is_contiguous()
            assert warm.numel() == self.batch * self.warm_size()
        _check(_lib.ripm_start(self.handle, _ptr(self.x0), _ptr(self.goal), _ptr(warm), _ptr(self.eb),
                               _stream(stream)), "ripm_start")

    def iterate(self, stream=None) -> int:
        act = ctypes.c_int32(0)
        _check(_lib.ripm_iterate(self.handle, ctypes.byref(act), _stream(stream)), "ripm_iterate")
        return int(act.value)

    def solve(self, max_iter: int = 200, stream=None):
        iters = np.zeros(self.batch, dtype=np.int32)
        conv = np.zeros(self.batch, dtype=np.int32)
        _check(_lib.ripm_solve(self.handle, int(max_iter), iters.ctypes.data, conv.ctypes.data, _stream(stream)),
               "ripm_solve")
        return iters, conv

    def solution(self, stream=None):
        torch = self.torch
        B, N, n, m, ng = self.batch, self.N, self.n, self.m, self.ng
        x = torch.empty(B, N + 1, n, dtype=torch.float64, device=self.device)
        u = torch.empty(B, N, m, dtype=torch.float64, device=self.device)
        y = torch.empty(B, N + 1, n, dtype=torch.float64, device=self.device)
        z = torch.empty(B, N + 1, ng, dtype=torch.float64, device=self.device)
        ye = torch.empty(B, N, max(self.ne, 1), dtype=torch.float64, device=self.device) if self.ne else None
        _check(_lib.ripm_solution(self.handle, _ptr(x), _ptr(u), _ptr(y), _ptr(z), _ptr(ye), _stream(stream)),
               "ripm_solution")
        if self.ne:
            self.ye = ye
        return x, u, y, z


# ------------------------------------------------------------- network kernels (include/rmlp.h)

RMLP_F32, RMLP_BF16 = 0, 1
RMLP_ACT_NONE, RMLP_ACT_TANH = 0, 1
_lib.rmlp_gemm.argtypes = [ctypes.c_int32] * 6 + [_vp, ctypes.c_int32, _vp, ctypes.c_int32, ctypes.c_float,
                                                  ctypes.c_float, _vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp]
_lib.rmlp_tanh_backward.argtypes = [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
_lib.rmlp_colsum.argtypes = [ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp]
_lib.rmlp_mse.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.rmlp_adam.argtypes = [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, ctypes.c_float, ctypes.c_int32, _vp]
_lib.rmlp_affine_cols.argtypes = [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp]
_lib.rmlp_cast.argtypes = [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp]
for _f in ("rmlp_gemm", "rmlp_tanh_backward", "rmlp_colsum", "rmlp_mse", "rmlp_adam", "rmlp_affine_cols", "rmlp_cast"):
    getattr(_lib, _f).restype = ctypes.c_int
MLP_EXPORTED = ("rmlp_gemm", "rmlp_tanh_backward", "rmlp_colsum", "rmlp_mse", "rmlp_adam", "rmlp_affine_cols",
                "rmlp_cast")


def rmlp_gemm(dtype, transA, transB, M, N, K, A, lda, B, ldb, alpha, beta, C, ldc, bias=None, act=0, Cq=None,
              stream=None):
    _check(_lib.rmlp_gemm(dtype, int(transA), int(transB), M, N, K, _ptr(A), lda, _ptr(B), ldb, float(alpha),
                          float(beta), _ptr(C), ldc, _ptr(bias), act, _ptr(Cq), _stream(stream)), "rmlp_gemm")


def rmlp_tanh_backward(dtype, count, dh, h, dpre, dpreq=None, stream=None):
    _check(_lib.rmlp_tanh_backward(dtype, count, _ptr(dh), _ptr(h), _ptr(dpre), _ptr(dpreq), _stream(stream)),
           "rmlp_tanh_backward")


def rmlp_colsum(M, N, X, ldx, out, stream=None):
    _check(_lib.rmlp_colsum(M, N, _ptr(X), ldx, _ptr(out), _stream(stream)), "rmlp_colsum")


def rmlp_mse(dtype, M, N, pred, target, dpred, dpredq, loss, stream=None):
    _check(_lib.rmlp_mse(dtype, M, N, _ptr(pred), _ptr(target), _ptr(dpred), _ptr(dpredq), _ptr(loss),
                         _stream(stream)), "rmlp_mse")


def rmlp_adam(dtype, count, w, wq, g, m, v, lr, beta1, beta2, eps, t, stream=None):
    _check(_lib.rmlp_adam(dtype, count, _ptr(w), _ptr(wq), _ptr(g), _ptr(m), _ptr(v), float(lr), float(beta1),
                          float(beta2), float(eps), int(t), _stream(stream)), "rmlp_adam")


def rmlp_affine_cols(M, N, X, scale, shift, Y, stream=None):
    _check(_lib.rmlp_affine_cols(M, N, _ptr(X), _ptr(scale), _ptr(shift), _ptr(Y), _stream(stream)),
           "rmlp_affine_cols")


def rmlp_cast(dtype, count, x, y, stream=None):
    _check(_lib.rmlp_cast(dtype, count, _ptr(x), _ptr(y), _stream(stream)), "rmlp_cast")
