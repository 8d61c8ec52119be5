"""FP64 CPU oracle for dual-regularized LQR -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The library under `paper_2509_16370_amd` never does, and
this package imports nothing from it except the seeded input generators
(`workloads`), which hold no solver arithmetic.

Contents
  * rlqr_oracle.c (built to liboracle.so with gcc): the sequential recursion,
    the parallel algorithm run serially, the residual, and a batch driver.
    See that file's header for the passages of the paper each part follows.
  * dense.py: the plain definition -- the KKT matrix of eqs.
    primal-dual-linear-system / optimal-control-specialization assembled
    densely, solved with numpy, inertia by eigenvalues and by scipy's LDL^T.
  * crossstage.py: the arrowhead step with cross-stage variables (Section
    "Cross-Stage Variables"), densely and by the paper's Schur route.
  * eqstep.py: stagewise equality rows eliminated into a dual-regularized
    LQR (Section "Applying the regularized IPM to optimal control"),
    densely and by the elimination route.
  * certificate(): the pivot test of Theorem
    "riccati-inertia-certification-theorem" from the oracle's pivots.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rlqr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# A pivot is "zero" when |d| <= ZERO_PIVOT_FACTOR * dim * eps64 * max|diag|.
ZERO_PIVOT_FACTOR = 1.0e3

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP for the batch driver)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        llp = ctypes.POINTER(ctypes.c_longlong)
        i, d = ctypes.c_int, ctypes.c_double
        lib.rlqr_oracle_seq.argtypes = [i, i, i, d] + [dp] * 8 + [dp] * 3 + [dp] * 6
        lib.rlqr_oracle_seq.restype = i
        lib.rlqr_oracle_par.argtypes = [i, i, i, d] + [dp] * 8 + [i, i] + [dp] * 3 + [dp] * 6
        lib.rlqr_oracle_par.restype = i
        lib.rlqr_oracle_residual.argtypes = [i, i, i, d] + [dp] * 8 + [dp] * 3 + [dp]
        lib.rlqr_oracle_residual.restype = None
        lib.rlqr_oracle_combine.argtypes = [i] + [dp] * 15
        lib.rlqr_oracle_combine.restype = i
        lib.rlqr_oracle_seq_diag.argtypes = [i, i, i, dp] + [dp] * 8 + [dp] * 3 + [dp] * 6
        lib.rlqr_oracle_seq_diag.restype = i
        lib.rlqr_oracle_residual_diag.argtypes = [i, i, i, dp] + [dp] * 8 + [dp] * 3 + [dp]
        lib.rlqr_oracle_residual_diag.restype = None
        lib.rlqr_oracle_seq_batch.argtypes = ([i, ip, ip, ip, dp] + [dp] * 8 + [llp] * 11
                                              + [dp] * 3 + [ip, i, dp, dp, dp])
        lib.rlqr_oracle_seq_batch.restype = i
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _data(inst):
    return [np.ascontiguousarray(getattr(inst, k), dtype=np.float64)
            for k in ("Q", "M", "R", "A", "B", "q", "r", "c")]


def _outputs(n, m, N):
    return dict(
        x=np.zeros((N + 1, n)), u=np.zeros((N, m)), y=np.zeros((N + 1, n)),
        P=np.zeros((N + 1, n, n)), p=np.zeros((N + 1, n)),
        K=np.zeros((N, m, n)), k=np.zeros((N, m)),
        dS=np.zeros((N + 1, n)), dG=np.zeros((N, m)))


def _diag(inst) -> Optional[np.ndarray]:
    """The instance's per-stage diagonals Delta_i, (N+1, n), or None (delta I)."""
    dd = getattr(inst, "delta_diag", None)
    if dd is None:
        return None
    dd = np.ascontiguousarray(dd, dtype=np.float64)
    assert dd.shape == (inst.N + 1, inst.n) and (dd > 0).all()
    return dd


def seq(inst) -> Dict[str, np.ndarray]:
    """Sequential dual-regularized Riccati (FP64). Returns x, u, y, P, p, K, k,
    state pivots dS, control pivots dG and `status` (0, or 1 on a zero pivot).
    With `inst.delta_diag` set, Delta_i = diag(delta_diag[i]) and dS holds the
    pivots of I + Delta_i^{1/2} P_i Delta_i^{1/2}."""
    lib = _load()
    n, m, N = inst.n, inst.m, inst.N
    data = _data(inst)
    o = _outputs(n, m, N)
    dd = _diag(inst)
    outs = (_p(o["x"]), _p(o["u"]), _p(o["y"]), _p(o["P"]), _p(o["p"]), _p(o["K"]), _p(o["k"]),
            _p(o["dS"]), _p(o["dG"]))
    if dd is None:
        st = lib.rlqr_oracle_seq(n, m, N, float(inst.delta), *[_p(a) for a in data], *outs)
    else:
        st = lib.rlqr_oracle_seq_diag(n, m, N, _p(dd), *[_p(a) for a in data], *outs)
    o["status"] = st
    return o


def par(inst, bracketing: int = 1, p_mode: int = 1) -> Dict[str, np.ndarray]:
    """Parallel algorithm run serially. bracketing 0 = fold, 1 = Hillis-Steele
    rounds; p_mode 0 = p from the scan's p-combine, 1 = from the p-recurrence."""
    lib = _load()
    n, m, N = inst.n, inst.m, inst.N
    data = _data(inst)
    o = _outputs(n, m, N)
    st = lib.rlqr_oracle_par(n, m, N, float(inst.delta), *[_p(a) for a in data],
                             int(bracketing), int(p_mode),
                             _p(o["x"]), _p(o["u"]), _p(o["y"]),
                             _p(o["P"]), _p(o["p"]), _p(o["K"]), _p(o["k"]),
                             _p(o["dS"]), _p(o["dG"]))
    o["status"] = st
    return o


def combine(n, e1, e2):
    """One combine of interval elements e = (P, p, A, C, c) (eq. lqr-gpu-combo,
    single-inversion form). Returns the combined tuple."""
    lib = _load()
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (*e1, *e2)]
    out = (np.zeros((n, n)), np.zeros(n), np.zeros((n, n)), np.zeros((n, n)), np.zeros(n))
    st = lib.rlqr_oracle_combine(n, *[_p(v) for v in a], *[_p(v) for v in out])
    if st:
        raise np.linalg.LinAlgError("singular I + C P in combine")
    return out


def residual(inst, x, u, y) -> np.ndarray:
    """Stagewise KKT residual (Section "Residual Computation"), ordering:
    [x_i-row; u_i-row] for i < N, x_N-row, c_0-row, dynamics rows i = 0..N-1."""
    lib = _load()
    n, m, N = inst.n, inst.m, inst.N
    data = _data(inst)
    res = np.zeros(N * (n + m) + n + (N + 1) * n)
    xs = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, u, y)]
    dd = _diag(inst)
    if dd is None:
        lib.rlqr_oracle_residual(n, m, N, float(inst.delta), *[_p(a) for a in data],
                                 *[_p(v) for v in xs], _p(res))
    else:
        lib.rlqr_oracle_residual_diag(n, m, N, _p(dd), *[_p(a) for a in data],
                                      *[_p(v) for v in xs], _p(res))
    return res


def rhs_norm(inst) -> float:
    """||[s; c]||_inf of the right-hand side."""
    return float(max(np.abs(inst.q).max(), np.abs(inst.r).max() if inst.N else 0.0,
                     np.abs(inst.c).max()))


def rel_residual(inst, x, u, y) -> float:
    """||residual||_inf / ||[s; c]||_inf (the relative KKT residual)."""
    return float(np.abs(residual(inst, x, u, y)).max() / max(rhs_norm(inst), 1e-300))


def certificate(inst, dS: np.ndarray, dG: np.ndarray):
    """Pivot test of Theorem "riccati-inertia-certification-theorem".

    dS: (N+1, n) LDL^T pivots of S_hat_i = I + delta P_i (with a per-stage
    diagonal Delta_i: I + Delta_i^{1/2} P_i Delta_i^{1/2}); dG: (N, m) pivots of G_i.
    Returns (verdict, first_bad, inertia) where verdict is True iff every pivot
    is positive, first_bad is the code of the first failing pivot in the order
    the backward pass meets them (S_hat_N, G_{N-1}, S_hat_{N-1}, ..., G_0,
    S_hat_0; code 2i for S_hat_i, 2i+1 for G_i; -1 if none), and inertia is
    (0, (N+1) n, 0) plus the sign counts of all pivots.
    """
    n, m, N = inst.n, inst.m, inst.N
    npos, nneg, nzero = 0, (N + 1) * n, 0
    first_bad = -1
    order = []
    for i in range(N, -1, -1):
        order.append((2 * i, dS[i]))
        if i > 0:
            order.append((2 * (i - 1) + 1, dG[i - 1]))
    for code, d in order:
        d = np.asarray(d)
        pos = int(np.sum(d > 0))
        neg = int(np.sum(d < 0))
        zer = int(d.size - pos - neg)
        npos += pos
        nneg += neg
        nzero += zer
        if first_bad < 0 and (neg or zer):
            first_bad = code
    return first_bad < 0, first_bad, (npos, nneg, nzero)


def seq_batch(packed, nthreads: int = 0, pivots: bool = False):
    """Sequential oracle over a packed batch, instances spread over threads.
    Returns (x, u, y, status, threads_used); with pivots=True also (dS, dG),
    the pivots of every instance laid out like x and u (see certificate_batch)."""
    lib = _load()
    a = packed.arrays
    o = packed.offsets
    x = np.zeros(o["x"][-1])
    u = np.zeros(o["u"][-1])
    y = np.zeros(o["y"][-1])
    dS = np.zeros(o["x"][-1]) if pivots else None
    dG = np.zeros(o["u"][-1]) if pivots else None
    status = np.zeros(packed.batch, dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int)
    llp = ctypes.POINTER(ctypes.c_longlong)
    N = np.ascontiguousarray(packed.N, dtype=np.int32)
    nx = np.ascontiguousarray(packed.n, dtype=np.int32)
    nu = np.ascontiguousarray(packed.m, dtype=np.int32)
    offs = [np.ascontiguousarray(o[k], dtype=np.int64) for k in
            ("Q", "M", "R", "A", "B", "q", "r", "c", "x", "u", "y")]
    dd = packed.arrays.get("delta_diag")
    used = lib.rlqr_oracle_seq_batch(
        packed.batch, N.ctypes.data_as(ip), nx.ctypes.data_as(ip), nu.ctypes.data_as(ip),
        _p(np.ascontiguousarray(packed.delta)),
        *[_p(a[k]) for k in ("Q", "M", "R", "A", "B", "q", "r", "c")],
        *[v.ctypes.data_as(llp) for v in offs],
        _p(x), _p(u), _p(y), status.ctypes.data_as(ip), int(nthreads),
        None if dd is None else _p(np.ascontiguousarray(dd, dtype=np.float64)), _p(dS), _p(dG))
    if pivots:
        return x, u, y, status, used, dS, dG
    return x, u, y, status, used


def certificate_batch(packed, insts, dS, dG):
    """certificate() of every instance of a packed batch from the pivots
    seq_batch(..., pivots=True) returned: lists of (verdict, first_bad, inertia)."""
    o = packed.offsets
    out = []
    for b, inst in enumerate(insts):
        n, m, N = inst.n, inst.m, inst.N
        s = dS[o["x"][b]:o["x"][b + 1]].reshape(N + 1, n)
        g = dG[o["u"][b]:o["u"][b + 1]].reshape(N, m)
        out.append(certificate(inst, s, g))
    return out
