"""Cross-stage variables (Section "Cross-Stage Variables") -- TEST INFRASTRUCTURE ONLY.

The Newton step with p variables theta shared by every stage is the arrowhead
system of eq. cross-stage-kkt,

    [[K, J], [J^T, H]] [dw; dtheta] = -[r_w; r_theta],

with K the dual-regularized LQR matrix of eq. primal-dual-linear-system. Each
column J_j of J, and r_w, lives in the row space of K and is given in the
layout of an LQR right-hand side: (Jq (N+1, n), Jr (N, m), Jc (N+1, n)) for
the x-rows, u-rows and dual (dynamics) rows; dw = (x, u, y) in the solution
layout. H is p x p symmetric, r_theta and dtheta have p entries.

Two routes, sharing nothing but the C oracle's sequential recursion:
  * dense(): the plain definition -- the arrowhead matrix assembled from the
    dense LQR matrix of oracle.dense and solved with numpy;
  * schur(): the paper's route, eq. cross-stage-schur and the two formulas
    after it, in their order: K^{-1} J and K^{-1} r_w by sequential Riccati
    solves, S = H - J^T K^{-1} J, dtheta = -S^{-1}(r_theta - J^T K^{-1} r_w),
    dw = -K^{-1}(r_w + J dtheta) (one more solve).
Inertia: eigenvalues of the dense arrowhead matrix; by Haynsworth's formula
it equals In(K) + In(S) when K is nonsingular.
Only tests/, the smoke check and the benchmark's CPU leg may import this.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

import oracle
from oracle import dense as odense

Vec = Tuple[np.ndarray, np.ndarray, np.ndarray]  # (q-or-x, r-or-u, c-or-y) blocks


def _with_rhs(inst, v: Vec):
    q, r, c = (np.ascontiguousarray(a, dtype=np.float64) for a in v)
    return dataclasses.replace(inst, q=q.reshape(inst.N + 1, inst.n), r=r.reshape(inst.N, inst.m),
                               c=c.reshape(inst.N + 1, inst.n))


def kinv(inst, v: Vec) -> Vec:
    """K^{-1} v by the sequential recursion: the oracle returns z with
    K z = -v, so K^{-1} v = -z."""
    o = oracle.seq(_with_rhs(inst, v))
    if o["status"]:
        raise np.linalg.LinAlgError("zero pivot in the sequential recursion")
    return -o["x"], -o["u"], -o["y"]


def dot(a: Vec, b: Vec) -> float:
    """Inner product of a row-space vector with a solution-space vector
    (x-rows with x, u-rows with u, dual rows with y)."""
    return float(sum(np.sum(np.asarray(s) * np.asarray(t)) for s, t in zip(a, b)))


def _axpy(a: Vec, coef: Sequence[float], cols: List[Vec]) -> Vec:
    out = [np.array(s, dtype=np.float64, copy=True) for s in a]
    for cj, col in zip(coef, cols):
        for k in range(3):
            out[k] = out[k] + cj * np.asarray(col[k])
    return tuple(out)


def schur(inst, J: List[Vec], H: np.ndarray, rw: Vec, rth: np.ndarray):
    """The paper's Schur-complement route; returns (dw, dtheta, S)."""
    p = len(J)
    KJ = [kinv(inst, J[j]) for j in range(p)]
    S = np.array([[H[i, j] - dot(J[i], KJ[j]) for j in range(p)] for i in range(p)])
    Krw = kinv(inst, rw)
    t = np.asarray(rth, dtype=np.float64) - np.array([dot(J[i], Krw) for i in range(p)])
    dtheta = -np.linalg.solve(S, t)
    w = kinv(inst, _axpy(rw, dtheta, J))
    dw = tuple(-a for a in w)
    return dw, dtheta, S


def assemble(inst, J: List[Vec], H: np.ndarray, rw: Vec, rth: np.ndarray):
    """Dense arrowhead matrix and right-hand side -[r_w; r_theta]."""
    K, _ = odense.assemble(inst)
    cols = [odense.join(inst, *Jj) for Jj in J]
    Jm = np.stack(cols, axis=1) if cols else np.zeros((K.shape[0], 0))
    A = np.block([[K, Jm], [Jm.T, np.asarray(H, dtype=np.float64)]])
    b = -np.concatenate([odense.join(inst, *rw), np.asarray(rth, dtype=np.float64)])
    return A, b


def dense(inst, J: List[Vec], H: np.ndarray, rw: Vec, rth: np.ndarray):
    """The plain definition; returns (dw, dtheta)."""
    A, b = assemble(inst, J, H, rw, rth)
    z = np.linalg.solve(A, b)
    nk = A.shape[0] - len(J)
    return odense.split(inst, z[:nk]), z[nk:]


def inertia(inst, J: List[Vec], H: np.ndarray):
    """(n+, n-, n0) of the arrowhead matrix from its eigenvalues."""
    A, _ = assemble(inst, J, H, (inst.q, inst.r, inst.c), np.zeros(len(J)))
    return odense.inertia_eig(A)


def target_inertia(inst, p: int):
    """Inertia of a step whose primal block is positive definite on the null
    space of the constraints: the LQR target with p more positive values."""
    a, b, c = odense.target_inertia(inst)
    return (a + p, b, c)


def residual(inst, J: List[Vec], H: np.ndarray, rw: Vec, rth: np.ndarray, dw: Vec, dtheta: np.ndarray):
    """(res_w, res_theta) = [[K, J], [J^T, H]] [dw; dtheta] + [r_w; r_theta],
    res_w in the order of the LQR residual (Section "Residual Computation")."""
    res_w = oracle.residual(_with_rhs(inst, _axpy(rw, dtheta, J)), *dw)
    res_t = np.array([dot(J[i], dw) for i in range(len(J))]) + np.asarray(H) @ dtheta + np.asarray(rth)
    return res_w, res_t


def rel_residual(inst, J, H, rw, rth, dw, dtheta) -> float:
    res_w, res_t = residual(inst, J, H, rw, rth, dw, dtheta)
    num = max(np.abs(res_w).max(), np.abs(res_t).max() if len(res_t) else 0.0)
    den = max(max(np.abs(np.asarray(a)).max() if np.asarray(a).size else 0.0 for a in rw),
              np.abs(np.asarray(rth)).max() if len(rth) else 0.0)
    return float(num / max(den, 1e-300))
