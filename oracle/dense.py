"""Dense brute force for dual-regularized LQR -- TEST INFRASTRUCTURE ONLY.

The plain definition of what every solver must return: the first-order
conditions of the dual-regularized LQR problem (eq. primal-dual-linear-system)
with the block layout of eq. optimal-control-specialization,

    [[P, C^T], [C, -Delta]] [x; y] = -[s; c],

with Delta = blockdiag(Delta_0, ..., Delta_N): delta I, or the instance's
per-stage diagonals or full SPD blocks when it carries them (Definition
"dual-regularized LQR" lets every Delta_i be any SPD matrix),

assembled as a dense matrix and solved with numpy. Inertia comes from the
eigenvalues (numpy.linalg.eigvalsh) and, independently, from the block
diagonal of scipy's symmetric-indefinite LDL^T. Small sizes only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def _primal_index(n, m, N):
    """Offsets of x_i and u_i inside the primal vector [x_0, u_0, ..., x_{N-1}, u_{N-1}, x_N]."""
    xo = [i * (n + m) for i in range(N + 1)]
    uo = [i * (n + m) + n for i in range(N)]
    return xo, uo


def assemble(inst):
    """Return (K, rhs) with K the KKT matrix and rhs = -[s; c]."""
    n, m, N, d = inst.n, inst.m, inst.N, inst.delta
    nxp = N * (n + m) + n
    ny = (N + 1) * n
    xo, uo = _primal_index(n, m, N)
    P = np.zeros((nxp, nxp))
    s = np.zeros(nxp)
    for i in range(N):
        P[xo[i]:xo[i] + n, xo[i]:xo[i] + n] = inst.Q[i]
        P[xo[i]:xo[i] + n, uo[i]:uo[i] + m] = inst.M[i]
        P[uo[i]:uo[i] + m, xo[i]:xo[i] + n] = inst.M[i].T
        P[uo[i]:uo[i] + m, uo[i]:uo[i] + m] = inst.R[i]
        s[xo[i]:xo[i] + n] = inst.q[i]
        s[uo[i]:uo[i] + m] = inst.r[i]
    P[xo[N]:xo[N] + n, xo[N]:xo[N] + n] = inst.Q[N]
    s[xo[N]:xo[N] + n] = inst.q[N]
    C = np.zeros((ny, nxp))
    C[0:n, xo[0]:xo[0] + n] = -np.eye(n)
    for i in range(N):
        C[(i + 1) * n:(i + 2) * n, xo[i]:xo[i] + n] = inst.A[i]
        C[(i + 1) * n:(i + 2) * n, uo[i]:uo[i] + m] = inst.B[i]
        C[(i + 1) * n:(i + 2) * n, xo[i + 1]:xo[i + 1] + n] = -np.eye(n)
    dd = getattr(inst, "delta_diag", None)
    df = getattr(inst, "delta_full", None)
    if df is not None:  # full SPD blocks Delta_i
        Delta = scipy.linalg.block_diag(*np.asarray(df, dtype=np.float64))
    else:
        Delta = d * np.eye(ny) if dd is None else np.diag(np.asarray(dd, dtype=np.float64).reshape(-1))
    K = np.block([[P, C.T], [C, -Delta]])
    rhs = -np.concatenate([s, inst.c.reshape(-1)])
    return K, rhs


def solve(inst):
    """Dense solve; returns x (N+1,n), u (N,m), y (N+1,n)."""
    n, m, N = inst.n, inst.m, inst.N
    K, rhs = assemble(inst)
    z = np.linalg.solve(K, rhs)
    return split(inst, z)


def split(inst, z):
    n, m, N = inst.n, inst.m, inst.N
    nxp = N * (n + m) + n
    xo, uo = _primal_index(n, m, N)
    x = np.stack([z[xo[i]:xo[i] + n] for i in range(N + 1)])
    u = np.stack([z[uo[i]:uo[i] + m] for i in range(N)]) if N else np.zeros((0, m))
    y = z[nxp:].reshape(N + 1, n)
    return x, u, y


def join(inst, x, u, y):
    n, m, N = inst.n, inst.m, inst.N
    parts = []
    for i in range(N):
        parts += [x[i], u[i]]
    parts.append(x[N])
    return np.concatenate(parts + [np.asarray(y).reshape(-1)])


def inertia_eig(K, rel_tol=1e-9):
    """(n+, n-, n0) from eigenvalues, zero meaning |lambda| <= rel_tol * ||K||_2."""
    w = np.linalg.eigvalsh(K)
    tol = rel_tol * max(np.abs(w).max(), 1e-300)
    return int(np.sum(w > tol)), int(np.sum(w < -tol)), int(np.sum(np.abs(w) <= tol))


def inertia_ldl(K, rel_tol=1e-9):
    """(n+, n-, n0) from the block diagonal of scipy's Bunch-Kaufman LDL^T
    (Sylvester: congruent matrices share inertia)."""
    _, D, _ = scipy.linalg.ldl(K)
    w = np.linalg.eigvalsh(D)  # D is block diagonal with 1x1 and 2x2 blocks
    tol = rel_tol * max(np.abs(np.linalg.eigvalsh(K)).max(), 1e-300)
    return int(np.sum(w > tol)), int(np.sum(w < -tol)), int(np.sum(np.abs(w) <= tol))


def target_inertia(inst):
    n, m, N = inst.n, inst.m, inst.N
    return (N * (n + m) + n, (N + 1) * n, 0)
