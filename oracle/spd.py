"""General SPD per-stage regularization Delta_i -- TEST INFRASTRUCTURE ONLY.

The definition of a dual-regularized LQR problem (Section "Dual-Regularized
LQR") lets every Delta_i be any symmetric positive definite matrix. This
module is the plain float64 CPU reference for that case, written with numpy
from the paper's formulas, independent of the HIP library:

  * seq(): the sequential recursion of Theorem "main-seq-theorem" with the
    full matrices Delta_i, in the paper's order -- W_{k+1} =
    P_{k+1}(I + Delta_{k+1} P_{k+1})^{-1}, g_{k+1} = p_{k+1} + W_{k+1}(c_{k+1} -
    Delta_{k+1} p_{k+1}), G_k, H_k, h_k, K_k, k_k, then P_k and p_k
    (eqs. value-fn-formulas) -- and the forward rollout x_0 = (I + Delta_0
    P_0)^{-1}(c_0 - Delta_0 p_0), u_k = K_k x_k + k_k, x_{k+1} = (I +
    Delta_{k+1} P_{k+1})^{-1}(A_k x_k + B_k u_k + c_{k+1} - Delta_{k+1}
    p_{k+1}), y_k = P_k x_k + p_k. The nonsymmetric I + Delta P is applied by
    LU (numpy.linalg.solve); W, G and P are symmetrized every stage (the
    paper proves them symmetric, its evaluation order is not).
  * The certificate's state pivots: unpivoted LDL^T of the symmetric matrix
    S_hat_i = I + L_i^T P_i L_i, with L_i the Cholesky factor of Delta_i
    (Delta_i = L_i L_i^T). L_i^T S_i L_i = S_hat_i for S_i = P_i + Delta_i^{-1},
    so S_hat_i is congruent to the state pivot S_i of Theorem
    "riccati-inertia-certification-theorem" (same inertia, Sylvester), and
    S_hat_i = L_i^{-1}(I + Delta_i P_i)L_i is similar to I + Delta_i P_i;
    Section "Inertia Certification" allows checking PD-ness on any such
    symmetric representative.
    For a diagonal Delta_i, L_i = Delta_i^{1/2} and this is the paper's
    Delta_i^{1/2} P_i Delta_i^{1/2}.
  * residual(): the stagewise residual of Section "Residual Computation" with
    Delta_i y_i as a matrix-vector product.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

# a pivot counts as zero when |d| <= ZERO_PIVOT_FACTOR * dim * eps64 * max|diag|
ZERO_PIVOT_FACTOR = 1.0e3


def ldl_pivots(S: np.ndarray):
    """Diagonal of the unpivoted LDL^T factorization of the symmetric S
    (plain loops); returns (d, zero) where zero is True when a pivot is
    below the zero threshold (the factorization then stops)."""
    n = S.shape[0]
    L = np.eye(n)
    d = np.zeros(n)
    scale = np.abs(np.diag(S)).max() if n else 0.0
    thr = ZERO_PIVOT_FACTOR * n * np.finfo(float).eps * max(scale, 1e-300)
    for j in range(n):
        d[j] = S[j, j] - np.sum(L[j, :j] ** 2 * d[:j])
        if abs(d[j]) <= thr:
            return d, True
        for i in range(j + 1, n):
            L[i, j] = (S[i, j] - np.sum(L[i, :j] * L[j, :j] * d[:j])) / d[j]
    return d, False


def _sym(X):
    return 0.5 * (X + X.T)


def seq(inst) -> Dict[str, np.ndarray]:
    """Sequential dual-regularized Riccati with full SPD Delta_i (inst.delta_full,
    (N+1, n, n)). Returns x, u, y, P, p, K, k, dS (pivots of S_hat_i), dG
    (pivots of G_i) and status (1 on a zero pivot, else 0)."""
    n, m, N = inst.n, inst.m, inst.N
    D = np.asarray(inst.delta_full, dtype=np.float64)
    assert D.shape == (N + 1, n, n)
    I = np.eye(n)
    P = np.zeros((N + 1, n, n))
    p = np.zeros((N + 1, n))
    K = np.zeros((N, m, n))
    k = np.zeros((N, m))
    dS = np.zeros((N + 1, n))
    dG = np.zeros((N, m))
    status = 0
    P[N] = inst.Q[N]
    p[N] = inst.q[N]
    for i in range(N - 1, -1, -1):
        P1, p1, D1 = P[i + 1], p[i + 1], D[i + 1]
        # W = P (I + Delta P)^{-1}: W^T = (I + P Delta)^{-1} P, solved by LU
        W = _sym(np.linalg.solve(I + P1 @ D1, P1).T)
        A, B = inst.A[i], inst.B[i]
        G = _sym(inst.R[i] + B.T @ W @ B)
        H = B.T @ W @ A + inst.M[i].T
        g = p1 + W @ (inst.c[i + 1] - D1 @ p1)
        h = inst.r[i] + B.T @ g
        K[i] = -np.linalg.solve(G, H)
        k[i] = -np.linalg.solve(G, h)
        P[i] = _sym(A.T @ W @ A + inst.Q[i] + H.T @ K[i])
        p[i] = inst.q[i] + A.T @ g + H.T @ k[i]
        dG[i], z = ldl_pivots(G)
        status |= int(z)
    for i in range(N + 1):
        L = np.linalg.cholesky(D[i])
        dS[i], z = ldl_pivots(_sym(I + L.T @ P[i] @ L))
        status |= int(z)
    x = np.zeros((N + 1, n))
    u = np.zeros((N, m))
    y = np.zeros((N + 1, n))
    x[0] = np.linalg.solve(I + D[0] @ P[0], inst.c[0] - D[0] @ p[0])
    for i in range(N):
        u[i] = K[i] @ x[i] + k[i]
        x[i + 1] = np.linalg.solve(I + D[i + 1] @ P[i + 1],
                                   inst.A[i] @ x[i] + inst.B[i] @ u[i] + inst.c[i + 1] - D[i + 1] @ p[i + 1])
    for i in range(N + 1):
        y[i] = P[i] @ x[i] + p[i]
    return dict(x=x, u=u, y=y, P=P, p=p, K=K, k=k, dS=dS, dG=dG, status=status)


def residual(inst, x, u, y) -> np.ndarray:
    """Stagewise residual (Section "Residual Computation") with full Delta_i,
    in the library's row order: [x_i-row; u_i-row] for i < N, the x_N row,
    the c_0 row, the dynamics rows i = 0..N-1."""
    n, m, N = inst.n, inst.m, inst.N
    D = np.asarray(inst.delta_full, dtype=np.float64)
    x = np.asarray(x).reshape(N + 1, n)
    u = np.asarray(u).reshape(N, m)
    y = np.asarray(y).reshape(N + 1, n)
    rows = []
    for i in range(N):
        rows.append(inst.Q[i] @ x[i] + inst.M[i] @ u[i] + inst.A[i].T @ y[i + 1] + inst.q[i] - y[i])
        rows.append(inst.M[i].T @ x[i] + inst.R[i] @ u[i] + inst.B[i].T @ y[i + 1] + inst.r[i])
    rows.append(inst.Q[N] @ x[N] + inst.q[N] - y[N])
    rows.append(inst.c[0] - D[0] @ y[0] - x[0])
    for i in range(N):
        rows.append(inst.A[i] @ x[i] + inst.B[i] @ u[i] + inst.c[i + 1] - D[i + 1] @ y[i + 1] - x[i + 1])
    return np.concatenate(rows) if rows else np.zeros(0)


def rel_residual(inst, x, u, y) -> float:
    """||residual||_inf / ||[s; c]||_inf."""
    b = max(np.abs(inst.q).max(), np.abs(inst.r).max() if inst.N else 0.0, np.abs(inst.c).max())
    return float(np.abs(residual(inst, x, u, y)).max() / max(b, 1e-300))


def certificate(inst, dS, dG):
    """(verdict, first_bad, inertia) from the pivots, in the elimination order
    S_hat_N, G_{N-1}, S_hat_{N-1}, ..., G_0, S_hat_0 (codes 2i and 2i+1)."""
    n, N = inst.n, inst.N
    npos, nneg, nzero = 0, (N + 1) * n, 0
    first_bad = -1
    for i in range(N, -1, -1):
        blocks = [(2 * i, dS[i])] + ([(2 * (i - 1) + 1, dG[i - 1])] if i > 0 else [])
        for code, d in blocks:
            pos, neg = int(np.sum(d > 0)), int(np.sum(d < 0))
            npos += pos
            nneg += neg
            nzero += len(d) - pos - neg
            if first_bad < 0 and pos < len(d):
                first_bad = code
    return first_bad < 0, first_bad, (npos, nneg, nzero)
