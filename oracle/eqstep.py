"""Stagewise equality constraints eliminated into a dual-regularized LQR --
TEST INFRASTRUCTURE ONLY.

Section "Applying the regularized IPM to optimal control": the Newton-KKT
system of the regularized interior-point method carries, besides the
dynamics, the rows of the other equality constraints with the diagonal
-Delta_C^{-1} of the dual regularization. For a stagewise constraint of
stage i with Jacobian E_i = [E_x | E_u] (ne x (n + m); stage N: E_x only),
residual r_e and penalty D = diag(eta) (regularization D^{-1}), the system
in the library's sign convention is

    [[P, C^T, E^T], [C, -Delta, 0], [E, 0, -D^{-1}]] [z; y; w] = -[s; c; r_e],

with [[P, C^T], [C, -Delta]] the dual-regularized LQR matrix of eq.
primal-dual-linear-system. Its last row gives w = D (E z + r_e); putting
that into the first row leaves a dual-regularized LQR with the stage
Hessian [[Q, M], [M^T, R]] + E^T D E and the gradient (q, r) + E^T D r_e
(the elimination the paper describes after the one of dz; E stagewise and D
diagonal keep the problem stagewise).

Two routes sharing nothing but the C oracle's sequential recursion:
  * dense(): the plain definition -- the full matrix assembled densely and
    solved with numpy;
  * route(): reduce(), the sequential oracle, recover().
Inertia: eigenvalues of the dense matrices; eliminating the negative
definite -D^{-1} block adds ne (N + 1) negative eigenvalues (Haynsworth).
Only tests/, the smoke check and the benchmark's CPU leg may import this.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle
from oracle import dense as odense


def full_matrix(inst, eq):
    """Dense [[K, F^T], [F, -D^{-1}]] and right-hand side -[s; c; r_e], where
    K, -[s; c] come from oracle.dense.assemble and F places E_i on the
    (x_i, u_i) columns."""
    n, m, N, ne = inst.n, inst.m, inst.N, eq.ne
    K, rhs = odense.assemble(inst)
    xo, uo = odense._primal_index(n, m, N)
    nk = K.shape[0]
    nw = (N + 1) * ne
    F = np.zeros((nw, nk))
    for i in range(N + 1):
        rows = slice(i * ne, (i + 1) * ne)
        F[rows, xo[i]:xo[i] + n] = eq.Ex[i]
        if i < N:
            F[rows, uo[i]:uo[i] + m] = eq.Eu[i]
    D = np.asarray(eq.eta, dtype=np.float64).reshape(-1)
    full = np.block([[K, F.T], [F, -np.diag(1.0 / D)]])
    b = np.concatenate([rhs, -np.asarray(eq.r, dtype=np.float64).reshape(-1)])
    return full, b


def dense(inst, eq):
    """Plain definition: returns x (N+1,n), u (N,m), y (N+1,n), w (N+1,ne)."""
    full, b = full_matrix(inst, eq)
    sol = np.linalg.solve(full, b)
    nk = full.shape[0] - (inst.N + 1) * eq.ne
    x, u, y = odense.split(inst, sol[:nk])
    return x, u, y, sol[nk:].reshape(inst.N + 1, eq.ne)


def reduce(inst, eq):
    """The dual-regularized LQR left after eliminating w (stagewise)."""
    N = inst.N
    D = np.asarray(eq.eta, dtype=np.float64)
    Q = inst.Q.copy()
    q = inst.q.copy()
    M = inst.M.copy()
    R = inst.R.copy()
    r = inst.r.copy()
    for i in range(N + 1):
        Ex = eq.Ex[i]
        Q[i] += Ex.T @ np.diag(D[i]) @ Ex
        q[i] += Ex.T @ (D[i] * eq.r[i])
        if i < N:
            Eu = eq.Eu[i]
            M[i] += Ex.T @ np.diag(D[i]) @ Eu
            R[i] += Eu.T @ np.diag(D[i]) @ Eu
            r[i] += Eu.T @ (D[i] * eq.r[i])
    return dataclasses.replace(inst, Q=Q, M=M, R=R, q=q, r=r)


def recover(inst, eq, x, u):
    """w_i = D_i (E_i z_i + r_e,i)."""
    w = np.zeros((inst.N + 1, eq.ne))
    for i in range(inst.N + 1):
        ez = eq.Ex[i] @ x[i]
        if i < inst.N:
            ez = ez + eq.Eu[i] @ u[i]
        w[i] = eq.eta[i] * (ez + eq.r[i])
    return w


def route(inst, eq):
    """Reduce, solve with the sequential oracle, recover w. Also returns the
    oracle's output dict of the reduced problem (pivots, status)."""
    red = reduce(inst, eq)
    o = oracle.seq(red)
    w = recover(inst, eq, o["x"], o["u"])
    return o["x"], o["u"], o["y"], w, o


def inertia_full(inst, eq, rel_tol=1e-9):
    full, _ = full_matrix(inst, eq)
    return odense.inertia_eig(full, rel_tol)
