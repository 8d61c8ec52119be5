"""Plain float64 CPU regularized primal-dual interior-point method for the
constrained trajectory problems of `workloads.TrajectorySet`.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
benchmark's CPU-baseline leg, never by the product path.

The method is the regularized IPM of Section "The Regularized Interior Point
Method": the Barrier-Lagrangian L = f - mu sum log s + y^T c + z^T (g + s),
the augmented barrier-Lagrangian merit A = L + 1/2 eta (|c|^2 + |g + s|^2)
(Delta_C = Delta_G = eta I), and the Newton-KKT system (eq.
ipm-4x4-newton-kkt) reduced by eliminating ds (eq. ipm-3x3-newton-kkt) and
then dz (Section "Applying the regularized IPM to optimal control"), which
leaves a dual-regularized LQR with delta = 1/eta solved by the sequential
oracle; its pivot certificate is the inertia test of Theorem
inertia-al-descent-theorem, answered by adding rho I to the Hessian.

Choices the paper leaves open (the readings documented with the driver):
eta = 1e3 (LQR delta = 1e-3); exact Lagrangian Hessian (with the tanh second
derivatives); rho = 0 initially, rho <- max(1e-8, 10 rho) while the
certificate fails, rho <- rho / 3 after a success; fraction to the boundary
tau = max(0.99, 1 - mu) for s (primal step) and z (dual step); Armijo
(c1 = 1e-4) on the merit along (dx, ds) over the ladder alpha_max 2^-k,
k = 0..11 (the last one if none passes); the equality multipliers take the
full step y <- y + dy, z its own step to the boundary; mu0 = 0.1 (cold) and
mu <- max(mu / 10, 1e-9) when the barrier error is <= 10 mu; converged when
|grad_x L|_inf, |c|_inf, |g + s|_inf and |s z|_inf are all <= 1e-6; at most
200 iterations. Cold start: x_i = x0, u_i = 0, y = 0, s = max(-g, 1e-2),
z = mu0 / s.

Optional stagewise equality rows e_i(u) = E_u u_i - b_i = 0 (i < N), ne rows
per stage with multipliers y_e: their rows of the Newton-KKT system carry the
same -1/eta dual regularization and are eliminated into the LQR (Section
"Applying the regularized IPM to optimal control"): R_i += eta E_u^T E_u,
r_i += eta E_u^T e_i, then dy_e = eta (E_u du_i + e_i) with the full step
y_e <- y_e + dy_e; the merit gains y_e^T e + eta/2 |e|^2 and the
convergence test |e|_inf.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

from . import seq as lqr_seq, certificate as lqr_certificate

ETA = 1.0e3
TOL = 1.0e-6
MAX_ITER = 200
C1 = 1.0e-4
LADDER = 12


@dataclasses.dataclass
class State:
    x: np.ndarray   # (N+1, n)
    u: np.ndarray   # (N, m)
    y: np.ndarray   # (N+1, n)  y_0 for x_0 = x0, y_{i+1} for the dynamics of step i
    s: np.ndarray   # (N+1, ng) slacks (row N: only the 2 state rows are used)
    z: np.ndarray   # (N+1, ng)
    mu: float
    rho: float = 0.0
    ye: Optional[np.ndarray] = None  # (N, ne) multipliers of the stagewise equality rows


class Problem:
    """One problem b of a TrajectorySet: f, c, g and their derivatives."""

    def __init__(self, ts, b: int, eq=None):
        """eq: optional (E_u (ne, m), b (N, ne)) stagewise equality rows E_u u_i = b_i."""
        self.ts = ts
        self.Eu = None if eq is None else np.atleast_2d(np.asarray(eq[0], dtype=float))
        self.eb = None if eq is None else np.asarray(eq[1], dtype=float).reshape(ts.N, -1)
        self.n, self.m, self.N = ts.n, ts.m, ts.N
        self.ng = 2 + 2 * ts.m
        self.x0 = ts.x0[b].astype(float)
        self.goal = ts.goal[b].astype(float)
        n, m = self.n, self.m
        # inequality Jacobians (constant): stage rows [a; u - umax; -u - umax]
        self.Gx = np.zeros((self.ng, n))
        self.Gx[:2] = ts.a
        self.Gu = np.zeros((self.ng, m))
        self.Gu[2:2 + m] = np.eye(m)
        self.Gu[2 + m:] = -np.eye(m)
        # the terminal stage has only the two state rows
        self.mask = np.ones((self.N + 1, self.ng))
        self.mask[self.N, 2:] = 0.0

    # ---- model
    def dyn(self, x, u):
        """d(x, u) = x + dt tanh(A x + B u), its Jacobians and the tanh terms."""
        ts = self.ts
        v = x @ ts.A.T + u @ ts.B.T
        th = np.tanh(v)
        sech2 = 1.0 - th * th
        return x + ts.dt * th, th, sech2

    def g(self, x, u):
        """Inequalities g <= 0, (N+1, ng); padded rows of stage N are 0."""
        ts = self.ts
        G = np.zeros((self.N + 1, self.ng))
        G[:, :2] = x @ ts.a.T - ts.xmax
        G[:self.N, 2:2 + self.m] = u - ts.umax
        G[:self.N, 2 + self.m:] = -u - ts.umax
        return G

    def c(self, x, u):
        """Equalities: c_0 = x0 - x_0, c_{i+1} = d(x_i, u_i) - x_{i+1}."""
        C = np.empty((self.N + 1, self.n))
        C[0] = self.x0 - x[0]
        d, _, _ = self.dyn(x[:-1], u)
        C[1:] = d - x[1:]
        return C

    def f(self, x, u):
        ts = self.ts
        ex = x - self.goal
        return (0.5 * ts.wx * np.sum(ex[:-1] ** 2) + 0.5 * ts.wu * np.sum(u ** 2)
                + 0.5 * ts.wN * np.sum(ex[-1] ** 2))

    def grad_f(self, x, u):
        ts = self.ts
        gx = ts.wx * (x - self.goal)
        gx[-1] = ts.wN * (x[-1] - self.goal)
        return gx, ts.wu * u

    def jac_c_T(self, x, u, w):
        """(J_c^T w) split into x and u parts, w (N+1, n)."""
        ts = self.ts
        _, th, sech2 = self.dyn(x[:-1], u)
        D = ts.dt * sech2 * w[1:]            # (N, n): dt sech^2 (.) w_{i+1}
        jx = np.zeros_like(x)
        jx[0] -= w[0]
        jx[:-1] += w[1:] + D @ ts.A           # (I + dt diag(sech2) A)^T w_{i+1}
        jx[1:] -= w[1:]
        ju = D @ ts.B
        return jx, ju

    def jac_g_T(self, w):
        """(G^T w) split into x and u parts, w (N+1, ng)."""
        w = w * self.mask
        return w @ self.Gx, w[:-1] @ self.Gu

    # ---- IPM quantities
    def e(self, u):
        """Stagewise equality residuals E_u u_i - b_i, (N, ne)."""
        return u @ self.Eu.T - self.eb

    def grad_L(self, st: State):
        gx, gu = self.grad_f(st.x, st.u)
        cx, cu = self.jac_c_T(st.x, st.u, st.y)
        zx, zu = self.jac_g_T(st.z)
        gu = gu + cu + zu
        if self.Eu is not None:
            gu = gu + st.ye @ self.Eu
        return gx + cx + zx, gu

    def errors(self, st: State, mu: Optional[float] = None):
        """(|grad L|, |c|, |g + s|, |s z - mu|) in the inf-norm; mu = 0 gives |s z|."""
        gx, gu = self.grad_L(st)
        c = self.c(st.x, st.u)
        gs = (self.g(st.x, st.u) + st.s) * self.mask
        sz = (st.s * st.z - (mu or 0.0)) * self.mask
        err = (max(np.abs(gx).max(), np.abs(gu).max() if gu.size else 0.0), np.abs(c).max(),
               np.abs(gs).max(), np.abs(sz).max())
        if self.Eu is not None and self.N:
            err = err + (np.abs(self.e(st.u)).max(),)
        return err

    def merit(self, x, u, s, st: State, mu: float):
        c = self.c(x, u)
        gs = (self.g(x, u) + s) * self.mask
        logs = np.sum(np.log(np.where(self.mask > 0, s, 1.0)))
        val = (self.f(x, u) - mu * logs + np.sum(st.y * c) + np.sum(st.z * gs)
               + 0.5 * ETA * (np.sum(c * c) + np.sum(gs * gs)))
        if self.Eu is not None:
            e = self.e(u)
            val += np.sum(st.ye * e) + 0.5 * ETA * np.sum(e * e)
        return val

    def merit_slope(self, st: State, mu, dx, du, ds):
        """Directional derivative of the merit along (dx, du, ds) at st (y, z fixed)."""
        c = self.c(st.x, st.u)
        gs = (self.g(st.x, st.u) + st.s) * self.mask
        gx, gu = self.grad_f(st.x, st.u)
        cx, cu = self.jac_c_T(st.x, st.u, st.y + ETA * c)
        zx, zu = self.jac_g_T(st.z + ETA * gs)
        dsg = (-mu / np.where(self.mask > 0, st.s, 1.0) + st.z + ETA * gs) * self.mask
        eu = 0.0
        if self.Eu is not None:
            eu = (st.ye + ETA * self.e(st.u)) @ self.Eu
        return np.sum((gx + cx + zx) * dx) + np.sum((gu + cu + zu + eu) * du) + np.sum(dsg * ds)

    def newton_lqr(self, st: State, mu: float, rho: float):
        """The dual-regularized LQR of the reduced Newton-KKT system, as an
        oracle Instance, plus the pieces needed to recover dz."""
        from paper_2509_16370_amd.workloads import Instance
        ts = self.ts
        n, m, N = self.n, self.m, self.N
        x, u = st.x, st.u
        _, th, sech2 = self.dyn(x[:-1], u)
        # Sigma = (W + Delta_G^{-1})^{-1}, W = S Z^{-1}; r_z = g + s + W (mu S^{-1} e - z) = g + mu / z
        zs = np.where(self.mask > 0, st.z, 1.0)
        Sig = self.mask / (np.where(self.mask > 0, st.s, 1.0) / zs + 1.0 / ETA)
        rz = (self.g(x, u) + mu / zs) * self.mask
        gx, gu = self.grad_L(st)
        AB = np.concatenate([ts.A, ts.B], axis=1)              # (n, n+m)
        Q = np.empty((N + 1, n, n))
        M = np.empty((N, n, m))
        R = np.empty((N, m, m))
        for i in range(N):
            wdd = ts.dt * st.y[i + 1] * (-2.0 * th[i] * sech2[i])   # second derivative weights
            H = AB.T @ (wdd[:, None] * AB)
            Q[i] = ts.wx * np.eye(n) + H[:n, :n] + self.Gx.T @ (Sig[i][:, None] * self.Gx) + rho * np.eye(n)
            M[i] = H[:n, n:] + self.Gx.T @ (Sig[i][:, None] * self.Gu)
            R[i] = ts.wu * np.eye(m) + H[n:, n:] + self.Gu.T @ (Sig[i][:, None] * self.Gu) + rho * np.eye(m)
        Q[N] = ts.wN * np.eye(n) + self.Gx.T @ (Sig[N][:, None] * self.Gx) + rho * np.eye(n)
        Q = 0.5 * (Q + np.swapaxes(Q, 1, 2))
        R = 0.5 * (R + np.swapaxes(R, 1, 2))
        Adyn = np.eye(n)[None] + ts.dt * sech2[:, :, None] * ts.A[None]
        Bdyn = ts.dt * sech2[:, :, None] * ts.B[None]
        q = gx + (Sig * rz) @ self.Gx
        r = gu + (Sig[:N] * rz[:N]) @ self.Gu
        if self.Eu is not None:  # the equality rows, eliminated through their -1/eta block
            R = R + ETA * (self.Eu.T @ self.Eu)[None]
            r = r + ETA * self.e(u) @ self.Eu
        c = self.c(x, u)
        inst = Instance(n, m, N, 1.0 / ETA, Q, M, R, Adyn, Bdyn, q, r, c)
        return inst, Sig, rz


def cold_start(p: Problem, mu0: float = 0.1) -> State:
    N, n, m = p.N, p.n, p.m
    x = np.tile(p.x0, (N + 1, 1))
    u = np.zeros((N, m))
    s = np.maximum(-p.g(x, u), 1e-2) * p.mask + (1 - p.mask)
    z = (mu0 / s) * p.mask
    ye = None if p.Eu is None else np.zeros((N, p.Eu.shape[0]))
    return State(x, u, np.zeros((N + 1, n)), s, z, mu0, ye=ye)


def warm_start(p: Problem, x, u, y, logz) -> State:
    """Initial point from a predicted trajectory: s = max(-g(x), 1e-2), z = exp(log z),
    mu0 = mean(s z) clipped to [1e-9, 0.1]."""
    s = np.maximum(-p.g(x, u), 1e-2) * p.mask + (1 - p.mask)
    z = np.exp(logz) * p.mask
    mu0 = float(np.clip(np.sum(s * z) / np.sum(p.mask), 1e-9, 0.1))
    ye = None if p.Eu is None else np.zeros((p.N, p.Eu.shape[0]))
    return State(x.copy(), u.copy(), y.copy(), s, z, mu0, ye=ye)


def frac_to_boundary(v, dv, tau, mask):
    neg = (dv < 0) & (mask > 0)
    if not neg.any():
        return 1.0
    return float(min(1.0, np.min(-tau * v[neg] / dv[neg])))


def direction(p: Problem, st: State, mu: float, rho: float):
    """Newton-KKT direction from the reduced dual-regularized LQR, with the
    inertia correction: rho grows until the pivot certificate holds.
    Returns (dx, du, dy, ds, dz, rho used)."""
    for _ in range(60):
        inst, Sig, rz = p.newton_lqr(st, mu, rho)
        sol = lqr_seq(inst)
        if sol["status"] == 0 and lqr_certificate(inst, sol["dS"], sol["dG"])[0]:
            break
        rho = max(1e-8, 10.0 * rho)
    dx, du, dy = sol["x"], sol["u"], sol["y"]
    dgx = dx @ p.Gx.T
    dgx[:-1] += du @ p.Gu.T
    dz = Sig * (dgx * p.mask + rz)                       # dz = (W + Delta_G^{-1})^{-1} (G dx + r_z)
    zs = np.where(p.mask > 0, st.z, 1.0)
    ds = (-(st.s / zs) * (dz + st.z) + mu / zs) * p.mask  # ds = -W (dz - mu S^{-1} e + z)
    return dx, du, dy, ds, dz, rho


def step(p: Problem, st: State, log=None) -> Dict:
    """One IPM iteration in place. Returns diagnostics."""
    mu = st.mu
    dx, du, dy, ds, dz, rho = direction(p, st, mu, st.rho)
    dye = None if p.Eu is None else ETA * (du @ p.Eu.T + p.e(st.u))
    tau = max(0.99, 1.0 - mu)
    a_s = frac_to_boundary(st.s, ds, tau, p.mask)
    a_z = frac_to_boundary(st.z, dz, tau, p.mask)
    m0 = p.merit(st.x, st.u, st.s, st, mu)
    slope = p.merit_slope(st, mu, dx, du, ds)
    a = a_s
    for k in range(LADDER):
        a = a_s * 0.5 ** k
        if p.merit(st.x + a * dx, st.u + a * du, st.s + a * ds, st, mu) <= m0 + C1 * a * slope:
            break
    st.x = st.x + a * dx
    st.u = st.u + a * du
    st.s = (st.s + a * ds) * p.mask + (1 - p.mask)
    st.y = st.y + dy
    if dye is not None:
        st.ye = st.ye + dye
    st.z = (st.z + a_z * dz) * p.mask
    st.rho = rho / 3.0
    err = p.errors(st, mu)
    if max(err) <= 10.0 * mu:
        st.mu = max(mu / 10.0, 1e-9)
    return dict(alpha=a, alpha_z=a_z, rho=rho, slope=slope, err=err)


def converged(p: Problem, st: State) -> bool:
    return max(p.errors(st, 0.0)) <= TOL


def solve(p: Problem, st: Optional[State] = None, max_iter: int = MAX_ITER):
    """Run the IPM to convergence; returns (state, iterations, converged)."""
    st = st or cold_start(p)
    for it in range(max_iter):
        if converged(p, st):
            return st, it, True
        step(p, st)
    return st, max_iter, converged(p, st)
