"""Seeded synthetic inputs for dual-regularized LQR problems.

This module only draws random problem data and packs it into the flat layout
that both the C-ABI library and the CPU oracle read. It holds none of the
solver's arithmetic (no Riccati step, no residual, no pivot test), so the GPU
path and the oracle can share it without sharing any of the method.

Problem data follow the dual-regularized LQR definition (Section "Dual-Regularized
LQR", Definition 1): stage blocks Q_i (n x n), M_i (n x m), R_i (m x m),
q_i, r_i, dynamics A_i (n x n), B_i (n x m), offsets c_0 .. c_N and the
regularization Delta_i = delta * I, or a positive diagonal Delta_i per stage
(`delta_diag`, (N+1, n); the definition allows any SPD Delta_i).

Flat layout (per instance, instances packed one after another, float64):

    Q : (N+1) * n * n     stage i is a row-major n x n block
    M : N * n * m         row-major n x m (cost term x^T M u)
    R : N * m * m
    A : N * n * n
    B : N * n * m
    q : (N+1) * n
    r : N * m
    c : (N+1) * n         c[0] is the initial-state target c_0,
                          c[i+1] the offset of the dynamics of step i
    x : (N+1) * n,  u : N * m,  y : (N+1) * n      (solution)
    delta_diag : (N+1) * n  (optional; laid out like x: the diagonal of Delta_i
                 at i * n; instances without one contribute delta repeated)

The element counts per instance are given by `counts(N, n, m)`; offsets are
exclusive prefix sums of those counts over the batch.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ARRAYS_LHS = ("Q", "M", "R", "A", "B")
ARRAYS_RHS = ("q", "r", "c")
ARRAYS_SOL = ("x", "u", "y")
ALL_ARRAYS = ARRAYS_LHS + ARRAYS_RHS + ARRAYS_SOL


def counts(N: int, n: int, m: int) -> Dict[str, int]:
    """Number of float64 elements each array holds for one instance."""
    return {
        "Q": (N + 1) * n * n, "M": N * n * m, "R": N * m * m,
        "A": N * n * n, "B": N * n * m,
        "q": (N + 1) * n, "r": N * m, "c": (N + 1) * n,
        "x": (N + 1) * n, "u": N * m, "y": (N + 1) * n,
    }


@dataclasses.dataclass
class Instance:
    """One dual-regularized LQR instance; arrays are stage-stacked."""
    n: int
    m: int
    N: int
    delta: float
    Q: np.ndarray  # (N+1, n, n)
    M: np.ndarray  # (N, n, m)
    R: np.ndarray  # (N, m, m)
    A: np.ndarray  # (N, n, n)
    B: np.ndarray  # (N, n, m)
    q: np.ndarray  # (N+1, n)
    r: np.ndarray  # (N, m)
    c: np.ndarray  # (N+1, n)
    indefinite: bool = False
    delta_diag: Optional[np.ndarray] = None  # (N+1, n): Delta_i = diag(delta_diag[i]); None: delta I
    delta_full: Optional[np.ndarray] = None  # (N+1, n, n): Delta_i any SPD matrix; overrides the others


def _rng(seed: Sequence[int]) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))


def _haar_orthogonal(rng: np.random.Generator, N: int, n: int) -> np.ndarray:
    g = rng.standard_normal((N, n, n))
    qm, rm = np.linalg.qr(g)
    s = np.sign(np.diagonal(rm, axis1=1, axis2=2))
    s[s == 0] = 1.0
    return qm * s[:, None, :]


def make_instance(n: int, m: int, N: int, delta: float, seed: Sequence[int],
                  indefinite: bool = False, diag_spread: Optional[float] = None,
                  spd_spread: Optional[float] = None) -> Instance:
    """Draw one instance with the stage recipe of the small single-instance workload.

    Recipe (all draws independent per stage, in this order):
      A_i = 0.95 * Haar-orthogonal + 0.05 * N(0,1)/sqrt(n)
      B_i ~ N(0,1)/sqrt(m)
      Q_i = W W^T / n + 1e-2 I,  W ~ N(0,1)   (i = 0..N, Q_N by the same recipe)
      R_i = V V^T / m + 1e-1 I,  V ~ N(0,1)
      M_i ~ N(0, 0.01^2)
      q_i ~ N(0,1) (i = 0..N),  r_i ~ N(0,1)
      c_0 ~ N(0,1),  c_1..c_N ~ N(0, 0.1^2)
    With indefinite=True every Q_i is shifted by -0.5 * lambda_max(Q_i) I.
    With diag_spread = s, Delta_i is diagonal with entries delta * 10^U(-s, s),
    drawn after everything else (the other data do not depend on s); they
    stand for separate penalty parameters per constraint.
    With spd_spread = s, Delta_i is a full SPD matrix delta * V_i diag(10^U(-s, s)) V_i^T
    with V_i Haar-orthogonal (drawn after everything else, per stage i = 0..N):
    penalties on combinations of the constraints (the definition allows any
    SPD Delta_i).
    """
    rng = _rng(seed)
    A = 0.95 * _haar_orthogonal(rng, N, n) + 0.05 * rng.standard_normal((N, n, n)) / np.sqrt(n)
    B = rng.standard_normal((N, n, m)) / np.sqrt(m)
    W = rng.standard_normal((N + 1, n, n))
    Q = W @ np.swapaxes(W, 1, 2) / n + 1e-2 * np.eye(n)
    V = rng.standard_normal((N, m, m))
    R = V @ np.swapaxes(V, 1, 2) / m + 1e-1 * np.eye(m)
    M = 0.01 * rng.standard_normal((N, n, m))
    q = rng.standard_normal((N + 1, n))
    r = rng.standard_normal((N, m))
    c = np.empty((N + 1, n))
    c[0] = rng.standard_normal(n)
    c[1:] = 0.1 * rng.standard_normal((N, n))
    if indefinite:
        lmax = np.linalg.eigvalsh(Q)[:, -1]
        Q = Q - 0.5 * lmax[:, None, None] * np.eye(n)
    # exact symmetry of the symmetric blocks
    Q = 0.5 * (Q + np.swapaxes(Q, 1, 2))
    R = 0.5 * (R + np.swapaxes(R, 1, 2))
    dd = None
    if diag_spread is not None:
        dd = float(delta) * 10.0 ** rng.uniform(-diag_spread, diag_spread, size=(N + 1, n))
    df = None
    if spd_spread is not None:
        Vd = _haar_orthogonal(rng, N + 1, n)
        ev = float(delta) * 10.0 ** rng.uniform(-spd_spread, spd_spread, size=(N + 1, n))
        df = (Vd * ev[:, None, :]) @ np.swapaxes(Vd, 1, 2)
        df = 0.5 * (df + np.swapaxes(df, 1, 2))
    return Instance(n, m, N, float(delta), Q, M, R, A, B, q, r, c, indefinite, dd, df)


# ---------------------------------------------------------------- workloads

def single_small(run: int = 0) -> List[Instance]:
    """One instance, n=4, m=2, N=32, delta=1e-6."""
    return [make_instance(4, 2, 32, 1e-6, (0, 0, run))]


def batched_uniform(batch: int = 4096, n: int = 12, m: int = 4, N: int = 128,
                    delta: float = 1e-8, run: int = 0) -> List[Instance]:
    """Uniform batch (quadrotor-sized: n=12, m=4, N=128), per-instance seeds."""
    return [make_instance(n, m, N, delta, (1, b, run)) for b in range(batch)]


def batched_ragged(batch: int = 1024, delta: float = 1e-4, run: int = 0,
                   n_choices=(8, 16, 32), m_choices=(2, 4, 8), N_range=(50, 1000),
                   indefinite_frac: float = 0.2) -> List[Instance]:
    """Ragged batch: N ~ U{50..1000}, n and m uniform over the choices,
    round(0.2*batch) instances (seeded permutation) with indefinite Q."""
    rng = _rng((2, 1 << 20, run))
    Ns = rng.integers(N_range[0], N_range[1] + 1, size=batch)
    ns = rng.choice(np.asarray(n_choices), size=batch)
    ms = rng.choice(np.asarray(m_choices), size=batch)
    n_indef = int(round(indefinite_frac * batch))
    indef = np.zeros(batch, dtype=bool)
    indef[rng.permutation(batch)[:n_indef]] = True
    return [make_instance(int(ns[b]), int(ms[b]), int(Ns[b]), delta, (2, b, run),
                          indefinite=bool(indef[b])) for b in range(batch)]


def long_horizon(N: int = 16384, n: int = 64, m: int = 32, delta: float = 1e-6,
                 run: int = 0) -> List[Instance]:
    """One long-horizon instance (n=64, m=32, N=16384 at full size)."""
    return [make_instance(n, m, N, delta, (3, 0, run))]


# ---------------------------------------------------------------- packing

@dataclasses.dataclass
class Packed:
    """A batch in the flat layout: shapes (int32) + one float64 array per name."""
    N: np.ndarray
    n: np.ndarray
    m: np.ndarray
    delta: np.ndarray
    arrays: Dict[str, np.ndarray]
    offsets: Dict[str, np.ndarray]  # name -> int64[B+1]

    @property
    def batch(self) -> int:
        return int(self.N.shape[0])

    def stage_count(self) -> int:
        return int(self.N.sum())


def layout_offsets(N, n, m) -> Dict[str, np.ndarray]:
    N = np.asarray(N, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    m = np.asarray(m, dtype=np.int64)
    per = {
        "Q": (N + 1) * n * n, "M": N * n * m, "R": N * m * m,
        "A": N * n * n, "B": N * n * m,
        "q": (N + 1) * n, "r": N * m, "c": (N + 1) * n,
        "x": (N + 1) * n, "u": N * m, "y": (N + 1) * n,
    }
    out = {}
    for k, v in per.items():
        o = np.zeros(len(N) + 1, dtype=np.int64)
        np.cumsum(v, out=o[1:])
        out[k] = o
    return out


def pack(instances: List[Instance]) -> Packed:
    N = np.array([i.N for i in instances], dtype=np.int32)
    n = np.array([i.n for i in instances], dtype=np.int32)
    m = np.array([i.m for i in instances], dtype=np.int32)
    delta = np.array([i.delta for i in instances], dtype=np.float64)
    offs = layout_offsets(N, n, m)
    arrays = {}
    for name in ARRAYS_LHS + ARRAYS_RHS:
        arrays[name] = np.concatenate(
            [getattr(i, name).reshape(-1) for i in instances]).astype(np.float64)
        assert arrays[name].shape[0] == offs[name][-1]
    if any(i.delta_diag is not None for i in instances):
        arrays["delta_diag"] = _pack_diag(instances)
        assert arrays["delta_diag"].shape[0] == offs["x"][-1]
    if any(i.delta_full is not None for i in instances):
        arrays["delta_full"] = _pack_full(instances)
        assert arrays["delta_full"].shape[0] == offs["Q"][-1]
    return Packed(N, n, m, delta, arrays, offs)


def _pack_full(instances: List[Instance]) -> np.ndarray:
    """Full Delta_i of every instance, laid out like Q ((N+1) n n per
    instance); an instance without them contributes its delta I (or its
    per-stage diagonal)."""
    parts = []
    for i in instances:
        if i.delta_full is not None:
            parts.append(np.asarray(i.delta_full, dtype=np.float64).reshape(-1))
        elif i.delta_diag is not None:
            parts.append(np.stack([np.diag(d) for d in i.delta_diag]).reshape(-1))
        else:
            parts.append(np.tile(i.delta * np.eye(i.n), (i.N + 1, 1, 1)).reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0)


def _pack_diag(instances: List[Instance]) -> np.ndarray:
    return np.concatenate([
        (i.delta_diag if i.delta_diag is not None else np.full((i.N + 1, i.n), i.delta)).reshape(-1)
        for i in instances]).astype(np.float64)


def unpack_solution(p: Packed, x: np.ndarray, u: np.ndarray, y: np.ndarray):
    """Split flat x, u, y into per-instance (N+1,n), (N,m), (N+1,n) arrays."""
    out = []
    for b in range(p.batch):
        N, n, m = int(p.N[b]), int(p.n[b]), int(p.m[b])
        ox, ou, oy = p.offsets["x"][b], p.offsets["u"][b], p.offsets["y"][b]
        out.append((x[ox:ox + (N + 1) * n].reshape(N + 1, n),
                    u[ou:ou + N * m].reshape(N, m),
                    y[oy:oy + (N + 1) * n].reshape(N + 1, n)))
    return out


# ---------------------------------------------------------------- parallel packing

def _pack_chunk(specs):
    p = pack([make_instance(*s) for s in specs])
    return p.N, p.n, p.m, p.delta, p.arrays


def uniform_specs(batch=4096, n=12, m=4, N=128, delta=1e-8, run=0, cfg_id=1):
    """Specs (n, m, N, delta, seed) of `batched_uniform`, for `pack_parallel`."""
    return [(n, m, N, delta, (cfg_id, b, run)) for b in range(batch)]


def pack_parallel(specs, workers: int = 8) -> Packed:
    """Generate and pack instances given as make_instance argument tuples, in
    worker processes; identical to pack([make_instance(*s) for s in specs])."""
    import concurrent.futures as cf
    workers = max(1, min(workers, len(specs)))
    if workers == 1 or len(specs) < 64:
        return pack([make_instance(*s) for s in specs])
    chunk = (len(specs) + workers - 1) // workers
    parts = [specs[i:i + chunk] for i in range(0, len(specs), chunk)]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(_pack_chunk, parts))
    N = np.concatenate([r[0] for r in res])
    n = np.concatenate([r[1] for r in res])
    m = np.concatenate([r[2] for r in res])
    delta = np.concatenate([r[3] for r in res])
    keys = list(ARRAYS_LHS + ARRAYS_RHS)
    if any("delta_diag" in r[4] for r in res):
        if not all("delta_diag" in r[4] for r in res):
            raise ValueError("pack_parallel: mix of chunks with and without delta_diag")
        keys.append("delta_diag")
    arrays = {k: np.concatenate([r[4][k] for r in res]) for k in keys}
    return Packed(N, n, m, delta, arrays, layout_offsets(N, n, m))


# ---------------------------------------------------------------- stagewise equality constraints

@dataclasses.dataclass
class StageEq:
    """ne equality rows per stage for one instance (no solver arithmetic):
    Jacobians E_i = [Ex_i | Eu_i] (stage N: Ex only), residuals r_e and the
    penalties eta (the dual regularization is 1 / eta)."""
    ne: int
    Ex: np.ndarray   # (N+1, ne, n)
    Eu: np.ndarray   # (N, ne, m)
    r: np.ndarray    # (N+1, ne)
    eta: np.ndarray  # (N+1, ne) > 0


def make_stage_eq(inst: Instance, ne: int, seed: Sequence[int], eta: float = 1e3) -> StageEq:
    """Draw ne stagewise equality rows for every stage of `inst`.

    Recipe (in this order, from their own seed stream): Ex_i ~ N(0,1)/sqrt(n+m),
    Eu_i ~ N(0,1)/sqrt(n+m), r_e ~ N(0, 0.1^2), penalties eta * 10^U(-1, 1)
    (one penalty per constraint, as the regularized IPM allows).
    """
    rng = _rng(list(seed) + [5])
    n, m, N = inst.n, inst.m, inst.N
    Ex = rng.standard_normal((N + 1, ne, n)) / np.sqrt(n + m)
    Eu = rng.standard_normal((N, ne, m)) / np.sqrt(n + m)
    r = 0.1 * rng.standard_normal((N + 1, ne))
    pen = eta * 10.0 ** rng.uniform(-1.0, 1.0, size=(N + 1, ne))
    return StageEq(ne, Ex, Eu, r, pen)


def pack_stage_eq(packed: Packed, eqs: List[StageEq]) -> Dict[str, np.ndarray]:
    """Flat arrays of the batch's equality rows. Per instance: E stage-stacked
    (stage i < N an ne x (n+m) row-major block [Ex_i | Eu_i], stage N an
    ne x n block), r and eta (N+1) * ne each; offsets by exclusive prefix
    sums (`E_off`, `v_off`)."""
    E, r, eta = [], [], []
    e_off = [0]
    v_off = [0]
    for b, eq in enumerate(eqs):
        N = int(packed.N[b])
        blocks = [np.concatenate([eq.Ex[i], eq.Eu[i]], axis=1).reshape(-1) for i in range(N)]
        blocks.append(eq.Ex[N].reshape(-1))
        E.append(np.concatenate(blocks) if blocks else np.zeros(0))
        r.append(eq.r.reshape(-1))
        eta.append(eq.eta.reshape(-1))
        e_off.append(e_off[-1] + E[-1].size)
        v_off.append(v_off[-1] + r[-1].size)
    return {"E": np.concatenate(E).astype(np.float64), "r": np.concatenate(r).astype(np.float64),
            "eta": np.concatenate(eta).astype(np.float64),
            "E_off": np.asarray(e_off, dtype=np.int64), "v_off": np.asarray(v_off, dtype=np.int64)}


# ---------------------------------------------------------------- cross-stage variables

@dataclasses.dataclass
class CrossStage:
    """Data of p cross-stage variables for one instance (no solver arithmetic):
    the columns of J_theta in the layout of an LQR right-hand side, H_theta_theta
    and r_theta."""
    J: List[Tuple[np.ndarray, np.ndarray, np.ndarray]]  # p x (Jq (N+1,n), Jr (N,m), Jc (N+1,n))
    H: np.ndarray    # (p, p) symmetric
    rth: np.ndarray  # (p,)


def make_cross_stage(inst: Instance, p: int, seed: Sequence[int], indefinite: bool = False) -> CrossStage:
    """Draw J, H, r_theta for p variables shared by every stage of `inst`.

    Recipe (in this order, from their own seed stream):
      Jq, Jr ~ 0.5 N(0,1)/sqrt(T), T = (N+1) n + N m (the variables enter
        every stage's cost; each column has norm about 0.5),
      Jc ~ 0.05 N(0,1)/sqrt(T) (and, weakly, every step's dynamics),
      H = W W^T / p + I, W ~ N(0,1) (p x p); with indefinite=True, H <- -H,
      r_theta ~ N(0,1).
    The column scale keeps J^T K^{-1} J of order 0.1-1 at any horizon and
    size: S = H - J^T K^{-1} J is usually, not always, positive definite."""
    n, m, N = inst.n, inst.m, inst.N
    rng = _rng(tuple(seed) + (17,))
    sc = 0.5 / np.sqrt((N + 1.0) * n + N * m)
    J = []
    for _ in range(p):
        Jq = sc * rng.standard_normal((N + 1, n))
        Jr = sc * rng.standard_normal((N, m))
        Jc = 0.1 * sc * rng.standard_normal((N + 1, n))
        J.append((Jq, Jr, Jc))
    W = rng.standard_normal((p, p))
    H = W @ W.T / p + np.eye(p)
    if indefinite:
        H = -H
    H = 0.5 * (H + H.T)
    rth = rng.standard_normal(p)
    return CrossStage(J, H, rth)


def pack_cross_stage(packed: Packed, xs: List[CrossStage]) -> Dict[str, np.ndarray]:
    """Stack the cross-stage data of a packed batch (all instances share p):
    column j of J occupies [j*L, (j+1)*L) of Jq / Jr / Jc (L = the batch's
    q / r / c length, instances at their usual offsets); H is (B, p, p) and
    r_theta (B, p), flattened."""
    B = packed.batch
    p = len(xs[0].J) if B else 0
    out = {}
    for k, name in enumerate(("q", "r", "c")):
        L = int(packed.offsets[name][-1])
        a = np.zeros(p * L)
        for b in range(B):
            o0, o1 = packed.offsets[name][b], packed.offsets[name][b + 1]
            for j in range(p):
                a[j * L + o0:j * L + o1] = xs[b].J[j][k].reshape(-1)
        out["J" + name] = a
    out["H"] = np.concatenate([x.H.reshape(-1) for x in xs]) if B else np.zeros(0)
    out["rth"] = np.concatenate([x.rth for x in xs]) if B else np.zeros(0)
    return out


# ---------------------------------------------------------------- constrained trajectory problems

@dataclasses.dataclass
class TrajectorySet:
    """Constrained trajectory problems sharing one model (no solver arithmetic here).

    For each problem b: minimize
        sum_{i<N} 1/2 wx |x_i - goal_b|^2 + 1/2 wu |u_i|^2 + 1/2 wN |x_N - goal_b|^2
    subject to x_0 = x0_b, x_{i+1} = x_i + dt * tanh(A x_i + B u_i),
    a_j^T x_i <= xmax (j = 1, 2; every stage i = 0..N) and |u_i| <= umax (componentwise).
    """
    n: int
    m: int
    N: int
    dt: float
    A: np.ndarray      # (n, n)
    B: np.ndarray      # (n, m)
    a: np.ndarray      # (2, n) unit normals of the state half-spaces
    x0: np.ndarray     # (batch, n)
    goal: np.ndarray   # (batch, n)
    wx: float = 1.0
    wu: float = 0.1
    wN: float = 10.0
    xmax: float = 1.5
    umax: float = 1.0

    @property
    def batch(self) -> int:
        return int(self.x0.shape[0])

    def take(self, ids) -> "TrajectorySet":
        ids = np.asarray(ids)
        return dataclasses.replace(self, x0=self.x0[ids].copy(), goal=self.goal[ids].copy())


def trajectory_model(n: int = 12, m: int = 4, seed: int = 0):
    """Shared model: A = -I + 0.5 (W - W^T) / sqrt(n) with W ~ N(0,1) (a damped
    rotation, so the uncontrolled flow is stable), B ~ N(0,1)/sqrt(m), and two
    seeded unit normals a_1, a_2 of the state half-spaces."""
    rng = _rng((4, 0, seed))
    W = rng.standard_normal((n, n))
    A = -np.eye(n) + 0.5 * (W - W.T) / np.sqrt(n)
    B = rng.standard_normal((n, m)) / np.sqrt(m)
    a = rng.standard_normal((2, n))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    return A, B, a


def trajectory_problems(count: int, N: int = 256, n: int = 12, m: int = 4, dt: float = 0.05,
                        stream: int = 0, model_seed: int = 0, margin: float = 0.1,
                        xmax: float = 0.5, first: int = 0) -> TrajectorySet:
    """`count` (x0, goal) pairs. x0 ~ N(0, 0.5^2 I); goal = -A^{-1} B u_g with
    u_g ~ U(-0.5, 0.5)^m, a steady state of the dynamics held by an admissible
    control; both rejection-sampled so that a_j^T v <= xmax - margin. Streams:
    0 = evaluation pairs, 1 = training pairs (disjoint seed streams). Problems
    first .. first + count - 1 of the stream are returned."""
    A, B, a = trajectory_model(n, m, model_seed)
    Ainv_B = np.linalg.solve(A, B)
    x0 = np.empty((count, n))
    goal = np.empty((count, n))
    for b in range(count):  # problem b depends only on (stream, model_seed, b)
        rng = _rng((4, 2 + stream, model_seed, first + b))
        while True:
            v = 0.5 * rng.standard_normal(n)
            if (a @ v <= xmax - margin).all():
                x0[b] = v
                break
        while True:
            v = -Ainv_B @ rng.uniform(-0.5, 0.5, m)
            if (a @ v <= xmax - margin).all():
                goal[b] = v
                break
    return TrajectorySet(n, m, N, dt, A, B, a, x0, goal, xmax=xmax)
