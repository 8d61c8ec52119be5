"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check goes against a
printed example, a textbook routine (DARE), a reduction to a different
problem, the dense definition, or an identity the paper proves.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle import dense
from paper_2509_16370_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _inst_from_json(d, q=None, r=None, c=None):
    n, m, N = d["n"], d["m"], d["N"]
    arr = lambda k, shape: np.asarray(d[k], dtype=np.float64).reshape(shape)
    return wl.Instance(
        n, m, N, float(d["delta"]),
        arr("Q", (N + 1, n, n)), arr("M", (N, n, m)), arr("R", (N, m, m)),
        arr("A", (N, n, n)), arr("B", (N, n, m)),
        np.asarray(d["q"], float).reshape(N + 1, n) if "q" in d else (q if q is not None else np.zeros((N + 1, n))),
        np.asarray(d["r"], float).reshape(N, m) if "r" in d else (r if r is not None else np.zeros((N, m))),
        np.asarray(d["c"], float).reshape(N + 1, n) if "c" in d else (c if c is not None else np.zeros((N + 1, n))),
    )


def _tiny(seed, n=3, m=2, N=5, delta=1e-4, indefinite=False):
    return wl.make_instance(n, m, N, delta, (99, seed, 0), indefinite=indefinite)


def _solution_close(a, b, tol):
    for va, vb in zip(a, b):
        scale = max(1.0, np.abs(vb).max())
        assert np.abs(np.asarray(va) - np.asarray(vb)).max() <= tol * scale


# ----------------------------------------------------------------- P1 example

def test_example_newton_kkt_reproduced():
    g = json.load(open(os.path.join(GOLD, "example_newton_kkt_descent.json")))
    inst = _inst_from_json(g["lqr"])
    K, rhs = dense.assemble(inst)
    # the reading of the example reproduces the printed system exactly
    assert np.array_equal(K, np.asarray(g["printed_matrix"], float))
    assert np.array_equal(rhs, np.asarray(g["printed_rhs"], float))
    z_ref = np.asarray(g["printed_solution"], float)
    assert np.allclose(np.linalg.solve(K, rhs), z_ref, atol=1e-14)
    for out in (oracle.seq(inst), oracle.par(inst, 0, 0), oracle.par(inst, 1, 1)):
        assert out["status"] == 0
        z = dense.join(inst, out["x"], out["u"], out["y"])
        assert np.allclose(z, z_ref, atol=1e-14)
    # intermediate values stated for this example: P_1 = 1, G_0 = 2, K_0 = -1/2, P_0 = 3/2, p_0 = 0
    o = oracle.seq(inst)
    assert np.isclose(o["P"][1, 0, 0], 1.0) and np.isclose(o["dG"][0, 0], 2.0)
    assert np.isclose(o["K"][0, 0, 0], -0.5) and np.isclose(o["P"][0, 0, 0], 1.5)
    assert abs(o["p"][0, 0]) < 1e-15


# ----------------------------------------------------------- P2/P3 inertia example

def test_example_indefinite_R_inertia():
    g = json.load(open(os.path.join(GOLD, "example_indefinite_R_inertia.json")))
    inst = _inst_from_json(g["lqr"])
    K, _ = dense.assemble(inst)
    nxp = inst.N * (inst.n + inst.m) + inst.n
    P = K[:nxp, :nxp]
    C = K[nxp:, :nxp]
    assert np.array_equal(P, np.asarray(g["printed_P"], float))
    assert np.array_equal(C, np.asarray(g["printed_C"], float))
    PC = P + C.T @ C
    assert np.array_equal(PC, np.asarray(g["printed_P_plus_CtC"], float))
    minors = [np.linalg.det(PC[:k, :k]) for k in (1, 2, 3)]
    assert np.allclose(minors, g["printed_leading_minors"])
    assert dense.inertia_eig(K) == tuple(g["printed_inertia"])
    assert dense.inertia_ldl(K) == tuple(g["printed_inertia"])
    o = oracle.seq(inst)
    verdict, first_bad, inertia = oracle.certificate(inst, o["dS"], o["dG"])
    assert verdict and first_bad == -1 and inertia == tuple(g["printed_inertia"])
    # pivots S_hat_1 = 1 + 1*1 = 2, G_0 = -1 + 4 * W_1 = -1 + 4 * 0.5 = 1, S_hat_0 = 2;
    # with Delta = 1 the product equals det(P + C^T C) = 4
    assert np.allclose([o["dS"][1, 0], o["dG"][0, 0], o["dS"][0, 0]], [2.0, 1.0, 2.0])
    assert np.isclose(np.prod(o["dS"]) * np.prod(o["dG"]), np.linalg.det(PC))


def test_example_variants_false_verdict_and_singular():
    g = json.load(open(os.path.join(GOLD, "example_indefinite_R_inertia.json")))
    d = dict(g["lqr"])
    d["R"] = [[[-3.0]]]      # G_0 = -3 + 2 = -1: solvable, wrong inertia
    inst = _inst_from_json(d, q=np.array([[0.3], [-0.2]]), r=np.array([[0.5]]), c=np.array([[1.0], [0.2]]))
    K, rhs = dense.assemble(inst)
    assert dense.inertia_eig(K) == (2, 3, 0)
    o = oracle.seq(inst)
    assert o["status"] == 0
    verdict, first_bad, inertia = oracle.certificate(inst, o["dS"], o["dG"])
    assert not verdict and first_bad == 1 and inertia == (2, 3, 0)
    # the recursion still returns the unique KKT solution (Theorem on the rational identity)
    _solution_close((o["x"], o["u"], o["y"]), dense.split(inst, np.linalg.solve(K, rhs)), 1e-13)
    d["R"] = [[[-2.0]]]      # G_0 = 0: the KKT matrix is singular
    inst = _inst_from_json(d)
    K, _ = dense.assemble(inst)
    assert dense.inertia_eig(K) == (2, 2, 1)
    assert oracle.seq(inst)["status"] == 1


# ------------------------------------------------------- P4 delta = 0 -> DARE

def test_delta_zero_time_invariant_reaches_dare():
    rng = np.random.default_rng(4)
    n, m, N = 4, 2, 400
    base = wl.make_instance(n, m, 1, 0.0, (4, 0, 0))
    A, B, Q, R = base.A[0], base.B[0], base.Q[0], base.R[0]
    inst = wl.Instance(n, m, N, 0.0, np.repeat(Q[None], N + 1, 0), np.zeros((N, n, m)),
                       np.repeat(R[None], N, 0), np.repeat(A[None], N, 0), np.repeat(B[None], N, 0),
                       rng.standard_normal((N + 1, n)), rng.standard_normal((N, m)),
                       np.zeros((N + 1, n)))
    X = scipy.linalg.solve_discrete_are(A, B, Q, R)
    o = oracle.seq(inst)
    assert np.abs(o["P"][0] - X).max() <= 1e-10 * np.abs(X).max()
    op = oracle.par(inst, 1, 1)
    assert np.abs(op["P"][0] - X).max() <= 1e-10 * np.abs(X).max()
    # textbook gain K = -(R + B^T X B)^{-1} B^T X A
    Kd = -np.linalg.solve(R + B.T @ X @ B, B.T @ X @ A)
    assert np.abs(o["K"][0] - Kd).max() <= 1e-10 * max(1, np.abs(Kd).max())


# ----------------------------- P5 delta > 0 == standard LQR with augmented control

def _augment(inst):
    """Standard (delta = 0) LQR whose solution carries the delta > 0 solution:
    one pre-stage sets x_0 = c_0 + w_{-1}, every dynamics step gets an extra
    control w_i entering with identity and costing (1/2) w^T Delta^{-1} w."""
    n, m, N, d = inst.n, inst.m, inst.N, inst.delta
    ma = m + n
    Q = np.zeros((N + 2, n, n)); M = np.zeros((N + 1, n, ma)); R = np.zeros((N + 1, ma, ma))
    A = np.zeros((N + 1, n, n)); B = np.zeros((N + 1, n, ma))
    q = np.zeros((N + 2, n)); r = np.zeros((N + 1, ma)); c = np.zeros((N + 2, n))
    Q[0] = np.eye(n)
    R[0, :m, :m] = np.eye(m); R[0, m:, m:] = np.eye(n) / d
    B[0, :, m:] = np.eye(n)
    c[1] = inst.c[0]
    for i in range(N):
        Q[i + 1] = inst.Q[i]; M[i + 1, :, :m] = inst.M[i]
        R[i + 1, :m, :m] = inst.R[i]; R[i + 1, m:, m:] = np.eye(n) / d
        A[i + 1] = inst.A[i]; B[i + 1, :, :m] = inst.B[i]; B[i + 1, :, m:] = np.eye(n)
        q[i + 1] = inst.q[i]; r[i + 1, :m] = inst.r[i]; c[i + 2] = inst.c[i + 1]
    Q[N + 1] = inst.Q[N]; q[N + 1] = inst.q[N]
    return wl.Instance(n, ma, N + 1, 0.0, Q, M, R, A, B, q, r, c)


@pytest.mark.parametrize("delta", [1e-2, 1e-1, 1.0])
def test_delta_positive_equals_augmented_standard_lqr(delta):
    inst = _tiny(5, n=3, m=2, N=6, delta=delta)
    aug = _augment(inst)
    oa = oracle.seq(aug)
    assert oa["status"] == 0
    # the augmented reduction is itself checked densely
    _solution_close((oa["x"], oa["u"], oa["y"]), dense.solve(aug), 1e-11)
    o = oracle.seq(inst)
    n, m = inst.n, inst.m
    _solution_close((o["x"],), (oa["x"][1:],), 1e-11)
    _solution_close((o["u"],), (oa["u"][1:, :m],), 1e-11)
    # y_{i+1} = -Delta^{-1} w_i and y_0 = -Delta^{-1} w_{-1}
    y_from_w = -oa["u"][:, m:] / delta
    _solution_close((o["y"],), (y_from_w,), 1e-10)


# ----------------------------------------------------- P6 whole solve vs dense

@pytest.mark.parametrize("delta", [0.0, 1e-8, 1e-4, 0.1, 1.0])
@pytest.mark.parametrize("indef", [False, True])
def test_seq_and_par_match_dense(delta, indef):
    for seed in range(6):
        n, m, N = [(3, 2, 5), (4, 1, 7), (2, 3, 4), (4, 3, 8), (1, 1, 3), (3, 3, 1)][seed]
        inst = _tiny(seed, n, m, N, delta, indefinite=indef)
        K, rhs = dense.assemble(inst)
        if np.linalg.cond(K) > 1e10:
            continue
        ref = dense.split(inst, np.linalg.solve(K, rhs))
        o = oracle.seq(inst)
        assert o["status"] == 0
        _solution_close((o["x"], o["u"], o["y"]), ref, 1e-10)
        for br, pm in ((0, 0), (1, 0), (1, 1)):
            op = oracle.par(inst, br, pm)
            assert op["status"] == 0
            _solution_close((op["x"], op["u"], op["y"]), ref, 1e-9)


# ------------------------------------------------ P7 / P12 parallel == sequential

@pytest.mark.parametrize("delta", [0.0, 1e-6, 1e-2])
def test_par_matches_seq_factors(delta):
    inst = wl.make_instance(5, 3, 37, delta, (7, 1, 0))
    o = oracle.seq(inst)
    for br in (0, 1):
        for pm in (0, 1):
            op = oracle.par(inst, br, pm)
            for key in ("P", "p", "K", "k", "x", "u", "y", "dS", "dG"):
                s = max(1.0, np.abs(o[key]).max())
                assert np.abs(op[key] - o[key]).max() <= 1e-11 * s, key


def test_p_combine_equals_p_recurrence():
    inst = wl.make_instance(4, 2, 21, 1e-3, (8, 0, 0))
    a = oracle.par(inst, 1, 0)["p"]
    b = oracle.par(inst, 1, 1)["p"]
    assert np.abs(a - b).max() <= 1e-11 * max(1, np.abs(a).max())


# ------------------------------------------------------------ P8 inertia

@pytest.mark.parametrize("delta", [1e-4, 1e-2, 1.0])
def test_certificate_matches_dense_inertia(delta):
    agree = 0
    nonpd = 0
    for seed in range(40):
        inst = _tiny(100 + seed, n=3, m=2, N=4, delta=delta, indefinite=(seed % 2 == 1))
        K, _ = dense.assemble(inst)
        o = oracle.seq(inst)
        if o["status"]:
            continue
        verdict, first_bad, inertia = oracle.certificate(inst, o["dS"], o["dG"])
        ie = dense.inertia_eig(K)
        assert inertia == ie == dense.inertia_ldl(K)
        assert verdict == (ie == dense.target_inertia(inst))
        nonpd += (not verdict)
        agree += 1
    assert agree >= 35 and nonpd >= 5  # non-vacuous on both sides


def test_certificate_determinant_identity():
    inst = _tiny(7, n=3, m=2, N=5, delta=1e-2, indefinite=True)
    K, _ = dense.assemble(inst)
    nxp = inst.N * (inst.n + inst.m) + inst.n
    P, C = K[:nxp, :nxp], K[nxp:, :nxp]
    red = P + C.T @ C / inst.delta
    o = oracle.seq(inst)
    # det S_i = det(S_hat_i) / delta^n with S_i = P_i + Delta^{-1}
    sign_d, logdet = np.linalg.slogdet(red)
    piv = np.concatenate([o["dS"].ravel() / inst.delta, o["dG"].ravel()])
    assert sign_d == np.prod(np.sign(piv))
    assert np.isclose(logdet, np.sum(np.log(np.abs(piv))), rtol=1e-10)


def test_delta_zero_verdict_is_control_pivots_only():
    for seed in range(30):
        inst = _tiny(300 + seed, n=3, m=2, N=4, delta=0.0, indefinite=(seed % 2 == 0))
        K, _ = dense.assemble(inst)
        o = oracle.seq(inst)
        if o["status"]:
            continue
        assert np.all(o["dS"] == 1.0)  # S_hat = I at delta = 0
        verdict, _, inertia = oracle.certificate(inst, o["dS"], o["dG"])
        assert inertia == dense.inertia_eig(K)
        assert verdict == bool(np.all(o["dG"] > 0))


# ------------------------------------------------------------ P9 residual

def test_residual_equals_dense_matrix_product():
    inst = _tiny(11, n=3, m=2, N=6, delta=1e-3)
    K, rhs = dense.assemble(inst)
    rng = np.random.default_rng(0)
    z = rng.standard_normal(K.shape[0])
    x, u, y = dense.split(inst, z)
    res = oracle.residual(inst, x, u, y)
    assert np.allclose(res, K @ z - rhs, atol=1e-13)
    z0 = np.linalg.solve(K, rhs)
    x, u, y = dense.split(inst, z0)
    assert oracle.rel_residual(inst, x, u, y) < 1e-13


# ------------------------------------------------------- P10 associativity

def _rand_elem(rng, n):
    G = rng.standard_normal((n, n)); P = G @ G.T / n
    H = rng.standard_normal((n, n)); C = H @ H.T / n + 1e-3 * np.eye(n)
    return (P, rng.standard_normal(n), rng.standard_normal((n, n)) / np.sqrt(n), C, rng.standard_normal(n))


def test_combine_associative():
    rng = np.random.default_rng(1)
    n = 4
    for _ in range(5):
        a, b, c = (_rand_elem(rng, n) for _ in range(3))
        left = oracle.combine(n, oracle.combine(n, a, b), c)
        right = oracle.combine(n, a, oracle.combine(n, b, c))
        for l, r in zip(left, right):
            assert np.abs(l - r).max() <= 1e-12 * max(1, np.abs(l).max())


def test_combine_with_terminal_is_riccati_step():
    """(i -> i+1) (+) (terminal) has P = A^T P_N (I + C P_N)^{-1} A + P_{i->i+1}:
    for M = 0 this is Q + A^T (P_N^{-1} + B R^{-1} B^T + Delta)^{-1} A (Woodbury)."""
    rng = np.random.default_rng(2)
    n, m = 3, 2
    inst = wl.make_instance(n, m, 1, 0.05, (9, 0, 0))
    Q0, R0, A0, B0, QN = inst.Q[0], inst.R[0], inst.A[0], inst.B[0], inst.Q[1]
    C = B0 @ np.linalg.solve(R0, B0.T) + 0.05 * np.eye(n)
    e0 = (Q0, np.zeros(n), A0, C, np.zeros(n))
    eN = (QN, np.zeros(n), np.zeros((n, n)), np.zeros((n, n)), np.zeros(n))
    P = oracle.combine(n, e0, eN)[0]
    expect = Q0 + A0.T @ np.linalg.inv(np.linalg.inv(QN) + C) @ A0
    assert np.allclose(P, expect, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------- P11 structure

def test_value_function_hessians_psd_for_psd_data():
    inst = wl.make_instance(4, 2, 30, 1e-3, (10, 0, 0))
    inst.M[:] = 0.0  # Q, R PSD, M = 0 -> the stage Hessians are PSD
    o = oracle.seq(inst)
    for P in o["P"]:
        assert np.array_equal(P, P.T)
        assert np.linalg.eigvalsh(P).min() >= -1e-12 * np.abs(P).max()


# ------------------------------------------------------- P13 delta -> 0

def test_delta_to_zero_continuity():
    inst0 = wl.make_instance(3, 2, 10, 0.0, (12, 0, 0))
    o0 = oracle.seq(inst0)
    for d in (1e-6, 1e-9, 1e-12):
        inst = wl.make_instance(3, 2, 10, d, (12, 0, 0))
        o = oracle.seq(inst)
        err = max(np.abs(o[k] - o0[k]).max() for k in ("x", "u", "y"))
        assert err <= 1e3 * d + 1e-12


def test_batch_pivots_give_dense_inertia():
    """The batch driver's pivots (every instance of a ragged batch, PD and
    indefinite, delta = 0 included) give the eigenvalue inertia of each
    instance's dense KKT matrix, and equal the single-instance pivots."""
    rng = np.random.default_rng(23)
    insts = []
    for i in range(24):
        n, m = int(rng.integers(2, 5)), int(rng.integers(1, 4))
        N = int(rng.integers(0, 7))
        delta = float(rng.choice([0.0, 1e-4, 0.1]))
        insts.append(wl.make_instance(n, m, N, delta, (94, i, 0), indefinite=bool(i % 2 == 1)))
    packed = wl.pack(insts)
    x, u, y, st, _, dS, dG = oracle.seq_batch(packed, nthreads=2, pivots=True)
    certs = oracle.certificate_batch(packed, insts, dS, dG)
    nfalse = 0
    for b, inst in enumerate(insts):
        ref = oracle.seq(inst)
        assert st[b] == ref["status"]
        o = packed.offsets
        assert np.array_equal(dS[o["x"][b]:o["x"][b + 1]], ref["dS"].ravel())
        assert np.array_equal(dG[o["u"][b]:o["u"][b + 1]], ref["dG"].ravel())
        if ref["status"]:
            continue
        verdict, first_bad, inertia = certs[b]
        K, _ = dense.assemble(inst)
        assert inertia == dense.inertia_eig(K), b
        assert verdict == (inertia == dense.target_inertia(inst))
        nfalse += not verdict
    assert nfalse >= 3
