"""Pins of the oracle's general SPD per-stage regularization Delta_i
(oracle/spd.py; Definition in Section "Dual-Regularized LQR": any SPD
Delta_i).

Each pin ties the oracle to something other than itself:
  * the dense KKT system with the full blocks -Delta_i (the plain definition),
    and its residual K z + [s; c] at an arbitrary z;
  * a congruence to Delta = I: with Delta_i = L_i L_i^T (Cholesky), the change
    of variables x = L_i x~, y = L_i^{-T} y~ maps the problem to one with
    Delta = I and data A~_i = L_{i+1}^{-1} A_i L_i, B~_i = L_{i+1}^{-1} B_i,
    Q~_i = L_i^T Q_i L_i, M~_i = L_i^T M_i, q~_i = L_i^T q_i, c~_i =
    L_i^{-1} c_i (R, r unchanged), solved by the C oracle's scalar path (pinned
    on its own); its P~_i = L_i^T P_i L_i, its state pivots are those of
    I + L_i^T P_i L_i and its control pivots those of G_i;
  * a diagonal Delta_i reproduces the C oracle's diagonal path, pivots included;
  * pivot signs give the dense KKT inertia (Theorem
    "riccati-inertia-certification-theorem");
  * the product of the state pivots of stage i is det(I + Delta_i P_i).
A dropped Delta term, a transposed Delta or L, or a wrong stage index in any
of the recursion's Delta products fails the dense comparison; a wrong
representative for the pivots fails the congruence and determinant pins.
"""
import numpy as np
import pytest

import oracle
from oracle import dense, spd
from paper_2509_16370_amd import workloads as wl


def _inst(seed, n=4, m=2, N=6, delta=1e-2, spread=1.0, indefinite=False):
    return wl.make_instance(n, m, N, delta, (78, seed, 0), indefinite, spd_spread=spread)


def _close(got, ref, tol):
    for g, r in zip(got, ref):
        if np.asarray(r).size:
            assert np.abs(np.asarray(g) - r).max() <= tol * max(1.0, np.abs(r).max())


def _congruent(inst):
    """The Delta = I problem the SPD one maps to (see the module docstring)."""
    N, n = inst.N, inst.n
    L = np.linalg.cholesky(inst.delta_full)
    Li = np.linalg.inv(L)
    A = np.stack([Li[i + 1] @ inst.A[i] @ L[i] for i in range(N)]) if N else inst.A
    B = np.stack([Li[i + 1] @ inst.B[i] for i in range(N)]) if N else inst.B
    Q = np.stack([L[i].T @ inst.Q[i] @ L[i] for i in range(N + 1)])
    Q = 0.5 * (Q + np.swapaxes(Q, 1, 2))
    M = np.stack([L[i].T @ inst.M[i] for i in range(N)]) if N else inst.M
    q = np.stack([L[i].T @ inst.q[i] for i in range(N + 1)])
    c = np.stack([Li[i] @ inst.c[i] for i in range(N + 1)])
    return wl.Instance(n, inst.m, N, 1.0, Q, M, inst.R.copy(), A, B, q, inst.r.copy(), c, inst.indefinite), L


def test_generator_gives_spd_blocks():
    inst = _inst(1, n=5, spread=2.0)
    for D in inst.delta_full:
        assert np.array_equal(D, D.T)
        w = np.linalg.eigvalsh(D)
        assert w.min() > 0 and w.max() / w.min() <= 10 ** 4.0 + 1e-6


@pytest.mark.parametrize("spread", [0.0, 1.0, 2.0])
@pytest.mark.parametrize("indef", [False, True])
@pytest.mark.parametrize("shape", [(4, 2, 6), (3, 1, 1), (5, 3, 0), (6, 2, 9)])
def test_spd_matches_dense(spread, indef, shape):
    n, m, N = shape
    inst = _inst(13 * n + N, n, m, N, spread=spread, indefinite=indef)
    r = spd.seq(inst)
    assert r["status"] == 0
    _close((r["x"], r["u"], r["y"]), dense.solve(inst), 1e-9)
    assert spd.rel_residual(inst, r["x"], r["u"], r["y"]) <= 1e-12


def test_spd_residual_is_dense_kkt_residual():
    inst = _inst(2, n=4, m=3, N=5, spread=1.5, indefinite=True)
    rng = np.random.default_rng(0)
    x, u, y = rng.standard_normal((inst.N + 1, 4)), rng.standard_normal((inst.N, 3)), rng.standard_normal((inst.N + 1, 4))
    K, rhs = dense.assemble(inst)
    z = dense.join(inst, x, u, y)
    np.testing.assert_allclose(spd.residual(inst, x, u, y), K @ z - rhs, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("indef", [False, True])
def test_spd_congruence_to_unit_delta(indef):
    inst = _inst(3, n=5, m=2, N=8, delta=1e-2, spread=2.0, indefinite=indef)
    r = spd.seq(inst)
    t_inst, L = _congruent(inst)
    t = oracle.seq(t_inst)
    assert r["status"] == 0 and t["status"] == 0
    x = np.einsum("nij,nj->ni", L, t["x"])
    y = np.stack([np.linalg.solve(L[i].T, t["y"][i]) for i in range(inst.N + 1)])
    _close((r["x"], r["u"], r["y"]), (x, t["u"], y), 1e-9)
    _close((np.einsum("nji,njk,nkl->nil", L, r["P"], L),), (t["P"],), 1e-9)
    np.testing.assert_allclose(r["dS"], t["dS"], rtol=1e-8, atol=1e-11)
    np.testing.assert_allclose(r["dG"], t["dG"], rtol=1e-8, atol=1e-11)


def test_spd_diagonal_reproduces_diag_path():
    dinst = wl.make_instance(4, 3, 7, 3e-3, (78, 40, 0), True, diag_spread=1.0)
    full = wl.Instance(*[getattr(dinst, f) for f in ("n", "m", "N", "delta", "Q", "M", "R", "A", "B", "q",
                                                      "r", "c", "indefinite")],
                       delta_full=np.stack([np.diag(d) for d in dinst.delta_diag]))
    r = spd.seq(full)
    s = oracle.seq(dinst)
    _close((r["x"], r["u"], r["y"], r["P"]), (s["x"], s["u"], s["y"], s["P"]), 1e-10)
    np.testing.assert_allclose(r["dS"], s["dS"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r["dG"], s["dG"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("indef", [False, True])
def test_spd_certificate_matches_dense_inertia(indef):
    inst = _inst(5, n=3, m=2, N=5, delta=1e-1, spread=1.5, indefinite=indef)
    r = spd.seq(inst)
    ok, first_bad, inertia = spd.certificate(inst, r["dS"], r["dG"])
    K, _ = dense.assemble(inst)
    assert inertia == dense.inertia_eig(K)
    assert ok == (inertia == dense.target_inertia(inst))
    assert (first_bad >= 0) == (not ok)
    if indef:
        assert not ok  # the shifted Q makes the certificate fail (non-vacuous)


def test_spd_pivot_product_is_similarity_determinant():
    inst = _inst(7, n=4, m=2, N=5, delta=1e-1, spread=1.0, indefinite=True)
    r = spd.seq(inst)
    for i in range(inst.N + 1):
        det = np.linalg.det(np.eye(inst.n) + inst.delta_full[i] @ r["P"][i])
        assert np.prod(r["dS"][i]) == pytest.approx(det, rel=1e-10)


def test_spd_certificate_agrees_with_oracle_certificate_function():
    """spd.certificate and oracle.certificate count the same pivots the same way."""
    inst = _inst(8, n=3, m=2, N=4, delta=1e-1, spread=1.0, indefinite=True)
    r = spd.seq(inst)
    assert spd.certificate(inst, r["dS"], r["dG"]) == oracle.certificate(inst, r["dS"], r["dG"])
