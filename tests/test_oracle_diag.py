"""Pins of the oracle's per-stage diagonal regularization Delta_i.

The definition of a dual-regularized LQR problem allows any SPD Delta_i;
the oracle's path for a positive diagonal Delta_i is checked here against
  * the dense KKT system with the blocks -Delta_i (the plain definition),
  * a reduction to the scalar case: with D_i = Delta_i^{1/2}, the change of
    variables x~_i = D_i^{-1} x_i, y~_i = D_i y_i turns the problem into one
    with Delta = I and data A~_i = D_{i+1}^{-1} A_i D_i, B~_i = D_{i+1}^{-1} B_i,
    Q~_i = D_i Q_i D_i, M~_i = D_i M_i, q~_i = D_i q_i, c~_i = D_i^{-1} c_i
    (R, r unchanged), solved by the oracle's scalar path, which is pinned on
    its own; the state pivots of that problem are those of
    I + D_i P_i D_i (Section "Inertia Certification"),
  * the inertia of the dense KKT matrix (Theorem
    "riccati-inertia-certification-theorem": pivot signs give the inertia),
  * the similarity I + Delta_i P_i = D_i S_hat_i D_i^{-1}: the product of the
    state pivots equals det(I + Delta_i P_i),
  * equal diagonal entries reproducing the scalar path.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2509_16370_amd import workloads as wl


def _inst(seed, n=4, m=2, N=6, delta=1e-3, spread=1.0, indefinite=False):
    return wl.make_instance(n, m, N, delta, (77, seed, 0), indefinite, diag_spread=spread)


def _close(got, ref, tol):
    for g, r in zip(got, ref):
        if np.asarray(r).size:
            assert np.abs(np.asarray(g) - r).max() <= tol * max(1.0, np.abs(r).max())


def _scaled(inst):
    """The Delta = I problem the diagonal one maps to (see the module docstring)."""
    D = np.sqrt(inst.delta_diag)
    N = inst.N
    A = np.stack([inst.A[i] * D[i][None, :] / D[i + 1][:, None] for i in range(N)]) if N else inst.A
    B = np.stack([inst.B[i] / D[i + 1][:, None] for i in range(N)]) if N else inst.B
    Q = inst.Q * D[:, :, None] * D[:, None, :]
    M = inst.M * D[:N, :, None]
    q = inst.q * D
    c = inst.c / D
    return wl.Instance(inst.n, inst.m, N, 1.0, Q, M, inst.R.copy(), A, B, q, inst.r.copy(), c,
                       inst.indefinite), D


@pytest.mark.parametrize("spread", [0.0, 1.0, 3.0])
@pytest.mark.parametrize("indef", [False, True])
@pytest.mark.parametrize("shape", [(4, 2, 6), (3, 1, 1), (5, 3, 0), (6, 2, 9)])
def test_diag_matches_dense(spread, indef, shape):
    n, m, N = shape
    inst = _inst(11 * n + N, n, m, N, spread=spread, indefinite=indef)
    r = oracle.seq(inst)
    assert r["status"] == 0
    _close((r["x"], r["u"], r["y"]), dense.solve(inst), 1e-9)
    assert oracle.rel_residual(inst, r["x"], r["u"], r["y"]) <= 1e-12


@pytest.mark.parametrize("indef", [False, True])
def test_diag_reduces_to_unit_delta_by_scaling(indef):
    inst = _inst(3, n=5, m=2, N=8, delta=1e-2, spread=2.0, indefinite=indef)
    r = oracle.seq(inst)
    sc, D = _scaled(inst)
    t = oracle.seq(sc)
    assert r["status"] == 0 and t["status"] == 0
    # x = D x~, y = D^{-1} y~, u unchanged; P~ = D P D
    _close((r["x"], r["u"], r["y"]), (D * t["x"], t["u"], t["y"] / D), 1e-9)
    _close((r["P"] * D[:, :, None] * D[:, None, :],), (t["P"],), 1e-9)
    # the same pivots: S_hat_i = I + D P_i D = I + P~_i, and G_i is unchanged
    np.testing.assert_allclose(r["dS"], t["dS"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r["dG"], t["dG"], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("indef", [False, True])
def test_diag_certificate_matches_dense_inertia(indef):
    inst = _inst(5, n=3, m=2, N=5, delta=1e-2, spread=1.5, indefinite=indef)
    r = oracle.seq(inst)
    ok, first_bad, inertia = oracle.certificate(inst, r["dS"], r["dG"])
    K, _ = dense.assemble(inst)
    assert inertia == dense.inertia_eig(K)
    assert ok == (inertia == dense.target_inertia(inst))
    assert (first_bad >= 0) == (not ok)


def test_diag_pivot_product_is_similarity_determinant():
    inst = _inst(7, n=4, m=2, N=5, delta=1e-1, spread=1.0, indefinite=True)
    r = oracle.seq(inst)
    for i in range(inst.N + 1):
        det = np.linalg.det(np.eye(inst.n) + np.diag(inst.delta_diag[i]) @ r["P"][i])
        assert np.prod(r["dS"][i]) == pytest.approx(det, rel=1e-10)


def test_equal_diagonal_is_scalar_delta():
    inst = _inst(9, n=4, m=3, N=7, delta=3e-3, spread=0.0, indefinite=True)
    assert np.all(inst.delta_diag == inst.delta)
    r = oracle.seq(inst)
    s = oracle.seq(wl.Instance(*[getattr(inst, f) for f in
                                 ("n", "m", "N", "delta", "Q", "M", "R", "A", "B", "q", "r", "c",
                                  "indefinite")]))
    _close((r["x"], r["u"], r["y"], r["P"], r["dS"], r["dG"]),
           (s["x"], s["u"], s["y"], s["P"], s["dS"], s["dG"]), 1e-12)


def test_diag_batch_driver_matches_single():
    insts = [_inst(20 + b, n=3 + b % 3, m=1 + b % 2, N=4 + b, spread=1.0 if b % 2 else None)
             for b in range(5)]
    packed = wl.pack(insts)
    assert "delta_diag" in packed.arrays
    x, u, y, st, _ = oracle.seq_batch(packed, nthreads=2)
    assert (st == 0).all()
    sols = wl.unpack_solution(packed, x, u, y)
    for inst, sol in zip(insts, sols):
        r = oracle.seq(inst)
        _close(sol, (r["x"], r["u"], r["y"]), 1e-13)
