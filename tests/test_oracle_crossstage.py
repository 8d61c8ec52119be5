"""Pins of the cross-stage (arrowhead) oracle.

The Schur route of the paper and the dense definition are checked against a
hand-derived example, against each other on random instances, against the
plain LQR solve when J = 0, and against Haynsworth's inertia formula.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import crossstage as ocs
from oracle import dense
from paper_2509_16370_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _inst(d):
    n, m, N = d["n"], d["m"], d["N"]
    a = lambda k, shape: np.asarray(d[k], dtype=np.float64).reshape(shape)
    return wl.Instance(n, m, N, float(d["delta"]), a("Q", (N + 1, n, n)), a("M", (N, n, m)),
                       a("R", (N, m, m)), a("A", (N, n, n)), a("B", (N, n, m)),
                       a("q", (N + 1, n)), a("r", (N, m)), a("c", (N + 1, n)))


def _close(a, b, tol):
    for va, vb in zip(a, b):
        scale = max(1.0, np.abs(np.asarray(vb)).max())
        assert np.abs(np.asarray(va) - np.asarray(vb)).max() <= tol * scale


@pytest.mark.parametrize("case", [0, 1])
def test_hand_example(case):
    g = json.load(open(os.path.join(GOLD, "example_cross_stage.json")))
    inst = _inst(g["lqr"])
    c = g["cases"][case]
    J = [(np.asarray(c["Jq"], float), np.asarray(c["Jr"], float), np.asarray(c["Jc"], float))]
    H = np.asarray(c["H"], float)
    rth = np.asarray(c["rtheta"], float)
    rw = (inst.q, inst.r, inst.c)
    want = (np.asarray(c["x"], float), np.asarray(c["u"], float), np.asarray(c["y"], float))
    for dw, th in (ocs.dense(inst, J, H, rw, rth), ocs.schur(inst, J, H, rw, rth)[:2]):
        _close(dw, want, 1e-13)
        assert np.allclose(th, c["theta"], atol=1e-13)
    S = ocs.schur(inst, J, H, rw, rth)[2]
    assert np.allclose(S, c["schur_complement"], atol=1e-13)
    # the Schur complement is the theta-block Schur complement of the reduced Hessian
    Hr = np.asarray(c["reduced_hessian_u0_theta"], float)
    assert np.isclose(S[0, 0], Hr[1, 1] - Hr[0, 1] ** 2 / Hr[0, 0])


def _random(seed, n=3, m=2, N=5, delta=1e-4, p=2, indefinite=False, indef_h=False):
    inst = wl.make_instance(n, m, N, delta, (98, seed, 0), indefinite=indefinite)
    xs = wl.make_cross_stage(inst, p, (98, seed, 0), indefinite=indef_h)
    return inst, xs


@pytest.mark.parametrize("delta", [0.0, 1e-8, 1e-4, 0.1])
@pytest.mark.parametrize("p", [1, 3])
def test_schur_matches_dense(delta, p):
    for seed in range(4):
        inst, xs = _random(seed, delta=delta, p=p, indefinite=(seed == 3))
        rw = (inst.q, inst.r, inst.c)
        dw_d, th_d = ocs.dense(inst, xs.J, xs.H, rw, xs.rth)
        dw_s, th_s, _ = ocs.schur(inst, xs.J, xs.H, rw, xs.rth)
        _close(dw_s, dw_d, 1e-9)
        assert np.abs(th_s - th_d).max() <= 1e-9 * max(1.0, np.abs(th_d).max())
        assert ocs.rel_residual(inst, xs.J, xs.H, rw, xs.rth, dw_s, th_s) <= 1e-12


def test_zero_coupling_reduces_to_lqr():
    """J = 0: dtheta = -H^{-1} r_theta and dw is the plain LQR solution."""
    inst, xs = _random(7, p=2)
    J0 = [tuple(np.zeros_like(a) for a in col) for col in xs.J]
    rw = (inst.q, inst.r, inst.c)
    for dw, th in (ocs.dense(inst, J0, xs.H, rw, xs.rth), ocs.schur(inst, J0, xs.H, rw, xs.rth)[:2]):
        assert np.allclose(th, -np.linalg.solve(xs.H, xs.rth), atol=1e-13)
        _close(dw, dense.solve(inst), 1e-12)


@pytest.mark.parametrize("indef_h", [False, True])
def test_haynsworth_inertia(indef_h):
    """In([[K, J], [J^T, H]]) = In(K) + In(S) (K nonsingular)."""
    for seed in range(5):
        inst, xs = _random(seed, p=3, delta=1e-3, indefinite=(seed % 2 == 1), indef_h=indef_h)
        rw = (inst.q, inst.r, inst.c)
        S = ocs.schur(inst, xs.J, xs.H, rw, xs.rth)[2]
        K, _ = dense.assemble(inst)
        kin = dense.inertia_eig(K)
        w = np.linalg.eigvalsh(0.5 * (S + S.T))
        sin = (int(np.sum(w > 0)), int(np.sum(w < 0)), 0)
        want = tuple(a + b for a, b in zip(kin, sin))
        assert ocs.inertia(inst, xs.J, xs.H) == want
        if indef_h:  # H negative definite and J^T K^{-1} J >= 0 on a PD LQR: S is negative definite
            if seed % 2 == 0:
                assert sin[1] == 3
        elif seed % 2 == 0:
            assert ocs.inertia(inst, xs.J, xs.H) == ocs.target_inertia(inst, 3)
