"""Pins of the stagewise-equality elimination oracle (oracle/eqstep.py).

Checks against things other than the route itself: a hand-derived case
(golden file, derivation inside), the dense definition of the full
Newton-KKT system with the equality rows, the reduction to the plain LQR
when the Jacobians vanish, and Haynsworth's inertia formula for the
elimination of the negative definite -D^{-1} block.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import dense, eqstep
from paper_2509_16370_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_derived_example():
    g = json.load(open(os.path.join(GOLD, "example_stage_equality.json")))
    d, e, want = g["lqr"], g["eq"], g["expect"]
    inst = wl.Instance(1, 1, 0, d["delta"], np.array(d["Q"]), np.zeros((0, 1, 1)), np.zeros((0, 1, 1)),
                       np.zeros((0, 1, 1)), np.zeros((0, 1, 1)), np.array(d["q"]), np.zeros((0, 1)),
                       np.array(d["c"]))
    eq = wl.StageEq(1, np.array(e["Ex"]), np.zeros((0, 1, 1)), np.array(e["r"]), np.array(e["eta"]))
    red = eqstep.reduce(inst, eq)
    assert red.Q[0, 0, 0] == pytest.approx(want["Q0_reduced"]) and red.q[0, 0] == pytest.approx(want["q0_reduced"])
    for route in (eqstep.dense(inst, eq), eqstep.route(inst, eq)[:4]):
        x, u, y, w = route
        assert x[0, 0] == pytest.approx(want["x0"], rel=1e-12)
        assert y[0, 0] == pytest.approx(want["y0"], rel=1e-12)
        assert w[0, 0] == pytest.approx(want["w0"], rel=1e-12)


@pytest.mark.parametrize("ne", [1, 3])
@pytest.mark.parametrize("indef", [False, True])
@pytest.mark.parametrize("N", [0, 1, 6])
def test_route_matches_dense_definition(ne, indef, N):
    inst = wl.make_instance(4, 2, N, 1e-3, (91, N, ne), indef)
    eq = wl.make_stage_eq(inst, ne, (91, N, ne))
    x, u, y, w = eqstep.dense(inst, eq)
    x2, u2, y2, w2, o = eqstep.route(inst, eq)
    assert o["status"] == 0
    for a, b in ((x, x2), (u, u2), (y, y2), (w, w2)):
        if b.size:
            assert np.abs(a - b).max() <= 1e-8 * max(1.0, np.abs(a).max())


def test_zero_jacobian_is_plain_lqr():
    inst = wl.make_instance(3, 2, 5, 1e-4, (92, 0, 0))
    eq = wl.make_stage_eq(inst, 2, (92, 0, 0))
    eq = wl.StageEq(2, np.zeros_like(eq.Ex), np.zeros_like(eq.Eu), eq.r, eq.eta)
    x, u, y, w, _ = eqstep.route(inst, eq)
    ref = oracle.seq(inst)
    np.testing.assert_allclose(x, ref["x"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(y, ref["y"], rtol=0, atol=1e-14)
    np.testing.assert_array_equal(w, eq.eta * eq.r)
    xd, ud, yd, wd = eqstep.dense(inst, eq)
    np.testing.assert_allclose(wd, eq.eta * eq.r, rtol=1e-10)


@pytest.mark.parametrize("indef", [False, True])
def test_haynsworth_inertia(indef):
    inst = wl.make_instance(3, 2, 4, 1e-2, (93, 1, 0), indef)
    eq = wl.make_stage_eq(inst, 2, (93, 1, 0))
    full = eqstep.inertia_full(inst, eq)
    K, _ = dense.assemble(eqstep.reduce(inst, eq))
    kin = dense.inertia_eig(K)
    assert full == (kin[0], kin[1] + (inst.N + 1) * eq.ne, kin[2])
    # and the certificate of the reduced LQR (pivot signs) gives In(K_red)
    o = oracle.seq(eqstep.reduce(inst, eq))
    assert oracle.certificate(inst, o["dS"], o["dG"])[2] == kin
