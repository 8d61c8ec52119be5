"""GPU parity of the stagewise-equality elimination (include/rlqr_eq.h).

A Newton step with ne equality rows per stage runs as rlqr_eq_reduce ->
rlqr_factor / rlqr_solve on the reduced data -> rlqr_eq_recover, all through
the C ABI, and is checked against the oracle (oracle/eqstep.py, pinned on the
CPU against a hand-derived case, the dense definition and Haynsworth's
inertia): the reduced blocks to 1e-13 relative, the step (x, u, y, w)
element-wise against the oracle after refinement of the reduced LQR, and the
certificate of the reduced factorization against the oracle's,
with the full matrix's inertia = reduced inertia + ne (N + 1) negative values.

Tolerances. The penalties (eta up to 1e4 per row) add eta E^T E to the stage
Hessian and raise cond(K) by up to about two decades over the plain batches,
so a step refined to a relative residual of 1e-8 is good to about 1e-6 of
its scale element-wise; the tests that gate at 1e-7 refine to 1e-10 (the
float64 path meets that in its first pass).
"""
import numpy as np
import pytest

import oracle
from oracle import dense, eqstep
from paper_2509_16370_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_16370_amd import rlqr
    return rlqr


def _eq_device(rl, packed, eqs):
    import torch
    cs = wl.pack_stage_eq(packed, eqs)
    dev = {k: torch.from_numpy(cs[k] if cs[k].size else np.zeros(1)).to("cuda:0") for k in ("E", "r", "eta")}
    return cs, dev


def step(rl, insts, eqs, mode="fp64", in_place=False, max_refine=6, rel_tol=1e-10):
    import torch
    packed = wl.pack(insts)
    lhs, rhs = rl.to_device(packed)
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode)
    st = rl.StageEquality(s, [e.ne for e in eqs])
    cs, eqd = _eq_device(rl, packed, eqs)
    assert np.array_equal(st.offsets["E"], cs["E_off"]) and np.array_equal(st.offsets["v"], cs["v_off"])
    out = None
    if in_place:
        lhs = {k: v.clone() for k, v in lhs.items()}
        rhs = {k: v.clone() for k, v in rhs.items()}
        out = {"Q": lhs["Q"], "M": lhs["M"], "R": lhs["R"], "q": rhs["q"], "r": rhs["r"]}
    lhs2, rhs2 = st.reduce(lhs, rhs, eqd, out=out)
    s.factor(lhs2, rhs2)
    sol, status, relres = s.solve(rhs2, rel_tol=rel_tol, max_refine=max_refine)
    w = st.recover(eqd, sol)
    verdict, first_bad, inertia = s.pivot_inertia()
    torch.cuda.synchronize()
    B = packed.batch
    return dict(packed=packed, cs=cs, lhs2={k: lhs2[k].cpu().numpy() for k in ("Q", "M", "R")},
                rhs2={k: rhs2[k].cpu().numpy() for k in ("q", "r")},
                sols=wl.unpack_solution(packed, *(sol[k].cpu().numpy() for k in ("x", "u", "y"))),
                w=w.cpu().numpy(), relres=relres.cpu().numpy()[:B], status=status.cpu().numpy()[:B],
                verdict=verdict.cpu().numpy()[:B], first_bad=first_bad.cpu().numpy()[:B],
                inertia=inertia.cpu().numpy().reshape(-1, 3)[:B])


def check(insts, eqs, r, tol=1e-7, inertia_full=False, rel_tol=1e-10):
    p = r["packed"]
    for b, (inst, eq) in enumerate(zip(insts, eqs)):
        red = eqstep.reduce(inst, eq)
        # reduced blocks
        for k in ("Q", "M", "R"):
            o = p.offsets[k]
            got = r["lhs2"][k][o[b]:o[b + 1]]
            want = getattr(red, k).reshape(-1)
            if want.size:
                assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max()), (b, k)
        for k in ("q", "r"):
            o = p.offsets[k]
            got = r["rhs2"][k][o[b]:o[b + 1]]
            want = getattr(red, k).reshape(-1)
            if want.size:
                assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max()), (b, k)
        # the step
        x, u, y, w, o = eqstep.route(inst, eq)
        assert o["status"] == 0
        ok, fb, inr = oracle.certificate(red, o["dS"], o["dG"])
        assert r["verdict"][b] == int(ok) and r["first_bad"][b] == fb, b
        assert tuple(r["inertia"][b]) == inr, b
        assert r["relres"][b] <= rel_tol, (b, r["relres"][b])
        v = r["cs"]["v_off"]
        wg = r["w"][v[b]:v[b + 1]].reshape(inst.N + 1, eq.ne)
        ref = (x, u, y, w)
        got = tuple(r["sols"][b]) + (wg,)
        scale = max(1.0, *(np.abs(a).max() for a in ref if a.size))
        err = max(np.abs(g - a).max() if a.size else 0.0 for g, a in zip(got, ref))
        assert err <= tol * scale, (b, err, scale)
        if inertia_full:
            full = eqstep.inertia_full(inst, eq)
            assert full == (inr[0], inr[1] + (inst.N + 1) * eq.ne, inr[2]), b


SHAPES = [(4, 2, 0), (4, 2, 1), (12, 4, 30), (5, 3, 9), (20, 8, 7), (36, 10, 5), (3, 1, 17), (12, 4, 64)]


def _batch(seed, nes, eta=1e3, delta=1e-4):
    insts, eqs = [], []
    for b, ((n, m, N), ne) in enumerate(zip(SHAPES, nes)):
        inst = wl.make_instance(n, m, N, delta, (95, seed, b), indefinite=(b % 4 == 3))
        insts.append(inst)
        eqs.append(wl.make_stage_eq(inst, ne, (95, seed, b), eta=eta))
    return insts, eqs


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_stage_equality_step_matches_oracle(rl, mode):
    print(f"[gpu] stage equality step mode={mode}", flush=True)
    insts, eqs = _batch(1, [1, 2, 2, 3, 5, 2, 1, 4])
    r = step(rl, insts, eqs, mode=mode)
    check(insts, eqs, r, inertia_full=(mode == "fp64"))


def test_stage_equality_in_place_and_no_rows(rl):
    """Reduced blocks written over the inputs; instances with ne = 0 keep
    their data (the step is the plain LQR step, w empty)."""
    print("[gpu] stage equality in place", flush=True)
    insts, eqs = _batch(2, [0, 2, 0, 3, 1, 0, 16, 2])
    a = step(rl, insts, eqs, in_place=True)
    check(insts, eqs, a)
    b = step(rl, insts, eqs, in_place=False)
    for k in ("Q", "M", "R"):
        assert np.array_equal(a["lhs2"][k], b["lhs2"][k])
    assert np.array_equal(a["w"], b["w"])


def test_stage_equality_penalty_range(rl):
    """Penalties from 1e1 to 1e5 (the reduced Hessian's conditioning grows
    with eta; refinement keeps the gate)."""
    print("[gpu] stage equality penalties", flush=True)
    for seed, eta in ((3, 1e2), (4, 1e4)):
        insts, eqs = _batch(seed, [2] * len(SHAPES), eta=eta)
        r = step(rl, insts, eqs, max_refine=8)
        check(insts, eqs, r, tol=1e-6)


def test_stage_equality_full_size_sampled(rl):
    """The benchmark configuration (4096 instances, n = 12, m = 4, N = 128,
    ne = 2 rows per stage): every instance at 1e-8; reduced blocks, step and
    certificate on a sample against the oracle."""
    print("[gpu] stage equality full size", flush=True)
    insts = wl.batched_uniform(batch=4096, n=12, m=4, N=128, delta=1e-8)
    eqs = [wl.make_stage_eq(inst, 2, (1, b, 0)) for b, inst in enumerate(insts)]
    r = step(rl, insts, eqs, mode="mixed", max_refine=3, rel_tol=1e-8)
    assert (r["relres"] <= 1e-8).all(), r["relres"].max()
    rng = np.random.default_rng(17)
    idx = sorted(rng.choice(len(insts), 12, replace=False))
    sub = dict(r)
    for key in ("relres", "status", "verdict", "first_bad", "inertia"):
        sub[key] = r[key][idx]
    sub["sols"] = [r["sols"][i] for i in idx]
    p = r["packed"]
    sub_insts = [insts[i] for i in idx]
    sub_eqs = [eqs[i] for i in idx]
    # re-index the flat arrays to the sample
    sub["packed"] = wl.pack(sub_insts)
    sp = sub["packed"]
    sub["lhs2"] = {k: np.concatenate([r["lhs2"][k][p.offsets[k][i]:p.offsets[k][i + 1]] for i in idx])
                   for k in ("Q", "M", "R")}
    sub["rhs2"] = {k: np.concatenate([r["rhs2"][k][p.offsets[k][i]:p.offsets[k][i + 1]] for i in idx])
                   for k in ("q", "r")}
    v = r["cs"]["v_off"]
    sub["w"] = np.concatenate([r["w"][v[i]:v[i + 1]] for i in idx])
    sub["cs"] = wl.pack_stage_eq(sp, sub_eqs)
    check(sub_insts, sub_eqs, sub, tol=1e-6, rel_tol=1e-8)


def test_stage_equality_with_per_stage_diagonal(rl):
    """Equality rows eliminated into an LQR whose dynamics carry a per-stage
    diagonal Delta_i: the reduced lhs keeps delta_diag, the diagonal kernels
    run the step."""
    print("[gpu] stage equality with a per-stage diagonal", flush=True)
    insts, eqs = [], []
    for b, (n, m, N) in enumerate(SHAPES):
        inst = wl.make_instance(n, m, N, 1e-3, (96, 0, b), indefinite=(b % 4 == 3), diag_spread=1.0)
        insts.append(inst)
        eqs.append(wl.make_stage_eq(inst, 1 + b % 3, (96, 0, b)))
    r = step(rl, insts, eqs)
    check(insts, eqs, r, inertia_full=True)
