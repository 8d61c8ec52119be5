"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances. The gate the method states is the relative KKT residual
||K z + b||_inf / ||b||_inf <= 1e-8 after refinement; every instance must meet
it. Element-wise, z differs from the oracle by at most cond(K) times the
residual gap; the random instances here have cond(K) below ~1e4, so the
element-wise gate is 1e-7 * max(1, |z|) for refined results and 1e-10 for
the pure float64 path (about 1e6 unit roundoffs of headroom). Integer outputs
(verdict, first failing pivot, inertia) must match exactly.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2509_16370_amd import workloads as wl

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def rl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_16370_amd import rlqr
    return rlqr


def run(rl, insts, mode, rel_tol=1e-8, max_refine=3, fused=False):
    import torch
    packed = wl.pack(insts)
    lhs, rhs = rl.to_device(packed)
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode)
    s.factor(lhs, rhs if fused else None)
    out, status, relres = s.solve(rhs, rel_tol=rel_tol, max_refine=max_refine)
    verdict, first_bad, inertia = s.pivot_inertia()
    torch.cuda.synchronize()
    sols = wl.unpack_solution(packed, *(out[k].cpu().numpy() for k in ("x", "u", "y")))
    B = packed.batch
    return dict(sols=sols, status=status.cpu().numpy()[:B], relres=relres.cpu().numpy()[:B],
                verdict=verdict.cpu().numpy()[:B], first_bad=first_bad.cpu().numpy()[:B],
                inertia=inertia.cpu().numpy().reshape(-1, 3)[:B] if B else np.zeros((0, 3)),
                solver=s, lhs=lhs, rhs=rhs, out=out, packed=packed)


def compare(inst, sol, ref, tol):
    scale = max(1.0, *(np.abs(ref[k]).max() for k in ("x", "u", "y") if ref[k].size))
    err = max(np.abs(a - ref[k]).max() if a.size else 0.0 for a, k in zip(sol, ("x", "u", "y")))
    assert err <= tol * scale, f"max|gpu - oracle| = {err:.3e}, scale {scale:.3e}"


def residual_rounding_bound(inst, x, u, y):
    """How far two float64 evaluations of the relative residual of one z may
    differ: every residual row is a sum of at most 2n + m + 2 products, each
    evaluation errs by at most (2n + m + 2) eps64 times the row's sum of
    |terms| <= ||K||_inf ||z||_inf + ||b||_inf; two evaluations, relative to
    ||b||_inf. ||K||_inf from the stage blocks' absolute row sums."""
    n, m, N = inst.n, inst.m, inst.N
    d = float(inst.delta) if getattr(inst, "delta_diag", None) is None else float(np.max(inst.delta_diag))
    kinf = 1.0 + d
    if N:
        kinf = max(kinf, float(np.max(np.abs(inst.Q[:N]).sum(2) + np.abs(inst.M).sum(2) + np.abs(inst.A).sum(1))) + 1.0,
                   float(np.max(np.abs(inst.M).sum(1) + np.abs(inst.R).sum(2) + np.abs(inst.B).sum(1))),
                   float(np.max(np.abs(inst.A).sum(2) + np.abs(inst.B).sum(2))) + 1.0 + d)
    kinf = max(kinf, float(np.abs(inst.Q[N]).sum(1).max()) + 1.0)
    zinf = max(float(np.abs(v).max()) if np.asarray(v).size else 0.0 for v in (x, u, y))
    binf = max(oracle.rhs_norm(inst), 1e-300)
    return 2.0 * (2 * n + m + 2) * 2.220446049250313e-16 * (kinf * zinf + binf) / binf


# cond(K) bound of the random instances of these tests (see the module docstring)
COND_BOUND = 1.0e4


def check_instance(rl, inst, res, b, base_tol, rel_tol=1e-8):
    """Every gate for instance b, positive definite or not: status, verdict,
    first failing pivot and inertia equal to the oracle's; relative residual
    <= rel_tol; element-wise against the oracle within
    max(base_tol, COND_BOUND * (gpu residual + oracle residual)) * max(1, |z|)
    (two solutions of one system differ by at most cond(K) times the sum of
    their relative residuals; an indefinite KKT system still has one solution)."""
    ref = oracle.seq(inst)
    if ref["status"]:
        assert res["status"][b] == rl.INST_SINGULAR, b
        return
    ov, ofb, oin = oracle.certificate(inst, ref["dS"], ref["dG"])
    where = (b, inst.n, inst.m, inst.N, inst.delta, inst.indefinite)
    assert res["verdict"][b] == int(ov), where
    assert res["first_bad"][b] == ofb, where
    assert tuple(res["inertia"][b]) == oin, (where, tuple(res["inertia"][b]), oin)
    assert res["relres"][b] <= rel_tol, (where, res["relres"][b])
    assert res["status"][b] == (rl.INST_OK if ov else rl.INST_NOT_PD), where
    oracle_rel = oracle.rel_residual(inst, ref["x"], ref["u"], ref["y"])
    compare(inst, res["sols"][b], ref, max(base_tol, COND_BOUND * (res["relres"][b] + oracle_rel)))


def _load(name):
    return json.load(open(os.path.join(GOLD, name)))


def _inst(d, q=None, r=None, c=None):
    n, m, N = d["n"], d["m"], d["N"]
    f = lambda k, s: np.asarray(d[k], float).reshape(s)
    return wl.Instance(n, m, N, float(d["delta"]), f("Q", (N + 1, n, n)), f("M", (N, n, m)),
                       f("R", (N, m, m)), f("A", (N, n, n)), f("B", (N, n, m)),
                       f("q", (N + 1, n)) if "q" in d else q, f("r", (N, m)) if "r" in d else r,
                       f("c", (N + 1, n)) if "c" in d else c)


# --------------------------------------------------------- worked examples

@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_printed_examples(rl, mode):
    print(f"[gpu] printed examples mode={mode}", flush=True)
    g1 = _load("example_newton_kkt_descent.json")
    ex1 = _inst(g1["lqr"])
    g2 = _load("example_indefinite_R_inertia.json")
    q2, r2, c2 = np.array([[0.3], [-0.2]]), np.array([[0.5]]), np.array([[1.0], [0.2]])
    ex2 = _inst(g2["lqr"], q2, r2, c2)
    d3 = dict(g2["lqr"]); d3["R"] = [[[-3.0]]]
    ex3 = _inst(d3, q2, r2, c2)
    d4 = dict(g2["lqr"]); d4["R"] = [[[-2.0]]]
    ex4 = _inst(d4, q2, r2, c2)
    res = run(rl, [ex1, ex2, ex3, ex4], mode)
    x, u, y = res["sols"][0]
    z = dense.join(ex1, x, u, y)
    tol = 1e-12 if mode == "fp64" else 1e-8
    assert np.allclose(z, g1["printed_solution"], atol=tol)
    assert res["verdict"][1] == 1 and tuple(res["inertia"][1]) == tuple(g2["printed_inertia"])
    assert res["first_bad"][1] == -1 and res["status"][1] == rl.INST_OK
    assert res["verdict"][2] == 0 and res["first_bad"][2] == 1 and tuple(res["inertia"][2]) == (2, 3, 0)
    assert res["status"][2] == rl.INST_NOT_PD
    compare(ex3, res["sols"][2], oracle.seq(ex3), 1e-10 if mode == "fp64" else 1e-7)
    assert res["status"][3] == rl.INST_SINGULAR and res["verdict"][3] == 0
    assert np.isnan(res["sols"][3][0]).all()


# --------------------------------------------------------- random ragged batches

def _random_batch(seed, count=48):
    rng = np.random.default_rng(seed)
    insts = []
    for i in range(count):
        n = int(rng.integers(1, 13))
        m = int(rng.integers(1, min(8, 16 - n) + 1))
        N = int(rng.choice([0, 1, 2, 7, 33, 64, 100]))
        delta = float(rng.choice([0.0, 1e-8, 1e-4, 1e-1, 1.0]))
        insts.append(wl.make_instance(n, m, N, delta, (50, seed, i), indefinite=bool(rng.random() < 0.25)))
    return insts


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_random_ragged_batch_matches_oracle(rl, mode):
    print(f"[gpu] random ragged batch mode={mode}", flush=True)
    insts = _random_batch(1)
    res = run(rl, insts, mode)
    for b, inst in enumerate(insts):
        check_instance(rl, inst, res, b, 1e-10 if mode == "fp64" else 1e-7)


@pytest.mark.parametrize("mode", ["fp64", "mixed", "scan"])
@pytest.mark.parametrize("shape", [(4, 1), (8, 2), (12, 4)])
def test_fixed_shape_kernels_match_oracle(rl, mode, shape):
    """A batch whose one-wavefront instances all share one of the stage shapes
    compiled with n and m fixed takes those kernels; ragged N (including 0
    and 1), deltas from 0 to 0.1 and indefinite instances."""
    n, m = shape
    print(f"[gpu] fixed shape n={n} m={m} mode={mode}", flush=True)
    rng = np.random.default_rng(n * 10 + m)
    insts = []
    for i in range(20):
        N = int(rng.choice([0, 1, 2, 7, 31, 64, 130]))
        delta = float(rng.choice([0.0, 1e-8, 1e-4, 1e-1]))
        insts.append(wl.make_instance(n, m, N, delta, (57, n * 10 + m, i), indefinite=bool(rng.random() < 0.2)))
    res = run(rl, insts, mode)
    for b, inst in enumerate(insts):
        check_instance(rl, inst, res, b, 1e-10 if mode == "fp64" else 1e-7)


@pytest.mark.parametrize("mode", ["fp64", "mixed", "scan"])
@pytest.mark.parametrize("uniform", [False, True])
def test_factor_rhs_matches_factor_then_solve(rl, mode, uniform):
    """rlqr_factor_rhs (the backward vector pass inside the factorization's
    stage loop) gives the results of rlqr_factor + rlqr_solve: a ragged batch
    mixing one-wavefront and multi-wavefront instances, and a uniform
    quadrotor-shaped batch (fixed-shape kernels); both against the oracle."""
    print(f"[gpu] factor_rhs mode={mode} uniform={uniform}", flush=True)
    if uniform:
        insts = [wl.make_instance(12, 4, N, d, (58, i, 0), indefinite=(i % 5 == 4))
                 for i, (N, d) in enumerate([(0, 1e-8), (1, 1e-4), (9, 0.0), (40, 1e-8), (128, 1e-8),
                                             (128, 1e-4), (77, 1e-1), (128, 1e-8), (3, 1.0), (64, 1e-6)])]
    else:
        insts = _random_batch(6, count=24) + [wl.make_instance(n, m, N, 1e-6, (59, n, N))
                                              for n, m, N in [(20, 10, 9), (33, 5, 17), (24, 20, 0)]]
    a = run(rl, insts, mode)
    b = run(rl, insts, mode, fused=True)
    for k in ("status", "verdict", "first_bad"):
        assert np.array_equal(a[k], b[k]), k
    assert np.all((b["relres"] <= 1e-8) | ~(a["relres"] <= 1e-8)), (a["relres"], b["relres"])
    for i, inst in enumerate(insts):
        if a["status"][i] == rl.INST_SINGULAR:
            continue
        ref = dict(zip(("x", "u", "y"), a["sols"][i]))
        compare(inst, b["sols"][i], ref, 1e-12 if mode == "fp64" else 1e-8)
        # the reported residual is that of the returned solution (float64 residual
        # of the oracle on the same z, up to the rounding of the residual itself)
        orel = oracle.rel_residual(inst, *b["sols"][i])
        gap = residual_rounding_bound(inst, *b["sols"][i])
        assert abs(b["relres"][i] - orel) <= 1e-3 * orel + gap, (i, b["relres"][i], orel, gap)
        check_instance(rl, inst, b, i, 1e-10 if mode == "fp64" else 1e-7)


def test_fp64_unrefined_is_accurate(rl):
    """With no refinement the float64 path alone reaches ~1e-13 relative residual."""
    print("[gpu] fp64 without refinement", flush=True)
    insts = [wl.make_instance(12, 4, 128, d, (51, i, 0)) for i, d in enumerate([0.0, 1e-8, 1e-4, 1.0])]
    res = run(rl, insts, "fp64", max_refine=0)
    assert (res["relres"] <= 1e-12).all(), res["relres"]
    for b, inst in enumerate(insts):
        compare(inst, res["sols"][b], oracle.seq(inst), 1e-11)


# --------------------------------------------------------- residual entry point

def test_residual_entry_matches_oracle(rl):
    import torch
    print("[gpu] residual entry", flush=True)
    insts = _random_batch(2, count=12)
    packed = wl.pack(insts)
    lhs, rhs = rl.to_device(packed)
    s = rl.Solver(packed.N, packed.n, packed.m, mode="fp64")
    s.factor(lhs)
    rng = np.random.default_rng(3)
    z = {k: rng.standard_normal(max(int(packed.offsets[k][-1]), 1)) for k in ("x", "u", "y")}
    zt = {k: torch.from_numpy(v).cuda() for k, v in z.items()}
    res, relres = s.residual(rhs, zt)
    torch.cuda.synchronize()
    res = res.cpu().numpy()
    roff = s.offsets["res"]
    sols = wl.unpack_solution(packed, z["x"], z["u"], z["y"])
    for b, inst in enumerate(insts):
        ref = oracle.residual(inst, *sols[b])
        got = res[roff[b]:roff[b + 1]]
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13 * max(1, np.abs(ref).max()))
        rel = np.abs(ref).max() / oracle.rhs_norm(inst)
        assert np.isclose(float(relres[b]), rel, rtol=1e-12)


# --------------------------------------------------------- edge cases

def test_empty_batch_and_zero_horizon(rl):
    import torch
    print("[gpu] empty batch / N=0", flush=True)
    s = rl.Solver(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    dummy = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.factor({k: dummy for k in ("Q", "M", "R", "A", "B", "delta")})
    s.solve({k: dummy for k in ("q", "r", "c")})
    torch.cuda.synchronize()
    insts = [wl.make_instance(3, 2, 0, 1e-3, (52, 0, 0)), wl.make_instance(5, 1, 1, 0.0, (52, 1, 0))]
    res = run(rl, insts, "fp64")
    for b, inst in enumerate(insts):
        compare(inst, res["sols"][b], oracle.seq(inst), 1e-12)


def test_solve_before_factor_is_state_error(rl):
    import torch
    s = rl.Solver([3], [2], [1])
    t = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(rl.RlqrError) as e:
        rl.rlqr_solve(s.handle, t, t, t, t, t, t, 1e-8, 0)
    assert e.value.code == rl.RLQR_E_STATE


def test_deterministic(rl):
    print("[gpu] determinism", flush=True)
    insts = _random_batch(4, count=16)
    a = run(rl, insts, "mixed")
    b = run(rl, insts, "mixed")
    for sa, sb in zip(a["sols"], b["sols"]):
        for va, vb in zip(sa, sb):
            assert np.array_equal(va, vb, equal_nan=True)


# --------------------------------------------------------- full size, sampled

@pytest.mark.parametrize("mode", ["fp64", "mixed"])
@pytest.mark.parametrize("delta", [1e-8, 1e-4])
def test_full_size_uniform_batch(rl, mode, delta):
    """4096 instances, n=12, m=4, N=128 (the benchmark's launch configuration):
    every instance meets 1e-8; a sample is checked element-wise and for
    certificate parity against the oracle."""
    print(f"[gpu] full-size uniform batch mode={mode} delta={delta}", flush=True)
    insts = _full_size(delta)
    res = run(rl, insts, mode)
    assert (res["relres"] <= 1e-8).all(), res["relres"].max()
    rng = np.random.default_rng(7)
    for b in rng.choice(len(insts), 24, replace=False):
        check_instance(rl, insts[b], res, b, 1e-10 if mode == "fp64" else 1e-7)


_FULL = {}


def _full_size(delta):
    if delta not in _FULL:
        insts = wl.batched_uniform(delta=delta)
        _FULL.clear()
        _FULL[delta] = insts
    return _FULL[delta]


# --------------------------------------------------------- larger stages (multi-wavefront kernels)

_CLASS_SHAPES = [(10, 12), (20, 10), (24, 20), (40, 6), (50, 14), (64, 32)]


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_multiwave_tile_classes_match_oracle(rl, mode):
    """One instance set per tile class (n + m from 22 to 96), ragged N, PD and
    indefinite data, delta in {0, 1e-6, 1e-2}."""
    print(f"[gpu] multi-wavefront tile classes mode={mode}", flush=True)
    insts = []
    for ci, (n, m) in enumerate(_CLASS_SHAPES):
        for j, (N, delta, indef) in enumerate([(0, 1e-6, False), (1, 0.0, False), (6, 1e-2, True), (19, 1e-6, False)]):
            insts.append(wl.make_instance(n, m, N, delta, (60, ci, j), indefinite=indef))
    res = run(rl, insts, mode)
    for b, inst in enumerate(insts):
        check_instance(rl, inst, res, b, 1e-10 if mode == "fp64" else 1e-7)


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_wavefront_counts_match_four(rl, mode):
    """rlqr_tuning.mw_waves = 1, 2 or 8 (stages with 16 < n + m <= 48) gives
    the results of the default four wavefronts: identical certificates,
    solutions within float64 rounding of each other, and the oracle's gates."""
    import torch
    print(f"[gpu] wavefront counts mode={mode}", flush=True)
    insts = []
    for ci, (n, m) in enumerate([(10, 12), (16, 8), (20, 10), (24, 20), (32, 8), (32, 2)]):
        for j, (N, delta, indef) in enumerate([(0, 1e-6, False), (9, 1e-4, False), (13, 1e-2, True), (40, 1e-8, False)]):
            insts.append(wl.make_instance(n, m, N, delta, (61, ci, j), indefinite=indef))
    packed = wl.pack(insts)
    lhs, rhs = rl.to_device(packed)
    res = {}
    for w in (4, 8, 1, 2):
        s = rl.Solver(packed.N, packed.n, packed.m, mode=mode, mw_waves=w)
        assert s.tuning["mw_waves"] == w
        s.factor(lhs)
        out, status, relres = s.solve(rhs, rel_tol=1e-8, max_refine=3)
        verdict, first_bad, inertia = s.pivot_inertia()
        torch.cuda.synchronize()
        B = packed.batch
        res[w] = dict(sols=wl.unpack_solution(packed, *(out[k].cpu().numpy() for k in ("x", "u", "y"))),
                      status=status.cpu().numpy()[:B], relres=relres.cpu().numpy()[:B],
                      verdict=verdict.cpu().numpy()[:B], first_bad=first_bad.cpu().numpy()[:B],
                      inertia=inertia.cpu().numpy().reshape(-1, 3)[:B])
    for w in (8, 1, 2):
        for k in ("status", "verdict", "first_bad", "inertia"):
            assert np.array_equal(res[4][k], res[w][k]), (w, k)
        for b, inst in enumerate(insts):
            compare(inst, res[w]["sols"][b], dict(zip(("x", "u", "y"), res[4]["sols"][b])),
                    1e-12 if mode == "fp64" else 1e-8)
            check_instance(rl, inst, res[w], b, 1e-10 if mode == "fp64" else 1e-7)
