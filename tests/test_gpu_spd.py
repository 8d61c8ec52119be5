"""GPU parity of general SPD per-stage regularization Delta_i
(include/rlqr_spd.h) against the float64 CPU oracle oracle/spd.py.

The library factors Delta_i = L_i D_i L_i^T, solves the congruent problem
with the diagonal regularization D_i in the handle's mode and refines
against the original system's float64 residual. Gates, per instance: the
certificate (verdict, first failing pivot, inertia) equal to the oracle's
(whose state pivots are those of I + C_i^T P_i C_i, C_i the Cholesky factor:
the same matrices the GPU sweeps), the library's relative residual <= 1e-8
and the oracle's own residual of the returned z <= 1e-8, and element-wise
1e-7 * max(1, |z|) against the oracle's solution (cond(K) of these
instances is below ~1e4; indefinite ones included, their solution is still
the unique KKT solution).
"""
import numpy as np
import pytest

from oracle import spd
from paper_2509_16370_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_16370_amd import rlqr
    return rlqr


def run(rl, insts, mode, chunk=0, rel_tol=1e-8, max_refine=3):
    import torch
    packed = wl.pack(insts)
    lhs, rhs = rl.to_device(packed)
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode, scan_chunk=chunk)
    sp = rl.SpdRegularized(s)
    sp.factor(lhs, lhs["delta_full"])
    out, status, relres = sp.solve(rhs, rel_tol=rel_tol, max_refine=max_refine)
    verdict, first_bad, inertia = s.pivot_inertia()
    torch.cuda.synchronize()
    B = packed.batch
    sols = wl.unpack_solution(packed, *(out[k].cpu().numpy() for k in ("x", "u", "y")))
    return dict(sols=sols, status=status.cpu().numpy()[:B], relres=relres.cpu().numpy()[:B],
                verdict=verdict.cpu().numpy()[:B], first_bad=first_bad.cpu().numpy()[:B],
                inertia=inertia.cpu().numpy().reshape(-1, 3)[:B], packed=packed, lhs=lhs, rhs=rhs, out=out,
                sp=sp)


def check(rl, insts, res, tol=1e-7, rel_tol=1e-8, elementwise=True):
    for b, inst in enumerate(insts):
        ref = spd.seq(inst)
        assert ref["status"] == 0
        ov, ofb, oin = spd.certificate(inst, ref["dS"], ref["dG"])
        where = (b, inst.n, inst.m, inst.N, inst.delta, inst.indefinite)
        assert res["verdict"][b] == int(ov), where
        assert res["first_bad"][b] == ofb, where
        assert tuple(res["inertia"][b]) == oin, where
        assert res["status"][b] == (rl.INST_OK if ov else rl.INST_NOT_PD), (where, res["status"][b])
        assert res["relres"][b] <= rel_tol, (where, res["relres"][b])
        x, u, y = res["sols"][b]
        orr = spd.rel_residual(inst, x, u, y)
        assert orr <= rel_tol, (where, orr)
        assert res["relres"][b] == pytest.approx(orr, rel=1e-3, abs=1e-14), where
        if elementwise:
            scale = max(1.0, *(np.abs(ref[k]).max() for k in ("x", "u", "y") if ref[k].size))
            err = max(np.abs(a - ref[k]).max() if a.size else 0.0 for a, k in zip((x, u, y), ("x", "u", "y")))
            assert err <= tol * scale, (where, err, scale)


def _batch(tag, shapes, spread=1.0):
    out = []
    for i, (n, m, N, delta) in enumerate(shapes):
        out.append(wl.make_instance(n, m, N, delta, (79, tag, i), indefinite=(i % 4 == 3), spd_spread=spread))
    return out


SHAPES = [(4, 2, 12, 1e-2), (12, 4, 30, 1e-4), (20, 10, 9, 1e-2), (6, 3, 0, 1e-1), (40, 6, 7, 1e-3),
          (12, 4, 17, 1e-6), (8, 2, 25, 1e-4), (33, 2, 5, 1e-2), (1, 1, 6, 1e-1), (64, 32, 4, 1e-3)]


@pytest.mark.parametrize("mode,chunk", [("fp64", 0), ("mixed", 0), ("scan", 3), ("scan_bf16", 4)])
def test_spd_matches_oracle(rl, mode, chunk):
    print(f"[gpu] spd mode={mode} chunk={chunk}", flush=True)
    insts = _batch(0, SHAPES)
    res = run(rl, insts, mode, chunk=chunk, max_refine=10 if mode == "scan_bf16" else 4)
    check(rl, insts, res)


def test_spd_condition_spread(rl):
    """Delta_i eigenvalues spread over 10^(+-2) (condition 10^4)."""
    print("[gpu] spd spread 2", flush=True)
    insts = _batch(1, [(12, 4, 40, 1e-3), (5, 3, 20, 1e-2), (24, 8, 10, 1e-4)], spread=2.0)
    res = run(rl, insts, "fp64", max_refine=4)
    check(rl, insts, res)


def test_spd_residual_entry_matches_oracle(rl):
    """rlqr_spd_residual at an arbitrary z against the oracle's residual, row by row."""
    import torch
    print("[gpu] spd residual entry", flush=True)
    insts = _batch(2, SHAPES[:6])
    res = run(rl, insts, "fp64")
    gen = torch.Generator(device="cpu").manual_seed(3)
    z = {k: (v + torch.randn(v.shape, generator=gen, dtype=torch.float64).to(v.device)) for k, v in res["out"].items()}
    r, rr = res["sp"].residual(res["rhs"], z)
    torch.cuda.synchronize()
    packed = res["packed"]
    o = packed.offsets
    sols = wl.unpack_solution(packed, *(z[k].cpu().numpy() for k in ("x", "u", "y")))
    rc = r.cpu().numpy()
    roff = np.zeros(packed.batch + 1, dtype=np.int64)
    np.cumsum([i.N * (i.n + i.m) + i.n + (i.N + 1) * i.n for i in insts], out=roff[1:])
    for b, inst in enumerate(insts):
        ref = spd.residual(inst, *sols[b])
        got = rc[roff[b]:roff[b + 1]]
        np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11 * max(1.0, np.abs(ref).max()))
        assert rr.cpu().numpy()[b] == pytest.approx(spd.rel_residual(inst, *sols[b]), rel=1e-11)
    del o


def test_spd_diagonal_blocks_match_diagonal_path(rl):
    """Diagonal Delta_i given as full blocks: the same certificate and the same
    solution (to refinement tolerance) as the per-stage diagonal path."""
    import torch
    print("[gpu] spd diagonal blocks", flush=True)
    dinsts = [wl.make_instance(n, m, N, 1e-3, (79, 3, i), indefinite=(i == 2), diag_spread=1.0)
              for i, (n, m, N) in enumerate([(12, 4, 20), (6, 2, 9), (20, 10, 7)])]
    finsts = [wl.Instance(*[getattr(d, f) for f in ("n", "m", "N", "delta", "Q", "M", "R", "A", "B", "q", "r",
                                                    "c", "indefinite")],
                          delta_full=np.stack([np.diag(v) for v in d.delta_diag])) for d in dinsts]
    res = run(rl, finsts, "fp64")
    check(rl, finsts, res)
    packed = wl.pack(dinsts)
    lhs, rhs = rl.to_device(packed)
    s = rl.Solver(packed.N, packed.n, packed.m, mode="fp64")
    s.factor(lhs)
    out, st, rr = s.solve(rhs, rel_tol=1e-8, max_refine=3)
    v, fb, ine = s.pivot_inertia()
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy()[:3], res["verdict"])
    assert np.array_equal(fb.cpu().numpy()[:3], res["first_bad"])
    assert np.array_equal(ine.cpu().numpy().reshape(-1, 3)[:3], res["inertia"])
    sols = wl.unpack_solution(packed, *(out[k].cpu().numpy() for k in ("x", "u", "y")))
    for a, b in zip(sols, res["sols"]):
        for va, vb in zip(a, b):
            assert np.abs(va - vb).max() <= 1e-8 * max(1.0, np.abs(va).max())


def test_spd_uniform_batch_full_size(rl):
    """The uniform benchmark batch (4096 x n=12, m=4, N=128, delta=1e-8) with
    full SPD Delta_i (spread 10^(+-1)), float64 and mixed: every instance at
    <= 1e-8, every verdict PD, 32 sampled instances element-wise and by
    certificate against the oracle."""
    import torch
    print("[gpu] spd uniform full size", flush=True)
    insts = [wl.make_instance(12, 4, 128, 1e-8, (1, b, 0), spd_spread=1.0) for b in range(4096)]
    rng = np.random.default_rng(17)
    sample = rng.choice(len(insts), 32, replace=False)
    for mode in ("fp64", "mixed"):
        res = run(rl, insts, mode, max_refine=3)
        assert (res["relres"] <= 1e-8).all(), res["relres"].max()
        assert (res["verdict"] == 1).all()
        sub = {k: (v[sample] if isinstance(v, np.ndarray) else [v[i] for i in sample])
               for k, v in res.items() if k in ("sols", "status", "relres", "verdict", "first_bad", "inertia")}
        check(rl, [insts[i] for i in sample], sub)
        del res
        torch.cuda.empty_cache()
