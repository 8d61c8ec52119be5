"""GPU: graph capture of the whole launch sequence and the autotuned ragged batch.

Graph replays are checked against eager runs on the same data, several
replays in a row with the program's own eager work and synchronizations in
between, each replay after the inputs changed in place. The autotuned ragged
batch (the ragged workload's recipe at reduced size: N ~ U{50..200},
n in {8, 16, 32}, m in {2, 4, 8}, 20% indefinite Q, delta = 1e-4) is checked
against the FP64 oracle instance by instance to the gates of the other
parity tests.
"""
import numpy as np
import pytest

import oracle
from paper_2509_16370_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_16370_amd import rlqr
    return rlqr


@pytest.mark.parametrize("mode,chunk", [("fp64", 0), ("mixed", 0), ("scan", 8)])
def test_graph_replays_match_eager(rl, mode, chunk):
    import torch
    print(f"[gpu] graph replay mode={mode}", flush=True)
    insts = [wl.make_instance(n, m, N, 1e-6, (81, i, 0))
             for i, (n, m, N) in enumerate([(4, 2, 40), (12, 4, 64), (20, 10, 33), (6, 3, 0)])]
    packed = wl.pack(insts)
    lhs, rhs = rl.to_device(packed)
    g = rl.Solver(packed.N, packed.n, packed.m, mode=mode, scan_chunk=chunk)
    e = rl.Solver(packed.N, packed.n, packed.m, mode=mode, scan_chunk=chunk)
    out = {k: g.empty(k) for k in ("x", "u", "y")}
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        status, relres = g.capture(lhs, rhs, out, rel_tol=1e-8, max_refine=3, stream=stream)
    stream.synchronize()
    for rep in range(3):
        # change the data in place between replays (eager torch work on the default stream)
        rhs["q"].mul_(1.0 + 0.5 * rep)
        rhs["c"].add_(0.1)
        lhs["Q"].mul_(1.01)
        torch.cuda.synchronize()
        stream.wait_stream(torch.cuda.current_stream())
        g.replay(stream=stream)
        stream.synchronize()
        e.factor(lhs)
        ref, st_e, rr_e = e.solve(rhs, rel_tol=1e-8, max_refine=3)
        torch.cuda.synchronize()
        for k in ("x", "u", "y"):
            a, b = out[k].cpu().numpy(), ref[k].cpu().numpy()
            assert np.array_equal(a, b), (rep, k, np.abs(a - b).max())
        assert np.array_equal(status.cpu().numpy(), st_e.cpu().numpy())
        assert np.array_equal(relres.cpu().numpy(), rr_e.cpu().numpy())
        assert (relres.cpu().numpy()[:packed.batch] <= 1e-8).all()


def _ragged(count, seed):
    rng = np.random.default_rng(seed)
    ns = rng.choice([8, 16, 32], count)
    ms = rng.choice([2, 4, 8], count)
    Ns = rng.integers(50, 201, count)
    indef = rng.permutation(count) < round(0.2 * count)
    return [wl.make_instance(int(ns[b]), int(ms[b]), int(Ns[b]), 1e-4, (82, b, seed), indefinite=bool(indef[b]))
            for b in range(count)]


def test_autotuned_ragged_batch_matches_oracle(rl):
    import torch
    from paper_2509_16370_amd import tune
    print("[gpu] autotuned ragged batch", flush=True)
    insts = _ragged(72, 0)
    packed = wl.pack(insts)
    plan = tune.tune(packed, rel_tol=1e-8, max_refine=3, reps=1, lengths=(16, 64), log=print)
    assert set(plan) == set(tune.buckets(packed))
    assert all(np.isfinite(c.ms) for c in plan.values())
    lhs, rhs = rl.to_device(packed)
    tb = tune.TunedBatch(packed, plan, lhs, rhs, rel_tol=1e-8, max_refine=3)
    for rep in range(2):
        out, status, relres = tb.run()
        torch.cuda.synchronize()
    sols = wl.unpack_solution(packed, *(out[k].cpu().numpy() for k in ("x", "u", "y")))
    verdict, first_bad, inertia = tb.solver.pivot_inertia()
    torch.cuda.synchronize()
    verdict, first_bad = verdict.cpu().numpy(), first_bad.cpu().numpy()
    inertia = inertia.cpu().numpy().reshape(-1, 3)
    status, relres = status.cpu().numpy(), relres.cpu().numpy()
    for b, inst in enumerate(insts):
        ref = oracle.seq(inst)
        if ref["status"]:
            assert status[b] == rl.INST_SINGULAR
            continue
        ov, ofb, oin = oracle.certificate(inst, ref["dS"], ref["dG"])
        assert verdict[b] == int(ov) and first_bad[b] == ofb, (b, inst.n, inst.m, inst.N)
        if ov:
            assert tuple(inertia[b]) == oin
        assert relres[b] <= 1e-8, (b, relres[b])
        if ov:
            scale = max(1.0, *(np.abs(ref[k]).max() for k in ("x", "u", "y")))
            err = max(np.abs(a - ref[k]).max() for a, k in zip(sols[b], ("x", "u", "y")))
            assert err <= 1e-7 * scale, (b, err)


_RAGGED = {}


def _full_ragged():
    """The ragged benchmark batch and the oracle's solution, certificate and
    residual of every instance (computed once per module)."""
    if not _RAGGED:
        insts = wl.batched_ragged()
        packed = wl.pack(insts)
        x, u, y, ost, _, dS, dG = oracle.seq_batch(packed, pivots=True)
        certs = oracle.certificate_batch(packed, insts, dS, dG)
        refs = wl.unpack_solution(packed, x, u, y)
        orel = np.array([oracle.rel_residual(inst, *refs[b]) for b, inst in enumerate(insts)])
        _RAGGED.update(insts=insts, packed=packed, certs=certs, refs=refs, orel=orel, ost=ost)
    return _RAGGED


def _check_full_ragged(rl, out, status, relres, verdict, first_bad, inertia):
    """Every instance of the full ragged batch: certificate (verdict, first
    failing pivot, inertia) equal to the oracle's, status, relative residual
    <= 1e-8, and the solution element-wise within max(1e-7, 1e4 * (gpu +
    oracle relative residual)) * max(1, |z|) of the oracle's -- indefinite
    instances included (their KKT system has one solution; the oracle's own
    residual on the worst of them is ~4e-7, which the bound accounts for)."""
    import torch
    torch.cuda.synchronize()
    R = _full_ragged()
    insts, packed = R["insts"], R["packed"]
    B = packed.batch
    rr = relres.cpu().numpy()[:B]
    st = status.cpu().numpy()[:B]
    vd, fb = verdict.cpu().numpy()[:B], first_bad.cpu().numpy()[:B]
    ine = inertia.cpu().numpy().reshape(-1, 3)[:B]
    assert (rr <= 1e-8).all(), rr.max()
    assert (R["ost"] == 0).all()
    sols = wl.unpack_solution(packed, *(out[k].cpu().numpy() for k in ("x", "u", "y")))
    nfalse = 0
    for b, inst in enumerate(insts):
        ov, ofb, oin = R["certs"][b]
        assert vd[b] == int(ov) and fb[b] == ofb, (b, vd[b], ofb)
        assert tuple(ine[b]) == oin, (b, tuple(ine[b]), oin)
        assert st[b] == (rl.INST_OK if ov else rl.INST_NOT_PD), (b, st[b])
        nfalse += 0 if ov else 1
        ref = R["refs"][b]
        scale = max(1.0, *(np.abs(a).max() for a in ref if a.size))
        err = max(np.abs(a - c).max() if a.size else 0.0 for a, c in zip(sols[b], ref))
        assert err <= max(1e-7, 1e4 * (rr[b] + R["orel"][b])) * scale, (b, err, scale)
    # every indefinite instance fails the certificate (the parity is not vacuous)
    assert nfalse >= sum(1 for i in insts if i.indefinite)


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_full_size_ragged_batch(rl, mode):
    """The ragged benchmark batch at full size (1024 instances, N up to 1000,
    205 indefinite, delta = 1e-4), tile classes on their concurrent streams,
    every instance checked against the oracle (see _check_full_ragged)."""
    import torch
    print(f"[gpu] full-size ragged batch mode={mode}", flush=True)
    R = _full_ragged()
    packed = R["packed"]
    lhs, rhs = rl.to_device(packed)
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode)
    s.factor(lhs)
    out, status, relres = s.solve(rhs, rel_tol=1e-8, max_refine=3)
    verdict, first_bad, inertia = s.pivot_inertia()
    _check_full_ragged(rl, out, status, relres, verdict, first_bad, inertia)
    del s
    torch.cuda.empty_cache()


@pytest.mark.parametrize("source", ["tuner", "mixed_paths"])
def test_full_size_tuned_graph(rl, source):
    """The ragged benchmark batch at full size through one captured graph of
    one handle under a tuning plan: the plan the coordinate-descent tuner
    picks (one round, candidates float64 / mixed / scan with L = 64), and a
    fixed plan that puts every path into the one graph (float64 for n = 32,
    the float32-product recursion for n = 16, the scan with L = 32 for n = 8).
    Two replays with the graph's own eager synchronizations between them;
    every instance checked against the oracle."""
    import torch
    from paper_2509_16370_amd import tune
    print(f"[gpu] full-size tuned graph source={source}", flush=True)
    R = _full_ragged()
    packed = R["packed"]
    lhs, rhs = rl.to_device(packed)
    if source == "tuner":
        plan = tune.tune_batch(packed, lhs, rhs, rel_tol=1e-8, max_refine=3, reps=1, lengths=(64,), rounds=1,
                               log=print)
    else:
        plan = {bk: (tune.Choice("fp64") if bk[0] == 32 else
                     tune.Choice("mixed") if bk[0] == 16 else tune.Choice("scan", 32))
                for bk in tune.buckets(packed)}
    print(f"[gpu] plan: { {f'{k[0]},{k[1]}': c.key() for k, c in plan.items()} }", flush=True)
    tb = tune.TunedBatch(packed, plan, lhs, rhs, rel_tol=1e-8, max_refine=3)
    for rep in range(2):
        out, status, relres = tb.run()
        torch.cuda.synchronize()
    verdict, first_bad, inertia = tb.solver.pivot_inertia()
    _check_full_ragged(rl, out, status, relres, verdict, first_bad, inertia)
    del tb
    torch.cuda.empty_cache()
