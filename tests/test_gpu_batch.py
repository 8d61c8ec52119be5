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


@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_full_size_ragged_batch(rl, mode):
    """The ragged benchmark batch at full size (1024 instances, N up to 1000,
    205 indefinite, delta = 1e-4), tile classes on their concurrent streams:
    every instance meets 1e-8; certificate parity on a sample against the
    oracle's pivots; every positive definite instance element-wise against
    the oracle's batch solve."""
    import torch
    print(f"[gpu] full-size ragged batch mode={mode}", flush=True)
    insts = wl.batched_ragged()
    packed = wl.pack(insts)
    lhs, rhs = rl.to_device(packed)
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode)
    s.factor(lhs)
    out, status, relres = s.solve(rhs, rel_tol=1e-8, max_refine=3)
    verdict, first_bad, _ = s.pivot_inertia()
    torch.cuda.synchronize()
    B = packed.batch
    rr = relres.cpu().numpy()[:B]
    assert (rr <= 1e-8).all(), rr.max()
    vd, fb = verdict.cpu().numpy()[:B], first_bad.cpu().numpy()[:B]
    st = status.cpu().numpy()[:B]
    assert (vd[[b for b, i in enumerate(insts) if i.indefinite]] == 0).all()
    rng = np.random.default_rng(11)
    for b in rng.choice(B, 48, replace=False):
        ref = oracle.seq(insts[b])
        ov, ofb, _ = oracle.certificate(insts[b], ref["dS"], ref["dG"])
        assert vd[b] == int(ov) and fb[b] == ofb, b
        assert st[b] == (0 if ov else 1), b
    x, u, y, ost, _ = oracle.seq_batch(packed)
    sols = wl.unpack_solution(packed, *(out[k].cpu().numpy() for k in ("x", "u", "y")))
    refs = wl.unpack_solution(packed, x, u, y)
    for b, inst in enumerate(insts):
        if inst.indefinite:
            continue
        scale = max(1.0, *(np.abs(a).max() for a in refs[b] if a.size))
        err = max(np.abs(a - c).max() if a.size else 0.0 for a, c in zip(sols[b], refs[b]))
        assert err <= 1e-7 * scale, (b, err)
