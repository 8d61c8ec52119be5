#!/usr/bin/env python
"""Benchmark: dual-regularized LQR stage-solves per second at 1e-8 relative KKT
residual, mixed precision vs plain float64, on one MI355X.

Workload: a uniform batch of 4096 independent instances, n=12, m=4, N=128
(quadrotor-sized), delta=1e-8, generated with the seeded recipe of
paper_2509_16370_amd.workloads; inputs are resident in HBM before timing.
One step = rlqr_factor_rhs + rlqr_solve (the factorization with the solve's
backward vector pass in its stage loop, then the forward rollout, float64
residual and iterative refinement until every instance reaches
||K z + b||_inf <= 1e-8 ||b||_inf). A stage-solve is one stage of one
instance carried through that step; instances that miss the tolerance are
not counted.

Prints ONE JSON line. `value` is the mixed path; the plain float64 path, the
roofline of the dominant kernel (the factorization) and the CPU oracle
baseline are reported beside it.

Other workloads (--workload): long_horizon (one instance, n=64, m=32,
N=16384, delta=1e-6, refined to 1e-10; the parallel-in-time scan, with float32
and with bfloat16 combine products, and with p and c carried through the scan
(scan_pc) instead of the p-recurrence, against the float64 sequential recursion) and batched_ragged (1024 instances,
N ~ U{50..1000}, n in {8,16,32}, m in {2,4,8}, 20% indefinite Q, delta=1e-4;
the autotuned single-graph launch against the float64 sequential path) and
cross_stage (the uniform batch with p = 4 variables shared by every stage:
the arrowhead step of Section "Cross-Stage Variables", factor + solve +
refinement of the whole system, float64 and mixed). --diag-spread s gives the
uniform batch a per-stage diagonal Delta_i (entries delta * 10^U(-s, s), the
separate per-constraint penalties the definition allows). stage_eq: the
uniform batch with --ne equality rows per stage eliminated into the LQR
(rlqr_eq_reduce, factor, solve, rlqr_eq_recover). single_small: one instance
n=4, m=2, N=32, delta=1e-6 (a latency measurement: float64 and mixed).
ipm: the regularized interior-point method on 2048 trajectory problems
(n=12, m=4, N=256, tolerance 1e-6), cold start against the learned warm
start (network trained first on --train method-generated solutions); the
line reports both runs' iterations and wall times.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "dual-reg LQR stage-solves/s at 1e-8 KKT residual, mixed vs FP64 plain"
MW_WAVES = 0  # --mw-waves: wavefronts per instance for 16 < n + m <= 48 (0: the library's default)
HBM_PEAK_GBS = 8000.0
REL_TOL = 1e-8


def factor_algorithmic_bytes(n, m, elem_bytes, with_rhs=True, diag=False):
    """Per stage: read Q, M, R, A, B (float64) and write the minimal
    factorization a solve needs -- K (m x n), the symmetric P and S_hat^{-1}
    (n(n+1)/2 each) and the symmetric G^{-1} (m(m+1)/2) -- in the working
    precision; with the right-hand side (rlqr_factor_rhs) also read q, r, c
    and write p, k (float64); with a per-stage diagonal Delta_i also read its
    n entries (float64)."""
    lhs = 8 * (n * n + n * m + m * m + n * n + n * m) + (8 * n if diag else 0)
    handoff = elem_bytes * (m * n + n * (n + 1) + m * (m + 1) // 2)
    vec = 8 * ((2 * n + m) + (n + m)) if with_rhs else 0
    return lhs + handoff + vec


def run_mode(torch, rl, packed, lhs, rhs, mode, steps, warmup, max_refine, rel_tol=REL_TOL, chunk=0, plan=None):
    stream = torch.cuda.current_stream()
    if plan is not None:  # autotuned: one handle, one graph launch per step
        from paper_2509_16370_amd import tune
        tb = tune.TunedBatch(packed, plan, lhs, rhs, rel_tol=rel_tol, max_refine=max_refine)
        s = tb.solver

        def step(ev=None):
            if ev:
                ev[0].record(stream)
                ev[1].record(stream)
            out, st, rr = tb.run()
            if ev:
                ev[2].record(stream)
            return out, st, rr
    else:
        # scan_pc: the scan mode carrying p and c through the reverse scan
        s = rl.Solver(packed.N, packed.n, packed.m, mode="scan" if mode == "scan_pc" else mode,
                      scan_chunk=chunk, scan_carry_pc=mode == "scan_pc", mw_waves=MW_WAVES)
        out = {k: s.empty(k) for k in ("x", "u", "y")}

        def step(ev=None):
            if ev:
                ev[0].record(stream)
            s.factor(lhs, rhs)  # rlqr_factor_rhs: the solve's backward vector pass rides in the factor
            if ev:
                ev[1].record(stream)
            res = s.solve(rhs, out=out, rel_tol=rel_tol, max_refine=max_refine)
            if ev:
                ev[2].record(stream)
            return res

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        _, status, relres = step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    factor_ms = [e[0].elapsed_time(e[1]) for e in evs]
    solve_ms = [e[1].elapsed_time(e[2]) for e in evs]
    if plan is not None:
        # the graph has no split point: time the same handle's factorization
        # eagerly (same kernels, same launch configuration) for the roofline
        fev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(max(steps, 1))]
        for e in fev:
            e[0].record(stream)
            s.factor(lhs, rhs)
            e[1].record(stream)
        torch.cuda.synchronize()
        factor_ms = [e[0].elapsed_time(e[1]) for e in fev]
        solve_ms = None
    status = status.cpu().numpy()[:packed.batch]
    relres = relres.cpu().numpy()[:packed.batch]
    ok = (relres <= rel_tol) & ((status == rl.INST_OK) | (status == rl.INST_NOT_PD))
    stages = int(packed.N[ok].sum())
    ms_per_step = 1e3 * wall / steps
    import numpy as np
    path = s.precision_path()
    torch.cuda.synchronize()
    path = path.cpu().numpy()[:packed.batch]
    paths = {name: int((path == code).sum()) for name, code in
             (("fp32", rl.PATH_FP32), ("fp64", rl.PATH_FP64), ("fp64_guard", rl.PATH_FP64_GUARD),
              ("fp64_redo", rl.PATH_FP64_REDO))}
    return dict(
        precision_paths=paths,
        value=stages / (ms_per_step * 1e-3),
        ms_per_step=ms_per_step,
        factor_ms=float(np.median(factor_ms)),
        solve_ms=float(np.median(solve_ms)) if solve_ms is not None else None,
        instances_ok=int(ok.sum()),
        max_relres=float(relres.max()),
        median_relres=float(np.median(relres)),
        status_counts={int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
        workspace_bytes=s.workspace_bytes,
        tuning=s.tuning,
    )


def run_xs_mode(torch, rl, packed, lhs, rhs, xsd, mode, steps, warmup, max_refine, rel_tol=REL_TOL):
    """Cross-stage step: rlqr_xs_factor (LQR factor + p column solves + S) and
    rlqr_xs_solve (one LQR solve, the p x p step, arrowhead refinement)."""
    import numpy as np
    stream = torch.cuda.current_stream()
    p = xsd["p"]
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode, max_rhs=p)  # the p column solves run together
    x = rl.CrossStage(s, p)
    out = {k: s.empty(k) for k in ("x", "u", "y")}
    out["theta"] = torch.empty(packed.batch * p, dtype=torch.float64, device="cuda:0")
    J = {k: xsd[k] for k in ("Jq", "Jr", "Jc")}

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        x.factor(lhs, J, xsd["H"], rel_tol=rel_tol, max_refine=max_refine)
        if ev:
            ev[1].record(stream)
        res = x.solve(rhs, xsd["rth"], out=out, rel_tol=rel_tol, max_refine=max_refine)
        if ev:
            ev[2].record(stream)
        return res

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        _, status, relres = step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = status.cpu().numpy()[:packed.batch]
    relres = relres.cpu().numpy()[:packed.batch]
    ok = (relres <= rel_tol) & ((status == rl.INST_OK) | (status == rl.INST_NOT_PD))
    stages = int(packed.N[ok].sum())
    ms_per_step = 1e3 * wall / steps
    return dict(
        value=stages / (ms_per_step * 1e-3),
        ms_per_step=ms_per_step,
        factor_ms=float(np.median([e[0].elapsed_time(e[1]) for e in evs])),
        solve_ms=float(np.median([e[1].elapsed_time(e[2]) for e in evs])),
        instances_ok=int(ok.sum()),
        max_relres=float(relres.max()),
        median_relres=float(np.median(relres)),
        status_counts={int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
        workspace_bytes=s.workspace_bytes + x.workspace_bytes,
    )


def run_eq_mode(torch, rl, packed, lhs, rhs, eqd, ne, mode, steps, warmup, max_refine, rel_tol=REL_TOL):
    """Newton step with stagewise equality rows: rlqr_eq_reduce (into
    preallocated reduced blocks), rlqr_factor_rhs + rlqr_solve on the reduced
    LQR, rlqr_eq_recover. Events: reduce | factor | solve + recover."""
    import numpy as np
    stream = torch.cuda.current_stream()
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode)
    st = rl.StageEquality(s, [ne] * packed.batch)
    red = {k: torch.empty_like(lhs[k]) for k in ("Q", "M", "R")}
    red.update({k: torch.empty_like(rhs[k]) for k in ("q", "r")})
    out = {k: s.empty(k) for k in ("x", "u", "y")}
    w = torch.empty(max(int(st.offsets["v"][-1]), 1), dtype=torch.float64, device="cuda:0")

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        lhs2, rhs2 = st.reduce(lhs, rhs, eqd, out=red)
        if ev:
            ev[1].record(stream)
        s.factor(lhs2, rhs2)
        if ev:
            ev[2].record(stream)
        res = s.solve(rhs2, out=out, rel_tol=rel_tol, max_refine=max_refine)
        st.recover(eqd, out, w=w)
        if ev:
            ev[3].record(stream)
        return res

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        _, status, relres = step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = status.cpu().numpy()[:packed.batch]
    relres = relres.cpu().numpy()[:packed.batch]
    ok = (relres <= rel_tol) & ((status == rl.INST_OK) | (status == rl.INST_NOT_PD))
    stages = int(packed.N[ok].sum())
    ms_per_step = 1e3 * wall / steps
    return dict(
        value=stages / (ms_per_step * 1e-3),
        ms_per_step=ms_per_step,
        reduce_ms=float(np.median([e[0].elapsed_time(e[1]) for e in evs])),
        factor_ms=float(np.median([e[1].elapsed_time(e[2]) for e in evs])),
        solve_ms=float(np.median([e[2].elapsed_time(e[3]) for e in evs])),
        instances_ok=int(ok.sum()),
        max_relres=float(relres.max()),
        median_relres=float(np.median(relres)),
        status_counts={int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
        workspace_bytes=s.workspace_bytes + st.workspace_bytes,
    )


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline_eq(insts, eqs, count=512):
    """The elimination oracle (reduce in numpy, the sequential C oracle over
    the reduced batch on all host threads, recover) on the first `count`
    instances."""
    import oracle
    from oracle import eqstep
    from paper_2509_16370_amd import workloads as wl
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
    t0 = time.perf_counter()
    red = [eqstep.reduce(i, e) for i, e in zip(insts[:count], eqs[:count])]
    packed = wl.pack(red)
    x, u, y, st, used = oracle.seq_batch(packed, nthreads=threads)
    for b, (xb, ub, yb) in enumerate(wl.unpack_solution(packed, x, u, y)):
        eqstep.recover(red[b], eqs[b], xb, ub)
    t = time.perf_counter() - t0
    stages = int(packed.N.sum())
    return dict(value=stages / t, unit="stage-solves/s", cores=int(used), kind="oracle", cpu_model=cpu_model(),
                sample=f"first {count} instances of the batch: numpy reduction, the sequential FP64 oracle "
                       f"over the reduced batch on {used} threads, numpy recovery of w",
                seconds=t)


def cpu_baseline_xs(insts, xs, count=256):
    """The cross-stage oracle (the paper's Schur route, p + 2 sequential
    Riccati solves per instance) on the first `count` instances, one thread."""
    from oracle import crossstage as ocs
    t0 = time.perf_counter()
    stages = 0
    for inst, x in zip(insts[:count], xs[:count]):
        ocs.schur(inst, x.J, x.H, (inst.q, inst.r, inst.c), x.rth)
        stages += inst.N
    t = time.perf_counter() - t0
    return dict(value=stages / t, unit="stage-solves/s", cores=1, kind="oracle", cpu_model=cpu_model(),
                sample=f"first {count} instances of the batch, the cross-stage oracle's Schur route "
                       f"(p + 2 sequential float64 Riccati solves each), one thread",
                seconds=t)


def cpu_baseline(packed, seconds_target=10.0, sample=None, threads=0):
    """The FP64 oracle, as it stands, over the same batch (or the named sample) on the host cores."""
    import numpy as np
    import oracle
    threads = threads or int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
    times = []
    used = 1
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        x, u, y, st, used = oracle.seq_batch(packed, nthreads=threads)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > seconds_target or len(times) >= (5 if packed.batch > 1 else 200):
            break
    t = float(np.median(times))
    stages = int(packed.N.sum())
    what = sample or f"full batch ({packed.batch} instances, {stages} stages)"
    return dict(value=stages / t, unit="stage-solves/s", cores=int(used), kind="oracle", cpu_model=cpu_model(),
                sample=f"{what}, median of {len(times)} runs of the sequential FP64 oracle, instances spread "
                       f"over {used} threads",
                seconds=t)


def run_ipm(torch, rl, args):
    """Interior-point workload: train the warm-start network on method-generated
    solutions (untimed), then solve the 2048 evaluation problems cold and warm.
    Returns the JSON line's fields."""
    import numpy as np
    from paper_2509_16370_amd import warmstart as wsm
    from paper_2509_16370_amd import workloads as wl
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    F, T = wsm.make_dataset(args.train, log=log)
    log(f"[bench] {F.shape[0]} training solutions in {time.perf_counter() - t0:.1f} s")
    net = wsm.WarmStart(F.shape[1], T.shape[1], dtype="bf16")
    t0 = time.perf_counter()
    hist = net.fit(F, T, epochs=args.epochs, log=log)
    train_s = time.perf_counter() - t0
    ts = wl.trajectory_problems(2048, stream=0)
    wsm.solve_batch(ts, max_iter=3)  # warm the driver and the library up (untimed)
    torch.cuda.synchronize()
    ic, cc, _, _, _, _, tc = wsm.solve_batch(ts)
    Fe = torch.from_numpy(wsm.features(ts)).cuda()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    warm = net.predict(Fe)
    torch.cuda.synchronize()
    tpred = time.perf_counter() - t1
    iw, cw, _, _, _, _, tw = wsm.solve_batch(ts, warm=warm)
    tw += tpred
    both = (cc > 0) & (cw > 0)
    N = ts.N
    res = dict(
        problems=int(ts.batch), cold_converged=int(cc.sum()), warm_converged=int(cw.sum()),
        cold_mean_iterations=float(ic[both].mean()), warm_mean_iterations=float(iw[both].mean()),
        cold_seconds=tc, warm_seconds=tw, predict_seconds=tpred, train_solutions=int(F.shape[0]),
        train_epochs=args.epochs, train_seconds=train_s, final_loss=float(hist[-1]),
        cold_stage_solves_per_s=float(ic.sum()) * N / tc, warm_stage_solves_per_s=float(iw.sum()) * N / tw)
    return res, ts


def cpu_baseline_ipm(ts, count=8):
    """The CPU interior-point oracle (numpy, the sequential C oracle for each
    Newton step's LQR) on the first `count` problems, cold start, one thread."""
    from oracle import ipm as oipm
    t0 = time.perf_counter()
    stage_solves = 0
    for b in range(count):
        st, it, ok = oipm.solve(oipm.Problem(ts, b))
        stage_solves += it * ts.N
    t = time.perf_counter() - t0
    return dict(value=stage_solves / t, unit="stage-solves/s", cores=1, kind="oracle", cpu_model=cpu_model(),
                sample=f"first {count} of the 2048 problems, the CPU interior-point oracle from a cold start "
                       f"(Newton-step LQR stage-solves per second), one thread", seconds=t)


def scan_factor_flops(n, m):
    """Algorithmic flops per stage of the parallel-in-time factorization:
    one interval combine (single inversion of I + C P and six n x n products,
    about 16.7 n^3), the segment recursion (6.3 n^3 + 6 n^2 m + 4 n m^2 + m^3/3)
    and the transfer-matrix product (4 n^3 + 2 n^2 m)."""
    return 16.7 * n ** 3 + 6.3 * n ** 3 + 6 * n * n * m + 4 * n * m * m + m ** 3 / 3 + 4 * n ** 3 + 2 * n * n * m


def load_counters(name):
    """HBM traffic per launch from a committed counter summary, or None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = dict(line.split("=", 1) for line in open(path).read().splitlines() if "=" in line and not line.startswith("#"))
    srcs = kv.get("sources", "").split(",")
    h = hashlib.sha256()
    for f in srcs:
        fp = os.path.join(ROOT, f.strip())
        if not os.path.exists(fp):
            return None
        h.update(open(fp, "rb").read())
    if h.hexdigest() != kv.get("source_sha256", "").strip():
        return None
    return float(kv["hbm_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched_uniform",
                    choices=["batched_uniform", "long_horizon", "batched_ragged", "cross_stage", "stage_eq",
                             "single_small", "ipm"])
    ap.add_argument("--train", type=int, default=50000, help="ipm: training problems for the warm start")
    ap.add_argument("--epochs", type=int, default=40, help="ipm: training epochs")
    ap.add_argument("--ne", type=int, default=2, help="stage_eq: equality rows per stage")
    ap.add_argument("--p", type=int, default=4, help="cross_stage: number of cross-stage variables")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--nx", type=int, default=12, help="batched_uniform: state size")
    ap.add_argument("--nu", type=int, default=4, help="batched_uniform: control size")
    ap.add_argument("--horizon", type=int, default=128, help="batched_uniform: N")
    ap.add_argument("--chunk", type=int, default=0,
                    help="scan modes: stages per segment L (0: the library's default)")
    ap.add_argument("--delta", type=float, default=1e-8)
    ap.add_argument("--diag-spread", type=float, default=None,
                    help="batched_uniform: per-stage diagonal Delta_i with entries delta * 10^U(-s, s)")
    ap.add_argument("--max-refine", type=int, default=3)
    ap.add_argument("--modes", default=None)
    ap.add_argument("--mw-waves", type=int, default=0,
                    help="wavefronts per instance of the kernels for 16 < n + m <= 48 (4 or 8; 0: default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="launch one plain 1 GiB float32 copy kernel (rmlp_cast) for counter calibration")
    args = ap.parse_args()
    global MW_WAVES
    MW_WAVES = args.mw_waves
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batch is "
              "independent instances and would shard by instance across GPUs, which this "
              "build does not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2509_16370_amd import workloads as wl
    from paper_2509_16370_amd import rlqr as rl

    wk = args.workload
    t0 = time.perf_counter()
    rel_tol, max_refine = REL_TOL, args.max_refine
    diag = args.diag_spread is not None
    if diag and wk != "batched_uniform":
        print("--diag-spread applies to the batched_uniform workload only", file=sys.stderr)
        sys.exit(2)
    if wk == "batched_uniform":
        n, m, N = args.nx, args.nu, args.horizon
        specs = wl.uniform_specs(batch=args.batch, n=n, m=m, N=N, delta=args.delta)
        if diag:
            specs = [s + (False, args.diag_spread) for s in specs]
        packed = wl.pack_parallel(specs, workers=args.workers)
        modes = (args.modes or "fp64,mixed").split(",")
        head = "mixed"
        reg = (f"per-stage diagonal Delta_i with entries delta * 10^U(-{args.diag_spread:g}, {args.diag_spread:g}), "
               f"delta={args.delta:g}") if diag else f"delta={args.delta:g}"
        desc = (f"batched uniform dual-regularized LQR: {args.batch} instances, n={n}, m={m}, N={N}, "
                f"{reg}, refined to {REL_TOL:g} relative KKT residual")
        cfg = {"batch": args.batch, "nx": n, "nu": m, "N": N, "delta": args.delta}
        if diag:
            cfg["delta_diag_spread"] = args.diag_spread
    elif wk == "stage_eq":
        n, m, N = args.nx, args.nu, args.horizon
        insts = wl.batched_uniform(batch=args.batch, n=n, m=m, N=N, delta=args.delta)
        packed = wl.pack(insts)
        eqs = [wl.make_stage_eq(inst, args.ne, (1, b, 0)) for b, inst in enumerate(insts)]
        modes = (args.modes or "fp64,mixed").split(",")
        head = "fp64"
        desc = (f"Newton step with stagewise equality rows: {args.batch} instances, n={n}, m={m}, N={N}, "
                f"delta={args.delta:g}, {args.ne} equality rows per stage (penalties 1e3 * 10^U(-1, 1)), "
                f"eliminated into the LQR, refined to {REL_TOL:g} relative KKT residual, multipliers recovered")
        cfg = {"batch": args.batch, "nx": n, "nu": m, "N": N, "delta": args.delta, "ne": args.ne}
    elif wk == "single_small":
        insts = wl.single_small()
        packed = wl.pack(insts)
        args.delta = 1e-6
        modes = (args.modes or "fp64,mixed").split(",")
        head = "fp64"
        desc = ("single small dual-regularized LQR: n=4, m=2, N=32, delta=1e-6, refined to 1e-8 "
                "(one instance: a latency measurement)")
        cfg = {"batch": 1, "nx": 4, "nu": 2, "N": 32, "delta": 1e-6}
    elif wk == "ipm":
        res, ts = run_ipm(torch, rl, args)
        fb = factor_algorithmic_bytes(ts.n, ts.m, 8)
        achieved = res["warm_stage_solves_per_s"] * fb / 1e9
        line = {
            "metric": METRIC, "value": res["warm_stage_solves_per_s"], "unit": "stage-solves/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": 1e3 * res["warm_seconds"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "regularized interior-point method, 2048 trajectory problems (n=12, m=4, "
                                   "N=256, x+ = x + 0.05 tanh(A x + B u), |u| <= 1, 2 state rows per stage), "
                                   "tolerance 1e-6, learned warm start vs cold start; value = Newton-step "
                                   "LQR stage-solves per second of the warm run",
                       "batch": 2048, "nx": ts.n, "nu": ts.m, "N": ts.N, "tol": 1e-6},
            "ipm": res,
            "roofline": {"kernel": "interior-point loop (all launches; factorization bytes per stage-solve)",
                         "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                         "algorithmic_bytes_per_stage_solve": fb},
        }
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_ipm(ts)
        print(json.dumps(line), flush=True)
        return
    elif wk == "long_horizon":
        inst = wl.long_horizon()[0]
        packed = wl.pack([inst])
        rel_tol, max_refine = 1e-10, 6
        modes = (args.modes or "fp64,scan,scan_pc,scan_bf16").split(",")
        head = "scan"
        desc = ("single long-horizon dual-regularized LQR: n=64, m=32, N=16384, delta=1e-6, "
                "refined to 1e-10 relative KKT residual; parallel-in-time scan vs float64 sequential")
        cfg = {"batch": 1, "nx": 64, "nu": 32, "N": 16384, "delta": 1e-6}
    elif wk == "cross_stage":
        n, m, N = args.nx, args.nu, args.horizon
        insts = wl.batched_uniform(batch=args.batch, n=n, m=m, N=N, delta=args.delta)
        packed = wl.pack(insts)
        xs_data = [wl.make_cross_stage(inst, args.p, (1, b, 0)) for b, inst in enumerate(insts)]
        modes = (args.modes or "fp64,mixed").split(",")
        head = "fp64"
        desc = (f"cross-stage Newton step: {args.batch} instances, n={n}, m={m}, N={N}, delta={args.delta:g}, "
                f"p={args.p} variables shared by all stages (arrowhead Schur route), refined to "
                f"{REL_TOL:g} relative residual of the whole system")
        cfg = {"batch": args.batch, "nx": n, "nu": m, "N": N, "delta": args.delta, "p": args.p}
    else:
        insts = wl.batched_ragged()
        packed = wl.pack(insts)
        args.delta = 1e-4
        modes = (args.modes or "fp64,mixed,tuned").split(",")
        head = "tuned"
        desc = ("batched ragged dual-regularized LQR: 1024 instances, N ~ U{50..1000}, n in {8,16,32}, "
                "m in {2,4,8}, 20% indefinite Q, delta=1e-4, refined to 1e-8; autotuned single-graph launch")
        cfg = {"batch": packed.batch, "stages": int(packed.N.sum()), "delta": 1e-4}
    print(f"[bench] generated {wk} in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    lhs, rhs = rl.to_device(packed, "cuda:0")
    torch.cuda.synchronize()
    if args.calibrate_copy:
        cnt = 1 << 28
        src = torch.ones(cnt, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        rl.rmlp_cast(rl.RMLP_F32, cnt, src, dst)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {cnt * 4} bytes read, {cnt * 4} bytes written", file=sys.stderr, flush=True)
        del src, dst

    eqd = None
    if wk == "stage_eq":
        cs = wl.pack_stage_eq(packed, eqs)
        eqd = {k: torch.from_numpy(cs[k]).to("cuda:0") for k in ("E", "r", "eta")}
        torch.cuda.synchronize()
    xsd = None
    if wk == "cross_stage":
        cs = wl.pack_cross_stage(packed, xs_data)
        xsd = {k: torch.from_numpy(v).to("cuda:0") for k, v in cs.items()}
        xsd["p"] = args.p
        torch.cuda.synchronize()

    results = {}
    for mode in modes:
        steps, warmup = args.steps, args.warmup
        if wk == "long_horizon" and mode == "fp64":  # the sequential float64 recursion takes seconds per step
            steps, warmup = max(1, args.steps // 10), 1
        plan = None
        if mode == "tuned":
            from paper_2509_16370_amd import tune
            t1 = time.perf_counter()
            plan = tune.tune_batch(packed, lhs, rhs, rel_tol=rel_tol, max_refine=max_refine, reps=2,
                                   log=lambda msg: print(msg, file=sys.stderr, flush=True))
            print(f"[bench] tuned {len(plan)} buckets in {time.perf_counter() - t1:.1f}s: "
                  + ", ".join(f"{k}: {c.key()}" for k, c in plan.items())
                  + f"; waves per instance {plan.mw_waves or 4}", file=sys.stderr, flush=True)
        if eqd is not None:
            results[mode] = run_eq_mode(torch, rl, packed, lhs, rhs, eqd, args.ne, mode, steps, warmup,
                                        max_refine, rel_tol=rel_tol)
        elif xsd is not None:
            results[mode] = run_xs_mode(torch, rl, packed, lhs, rhs, xsd, mode, steps, warmup, max_refine,
                                        rel_tol=rel_tol)
        else:
            results[mode] = run_mode(torch, rl, packed, lhs, rhs, mode, steps, warmup, max_refine,
                                     rel_tol=rel_tol, chunk=args.chunk, plan=plan)
        if plan is not None:
            results[mode]["plan"] = {f"{k[0]},{k[1]}": c.key() for k, c in plan.items()}
            results[mode]["plan"]["waves_per_instance"] = plan.mw_waves or 4
        print(f"[bench] {mode}: {json.dumps(results[mode])}", file=sys.stderr, flush=True)

    head = head if head in results else modes[0]
    r = results[head]
    if wk == "long_horizon":
        flops = scan_factor_flops(64, 32) * 16384
        achieved = flops / (r["factor_ms"] * 1e-3) / 1e12
        roof = {"kernel": "rlqr_factor (scan elements, chunk reduce, scan tree, segment recursion, transfer)",
                "bound": "mfma", "achieved": achieved, "peak": 157.3, "unit": "TFLOP/s", "frac": achieved / 157.3,
                "traffic": None, "algorithmic_flops_per_stage": scan_factor_flops(64, 32),
                "launch_ms": r["factor_ms"]}
        dtype = "f32+f64"
    elif wk == "cross_stage":
        # the whole step against HBM, per stage: the factorization (LHS read,
        # factorization written); two solve passes (the p stacked column
        # solves, then the r_w solve), each reading the factorization and A, B
        # twice (backward and forward) and Q, M, R once (its residual), plus
        # per right-hand side its q, r, c read and x, u, y written; the
        # arrowhead residual re-reading the LHS; the cross-stage vector passes
        # (6p + 10 vectors of the right-hand-side length read or written)
        elem = 8 if head == "fp64" else 4
        p = args.p
        handoff = elem * (m * n + n * (n + 1) + m * (m + 1) // 2)
        lhs_b = 8 * (2 * n * n + 2 * n * m + m * m)
        vec_b = 8 * (2 * n + m)
        per_stage = (factor_algorithmic_bytes(n, m, elem, with_rhs=False)
                     + 2 * (2 * handoff + 16 * (n * n + n * m) + 8 * (n * n + n * m + m * m))
                     + (p + 1) * 2 * vec_b + lhs_b + (6 * p + 10) * vec_b)
        alg_bytes = float(per_stage * packed.N.sum())
        achieved = alg_bytes / (r["ms_per_step"] * 1e-3) / 1e9
        roof = {"kernel": "whole cross-stage step (all launches)", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes_per_step": alg_bytes, "step_ms": r["ms_per_step"]}
        dtype = "f64" if head == "fp64" else "f32+f64"
    else:
        elem = 8 if head == "fp64" else 4
        alg_bytes = float(sum(factor_algorithmic_bytes(int(packed.n[b]), int(packed.m[b]), elem, diag=diag)
                              * int(packed.N[b]) for b in range(packed.batch)))
        achieved = alg_bytes / (r["factor_ms"] * 1e-3) / 1e9
        default_uniform = (wk == "batched_uniform" and not diag
                           and (args.nx, args.nu, args.horizon, args.batch) == (12, 4, 128, 4096))
        if wk in ("batched_uniform", "stage_eq"):
            kern = ("k_factor16<%s>" if args.nx + args.nu <= 16 else "k_factor_mw<%s>") % (
                ("double" if head == "fp64" else "float") + (", diagonal Delta" if diag else ""))
        else:
            kern = "rlqr_factor (all tile classes)"
        traffic = (load_counters("k_factor16_float.batched_uniform.counters.txt")
                   if default_uniform and head == "mixed" else None)
        roof = {"kernel": kern, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": alg_bytes, "launch_ms": r["factor_ms"]}
        if wk == "stage_eq":
            # the elimination kernel beside it: per stage Q, M, R, q, r read and
            # written, E (ne x (n + m)), r_e and eta read
            n, m, ne = args.nx, args.nu, args.ne
            red_b = 8 * (2 * (n * n + n * m + m * m + n + m) + ne * (n + m) + 2 * ne)
            roof["reduce_kernel"] = "k_eq_reduce"
            roof["reduce_algorithmic_bytes_per_launch"] = float(red_b * packed.N.sum())
            roof["reduce_gbs"] = red_b * float(packed.N.sum()) / (r["reduce_ms"] * 1e-3) / 1e9
            roof["reduce_ms"] = r["reduce_ms"]
        dtype = "f64" if head == "fp64" else "f32+f64"
    cfg.update({"workload": desc, "rel_tol": rel_tol, "max_refine": max_refine, "path": head})
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "stage-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": cfg,
        "modes": results,
        "roofline": roof,
    }
    if "fp64" in results:
        line[f"{head}_over_fp64"] = results[head]["value"] / results["fp64"]["value"]
    if not args.no_cpu_baseline:
        if wk == "cross_stage":
            line["cpu_baseline"] = cpu_baseline_xs(insts, xs_data)
        elif wk == "stage_eq":
            line["cpu_baseline"] = cpu_baseline_eq(insts, eqs)
        elif wk == "long_horizon":
            line["cpu_baseline"] = cpu_baseline(wl.pack([wl.make_instance(64, 32, 2048, 1e-6, (3, 0, 0))]),
                                                sample="one instance of the long-horizon shape at N=2048")
        elif wk == "single_small":
            line["cpu_baseline"] = cpu_baseline(packed, seconds_target=2.0, threads=1,
                                                sample="the same single instance")
        else:
            line["cpu_baseline"] = cpu_baseline(packed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
