#!/usr/bin/env python
"""Benchmark: dual-regularized LQR stage-solves per second at 1e-8 relative KKT
residual, mixed precision vs plain float64, on one MI355X.

Workload: a uniform batch of 4096 independent instances, n=12, m=4, N=128
(quadrotor-sized), delta=1e-8, generated with the seeded recipe of
paper_2509_16370_amd.workloads; inputs are resident in HBM before timing.
One step = rlqr_factor + rlqr_solve (backward/forward passes, float64
residual and iterative refinement until every instance reaches
||K z + b||_inf <= 1e-8 ||b||_inf). A stage-solve is one stage of one
instance carried through that step; instances that miss the tolerance are
not counted.

Prints ONE JSON line. `value` is the mixed path; the plain float64 path, the
roofline of the dominant kernel (the factorization) and the CPU oracle
baseline are reported beside it.
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
HBM_PEAK_GBS = 8000.0
REL_TOL = 1e-8


def factor_algorithmic_bytes(n, m, elem_bytes):
    """Per stage: read Q, M, R, A, B (float64) and write the minimal
    factorization a solve needs -- K (m x n), the symmetric P and S_hat^{-1}
    (n(n+1)/2 each) and the symmetric G^{-1} (m(m+1)/2) -- in the working precision."""
    lhs = 8 * (n * n + n * m + m * m + n * n + n * m)
    handoff = elem_bytes * (m * n + n * (n + 1) + m * (m + 1) // 2)
    return lhs + handoff


def run_mode(torch, rl, packed, lhs, rhs, mode, steps, warmup, max_refine):
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode)
    out = {k: s.empty(k) for k in ("x", "u", "y")}
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        s.factor(lhs)
        if ev:
            ev[1].record(stream)
        res = s.solve(rhs, out=out, rel_tol=REL_TOL, max_refine=max_refine)
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
    status = status.cpu().numpy()[:packed.batch]
    relres = relres.cpu().numpy()[:packed.batch]
    ok = (relres <= REL_TOL) & ((status == rl.INST_OK) | (status == rl.INST_NOT_PD))
    stages = int(packed.N[ok].sum())
    ms_per_step = 1e3 * wall / steps
    import numpy as np
    return dict(
        value=stages / (ms_per_step * 1e-3),
        ms_per_step=ms_per_step,
        factor_ms=float(np.median(factor_ms)),
        solve_ms=float(np.median(solve_ms)),
        instances_ok=int(ok.sum()),
        max_relres=float(relres.max()),
        median_relres=float(np.median(relres)),
        status_counts={int(k): int(v) for k, v in zip(*np.unique(status, return_counts=True))},
        workspace_bytes=s.workspace_bytes,
    )


def cpu_baseline(packed, seconds_target=10.0):
    """The FP64 oracle, as it stands, over the same batch on the host cores."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
    times = []
    used = 1
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        x, u, y, st, used = oracle.seq_batch(packed, nthreads=threads)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > seconds_target or len(times) >= 5:
            break
    t = float(np.median(times))
    stages = int(packed.N.sum())
    return dict(value=stages / t, unit="stage-solves/s", cores=int(used), kind="oracle",
                sample=f"full batch ({packed.batch} instances, {stages} stages), median of {len(times)} runs "
                       f"of the sequential FP64 oracle, instances spread over {used} threads",
                seconds=t)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--delta", type=float, default=1e-8)
    ap.add_argument("--max-refine", type=int, default=3)
    ap.add_argument("--modes", default="fp64,mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the batch is "
              "independent instances and would shard by instance across GPUs, which this "
              "build does not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2509_16370_amd import workloads as wl
    from paper_2509_16370_amd import rlqr as rl

    n, m, N = 12, 4, 128
    t0 = time.perf_counter()
    packed = wl.pack_parallel(wl.uniform_specs(batch=args.batch, n=n, m=m, N=N, delta=args.delta),
                              workers=args.workers)
    print(f"[bench] generated {args.batch} instances in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
          flush=True)
    lhs, rhs = rl.to_device(packed, "cuda:0")
    torch.cuda.synchronize()

    modes = [md for md in args.modes.split(",") if md]
    results = {}
    for mode in modes:
        results[mode] = run_mode(torch, rl, packed, lhs, rhs, mode, args.steps, args.warmup, args.max_refine)
        print(f"[bench] {mode}: {json.dumps(results[mode])}", file=sys.stderr, flush=True)

    head = "mixed" if "mixed" in results else modes[0]
    r = results[head]
    units = args.batch * N
    elem = 4 if head == "mixed" else 8
    alg_bytes = factor_algorithmic_bytes(n, m, elem) * units
    achieved = alg_bytes / (r["factor_ms"] * 1e-3) / 1e9
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
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"batched uniform dual-regularized LQR: {args.batch} instances, n={n}, m={m}, "
                        f"N={N}, delta={args.delta:g}, refined to {REL_TOL:g} relative KKT residual",
            "batch": args.batch, "nx": n, "nu": m, "N": N, "delta": args.delta,
            "rel_tol": REL_TOL, "max_refine": args.max_refine, "path": head,
        },
        "modes": results,
        "roofline": {
            "kernel": "k_factor16<float>" if head == "mixed" else "k_factor16<double>",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_stage": factor_algorithmic_bytes(n, m, elem),
            "launch_ms": r["factor_ms"],
        },
    }
    if "fp64" in results and "mixed" in results:
        line["mixed_over_fp64"] = results["mixed"]["value"] / results["fp64"]["value"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(packed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
