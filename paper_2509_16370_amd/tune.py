"""Autotuner and graph driver for batched, ragged launches.

Instances are grouped into buckets by (n, m); each bucket takes one of the
candidate paths -- float64 sequential, the float32-product sequential
recursion, or the parallel-in-time scan with segment length L -- carried to
the requested relative KKT residual. The choices become per-instance tuning
arrays of ONE handle in RLQR_SCAN_FP32 mode (`inst_fp64` = 1 for the float64
path, `inst_chunk` = 0 for one segment, L for the scan), so the whole ragged
batch is one handle and its factor + solve + refinement is captured into one
HIP graph.

Buckets share launches (one launch per tile class covers every bucket of that
class), so a bucket's best path depends on the others: the tuner starts from
all-float64 and does coordinate descent over the buckets, timing the whole
batch's graph for every candidate of one bucket with the others fixed, and
keeps a change only if it shortens the batch and every instance still
reaches the tolerance (`tune_batch`). `tune` (buckets timed on their own) is
kept as the cheaper first guess.

Host-side orchestration only: every step of the solve runs in the library's
HIP kernels.
"""
from __future__ import annotations

import dataclasses
import json
import time
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import workloads as wl

Bucket = Tuple[int, int]


class Plan(dict):
    """Bucket -> Choice, plus the batch-level schedule: mw_waves, the
    wavefronts per instance of the multi-wavefront kernels for stages with
    16 < n + m <= 48 (0: the library's default of four, or 8)."""

    def __init__(self, *args, mw_waves: int = 0, **kw):
        super().__init__(*args, **kw)
        self.mw_waves = mw_waves


@dataclasses.dataclass
class Choice:
    path: str          # "fp64", "mixed" or "scan"
    L: int = 0         # segment length for "scan"
    ms: float = float("nan")

    def key(self) -> str:
        return f"{self.path}:{self.L}" if self.path == "scan" else self.path


def buckets(packed: wl.Packed) -> Dict[Bucket, np.ndarray]:
    """Instance ids per (n, m), in batch order."""
    out: Dict[Bucket, List[int]] = {}
    for b in range(packed.batch):
        out.setdefault((int(packed.n[b]), int(packed.m[b])), []).append(b)
    return {k: np.asarray(v, dtype=np.int64) for k, v in sorted(out.items())}


def candidates(n: int, m: int, Nmax: int, lengths=(16, 32, 64, 128, 256)) -> List[Choice]:
    cands = [Choice("fp64"), Choice("mixed")]
    cands += [Choice("scan", L) for L in lengths if L < Nmax]
    return cands


def plan_arrays(packed: wl.Packed, plan: Dict[Bucket, Choice]) -> Tuple[np.ndarray, np.ndarray]:
    """Per-instance (inst_chunk, inst_fp64) for one RLQR_SCAN_FP32 handle."""
    chunk = np.zeros(packed.batch, dtype=np.int32)
    fp64 = np.zeros(packed.batch, dtype=np.int32)
    for bk, ids in buckets(packed).items():
        c = plan[bk]
        if c.path == "fp64":
            fp64[ids] = 1
        elif c.path == "scan":
            chunk[ids] = c.L
    return chunk, fp64


def subset(packed: wl.Packed, ids: np.ndarray) -> wl.Packed:
    """The instances `ids` of a packed batch, repacked."""
    ids = np.asarray(ids, dtype=np.int64)
    arrays = {}
    offsets = wl.layout_offsets(packed.N[ids], packed.n[ids], packed.m[ids])
    for k, a in packed.arrays.items():
        off = packed.offsets[k]
        arrays[k] = np.concatenate([a[off[b]:off[b + 1]] for b in ids]) if len(ids) else np.zeros(0)
    return wl.Packed(packed.N[ids].copy(), packed.n[ids].copy(), packed.m[ids].copy(), packed.delta[ids].copy(),
                     arrays, offsets)


def _time_choice(rl, torch, packed, lhs, rhs, c: Choice, rel_tol, max_refine, reps) -> float:
    mode = "scan" if c.path == "scan" else c.path
    s = rl.Solver(packed.N, packed.n, packed.m, mode=mode, scan_chunk=c.L)
    out = {k: s.empty(k) for k in ("x", "u", "y")}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for r in range(reps + 1):
        ev[0].record()
        s.factor(lhs)
        _, status, relres = s.solve(rhs, out=out, rel_tol=rel_tol, max_refine=max_refine)
        ev[1].record()
        torch.cuda.synchronize()
        if r:
            times.append(ev[0].elapsed_time(ev[1]))
    st = status.cpu().numpy()[:packed.batch]
    rr = relres.cpu().numpy()[:packed.batch]
    solved = (st == rl.INST_OK) | (st == rl.INST_NOT_PD)
    if not np.all((rr <= rel_tol) | ~solved) or np.any(st == rl.INST_NOT_CONVERGED):
        return float("inf")
    return float(np.median(times))


def tune(packed: wl.Packed, rel_tol: float = 1e-8, max_refine: int = 3, reps: int = 3,
         lengths=(16, 32, 64, 128, 256), device: str = "cuda:0", log=None) -> Dict[Bucket, Choice]:
    """Time every candidate on each bucket's instances; return the plan."""
    import torch
    from . import rlqr as rl
    plan = Plan()
    for bk, ids in buckets(packed).items():
        sub = subset(packed, ids)
        lhs, rhs = rl.to_device(sub, device)
        best = None
        for c in candidates(bk[0], bk[1], int(sub.N.max()), lengths):
            c.ms = _time_choice(rl, torch, sub, lhs, rhs, c, rel_tol, max_refine, reps)
            if log:
                log(f"[tune] bucket n={bk[0]} m={bk[1]} ({len(ids)} instances): {c.key()} {c.ms:.3f} ms")
            if best is None or c.ms < best.ms:
                best = c
        plan[bk] = best
    return plan


def time_plan(packed, plan, lhs, rhs, rel_tol, max_refine, reps, device="cuda:0") -> float:
    """Median graph-launch time of the whole batch under `plan` (inf if an
    instance misses the tolerance)."""
    import torch
    from . import rlqr as rl
    tb = TunedBatch(packed, plan, lhs, rhs, rel_tol=rel_tol, max_refine=max_refine, device=device)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for r in range(reps + 1):
        ev[0].record(tb.stream)
        tb.solver.replay(stream=tb.stream)
        ev[1].record(tb.stream)
        tb.stream.synchronize()
        if r:
            times.append(ev[0].elapsed_time(ev[1]))
    st = tb.status.cpu().numpy()[:packed.batch]
    rr = tb.relres.cpu().numpy()[:packed.batch]
    solved = (st == rl.INST_OK) | (st == rl.INST_NOT_PD)
    del tb
    if np.any(st == rl.INST_NOT_CONVERGED) or not np.all((rr <= rel_tol) | ~solved):
        return float("inf")
    return float(np.median(times))


def tune_batch(packed: wl.Packed, lhs, rhs, rel_tol: float = 1e-8, max_refine: int = 3, reps: int = 2,
               lengths=(32, 128), rounds: int = 1, device: str = "cuda:0", log=None) -> Dict[Bucket, Choice]:
    """Coordinate descent over the buckets with whole-batch timing (see module doc)."""
    bks = buckets(packed)
    work = {bk: float(sum(int(packed.N[b]) * (bk[0] + bk[1]) ** 3 for b in ids)) for bk, ids in bks.items()}
    plan = Plan({bk: Choice("fp64") for bk in bks})
    best = time_plan(packed, plan, lhs, rhs, rel_tol, max_refine, reps, device)
    if log:
        log(f"[tune] all-fp64: {best:.3f} ms")
    for _ in range(rounds):
        for bk in sorted(bks, key=lambda k: -work[k]):
            Nmax = int(packed.N[bks[bk]].max())
            for c in candidates(bk[0], bk[1], Nmax, lengths):
                if c.key() == plan[bk].key():
                    continue
                trial = Plan(plan, mw_waves=plan.mw_waves)
                trial[bk] = c
                t = time_plan(packed, trial, lhs, rhs, rel_tol, max_refine, reps, device)
                if log:
                    log(f"[tune] bucket {bk} -> {c.key()}: {t:.3f} ms (best {best:.3f})")
                if t < 0.98 * best:
                    best, plan = t, trial
                    plan[bk].ms = t
    # schedule: wavefronts per instance for the stages with 16 < n + m <= 48
    # (one for the 16-wide states, two for the 32-wide ones; or eight)
    if any(16 < n + m <= 48 and n <= 32 for n, m in bks):
        for w in (1, 8):
            trial = Plan(plan, mw_waves=w)
            t = time_plan(packed, trial, lhs, rhs, rel_tol, max_refine, reps, device)
            if log:
                log(f"[tune] {w} wavefront(s) per instance: {t:.3f} ms (best {best:.3f})")
            if t < 0.98 * best:
                best, plan = t, trial
    return plan


def save_plan(plan: Dict[Bucket, Choice], path: str) -> None:
    d = {f"{n},{m}": dataclasses.asdict(c) for (n, m), c in plan.items()}
    d["mw_waves"] = int(getattr(plan, "mw_waves", 0))
    json.dump(d, open(path, "w"), indent=1)


def load_plan(path: str) -> "Plan":
    d = json.load(open(path))
    w = int(d.pop("mw_waves", 0))
    return Plan({tuple(int(v) for v in k.split(",")): Choice(**c) for k, c in d.items()}, mw_waves=w)


class TunedBatch:
    """One handle for a ragged batch under a tuning plan, with its factor +
    solve + refinement captured into one HIP graph."""

    def __init__(self, packed: wl.Packed, plan: Dict[Bucket, Choice], lhs, rhs, rel_tol: float = 1e-8,
                 max_refine: int = 3, device: str = "cuda:0"):
        import torch
        from . import rlqr as rl
        self.torch = torch
        chunk, fp64 = plan_arrays(packed, plan)
        self.solver = rl.Solver(packed.N, packed.n, packed.m, mode="scan", device=device,
                                inst_chunk=chunk, inst_fp64=fp64, mw_waves=getattr(plan, "mw_waves", 0))
        self.lhs, self.rhs = lhs, rhs
        self.out = {k: self.solver.empty(k) for k in ("x", "u", "y")}
        self.stream = torch.cuda.Stream(device=device)
        self.rel_tol, self.max_refine = rel_tol, max_refine
        with torch.cuda.stream(self.stream):
            self.status, self.relres = self.solver.capture(lhs, rhs, self.out, rel_tol, max_refine,
                                                           stream=self.stream)
        self.stream.synchronize()

    def run(self):
        """Replay the graph on the batch's stream (after the current stream's work)."""
        torch = self.torch
        self.stream.wait_stream(torch.cuda.current_stream())
        self.solver.replay(stream=self.stream)
        torch.cuda.current_stream().wait_stream(self.stream)
        return self.out, self.status, self.relres

    def eager(self):
        return self.solver.factor(self.lhs), self.solver.solve(self.rhs, rel_tol=self.rel_tol,
                                                               max_refine=self.max_refine)
