"""Learned warm start for the interior-point driver.

A multilayer perceptron maps a problem's (x0, goal) to the initial primal and
dual trajectory of the interior-point driver (x, u, y and log z, in the warm
layout of ripm_start). It is trained on converged solutions that the driver
itself produces, with the hand-written kernels of include/rmlp.h for the
forward pass, the backward pass and Adam; targets are standardized per
output. A cold start remains the fallback (warm=None), and the plain cold-start
run is the reference the warm start is judged against.

Host-side orchestration only: every layer, gradient and update runs in the
library's kernels; torch provides device memory and the stream.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional

import numpy as np

from . import rlqr as rl
from . import workloads as wl

HIDDEN = (256, 256, 256)


def layout_size(ts) -> int:
    N, n, m = ts.N, ts.n, ts.m
    return (N + 1) * n * 2 + N * m + (N + 1) * (2 + 2 * m)


class Net:
    """Dense tanh network with float32 master weights, operand copies in
    `dtype` ("bf16" or "f32") and Adam moments, all on the device."""

    def __init__(self, sizes, dtype: str = "bf16", seed: int = 0, max_batch: int = 256, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.sizes = list(sizes)
        self.dt = rl.RMLP_BF16 if dtype == "bf16" else rl.RMLP_F32
        self.qdtype = torch.int16 if dtype == "bf16" else torch.float32
        self.max_batch = max_batch
        rng = np.random.default_rng(seed)
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.W, self.b, self.Wq, self.mW, self.vW, self.mb, self.vb, self.gW, self.gb = ([] for _ in range(9))
        for a, c in zip(self.sizes[:-1], self.sizes[1:]):
            lim = np.sqrt(6.0 / (a + c))
            W = torch.from_numpy(rng.uniform(-lim, lim, (a, c)).astype(np.float32)).to(self.dev)
            self.W.append(W)
            self.b.append(torch.zeros(c, **f32))
            self.Wq.append(self._q(W))
            for lst, shape in ((self.mW, (a, c)), (self.vW, (a, c)), (self.gW, (a, c))):
                lst.append(torch.zeros(shape, **f32))
            for lst in (self.mb, self.vb, self.gb):
                lst.append(torch.zeros(c, **f32))
        self.t = 0
        self._alloc(max_batch)

    def _q(self, x):
        """Operand copy of a float32 tensor in the network dtype."""
        if self.dt == rl.RMLP_F32:
            return x
        q = self.torch.empty(x.shape, dtype=self.qdtype, device=self.dev)
        rl.rmlp_cast(self.dt, x.numel(), x, q)
        return q

    def _alloc(self, M):
        torch = self.torch
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.H = [torch.empty(M, s, **f32) for s in self.sizes]
        self.Hq = [h if self.dt == rl.RMLP_F32 else torch.empty(h.shape, dtype=self.qdtype, device=self.dev)
                   for h in self.H]
        self.dZ = [torch.empty(M, s, **f32) for s in self.sizes[1:]]
        self.dZq = [d if self.dt == rl.RMLP_F32 else torch.empty(d.shape, dtype=self.qdtype, device=self.dev)
                    for d in self.dZ]
        self.dH = [torch.empty(M, s, **f32) for s in self.sizes[1:-1]]
        self.loss = torch.zeros(M + 1, dtype=torch.float64, device=self.dev)

    def forward(self, X):
        """X: float32 [M, in] on the device (M <= max_batch). Returns the output view."""
        M = X.shape[0]
        L = len(self.W)
        self.H[0][:M].copy_(X)
        if self.dt != rl.RMLP_F32:
            rl.rmlp_cast(self.dt, M * self.sizes[0], self.H[0], self.Hq[0])
        for l in range(L):
            a, c = self.sizes[l], self.sizes[l + 1]
            act = rl.RMLP_ACT_TANH if l < L - 1 else rl.RMLP_ACT_NONE
            rl.rmlp_gemm(self.dt, 0, 0, M, c, a, self.Hq[l], a, self.Wq[l], c, 1.0, 0.0, self.H[l + 1], c,
                         self.b[l], act, None if self.dt == rl.RMLP_F32 else self.Hq[l + 1])
        return self.H[L][:M]

    def backward(self, M):
        """Gradients of the loss whose output gradient is in dZ[-1] / dZq[-1]."""
        L = len(self.W)
        for l in range(L - 1, -1, -1):
            a, c = self.sizes[l], self.sizes[l + 1]
            # dW = H_l^T dZ_l, db = column sums of dZ_l
            rl.rmlp_gemm(self.dt, 1, 0, a, c, M, self.Hq[l], a, self.dZq[l], c, 1.0, 0.0, self.gW[l], c)
            rl.rmlp_colsum(M, c, self.dZ[l], c, self.gb[l])
            if l > 0:
                # dH_l = dZ_l W_l^T, dZ_{l-1} = dH_l (1 - H_l^2)
                rl.rmlp_gemm(self.dt, 0, 1, M, a, c, self.dZq[l], c, self.Wq[l], c, 1.0, 0.0, self.dH[l - 1], a)
                rl.rmlp_tanh_backward(self.dt, M * a, self.dH[l - 1], self.H[l], self.dZ[l - 1],
                                      None if self.dt == rl.RMLP_F32 else self.dZq[l - 1])

    def loss_and_grads(self, X, T):
        M = X.shape[0]
        pred = self.forward(X)
        rl.rmlp_mse(self.dt, M, self.sizes[-1], pred, T, self.dZ[-1],
                    None if self.dt == rl.RMLP_F32 else self.dZq[-1], self.loss)
        self.backward(M)
        return self.loss[0]

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        for l in range(len(self.W)):
            rl.rmlp_adam(self.dt, self.W[l].numel(), self.W[l], None if self.dt == rl.RMLP_F32 else self.Wq[l],
                         self.gW[l], self.mW[l], self.vW[l], lr, beta1, beta2, eps, self.t)
            rl.rmlp_adam(rl.RMLP_F32, self.b[l].numel(), self.b[l], None, self.gb[l], self.mb[l], self.vb[l], lr,
                         beta1, beta2, eps, self.t)


# ---------------------------------------------------------------- data from the method itself

def features(ts):
    return np.concatenate([ts.x0, ts.goal], axis=1).astype(np.float32)


def solve_batch(ts, lqr="fp64", max_iter=200, warm=None):
    """Run the GPU interior-point driver; returns (iters, converged, x, u, y, z, seconds)."""
    import torch
    drv = rl.IPM(ts, lqr=lqr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    drv.start(warm=warm)
    iters, conv = drv.solve(max_iter=max_iter)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    x, u, y, z = drv.solution()
    return iters, conv, x, u, y, z, secs


def targets_from_solution(x, u, y, z, zmin=1e-12):
    """Warm layout rows (x, u, y, log z) as a float32 device tensor [B, size]."""
    import torch
    B = x.shape[0]
    logz = torch.log(torch.clamp(z, min=zmin))
    return torch.cat([x.reshape(B, -1), u.reshape(B, -1), y.reshape(B, -1), logz.reshape(B, -1)], 1).float()


def make_dataset(count, N=256, n=12, m=4, stream=1, chunk=2048, log=None):
    """Converged interior-point solutions of `count` training problems (seed
    stream disjoint from the evaluation pairs). Returns (features, targets)
    of the converged problems as device tensors."""
    import torch
    feats, tgts = [], []
    for start in range(0, count, chunk):
        ts = wl.trajectory_problems(min(chunk, count - start), N=N, n=n, m=m, stream=stream, first=start)
        iters, conv, x, u, y, z, secs = solve_batch(ts)
        ok = torch.from_numpy(conv.astype(bool)).to(x.device)
        feats.append(torch.from_numpy(features(ts)).to(x.device)[ok])
        tgts.append(targets_from_solution(x, u, y, z)[ok])
        if log:
            log(f"[data] problems {start}..{start + ts.batch}: {int(conv.sum())} converged, "
                f"mean iterations {iters.mean():.2f}, {secs:.2f} s")
    return torch.cat(feats), torch.cat(tgts)


class WarmStart:
    """Standardization + network + training loop + prediction in the warm layout."""

    def __init__(self, in_size, out_size, hidden=HIDDEN, dtype="bf16", seed=0, batch=256, device="cuda:0"):
        import torch
        self.torch = torch
        self.net = Net([in_size, *hidden, out_size], dtype=dtype, seed=seed, max_batch=batch, device=device)
        self.batch = batch
        self.mean = self.std = None

    def fit(self, F, T, epochs=20, lr=1e-3, lr_min=1e-5, seed=0, log=None):
        """Adam on minibatches of the standardized targets; the step size
        follows a cosine from lr down to lr_min over the epochs."""
        torch = self.torch
        # per-output standardization constants of the training targets
        Tn = T.cpu().numpy().astype(np.float64)
        mean = Tn.mean(0)
        std = np.maximum(Tn.std(0), 1e-6)
        self.mean = torch.from_numpy(mean.astype(np.float32)).to(T.device)
        self.std = torch.from_numpy(std.astype(np.float32)).to(T.device)
        inv = torch.from_numpy((1.0 / std).astype(np.float32)).to(T.device)
        shift = torch.from_numpy((-mean / std).astype(np.float32)).to(T.device)
        Ts = torch.empty_like(T)
        rl.rmlp_affine_cols(T.shape[0], T.shape[1], T, inv, shift, Ts)
        rng = np.random.default_rng(seed)
        Mtot = F.shape[0]
        history = []
        for ep in range(epochs):
            lr_ep = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * ep / max(epochs, 1)))
            perm = torch.from_numpy(rng.permutation(Mtot)).to(F.device)
            tot, cnt = 0.0, 0
            for s in range(0, Mtot - self.batch + 1, self.batch):
                idx = perm[s:s + self.batch]
                loss = self.net.loss_and_grads(F[idx].contiguous(), Ts[idx].contiguous())
                self.net.adam(lr=lr_ep)
                tot += float(loss) if (s // self.batch) % 50 == 0 else 0.0
                cnt += 1 if (s // self.batch) % 50 == 0 else 0
            history.append(tot / max(cnt, 1))
            if log:
                log(f"[train] epoch {ep}: lr {lr_ep:.2e}, sampled loss {history[-1]:.4e}")
        return history

    def predict(self, F):
        """Warm layout rows (float64) for features F [B, in] (float32 device tensor)."""
        torch = self.torch
        out = []
        for s in range(0, F.shape[0], self.batch):
            Fi = F[s:s + self.batch].contiguous()
            P = self.net.forward(Fi)
            Y = torch.empty_like(P)
            rl.rmlp_affine_cols(P.shape[0], P.shape[1], P, self.std, self.mean, Y)
            out.append(Y.double())
        return torch.cat(out).contiguous()


def evaluate(ws: WarmStart, ts, log=None):
    """Cold vs warm starts of the driver on the problems of ts."""
    import torch
    ic, cc, _, _, _, _, tc = solve_batch(ts)
    F = torch.from_numpy(features(ts)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    warm = ws.predict(F)
    torch.cuda.synchronize()
    tpred = time.perf_counter() - t0
    iw, cw, _, _, _, _, tw = solve_batch(ts, warm=warm)
    both = (cc > 0) & (cw > 0)
    res = dict(problems=int(ts.batch), cold_converged=int(cc.sum()), warm_converged=int(cw.sum()),
               cold_mean_iters=float(ic[both].mean()), warm_mean_iters=float(iw[both].mean()),
               cold_seconds=tc, warm_seconds=tw + tpred, predict_seconds=tpred)
    if log:
        log(f"[eval] {res}")
    return res


def main(argv=None):
    """Train on method-generated solutions and compare warm vs cold starts.
    python -m paper_2509_16370_amd.warmstart [--train 50000] [--eval 2048] [--epochs 20]"""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=50000)
    ap.add_argument("--eval", type=int, default=2048)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--dtype", default="bf16")
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    t0 = time.perf_counter()
    F, T = make_dataset(args.train, N=args.N, log=log)
    log(f"[data] {F.shape[0]} training pairs in {time.perf_counter() - t0:.1f} s")
    ws = WarmStart(F.shape[1], T.shape[1], dtype=args.dtype)
    t0 = time.perf_counter()
    hist = ws.fit(F, T, epochs=args.epochs, log=log)
    log(f"[train] {time.perf_counter() - t0:.1f} s")
    ts = wl.trajectory_problems(args.eval, N=args.N, stream=0)
    res = evaluate(ws, ts, log=log)
    res.update(train_pairs=int(F.shape[0]), epochs=args.epochs, final_loss=hist[-1], dtype=args.dtype)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
