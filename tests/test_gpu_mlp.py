"""GPU kernels of the warm-start network against the CPU oracle (oracle/mlp.py).

GEMM: every transpose combination, ragged sizes, both operand types; the
bfloat16 reference uses the same bf16-rounded operands in float64, so only
the float32 accumulation order separates them. Gradients: the float32
kernels agree with the float64 oracle to 1e-4 (normwise per tensor); the
bfloat16 kernels to 3e-2, the rounding of bf16 activations and weights.
The end-to-end test trains on solutions the interior-point driver produced
and checks that the warm start needs fewer iterations than the cold start.
"""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2509_16370_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_16370_amd import rlqr
    return rlqr


def _bf16_round(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def _to_bf16_bits(a, torch):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return torch.from_numpy(u.view(np.int16)).cuda()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_gemm_matches_reference(rl, dtype, ta, tb):
    import torch
    rng = np.random.default_rng(ta * 2 + tb)
    M, N, K = 70, 45, 33
    A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    bias = rng.standard_normal(N).astype(np.float32)
    dt = rl.RMLP_F32 if dtype == "f32" else rl.RMLP_BF16
    if dtype == "f32":
        Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        Ar, Br = A.astype(np.float64), B.astype(np.float64)
    else:
        Ad, Bd = _to_bf16_bits(A, torch), _to_bf16_bits(B, torch)
        Ar, Br = _bf16_round(A).astype(np.float64), _bf16_round(B).astype(np.float64)
    C = torch.from_numpy(C0.copy()).cuda()
    lda, ldb = A.shape[1], B.shape[1]
    rl.rmlp_gemm(dt, ta, tb, M, N, K, Ad, lda, Bd, ldb, 0.5, 2.0, C, N, torch.from_numpy(bias).cuda(),
                 rl.RMLP_ACT_TANH)
    torch.cuda.synchronize()
    opA = Ar.T if ta else Ar
    opB = Br.T if tb else Br
    ref = np.tanh(0.5 * opA @ opB + 2.0 * C0 + bias)
    assert np.abs(C.cpu().numpy() - ref).max() <= 5e-5


def _net_and_oracle(rl, dtype, sizes, seed=0):
    from paper_2509_16370_amd.warmstart import Net
    net = Net(sizes, dtype=dtype, seed=seed, max_batch=64)
    params = [(W.double().cpu().numpy(), b.double().cpu().numpy()) for W, b in zip(net.W, net.b)]
    return net, params


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("bf16", 3e-2)])
def test_gradients_match_oracle(rl, dtype, tol):
    import torch
    sizes = [24, 64, 64, 64, 100]
    net, params = _net_and_oracle(rl, dtype, sizes)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((48, 24)).astype(np.float32)
    T = rng.standard_normal((48, 100)).astype(np.float32)
    if dtype == "bf16":  # the oracle sees the operands the kernels see
        Xo = _bf16_round(X).astype(np.float64)
        params = [(_bf16_round(W.astype(np.float32)).astype(np.float64), b) for W, b in params]
    else:
        Xo = X.astype(np.float64)
    loss = net.loss_and_grads(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    torch.cuda.synchronize()
    oloss, ograds = omlp.loss_and_grads(params, Xo, T.astype(np.float64))
    assert abs(float(loss) - oloss) <= tol * abs(oloss)
    for l, (gW, gb) in enumerate(ograds):
        dW = net.gW[l].double().cpu().numpy()
        db = net.gb[l].double().cpu().numpy()
        assert np.linalg.norm(dW - gW) <= tol * np.linalg.norm(gW), l
        assert np.linalg.norm(db - gb) <= tol * np.linalg.norm(gb) + 1e-7, l


def test_adam_matches_reference(rl):
    import torch
    rng = np.random.default_rng(4)
    w = rng.standard_normal(1000).astype(np.float32)
    g = rng.standard_normal(1000).astype(np.float32)
    m = np.zeros(1000, np.float32)
    v = np.zeros(1000, np.float32)
    wd, gd, md, vd = (torch.from_numpy(a.copy()).cuda() for a in (w, g, m, v))
    for t in (1, 2, 3):
        rl.rmlp_adam(rl.RMLP_F32, 1000, wd, None, gd, md, vd, 1e-3, 0.9, 0.999, 1e-8, t)
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        w = w - 1e-3 * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-8)
    torch.cuda.synchronize()
    assert np.allclose(wd.cpu().numpy(), w, rtol=1e-5, atol=1e-6)


def test_warm_start_reduces_iterations(rl):
    """Train on converged driver solutions (seed stream 1) and evaluate on
    held-out problems (stream 0): fewer interior-point iterations than the
    cold start, every problem still converging."""
    from paper_2509_16370_amd import warmstart
    print("[gpu] warm start end to end", flush=True)
    F, T = warmstart.make_dataset(1024, N=32, chunk=1024)
    assert F.shape[0] >= 1000
    ws = warmstart.WarmStart(F.shape[1], T.shape[1], hidden=(128, 128, 128), dtype="bf16", batch=128)
    hist = ws.fit(F, T, epochs=40, lr=2e-3)
    assert hist[-1] < hist[0]
    ts = wl.trajectory_problems(128, N=32, stream=0)
    res = warmstart.evaluate(ws, ts)
    print(res, flush=True)
    assert res["warm_converged"] == res["problems"] and res["cold_converged"] == res["problems"]
    assert res["warm_mean_iters"] < res["cold_mean_iters"]
