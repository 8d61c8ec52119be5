"""GPU interior-point driver (include/ripm.h) against the CPU IPM oracle.

The driver follows the oracle's iteration rules; its Newton LQR is solved by
the library (refined to 1e-10), so iterates agree with the oracle's to
roundoff and the step decisions match except at razor-edge comparisons:
iteration counts are compared with a slack of two. Converged points are
checked by the oracle's own error measures (gradient of the Lagrangian,
constraint values, slack residual, complementarity) and against the
oracle's converged solutions.
"""
import numpy as np
import pytest

from oracle import ipm as oipm
from paper_2509_16370_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_16370_amd import rlqr
    return rlqr


def _check_kkt(p, x, u, y, z, tol):
    gx, gu = p.grad_L(oipm.State(x, u, y, np.ones_like(z), z * p.mask, 0.0))
    assert max(np.abs(gx).max(), np.abs(gu).max()) <= tol
    assert np.abs(p.c(x, u)).max() <= tol
    g = p.g(x, u)[p.mask > 0]
    zz = z[p.mask > 0]
    assert g.max() <= tol and zz.min() >= 0.0
    assert np.abs(g * zz).max() <= 2 * tol


@pytest.mark.parametrize("lqr", ["fp64", "mixed"])
def test_ipm_matches_oracle_small(rl, lqr):
    print(f"[gpu] ipm small lqr={lqr}", flush=True)
    ts = wl.trajectory_problems(6, N=32, n=6, m=2)
    drv = rl.IPM(ts, lqr=lqr, eta=oipm.ETA, tol=oipm.TOL)
    drv.start()
    iters, conv = drv.solve(max_iter=oipm.MAX_ITER)
    x, u, y, z = (t.cpu().numpy() for t in drv.solution())
    assert conv.all(), conv
    for b in range(ts.batch):
        p = oipm.Problem(ts, b)
        st, it, ok = oipm.solve(p)
        assert ok
        assert abs(int(iters[b]) - it) <= 2, (b, int(iters[b]), it)
        _check_kkt(p, x[b], u[b], y[b], z[b], 1e-6)
        assert np.allclose(x[b], st.x, atol=1e-5) and np.allclose(u[b], st.u, atol=1e-5)


def test_ipm_full_shape_batch(rl):
    """N = 256, n = 12, m = 4: every problem converges; four of them against
    the oracle's solutions."""
    print("[gpu] ipm full shape", flush=True)
    ts = wl.trajectory_problems(64, N=256)
    drv = rl.IPM(ts, lqr="mixed")
    drv.start()
    iters, conv = drv.solve(max_iter=200)
    assert conv.all(), (conv == 0).sum()
    x, u, y, z = (t.cpu().numpy() for t in drv.solution())
    for b in range(ts.batch):
        _check_kkt(oipm.Problem(ts, b), x[b], u[b], y[b], z[b], 1e-6)
    for b in (0, 17, 40, 63):
        st, it, ok = oipm.solve(oipm.Problem(ts, b))
        assert ok
        assert np.allclose(x[b], st.x, atol=1e-5) and np.allclose(u[b], st.u, atol=1e-5)


def test_warm_start_from_solution_converges_at_once(rl):
    import torch
    print("[gpu] ipm warm start", flush=True)
    ts = wl.trajectory_problems(8, N=64)
    drv = rl.IPM(ts, lqr="mixed")
    drv.start()
    it0, conv0 = drv.solve(max_iter=200)
    assert conv0.all()
    x, u, y, z = drv.solution()
    B = ts.batch
    logz = torch.log(torch.clamp(z, min=1e-300))
    warm = torch.cat([x.reshape(B, -1), u.reshape(B, -1), y.reshape(B, -1), logz.reshape(B, -1)], 1).contiguous()
    drv2 = rl.IPM(ts, lqr="mixed")
    drv2.start(warm=warm)
    it1, conv1 = drv2.solve(max_iter=200)
    assert conv1.all()
    assert (it1 <= 8).all() and it1.mean() < it0.mean(), (it1, it0)


# ---- stagewise equality rows E_u u_i = b_i (eliminated into the Newton LQR)

def _eq(ts, ne=1, bval=0.1):
    Eu = np.zeros((ne, ts.m))
    for k in range(ne):
        Eu[k, k], Eu[k, k + 1] = 1.0 / np.sqrt(2), -1.0 / np.sqrt(2)
    return Eu, np.full((ts.N, ne), bval)


def _check_kkt_eq(p, x, u, y, z, ye, tol):
    gx, gu = p.grad_L(oipm.State(x, u, y, np.ones_like(z), z * p.mask, 0.0, ye=ye))
    assert max(np.abs(gx).max(), np.abs(gu).max()) <= tol
    assert np.abs(p.c(x, u)).max() <= tol and np.abs(p.e(u)).max() <= tol
    g = p.g(x, u)[p.mask > 0]
    zz = z[p.mask > 0]
    assert g.max() <= tol and zz.min() >= 0.0
    assert np.abs(g * zz).max() <= 2 * tol


@pytest.mark.parametrize("lqr,ne", [("fp64", 1), ("mixed", 1), ("fp64", 2)])
def test_ipm_stage_equalities_match_oracle(rl, lqr, ne):
    """Equality rows carried through the whole GPU loop: iterations within
    two of the CPU oracle's, the converged x, u and y_e equal the oracle's,
    and the point meets the NLP's first-order conditions."""
    print(f"[gpu] ipm stage equalities lqr={lqr} ne={ne}", flush=True)
    ts = wl.trajectory_problems(6, N=32, n=6, m=3)
    Eu, eb = _eq(ts, ne=ne, bval=0.05)
    drv = rl.IPM(ts, lqr=lqr, eta=oipm.ETA, tol=oipm.TOL, eq=(Eu, eb))
    drv.start()
    iters, conv = drv.solve(max_iter=oipm.MAX_ITER)
    x, u, y, z = (t.cpu().numpy() for t in drv.solution())
    ye = drv.ye.cpu().numpy()
    assert conv.all(), conv
    for b in range(ts.batch):
        p = oipm.Problem(ts, b, eq=(Eu, eb))
        st, it, ok = oipm.solve(p)
        assert ok
        assert abs(int(iters[b]) - it) <= 2, (b, int(iters[b]), it)
        _check_kkt_eq(p, x[b], u[b], y[b], z[b], ye[b], 1e-6)
        assert np.allclose(x[b], st.x, atol=1e-5) and np.allclose(u[b], st.u, atol=1e-5)
        assert np.allclose(ye[b], st.ye, atol=1e-4 * max(1.0, np.abs(st.ye).max()))


def test_ipm_stage_equalities_full_shape(rl):
    """N = 256, n = 12, m = 4 with one equality row per stage: every problem
    converges to a first-order point; two of them against the oracle."""
    print("[gpu] ipm stage equalities full shape", flush=True)
    ts = wl.trajectory_problems(32, N=256)
    Eu, eb = _eq(ts)
    drv = rl.IPM(ts, lqr="fp64", eq=(Eu, eb))
    drv.start()
    iters, conv = drv.solve(max_iter=200)
    assert conv.all(), (conv == 0).sum()
    x, u, y, z = (t.cpu().numpy() for t in drv.solution())
    ye = drv.ye.cpu().numpy()
    for b in range(ts.batch):
        _check_kkt_eq(oipm.Problem(ts, b, eq=(Eu, eb)), x[b], u[b], y[b], z[b], ye[b], 1e-6)
    for b in (0, 21):
        st, it, ok = oipm.solve(oipm.Problem(ts, b, eq=(Eu, eb)))
        assert ok and abs(int(iters[b]) - it) <= 2, (b, int(iters[b]), it)
        assert np.allclose(x[b], st.x, atol=1e-5) and np.allclose(u[b], st.u, atol=1e-5)
