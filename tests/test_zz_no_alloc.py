"""GPU: rlqr_residual_noalloc (no handle, no device allocation) against
rlqr_residual on a handle of the same shapes.

Both run the same residual kernels, so the residual vectors and the
per-instance relative residuals must agree bit for bit; the relative
residual is also checked against the float64 CPU oracle's. Two calls in a
row go through the shared scratch array, the second with a smaller batch
(fewer instances, shorter horizons, other shapes), so stale metadata of the
first call would show.
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


def _batch(shapes, tag, delta=1e-6, diag=False):
    return [wl.make_instance(n, m, N, delta, (97, tag, i), indefinite=(i % 5 == 3),
                             diag_spread=1.0 if diag else None)
            for i, (n, m, N) in enumerate(shapes)]


def _check_pair(rl, insts):
    import torch
    packed = wl.pack(insts)
    lhs, rhs = rl.to_device(packed)
    s = rl.Solver(packed.N, packed.n, packed.m, mode="fp64")
    s.factor(lhs)
    out, _, _ = s.solve(rhs, rel_tol=1e-8, max_refine=2)
    # perturb z so that the residual is far from zero and every row matters
    gen = torch.Generator(device="cpu").manual_seed(5)
    for k in ("x", "u", "y"):
        out[k] += (1e-3 * torch.randn(out[k].shape, generator=gen, dtype=torch.float64)).to(out[k].device)
    res_h, rel_h = s.residual(rhs, out)
    res_n = torch.full_like(res_h, float("nan"))
    rel_n = torch.full((max(packed.batch, 1),), float("nan"), dtype=torch.float64, device=res_h.device)
    rl.rlqr_residual_noalloc(packed.N, packed.n, packed.m, lhs["Q"], lhs["M"], lhs["R"], lhs["A"], lhs["B"],
                             lhs["delta"], rhs["q"], rhs["r"], rhs["c"], out["x"], out["u"], out["y"],
                             res_n, rel_n, delta_diag=lhs.get("delta_diag"))
    torch.cuda.synchronize()
    B = packed.batch
    L = s.size("res")
    a, b = res_h.cpu().numpy()[:L], res_n.cpu().numpy()[:L]
    assert np.array_equal(a, b), np.nanmax(np.abs(a - b))
    ra, rb = rel_h.cpu().numpy()[:B], rel_n.cpu().numpy()[:B]
    assert np.array_equal(ra, rb)
    sols = wl.unpack_solution(packed, *(out[k].cpu().numpy() for k in ("x", "u", "y")))
    for i, inst in enumerate(insts):
        ref = oracle.rel_residual(inst, *sols[i])
        assert rb[i] == pytest.approx(ref, rel=1e-10), (i, rb[i], ref)
    return B


def test_noalloc_residual_matches_handle_two_calls(rl):
    """First call: one-wavefront and multi-wavefront instances mixed; second
    call: fewer, shorter instances of one fixed shape (the fixed-shape kernel)."""
    print("[gpu] no-alloc residual: two calls, second smaller", flush=True)
    first = _batch([(12, 4, 130), (4, 2, 33), (20, 10, 17), (40, 6, 9), (8, 2, 0), (12, 4, 64)] * 3, 0)
    second = _batch([(12, 4, 7), (12, 4, 1), (12, 4, 20)], 1)
    assert _check_pair(rl, first) == 18
    assert _check_pair(rl, second) == 3


def test_noalloc_residual_per_stage_diagonal(rl):
    print("[gpu] no-alloc residual: per-stage diagonal", flush=True)
    _check_pair(rl, _batch([(12, 4, 40), (6, 3, 11), (24, 20, 5)], 2, diag=True))
    _check_pair(rl, _batch([(4, 1, 3)], 3, diag=True))


def test_noalloc_residual_rejects_oversized_batch(rl):
    """A batch beyond the scratch array returns RLQR_E_INVALID before any GPU work."""
    import torch
    B = 200000
    one = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(rl.RlqrError) as e:
        rl.rlqr_residual_noalloc(np.full(B, 1), np.full(B, 2), np.full(B, 1), *([one] * 12))
    assert e.value.code == rl.RLQR_E_INVALID
