"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and rejects bad arguments before touching the GPU. No compute calls."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlqr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rlqr_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2509_16370_amd import rlqr
    names = _declared()
    assert set(names) >= {"rlqr_create", "rlqr_factor", "rlqr_solve", "rlqr_pivot_inertia",
                          "rlqr_residual", "rlqr_destroy", "rlqr_layout_offsets"}
    lib = ctypes.CDLL(rlqr.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(rlqr.EXPORTED) == set(names)


def test_status_strings():
    from paper_2509_16370_amd import rlqr
    for code in (0, -1, -2, -3, -4, -5):
        assert rlqr._lib.rlqr_status_string(code)


@pytest.mark.parametrize("N,nx,nu,mode", [
    ([4], [65], [5], 0),     # n > 64
    ([4], [60], [40], 0),    # n + m > 96
    ([4], [0], [2], 0),      # n < 1
    ([4], [3], [0], 0),      # m < 1
    ([-1], [3], [2], 0),     # N < 0
    ([4], [3], [2], 7),      # unknown mode
])
def test_create_rejects_bad_shapes(N, nx, nu, mode):
    from paper_2509_16370_amd import rlqr
    with pytest.raises(rlqr.RlqrError) as e:
        rlqr.rlqr_create(N, nx, nu, mode)
    assert e.value.code == rlqr.RLQR_E_INVALID


def test_null_arguments_rejected():
    from paper_2509_16370_amd import rlqr
    lib = rlqr._lib
    assert lib.rlqr_create(None, None, 0, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_factor(None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_solve(None, None, None, 1e-8, 0, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_pivot_inertia(None, None, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_residual(None, None, None, None, None, None) == rlqr.RLQR_E_INVALID
    lib.rlqr_destroy(None)


def test_layout_offsets_formula_matches_workloads():
    """The packing rule the generators use is the one the header states."""
    from paper_2509_16370_amd import workloads as wl
    N, n, m = [3, 0, 5], [2, 4, 1], [1, 3, 2]
    off = wl.layout_offsets(N, n, m)
    for b in range(3):
        c = wl.counts(N[b], n[b], m[b])
        for k, v in c.items():
            assert off[k][b + 1] - off[k][b] == v
