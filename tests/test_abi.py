"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and rejects bad arguments before touching the GPU. No compute calls."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlqr.h")
IPM_HEADER = os.path.join(ROOT, "include", "ripm.h")


def _declared(path=HEADER, prefix="rlqr_"):
    src = open(path).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2509_16370_amd import rlqr
    names = _declared()
    assert set(names) >= {"rlqr_create", "rlqr_factor", "rlqr_solve", "rlqr_pivot_inertia",
                          "rlqr_residual", "rlqr_destroy", "rlqr_layout_offsets"}
    lib = ctypes.CDLL(rlqr.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(rlqr.EXPORTED) == set(names)


def test_library_exports_every_ipm_symbol():
    from paper_2509_16370_amd import rlqr
    names = _declared(IPM_HEADER, "ripm_")
    assert set(names) == set(rlqr.IPM_EXPORTED)
    lib = ctypes.CDLL(rlqr.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_library_exports_every_cross_stage_symbol():
    from paper_2509_16370_amd import rlqr
    names = _declared(os.path.join(ROOT, "include", "rlqr_xs.h"), "rlqr_xs_")
    assert set(names) == set(rlqr.XS_EXPORTED)
    lib = ctypes.CDLL(rlqr.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_cross_stage_rejects_bad_arguments():
    from paper_2509_16370_amd import rlqr
    lib = rlqr._lib
    x = ctypes.c_void_p()
    assert lib.rlqr_xs_create(ctypes.byref(x), None, 2, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_xs_create(None, None, 2, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_xs_factor(None, None, None, 1e-8, 0, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_xs_solve(None, None, None, None, None, 1e-8, 0, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_xs_inertia(None, None, None, None) == rlqr.RLQR_E_INVALID
    lib.rlqr_xs_destroy(None)
    assert lib.rlqr_solve_multi(None, 1, None, None, 1e-8, 0, None, None, None) == rlqr.RLQR_E_INVALID


def test_library_exports_every_stage_equality_symbol():
    from paper_2509_16370_amd import rlqr
    names = _declared(os.path.join(ROOT, "include", "rlqr_eq.h"), "rlqr_eq_")
    assert set(names) == set(rlqr.EQ_EXPORTED)
    lib = ctypes.CDLL(rlqr.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_stage_equality_rejects_bad_arguments():
    from paper_2509_16370_amd import rlqr
    lib = rlqr._lib
    x = ctypes.c_void_p()
    assert lib.rlqr_eq_create(ctypes.byref(x), None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_eq_create(None, None, None, None) == rlqr.RLQR_E_INVALID
    off = (ctypes.c_int64 * 2)()
    assert lib.rlqr_eq_offsets(None, 0, off) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_eq_reduce(None, None, None, None, None, None, None, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_eq_recover(None, None, None, None, None) == rlqr.RLQR_E_INVALID
    lib.rlqr_eq_destroy(None)


def test_library_exports_every_network_kernel_symbol():
    from paper_2509_16370_amd import rlqr
    names = _declared(os.path.join(ROOT, "include", "rmlp.h"), "rmlp_")
    assert set(names) == set(rlqr.MLP_EXPORTED)
    lib = ctypes.CDLL(rlqr.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_network_kernels_reject_bad_arguments():
    from paper_2509_16370_amd import rlqr
    lib = rlqr._lib
    assert lib.rmlp_gemm(5, 0, 0, 4, 4, 4, None, 4, None, 4, 1.0, 0.0, None, 4, None, 0, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rmlp_gemm(0, 0, 0, -1, 4, 4, None, 4, None, 4, 1.0, 0.0, None, 4, None, 0, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rmlp_gemm(0, 0, 0, 4, 4, 4, None, 4, None, 4, 1.0, 0.0, None, 4, None, 0, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rmlp_gemm(0, 0, 0, 4, 4, 4, None, 4, None, 4, 1.0, 0.0, None, 4, None, 3, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rmlp_mse(0, 0, 4, None, None, None, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rmlp_adam(0, 10, None, None, None, None, None, 1e-3, 0.9, 0.999, 1e-8, 0, None) == rlqr.RLQR_E_INVALID
    assert lib.rmlp_cast(2, 10, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rmlp_gemm(0, 0, 0, 0, 4, 4, None, 4, None, 4, 1.0, 0.0, None, 4, None, 0, None, None) == rlqr.RLQR_OK


def test_ipm_create_rejects_bad_problems():
    from paper_2509_16370_amd import rlqr
    lib = rlqr._lib
    assert lib.ripm_create(None, None, None) == rlqr.RLQR_E_INVALID
    A = np.eye(3); B = np.ones((3, 1)); a = np.ones((2, 3))
    dp = rlqr._dp
    good = dict(batch=2, N=4, n=3, m=1, dt=0.05, wx=1.0, wu=0.1, wN=10.0, xmax=0.5, umax=1.0, eta=1e3, tol=1e-6,
                lqr_mode=1)
    for bad in (dict(batch=0), dict(N=0), dict(n=30, m=3), dict(eta=0.0), dict(lqr_mode=2), dict(umax=-1.0)):
        kw = dict(good, **bad)
        p = rlqr._IpmProblem(kw["batch"], kw["N"], kw["n"], kw["m"], kw["dt"], kw["wx"], kw["wu"], kw["wN"],
                             kw["xmax"], kw["umax"], A.ctypes.data_as(dp), B.ctypes.data_as(dp), a.ctypes.data_as(dp),
                             kw["eta"], kw["tol"], kw["lqr_mode"])
        h = rlqr._vp()
        assert lib.ripm_create(ctypes.byref(h), ctypes.byref(p), None) == rlqr.RLQR_E_INVALID, bad
    # stagewise equality rows: more rows than controls, or no E_u
    kw = good
    Eu = np.ones((2, 1))
    for ne, E in ((2, Eu), (1, None), (9, Eu), (-1, Eu)):
        p = rlqr._IpmProblem(kw["batch"], kw["N"], kw["n"], kw["m"], kw["dt"], kw["wx"], kw["wu"], kw["wN"],
                             kw["xmax"], kw["umax"], A.ctypes.data_as(dp), B.ctypes.data_as(dp), a.ctypes.data_as(dp),
                             kw["eta"], kw["tol"], kw["lqr_mode"], ne, None if E is None else E.ctypes.data_as(dp))
        h = rlqr._vp()
        assert lib.ripm_create(ctypes.byref(h), ctypes.byref(p), None) == rlqr.RLQR_E_INVALID, ne
    lib.ripm_destroy(None)


def test_tuned_create_rejects_negative_segment_lengths():
    from paper_2509_16370_amd import rlqr
    with pytest.raises(rlqr.RlqrError) as e:
        rlqr.rlqr_create_tuned([8], [3], [2], rlqr.RLQR_SCAN_FP32, scan_chunk=-1)
    assert e.value.code == rlqr.RLQR_E_INVALID
    with pytest.raises(rlqr.RlqrError) as e:
        rlqr.rlqr_create_tuned([8, 9], [3, 3], [2, 2], rlqr.RLQR_SCAN_FP32, inst_chunk=[4, -2])
    assert e.value.code == rlqr.RLQR_E_INVALID


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
    ([4], [3], [2], 4),      # unknown mode
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
    assert lib.rlqr_factor_rhs(None, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_solve(None, None, None, 1e-8, 0, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_pivot_inertia(None, None, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_residual(None, None, None, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_graph_capture(None, None, None, None, 1e-8, 0, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_graph_launch(None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_get_tuning(None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_precision_path(None, None, None) == rlqr.RLQR_E_INVALID
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


def test_package_binds_to_a_single_hip_runtime():
    """Importing the binding before torch must leave exactly one HIP runtime
    mapped in the process once torch is loaded too."""
    import subprocess
    import sys
    code = ("import paper_2509_16370_amd.rlqr\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_residual_noalloc_rejects_bad_arguments_before_gpu_work():
    """NULL arguments, shapes out of range and a batch beyond the scratch
    array are rejected on the host (no pointer is dereferenced)."""
    from paper_2509_16370_amd import rlqr
    lib = rlqr._lib
    lhs = rlqr._Lhs(*(8 for _ in range(7)))
    rhs = rlqr._Rhs(8, 8, 8)
    sol = rlqr._Sol(8, 8, 8)
    assert lib.rlqr_residual_noalloc(None, None, None, None, None, None, None) == rlqr.RLQR_E_INVALID
    for N, nx, nu in [(-1, 2, 1), (3, 0, 1), (3, 65, 1), (3, 60, 40)]:
        shape, _keep = rlqr._shape([N], [nx], [nu])
        assert lib.rlqr_residual_noalloc(ctypes.byref(shape), ctypes.byref(lhs), ctypes.byref(rhs),
                                         ctypes.byref(sol), None, None, None) == rlqr.RLQR_E_INVALID
    B = 200000  # 200000 instances need > 32 MB of metadata alone
    shape, _keep = rlqr._shape(np.full(B, 1), np.full(B, 2), np.full(B, 1))
    assert lib.rlqr_residual_noalloc(ctypes.byref(shape), ctypes.byref(lhs), ctypes.byref(rhs),
                                     ctypes.byref(sol), None, None, None) == rlqr.RLQR_E_INVALID
    bad_lhs = rlqr._Lhs(8, 8, 8, 8, 8, None, None)  # neither delta nor delta_diag
    shape, _keep = rlqr._shape([3], [2], [1])
    assert lib.rlqr_residual_noalloc(ctypes.byref(shape), ctypes.byref(bad_lhs), ctypes.byref(rhs),
                                     ctypes.byref(sol), None, None, None) == rlqr.RLQR_E_INVALID


def test_library_exports_every_spd_symbol():
    from paper_2509_16370_amd import rlqr
    names = _declared(os.path.join(ROOT, "include", "rlqr_spd.h"), "rlqr_spd_")
    assert set(names) == set(rlqr.SPD_EXPORTED)
    lib = ctypes.CDLL(rlqr.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_spd_rejects_bad_arguments():
    from paper_2509_16370_amd import rlqr
    lib = rlqr._lib
    x = ctypes.c_void_p()
    assert lib.rlqr_spd_create(ctypes.byref(x), None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_spd_create(None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_spd_factor(None, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_spd_solve(None, None, None, 1e-8, 0, None, None, None) == rlqr.RLQR_E_INVALID
    assert lib.rlqr_spd_residual(None, None, None, None, None, None) == rlqr.RLQR_E_INVALID
    lib.rlqr_spd_destroy(None)
