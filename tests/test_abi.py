"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/axipcg.h, and rejects invalid arguments before touching
the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "axipcg.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(axipcg_[A-Za-z_0-9]+)\s*\(", hdr)))


@pytest.fixture(scope="module")
def ax():
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


def test_header_declares_the_boundary():
    names = _declared()
    for expected in ("axipcg_op_create", "axipcg_precond_apply", "axipcg_pcg_solve", "axipcg_apply_A",
                     "axipcg_laguerre_rhs", "axipcg_laguerre_coeffs", "axipcg_residual_norm"):
        assert expected in names


def test_every_declared_symbol_is_exported(ax):
    h = ctypes.CDLL(ax.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(h, n)]
    assert not missing, missing
    # and the binding covers them with the same names
    assert set(_declared()) <= set(ax.SIGNATURES)


def test_binding_never_imports_the_oracle():
    import paper_1002_3094_amd.axipcg as b
    src = open(b.__file__).read()
    assert "oracle" not in src.replace("no CPU fallback", "")


def test_product_and_oracle_share_no_code():
    """No product source imports or includes the oracle, and the oracle
    neither imports the package nor includes the library's headers; the
    seeded input generators (synth) are the only code both sides use."""
    import glob
    import re
    pkg = os.path.join(ROOT, "paper_1002_3094_amd")
    product = glob.glob(os.path.join(pkg, "*.py")) + glob.glob(os.path.join(pkg, "csrc", "*")) + \
        glob.glob(os.path.join(ROOT, "include", "*.h"))
    py_import = re.compile(r"^\s*(import|from)\s+(\S+)", re.M)
    c_include = re.compile(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', re.M)
    for path in product:
        if path.endswith((".so", ".o")) or os.path.isdir(path):
            continue
        src = open(path, errors="replace").read()
        assert not any(m.group(2).split(".")[0] == "oracle" for m in py_import.finditer(src)), path
        assert not any("oracle" in m.group(1) for m in c_include.finditer(src)), path
    for path in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if not path.endswith((".py", ".c", ".h")):
            continue
        src = open(path).read()
        assert not any(m.group(2).split(".")[0] == "paper_1002_3094_amd" for m in py_import.finditer(src)), path
        for m in c_include.finditer(src):
            assert "axipcg" not in m.group(1) and "csrc" not in m.group(1), path


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library every entry point raises: there is no CPU
    fallback to land on."""
    import paper_1002_3094_amd.axipcg as b
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "LIB_PATH", os.path.join(ROOT, "_no_such_dir", "libaxipcg.so"))
    with pytest.raises(ImportError):
        b.lib()
    with pytest.raises(ImportError):
        b.strerror(0)
    with pytest.raises(ImportError):
        b.laguerre_coeffs(4, 10.0, np.ones(5), 1.0)


def test_strerror(ax):
    assert ax.strerror(ax.EINVAL) == "invalid argument"
    assert ax.strerror(ax.ENOTCONV) == "not converged within maxit"
    assert ax.strerror(12345) == "unknown status"


@pytest.mark.parametrize("case", ["nz_not_pow2", "nz_too_large", "kappa_nonpositive", "q_negative", "nan", "nr_small",
                                  "bc"])
def test_op_create_validates_before_device_work(ax, case):
    nr, nz, bc = 8, 8, 0
    kappa = np.ones((nr, nz))
    q = np.zeros((nr, nz))
    if case == "nz_not_pow2":
        nz = 12
        kappa = np.ones((nr, nz))
        q = np.zeros((nr, nz))
    elif case == "nz_too_large":
        nz = 8192
        kappa = np.ones((nr, nz))
        q = np.zeros((nr, nz))
    elif case == "kappa_nonpositive":
        kappa[3, 3] = 0.0
    elif case == "q_negative":
        q[1, 2] = -1e-3
    elif case == "nan":
        kappa[0, 0] = np.nan
    elif case == "nr_small":
        nr = 1
        kappa = np.ones((nr, nz))
        q = np.zeros((nr, nz))
    elif case == "bc":
        bc = 7
    out = ctypes.c_void_p()
    lib = ax.lib()
    code = lib.axipcg_op_create(nr, nz, 1.0, 1.0, bc, kappa.ctypes.data_as(ax._dp), q.ctypes.data_as(ax._dp),
                                -1.0, -1.0, None, ctypes.byref(out))
    assert code == ax.EINVAL
    assert out.value is None
    assert ax.last_error() != ""


def test_null_handles_rejected(ax):
    lib = ax.lib()
    assert lib.axipcg_apply_A(None, None, None, None) == ax.EINVAL
    assert lib.axipcg_pcg_solve(None, None, None, 1e-10, 10, 1, 0, None, None) == ax.EINVAL
    assert lib.axipcg_precond_apply(None, None, None, 1, None) == ax.EINVAL
    lib.axipcg_op_destroy(None)  # NULL-safe
    assert lib.axipcg_op_bounds_lanczos(None, None, 10, 1, None, None, None, None) == ax.EINVAL
    # batched solves: NULL arrays, a NULL member, bad counts, flags and bounds
    n1 = (ax._vp * 1)(None)
    assert lib.axipcg_batch_solve(1, None, None, None, 1e-10, 10, 1, 0, None, None) == ax.EINVAL
    assert lib.axipcg_batch_solve(1, n1, n1, n1, 1e-10, 10, 1, 0, None, None) == ax.EINVAL
    assert lib.axipcg_batch_solve(0, n1, n1, n1, 1e-10, 10, 1, 0, None, None) == ax.EINVAL
    assert lib.axipcg_batch_solve(1, n1, n1, n1, 1e-10, 10, 1, 8, None, None) == ax.EINVAL
    assert lib.axipcg_batch_cheb_solve(1, None, None, None, None, None, 1e-10, 10, 1, 0, None, None) == ax.EINVAL
    assert lib.axipcg_batch_cheb_solve(1, n1, n1, n1, None, None, 1e-10, 10, 1, 0, None, None) == ax.EINVAL
    assert lib.axipcg_batch_cheb_solve(1, n1, n1, n1, None, None, 1e-10, 10, 1, 2, None, None) == ax.EINVAL
    assert lib.axipcg_batch_cheb_solve(1, n1, n1, n1, None, None, 2.0, 10, 1, 0, None, None) == ax.EINVAL


def test_laguerre_coeffs_validates(ax):
    lib = ax.lib()
    f = np.zeros(2)
    g = np.zeros(4)
    assert lib.axipcg_laguerre_coeffs(4, 10.0, 2, 0.2, f.ctypes.data_as(ax._dp), g.ctypes.data_as(ax._dp),
                                      None) == ax.EINVAL
    assert lib.axipcg_laguerre_coeffs(0, 10.0, 8, 0.2, f.ctypes.data_as(ax._dp), g.ctypes.data_as(ax._dp),
                                      None) == ax.EINVAL


def test_nn_entry_points_validate_before_device_work(ax):
    lib = ax.lib()
    n = lib.axipcg_nn_num_params()
    assert n == 38465
    p = np.zeros(n, dtype=np.float32)
    out = ctypes.c_void_p()
    for nr, nz in ((0, 64), (8, 65), (8, 32), (9000, 64), (8, 8256)):
        assert lib.axipcg_nn_create(nr, nz, ax._fp(p), ctypes.byref(out)) == ax.EINVAL
        assert out.value is None
    p[100] = np.inf
    assert lib.axipcg_nn_create(8, 64, ax._fp(p), ctypes.byref(out)) == ax.EINVAL
    assert "non-finite" in ax.last_error()
    assert lib.axipcg_nn_create(8, 64, None, ctypes.byref(out)) == ax.EINVAL
    assert lib.axipcg_nn_forward(None, None, None, None, None, None, None) == ax.EINVAL
    assert lib.axipcg_nn_backward(None, None, None, None, None, None, None) == ax.EINVAL
    assert lib.axipcg_nn_adam(None, 1e-3, 0.9, 0.999, 1e-8, None) == ax.EINVAL
    assert lib.axipcg_nn_set_base(None, 2) == ax.EINVAL
    assert lib.axipcg_nn_get_base(None) == ax.EINVAL
    assert lib.axipcg_nn_backward_poly(None, None, None, 3, None, None, None) == ax.EINVAL
    assert lib.axipcg_nn_guess(None, None, None, None, None, None, None, None, None, None) == ax.EINVAL
    lib.axipcg_nn_destroy(None)  # NULL-safe


def test_series_runs_validate_before_device_work(ax):
    lib = ax.lib()
    VP = ctypes.c_void_p
    g = np.ones(3)
    a, b, c = VP(1 << 20), VP(2 << 20), VP(3 << 20)       # never dereferenced: rejected first
    same = (VP * 3)(a, a, c)
    done = ctypes.c_int(-1)
    code = lib.axipcg_series_run(None, None, 0, -1, g.ctypes.data_as(ax._dp), 0, 0, None, a, b, c, same, None, 1, 0,
                                 1e-10, 10, 1, None, ctypes.byref(done), None)
    assert code == ax.EINVAL and done.value == 0
    code = lib.axipcg_series_run(None, None, 0, 2, g.ctypes.data_as(ax._dp), 0, 0, None, a, b, c, same, None, 1, 0,
                                 1e-10, 10, 1, None, None, None)
    assert code == ax.EINVAL                                 # the three u arrays must be distinct
    two = (VP * 2)(a, b)
    code = lib.axipcg_series_run_alpha(None, 0, 2, 5, g.ctypes.data_as(ax._dp), 0, 0, None, a, b, c, two, None, 0,
                                       None, 0, 0, 1e-10, 10, 1, None, ctypes.byref(done), None)
    assert code == ax.EINVAL and done.value == 0             # NULL operator


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
