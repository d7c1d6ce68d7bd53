"""The allocation-free Laguerre-coefficient entry point against the
allocating one, through the C-ABI: identical outputs (the same kernel on the
same samples) on two calls in a row, the second smaller, and the size limit
of its fixed scratch array."""
import ctypes

import numpy as np
import pytest

import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1002_3094_amd import axipcg
    return axipcg


def _call(ax, name, n, alpha, eta, f, t_max):
    g = np.full(n, np.nan)
    f = np.ascontiguousarray(f, dtype=np.float64)
    code = getattr(ax.lib(), name)(n, alpha, eta, len(f), t_max, f.ctypes.data_as(ax._dp), g.ctypes.data_as(ax._dp),
                                   None)
    return code, g


def test_noalloc_matches_allocating_entry_point_twice(lib):
    ax = lib
    t, ft = synth.gauss_sine_pulse_samples()                 # 4001 samples on [0, 0.4]
    tr, fr = synth.ricker_pulse_samples()
    cases = [(2000, 5, 300.0, ft, t[-1]),                    # the paper's experiment
             (37, 0, 10.0, fr[:1201], tr[1200])]             # smaller: fewer harmonics, fewer samples
    for n, alpha, eta, f, t_max in cases:
        log(f"noalloc laguerre coeffs n={n} alpha={alpha} nt={len(f)}")
        c1, g_noalloc = _call(ax, "axipcg_laguerre_coeffs_alpha_noalloc", n, alpha, eta, f, t_max)
        c2, g_ref = _call(ax, "axipcg_laguerre_coeffs_alpha", n, alpha, eta, f, t_max)
        assert c1 == ax.OK and c2 == ax.OK
        assert np.all(np.isfinite(g_noalloc))
        np.testing.assert_array_equal(g_noalloc, g_ref)


def test_noalloc_rejects_sizes_beyond_its_scratch(lib):
    ax = lib
    f = np.zeros(131072 - 9)
    code, g = _call(ax, "axipcg_laguerre_coeffs_alpha_noalloc", 10, 0, 10.0, f, 1.0)
    assert code == ax.EINVAL and "scratch" in ax.last_error()
    assert np.all(np.isnan(g))
    code, g = _call(ax, "axipcg_laguerre_coeffs_alpha_noalloc", 9, 0, 10.0, f, 1.0)
    assert code == ax.OK and np.all(np.isfinite(g))
