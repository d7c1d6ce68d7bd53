"""The 4096 x 4096 grid (rows of 4096: the block-wide transforms of 512
threads, the per-mode r-solve at the most rows op_create accepts), through
the C-ABI.

* the standalone preconditioner against the oracle's over the whole grid, in
  both precisions and both z-boundaries, by the normwise backward error (the
  bounds of the other preconditioner tests: 1e-14 FP64, 2e-6 FP32; the
  forward error of the low modes' r-systems grows as nr^2 and is not bounded
  at this size);
* a PCG solve with each preconditioner: both converge to 1e-10, the oracle's
  own apply of A gives a true residual within 1e-9 of ||b|| for each, and the
  two solutions of the same system agree to 1e-8 (the solve's parity
  property at any size; the oracle's full solve at 16.8 M points would take
  minutes);
* solves whose row count leaves the SpMV's 16-row tiles ragged (2063 x 2048,
  1031 x 4096), checked the same way.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, log, rel, spectral_norm_estimate

pytestmark = pytest.mark.gpu

N = 4096


@pytest.fixture(scope="module")
def ax():
    import torch
    assert torch.cuda.is_available()
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


@pytest.fixture(scope="module")
def medium():
    kappa, q = synth.medium_layered(N, N, 3)
    return kappa, q


@pytest.mark.parametrize("bc", [0, 1])
def test_precond_4096(ax, orc, medium, bc):
    kappa, q = medium
    r = np.random.default_rng(40 + bc).standard_normal((N, N))
    oop = orc.operator_from_cells(kappa, q, bc_z=bc)
    B = orc.operator_from_cells(np.full((N, N), oop.kbar), np.full((N, N), oop.qbar), bc_z=bc,
                                kbar=oop.kbar, qbar=oop.qbar)
    nB = spectral_norm_estimate(lambda v: orc.apply(B, v), (N, N), iters=20) * 1.1
    with ax.op_create(kappa, q, bc_z=bc) as op:
        z = dev(np.zeros((N, N)))
        for prec, bound in ((ax.PREC_FP64, 1e-14), (ax.PREC_FP32, 2e-6)):
            log(f"precond {N}x{N} bc={bc} prec={prec}")
            ax.precond_apply(op, dev(r), z, prec)
            zg = host(z)
            back = np.linalg.norm(orc.apply(B, zg) - r) / (nB * np.linalg.norm(zg) + np.linalg.norm(r))
            log(f"  backward={back:.2e}")
            assert np.all(np.isfinite(zg))
            assert back <= bound


def test_pcg_4096(ax, orc, medium):
    kappa, q = medium
    f = synth.ricker_source(N, N, 1.0, 1.0, 0.3, 0.01)
    oop = orc.operator_from_cells(kappa, q)
    bo = orc.rhs(oop, f)
    sols = {}
    with ax.op_create(kappa, q) as op:
        for prec in (ax.PREC_FP64, ax.PREC_FP32):
            x = dev(np.zeros((N, N)))
            st = ax.pcg_solve(op, dev(bo), x, rtol=1e-10, maxit=500, prec=prec, flags=ax.FLAG_TRUE_RESIDUAL)
            xg = host(x)
            true = np.linalg.norm(bo - orc.apply(oop, xg)) / np.linalg.norm(bo)
            log(f"pcg {N}x{N} prec={prec}: iters={st['iters']} relres={st['relres_rec']:.2e} "
                f"oracle true residual={true:.2e}")
            assert st["code"] == ax.OK and st["relres_rec"] <= 1e-10
            assert true <= 1e-9
            sols[prec] = xg
    d = rel(sols[ax.PREC_FP32], sols[ax.PREC_FP64])
    log(f"  FP32 vs FP64 preconditioner solutions: {d:.2e}")
    assert d <= 1e-8


# 2063 = 128 * 16 + 15 rows of 2048 (and 1031 = 64 * 16 + 7 of 4096): the
# SpMV takes tiles of 16 rows there, the last one partly empty
@pytest.mark.parametrize("nr,nz", [(2063, 2048), (1031, 4096)])
def test_pcg_ragged_spmv_tiles(ax, orc, nr, nz):
    kappa, q = synth.medium_layered(nr, nz, 5)
    f = synth.ricker_source(nr, nz, 1.0, 1.0, 0.3, 0.01)
    oop = orc.operator_from_cells(kappa, q, bc_z=1)
    bo = orc.rhs(oop, f)
    with ax.op_create(kappa, q, bc_z=1) as op:
        x = dev(np.zeros((nr, nz)))
        st = ax.pcg_solve(op, dev(bo), x, rtol=1e-10, maxit=500, prec=ax.PREC_FP32, flags=ax.FLAG_TRUE_RESIDUAL)
        xg = host(x)
    true = np.linalg.norm(bo - orc.apply(oop, xg)) / np.linalg.norm(bo)
    log(f"pcg {nr}x{nz}: iters={st['iters']} relres={st['relres_rec']:.2e} oracle true residual={true:.2e}")
    assert st["code"] == ax.OK and st["relres_rec"] <= 1e-10
    assert true <= 1e-9
