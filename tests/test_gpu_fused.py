"""Single-pass (cooperative, opt-in) preconditioner against the oracle and
against the three-launch form.

The fused form eliminates each strip's interior rows against the strip's
boundary rows and solves the reduced system of those boundary rows per mode;
the three-launch form eliminates per lane segment inside one wavefront.  Both
compute B^{-1} r, so the bounds are those of the preconditioner tests: FP64
backward error <= 1e-14 and forward <= 1e-9 (and the two forms within 1e-12
of each other), FP32 backward <= 32 eps32 log2 nz and forward <= 2e-3.
"""
import math

import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, log, rel, spectral_norm_estimate

pytestmark = pytest.mark.gpu
EPS32 = float(np.finfo(np.float32).eps)


@pytest.fixture(scope="module")
def ax():
    import torch
    assert torch.cuda.is_available()
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


# (nr, nz, bc, prec) whose geometry the single-pass form accepts
FUSED_CASES = [(64, 64, 0, 0), (64, 64, 1, 1), (256, 128, 0, 1), (128, 512, 1, 0), (32, 16, 0, 0),
               (2048, 128, 1, 1), (1024, 1024, 0, 1), (1024, 1024, 1, 0), (2048, 2048, 0, 1), (512, 2048, 1, 1)]


@pytest.mark.parametrize("nr,nz,bc,prec", FUSED_CASES)
def test_fused_precond(ax, orc, nr, nz, bc, prec):
    log(f"fused precond {nr}x{nz} bc={bc} prec={prec}")
    kappa, q = synth.medium_layered(nr, nz, 7)
    r = np.random.default_rng(11).standard_normal((nr, nz))
    with ax.op_create(kappa, q, bc_z=bc) as op:
        assert not ax.op_fused_info(op, prec)[0]        # opt-in
        ax.op_set_fused(op, True)
        active, strips, _ = ax.op_fused_info(op, prec)
        log(f"  single-pass active={active} strips={strips}")
        assert active
        z = dev(np.zeros((nr, nz)))
        ax.precond_apply(op, dev(r), z, prec)
        zf = host(z)
        ax.op_set_fused(op, False)
        ax.precond_apply(op, dev(r), z, prec)
        z3 = host(z)
        _, _, errs = ax.op_fused_info(op, prec, want_errors=True)
        assert errs == 0
    oop = orc.operator_from_cells(kappa, q, bc_z=bc)
    zo = orc.precond(oop, r)
    B = orc.operator_from_cells(np.full((nr, nz), oop.kbar), np.full((nr, nz), oop.qbar), bc_z=bc,
                                kbar=oop.kbar, qbar=oop.qbar)
    res = orc.apply(B, zf) - r
    nB = spectral_norm_estimate(lambda v: orc.apply(B, v), (nr, nz)) * 1.1
    back = np.linalg.norm(res) / (nB * np.linalg.norm(zf) + np.linalg.norm(r))
    fwd = rel(zf, zo)
    log(f"  backward={back:.2e} forward={fwd:.2e} fused-vs-three={rel(zf, z3):.2e}")
    if prec == ax.PREC_FP64:
        assert back <= 1e-14 and fwd <= 1e-9 and rel(zf, z3) <= 1e-12
    else:
        assert back <= 32 * EPS32 * max(1.0, math.log2(nz)) and fwd <= 2e-3


def test_fused_inactive_geometry_falls_back(ax, orc):
    # 100 rows: no power-of-two strip count divides it; the three launches run
    kappa, q = synth.medium_layered(100, 64, 2)
    with ax.op_create(kappa, q) as op:
        ax.op_set_fused(op, True)
        active, strips, _ = ax.op_fused_info(op, ax.PREC_FP32)
        assert not active and strips == 0
        r = np.random.default_rng(1).standard_normal((100, 64))
        z = dev(np.zeros((100, 64)))
        ax.precond_apply(op, dev(r), z, ax.PREC_FP32)
        oop = orc.operator_from_cells(kappa, q)
        assert rel(host(z), orc.precond(oop, r)) <= 2e-3
