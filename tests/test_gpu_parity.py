"""GPU parity of the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances:
  * operator application: 1e-13 relative L2 (FP64, different summation order);
  * FP64 preconditioner: normwise backward error ||B z - r|| / (||B|| ||z|| +
    ||r||) <= 1e-14, and forward error vs the oracle <= 1e-9 (the r-systems of
    the low modes have condition numbers up to ~1e7);
  * FP32 preconditioner: backward error <= 2e-6 (about eps_32 log2(nz) for
    the orthogonal transforms, plus backward-stable tridiagonal elimination),
    forward error <= 2e-3;
  * PCG solutions converged to ||r||/||b|| <= 1e-10: relative L2 error <=
    1e-8 against the oracle solution converged to 1e-13.
"""
import math

import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, log, rel, spectral_norm_estimate

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def ax():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


def _problem(kind, nr, nz, bc=0, seed=0):
    if kind == "smooth":
        kappa, q = synth.medium_smooth_small(nr, seed) if nr == nz else synth.medium_layered(nr, nz, seed)
        f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.0, 0.5, 0.05)
    else:
        kappa, q = synth.medium_layered(nr, nz, seed)
        f = synth.ricker_source(nr, nz, 1.0, 1.0, 0.3, 0.01 if nr >= 512 else 0.05)
    return synth.Problem(nr, nz, 1.0, 1.0, kappa, q, np.ascontiguousarray(f), bc, seed, kind)


SHAPES = [("smooth", 64, 64, 0), ("layered", 256, 128, 0), ("layered", 128, 256, 1),
          ("layered", 100, 64, 0), ("layered", 37, 32, 1), ("layered", 2, 2, 0), ("layered", 3, 8, 1)]


@pytest.mark.parametrize("kind,nr,nz,bc", SHAPES)
def test_apply_A_matches_oracle(ax, orc, kind, nr, nz, bc):
    log(f"apply_A {kind} {nr}x{nz} bc={bc}")
    p = _problem(kind, nr, nz, bc)
    x = np.random.default_rng(1).standard_normal((nr, nz))
    with ax.op_create(p.kappa, p.q, bc_z=bc) as op:
        y = dev(np.zeros((nr, nz)))
        ax.apply_A(op, dev(x), y)
        yg = host(y)
    oop = orc.operator_from_cells(p.kappa, p.q, bc_z=bc)
    assert rel(yg, orc.apply(oop, x)) <= 1e-13


@pytest.mark.parametrize("kind,nr,nz,bc", SHAPES)
def test_rhs_and_residual_norm(ax, orc, kind, nr, nz, bc):
    log(f"rhs/residual {kind} {nr}x{nz} bc={bc}")
    p = _problem(kind, nr, nz, bc)
    x = np.random.default_rng(2).standard_normal((nr, nz))
    with ax.op_create(p.kappa, p.q, bc_z=bc) as op:
        b = dev(np.zeros((nr, nz)))
        ax.rhs_from_f(op, dev(p.f), b)
        bg = host(b)
        rn, bn = ax.residual_norm(op, b, dev(x))
    oop = orc.operator_from_cells(p.kappa, p.q, bc_z=bc)
    bo = orc.rhs(oop, p.f)
    assert rel(bg, bo) <= 1e-15
    assert math.isclose(bn, np.linalg.norm(bo), rel_tol=1e-13)
    assert math.isclose(rn, np.linalg.norm(bo - orc.apply(oop, x)), rel_tol=1e-12)


def _precond_case(ax, orc, nr, nz, bc, prec, seed=3):
    p = _problem("layered", nr, nz, bc, seed)
    r = np.random.default_rng(seed).standard_normal((nr, nz))
    with ax.op_create(p.kappa, p.q, bc_z=bc) as op:
        z = dev(np.zeros((nr, nz)))
        ax.precond_apply(op, dev(r), z, prec)
        zg = host(z)
    oop = orc.operator_from_cells(p.kappa, p.q, bc_z=bc)
    zo = orc.precond(oop, r)
    B = orc.operator_from_cells(np.full((nr, nz), oop.kbar), np.full((nr, nz), oop.qbar), bc_z=bc,
                                kbar=oop.kbar, qbar=oop.qbar)
    res = orc.apply(B, zg) - r
    nB = spectral_norm_estimate(lambda v: orc.apply(B, v), (nr, nz)) * 1.1
    back = np.linalg.norm(res) / (nB * np.linalg.norm(zg) + np.linalg.norm(r))
    fwd = rel(zg, zo)
    return back, fwd


PC_SHAPES = [(64, 64, 0), (64, 64, 1), (256, 128, 0), (128, 512, 1), (100, 64, 0), (1000, 256, 0),
             (2048, 128, 1), (4, 4, 0), (2, 2, 1), (7, 16, 0),
             # one-wave transforms (nz = 512, 1024, 2048), row counts that leave a
             # workgroup partly empty
             (130, 512, 0), (3, 512, 1), (64, 1024, 0), (37, 1024, 1), (6, 2048, 0), (33, 2048, 1),
             # rows of 4096: block-wide transforms of 512 threads, FP64 LDS above 64 KiB
             (16, 4096, 0), (9, 4096, 1)]


@pytest.mark.parametrize("nr,nz,bc", PC_SHAPES)
def test_precond_fp64(ax, orc, nr, nz, bc):
    log(f"precond fp64 {nr}x{nz} bc={bc}")
    back, fwd = _precond_case(ax, orc, nr, nz, bc, ax.PREC_FP64)
    log(f"  backward={back:.2e} forward={fwd:.2e}")
    assert back <= 1e-14
    assert fwd <= 1e-9


@pytest.mark.parametrize("nr,nz,bc", PC_SHAPES)
def test_precond_fp32(ax, orc, nr, nz, bc):
    log(f"precond fp32 {nr}x{nz} bc={bc}")
    back, fwd = _precond_case(ax, orc, nr, nz, bc, ax.PREC_FP32)
    log(f"  backward={back:.2e} forward={fwd:.2e}")
    assert back <= 2e-6   # FP32 transforms: normwise backward error (about eps32 log2 N)
    assert fwd <= 2e-3


SOLVE_CASES = [("smooth", 64, 64, 0), ("layered", 256, 256, 0), ("layered", 128, 64, 1),
               ("layered", 96, 256, 0), ("layered", 100, 128, 1), ("layered", 8, 4, 0),
               ("layered", 66, 1024, 0), ("layered", 30, 2048, 1), ("layered", 45, 512, 1),
               ("layered", 24, 4096, 0), ("layered", 13, 4096, 1),
               # the most rows op_create accepts (64 per r-solve lane), and a
               # ragged row count in the same r-solve variant
               ("layered", 4096, 32, 0), ("layered", 3000, 64, 1)]


# The most rows op_create accepts, and a ragged count in the same r-solve
# variant (segments of 46 and 47 rows).  Only the backward error is bounded:
# the forward error of a correct solve grows with the condition number of the
# r-systems (about nr^2), so a fixed forward bound would not hold at any size.
@pytest.mark.parametrize("nr,nz,bc", [(4096, 32, 0), (3000, 64, 1)])
@pytest.mark.parametrize("prec", [0, 1])
def test_precond_max_rows(ax, orc, nr, nz, bc, prec):
    log(f"precond max rows {nr}x{nz} bc={bc} prec={prec}")
    back, fwd = _precond_case(ax, orc, nr, nz, bc, prec)
    log(f"  backward={back:.2e} forward={fwd:.2e}")
    assert back <= (1e-14 if prec == ax.PREC_FP64 else 2e-6)


@pytest.mark.parametrize("kind,nr,nz,bc", SOLVE_CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_pcg_matches_oracle(ax, orc, kind, nr, nz, bc, prec):
    log(f"pcg {kind} {nr}x{nz} bc={bc} prec={prec}")
    p = _problem(kind, nr, nz, bc)
    oop = orc.operator_from_cells(p.kappa, p.q, bc_z=bc)
    bo = orc.rhs(oop, p.f)
    xr = orc.solve_reference(oop, bo)
    with ax.op_create(p.kappa, p.q, bc_z=bc) as op:
        b = dev(np.zeros((nr, nz)))
        ax.rhs_from_f(op, dev(p.f), b)
        x = dev(np.zeros((nr, nz)))
        st = ax.pcg_solve(op, b, x, rtol=1e-10, maxit=500, prec=prec, flags=ax.FLAG_TRUE_RESIDUAL)
        xg = host(x)
    log(f"  iters={st['iters']} relres={st['relres_rec']:.2e} true={st['relres_true']:.2e} err={rel(xg, xr):.2e}")
    assert st["code"] == ax.OK
    assert st["relres_rec"] <= 1e-10
    assert st["relres_true"] <= 1e-9
    assert rel(xg, xr) <= 1e-8


def test_pcg_polak_ribiere(ax, orc):
    log("pcg polak-ribiere 256x256")
    p = _problem("layered", 256, 256)
    oop = orc.operator_from_cells(p.kappa, p.q)
    xr = orc.solve_reference(oop, orc.rhs(oop, p.f))
    with ax.op_create(p.kappa, p.q) as op:
        b = dev(np.zeros((256, 256)))
        ax.rhs_from_f(op, dev(p.f), b)
        x = dev(np.zeros((256, 256)))
        st = ax.pcg_solve(op, b, x, 1e-10, 500, ax.PREC_FP32, ax.FLAG_POLAK_RIBIERE)
        assert st["code"] == ax.OK
        assert rel(host(x), xr) <= 1e-8


def test_pcg_edge_cases(ax, orc):
    log("pcg edge cases 64x64")
    p = _problem("smooth", 64, 64)
    oop = orc.operator_from_cells(p.kappa, p.q)
    bo = orc.rhs(oop, p.f)
    xr = orc.solve_reference(oop, bo)
    with ax.op_create(p.kappa, p.q) as op:
        b = dev(bo)
        # zero right-hand side: x = 0 whatever the guess
        x = dev(np.ones((64, 64)))
        st = ax.pcg_solve(op, dev(np.zeros((64, 64))), x, 1e-10, 50, ax.PREC_FP32)
        assert st["code"] == ax.OK and st["iters"] == 0 and not host(x).any()
        # the exact answer as the guess: no iteration
        x = dev(xr)
        st = ax.pcg_solve(op, b, x, 1e-10, 50, ax.PREC_FP32)
        assert st["code"] == ax.OK and st["iters"] == 0
        # maxit reached: positive status, last iterate returned
        x = dev(np.zeros((64, 64)))
        st = ax.pcg_solve(op, b, x, 1e-10, 2, ax.PREC_FP32)
        assert st["code"] == ax.ENOTCONV and st["iters"] == 2 and st["relres_rec"] > 1e-10
        # continuing from that iterate converges to the same answer
        st = ax.pcg_solve(op, b, x, 1e-10, 200, ax.PREC_FP32)
        assert st["code"] == ax.OK and rel(host(x), xr) <= 1e-8
        # invalid arguments
        with pytest.raises(ax.AxipcgError):
            ax.pcg_solve(op, b, x, -1.0, 10)
        with pytest.raises(ax.AxipcgError):
            ax.pcg_solve(op, b, x, 1e-10, 10, prec=7)


def test_results_are_bitwise_reproducible(ax):
    log("determinism 256x128")
    p = _problem("layered", 256, 128)
    outs = []
    with ax.op_create(p.kappa, p.q) as op:
        b = dev(np.zeros((256, 128)))
        ax.rhs_from_f(op, dev(p.f), b)
        for _ in range(2):
            x = dev(np.zeros((256, 128)))
            st = ax.pcg_solve(op, b, x, 1e-10, 300, ax.PREC_FP32)
            outs.append((host(x), st["iters"]))
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])


def test_face_form_matches_oracle(ax, orc):
    log("op_create_faces 64x32")
    rng = np.random.default_rng(9)
    nr, nz = 64, 32
    kr = rng.uniform(1, 3, (nr, nz))
    kz = rng.uniform(1, 3, (nr, nz + 1))
    q = rng.uniform(0, 1, (nr, nz))
    x = rng.standard_normal((nr, nz))
    oop = orc.operator_from_faces(kr, kz, q, bc_z=0, kbar=2.0, qbar=0.5)
    with ax.op_create_faces(kr, kz, q, bc_z=0, kbar=2.0, qbar=0.5) as op:
        y = dev(np.zeros((nr, nz)))
        ax.apply_A(op, dev(x), y)
        assert rel(host(y), orc.apply(oop, x)) <= 1e-13
        z = dev(np.zeros((nr, nz)))
        ax.precond_apply(op, dev(x), z, ax.PREC_FP64)
        assert rel(host(z), orc.precond(oop, x)) <= 1e-10
