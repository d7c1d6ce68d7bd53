"""Chebyshev form of eq. (8) on the GPU against the oracle.

The GPU runs the iteration in increment form, the oracle in the paper's
three-layer form; they are the same polynomial in B^{-1}A, so with the FP64
preconditioner the k-th iterates agree to rounding (1e-11 relative after 25
steps, with the rounding of both preconditioners amplified by at most the
Chebyshev polynomial's bound, <= 1).  Converged answers (rtol 1e-10) match
the PCG reference to 1e-8 with either preconditioner.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, log, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ax():
    import torch
    assert torch.cuda.is_available()
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


# (512, 32) and (600, 64): FP64 transforms two rows per workgroup (one complex
# FFT for both), in the Chebyshev step and start modes too
CASES = [(64, 64, 0), (128, 256, 1), (96, 64, 0), (256, 256, 0), (42, 1024, 1), (20, 4096, 1), (512, 32, 1),
         (600, 64, 0)]


@pytest.mark.parametrize("nr,nz,bc", CASES)
def test_bounds_match_oracle(ax, orc, nr, nz, bc):
    kappa, q = synth.medium_layered(nr, nz, 5)
    with ax.op_create(kappa, q, bc_z=bc) as op:
        g = ax.op_bounds(op)
    go = orc.energy_bounds(orc.operator_from_cells(kappa, q, bc_z=bc))
    assert g[0] == pytest.approx(go[0], rel=1e-13) and g[1] == pytest.approx(go[1], rel=1e-13)


def test_bounds_face_form(ax, orc):
    nr, nz = 32, 64
    kappa, q = synth.medium_layered(nr, nz, 9)
    kr, kz = orc.face_kappa(kappa)
    with ax.op_create_faces(kr, kz, q, kbar=2.0, qbar=float(q.mean())) as op:
        g = ax.op_bounds(op)
    go = orc.energy_bounds(orc.operator_from_faces(kr, kz, q, kbar=2.0, qbar=float(q.mean())))
    assert g[0] == pytest.approx(go[0], rel=1e-13) and g[1] == pytest.approx(go[1], rel=1e-13)


@pytest.mark.parametrize("nr,nz,bc", CASES)
def test_iterates_match_oracle(ax, orc, nr, nz, bc):
    log(f"cheb iterates {nr}x{nz} bc={bc}")
    kappa, q = synth.medium_layered(nr, nz, 6)
    f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.1, 0.5, 0.05)
    oop = orc.operator_from_cells(kappa, q, bc_z=bc)
    b = orc.rhs(oop, f)
    x0 = np.random.default_rng(3).standard_normal((nr, nz)) * 1e-3
    g1, g2 = orc.energy_bounds(oop)
    k = 25
    yo, _, ko, _ = orc.cheb(oop, b, x0, g1, g2, iters=k)
    with ax.op_create(kappa, q, bc_z=bc) as op:
        x = dev(x0)
        st = ax.cheb_solve(op, dev(b), x, g1, g2, rtol=1e-30, maxit=k, prec=ax.PREC_FP64)
        assert st["code"] == ax.ENOTCONV and st["iters"] == k
        e = rel(host(x), yo)
    log(f"  after {k} steps: rel diff {e:.2e}")
    # two FP64 evaluations of the same 25-step polynomial differ by rounding
    # only; the per-step difference grows with the row length (the
    # transforms' log2 N rounding and the z-modes' spread, h_z^-2), so the
    # bound scales with nz beyond 1024
    assert e <= 1e-11 * max(1, nz // 1024)


@pytest.mark.parametrize("nr,nz,bc", CASES)
@pytest.mark.parametrize("prec", [0, 1])
def test_converged_matches_reference(ax, orc, nr, nz, bc, prec):
    kappa, q = synth.medium_layered(nr, nz, 7)
    f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.2, 0.4, 0.05)
    oop = orc.operator_from_cells(kappa, q, bc_z=bc)
    b = orc.rhs(oop, f)
    xr = orc.solve_reference(oop, b)
    with ax.op_create(kappa, q, bc_z=bc) as op:
        x = dev(np.zeros((nr, nz)))
        st = ax.cheb_solve(op, dev(b), x, rtol=1e-10, maxit=500, prec=prec)
        xs = dict(st)
        y = dev(np.zeros((nr, nz)))
        sp = ax.pcg_solve(op, dev(b), y, rtol=1e-10, maxit=500, prec=prec)
        rn, bn = ax.residual_norm(op, dev(b), x)
        err = rel(host(x), xr)
    log(f"cheb {nr}x{nz} bc={bc} prec={prec}: iters {xs['iters']} (pcg {sp['iters']}), true relres {rn / bn:.2e}, "
        f"err {err:.2e}")
    assert xs["code"] == ax.OK and xs["relres_rec"] <= 1e-10
    assert rn / bn <= 1e-9
    assert err <= 1e-8


def test_edge_cases(ax, orc):
    nr, nz = 32, 32
    kappa, q = synth.medium_layered(nr, nz, 2)
    with ax.op_create(kappa, q) as op:
        x = dev(np.ones((nr, nz)))
        st = ax.cheb_solve(op, dev(np.zeros((nr, nz))), x)
        assert st["code"] == ax.OK and st["iters"] == 0
        assert np.all(host(x) == 0.0)
        with pytest.raises(ax.AxipcgError):
            ax.cheb_solve(op, dev(np.ones((nr, nz))), x, gamma1=2.0, gamma2=1.0)
        with pytest.raises(ax.AxipcgError):
            ax.cheb_solve(op, dev(np.ones((nr, nz))), x, gamma1=-1.0, gamma2=1.0)
        # an interval below the whole spectrum: every eigencomponent is amplified
        # (|P_n| > 1 outside [gamma1, gamma2] on the far side of 0), the iteration
        # diverges and says so
        g1, g2 = ax.op_bounds(op)
        x = dev(np.zeros((nr, nz)))
        try:
            code = ax.cheb_solve(op, dev(np.ones((nr, nz))), x, 0.2 * g1, 0.21 * g1, maxit=300)["code"]
        except ax.AxipcgError as e:
            code = e.code
        assert code in (ax.ENOTCONV, ax.EBREAKDOWN)
