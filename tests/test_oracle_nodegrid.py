"""Pins of the oracle on the paper's node grid in r (§2.1: nodes at
(i - 1/2) h_r, h_r = l_1/(N_1 - 1/2), the last r-node on r = l_1 carrying
u = 0), z cell-centred with Neumann walls as in §4.1 eq. (32):

* the geometry of the grid: the boundary node sits exactly on r = l_r;
* the operator against the independent energy-form assembly (boundary node a
  full step away, so its face keeps the plain conductance);
* the preconditioner inverts the assembled constant-coefficient operator of
  that grid;
* second order on a closed form, u = J0(j01 r / l_r) cos(pi z / l_z), which
  vanishes on r = l_r and has du/dz = 0 at z = 0, l_z: the error ratio per
  halving lies in the band the paper's Table 2 (§4.3) brackets;
* a planted mistake (the cell grid's doubled outer face on the node grid's
  steps) fails the closed-form pin;
* the literal z-grid of §2.1 (h_z = l_2/(N_2 - 1/2)) with the one-sided
  boundary flux the paper prints (and its cosine basis, eq. (38), assumes)
  is first order: the reason the solver keeps z cell-centred.
"""
import numpy as np
import pytest
import scipy.special as ss

from tests import _assembly
from tests.test_oracle_convergence import J01, _second_order_band

NODES = 1


def test_node_grid_geometry(orc):
    for nr, nz, lr, lz in ((8, 16, 2.0, 1.5), (33, 7, 1.0, 1.0)):
        op = orc.operator_from_cells(np.ones((nr, nz)), np.zeros((nr, nz)), lr, lz, orc.Z_NEUMANN,
                                     grid=orc.GRID_NODES)
        assert op.hr == pytest.approx(lr / (nr + 0.5))
        assert op.r[-1] + op.hr == pytest.approx(lr, rel=1e-15)        # the boundary node on r = lr
        assert op.hz == pytest.approx(lz / nz)                          # z cell-centred
        assert op.r[0] == pytest.approx(0.5 * op.hr)                   # first node half a step off the axis


@pytest.mark.parametrize("shape", [(5, 7), (8, 8), (16, 12)])
def test_node_grid_apply_matches_energy_assembly(orc, shape):
    rng = np.random.default_rng(13)
    nr, nz = shape
    kr = rng.uniform(0.5, 3.0, (nr, nz))
    kz = rng.uniform(0.5, 3.0, (nr, nz + 1))
    q = rng.uniform(0.0, 2.0, (nr, nz))
    op = orc.operator_from_faces(kr, kz, q, 1.3, 0.7, orc.Z_NEUMANN, grid=orc.GRID_NODES)
    A = _assembly.assemble(kr, kz, q, 1.3, 0.7, 1, grid=NODES)
    for _ in range(3):
        x = rng.standard_normal((nr, nz))
        y = orc.apply(op, x)
        yref = (A @ x.ravel()).reshape(nr, nz)
        assert np.linalg.norm(y - yref) <= 1e-13 * np.linalg.norm(yref)
    # and the node grid differs from the cell grid exactly by its steps and
    # the outer face (so the pin above can tell them apart)
    opc = orc.operator_from_faces(kr, kz, q, 1.3, 0.7, orc.Z_NEUMANN)
    assert not np.allclose(orc.apply(opc, x), y)


@pytest.mark.parametrize("shape", [(6, 8), (16, 16), (31, 32)])
def test_node_grid_preconditioner_inverts_assembled_B(orc, shape):
    nr, nz = shape
    kbar, qbar = 1.7, 0.4
    op = orc.operator_from_cells(np.full((nr, nz), kbar), np.full((nr, nz), qbar), 1.0, 2.0, orc.Z_NEUMANN,
                                 kbar=kbar, qbar=qbar, grid=orc.GRID_NODES)
    B = _assembly.assemble(np.full((nr, nz), kbar), np.full((nr, nz + 1), kbar), np.full((nr, nz), qbar),
                           1.0, 2.0, 1, grid=NODES)
    r = np.random.default_rng(5).standard_normal((nr, nz))
    z = orc.precond(op, r)
    assert np.linalg.norm((B @ z.ravel()).reshape(nr, nz) - r) <= 1e-12 * np.linalg.norm(r)


def _bessel_cos_errors(orc, apply_fn=None):
    kap, q, lr, lz = 1.3, 0.7, 1.0, 1.0
    errs = []
    for N in (16, 32, 64):
        op = orc.operator_from_cells(np.full((N, N), kap), np.full((N, N), q), lr, lz, orc.Z_NEUMANN,
                                     grid=orc.GRID_NODES)
        r, z = op.r, (np.arange(N) + 0.5) * op.hz
        u = ss.j0(J01 * r / lr)[:, None] * np.cos(np.pi * z / lz)[None, :]
        f = (kap * ((J01 / lr) ** 2 + (np.pi / lz) ** 2) + q) * u
        b = orc.rhs(op, f)
        if apply_fn is None:
            x, st, it, rel = orc.pcg(op, b, rtol=1e-13)
        else:
            x = apply_fn(op, b)
        errs.append(np.linalg.norm(x - u) / np.linalg.norm(u))
    return errs


def test_node_grid_second_order_on_closed_form(orc):
    errs = _bessel_cos_errors(orc)
    lo, hi = _second_order_band()
    for e0, e1 in zip(errs, errs[1:]):
        assert lo <= e0 / e1 <= hi, errs


def test_planted_doubled_outer_face_fails_the_pin(orc):
    """The cell grid's doubled outer face (ghost half a step away) on the
    node grid's steps, planted in a copy of the operator: the closed-form pin
    then sees first order at best."""
    def solve_mutant(op, b):
        cr = op.cr.copy()
        cr[-1] *= 2.0
        import dataclasses
        bad = dataclasses.replace(op, cr=cr)
        A = _dense(orc, bad)
        return np.linalg.solve(A, b.ravel()).reshape(b.shape)

    errs = _bessel_cos_errors(orc, solve_mutant)
    lo, hi = _second_order_band()
    assert not all(lo <= e0 / e1 <= hi for e0, e1 in zip(errs, errs[1:])), errs


def _dense(orc, op):
    n = op.nr * op.nz
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = orc.apply(op, e.reshape(op.nr, op.nz)).ravel()
    return A


def test_literal_z_node_grid_is_first_order(orc):
    """The paper's z-grid taken literally: h_z = l_z/(N_2 - 1/2), the last
    node on z = l_z, and at that node the one-sided flux (1/h) a_2 y_zbar of
    eq. (5) over a full step.  That is the cell-centred Neumann operator with
    its wall at N_2 h_z = l_z + h_z/2, so against u = cos(pi z / l_z) the
    error halves (not quarters) per refinement."""
    kap, q, lz = 1.0, 0.3, 1.0
    errs = []
    for N in (16, 32, 64):
        hz = lz / (N - 0.5)
        z = (np.arange(N) + 0.5) * hz
        T = np.zeros((N, N))
        for k in range(N):
            if k > 0:
                T[k, k] += kap / hz**2
                T[k, k - 1] -= kap / hz**2
            if k < N - 1:
                T[k, k] += kap / hz**2
                T[k, k + 1] -= kap / hz**2
            T[k, k] += q
        u = np.cos(np.pi * z / lz)
        x = np.linalg.solve(T, (kap * (np.pi / lz) ** 2 + q) * u)
        errs.append(np.linalg.norm(x - u) / np.linalg.norm(u))
    ratios = [e0 / e1 for e0, e1 in zip(errs, errs[1:])]
    assert all(1.7 < r < 2.3 for r in ratios), ratios
    # the same operator on h_z = l_z / N (the wall on the face) is second order
    assert np.allclose(orc.mode_eig(8, 1.0, orc.Z_NEUMANN, grid=orc.GRID_NODES), orc.mode_eig(8, 1.0, orc.Z_NEUMANN))
