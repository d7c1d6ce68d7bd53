"""Pins of the oracle's Thomas solver, preconditioner (§4.2 eqs. (36)-(39))
and PCG (§2.2 eq. (8)) against library solvers and exact properties."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from tests import _assembly


def test_thomas_matches_solve_banded(orc):
    rng = np.random.default_rng(0)
    n = 257
    a = -rng.uniform(0.1, 1.0, n)
    c = -rng.uniform(0.1, 1.0, n)
    b = 2.5 + rng.uniform(0.0, 1.0, n)
    a[0] = 0.0
    c[-1] = 0.0
    f = rng.standard_normal(n)
    ab = np.zeros((3, n))
    ab[0, 1:] = c[:-1]
    ab[1] = b
    ab[2, :-1] = a[1:]
    ref = sla.solve_banded((1, 1), ab, f)
    assert np.abs(orc.thomas(a, b, c, f) - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [(8, 8), (24, 16), (17, 32)])
def test_precond_inverts_constant_coefficient_operator(orc, bc, shape):
    """B^{-1} is the exact inverse of the scheme's operator with kappa = kbar,
    q = qbar (eqs. (36)-(37)); B is assembled independently."""
    nr, nz = shape
    rng = np.random.default_rng(1)
    kbar, qbar = 1.7, 0.4
    op = orc.operator_from_cells(np.full((nr, nz), kbar), np.full((nr, nz), qbar), 1.0, 1.3, bc,
                                 kbar=kbar, qbar=qbar)
    assert op.kbar == pytest.approx(kbar, rel=1e-15) and op.qbar == pytest.approx(qbar, rel=1e-15)
    B = _assembly.assemble(np.full((nr, nz), kbar), np.full((nr, nz + 1), kbar),
                           np.full((nr, nz), qbar), 1.0, 1.3, bc)
    r = rng.standard_normal((nr, nz))
    z = orc.precond(op, r)
    res = B @ z.ravel() - r.ravel()
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(r)


@pytest.mark.parametrize("bc", [0, 1])
def test_precond_with_zero_qbar_neumann_is_definite(orc, bc):
    """With q = 0 and Neumann z the l = 0 mode relies on the Dirichlet face at
    r = l_r; the r-system stays nonsingular."""
    nr, nz = 16, 16
    op = orc.operator_from_cells(np.ones((nr, nz)), np.zeros((nr, nz)), bc_z=bc)
    B = _assembly.assemble(np.ones((nr, nz)), np.ones((nr, nz + 1)), np.zeros((nr, nz)), 1.0, 1.0, bc)
    r = np.random.default_rng(2).standard_normal((nr, nz))
    z = orc.precond(op, r)
    assert np.linalg.norm(B @ z.ravel() - r.ravel()) <= 1e-11 * np.linalg.norm(r)


@pytest.mark.parametrize("bc", [0, 1])
def test_pcg_constant_coefficients_converges_in_one_iteration(orc, bc):
    n = 32
    op = orc.operator_from_cells(np.full((n, n), 2.0), np.full((n, n), 0.3), bc_z=bc)
    b = np.random.default_rng(3).standard_normal((n, n))
    x, st, it, rel = orc.pcg(op, b, rtol=1e-10)
    assert st == 0 and it == 1 and rel <= 1e-10


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [(48, 32), (32, 64)])
def test_pcg_matches_sparse_direct(orc, bc, shape):
    nr, nz = shape
    rng = np.random.default_rng(4)
    kappa = 1.0 + 3.0 * rng.uniform(size=(nr, nz))
    q = rng.uniform(0.0, 1.0, (nr, nz))
    op = orc.operator_from_cells(kappa, q, 1.0, 0.5, bc)
    kr, kz = orc.face_kappa(kappa)
    A = _assembly.assemble(kr, kz, q, 1.0, 0.5, bc)
    b = rng.standard_normal((nr, nz))
    xref = spla.spsolve(A.tocsc(), b.ravel()).reshape(nr, nz)
    x, st, it, rel = orc.pcg(op, b, rtol=1e-13, maxit=300)
    assert st == 0
    assert np.linalg.norm(x - xref) <= 1e-11 * np.linalg.norm(xref)


def test_pcg_nonzero_guess_and_dense(orc):
    nr, nz = 6, 8
    rng = np.random.default_rng(5)
    kappa = rng.uniform(1, 4, (nr, nz))
    q = rng.uniform(0, 1, (nr, nz))
    op = orc.operator_from_cells(kappa, q)
    kr, kz = orc.face_kappa(kappa)
    A = _assembly.assemble(kr, kz, q).toarray()
    b = rng.standard_normal((nr, nz))
    xref = np.linalg.solve(A, b.ravel()).reshape(nr, nz)
    x, st, it, rel = orc.pcg(op, b, x0=xref + 1e-3 * rng.standard_normal((nr, nz)), rtol=1e-13)
    assert st == 0 and np.linalg.norm(x - xref) <= 1e-12 * np.linalg.norm(xref)


def test_pcg_zero_rhs(orc):
    op = orc.operator_from_cells(np.ones((8, 8)), np.ones((8, 8)))
    x, st, it, rel = orc.pcg(op, np.zeros((8, 8)), x0=np.ones((8, 8)))
    assert st == 0 and it == 0 and not x.any()


def test_pcg_maxit_reports_not_converged(orc):
    rng = np.random.default_rng(6)
    kappa = rng.uniform(1, 4, (32, 32))
    op = orc.operator_from_cells(kappa, np.zeros((32, 32)))
    x, st, it, rel = orc.pcg(op, rng.standard_normal((32, 32)), rtol=1e-12, maxit=2)
    assert st == 1 and it == 2 and rel > 1e-12
