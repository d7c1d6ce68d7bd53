"""Pins of the Chebyshev form of eq. (8) in the oracle.

* the energy bounds of eq. (10) contain every eigenvalue of B^{-1}A (dense
  generalized eigenproblem of the independently assembled matrices);
* after n steps the error is exactly P_n(B^{-1}A) e_0 with the scaled
  Chebyshev polynomial P_n(x) = T_n((g2 + g1 - 2x)/(g2 - g1)) / T_n((g2 + g1)/(g2 - g1))
  (closed form; a wrong alpha or tau anywhere breaks it);
* the converged answer equals the PCG reference.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from synth import medium_layered
from tests._assembly import assemble


def _setup(orc, nr, nz, seed, bc=0):
    kappa, q = medium_layered(nr, nz, seed)
    op = orc.operator_from_cells(kappa, q, bc_z=bc)
    kr, kz = orc.face_kappa(kappa)
    A = assemble(kr, kz, q, bc_z=bc).toarray()
    B = assemble(np.full_like(kr, op.kbar), np.full_like(kz, op.kbar), np.full_like(q, op.qbar), bc_z=bc).toarray()
    return op, A, B


@pytest.mark.parametrize("bc", [0, 1])
def test_energy_bounds_contain_spectrum(orc, bc):
    op, A, B = _setup(orc, 6, 8, 3, bc)
    lam = sla.eigh(A, B, eigvals_only=True)
    g1, g2 = orc.energy_bounds(op)
    assert g1 <= lam.min() * (1 + 1e-12) and lam.max() <= g2 * (1 + 1e-12)
    assert g1 > 0


def test_error_is_the_chebyshev_polynomial(orc):
    op, A, B = _setup(orc, 6, 8, 4)
    lam, V = sla.eigh(A, B)                     # A V = B V diag(lam), V^T B V = I
    g1, g2 = lam.min() * 0.97, lam.max() * 1.02
    rng = np.random.default_rng(0)
    u = rng.standard_normal(48)
    f = A @ u
    y0 = rng.standard_normal(48)
    c = V.T @ B @ (y0 - u)                      # coordinates of e_0
    for n in range(1, 11):
        y, _, k, _ = orc.cheb(op, f.reshape(6, 8), y0.reshape(6, 8), g1, g2, iters=n)
        assert k == n
        xs = (g2 + g1 - 2 * lam) / (g2 - g1)
        Pn = np.cos(n * np.arccos(np.clip(xs, -1, 1))) / np.cosh(n * np.arccosh((g2 + g1) / (g2 - g1)))
        pred = u + V @ (Pn * c)
        assert np.linalg.norm(y.ravel() - pred) <= 1e-10 * np.linalg.norm(y0 - u), n


def test_converges_to_reference(orc):
    kappa, q = medium_layered(32, 64, 6)
    op = orc.operator_from_cells(kappa, q)
    f = np.random.default_rng(1).standard_normal((32, 64))
    y, st, k, rel = orc.cheb(op, f, rtol=1e-11, maxit=400)
    ref = orc.solve_reference(op, f)
    assert st == 0 and rel <= 1e-11
    assert np.linalg.norm(y - ref) <= 1e-9 * np.linalg.norm(ref)
