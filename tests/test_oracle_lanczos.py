"""Pins of the oracle's Lanczos bounds of B^{-1} A (taken out of PCG steps,
§2.2 eq. (8) with conjugate-gradient parameters), for the Chebyshev form.

* after as many steps as unknowns, the extreme eigenvalues of the Lanczos
  matrix are those of the generalized eigenproblem A v = lambda B v of the
  independently assembled matrices (a wrong entry of T, or a wrong alpha or
  beta, moves them);
* after a few steps they lie inside that spectrum (Ritz values interlace);
* the energy bounds of eq. (10) contain them;
* with A = B (constant medium) every Ritz value is 1.
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
def test_full_lanczos_gives_the_spectrum_ends(orc, bc):
    op, A, B = _setup(orc, 6, 8, 11, bc)
    lam = sla.eigh(A, B, eigvals_only=True)
    b = np.random.default_rng(1).standard_normal((6, 8))
    lo, hi = orc.lanczos_bounds(op, b, 6 * 8)
    assert lo == pytest.approx(lam.min(), rel=1e-8)
    assert hi == pytest.approx(lam.max(), rel=1e-8)


@pytest.mark.parametrize("steps", [2, 5, 12])
def test_few_steps_lie_inside_the_spectrum_and_the_energy_bounds(orc, steps):
    op, A, B = _setup(orc, 8, 16, 12)
    lam = sla.eigh(A, B, eigvals_only=True)
    b = np.random.default_rng(2).standard_normal((8, 16))
    lo, hi = orc.lanczos_bounds(op, b, steps)
    g1, g2 = orc.energy_bounds(op)
    assert lam.min() * (1 - 1e-12) <= lo <= hi <= lam.max() * (1 + 1e-12)
    assert g1 <= lo and hi <= g2


def test_more_steps_widen_the_interval(orc):
    # the extreme Ritz values move monotonically outwards with the steps
    op, A, B = _setup(orc, 8, 16, 13)
    b = np.random.default_rng(3).standard_normal((8, 16))
    prev = None
    for k in (2, 4, 8, 16):
        lo, hi = orc.lanczos_bounds(op, b, k)
        if prev is not None:
            assert lo <= prev[0] * (1 + 1e-12) and hi >= prev[1] * (1 - 1e-12)
        prev = (lo, hi)


def test_identity_when_the_medium_is_constant(orc):
    nr, nz = 6, 8
    op = orc.operator_from_cells(np.full((nr, nz), 2.0), np.full((nr, nz), 0.5))
    b = np.random.default_rng(4).standard_normal((nr, nz))
    lo, hi = orc.lanczos_bounds(op, b, 3)
    assert lo == pytest.approx(1.0, abs=1e-10) and hi == pytest.approx(1.0, abs=1e-10)
