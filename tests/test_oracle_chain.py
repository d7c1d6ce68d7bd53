"""Pins of the oracle's Laguerre series drivers (§4.1 eq. (35), alpha = 0
and general alpha) against independent chains built on a sparse direct
solver."""
import math
from fractions import Fraction

import numpy as np
import scipy.sparse.linalg as spla

import synth
from tests import _assembly


def test_chain_matches_sparse_direct_chain(orc):
    inp = synth.laguerre_series_inputs(12, 16, seed=3)
    kappa, q, eta = inp["kappa"], inp["q"], inp["eta"]
    nr, nz = kappa.shape
    op = orc.operator_from_cells(kappa, q)
    g = orc.laguerre_coeffs(8, eta, inp["ft"], inp["t"][-1])
    us, stats = orc.laguerre_chain(op, kappa, g, eta, inp["src_i"], inp["src_k"], 8, rtol=1e-13)

    kr, kz = orc.face_kappa(kappa)
    A = _assembly.assemble(kr, kz, q).tocsc()
    lu = spla.splu(A)
    hr, hz = 1.0 / nr, 1.0 / nz
    r = (np.arange(nr) + 0.5) * hr
    ref = []
    for m in range(8):
        # the running-sum form S1_m = sum_{k<m} u_k, S2_m = S2_{m-1} + S1_m
        # equals sum_{k<m} (m-k) u_k; it is used here so that the two chains
        # do not share the way the history term is formed.
        if m == 0:
            S1 = np.zeros((nr, nz))
            S2 = np.zeros((nr, nz))
        else:
            S1 = S1 + ref[-1]
            S2 = S2 + S1
        f = -(eta * eta / kappa) * S2
        f[inp["src_i"], inp["src_k"]] += g[m] / (r[inp["src_i"]] * hr * hz)
        ref.append(lu.solve((r[:, None] * f).ravel()).reshape(nr, nz))
    for m in range(8):
        assert stats[m][0] == 0
        assert np.linalg.norm(us[m] - ref[m]) <= 1e-11 * np.linalg.norm(ref[m]), m


def _weight(m: int, k: int, alpha: int) -> float:
    """(m - k) sqrt(m! (k + alpha)! / ((m + alpha)! k!)), from exact integers."""
    ratio = Fraction(math.factorial(m) * math.factorial(k + alpha), math.factorial(m + alpha) * math.factorial(k))
    return (m - k) * math.sqrt(ratio)


def test_alpha_chain_matches_sparse_direct_chain(orc):
    """The general-alpha driver (§4.1 eq. (35), the paper's medium: rho = 1,
    Neumann in z) against a chain of sparse LU solves whose history weights
    are formed pairwise from exact factorials (the oracle splits them into a
    factor of m and a factor of k)."""
    n = 7
    inp = synth.paper_series_inputs(10, 16, seed=4, eta=30.0, alpha=5)
    kappa, q, coef, alpha = inp["kappa"], inp["q"], inp["coef"], inp["alpha"]
    nr, nz = kappa.shape
    # with rho = 1 the reaction term of eq. (35) is a quarter of the history coefficient
    np.testing.assert_array_equal(4.0 * q, coef)
    op = orc.operator_from_cells(kappa, q, lr=inp["lr"], lz=inp["lz"], bc_z=inp["bc_z"])
    g = orc.laguerre_coeffs_a(n, alpha, inp["eta"], inp["ft"], inp["t"][-1])
    us, stats = orc.laguerre_chain_a(op, coef, g, alpha, inp["src_i"], inp["src_k"], n)

    kr, kz = orc.face_kappa(kappa)
    lu = spla.splu(_assembly.assemble(kr, kz, q, inp["lr"], inp["lz"], inp["bc_z"]).tocsc())
    hr, hz = inp["lr"] / nr, inp["lz"] / nz
    r = (np.arange(nr) + 0.5) * hr
    ref = []
    for m in range(n):
        hist = np.zeros((nr, nz))
        for k in range(m):
            hist += _weight(m, k, alpha) * ref[k]
        f = -coef * hist
        f[inp["src_i"], inp["src_k"]] += g[m] / (r[inp["src_i"]] * hr * hz)
        ref.append(lu.solve((r[:, None] * f).ravel()).reshape(nr, nz))
    for m in range(n):
        assert stats[m][0] == 0
        assert np.linalg.norm(us[m] - ref[m]) <= 1e-11 * np.linalg.norm(ref[m]), m
    # the history term is exercised: the last harmonic without it is far off
    f = np.zeros((nr, nz))
    f[inp["src_i"], inp["src_k"]] = g[n - 1] / (r[inp["src_i"]] * hr * hz)
    bare = lu.solve((r[:, None] * f).ravel()).reshape(nr, nz)
    assert np.linalg.norm(us[-1] - bare) > 1e-3 * np.linalg.norm(us[-1])
