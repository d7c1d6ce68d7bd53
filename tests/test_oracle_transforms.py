"""Pins of the oracle's FFT, z-transforms (§4.2 eq. (38)) and mode eigenvalues
(eq. (39))."""
import numpy as np
import pytest
import scipy.fft as sfft

from tests import _assembly


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 64])
def test_fft_matches_dft_definition(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    j = np.arange(n)
    dft = np.exp(-2j * np.pi * np.outer(j, j) / n) @ x
    assert np.abs(orc.fft(x) - dft).max() <= 1e-13 * max(1.0, np.abs(dft).max())


def test_fft_matches_numpy_large(orc):
    x = np.random.default_rng(0).standard_normal(4096)
    ref = np.fft.fft(x)
    assert np.abs(orc.fft(x) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n", [2, 8, 64, 256, 2048])
def test_ztrans_matches_scipy(orc, n):
    x = np.random.default_rng(n).standard_normal((3, n))
    for bc, kind in ((0, "dst"), (1, "dct")):
        fn = getattr(sfft, kind)
        assert np.abs(orc.ztrans_fwd(x, bc) - fn(x, 2, norm="ortho", axis=-1)).max() < 1e-13
        assert np.abs(orc.ztrans_inv(x, bc) - fn(x, 3, norm="ortho", axis=-1)).max() < 1e-13


@pytest.mark.parametrize("bc", [0, 1])
def test_ztrans_orthonormal(orc, bc):
    x = np.random.default_rng(1).standard_normal((4, 128))
    X = orc.ztrans_fwd(x, bc)
    assert np.allclose(np.linalg.norm(X, axis=1), np.linalg.norm(x, axis=1), rtol=1e-14)
    assert np.abs(orc.ztrans_inv(X, bc) - x).max() < 1e-13


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("nz", [4, 16, 33 - 1])
def test_basis_diagonalises_the_z_operator(orc, bc, nz):
    """The inverse transform of a unit mode vector is an eigenvector of the
    scheme's z-part with eigenvalue r * kappa * mu_j (eq. (39)).  The operator
    is assembled independently with one r-cell: A = r0 * Lz + 2 C_r I."""
    lz = 0.8
    kr = np.ones((1, nz))
    kz = np.ones((1, nz + 1))
    q = np.zeros((1, nz))
    A = _assembly.assemble(kr, kz, q, 1.0, lz, bc).toarray()
    mu = orc.mode_eig(nz, lz, bc)
    r0, cr0 = 0.5, 1.0  # r_0 = h/2, rho_{1/2} kappa / h^2 with h = 1
    for j in range(nz):
        e = np.zeros(nz)
        e[j] = 1.0
        phi = orc.ztrans_inv(e, bc)
        lam = r0 * mu[j] + 2.0 * cr0
        assert np.abs(A @ phi - lam * phi).max() <= 1e-12 * lam
