"""Pins of the oracle's operator (§2.1 eqs. (4)-(6); §2.2 eq. (7): A = A^* > 0)."""
import numpy as np
import pytest

from tests import _assembly


def _rand_faces(rng, nr, nz):
    kr = rng.uniform(0.5, 3.0, (nr, nz))
    kz = rng.uniform(0.5, 3.0, (nr, nz + 1))
    q = rng.uniform(0.0, 2.0, (nr, nz))
    return kr, kz, q


@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("shape", [(5, 7), (8, 8), (16, 12)])
def test_apply_matches_energy_assembly(orc, bc, shape):
    rng = np.random.default_rng(3)
    nr, nz = shape
    kr, kz, q = _rand_faces(rng, nr, nz)
    op = orc.operator_from_faces(kr, kz, q, 1.3, 0.7, bc)
    A = _assembly.assemble(kr, kz, q, 1.3, 0.7, bc)
    for _ in range(3):
        x = rng.standard_normal((nr, nz))
        y = orc.apply(op, x)
        yref = (A @ x.ravel()).reshape(nr, nz)
        assert np.linalg.norm(y - yref) <= 1e-13 * np.linalg.norm(yref)


@pytest.mark.parametrize("bc", [0, 1])
def test_dense_symmetric_bitwise_and_spd(orc, bc):
    rng = np.random.default_rng(4)
    nr, nz = 9, 11
    kr, kz, q = _rand_faces(rng, nr, nz)
    q[:] = 0.0  # SPD must come from the Dirichlet face at r = l_r alone
    op = orc.operator_from_faces(kr, kz, q, 1.0, 1.0, bc)
    n = nr * nz
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = orc.apply(op, e.reshape(nr, nz)).ravel()
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0.0


@pytest.mark.parametrize("bc", [0, 1])
def test_energy_identity(orc, bc):
    rng = np.random.default_rng(5)
    nr, nz = 12, 10
    kr, kz, q = _rand_faces(rng, nr, nz)
    op = orc.operator_from_faces(kr, kz, q, 1.0, 2.0, bc)
    y = rng.standard_normal((nr, nz))
    e = _assembly.energy(kr, kz, q, y, 1.0, 2.0, bc)
    assert abs(np.sum(y * orc.apply(op, y)) - e) <= 1e-12 * e


def test_face_kappa_exact_for_linear_fields(orc):
    """Interpolating cell values to the face points (eq. (6) samples kappa at
    the faces) is exact for kappa linear in r and z; boundary faces take the
    adjacent cell's value."""
    nr, nz = 6, 5
    hr, hz = 1.0 / nr, 1.0 / nz
    r = (np.arange(nr) + 0.5) * hr
    z = (np.arange(nz) + 0.5) * hz
    kc = 2.0 + 0.3 * r[:, None] + 0.7 * z[None, :]
    kr, kz = orc.face_kappa(kc)
    rho = (np.arange(nr) + 1) * hr
    expect_r = 2.0 + 0.3 * rho[:, None] + 0.7 * z[None, :]
    assert np.allclose(kr[:-1], expect_r[:-1], rtol=0, atol=1e-14)
    assert np.allclose(kr[-1], kc[-1], rtol=0, atol=0)
    zf = np.arange(nz + 1) * hz
    expect_z = 2.0 + 0.3 * r[:, None] + 0.7 * zf[None, :]
    assert np.allclose(kz[:, 1:-1], expect_z[:, 1:-1], rtol=0, atol=1e-14)
    assert np.array_equal(kz[:, 0], kc[:, 0]) and np.array_equal(kz[:, -1], kc[:, -1])


def test_rhs_is_r_weighted(orc):
    """phi = r f (eq. (6)): the midpoint sum of phi over the cells equals the
    exact integral of r f dr dz for f linear in z."""
    nr, nz = 8, 4
    op = orc.operator_from_cells(np.ones((nr, nz)), np.zeros((nr, nz)))
    z = (np.arange(nz) + 0.5) / nz
    f = np.broadcast_to(1.0 + z[None, :], (nr, nz))
    b = orc.rhs(op, f)
    integral = 0.5 * 1.5  # int_0^1 r dr * int_0^1 (1+z) dz
    assert abs(b.sum() * op.hr * op.hz - integral) < 1e-14
