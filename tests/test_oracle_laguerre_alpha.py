"""Pins of the oracle's generalized Laguerre transform (§4.1 eqs. (34)-(35)
with integer alpha, the paper's experiment uses alpha = 5, h = 300).

* the projection kernel against scipy's generalized Laguerre polynomials and
  log-gamma normalisation;
* biorthogonality of the synthesis and projection functions;
* the recursion with alpha against the Laguerre transform of an ODE solution
  (the 0-D reduction of eq. (35));
* synthesis from the coefficients reproduces the pulse of eq. (40);
* alpha = 0 reduces to the functions of the alpha = 0 transform.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.special import eval_genlaguerre, gammaln

import synth


def test_psi_matches_library_polynomials(orc):
    eta, alpha = 300.0, 5
    t = np.linspace(0.0, 0.8, 161)
    P = orc.laguerre_psi(220, alpha, eta, t)
    for m in (0, 1, 2, 17, 120, 219):
        nrm = np.exp(0.5 * (np.log(eta) + gammaln(m + 1) - gammaln(m + alpha + 1)))
        ref = nrm * np.exp(-eta * t / 2) * eval_genlaguerre(m, alpha, eta * t)
        assert np.abs(P[m] - ref).max() <= 1e-9 * max(1e-300, np.abs(ref).max()), m


def test_alpha_zero_reduces_to_the_plain_functions(orc):
    t = np.linspace(0.0, 2.0, 101)
    np.testing.assert_allclose(orc.laguerre_psi(30, 0, 10.0, t), orc.laguerre_functions(30, 10.0, t),
                               rtol=1e-12, atol=1e-14)


def test_synthesis_and_projection_are_biorthogonal(orc):
    """int phi_m psi_n dt = delta_mn on [0, inf) (Simpson on a fine grid)."""
    eta, alpha, n = 300.0, 5, 40
    t = np.linspace(0.0, 1.0, 200001)     # the functions have decayed below 1e-20 by eta t = 300
    P = orc.laguerre_psi(n, alpha, eta, t)
    F = orc.laguerre_synthesis(n, alpha, eta, t)
    w = np.full(t.size, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    w *= (t[1] - t[0]) / 3.0
    G = (F * w) @ P.T
    assert np.abs(G - np.eye(n)).max() < 1e-9


@pytest.mark.parametrize("alpha", [2, 5])
def test_recursion_with_alpha_solves_zero_dimensional_wave_equation(orc, alpha):
    """0-D reduction of eq. (35): the space operator becomes -omega^2, so
        Q_m = (f_m - eta^2 c_m sum_{k<m} (m-k) d_k Q_k) / (omega^2 + eta^2/4),
    c_m = sqrt(m!/(m+alpha)!), d_k = sqrt((k+alpha)!/k!), must equal the
    projection onto psi_m of the solution of u'' = -omega^2 u + f(t),
    u(0) = u'(0) = 0 (eqs. (30)-(31)), computed by an ODE integrator."""
    eta, n, omega = 60.0, 50, 25.0
    f0, t0, T = 5.0, 0.3, 0.6
    t, ft = synth.ricker_pulse_samples(nt=30001, t_max=T, f0=f0, t0=t0)
    g = orc.laguerre_coeffs_a(n, alpha, eta, ft, T)
    c, d = orc.laguerre_weights(n, alpha)
    Q = np.zeros(n)
    for m in range(n):
        s = sum((m - k) * d[k] * Q[k] for k in range(m))
        Q[m] = (g[m] - eta**2 * c[m] * s) / (omega**2 + eta**2 / 4)

    def src(s):
        a = (np.pi * f0 * (s - t0)) ** 2
        return (1 - 2 * a) * np.exp(-a) if s <= T else 0.0

    TL = 4.0
    tt = np.linspace(0.0, TL, 200001)
    sol = solve_ivp(lambda s, y: [y[1], -omega**2 * y[0] + src(s)], [0, TL], [0.0, 0.0],
                    t_eval=tt, rtol=1e-12, atol=1e-15, max_step=5e-4, method="DOP853")
    P = orc.laguerre_psi(n, alpha, eta, tt)
    w = np.full(tt.size, tt[1] - tt[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    Qd = P @ (sol.y[0] * w)
    # agreement to the quadrature and integrator accuracy (measured 2e-5 for
    # alpha = 2, the transform identity itself holds to 1e-11)
    assert np.abs(Q - Qd).max() < 2e-4 * np.abs(Qd).max()
    # dropping the weights (the alpha = 0 recursion) is caught
    Qw = np.zeros(n)
    for m in range(n):
        s = sum((m - k) * Qw[k] for k in range(m))
        Qw[m] = (g[m] - eta**2 * s) / (omega**2 + eta**2 / 4)
    assert np.abs(Qw - Qd).max() > 1e-1 * np.abs(Qd).max()


def test_pulse_is_reproduced_by_its_series(orc):
    """f(t) = sum_m f_m phi_m(t) for the pulse of eq. (40) with the paper's
    alpha = 5, h = 300, once enough terms are kept."""
    t, ft = synth.gauss_sine_pulse_samples(nt=8001)
    g = orc.laguerre_coeffs_a(400, 5, 300.0, ft, t[-1])
    ts = t[::40]
    F = orc.laguerre_synthesis(400, 5, 300.0, ts)
    rec = g @ F
    err = np.abs(rec - ft[::40]).max()
    assert err < 1e-6 * np.abs(ft).max()


@pytest.mark.parametrize("alpha", [0, 2, 5])
def test_transform_of_second_derivative(orc, alpha):
    """The identity behind eq. (35): for u(0) = u'(0) = 0,
        int u'' psi_m dt = (eta^2/4) Q_m + eta^2 c_m sum_{k<m} (m-k) d_k Q_k,
    checked for u = Im(t^3 e^{s t}), s = -3 + 7i, whose u'' is written out."""
    eta, n = 60.0, 30
    t = np.linspace(0.0, 8.0, 400001)
    w = np.full(t.size, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    w *= (t[1] - t[0]) / 3.0
    s = -3.0 + 7.0j
    u = np.imag(t**3 * np.exp(s * t))
    upp = np.imag((6 * t + 6 * s * t**2 + s * s * t**3) * np.exp(s * t))
    P = orc.laguerre_psi(n, alpha, eta, t)
    Q, R = P @ (u * w), P @ (upp * w)
    c, d = orc.laguerre_weights(n, alpha)
    rhs = np.array([eta**2 / 4 * Q[m] + eta**2 * c[m] * sum((m - k) * d[k] * Q[k] for k in range(m))
                    for m in range(n)])
    assert np.abs(R - rhs).max() < 1e-9 * np.abs(R).max()
