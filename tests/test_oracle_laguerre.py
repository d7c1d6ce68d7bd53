"""Pins of the oracle's Laguerre machinery (§4.1 eqs. (34)-(35), alpha = 0)."""
import numpy as np
import pytest
from scipy.integrate import simpson, solve_ivp
from scipy.special import eval_laguerre

import synth


def test_laguerre_functions_match_library_polynomials(orc):
    eta = 10.0
    t = np.linspace(0.0, 3.0, 301)
    L = orc.laguerre_functions(40, eta, t)
    for m in (0, 1, 7, 39):
        ref = np.sqrt(eta) * np.exp(-eta * t / 2) * eval_laguerre(m, eta * t)
        assert np.abs(L[m] - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_laguerre_functions_orthonormal(orc):
    """l_m(t) = sqrt(eta) e^{-eta t/2} L_m(eta t) are orthonormal on [0, inf)."""
    eta, n = 10.0, 40
    t = np.linspace(0.0, 40.0, 400001)
    L = orc.laguerre_functions(n, eta, t)
    w = np.full(t.size, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    w *= (t[1] - t[0]) / 3.0          # composite Simpson weights
    G = (L * w) @ L.T
    assert abs(G[3, 5] - simpson(L[3] * L[5], x=t)) < 1e-13
    assert np.abs(G - np.eye(n)).max() < 1e-8


def test_coefficients_are_projections(orc):
    """g_m from the Simpson rule on [0, T] equals the projection of f onto l_m
    computed by a library quadrature (trapezoid on a 4x finer grid)."""
    eta, n = 10.0, 50
    t, ft = synth.ricker_pulse_samples()
    g = orc.laguerre_coeffs(n, eta, ft, t[-1])
    tf, ff = synth.ricker_pulse_samples(nt=4 * (len(t) - 1) + 1)
    L = orc.laguerre_functions(n, eta, tf)
    ref = np.trapezoid(L * ff, tf, axis=1)
    assert np.abs(g - ref).max() < 1e-9 * np.abs(ref).max()


def test_parseval_converges(orc):
    """sum g_m^2 -> int f^2 as the number of terms grows (completeness)."""
    t, ft = synth.ricker_pulse_samples(nt=20001, t_max=0.6, f0=5.0, t0=0.3)
    norm2 = np.trapezoid(ft * ft, t)
    eta = 50.0
    g = orc.laguerre_coeffs(800, eta, ft, t[-1])
    s = np.cumsum(g * g)
    assert s[-1] <= norm2 * (1 + 1e-9)
    assert abs(s[-1] - norm2) < 1e-3 * norm2
    assert abs(s[-1] - norm2) < abs(s[99] - norm2)


@pytest.mark.parametrize("omega", [8.0, 20.0])
def test_recursion_solves_zero_dimensional_wave_equation(orc, omega):
    """0-D reduction of eq. (35): the space operator becomes -omega^2, so
    Q_m = (g_m - eta^2 sum_{k<m} (m-k) Q_k) / (omega^2 + eta^2/4) must equal the
    Laguerre transform of the solution of u'' = -omega^2 u + f(t), u(0) =
    u'(0) = 0 (eqs. (30)-(31)), computed by an ODE integrator."""
    eta, n = 50.0, 60
    f0, t0, T = 5.0, 0.3, 0.6
    t, ft = synth.ricker_pulse_samples(nt=30001, t_max=T, f0=f0, t0=t0)
    g = orc.laguerre_coeffs(n, eta, ft, T)
    Q = np.zeros(n)
    for m in range(n):
        s = sum((m - k) * Q[k] for k in range(m))
        Q[m] = (g[m] - eta**2 * s) / (omega**2 + eta**2 / 4)

    def src(s):
        a = (np.pi * f0 * (s - t0)) ** 2
        return (1 - 2 * a) * np.exp(-a) if s <= T else 0.0

    TL = 16.0
    tt = np.linspace(0.0, TL, 320001)
    sol = solve_ivp(lambda s, y: [y[1], -omega**2 * y[0] + src(s)], [0, TL], [0.0, 0.0],
                    t_eval=tt, rtol=1e-12, atol=1e-15, max_step=5e-4, method="DOP853")
    L = orc.laguerre_functions(n, eta, tt)
    w = np.full(tt.size, tt[1] - tt[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    Qd = L @ (sol.y[0] * w)
    assert np.abs(Q - Qd).max() < 1e-7 * np.abs(Qd).max()
