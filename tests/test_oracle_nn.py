"""Pins of the learned-guess oracle (oracle/nn.py) against things other than itself.

* bfloat16 rounding against torch's own float32 -> bfloat16 conversion;
* the FP64 network against torch.nn.functional.conv2d, and the gradients of
  its energy-norm loss (matrix from the independent assembly in _assembly.py)
  against torch autograd and against central finite differences;
* Adam against torch.optim.Adam;
* the guard's pick against the error seen through A from a direct solve;
* special cases: a zero last layer returns the extrapolation exactly; the rounded
  network stays within bfloat16's error of the FP64 one; every stored
  activation is a bfloat16 value.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from oracle import nn as onn
from synth import nn_example
from tests._assembly import assemble


def _matrix(ex):
    """Scheme matrix for the example's kappa (independent assembly), q = 1."""
    kappa = ex["kappa"]
    nr, nz = kappa.shape
    kr = np.empty_like(kappa)
    kr[:-1] = 0.5 * (kappa[:-1] + kappa[1:])
    kr[-1] = kappa[-1]
    kz = np.empty((nr, nz + 1))
    kz[:, 1:-1] = 0.5 * (kappa[:, :-1] + kappa[:, 1:])
    kz[:, 0], kz[:, -1] = kappa[:, 0], kappa[:, -1]
    A = assemble(kr, kz, np.ones_like(kappa))
    return A, (lambda e: (A @ e.ravel()).reshape(e.shape))


def _torch_net(params):
    """The same network written with torch layers (FP64, CPU)."""
    layers = onn.unpack(params)
    ws = []
    for W, b in layers:
        # torch weight [co][ci][a][b] with t = 3 a + b
        w = torch.tensor(W.transpose(2, 1, 0).reshape(W.shape[2], W.shape[1], 3, 3), dtype=torch.float64)
        ws.append((w.clone().requires_grad_(True), torch.tensor(b, dtype=torch.float64).requires_grad_(True)))
    return ws


def _torch_forward(ws, x):
    h = torch.tensor(np.moveaxis(x, -1, 0)[None], dtype=torch.float64)
    for l, (w, b) in enumerate(ws):
        h = torch.nn.functional.conv2d(h, w, b, padding=1)
        if l < len(ws) - 1:
            h = torch.relu(h)
    return h[0, 0]


def _flat_grads(ws):
    parts = []
    for w, b in ws:
        g = w.grad.detach().numpy()            # [co][ci][3][3]
        parts.append(g.reshape(g.shape[0], g.shape[1], 9).transpose(2, 1, 0).ravel())
        parts.append(b.grad.detach().numpy())
    return np.concatenate(parts)


def test_param_count_matches_layout():
    assert onn.N_PARAMS == 38465
    assert onn.OFFSETS[1] == 9 * 4 * 32 + 32


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 1.0078125, 3.0e38, -7.5e-39]])
    # ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7 and must round to the even 1
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = onn.bf16_round(x)
    np.testing.assert_array_equal(got, ref)
    assert onn.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0


def test_forward_fp64_matches_torch_conv2d():
    ex = nn_example(12, 20, seed=5)
    params = onn.init_params(7, last_zero=False)
    guess, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    x, s = onn.inputs(ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    ws = _torch_net(params)
    out = _torch_forward(ws, x).detach().numpy()
    np.testing.assert_allclose(cache["out"], out, rtol=1e-12, atol=1e-12 * np.abs(out).max())
    np.testing.assert_allclose(guess, 2 * ex["u1"] - ex["u2"] + s * out, rtol=1e-12, atol=1e-14)


def test_backward_fp64_matches_torch_autograd():
    ex = nn_example(10, 16, seed=6)
    A, apply_A = _matrix(ex)
    params = onn.init_params(8, last_zero=False)
    _, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    loss, grads = onn.backward(params, cache, apply_A, ex["ut"])
    x, s = onn.inputs(ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    ws = _torch_net(params)
    out = _torch_forward(ws, x)
    guess = torch.tensor(2 * ex["u1"] - ex["u2"]) + s * out
    e = (guess - torch.tensor(ex["ut"])).reshape(-1)
    tA = torch.tensor(A.toarray())
    tl = (e @ (tA @ e)) / (s * s * e.numel())
    tl.backward()
    assert loss == pytest.approx(tl.item(), rel=1e-12)
    ref = _flat_grads(ws)
    np.testing.assert_allclose(grads, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_backward_fp64_finite_differences():
    ex = nn_example(8, 12, seed=9)
    _, apply_A = _matrix(ex)
    params = onn.init_params(10, last_zero=False).astype(np.float64)
    _, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    _, grads = onn.backward(params, cache, apply_A, ex["ut"])

    def loss_at(p):
        _, c = onn.forward(p, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
        return onn.backward(p, c, apply_A, ex["ut"])[0]

    rng = np.random.default_rng(0)
    idx = list(rng.choice(onn.N_PARAMS, 24, replace=False))
    idx += [onn.OFFSETS[l] + 9 * onn.CIN[l] * onn.COUT[l] for l in range(onn.N_LAYERS)]   # one bias per layer
    h = 1e-6
    for e in idx:
        pp, pm = params.copy(), params.copy()
        pp[e] += h
        pm[e] -= h
        fd = (loss_at(pp) - loss_at(pm)) / (2 * h)
        assert fd == pytest.approx(grads[e], rel=1e-5, abs=1e-9 * np.abs(grads).max()), e


def test_guard_picks_smallest_residual():
    ex = nn_example(12, 16, seed=17)
    A, apply_A = _matrix(ex)
    ustar = spla.spsolve(A.tocsc(), ex["b"].ravel()).reshape(ex["b"].shape)
    rng = np.random.default_rng(4)
    for trial in range(6):
        u1 = ustar + rng.standard_normal(ustar.shape) * 10.0 ** rng.uniform(-3, 0)
        u2 = ustar + rng.standard_normal(ustar.shape) * 10.0 ** rng.uniform(-3, 0)
        guess = ustar + rng.standard_normal(ustar.shape) * 10.0 ** rng.uniform(-3, 0)
        res, pick = onn.guard(ex["b"], u1, u2, guess, apply_A)
        # A (x - u*) = A x - b: the residual is the error seen through A
        cands = [u1, 2 * u1 - u2, guess]
        ref = [np.linalg.norm(A @ (x - ustar).ravel()) for x in cands]
        assert pick == int(np.argmin(ref))
        np.testing.assert_allclose((res[2], res[1], res[0]), ref, rtol=1e-8)
    # ties keep the simpler candidate
    res, pick = onn.guard(ex["b"], ustar, ustar, ustar, apply_A)
    assert pick == 0


def test_extrapolation_is_exact_for_polynomial_sequences():
    """Order p reproduces the next value of any sequence that is a polynomial
    of degree <= p in the harmonic index, and misses one of degree p + 1 by
    the (p+1)-th difference (the first dropped term of Newton's form)."""
    rng = np.random.default_rng(9)
    shape = (5, 7)
    for deg in range(5):
        coef = [rng.standard_normal(shape) for _ in range(deg + 1)]
        seq = lambda t: sum(c * float(t) ** d for d, c in enumerate(coef))  # noqa: E731
        m = 11
        hist = [seq(m - 1 - i) for i in range(5)]
        for p in range(5):
            x = onn.extrapolate(hist, p)
            if p >= deg:
                np.testing.assert_allclose(x, seq(m), rtol=1e-9, atol=1e-9 * np.abs(seq(m)).max())
            elif p == deg - 1:
                # error = leading coefficient * deg! (the deg-th difference of t^deg)
                err = seq(m) - x
                np.testing.assert_allclose(err, coef[deg] * math.factorial(deg), rtol=1e-8, atol=1e-8)
    assert np.array_equal(onn.extrapolate([np.ones(3), 5 * np.ones(3)], 1), -3 * np.ones(3))


def test_guard_poly_ranks_by_residual():
    ex = nn_example(12, 16, seed=19)
    A, apply_A = _matrix(ex)
    ustar = spla.spsolve(A.tocsc(), ex["b"].ravel()).reshape(ex["b"].shape)
    rng = np.random.default_rng(5)
    # u_{m-1-i} = u* + a cubic in (i + 1) + small noise: orders 0..2 miss the
    # cubic, order 3 only sees the noise, order 4 amplifies it more
    w = [rng.standard_normal(ustar.shape) * 0.1 for _ in range(3)]
    hist = [ustar + sum(wd * float(i + 1) ** (d + 1) for d, wd in enumerate(w))
            + 1e-5 * rng.standard_normal(ustar.shape) for i in range(5)]
    res, pick, cands = onn.guard_poly(ex["b"], hist, apply_A)
    ref = [np.linalg.norm(A @ (x - ustar).ravel()) for x in cands]
    np.testing.assert_allclose(res, ref, rtol=1e-8)
    assert pick == 3 == int(np.argmin(ref))
    # a network candidate is ranked last and wins only when strictly smaller
    res, pick, _ = onn.guard_poly(ex["b"], hist, apply_A, net_guess=ustar)
    assert pick == 5 and res[5] < 1e-8 * res[0]
    res, pick, _ = onn.guard_poly(ex["b"], [ustar] * 3, apply_A, net_guess=ustar)
    assert pick == 0


def _history(ex, n, seed):
    """u_{m-1} = ex's u1, u_{m-2} = u2 and n - 2 more smooth fields."""
    rng = np.random.default_rng(seed)
    more = [ex["u1"] + 0.3 * rng.standard_normal(ex["u1"].shape) for _ in range(n - 2)]
    return [ex["u1"], ex["u2"]] + more


def _fit_extrapolation(hist, p):
    """The value at t = 0 of the degree-p least-squares polynomial through
    (t, hist[i]) at t = -1 - i, i <= p (an interpolant: p + 1 points), by
    numpy's polynomial fit; independent of the oracle's Lagrange weights."""
    t = -1.0 - np.arange(p + 1)
    ys = np.stack([np.asarray(hist[i]).ravel() for i in range(p + 1)])
    c = np.polynomial.polynomial.polyfit(t, ys, p)
    return c[0].reshape(np.shape(hist[0]))


@pytest.mark.parametrize("order", [2, 4, 6])
def test_forward_base_order_matches_torch(order):
    """Order-P base: the guess is the network's (torch) output times s plus
    the degree-P polynomial through the last P + 1 harmonics at harmonic m."""
    ex = nn_example(12, 20, seed=21)
    hist = _history(ex, 7, order)
    params = onn.init_params(7, last_zero=False)
    guess, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False, hist=hist,
                               order=order)
    x, s = onn.inputs(ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    out = _torch_forward(_torch_net(params), x).detach().numpy()
    ref = _fit_extrapolation(hist, order) + s * out
    np.testing.assert_allclose(guess, ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


def test_backward_base_order_matches_torch_autograd():
    ex = nn_example(10, 16, seed=22)
    A, apply_A = _matrix(ex)
    hist = _history(ex, 5, 3)
    params = onn.init_params(8, last_zero=False)
    _, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False, hist=hist, order=4)
    loss, grads = onn.backward(params, cache, apply_A, ex["ut"])
    x, s = onn.inputs(ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    ws = _torch_net(params)
    guess = torch.tensor(_fit_extrapolation(hist, 4)) + s * _torch_forward(ws, x)
    e = (guess - torch.tensor(ex["ut"])).reshape(-1)
    tl = (e @ (torch.tensor(A.toarray()) @ e)) / (s * s * e.numel())
    tl.backward()
    assert loss == pytest.approx(tl.item(), rel=1e-9)
    ref = _flat_grads(ws)
    np.testing.assert_allclose(grads, ref, rtol=1e-7, atol=1e-10 * np.abs(ref).max())


def test_base_order_needs_history():
    ex = nn_example(4, 8, seed=23)
    params = onn.init_params(1)
    with pytest.raises(ValueError):
        onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], order=2)
    with pytest.raises(ValueError):
        onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], hist=_history(ex, 3, 0), order=3)


def test_zero_last_layer_returns_extrapolation():
    ex = nn_example(9, 14, seed=11)
    params = onn.init_params(12, last_zero=True)
    for bf in (False, True):
        guess, _ = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=bf)
        np.testing.assert_array_equal(guess, 2 * ex["u1"] - ex["u2"])
        hist = _history(ex, 7, 4)
        for p in range(1, 7):
            guess, _ = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=bf, hist=hist, order=p)
            np.testing.assert_array_equal(guess, onn.extrapolate(hist, p))


def test_rounded_network_close_to_fp64_and_on_bf16_grid():
    ex = nn_example(16, 24, seed=13)
    params = onn.init_params(14, last_zero=False)
    g64, c64 = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    g16, c16 = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=True)
    rel = np.linalg.norm(c16["out"] - c64["out"]) / np.linalg.norm(c64["out"])
    # every rounding is within 2^-9 relative; six layers of it stay well under 5 %
    assert 1e-5 < rel < 5e-2
    for a in c16["acts"]:
        np.testing.assert_array_equal(onn.bf16_round(a), a)
    # The energy loss weighs the output's grid-scale rounding noise by A, so the
    # gradients agree to bfloat16 accuracy when the correction is small next to
    # the extrapolation error (the regime the guess works in).
    params[onn.OFFSETS[5]:onn.OFFSETS[5] + 9 * 32] *= 0.01
    _, c64 = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    _, c16 = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=True)
    _, apply_A = _matrix(ex)
    l64, gr64 = onn.backward(params, c64, apply_A, ex["ut"])
    l16, gr16 = onn.backward(params, c16, apply_A, ex["ut"])
    assert l16 == pytest.approx(l64, rel=1e-3)
    assert np.linalg.norm(gr16 - gr64) / np.linalg.norm(gr64) < 5e-2


def test_adam_matches_torch():
    rng = np.random.default_rng(21)
    p0 = rng.standard_normal(50)
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m1, m2 = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        tp.grad = torch.tensor(g)
        opt.step()
        p, m1, m2 = onn.adam(p, g, m1, m2, step, 1e-2)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("bf16", [False, True])
def test_forward_at_equals_whole_grid_forward(bf16):
    """The windowed evaluation (six-cell receptive field, whole-grid scales,
    zero padding at the grid's edges only) gives the whole-grid output at
    every cell, corners and edges included."""
    ex = nn_example(19, 23, seed=31)
    params = onn.init_params(4, last_zero=False)
    params[onn.OFFSETS[5] + 9 * 32] = 0.25
    _, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=bf16)
    pts = [(i, k) for i in range(19) for k in range(23)]
    got = onn.forward_at(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], pts, bf16=bf16)
    want = cache["out"].ravel()
    if bf16:
        # FP64 sums of another length may round a hidden activation to the
        # neighbouring bfloat16 now and then
        assert np.linalg.norm(got - want) <= 1e-3 * np.linalg.norm(want)
    else:
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


# ---- the input normalisation (scales / inputs) -----------------------------------
# A hand-checked 2x2 case: u_{m-1} = 2 everywhere (RMS 2), u_{m-2} one 1 (RMS 1/2),
# b one 4 (RMS 2), kappa in {1, 2.5, 4}.  The channels are then u_{m-1}/2,
# u_{m-2}/2, b/2 and (kappa - 2.5)/1.5, all exact in bfloat16.
_U1 = np.full((2, 2), 2.0)
_U2 = np.array([[1.0, 0.0], [0.0, 0.0]])
_B = np.array([[0.0, 4.0], [0.0, 0.0]])
_K = np.array([[1.0, 2.5], [4.0, 1.0]])
_CH = np.array([[[1.0, 0.5, 0.0, -1.0], [1.0, 0.0, 2.0, 0.0]],
                [[1.0, 0.0, 0.0, 1.0], [1.0, 0.0, 0.0, -1.0]]])


def _normalisation_failures(inputs_fn, forward_fn):
    """Checks of the input normalisation that do not use its own formula:
    the hand-checked 2x2 channels, the zero-field fallbacks, and two exact
    invariances of the guess (scaling the earlier harmonics by 2^k scales
    the guess by 2^k; scaling b alone by 2^k leaves it unchanged).  Returns
    the names of the checks that fail."""
    bad = []
    for bf in (False, True):
        x, s = inputs_fn(_U1, _U2, _B, _K, bf16=bf)
        if s != 2.0 or not np.array_equal(x, _CH):
            bad.append(f"hand_2x2_bf16={bf}")
    x, s = inputs_fn(np.zeros((2, 2)), _U2, np.zeros((2, 2)), _K, bf16=False)
    if s != 1.0 or not np.array_equal(x[..., 1], _U2) or np.any(x[..., 2] != 0.0):
        bad.append("zero_fields")
    ex = nn_example(10, 14, seed=23)
    params = onn.init_params(6, last_zero=False)
    g0, _ = forward_fn(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=True)
    for c in (0.25, 8.0):
        gu, _ = forward_fn(params, c * ex["u1"], c * ex["u2"], ex["b"], ex["kappa"], bf16=True)
        if not np.array_equal(gu, c * g0):
            bad.append(f"scale_u_{c}")
        gb, _ = forward_fn(params, ex["u1"], ex["u2"], c * ex["b"], ex["kappa"], bf16=True)
        if not np.array_equal(gb, g0):
            bad.append(f"scale_b_{c}")
    return bad


def test_input_normalisation_pinned():
    assert _normalisation_failures(onn.inputs, onn.forward) == []


def _mutant_forward(mutant_inputs):
    """onn.forward with its input normalisation replaced (the rest unchanged)."""
    def fwd(params, u1, u2, b, kappa, bf16=True):
        saved = onn.inputs
        onn.inputs = mutant_inputs
        try:
            return onn.forward(params, u1, u2, b, kappa, bf16=bf16)
        finally:
            onn.inputs = saved
    return fwd


def _mutant(kind):
    def inputs(u1, u2, b, kappa, bf16=True, sc=None):
        rnd = onn.bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
        u1, u2, b, kappa = (np.asarray(a, dtype=np.float64) for a in (u1, u2, b, kappa))
        s, sb = onn.scales(u1, b)
        if kind == "b_over_s":
            sb = s
        elif kind == "s_from_u2":
            s = float(np.sqrt(np.mean(u2 * u2))) or 1.0
        elif kind == "kappa_shift":
            kappa = kappa + 1.5
        x = np.stack([u1 / s, u2 / s, b / sb, (kappa - 2.5) / 1.5], axis=-1)
        return rnd(x), s
    return inputs


@pytest.mark.parametrize("kind", ["b_over_s", "s_from_u2", "kappa_shift"])
def test_planted_normalisation_mistakes_are_caught(kind):
    """Each plausible misreading of the normalisation, planted in a copy of
    the oracle's input step, fails the pins above."""
    m = _mutant(kind)
    assert _normalisation_failures(m, _mutant_forward(m)) != []
