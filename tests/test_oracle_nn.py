"""Pins of the learned-guess oracle (oracle/nn.py) against things other than itself.

* bfloat16 rounding against torch's own float32 -> bfloat16 conversion;
* the FP64 network against torch.nn.functional.conv2d, and its gradients
  against torch autograd and against central finite differences;
* Adam against torch.optim.Adam;
* special cases: a zero last layer returns u_{m-1} exactly; the rounded
  network stays within bfloat16's error of the FP64 one; every stored
  activation is a bfloat16 value.
"""
import numpy as np
import pytest
import torch

from oracle import nn as onn
from synth import nn_example


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
    np.testing.assert_allclose(guess, ex["u1"] + s * out, rtol=1e-12, atol=1e-14)


def test_backward_fp64_matches_torch_autograd():
    ex = nn_example(10, 16, seed=6)
    params = onn.init_params(8, last_zero=False)
    _, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    loss, grads = onn.backward(params, cache, ex["u1"], ex["ut"])
    x, s = onn.inputs(ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    ws = _torch_net(params)
    out = _torch_forward(ws, x)
    target = torch.tensor((ex["ut"] - ex["u1"]) / s)
    tl = torch.mean((out - target) ** 2)
    tl.backward()
    assert loss == pytest.approx(tl.item(), rel=1e-12)
    ref = _flat_grads(ws)
    np.testing.assert_allclose(grads, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


def test_backward_fp64_finite_differences():
    ex = nn_example(8, 12, seed=9)
    params = onn.init_params(10, last_zero=False).astype(np.float64)
    _, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
    _, grads = onn.backward(params, cache, ex["u1"], ex["ut"])

    def loss_at(p):
        _, c = onn.forward(p, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=False)
        return onn.backward(p, c, ex["u1"], ex["ut"])[0]

    rng = np.random.default_rng(0)
    idx = list(rng.choice(onn.N_PARAMS, 24, replace=False))
    idx += [onn.OFFSETS[l] + 9 * onn.CIN[l] * onn.COUT[l] for l in range(onn.N_LAYERS)]   # one bias per layer
    h = 1e-6
    for e in idx:
        pp, pm = params.copy(), params.copy()
        pp[e] += h
        pm[e] -= h
        fd = (loss_at(pp) - loss_at(pm)) / (2 * h)
        assert fd == pytest.approx(grads[e], rel=1e-5, abs=1e-9), e


def test_zero_last_layer_returns_previous_harmonic():
    ex = nn_example(9, 14, seed=11)
    params = onn.init_params(12, last_zero=True)
    for bf in (False, True):
        guess, _ = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=bf)
        np.testing.assert_array_equal(guess, ex["u1"])


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
    l64, gr64 = onn.backward(params, c64, ex["u1"], ex["ut"])
    l16, gr16 = onn.backward(params, c16, ex["u1"], ex["ut"])
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
