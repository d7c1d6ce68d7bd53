"""CPU oracle of the learned initial guess (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU leg of ``bench.py``
may import this module; the product path never does.

The paper solves the Laguerre harmonics one after another (§4.1, eqs.
(34)-(35)) and starts each PCG run from zero; it has no learned component.
The network here is an extension whose definition is fixed by the library's
header rather than by the paper:

* inputs per cell, with s = RMS(u_{m-1}) and s_b = RMS(b_m) (1 when zero):
  u_{m-1}/s, u_{m-2}/s, b_m/s_b, (kappa - 2.5)/1.5;
* six 3x3 convolutions with zero "same" padding, 4 -> 32 -> ... -> 32 -> 1
  channels, ReLU after every layer but the last;
* guess = x_P + s * out: the network corrects the polynomial extrapolation
  in m of order P (``extrapolate``; P = 1, the default, is the linear
  2 u_{m-1} - u_{m-2}; a larger P reads u_{m-1}, ..., u_{m-1-P});
* loss: the energy norm of the guess error, L = e^T A e / (s^2 P) with
  e = guess - u_target, A the scheme's matrix and P the number of cells;
  Adam on the parameters;
* guard: of u_{m-1}, the extrapolation and the guess, the one with the
  smallest residual |b - A x|, a later candidate only when strictly smaller.

Parameters are a flat float32 vector: per layer W[t][ci][co] with
t = 3 (di + 1) + (dk + 1) for the neighbour (i + di, k + dk), then bias[co].

``bf16=True`` reproduces where the GPU library rounds to bfloat16 (inputs,
weights, hidden activations, the loss gradient seed and every hidden-layer
data gradient); the arithmetic between those points is FP64, so the oracle
is the exact value of the rounded network.  ``bf16=False`` is the same
network in plain FP64, which the CPU tests pin against torch's conv2d and
autograd and against finite differences.
"""
from __future__ import annotations

import numpy as np

N_LAYERS = 6
CIN = (4, 32, 32, 32, 32, 32)
COUT = (32, 32, 32, 32, 32, 1)


def layer_offsets():
    offs, o = [], 0
    for l in range(N_LAYERS):
        offs.append(o)
        o += 9 * CIN[l] * COUT[l] + COUT[l]
    return offs, o


OFFSETS, N_PARAMS = layer_offsets()


def unpack(params):
    """Split the flat vector into per-layer (W[9][cin][cout], bias[cout]) in FP64."""
    p = np.asarray(params, dtype=np.float64)
    assert p.size == N_PARAMS
    out = []
    for l in range(N_LAYERS):
        o = OFFSETS[l]
        nw = 9 * CIN[l] * COUT[l]
        out.append((p[o:o + nw].reshape(9, CIN[l], COUT[l]), p[o + nw:o + nw + COUT[l]]))
    return out


def init_params(seed: int, last_zero: bool = True) -> np.ndarray:
    """He-normal weights, zero biases; a zero last layer makes the guess the extrapolation."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS, dtype=np.float32)
    for l in range(N_LAYERS):
        o = OFFSETS[l]
        nw = 9 * CIN[l] * COUT[l]
        if l == N_LAYERS - 1 and last_zero:
            continue
        p[o:o + nw] = rng.standard_normal(nw) * np.sqrt(2.0 / (9 * CIN[l]))
    return p


def bf16_round(x):
    """Round to bfloat16 (nearest, ties to even) through float32, as FP64 values."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = np.isfinite(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(finite, r, u & 0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(x):
    return np.asarray(x, dtype=np.float64)


def shift(x, di, dk):
    """y[i][k] = x[i + di][k + dk], zero outside the grid (x is [nr][nz][c])."""
    nr, nz = x.shape[:2]
    y = np.zeros_like(x)
    i0, i1 = max(0, -di), min(nr, nr - di)
    k0, k1 = max(0, -dk), min(nz, nz - dk)
    if i0 < i1 and k0 < k1:
        y[i0:i1, k0:k1] = x[i0 + di:i1 + di, k0 + dk:k1 + dk]
    return y


def taps():
    return [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def conv3(x, W, bias=None):
    """Same-padded 3x3 correlation: y[p][co] = sum_t sum_ci x[p + off_t][ci] W[t][ci][co] (+ bias)."""
    y = np.zeros(x.shape[:2] + (W.shape[2],))
    for t, (di, dk) in enumerate(taps()):
        y += shift(x, di, dk) @ W[t]
    if bias is not None:
        y += bias
    return y


def scales(u1, b):
    """s = RMS(u_{m-1}) and s_b = RMS(b_m) over the whole grid (1 when zero)."""
    u1, b = np.asarray(u1, dtype=np.float64), np.asarray(b, dtype=np.float64)
    s = float(np.sqrt(np.mean(u1 * u1)))
    sb = float(np.sqrt(np.mean(b * b)))
    return (s if s > 0 else 1.0), (sb if sb > 0 else 1.0)


def inputs(u1, u2, b, kappa, bf16=True, sc=None):
    """Normalised input channels and the scale s (``sc`` = (s, s_b) when the
    arrays are a window of a larger grid)."""
    rnd = bf16_round if bf16 else _ident
    u1, u2, b, kappa = (np.asarray(a, dtype=np.float64) for a in (u1, u2, b, kappa))
    s, sb = scales(u1, b) if sc is None else sc
    x = np.stack([u1 / s, u2 / s, b / sb, (kappa - 2.5) / 1.5], axis=-1)
    return rnd(x), s


def base(u1, u2, hist=None, order=1):
    """The extrapolation x_P the network corrects: ``extrapolate`` of order
    P = ``order`` through hist = (u_{m-1}, u_{m-2}, ...) (u1, u2 when hist is
    None, which allows P = 1 only)."""
    h = (u1, u2) if hist is None else hist
    if not 1 <= order < len(h):
        raise ValueError("the base order needs order + 1 history arrays")
    return extrapolate(h, order)


def forward(params, u1, u2, b, kappa, bf16=True, hist=None, order=1):
    """Return (guess, cache) where cache holds what backward needs.  The
    network reads u1 = u_{m-1} and u2 = u_{m-2} whatever the base order;
    ``hist`` (hist[0] = u1, hist[1] = u2) is needed for order > 1."""
    rnd = bf16_round if bf16 else _ident
    layers = unpack(params)
    x, s = inputs(u1, u2, b, kappa, bf16)
    acts = [x]
    for l, (W, bias) in enumerate(layers):
        y = conv3(acts[-1], rnd(W), bias)
        if l < N_LAYERS - 1:
            acts.append(rnd(np.maximum(y, 0.0)))
        else:
            out = y[..., 0]
    guess = base(u1, u2, hist, order) + s * out
    return guess, {"acts": acts, "out": out, "s": s, "bf16": bf16, "guess": guess}


def forward_at(params, u1, u2, b, kappa, points, bf16=True):
    """The network output ``out`` at the cells ``points`` ((i, k) pairs) of a
    grid too large to evaluate whole.  The output of a cell depends only on
    the inputs within six cells in each direction (six 3x3 layers), so each
    point is evaluated on that window: its normalisation uses the scales of
    the whole grid, and zero padding falls at the grid's edges where the
    window meets them.  Values at the window's inner border are wrong after a
    layer, but they never reach the centre in the layers that remain."""
    rnd = bf16_round if bf16 else _ident
    layers = unpack(params)
    sc = scales(u1, b)
    nr, nz = np.shape(u1)
    out = np.empty(len(points))
    for j, (i, k) in enumerate(points):
        i0, i1 = max(0, i - N_LAYERS), min(nr, i + N_LAYERS + 1)
        k0, k1 = max(0, k - N_LAYERS), min(nz, k + N_LAYERS + 1)
        win = tuple(np.asarray(a)[i0:i1, k0:k1] for a in (u1, u2, b, kappa))
        x, _ = inputs(*win, bf16=bf16, sc=sc)
        for l, (W, bias) in enumerate(layers):
            y = conv3(x, rnd(W), bias)
            x = rnd(np.maximum(y, 0.0)) if l < N_LAYERS - 1 else y
        out[j] = x[i - i0, k - k0, 0]
    return out


def backward(params, cache, apply_A, u_target):
    """Energy-norm loss and its gradient w.r.t. the flat parameter vector.

    ``apply_A`` maps a [nr][nz] array to A times it (A symmetric), so that
    dL/d(out) = 2 s A e / (s^2 P)."""
    rnd = bf16_round if cache["bf16"] else _ident
    layers = unpack(params)
    acts, s = cache["acts"], cache["s"]
    e = cache["guess"] - np.asarray(u_target, dtype=np.float64)
    y = apply_A(e)
    P = e.size
    loss = float(np.sum(e * y)) / (s * s * P)
    g = rnd(2.0 * y / (s * P))[..., None]    # dL/d(out), channel axis last
    grads = np.zeros(N_PARAMS)
    for l in range(N_LAYERS - 1, -1, -1):
        W = rnd(layers[l][0])
        x = acts[l]
        o = OFFSETS[l]
        nw = 9 * CIN[l] * COUT[l]
        dW = np.zeros_like(W)
        for t, (di, dk) in enumerate(taps()):
            dW[t] = shift(x, di, dk).reshape(-1, CIN[l]).T @ g.reshape(-1, COUT[l])
        grads[o:o + nw] = dW.ravel()
        grads[o + nw:o + nw + COUT[l]] = g.reshape(-1, COUT[l]).sum(axis=0)
        if l > 0:
            # dx[q][ci] = sum_t sum_co g[q - off_t][co] W[t][ci][co]
            dx = np.zeros(x.shape)
            for t, (di, dk) in enumerate(taps()):
                dx += shift(g, -di, -dk) @ W[t].T
            g = rnd(dx * (x > 0))
    return loss, grads


def guard(b, u1, u2, guess, apply_A):
    """Residual norms of (guess, extrapolation, u1) and the pick: 0 u1,
    1 extrapolation, 2 guess; a later candidate must be strictly smaller."""
    u1, u2 = np.asarray(u1, dtype=np.float64), np.asarray(u2, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    cands = [u1, 2.0 * u1 - u2, np.asarray(guess, dtype=np.float64)]
    res = [float(np.sqrt(np.sum((b - apply_A(x)) ** 2))) for x in cands]
    pick, best = 0, res[0]
    for j in (1, 2):
        if res[j] < best:
            pick, best = j, res[j]
    return (res[2], res[1], res[0]), pick


def extrapolate(hist, p):
    """Order-p polynomial extrapolation to harmonic m through hist[i] =
    u_{m-1-i}, i <= p: the value at m of the degree-p polynomial in the
    harmonic index through the last p + 1 harmonics (Lagrange form on equally
    spaced nodes: weights (-1)^i C(p+1, i+1))."""
    from math import comb
    return sum((-1) ** i * comb(p + 1, i + 1) * np.asarray(hist[i], dtype=np.float64) for i in range(p + 1))


def guard_poly(b, hist, apply_A, net_guess=None):
    """Residual norms |b - A x| of the extrapolations of order 0 .. K-1
    (K = len(hist)) and, last, of net_guess; the pick takes them in that
    order, a later one replacing the choice only when strictly smaller.
    Returns (norms, pick, candidates)."""
    b = np.asarray(b, dtype=np.float64)
    cands = [extrapolate(hist, p) for p in range(len(hist))]
    if net_guess is not None:
        cands.append(np.asarray(net_guess, dtype=np.float64))
    res = [float(np.sqrt(np.sum((b - apply_A(x)) ** 2))) for x in cands]
    pick, best = 0, res[0]
    for j in range(1, len(res)):
        if res[j] < best:
            pick, best = j, res[j]
    return res, pick, cands


def adam(params, grads, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected moments); returns new (params, m1, m2)."""
    m1 = beta1 * m1 + (1 - beta1) * grads
    m2 = beta2 * m2 + (1 - beta2) * grads * grads
    mh = m1 / (1 - beta1 ** step)
    vh = m2 / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m1, m2
