"""Learned initial guess on the GPU against the CPU oracle (oracle/nn.py).

Forward: the network output of the GPU (BF16 MFMA, FP32 accumulation)
against the oracle's exact value of the same rounded network.  The two differ
only by FP32 accumulation order, which now and then moves a hidden BF16
activation by one unit in the last place (2^-8 relative); the tolerance is a
few of those on average (norm-wise 5e-3).  Gradients of the energy-norm loss:
per layer, norm-wise 2e-2 (the data gradient is rounded to BF16 at every
layer too), with a small last layer so that the loss is not dominated by the
output's rounding noise, which A amplifies.  Adam: FP32 arithmetic on the
same gradients, 1e-5.  Guard: the pick and residual norms against the oracle's.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, log, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ax():
    import torch
    assert torch.cuda.is_available()
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


@pytest.fixture(scope="module")
def onn():
    from oracle import nn
    return nn


def _ops(ax, orc, kappa, q):
    """The same operator on both sides: GPU handle and oracle operator."""
    return ax.op_create(kappa, q), orc.operator_from_cells(kappa, q)


SHAPES = [(37, 128), (1, 64), (70, 192), (128, 64)]


def _gpu_out(ax, net, ex):
    g = dev(np.zeros_like(ex["u1"]))
    ax.nn_forward(net, dev(ex["u1"]), dev(ex["u2"]), dev(ex["b"]), dev(ex["kappa"]), g)
    return host(g)


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(ax, onn, shape):
    nr, nz = shape
    log(f"nn forward {shape}")
    ex = synth.nn_example(nr, nz, seed=nr + nz)
    params = onn.init_params(3, last_zero=False)
    params[onn.OFFSETS[5] + 9 * 32] = 0.25          # a non-zero last bias
    net = ax.nn_create(nr, nz, params)
    guess = _gpu_out(ax, net, ex)
    ref, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=True)
    s = cache["s"]
    out_gpu = (guess - (2 * ex["u1"] - ex["u2"])) / s
    e = rel(out_gpu, cache["out"])
    log(f"  out rel err {e:.2e}")
    assert e < 5e-3
    assert np.abs(out_gpu - cache["out"]).max() < 0.05 * np.abs(cache["out"]).max()
    net.close()


def test_zero_last_layer_is_extrapolation(ax, onn):
    ex = synth.nn_example(33, 128, seed=2)
    net = ax.nn_create(33, 128, onn.init_params(4, last_zero=True))
    np.testing.assert_array_equal(_gpu_out(ax, net, ex), 2 * ex["u1"] - ex["u2"])


# (300, 256) has 1200 weight-gradient segments of 64 pixels, more than the
# 1024 partial-sum workgroups: workgroups then loop over one or two segments
# (an uneven split), as at the training size, and the partials' reduction
# sums 1024 rows.
@pytest.mark.parametrize("shape", [(37, 128), (64, 256), (300, 256)])
def test_backward_matches_oracle(ax, onn, orc, shape):
    nr, nz = shape
    log(f"nn backward {shape}")
    ex = synth.nn_example(nr, nz, seed=7 * nr + nz)
    op, oop = _ops(ax, orc, ex["kappa"], np.full((nr, nz), 0.5))
    params = onn.init_params(5, last_zero=False)
    params[onn.OFFSETS[5]:onn.OFFSETS[5] + 9 * 32] *= 0.001
    net = ax.nn_create(nr, nz, params)
    u1, u2 = dev(ex["u1"]), dev(ex["u2"])
    g = dev(np.zeros_like(ex["u1"]))
    ax.nn_forward(net, u1, u2, dev(ex["b"]), dev(ex["kappa"]), g)
    loss = ax.nn_backward(op, net, u1, u2, dev(ex["ut"]))
    _, grads = ax.nn_get_params(net)
    _, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=True)
    lref, gref = onn.backward(params, cache, lambda e: orc.apply(oop, e), ex["ut"])
    log(f"  loss {loss:.6e} vs {lref:.6e}")
    assert loss == pytest.approx(lref, rel=1e-3)
    for l in range(onn.N_LAYERS):
        o = onn.OFFSETS[l]
        nw = 9 * onn.CIN[l] * onn.COUT[l]
        ew = rel(grads[o:o + nw], gref[o:o + nw])
        eb = rel(grads[o + nw:o + nw + onn.COUT[l]], gref[o + nw:o + nw + onn.COUT[l]])
        log(f"  layer {l}: dW rel {ew:.2e}, db rel {eb:.2e}")
        assert ew < 2e-2 and eb < 2e-2
    net.close()
    op.close()


def test_adam_matches_oracle(ax, onn, orc):
    nr, nz = 16, 64
    ex = synth.nn_example(nr, nz, seed=31)
    op, _ = _ops(ax, orc, ex["kappa"], np.zeros((nr, nz)))
    params = onn.init_params(6, last_zero=False)
    net = ax.nn_create(nr, nz, params)
    u1, u2 = dev(ex["u1"]), dev(ex["u2"])
    g = dev(np.zeros_like(ex["u1"]))
    p = params.astype(np.float64)
    m1 = np.zeros_like(p)
    m2 = np.zeros_like(p)
    for step in range(1, 4):
        ax.nn_forward(net, u1, u2, dev(ex["b"]), dev(ex["kappa"]), g)
        ax.nn_backward(op, net, u1, u2, dev(ex["ut"]))
        _, grads = ax.nn_get_params(net)
        ax.nn_adam(net, lr=1e-3)
        got, _ = ax.nn_get_params(net)
        p, m1, m2 = onn.adam(p, grads.astype(np.float64), m1, m2, step, 1e-3)
        assert np.abs(got - p).max() < 1e-5 * max(1.0, np.abs(p).max())
        p = got.astype(np.float64)
    net.close()
    op.close()


def _bias_only(onn, c):
    p = np.zeros(onn.N_PARAMS, dtype=np.float32)
    p[onn.OFFSETS[5] + 9 * 32] = c
    return p


# several row pairs per thread (nz = 1024), an odd row count, more rows than
# residual workgroups (1100 > 1024)
GUARD_SHAPES = [(32, 64), (37, 1024), (1100, 64)]


@pytest.mark.parametrize("nr,nz", GUARD_SHAPES)
def test_guard_picks_smallest_residual(ax, onn, orc, nr, nz):
    kappa, q = synth.medium_layered(nr, nz, 3)
    op, oop = _ops(ax, orc, kappa, q)
    f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.2, 0.5, 0.05)
    b = orc.rhs(oop, f)
    ustar, status, _, _ = orc.pcg(oop, b, np.zeros_like(b), rtol=1e-14, maxit=2000)
    assert status == 0
    A = lambda x: orc.apply(oop, x)  # noqa: E731
    shift = 0.1 * np.abs(ustar).max()
    u1 = ustar - shift
    s = np.sqrt(np.mean(u1 * u1))
    kd, bd = dev(kappa), dev(b)
    x = dev(np.zeros_like(b))

    def run(params, u1, u2):
        ax.nn_set_params(net, params)
        phi, pick = ax.nn_guess(op, net, bd, dev(u1), dev(u2), kd, x)
        return phi, pick, host(x)

    # 1. u2 = u1 (extrapolation = u1) and out == shift / s: the network guess is
    #    u* up to the float32 rounding of the bias, and wins
    c32 = float(np.float32(shift / s))
    net = ax.nn_create(nr, nz, _bias_only(onn, shift / s))
    phi, pick, xh = run(_bias_only(onn, shift / s), u1, u1)
    guess_ref = u1 + s * c32
    phi_ref, pick_ref = onn.guard(b, u1, u1, guess_ref, A)
    log(f"guard: resid {phi} (oracle {phi_ref}), pick {pick}")
    assert pick == pick_ref == 2
    np.testing.assert_allclose(phi[1:], phi_ref[1:], rtol=1e-9)
    # the winner's residual is ~1e-8 of the others': cancellation leaves ~1e-5 relative
    assert phi[0] == pytest.approx(phi_ref[0], rel=1e-5)
    np.testing.assert_allclose(xh, guess_ref, rtol=1e-12, atol=1e-14 * np.abs(ustar).max())
    # 2. u2 = 2 u1 - u*: the extrapolation is u*; a zero network ties with it, so
    #    the extrapolation is kept
    u2 = 2 * u1 - ustar
    phi, pick, xh = run(_bias_only(onn, 0.0), u1, u2)
    phi_ref, pick_ref = onn.guard(b, u1, u2, 2 * u1 - u2, A)
    assert pick == pick_ref == 1
    # the extrapolation's residual is at rounding level: compare it against u1's
    np.testing.assert_allclose(phi[1:], phi_ref[1:], rtol=1e-9, atol=1e-12 * phi_ref[2])
    assert phi[0] == phi[1]
    np.testing.assert_array_equal(xh, 2 * u1 - u2)
    # 3. a network that blows the guess up (non-finite FP32 output) never wins
    p = _bias_only(onn, 0.0)
    p[onn.OFFSETS[4] + 9 * 32 * 32:onn.OFFSETS[5]] = 1.0     # hidden activations of 1 feed the last layer
    p[onn.OFFSETS[5]:onn.OFFSETS[5] + 9 * 32] = 3.0e38
    phi, pick, xh = run(p, u1, u1)
    log(f"guard (overflow): resid {phi}, pick {pick}")
    assert not np.isfinite(phi[0]) and pick == 0
    np.testing.assert_array_equal(xh, u1)
    # 4. all three equal: u1 is kept
    phi, pick, xh = run(_bias_only(onn, 0.0), u1, u1)
    assert pick == 0 and phi[0] == phi[1] == phi[2]
    np.testing.assert_array_equal(xh, u1)
    net.close()
    op.close()


@pytest.mark.parametrize("nr,nz", GUARD_SHAPES)
def test_extrapolation_guard(ax, onn, orc, nr, nz):
    kappa, q = synth.medium_layered(nr, nz, 5)
    op, oop = _ops(ax, orc, kappa, q)
    f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.3, 0.4, 0.05)
    b = orc.rhs(oop, f)
    ustar, status, _, _ = orc.pcg(oop, b, np.zeros_like(b), rtol=1e-14, maxit=2000)
    assert status == 0
    A = lambda x: orc.apply(oop, x)  # noqa: E731
    rng = np.random.default_rng(8)
    bd = dev(b)
    cases = [
        (ustar + 0.1 * rng.standard_normal(b.shape), None, 1),        # u2 = 2 u1 - u*: extrapolation exact
        (ustar + 0.1 * rng.standard_normal(b.shape), "same", 0),      # u2 = u1: tie, u1 kept
        (ustar + 1e-3 * rng.standard_normal(b.shape), "far", 0),      # u2 far off: u1 better
    ]
    for u1, kind, want in cases:
        u2 = 2 * u1 - ustar if kind is None else (u1 if kind == "same" else u1 + rng.standard_normal(b.shape))
        x = dev(np.zeros_like(b))
        res, pick = ax.guess_extrap(op, bd, dev(u1), dev(u2), x, want_info=True)
        res_ref, pick_ref = onn.guard(b, u1, u2, 2 * u1 - u2, A)
        log(f"extrap guard {kind}: resid {res} (oracle {res_ref[1:]}) pick {pick}")
        assert pick == want and pick_ref in (want, 2)
        np.testing.assert_allclose(res, res_ref[1:], rtol=1e-9, atol=1e-12 * res_ref[2])
        np.testing.assert_array_equal(host(x), u1 if want == 0 else 2 * u1 - u2)
    # x may alias u1: the choice is made before x is written
    u1 = ustar + 0.1 * rng.standard_normal(b.shape)
    u1d = dev(u1)
    ax.guess_extrap(op, bd, u1d, dev(2 * u1 - ustar), u1d)
    np.testing.assert_allclose(host(u1d), ustar, rtol=0, atol=1e-12 * np.abs(ustar).max())
    op.close()


@pytest.mark.parametrize("nr,nz", GUARD_SHAPES)
def test_poly_guard_matches_oracle(ax, onn, orc, nr, nz):
    """Extrapolations of every order against the oracle's: residual norms,
    the pick, and x = the chosen candidate."""
    kappa, q = synth.medium_layered(nr, nz, 6)
    op, oop = _ops(ax, orc, kappa, q)
    f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.25, 0.5, 0.05)
    b = orc.rhs(oop, f)
    ustar, status, _, _ = orc.pcg(oop, b, np.zeros_like(b), rtol=1e-14, maxit=2000)
    assert status == 0
    A = lambda x: orc.apply(oop, x)  # noqa: E731
    rng = np.random.default_rng(12)
    scale = np.abs(ustar).max()
    w = [rng.standard_normal(b.shape) * 0.1 * scale for _ in range(3)]
    hist = [ustar + sum(wd * float(i + 1) ** (d + 1) for d, wd in enumerate(w))
            + 1e-5 * scale * rng.standard_normal(b.shape) for i in range(7)]
    bd = dev(b)
    hd = [dev(h) for h in hist]
    for k in range(1, 8):
        x = dev(np.zeros_like(b))
        res, pick = ax.guess_poly(op, bd, hd[:k], x, want_info=True)
        res_ref, pick_ref, cands = onn.guard_poly(b, hist[:k], A)
        log(f"poly guard {nr}x{nz} K={k}: pick {pick} (oracle {pick_ref}) resid {res}")
        # orders >= 3 reproduce the cubic and differ only in the noise they amplify
        assert pick == pick_ref and (k < 4 or pick == 3)
        np.testing.assert_allclose(res, res_ref, rtol=1e-9)
        np.testing.assert_allclose(host(x), cands[pick], rtol=1e-13, atol=1e-14 * scale)
    # x may alias the newest history array
    x = hd[0].clone()
    h2 = [x] + hd[1:]
    ax.guess_poly(op, bd, h2, x)
    _, pick_ref, cands = onn.guard_poly(b, hist, A)
    np.testing.assert_allclose(host(x), cands[pick_ref], rtol=1e-13, atol=1e-14 * scale)
    with pytest.raises(ax.AxipcgError):
        ax.guess_poly(op, bd, hd + [hd[0]], dev(np.zeros_like(b)))   # eight arrays
    with pytest.raises(ax.AxipcgError):
        ax.guess_poly(op, bd, [bd], dev(np.zeros_like(b)))           # history aliasing b
    op.close()


def test_nn_poly_guard_matches_oracle(ax, onn, orc):
    nr, nz = 32, 64
    kappa, q = synth.medium_layered(nr, nz, 3)
    op, oop = _ops(ax, orc, kappa, q)
    f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.2, 0.5, 0.05)
    b = orc.rhs(oop, f)
    ustar, status, _, _ = orc.pcg(oop, b, np.zeros_like(b), rtol=1e-14, maxit=2000)
    assert status == 0
    A = lambda x: orc.apply(oop, x)  # noqa: E731
    shift = 0.1 * np.abs(ustar).max()
    u1 = ustar - shift
    s = np.sqrt(np.mean(u1 * u1))
    c32 = float(np.float32(shift / s))
    kd, bd = dev(kappa), dev(b)
    # a constant history: every extrapolation is u1; a bias-only network
    # whose correction is the shift makes the learned guess (nearly) u*
    hist = [u1] * 4
    net = ax.nn_create(nr, nz, _bias_only(onn, shift / s))
    x = dev(np.zeros_like(b))
    phi, pick = ax.nn_guess_poly(op, net, bd, [dev(h) for h in hist], kd, x)
    res_ref, pick_ref, _ = onn.guard_poly(b, hist, A, net_guess=u1 + s * c32)
    log(f"nn poly guard: resid {phi} (oracle {res_ref}), pick {pick}")
    assert pick == pick_ref == 4
    np.testing.assert_allclose(phi[:4], res_ref[:4], rtol=1e-9)
    assert phi[4] == pytest.approx(res_ref[4], rel=1e-5)
    np.testing.assert_allclose(host(x), u1 + s * c32, rtol=1e-12, atol=1e-14 * np.abs(ustar).max())
    # a zero network equals the linear extrapolation, which comes first: it never wins
    ax.nn_set_params(net, _bias_only(onn, 0.0))
    phi, pick = ax.nn_guess_poly(op, net, bd, [dev(h) for h in hist], kd, x)
    assert pick < 4
    np.testing.assert_allclose(host(x), u1, rtol=1e-14, atol=1e-15 * np.abs(ustar).max())
    with pytest.raises(ax.AxipcgError):       # the network needs two history arrays
        ax.nn_guess_poly(op, net, bd, [dev(u1)], kd, x)
    net.close()
    op.close()



def test_nn_base_order_guard_matches_oracle(ax, onn, orc):
    """Base order 4: the network's candidate is x_4 + s out.  A history that
    is u* - shift plus a cubic in the harmonic index makes x_3 .. x_6 equal
    u* - shift (orders 0..2 miss the cubic); a bias-only network whose
    correction is the shift makes its candidate (nearly) u*."""
    nr, nz = 32, 64
    kappa, q = synth.medium_layered(nr, nz, 4)
    op, oop = _ops(ax, orc, kappa, q)
    b = orc.rhs(oop, synth.gaussian_source(nr, nz, 1.0, 1.0, 0.2, 0.5, 0.05))
    ustar, status, _, _ = orc.pcg(oop, b, np.zeros_like(b), rtol=1e-14, maxit=2000)
    assert status == 0
    A = lambda x: orc.apply(oop, x)  # noqa: E731
    rng = np.random.default_rng(3)
    w = 0.05 * np.abs(ustar).max() * rng.standard_normal((3, nr, nz))
    shift = 0.1 * np.abs(ustar).max()
    hist = [ustar - shift + sum(w[d] * float(i + 1) ** (d + 1) for d in range(3)) for i in range(7)]
    s = np.sqrt(np.mean(hist[0] * hist[0]))
    c32 = float(np.float32(shift / s))
    net = ax.nn_create(nr, nz, _bias_only(onn, shift / s))
    assert ax.nn_get_base(net) == 1
    ax.nn_set_base(net, 4)
    assert ax.nn_get_base(net) == 4
    kd, bd, hd = dev(kappa), dev(b), [dev(h) for h in hist]
    x = dev(np.zeros_like(b))
    phi, pick = ax.nn_guess_poly(op, net, bd, hd, kd, x)
    base4 = onn.extrapolate(hist, 4)
    res_ref, pick_ref, _ = onn.guard_poly(b, hist, A, net_guess=base4 + s * c32)
    log(f"nn base-4 guard: resid {phi} (oracle {res_ref}), pick {pick}")
    assert pick == pick_ref == 7
    np.testing.assert_allclose(phi[:7], res_ref[:7], rtol=1e-8)
    assert phi[7] == pytest.approx(res_ref[7], rel=1e-5)
    np.testing.assert_allclose(host(x), base4 + s * c32, rtol=1e-12, atol=1e-13 * np.abs(ustar).max())
    # too few history arrays for the base, and the two-array calls, are refused
    with pytest.raises(ax.AxipcgError):
        ax.nn_guess_poly(op, net, bd, hd[:4], kd, x)
    with pytest.raises(ax.AxipcgError):
        ax.nn_guess(op, net, bd, hd[0], hd[1], kd, x)
    with pytest.raises(ax.AxipcgError):
        ax.nn_forward(net, hd[0], hd[1], bd, kd, x)
    with pytest.raises(ax.AxipcgError):
        ax.nn_backward(op, net, hd[0], hd[1], x)
    for bad in (0, 7):
        with pytest.raises(ax.AxipcgError):
            ax.nn_set_base(net, bad)
    assert ax.nn_get_base(net) == 4
    net.close()
    op.close()


@pytest.mark.parametrize("shape,order", [((37, 128), 2), ((64, 256), 6)])
def test_backward_base_order_matches_oracle(ax, onn, orc, shape, order):
    nr, nz = shape
    log(f"nn backward base order {order} {shape}")
    ex = synth.nn_example(nr, nz, seed=5 * nr + nz)
    rng = np.random.default_rng(order)
    hist = [ex["u1"], ex["u2"]] + [ex["u1"] + 0.3 * rng.standard_normal((nr, nz)) for _ in range(order - 1)]
    op, oop = _ops(ax, orc, ex["kappa"], np.full((nr, nz), 0.5))
    params = onn.init_params(5, last_zero=False)
    params[onn.OFFSETS[5]:onn.OFFSETS[5] + 9 * 32] *= 0.001
    net = ax.nn_create(nr, nz, params)
    ax.nn_set_base(net, order)
    hd = [dev(h) for h in hist]
    x = dev(np.zeros_like(ex["u1"]))
    ax.nn_guess_poly(op, net, dev(ex["b"]), hd, dev(ex["kappa"]), x)
    loss = ax.nn_backward_poly(op, net, hd, dev(ex["ut"]))
    _, grads = ax.nn_get_params(net)
    _, cache = onn.forward(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], bf16=True, hist=hist, order=order)
    lref, gref = onn.backward(params, cache, lambda e: orc.apply(oop, e), ex["ut"])
    log(f"  loss {loss:.6e} vs {lref:.6e}")
    assert loss == pytest.approx(lref, rel=1e-3)
    for l in range(onn.N_LAYERS):
        o = onn.OFFSETS[l]
        nw = 9 * onn.CIN[l] * onn.COUT[l]
        ew = rel(grads[o:o + nw], gref[o:o + nw])
        eb = rel(grads[o + nw:o + nw + onn.COUT[l]], gref[o + nw:o + nw + onn.COUT[l]])
        log(f"  layer {l}: dW rel {ew:.2e}, db rel {eb:.2e}")
        assert ew < 2e-2 and eb < 2e-2
    net.close()
    op.close()


def test_forward_1024_sampled(ax, onn):
    """Forward pass at the benchmark's 1024^2 grid against the oracle on
    sampled cells (corners, edges and seeded interior cells), each evaluated
    by the oracle on its receptive field; the bound is the one of the small
    shapes above."""
    n = 1024
    log("nn forward 1024^2 sampled")
    ex = synth.nn_example(n, n, seed=77)
    params = onn.init_params(5, last_zero=False)
    params[onn.OFFSETS[5] + 9 * 32] = 0.25
    net = ax.nn_create(n, n, params)
    guess = _gpu_out(ax, net, ex)
    net.close()
    s, _ = onn.scales(ex["u1"], ex["b"])
    out_gpu = (guess - (2 * ex["u1"] - ex["u2"])) / s
    rng = np.random.default_rng(77)
    edge = [0, 1, 5, 6, n // 2, n - 7, n - 2, n - 1]
    pts = [(i, k) for i in edge for k in edge] + [tuple(p) for p in rng.integers(0, n, size=(200, 2))]
    ref = onn.forward_at(params, ex["u1"], ex["u2"], ex["b"], ex["kappa"], pts, bf16=True)
    got = np.array([out_gpu[i, k] for i, k in pts])
    e = rel(got, ref)
    log(f"  {len(pts)} cells: out rel err {e:.2e}")
    assert e < 5e-3
    assert np.abs(got - ref).max() < 0.05 * np.abs(ref).max()
