"""The learned guess inside the Laguerre series (§4.1, eq. (35)) against the
method without it: the polynomial-extrapolation guard alone ("poly") versus
the same guard with the trained network's candidate added ("nn_poly", the
network correcting the order-6 extrapolation).

* online training in nn_poly mode on two media lowers the network's loss;
* on a held-out medium both modes converge to the oracle's harmonics (1e-8,
  like every chain parity test);
* the guard takes the network only when its residual is strictly smaller than
  every extrapolation's, and a harmonic where it does not starts PCG from the
  same array as "poly": the iterations are then the same;
* what the network gains is measured and logged: its pick count, the mean
  iterations of both modes, and the energy-norm error of the network's
  candidate relative to the best extrapolation's on the held-out harmonics.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import host, log, rel

pytestmark = pytest.mark.gpu

N = 256
N_TRAIN = 40
N_EVAL = 40
N_ORACLE = 20
BASE = 6


@pytest.fixture(scope="module")
def ax():
    import torch
    assert torch.cuda.is_available()
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


def _problem(ax, seed, n):
    inp = synth.laguerre_series_inputs(N, N, seed=seed)
    op = ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    g = ax.laguerre_coeffs(n, inp["eta"], inp["ft"], inp["t"][-1])
    return inp, op, g


def test_learned_guess_against_poly_guard(ax, orc):
    import torch
    from paper_1002_3094_amd.series import LaguerreSeries, SeriesStats, nn_init_params
    net = ax.nn_create(N, N, nn_init_params(0))
    ax.nn_set_base(net, BASE)
    for seed in (1, 2):
        inp, op, g = _problem(ax, seed, N_TRAIN)
        s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st = s.run(N_TRAIN, "nn_poly", ax.PREC_FP32, net=net, lr=1e-3, want_info=True)
        assert all(c == ax.OK for c in st.status)
        L = np.array(st.loss)
        log(f"train seed {seed}: loss first10 {L[2:12].mean():.3e} last10 {L[-10:].mean():.3e}, "
            f"iters {np.mean(st.iters):.2f}, picks {np.bincount(st.choice, minlength=8)}")
        if seed == 1:
            assert L[-10:].mean() < L[2:12].mean()
        op.close()

    inp, op, g = _problem(ax, 101, N_EVAL)
    runs = {}
    for mode in ("poly", "nn_poly"):
        s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st = SeriesStats()
        sols = []
        for _ in range(N_EVAL):
            s.step(mode, ax.PREC_FP32, 1e-10, 1000, st, net=net, want_info=True)
            if len(sols) < N_ORACLE:
                sols.append(host(s.u1).copy())
        assert all(c == ax.OK for c in st.status)
        runs[mode] = (st, sols)
    st_p, st_n = runs["poly"][0], runs["nn_poly"][0]
    picks_net = int(np.sum(np.array(st_n.choice) == ax.POLY_HISTORY))
    it_p, it_n = np.mean(st_p.iters), np.mean(st_n.iters)
    log(f"held-out: iters poly {it_p:.2f}, nn_poly {it_n:.2f} (change {it_n - it_p:+.2f}); "
        f"network picked on {picks_net} of {N_EVAL} harmonics; picks {np.bincount(st_n.choice, minlength=8)}")
    for m in range(N_EVAL):
        res_n = st_n.resid[m]
        if st_n.choice[m] == ax.POLY_HISTORY:
            assert res_n[ax.POLY_HISTORY] < min(res_n[:ax.POLY_HISTORY])
        else:
            # the same extrapolation from the same history: the same start
            assert st_n.choice[m] == st_p.choice[m]
            assert st_n.iters[m] == st_p.iters[m]

    # the network's own candidate x_6 + s out against the best extrapolation,
    # by the energy norm of their errors (CG's measure) and by the residual
    s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
    s.run_harmonics(N_EVAL - 10, "poly", ax.PREC_FP32, 1e-10, 1000, SeriesStats())
    z = lambda: torch.zeros((N, N), dtype=torch.float64, device="cuda")  # noqa: E731
    xb, gx, y = z(), z(), z()
    w6 = [7, -21, 35, -35, 21, -7, 1]
    ratios = []
    for _ in range(10):
        m = s.m
        ax.laguerre_rhs(op, s.g[m], s.src_i, s.src_k, s.S1, s.S2, s.b, u_prev=s.u1)
        ax.guess_poly(op, s.b, s.hist, xb)
        ax.nn_set_base(net, 1)                     # out from the two-array form
        ax.nn_forward(net, s.hist[0], s.hist[1], s.b, s.kappa, gx)
        ax.nn_set_base(net, BASE)
        xn = sum(c * s.hist[j] for j, c in enumerate(w6)) + (gx - (2 * s.hist[0] - s.hist[1]))
        s.u.copy_(xb)
        ax.pcg_solve(op, s.b, s.u, rtol=1e-12, prec=ax.PREC_FP64)
        en = []
        for x in (xb, xn):
            e = x - s.u
            ax.apply_A(op, e, y)
            en.append(float(torch.sqrt(torch.sum(e * y))))
        ratios.append(en[1] / en[0])
        s._rotate()
        s.m += 1
    log(f"  energy-norm error of the network candidate / best extrapolation: median {np.median(ratios):.3f} "
        f"(harmonics {N_EVAL - 10}..{N_EVAL - 1})")
    assert all(np.isfinite(ratios))

    oop = orc.operator_from_cells(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    go = orc.laguerre_coeffs(N_ORACLE, inp["eta"], inp["ft"], inp["t"][-1])
    uo, _ = orc.laguerre_chain(oop, inp["kappa"], go, inp["eta"], inp["src_i"], inp["src_k"], N_ORACLE,
                               rtol=1e-13)
    for mode in ("poly", "nn_poly"):
        errs = [rel(a, b) for a, b in zip(runs[mode][1], uo)]
        log(f"  {mode} harmonics vs oracle: max rel err {max(errs):.2e}")
        assert max(errs) <= 1e-8
    net.close()
    op.close()
