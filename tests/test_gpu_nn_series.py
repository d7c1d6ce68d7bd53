"""The learned guess inside the Laguerre series (§4.1, eq. (35)): online
training on two media, then a held-out medium solved from the guarded guess.

* training lowers the network's loss;
* every harmonic solved from the guarded guess converges to the oracle's
  harmonic (guess-independent answer, 1e-8 like every chain parity test);
* the guard never starts PCG from a larger residual than u_{m-1}, so the
  series needs no more iterations on average than the previous-harmonic guess
  (the measured gain is logged).
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


def test_trained_guess_in_series(ax, orc):
    from paper_1002_3094_amd.series import LaguerreSeries, SeriesStats, nn_init_params
    net = ax.nn_create(N, N, nn_init_params(0))
    for seed in (1, 2):
        inp, op, g = _problem(ax, seed, N_TRAIN)
        s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st = s.run(N_TRAIN, "nn", ax.PREC_FP32, net=net, lr=1e-3, want_info=True)
        assert all(c == ax.OK for c in st.status)
        L = np.array(st.loss)
        log(f"train seed {seed}: loss first10 {L[2:12].mean():.3e} last10 {L[-10:].mean():.3e}, "
            f"iters {np.mean(st.iters):.2f}, picks {np.bincount(st.choice, minlength=3)}")
        if seed == 1:
            assert L[-10:].mean() < L[2:12].mean()
        op.close()

    inp, op, g = _problem(ax, 101, N_EVAL)
    runs = {}
    for mode in ("prev", "nn"):
        s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st = SeriesStats()
        sols = []
        for _ in range(N_EVAL):
            s.step(mode, ax.PREC_FP32, 1e-10, 1000, st, net=net, want_info=True)
            if len(sols) < N_ORACLE:
                sols.append(host(s.u1).copy())
        assert all(c == ax.OK for c in st.status)
        runs[mode] = (st, sols)
    it_prev = np.mean(runs["prev"][0].iters)
    it_nn = np.mean(runs["nn"][0].iters)
    picks = np.bincount(runs["nn"][0].choice, minlength=3)
    log(f"held-out: iters prev {it_prev:.2f}, guarded guess {it_nn:.2f} (picks prev/extrap/net {picks})")
    assert it_nn <= it_prev + 0.25

    oop = orc.operator_from_cells(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    go = orc.laguerre_coeffs(N_ORACLE, inp["eta"], inp["ft"], inp["t"][-1])
    uo, _ = orc.laguerre_chain(oop, inp["kappa"], go, inp["eta"], inp["src_i"], inp["src_k"], N_ORACLE,
                               rtol=1e-13)
    errs = [rel(a, b) for a, b in zip(runs["nn"][1], uo)]
    log(f"  guarded-guess harmonics vs oracle: max rel err {max(errs):.2e}")
    assert max(errs) <= 1e-8
    net.close()
    op.close()
