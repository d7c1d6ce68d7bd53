"""``axipcg_series_step`` (one call per Laguerre harmonic) and
``axipcg_series_run`` (one call for several harmonics) against the same
harmonics made of separate calls: identical kernels in identical order, so the
solutions must agree bit for bit, with the same iteration counts."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, log

pytestmark = pytest.mark.gpu

N = 128
N_HARM = 5


@pytest.fixture(scope="module")
def ax():
    import torch
    assert torch.cuda.is_available()
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


@pytest.mark.parametrize("guess,solver", [("zero", "pcg"), ("prev", "pcg"), ("extrap", "pcg"), ("nn", "pcg"),
                                          ("extrap", "cheb")])
def test_series_step_matches_separate_calls(ax, guess, solver):
    from paper_1002_3094_amd.series import LaguerreSeries, SeriesStats, nn_init_params
    log(f"series_step guess={guess} solver={solver}")
    inp = synth.laguerre_series_inputs(N, N, seed=3)
    net = ax.nn_create(N, N, nn_init_params(5, last_zero=False)) if guess == "nn" else None
    with ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"]) as op:
        g = ax.laguerre_coeffs(N_HARM, inp["eta"], inp["ft"], inp["t"][-1])
        sols, its = {}, {}
        for path in ("separate", "one_call"):
            s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
            st = SeriesStats()
            out = []
            for _ in range(N_HARM):
                s.step(guess, ax.PREC_FP32, 1e-10, 1000, st, net=net, want_info=(path == "separate"), solver=solver)
                out.append(host(s.u1).copy())
            assert all(c == ax.OK for c in st.status)
            sols[path], its[path] = out, st.iters
        log(f"  iterations {its['one_call']}")
        assert its["separate"] == its["one_call"]
        for a, b in zip(sols["separate"], sols["one_call"]):
            np.testing.assert_array_equal(a, b)
    if net is not None:
        net.close()


@pytest.mark.parametrize("guess,solver,base", [("prev", "pcg", 1), ("nn", "pcg", 1), ("extrap", "cheb", 1),
                                               ("nn", "cheb", 1), ("poly", "pcg", 1), ("nn_poly", "pcg", 1),
                                               ("nn_poly", "pcg", 6), ("poly", "cheb", 1)])
def test_series_run_matches_steps(ax, guess, solver, base):
    """Harmonics 0..6 as one run of 2 and one of 5 against seven single steps
    (base: the order of the extrapolation the network corrects)."""
    from paper_1002_3094_amd.series import LaguerreSeries, SeriesStats, nn_init_params
    log(f"series_run guess={guess} solver={solver} base={base}")
    n_harm = 7
    inp = synth.laguerre_series_inputs(N, N, seed=4)
    net = ax.nn_create(N, N, nn_init_params(6, last_zero=False)) if guess in ("nn", "nn_poly") else None
    if net is not None:
        ax.nn_set_base(net, base)
    with ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"]) as op:
        g = ax.laguerre_coeffs(n_harm, inp["eta"], inp["ft"], inp["t"][-1])
        s1 = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st1 = SeriesStats()
        ref = []
        for _ in range(n_harm):
            s1.step(guess, ax.PREC_FP32, 1e-10, 1000, st1, net=net, solver=solver)
            ref.append((host(s1.u1).copy(), host(s1.u2).copy()))
        s2 = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st2 = SeriesStats()
        s2.run_harmonics(2, guess, ax.PREC_FP32, 1e-10, 1000, st2, net=net, solver=solver)
        np.testing.assert_array_equal(host(s2.u1), ref[1][0])
        np.testing.assert_array_equal(host(s2.u2), ref[1][1])
        s2.run_harmonics(5, guess, ax.PREC_FP32, 1e-10, 1000, st2, net=net, solver=solver)
        log(f"  iterations {st2.iters}")
        assert st2.iters == st1.iters and all(c == ax.OK for c in st2.status) and s2.m == n_harm
        np.testing.assert_array_equal(host(s2.u1), ref[-1][0])
        np.testing.assert_array_equal(host(s2.u2), ref[-1][1])
        assert len({s2.u1.data_ptr(), s2.u2.data_ptr(), s2.u.data_ptr()}) == 3
    if net is not None:
        net.close()


def test_series_run_edge_cases(ax):
    inp = synth.laguerre_series_inputs(32, 32, seed=2)
    with ax.op_create(inp["kappa"], inp["q"]) as op:
        z = lambda: dev(np.zeros((32, 32)))  # noqa: E731
        S1, S2, b = z(), z(), z()
        u = [z(), z(), z()]
        before = [t.data_ptr() for t in u]
        code, sts = ax.series_run(op, 0, [], inp["src_i"], inp["src_k"], S1, S2, b, u, "prev")
        assert code == ax.OK and sts == [] and [t.data_ptr() for t in u] == before
        with pytest.raises(ax.AxipcgError):   # two roles on one array
            ax.series_run(op, 0, [1.0], inp["src_i"], inp["src_k"], S1, S2, b, [u[0], u[0], u[2]], "prev")
        with pytest.raises(ax.AxipcgError):   # the learned guess without a network
            ax.series_run(op, 0, [1.0, 0.5], inp["src_i"], inp["src_k"], S1, S2, b, u, "nn")
        with pytest.raises(ValueError):       # polynomial guesses need eight arrays
            ax.series_run(op, 0, [1.0], inp["src_i"], inp["src_k"], S1, S2, b, u, "poly")
        with pytest.raises(ax.AxipcgError):   # and series_step cannot hold their history
            ax.series_step(op, 0, 1.0, inp["src_i"], inp["src_k"], S1, S2, b, u[0], u[1], u[2], "poly")
        assert [t.data_ptr() for t in u] == before
        # a harmonic that stops at maxit is kept and the run goes on
        code, sts = ax.series_run(op, 0, [1.0, 0.5, 0.25], inp["src_i"], inp["src_k"], S1, S2, b, u, "zero",
                                  maxit=2)
        assert code == ax.ENOTCONV and len(sts) == 3
        assert all(st["status"] == ax.ENOTCONV and st["iters"] == 2 for st in sts)


def test_series_step_rejects_bad_arguments(ax):
    inp = synth.laguerre_series_inputs(32, 32, seed=1)
    with ax.op_create(inp["kappa"], inp["q"]) as op:
        z = lambda: dev(np.zeros((32, 32)))  # noqa: E731
        S1, S2, b, u1, u2, x = z(), z(), z(), z(), z(), z()
        with pytest.raises(ax.AxipcgError):   # the learned guess without a network
            ax.series_step(op, 0, 1.0, inp["src_i"], inp["src_k"], S1, S2, b, u1, u2, x, "nn")
        with pytest.raises(ax.AxipcgError):   # x aliasing u1
            ax.series_step(op, 0, 1.0, inp["src_i"], inp["src_k"], S1, S2, b, u1, u2, u1, "prev")
        with pytest.raises(ax.AxipcgError):   # source cell out of range
            ax.series_step(op, 0, 1.0, 99, 0, S1, S2, b, u1, u2, x, "zero")
