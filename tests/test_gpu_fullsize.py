"""Parity at the benchmark's sizes, in the launch configuration bench.py times.

* single solve on the 1024^2 layered medium with the spatial Ricker source,
  FP64 and FP32 preconditioner, error <= 1e-8 vs the oracle;
* Laguerre source coefficients g_m (device trapezoid rule vs the oracle's
  Simpson rule on the same samples) to 1e-10 relative;
* the Laguerre series itself: the GPU chain (running-sum right-hand sides,
  previous-harmonic guess, FP32 preconditioner, rtol 1e-10) against the
  oracle's chain (direct history sum, FP64, rtol 1e-13) from the same seeded
  inputs, every harmonic within 1e-8 relative L2;
* the benchmark's launch configuration (one series_run call over the
  harmonics with the polynomial-extrapolation guard, with and without the
  learned candidate) against the same oracle chain, 1e-8 relative L2.
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


@pytest.mark.parametrize("prec", [0, 1])
def test_layered_1024_single_solve(ax, orc, prec):
    log(f"layered 1024^2 single solve prec={prec}")
    p = synth.problem_layered(1024, 1024, seed=0)
    oop = orc.operator_from_cells(p.kappa, p.q)
    bo = orc.rhs(oop, p.f)
    xr = orc.solve_reference(oop, bo, rtol=1e-13)
    with ax.op_create(p.kappa, p.q) as op:
        b = dev(np.zeros((1024, 1024)))
        ax.rhs_from_f(op, dev(p.f), b)
        x = dev(np.zeros((1024, 1024)))
        st = ax.pcg_solve(op, b, x, 1e-10, 500, prec, ax.FLAG_TRUE_RESIDUAL)
        xg = host(x)
    err = rel(xg, xr)
    log(f"  iters={st['iters']} relres_true={st['relres_true']:.2e} err={err:.2e}")
    assert st["code"] == ax.OK and err <= 1e-8


@pytest.mark.parametrize("n,eta", [(400, 10.0), (64, 300.0)])
def test_laguerre_coeffs_match_oracle(ax, orc, n, eta):
    log(f"laguerre coeffs n={n} eta={eta}")
    t, ft = synth.ricker_pulse_samples()
    gg = ax.laguerre_coeffs(n, eta, ft, t[-1])
    go = orc.laguerre_coeffs(n, eta, ft, t[-1])
    assert np.abs(gg - go).max() <= 1e-10 * np.abs(go).max()


def _gpu_chain(ax, inp, n_harm, prec=1):
    nr, nz = inp["kappa"].shape
    g = ax.laguerre_coeffs(n_harm, inp["eta"], inp["ft"], inp["t"][-1])
    out, stats = [], []
    with ax.op_create(inp["kappa"], inp["q"]) as op:
        S1 = dev(np.zeros((nr, nz)))
        S2 = dev(np.zeros((nr, nz)))
        b = dev(np.zeros((nr, nz)))
        u = dev(np.zeros((nr, nz)))
        for m in range(n_harm):
            ax.laguerre_rhs(op, float(g[m]), inp["src_i"], inp["src_k"], S1, S2, b, u_prev=(u if m else None))
            st = ax.pcg_solve(op, b, u, 1e-10, 1000, prec)
            assert st["code"] == ax.OK
            out.append(host(u).copy())
            stats.append(st["iters"])
    return out, stats


@pytest.mark.parametrize("nr,nz,n_harm", [(64, 64, 12), (1024, 1024, 3), (2048, 2048, 2)])
def test_laguerre_chain_matches_oracle(ax, orc, nr, nz, n_harm):
    log(f"laguerre chain {nr}x{nz} harmonics={n_harm}")
    inp = synth.laguerre_series_inputs(nr, nz, seed=0)
    ug, its = _gpu_chain(ax, inp, n_harm)
    oop = orc.operator_from_cells(inp["kappa"], inp["q"])
    go = orc.laguerre_coeffs(n_harm, inp["eta"], inp["ft"], inp["t"][-1])
    uo, ost = orc.laguerre_chain(oop, inp["kappa"], go, inp["eta"], inp["src_i"], inp["src_k"], n_harm,
                                 rtol=1e-13 if nr < 2048 else 1e-12)
    errs = [rel(a, b) for a, b in zip(ug, uo)]
    log(f"  iters={its} errs={[f'{e:.1e}' for e in errs]}")
    assert max(errs) <= 1e-8


# The benchmark's own launch configuration: the whole run of harmonics in one
# series_run call (right-hand side, guard over the seven-harmonic polynomial
# extrapolations -- and the learned candidate --, FP64 PCG with the FP32
# preconditioner, rtol 1e-10) on the 1024^2 layered medium.  The call keeps
# the last seven solutions; each must match the oracle's harmonic, since the
# answer does not depend on the guess.
N_HEAD = 9


@pytest.fixture(scope="module")
def head_oracle(orc):
    inp = synth.laguerre_series_inputs(1024, 1024, seed=0)
    oop = orc.operator_from_cells(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    go = orc.laguerre_coeffs(N_HEAD, inp["eta"], inp["ft"], inp["t"][-1])
    uo, _ = orc.laguerre_chain(oop, inp["kappa"], go, inp["eta"], inp["src_i"], inp["src_k"], N_HEAD,
                               rtol=1e-13)
    return inp, uo


@pytest.mark.parametrize("guess", ["nn_poly", "poly"])
def test_series_run_1024_matches_oracle(ax, head_oracle, guess):
    from paper_1002_3094_amd.series import LaguerreSeries, nn_init_params
    log(f"series_run 1024^2 guess={guess} harmonics={N_HEAD}")
    inp, uo = head_oracle
    net = ax.nn_create(1024, 1024, nn_init_params(0, last_zero=False)) if guess == "nn_poly" else None
    with ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"]) as op:
        g = ax.laguerre_coeffs(N_HEAD, inp["eta"], inp["ft"], inp["t"][-1])
        s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st = s.run(N_HEAD, guess, ax.PREC_FP32, rtol=1e-10, net=net)
        assert st.status == [ax.OK] * N_HEAD
        kept = [host(h).copy() for h in s.hist]   # u_8, u_7, ..., u_2
    if net is not None:
        net.close()
    errs = [rel(kept[j], uo[N_HEAD - 1 - j]) for j in range(len(kept))]
    log(f"  iters={st.iters} errs={[f'{e:.1e}' for e in errs]}")
    assert max(errs) <= 1e-8


# Per-step parity on a long chain (the oracle re-solves harmonic m from the
# GPU's own right-hand side b_m): the benchmark's configuration (one
# series_run call per chunk, polynomial guard with and without the learned
# candidate, FP32 preconditioner) over 160 harmonics of the 1024^2 medium,
# checked at harmonics spread over the run and at the last one.  The error of
# the chain as a whole compounds through the history sums and is not what
# this gates; each step's solve is.
PER_STEP_MARKS = (20, 59, 110, 159)


@pytest.mark.parametrize("guess", ["nn_poly", "poly"])
def test_series_run_per_step_parity_late_harmonics(ax, orc, guess):
    from paper_1002_3094_amd.series import LaguerreSeries, SeriesStats, nn_init_params
    log(f"per-step parity 1024^2 guess={guess} marks={PER_STEP_MARKS}")
    inp = synth.laguerre_series_inputs(1024, 1024, seed=0)
    oop = orc.operator_from_cells(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    net = ax.nn_create(1024, 1024, nn_init_params(0, last_zero=False)) if guess == "nn_poly" else None
    cases = []
    with ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"]) as op:
        g = ax.laguerre_coeffs(PER_STEP_MARKS[-1] + 1, inp["eta"], inp["ft"], inp["t"][-1])
        s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st = SeriesStats()
        for m in PER_STEP_MARKS:
            s.run_harmonics(m + 1 - s.m, guess, ax.PREC_FP32, 1e-10, 1000, st, net=net)
            cases.append((m, host(s.b).copy(), host(s.u1).copy()))
        assert all(c == ax.OK for c in st.status)
    if net is not None:
        net.close()
    errs = []
    for m, b, u in cases:
        ref = orc.solve_reference(oop, b, rtol=1e-13, maxit=1000)
        errs.append(rel(u, ref))
        assert np.linalg.norm(b) > 0
    log(f"  mean iters={np.mean(st.iters):.2f} errs={[f'{e:.1e}' for e in errs]}")
    assert max(errs) <= 1e-8
