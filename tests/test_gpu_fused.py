"""The single-launch (cooperative, opt-in) strip preconditioner against the
oracle and against the three-launch strip form, through the C-ABI.

Both forms run the same phases on the same strips (the single launch keeps
f' in LDS where the three launches pass it through global memory, and splits
the reduced systems' modes among the strips' workgroups).  A standalone
apply matches the three launches bit for bit; inside PCG the compiler may
contract the phases' multiply-adds differently in the larger kernel, so
solves are held to the oracle (1e-8), to the three launches' iteration count
within one, and to bitwise run-to-run reproducibility.  The oracle bound of
the applies is that of the preconditioner tests (FP32 normwise backward
error <= 2e-6).
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, host, log, rel, spectral_norm_estimate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ax():
    import torch
    assert torch.cuda.is_available()
    from paper_1002_3094_amd import axipcg
    axipcg.lib()
    return axipcg


# (nr, nz, bc): one strip, a strip count that is no power of two (G = 50),
# the benchmark's grids (2048^2 standalone: 8-row strips)
APPLY_CASES = [(4, 256, 0), (64, 256, 1), (200, 1024, 0), (256, 512, 1), (1024, 1024, 0), (2048, 2048, 1),
               (12, 2048, 0), (512, 2048, 1)]


@pytest.mark.parametrize("nr,nz,bc", APPLY_CASES)
def test_single_launch_apply(ax, orc, nr, nz, bc):
    log(f"single-launch apply {nr}x{nz} bc={bc}")
    kappa, q = synth.medium_layered(nr, nz, 7)
    r = np.random.default_rng(11).standard_normal((nr, nz))
    with ax.op_create(kappa, q, bc_z=bc) as op:
        assert not ax.op_fused_info(op, ax.FUSED_APPLY)[0]        # opt-in
        z = dev(np.zeros((nr, nz)))
        ax.precond_apply(op, dev(r), z, ax.PREC_FP32)
        z3 = host(z).copy()
        ax.op_set_fused(op, True)
        active, strips, _ = ax.op_fused_info(op, ax.FUSED_APPLY)
        log(f"  single launch active={active} strips={strips}")
        assert active and strips == nr // (8 if nz == 2048 and nr % 8 == 0 else 4)
        outs = []
        for _ in range(3):                     # barrier numbers keep growing across launches
            z.zero_()
            ax.precond_apply(op, dev(r), z, ax.PREC_FP32)
            outs.append(host(z).copy())
        _, _, errs = ax.op_fused_info(op, ax.FUSED_APPLY, want_errors=True)
        assert errs == 0
    for zf in outs:
        assert np.array_equal(zf, z3)
    oop = orc.operator_from_cells(kappa, q, bc_z=bc)
    B = orc.operator_from_cells(np.full((nr, nz), oop.kbar), np.full((nr, nz), oop.qbar), bc_z=bc,
                                kbar=oop.kbar, qbar=oop.qbar)
    nB = spectral_norm_estimate(lambda v: orc.apply(B, v), (nr, nz)) * 1.1
    back = np.linalg.norm(orc.apply(B, outs[0]) - r) / (nB * np.linalg.norm(outs[0]) + np.linalg.norm(r))
    log(f"  backward={back:.2e}")
    assert back <= 2e-6


@pytest.mark.parametrize("nr,nz,bc", [(64, 256, 0), (256, 512, 1), (1024, 1024, 0), (96, 2048, 1)])
def test_single_launch_pcg(ax, orc, nr, nz, bc):
    log(f"single-launch pcg {nr}x{nz} bc={bc}")
    kappa, q = synth.medium_layered(nr, nz, 8)
    f = synth.ricker_source(nr, nz, 1.0, 1.0, 0.3, 0.01 if nr >= 512 else 0.05)
    oop = orc.operator_from_cells(kappa, q, bc_z=bc)
    bo = orc.rhs(oop, f)
    xr = orc.solve_reference(oop, bo)
    res = {}
    with ax.op_create(kappa, q, bc_z=bc) as op:
        for fused in (False, True, True):
            ax.op_set_fused(op, fused)
            if fused:
                assert ax.op_fused_info(op, ax.FUSED_PCG)[:2] == (True, nr // 4)
            x = dev(np.zeros((nr, nz)))
            st = ax.pcg_solve(op, dev(bo), x, rtol=1e-10, maxit=500, prec=ax.PREC_FP32,
                              flags=ax.FLAG_TRUE_RESIDUAL)
            res.setdefault(fused, []).append((host(x).copy(), st))
        assert ax.op_fused_info(op, ax.FUSED_PCG, want_errors=True)[2] == 0
    (xf, stf), (xf2, stf2) = res[True]
    x3, st3 = res[False][0]
    log(f"  iters {stf['iters']} (three launches {st3['iters']}), err {rel(xf, xr):.2e}, "
        f"vs three launches {rel(xf, x3):.1e}")
    assert stf["code"] == ax.OK and rel(xf, xr) <= 1e-8 and stf["relres_true"] <= 1e-9
    assert abs(stf["iters"] - st3["iters"]) <= 1
    assert stf2["iters"] == stf["iters"] and np.array_equal(xf2, xf)


def test_single_launch_series_matches_oracle(ax, orc):
    """The benchmark's series configuration (polynomial guard, FP32, one
    series_run call) with single-launch iterations over 40 harmonics of the
    1024^2 layered medium: per-step parity of the last harmonic (the oracle
    re-solving from the GPU's right-hand side) and the iteration counts of
    the three launches within one per harmonic."""
    from paper_1002_3094_amd.series import LaguerreSeries
    inp = synth.laguerre_series_inputs(1024, 1024, seed=0)
    outs = {}
    with ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"]) as op:
        g = ax.laguerre_coeffs(40, inp["eta"], inp["ft"], inp["t"][-1])
        for fused in (False, True):
            ax.op_set_fused(op, fused)
            s = LaguerreSeries(op, g, inp["src_i"], inp["src_k"])
            st = s.run(40, "poly", ax.PREC_FP32)
            assert st.status == [ax.OK] * 40
            outs[fused] = (host(s.b).copy(), host(s.u1).copy(), st.iters)
    b, u, its = outs[True]
    oop = orc.operator_from_cells(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    err = rel(u, orc.solve_reference(oop, b, rtol=1e-13, maxit=1000))
    log(f"  iterations {its}, per-step error {err:.1e}")
    assert err <= 1e-8
    assert all(abs(a - c) <= 1 for a, c in zip(its, outs[False][2]))


def test_single_launch_inactive_falls_back(ax, orc):
    # nz = 128 has no one-wave transform: the per-mode three launches run
    kappa, q = synth.medium_layered(64, 128, 2)
    with ax.op_create(kappa, q) as op:
        ax.op_set_fused(op, True)
        for kind in (ax.FUSED_APPLY, ax.FUSED_PCG):
            active, strips, _ = ax.op_fused_info(op, kind)
            assert not active and strips == 0
        r = np.random.default_rng(1).standard_normal((64, 128))
        z = dev(np.zeros((64, 128)))
        ax.precond_apply(op, dev(r), z, ax.PREC_FP32)
        assert rel(host(z), orc.precond(orc.operator_from_cells(kappa, q), r)) <= 2e-3
        # FP64 applies never take the single launch
        ax.precond_apply(op, dev(r), z, ax.PREC_FP64)
        assert rel(host(z), orc.precond(orc.operator_from_cells(kappa, q), r)) <= 1e-9
