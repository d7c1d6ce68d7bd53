"""Lanczos estimates of the spectrum of B^{-1} A (axipcg_op_bounds_lanczos)
against the oracle's (the same PCG steps and Lanczos matrix in FP64), and
their use as the Chebyshev form's lower parameter on media where eq. (10)
gives none (cells with q = 0)."""
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


@pytest.mark.parametrize("nr,nz,bc", [(64, 64, 0), (37, 128, 1), (128, 256, 0)])
@pytest.mark.parametrize("steps", [5, 20])
def test_ritz_values_match_oracle(ax, orc, nr, nz, bc, steps):
    kappa, q = synth.medium_layered(nr, nz, 21)
    b = np.random.default_rng(5).standard_normal((nr, nz))
    oop = orc.operator_from_cells(kappa, q, bc_z=bc)
    lo, hi = orc.lanczos_bounds(oop, b, steps)
    g1e, g2e = orc.energy_bounds(oop)
    with ax.op_create(kappa, q, bc_z=bc) as op:
        g64 = ax.op_bounds_lanczos(op, dev(b), steps, ax.PREC_FP64)
        g32 = ax.op_bounds_lanczos(op, dev(b), steps, ax.PREC_FP32)
    log(f"lanczos {nr}x{nz} bc={bc} steps={steps}: oracle ({lo:.10f}, {hi:.10f}), FP64 ({g64[0]:.10f}, "
        f"{g64[1]:.10f}), FP32 ({g32[0]:.10f}, {g32[1]:.10f}); eq. (10) ({g1e:.4f}, {g2e:.4f})")
    assert g64[2] == steps and g32[2] == steps
    # the same steps in FP64: rounding only
    assert g64[0] == pytest.approx(lo, rel=1e-9) and g64[1] == pytest.approx(hi, rel=1e-9)
    # the FP32 preconditioner is B^-1 to about 1e-7 (relative)
    assert g32[0] == pytest.approx(lo, rel=1e-5) and g32[1] == pytest.approx(hi, rel=1e-5)
    assert g1e <= g64[0] <= g64[1] <= g2e


def test_constant_medium_gives_one(ax):
    nr, nz = 32, 64
    with ax.op_create(np.full((nr, nz), 2.0), np.full((nr, nz), 0.5)) as op:
        g1, g2, k = ax.op_bounds_lanczos(op, dev(np.random.default_rng(6).standard_normal((nr, nz))), 4,
                                         ax.PREC_FP64)
    assert g1 == pytest.approx(1.0, abs=1e-9) and g2 == pytest.approx(1.0, abs=1e-9)


def test_rejects_zero_b(ax):
    with ax.op_create(np.full((16, 16), 1.0), np.full((16, 16), 1.0)) as op:
        with pytest.raises(ax.AxipcgError):
            ax.op_bounds_lanczos(op, dev(np.zeros((16, 16))), 5)


def test_chebyshev_on_media_with_q_zero(ax, orc):
    """Batch members (q rescaled to [0, 1], so eq. (10) gives gamma1 = 0 for
    the default preconditioner): the Chebyshev form with gamma1 from 20
    Lanczos steps and eq. (10)'s gamma2 converges, single and batched, to the
    oracle's solution."""
    members = [synth.problem_batch_member(p) for p in range(3)]
    ops, bs, g1s, g2s, refs = [], [], [], [], []
    for pr in members:
        op = ax.op_create(pr.kappa, pr.q)
        oop = orc.operator_from_cells(pr.kappa, pr.q)
        assert ax.op_bounds(op)[0] == 0.0      # eq. (10) has no positive lower bound here
        b = dev(np.zeros((pr.nr, pr.nz)))
        ax.rhs_from_f(op, dev(pr.f), b)
        g1, _, _ = ax.op_bounds_lanczos(op, b, 20, ax.PREC_FP32)
        g2 = ax.op_bounds(op)[1]
        ops.append(op)
        bs.append(b)
        g1s.append(g1)
        g2s.append(g2)
        refs.append(orc.solve_reference(oop, host(b)))
    for k, op in enumerate(ops):
        x = dev(np.zeros(bs[k].shape))
        st = ax.cheb_solve(op, bs[k], x, g1s[k], g2s[k], rtol=1e-10, maxit=2000, prec=ax.PREC_FP32)
        y = dev(np.zeros(bs[k].shape))
        sp = ax.pcg_solve(op, bs[k], y, rtol=1e-10, maxit=2000, prec=ax.PREC_FP32)
        err = rel(host(x), refs[k])
        log(f"  member {k} {members[k].nr}x{members[k].nz}: gamma ({g1s[k]:.4f}, {g2s[k]:.4f}), Chebyshev "
            f"{st['iters']} iterations (PCG {sp['iters']}), err {err:.1e}")
        assert st["code"] == ax.OK and err <= 1e-8
    xs = [dev(np.zeros(b.shape)) for b in bs]
    code, stb = ax.batch_cheb_solve(ops, bs, xs, gamma1=g1s, gamma2=g2s, rtol=1e-10, maxit=2000,
                                    prec=ax.PREC_FP32)
    assert code == ax.OK
    for k in range(len(ops)):
        assert rel(host(xs[k]), refs[k]) <= 1e-8
    for op in ops:
        op.close()
