"""The batched solve in one cooperative launch (AXIPCG_FLAG_SINGLE_LAUNCH):
the same phases as the launch-per-phase batch, dealt to resident workgroups
with grid barriers between them.  Every problem goes through the same
operations in the same order as in the launch-per-phase form; only the
compiler's choice of fused multiply-adds differs between the two kernels'
code, so the two agree to rounding: the same iteration counts and statuses,
iterates to 1e-12 relative, and the recursive residuals ||r_k|| / ||b|| to
1e-13 (absolute: at convergence ||r_k|| is about 1e-10 ||b||, the
difference of vectors of size ||b||, so rounding of order 1e-16 ||b|| moves
it by about 1e-6 of itself once the preconditioner runs in FP32).  The launch-per-phase batch
itself is checked against the oracle in tests/test_gpu_batch.py, and a few
members here are checked against the oracle directly."""
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


def _members(ax, shapes, seed0):
    ops, bs, meta = [], [], []
    for i, ((nr, nz), bc) in enumerate(shapes):
        kappa, q = synth.medium_layered(nr, nz, seed0 + i)
        f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.1, 0.4, 0.05)
        op = ax.op_create(kappa, q, bc_z=bc)
        b = dev(np.zeros((nr, nz)))
        ax.rhs_from_f(op, dev(f), b)
        ops.append(op)
        bs.append(b)
        meta.append((kappa, q, f, bc))
    return ops, bs, meta


def _both(ax, ops, bs, x0s, rtol, maxit, prec, flags):
    """The launch-per-phase batch and the single launch from the same starts."""
    out = []
    for extra in (0, ax.FLAG_SINGLE_LAUNCH):
        xs = [dev(x0) for x0 in x0s]
        code, st = ax.batch_solve(ops, bs, xs, rtol, maxit, prec, flags | extra)
        out.append((code, st, [host(x) for x in xs]))
    return out


def _assert_same(multi, single):
    (cm, sm, xm), (cs, ss, xs) = multi, single
    assert cm == cs
    dr = dx = 0.0
    for k, (a, b) in enumerate(zip(sm, ss)):
        assert a["iters"] == b["iters"] and a["status"] == b["status"], (k, a, b)
        dr = max(dr, abs(a["relres_rec"] - b["relres_rec"]))
        if np.any(xm[k]):
            dx = max(dx, rel(xs[k], xm[k]))
        else:
            assert not np.any(xs[k]), k
    log(f"  single vs launch per phase: ||r||/||b|| {dr:.1e} apart, iterates {dx:.1e} (relative)")
    assert dr <= 1e-13 and dx <= 1e-12


# one-wave transform plans (rows of 256, 512, 1024) and block-wide ones (16,
# 32, 64, 128), ragged row counts, both z boundaries
SHAPES = [((64, 64), 0), ((128, 256), 1), ((256, 128), 0), ((96, 32), 1), ((256, 512), 1), ((32, 16), 0),
          ((18, 1024), 1), ((7, 1024), 0), ((40, 256), 0), ((300, 64), 1)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("pr", [False, True])
def test_single_launch_matches_launch_per_phase(ax, orc, prec, pr):
    log(f"single-launch batch prec={prec} polak_ribiere={pr}")
    ops, bs, meta = _members(ax, SHAPES, 80)
    flags = ax.FLAG_POLAK_RIBIERE if pr else 0
    x0s = [np.zeros(op_shape) for op_shape in ((op.nr, op.nz) for op in ops)]
    multi, single = _both(ax, ops, bs, x0s, 1e-10, 500, prec, flags)
    assert single[0] == ax.OK
    _assert_same(multi, single)
    log(f"  iterations {[s['iters'] for s in single[1]]}")
    # a few members against the oracle directly
    for k in (0, 3, 6):
        kappa, q, f, bc = meta[k]
        oop = orc.operator_from_cells(kappa, q, bc_z=bc)
        err = rel(single[2][k], orc.solve_reference(oop, orc.rhs(oop, f)))
        log(f"  member {k} {SHAPES[k]}: rel err vs oracle {err:.1e}")
        assert err <= 1e-8
    for op in ops:
        op.close()


def test_single_launch_edge_cases(ax):
    """A zero right-hand side (x = 0, no iterations), a start that already
    meets the test, maxit reached by one member only, and two solves in a
    row on the same handles; each as the launch-per-phase form does it."""
    log("single-launch batch edge cases")
    shapes = [((64, 64), 0), ((64, 64), 1), ((48, 256), 0)]
    ops, bs, _ = _members(ax, shapes, 5)
    bs[1].zero_()
    x0s = [np.zeros((64, 64)), np.ones((64, 64)), np.zeros((48, 256))]
    multi, single = _both(ax, ops, bs, x0s, 1e-10, 300, ax.PREC_FP32, 0)
    _assert_same(multi, single)
    assert single[0] == ax.OK and single[1][1]["iters"] == 0 and not single[2][1].any()
    # start from the converged answers: every member stops at its start test
    x0s = [single[2][0], np.zeros((64, 64)), single[2][2]]
    multi, single2 = _both(ax, ops, bs, x0s, 1e-8, 300, ax.PREC_FP32, 0)
    _assert_same(multi, single2)
    assert all(s["iters"] == 0 for s in single2[1])
    # maxit 3: the non-trivial members stop there
    x0s = [np.zeros((64, 64)), np.zeros((64, 64)), np.zeros((48, 256))]
    multi, single3 = _both(ax, ops, bs, x0s, 1e-10, 3, ax.PREC_FP64, ax.FLAG_TRUE_RESIDUAL)
    _assert_same(multi, single3)
    assert single3[0] == ax.ENOTCONV
    assert [s["status"] for s in single3[1]] == [ax.ENOTCONV, ax.OK, ax.ENOTCONV]
    assert [s["iters"] for s in single3[1]] == [3, 0, 3]
    # members with rows of 2048 are refused before anything runs
    k2, q2 = synth.medium_layered(8, 2048, 1)
    with ax.op_create(k2, q2) as op2:
        with pytest.raises(ax.AxipcgError):
            ax.batch_solve([ops[0], op2], [bs[0], dev(np.ones((8, 2048)))],
                           [dev(np.zeros((64, 64))), dev(np.zeros((8, 2048)))], 1e-10, 10, ax.PREC_FP32,
                           ax.FLAG_SINGLE_LAUNCH)
    for op in ops:
        op.close()


def test_single_launch_uneven_batch_of_64(ax):
    """The 64-member uneven batch (N_r, N_z ~ U{256,512,1024}, seeds
    1000+p) in one launch: the launch-per-phase result to rounding."""
    log("single-launch batch of 64 uneven problems")
    probs = [synth.problem_batch_member(p) for p in range(64)]
    ops, bs = [], []
    for pr in probs:
        op = ax.op_create(pr.kappa, pr.q)
        b = dev(np.zeros((pr.nr, pr.nz)))
        ax.rhs_from_f(op, dev(pr.f), b)
        ops.append(op)
        bs.append(b)
    x0s = [np.zeros((pr.nr, pr.nz)) for pr in probs]
    multi, single = _both(ax, ops, bs, x0s, 1e-10, 1000, ax.PREC_FP32, ax.FLAG_TRUE_RESIDUAL)
    assert single[0] == ax.OK
    _assert_same(multi, single)
    assert max(s["relres_true"] for s in single[1]) <= 1e-9
    log(f"  iterations min/max {min(s['iters'] for s in single[1])}/{max(s['iters'] for s in single[1])}")
    for op in ops:
        op.close()
