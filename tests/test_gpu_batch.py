"""Batched PCG over independent problems of different sizes, against the
oracle (each problem solved on its own) and against single-problem solves,
up to the largest member count a batch accepts."""
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


def _member(shape, bc, seed):
    nr, nz = shape
    kappa, q = synth.medium_layered(nr, nz, seed)
    f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.1, 0.4, 0.05)
    return kappa, q, f, bc


# z-lengths with a one-wave transform plan (256, 512, 1024, 2048 in FP32) and
# without (16, 64, 128; 2048 in FP64), so that every transform launch of a
# batch covers problems of one plan while the other launches mix them
SMALL = [((64, 64), 0), ((128, 256), 1), ((256, 128), 0), ((96, 64), 0), ((256, 512), 1), ((32, 16), 0),
         ((18, 1024), 1), ((8, 2048), 0), ((40, 256), 0)]


@pytest.mark.parametrize("prec", [0, 1])
def test_small_uneven_batch_matches_oracle(ax, orc, prec):
    log(f"batch small uneven prec={prec}")
    members = [_member(s, bc, 50 + i) for i, (s, bc) in enumerate(SMALL)]
    ops, bs, xs, refs = [], [], [], []
    for kappa, q, f, bc in members:
        op = ax.op_create(kappa, q, bc_z=bc)
        b = dev(np.zeros(kappa.shape))
        ax.rhs_from_f(op, dev(f), b)
        ops.append(op)
        bs.append(b)
        xs.append(dev(np.zeros(kappa.shape)))
        oop = orc.operator_from_cells(kappa, q, bc_z=bc)
        refs.append(orc.solve_reference(oop, orc.rhs(oop, f)))
    code, st = ax.batch_solve(ops, bs, xs, 1e-10, 500, prec, ax.FLAG_TRUE_RESIDUAL)
    assert code == ax.OK
    for k in range(len(ops)):
        err = rel(host(xs[k]), refs[k])
        log(f"  member {k} {SMALL[k]} iters={st[k]['iters']} true={st[k]['relres_true']:.1e} err={err:.1e}")
        assert st[k]["status"] == ax.OK and st[k]["relres_true"] <= 1e-9 and err <= 1e-8
    # a second solve on the same handles starts from their finished state
    # (stop flags set by the first): it must run the full iteration again
    first = [host(x).copy() for x in xs]
    for x in xs:
        x.zero_()
    code2, st2 = ax.batch_solve(ops, bs, xs, 1e-10, 500, prec, ax.FLAG_TRUE_RESIDUAL)
    assert code2 == ax.OK
    for k in range(len(ops)):
        assert st2[k]["iters"] == st[k]["iters"] and st2[k]["relres_true"] <= 1e-9
        np.testing.assert_array_equal(host(xs[k]), first[k])
    for op in ops:
        op.close()


def test_batch_edge_cases(ax):
    log("batch edge cases")
    kappa, q, f, bc = _member((64, 64), 0, 7)
    op1 = ax.op_create(kappa, q)
    op2 = ax.op_create(kappa, q)
    b1 = dev(np.zeros((64, 64)))
    ax.rhs_from_f(op1, dev(f), b1)
    b2 = dev(np.zeros((64, 64)))           # zero right-hand side
    x1 = dev(np.zeros((64, 64)))
    x2 = dev(np.ones((64, 64)))
    code, st = ax.batch_solve([op1, op2], [b1, b2], [x1, x2], 1e-10, 300)
    assert code == ax.OK and st[1]["iters"] == 0 and not host(x2).any()
    # maxit reached for the non-trivial member only
    x1.zero_()
    code, st = ax.batch_solve([op1, op2], [b1, b2], [x1, x2], 1e-10, 2)
    assert code == ax.ENOTCONV and st[0]["status"] == ax.ENOTCONV and st[1]["status"] == ax.OK
    with pytest.raises(ax.AxipcgError):
        ax.batch_solve([op1, op1], [b1, b1], [x1, x2], 1e-10, 10)   # same handle twice
    op1.close()
    op2.close()


def test_uneven_batch_of_64(ax, orc):
    """The 64-member uneven batch (N_r, N_z ~ U{256,512,1024}, seeds 1000+p):
    every member converges; the eight smallest match the oracle to 1e-8 and all
    agree with single-problem solves to 1e-9."""
    log("batch of 64 uneven problems")
    probs = [synth.problem_batch_member(p) for p in range(64)]
    ops, bs, xs = [], [], []
    for pr in probs:
        op = ax.op_create(pr.kappa, pr.q)
        b = dev(np.zeros((pr.nr, pr.nz)))
        ax.rhs_from_f(op, dev(pr.f), b)
        ops.append(op)
        bs.append(b)
        xs.append(dev(np.zeros((pr.nr, pr.nz))))
    code, st = ax.batch_solve(ops, bs, xs, 1e-10, 1000, ax.PREC_FP32, ax.FLAG_TRUE_RESIDUAL)
    assert code == ax.OK
    assert max(s["relres_true"] for s in st) <= 1e-9
    log(f"  iterations min/max {min(s['iters'] for s in st)}/{max(s['iters'] for s in st)}")
    order = sorted(range(64), key=lambda p: probs[p].nr * probs[p].nz)
    for p in order[:8]:
        pr = probs[p]
        oop = orc.operator_from_cells(pr.kappa, pr.q)
        xr = orc.solve_reference(oop, orc.rhs(oop, pr.f))
        assert rel(host(xs[p]), xr) <= 1e-8, p
    for p in range(64):
        xs1 = dev(np.zeros((probs[p].nr, probs[p].nz)))
        s1 = ax.pcg_solve(ops[p], bs[p], xs1, 1e-10, 1000, ax.PREC_FP32)
        # the batched r-solve sizes its segments for the batch, so partial
        # sums may be added in another order than in the single solve
        assert abs(s1["iters"] - st[p]["iters"]) <= 1
        assert rel(host(xs[p]), host(xs1)) <= 1e-9, p
    for op in ops:
        op.close()


def test_batch_of_the_most_members(ax, orc):
    """A batch of 4096 members (the most batch_solve accepts) of tiny mixed
    shapes and both z boundaries: every member converges by its true
    residual, and every 64th matches the oracle."""
    shapes = [(2, 4), (3, 8), (4, 4), (8, 4), (7, 16), (16, 32)]   # members need nz >= 4
    n = 4096
    log(f"batch of {n} members")
    ops, bs, xs, members = [], [], [], []
    for p in range(n):
        kappa, q, f, bc = _member(shapes[p % len(shapes)], (p // len(shapes)) % 2, 7000 + p)
        op = ax.op_create(kappa, q, bc_z=bc)
        b = dev(np.zeros(kappa.shape))
        ax.rhs_from_f(op, dev(f), b)
        ops.append(op)
        bs.append(b)
        xs.append(dev(np.zeros(kappa.shape)))
        members.append((kappa, q, f, bc))
    code, st = ax.batch_solve(ops, bs, xs, 1e-10, 500, ax.PREC_FP32, ax.FLAG_TRUE_RESIDUAL)
    assert code == ax.OK
    assert all(s["status"] == ax.OK and s["relres_true"] <= 1e-9 for s in st)
    errs = []
    for p in range(0, n, 64):
        kappa, q, f, bc = members[p]
        oop = orc.operator_from_cells(kappa, q, bc_z=bc)
        errs.append(rel(host(xs[p]), orc.solve_reference(oop, orc.rhs(oop, f))))
    log(f"  iters max {max(s['iters'] for s in st)}, sampled max rel err {max(errs):.1e}")
    assert max(errs) <= 1e-8
    for op in ops:
        op.close()
