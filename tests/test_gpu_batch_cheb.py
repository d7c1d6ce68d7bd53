"""The Chebyshev form of eq. (8) over a batch (axipcg_batch_cheb_solve), one
launch per phase over every member, against the oracle's Chebyshev iteration
(the same polynomial, member by member) and its reference solves, and against
single-problem Chebyshev solves."""
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


# one-wave transform plans (rows of 256, 512, 1024, 2048) and block-wide ones
# (16, 32, 64, 128), ragged row counts, both z boundaries
SHAPES = [((64, 64), 0), ((128, 256), 1), ((96, 32), 1), ((256, 512), 0), ((32, 16), 0), ((18, 1024), 1),
          ((8, 2048), 0), ((40, 128), 1)]


def _members(ax, orc, shapes, seed0, rhs="gauss"):
    ops, bs, meta = [], [], []
    for i, ((nr, nz), bc) in enumerate(shapes):
        kappa, q = synth.medium_layered(nr, nz, seed0 + i)
        f = synth.gaussian_source(nr, nz, 1.0, 1.0, 0.1, 0.4, 0.05)
        oop = orc.operator_from_cells(kappa, q, bc_z=bc)
        ops.append(ax.op_create(kappa, q, bc_z=bc))
        b = orc.rhs(oop, f)
        bs.append(b)
        meta.append(oop)
    return ops, bs, meta


def test_batch_iterates_match_oracle(ax, orc):
    """25 steps of every member (FP64 preconditioner, stop test never met)
    against the oracle's three-term iteration from the same start: the same
    polynomial in B^-1 A, so equal to rounding (the bound of the
    single-problem test, scaled as there with the row length)."""
    log("batch Chebyshev iterates vs oracle")
    ops, bs, meta = _members(ax, orc, SHAPES, 30)
    rng = np.random.default_rng(4)
    x0s = [rng.standard_normal(b.shape) * 1e-3 for b in bs]
    xs = [dev(x0) for x0 in x0s]
    k = 25
    code, st = ax.batch_cheb_solve(ops, [dev(b) for b in bs], xs, rtol=1e-30, maxit=k, prec=ax.PREC_FP64)
    assert code == ax.ENOTCONV
    for p, oop in enumerate(meta):
        g1, g2 = orc.energy_bounds(oop)
        yo, _, _, _ = orc.cheb(oop, bs[p], x0s[p], g1, g2, iters=k)
        e = rel(host(xs[p]), yo)
        log(f"  member {p} {SHAPES[p]}: {st[p]['iters']} steps, rel diff {e:.1e}")
        assert st[p]["iters"] == k and st[p]["status"] == ax.ENOTCONV
        assert e <= 1e-11 * max(1, SHAPES[p][0][1] // 1024)
    for op in ops:
        op.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_converged_matches_oracle_and_single_solves(ax, orc, prec):
    log(f"batch Chebyshev converged prec={prec}")
    ops, bs, meta = _members(ax, orc, SHAPES, 40)
    xs = [dev(np.zeros(b.shape)) for b in bs]
    code, st = ax.batch_cheb_solve(ops, [dev(b) for b in bs], xs, rtol=1e-10, maxit=1000, prec=prec,
                                   flags=ax.FLAG_TRUE_RESIDUAL)
    assert code == ax.OK
    for p, oop in enumerate(meta):
        xr = orc.solve_reference(oop, bs[p])
        err = rel(host(xs[p]), xr)
        y = dev(np.zeros(bs[p].shape))
        s1 = ax.cheb_solve(ops[p], dev(bs[p]), y, rtol=1e-10, maxit=1000, prec=prec)
        log(f"  member {p} {SHAPES[p]}: iters {st[p]['iters']} (single {s1['iters']}), "
            f"true relres {st[p]['relres_true']:.1e}, err {err:.1e}")
        assert st[p]["status"] == ax.OK and st[p]["relres_rec"] <= 1e-10 and st[p]["relres_true"] <= 1e-9
        assert err <= 1e-8
        # the single solve runs the r-solves in strips where the batch runs
        # them per mode: rounding may move the stop by one iteration
        assert abs(st[p]["iters"] - s1["iters"]) <= 1
        assert rel(host(xs[p]), host(y)) <= 1e-8
    for op in ops:
        op.close()


def test_batch_explicit_bounds_and_edge_cases(ax, orc):
    log("batch Chebyshev bounds and edge cases")
    shapes = [((64, 64), 0), ((64, 64), 1), ((48, 256), 0)]
    ops, bs, meta = _members(ax, orc, shapes, 9)
    bd = [dev(b) for b in bs]
    bd[1].zero_()
    # each member's own bounds passed explicitly: the same launches as NULL
    g = [ax.op_bounds(op) for op in ops]
    xa = [dev(np.zeros(b.shape)) for b in bs]
    xb = [dev(np.zeros(bs[0].shape)), dev(np.ones(bs[1].shape)), dev(np.zeros(bs[2].shape))]
    ca, sa = ax.batch_cheb_solve(ops, bd, xa, rtol=1e-10, prec=ax.PREC_FP32)
    cb, sb = ax.batch_cheb_solve(ops, bd, xb, gamma1=[v[0] for v in g], gamma2=[v[1] for v in g], rtol=1e-10,
                                 prec=ax.PREC_FP32)
    assert ca == cb == ax.OK
    # b = 0: x = 0 without iterating, from any start
    assert sb[1]["iters"] == 0 and not host(xb[1]).any()
    for p in (0, 2):
        assert sa[p]["iters"] == sb[p]["iters"]
        np.testing.assert_array_equal(host(xa[p]), host(xb[p]))
    # maxit reached by the non-trivial members only
    xc = [dev(np.zeros(b.shape)) for b in bs]
    code, sc = ax.batch_cheb_solve(ops, bd, xc, rtol=1e-10, maxit=3, prec=ax.PREC_FP64)
    assert code == ax.ENOTCONV
    assert [s["status"] for s in sc] == [ax.ENOTCONV, ax.OK, ax.ENOTCONV]
    assert [s["iters"] for s in sc] == [3, 0, 3]
    # an interval that is not a bound pair is refused before anything runs
    with pytest.raises(ax.AxipcgError):
        ax.batch_cheb_solve(ops, bd, xc, gamma1=[2.0, 2.0, 2.0], gamma2=[1.0, 1.0, 1.0])
    for op in ops:
        op.close()


def test_batch_cheb_uneven_batch_of_64(ax):
    """The 64-member uneven batch: every member converges by its true
    residual; the iterations against the batched PCG's on the same operators.
    These media have cells with q = 0, where eq. (10) bounds B^-1 A from below
    only when B has no q term: the operators take qbar = 0."""
    log("batch Chebyshev, 64 uneven problems")
    probs = [synth.problem_batch_member(p) for p in range(64)]
    ops, bs = [], []
    for pr in probs:
        op = ax.op_create(pr.kappa, pr.q, qbar=0.0)
        b = dev(np.zeros((pr.nr, pr.nz)))
        ax.rhs_from_f(op, dev(pr.f), b)
        ops.append(op)
        bs.append(b)
    xs = [dev(np.zeros((pr.nr, pr.nz))) for pr in probs]
    code, st = ax.batch_cheb_solve(ops, bs, xs, rtol=1e-10, maxit=1000, prec=ax.PREC_FP32,
                                   flags=ax.FLAG_TRUE_RESIDUAL)
    assert code == ax.OK and max(s["relres_true"] for s in st) <= 1e-9
    xp = [dev(np.zeros((pr.nr, pr.nz))) for pr in probs]
    code, sp = ax.batch_solve(ops, bs, xp, 1e-10, 1000, ax.PREC_FP32)
    assert code == ax.OK
    it_c = [s["iters"] for s in st]
    it_p = [s["iters"] for s in sp]
    log(f"  Chebyshev iterations {min(it_c)}-{max(it_c)}, PCG {min(it_p)}-{max(it_p)}")
    assert max(rel(host(a), host(b)) for a, b in zip(xs, xp)) <= 1e-8
    for op in ops:
        op.close()
