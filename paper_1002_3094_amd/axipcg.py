"""Thin ctypes binding of the axipcg C-ABI (``include/axipcg.h``).

Argument marshalling only: every numerical step runs in the HIP library
``libaxipcg.so`` built for gfx950.  Device arrays are torch tensors
(float64, contiguous, on the current HIP device); host arrays are numpy
arrays.  The stream defaults to torch's current stream.  Loading fails loudly
when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# AXIPCG_LIB selects another build of the same library (the host-sanitized
# one of build.build_host_sanitized, for CPU-only checks)
LIB_PATH = os.environ.get("AXIPCG_LIB") or os.path.join(_HERE, "libaxipcg.so")

OK, ENOTCONV, EINVAL, ENOMEM, EDEVICE, EBREAKDOWN = 0, 1, -1, -2, -3, -4
Z_DIRICHLET, Z_NEUMANN = 0, 1
GRID_NODES = 0x100   # OR into bc_z: the paper's node grid (h = l / (N - 1/2)); Neumann z only
PREC_FP64, PREC_FP32 = 0, 1
FLAG_TRUE_RESIDUAL, FLAG_POLAK_RIBIERE, FLAG_SINGLE_LAUNCH = 1, 2, 4
KERNEL_NONE, KERNEL_SPMV, KERNEL_ZFWD, KERNEL_TRIDIAG, KERNEL_ZINV = -1, 0, 1, 2, 3

_lib = None
# Handles still open: released by an exit hook, before the interpreter and
# the HIP runtime shut down, never from a finaliser during shutdown.
_live = weakref.WeakSet()


def _release_all():
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass


atexit.register(_release_all)


class AxipcgError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int),
                ("relres_rec", ctypes.c_double), ("relres_true", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i, _d, _u = ctypes.c_int, ctypes.c_double, ctypes.c_uint

SIGNATURES = {
    "axipcg_op_create": ([_i, _i, _d, _d, _i, _dp, _dp, _d, _d, _vp, ctypes.POINTER(_vp)], _i),
    "axipcg_op_create_faces": ([_i, _i, _d, _d, _i, _dp, _dp, _dp, _d, _d, _vp, ctypes.POINTER(_vp)], _i),
    "axipcg_op_destroy": ([_vp], None),
    "axipcg_op_info": ([_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), _dp, _dp], _i),
    "axipcg_apply_A": ([_vp, _vp, _vp, _vp], _i),
    "axipcg_rhs_from_f": ([_vp, _vp, _vp, _vp], _i),
    "axipcg_precond_apply": ([_vp, _vp, _vp, _i, _vp], _i),
    "axipcg_residual_norm": ([_vp, _vp, _vp, _dp, _vp], _i),
    "axipcg_op_set_fused": ([_vp, _i], _i),
    "axipcg_op_set_strips": ([_vp, _i], _i),
    "axipcg_op_strips_info": ([_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)], _i),
    "axipcg_op_bounds": ([_vp, _dp, _dp], _i),
    "axipcg_cheb_solve": ([_vp, _vp, _vp, _d, _d, _d, _i, _i, ctypes.POINTER(Stats), _vp], _i),
    "axipcg_op_fused_info": ([_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)], _i),
    "axipcg_pcg_solve": ([_vp, _vp, _vp, _d, _i, _i, _u, ctypes.POINTER(Stats), _vp], _i),
    "axipcg_batch_solve": ([_i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _d, _i, _i, _u,
                            ctypes.POINTER(Stats), _vp], _i),
    "axipcg_op_bounds_lanczos": ([_vp, _vp, _i, _i, _dp, _dp, ctypes.POINTER(_i), _vp], _i),
    "axipcg_batch_cheb_solve": ([_i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                 ctypes.POINTER(_d), ctypes.POINTER(_d), _d, _i, _i, _u, ctypes.POINTER(Stats), _vp],
                                _i),
    "axipcg_laguerre_coeffs": ([_i, _d, _i, _d, _dp, _dp, _vp], _i),
    "axipcg_laguerre_rhs": ([_vp, _d, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp], _i),
    "axipcg_guess_extrap": ([_vp, _vp, _vp, _vp, _vp, _dp, ctypes.POINTER(_i), _vp], _i),
    "axipcg_guess_poly": ([_vp, _vp, ctypes.POINTER(_vp), _i, _vp, _dp, ctypes.POINTER(_i), _vp], _i),
    "axipcg_laguerre_coeffs_alpha": ([_i, _i, _d, _i, _d, _dp, _dp, _vp], _i),
    "axipcg_laguerre_coeffs_alpha_noalloc": ([_i, _i, _d, _i, _d, _dp, _dp, _vp], _i),
    "axipcg_laguerre_rhs_alpha": ([_vp, _i, _i, _d, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp], _i),
    "axipcg_gather": ([_vp, _vp, _vp, _i, _vp, _vp], _i),
    "axipcg_laguerre_synth": ([_i, _i, _d, _i, _vp, _i, _d, _vp, _vp], _i),
    "axipcg_nn_num_params": ([], _i),
    "axipcg_nn_create": ([_i, _i, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_vp)], _i),
    "axipcg_nn_destroy": ([_vp], None),
    "axipcg_nn_get_params": ([_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)], _i),
    "axipcg_nn_set_params": ([_vp, ctypes.POINTER(ctypes.c_float)], _i),
    "axipcg_nn_forward": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], _i),
    "axipcg_nn_backward": ([_vp, _vp, _vp, _vp, _vp, _dp, _vp], _i),
    "axipcg_nn_adam": ([_vp, _d, _d, _d, _d, _vp], _i),
    "axipcg_nn_set_base": ([_vp, _i], _i),
    "axipcg_nn_get_base": ([_vp], _i),
    "axipcg_nn_backward_poly": ([_vp, _vp, ctypes.POINTER(_vp), _i, _vp, _dp, _vp], _i),
    "axipcg_nn_guess": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _dp, ctypes.POINTER(_i), _vp], _i),
    "axipcg_nn_guess_poly": ([_vp, _vp, _vp, ctypes.POINTER(_vp), _i, _vp, _vp, _dp, ctypes.POINTER(_i), _vp], _i),
    "axipcg_series_step": ([_vp, _vp, _i, _d, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i, _i, _d, _i, _i,
                            ctypes.POINTER(Stats), _vp], _i),
    "axipcg_series_run": ([_vp, _vp, _i, _i, _dp, _i, _i, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp), _vp, _i, _i,
                           _d, _i, _i, ctypes.POINTER(Stats), ctypes.POINTER(_i), _vp], _i),
    "axipcg_series_run_alpha": ([_vp, _i, _i, _i, _dp, _i, _i, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp), _vp, _i, _vp,
                                 _i, _i, _d, _i, _i, ctypes.POINTER(Stats), ctypes.POINTER(_i), _vp], _i),
    "axipcg_profile_select": ([_vp, _i, _i], _i),
    "axipcg_profile_read": ([_vp, _dp, ctypes.POINTER(ctypes.c_longlong), _i], _i),
    "axipcg_strerror": ([_i], ctypes.c_char_p),
    "axipcg_last_error": ([], ctypes.c_char_p),
}


def lib():
    """Load libaxipcg.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_1002_3094_amd/build.py")
        h = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = res
        _lib = h
    return _lib


def _check(code: int, where: str, allow=(OK,)):
    if code in allow:
        return code
    msg = lib().axipcg_last_error().decode() or lib().axipcg_strerror(code).decode()
    raise AxipcgError(code, where, msg)


def _host(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _hp(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _dev(t, name="array"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    return _vp(t.data_ptr())


def _opt_dev(t, name):
    return None if t is None else _dev(t, name)


def _stream(stream):
    if stream is not None:
        return _vp(stream if isinstance(stream, int) else stream.cuda_stream)
    import torch
    return _vp(torch.cuda.current_stream().cuda_stream)


class Op:
    """Owning wrapper of an axipcg_op_t handle."""

    def __init__(self, handle: int):
        self.handle = _vp(handle)
        _live.add(self)
        n_r, n_z, kb, qb = _i(), _i(), _d(), _d()
        _check(lib().axipcg_op_info(self.handle, ctypes.byref(n_r), ctypes.byref(n_z),
                                    ctypes.byref(kb), ctypes.byref(qb)), "op_info")
        self.nr, self.nz, self.kbar, self.qbar = n_r.value, n_z.value, kb.value, qb.value

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().axipcg_op_destroy(self.handle)
        self.handle = None
        _live.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the exit hook has already released it (or
        # the runtime is going away): touch nothing (the check is bound at
        # definition, since module globals may already be cleared then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def op_create(kappa, q, lr=1.0, lz=1.0, bc_z=Z_DIRICHLET, kbar=-1.0, qbar=-1.0, stream=None) -> Op:
    kappa, q = _host(kappa), _host(q)
    if kappa.ndim != 2 or q.shape != kappa.shape:
        raise ValueError("kappa and q must be [nr][nz] arrays of the same shape")
    nr, nz = kappa.shape
    out = _vp()
    _check(lib().axipcg_op_create(nr, nz, lr, lz, bc_z, _hp(kappa), _hp(q), kbar, qbar,
                                  _stream(stream), ctypes.byref(out)), "op_create")
    return Op(out.value)


def op_create_faces(kappa_r, kappa_z, q, lr=1.0, lz=1.0, bc_z=Z_DIRICHLET, kbar=1.0, qbar=0.0,
                    stream=None) -> Op:
    kappa_r, kappa_z, q = _host(kappa_r), _host(kappa_z), _host(q)
    nr, nz = q.shape
    if kappa_r.shape != (nr, nz) or kappa_z.shape != (nr, nz + 1):
        raise ValueError("kappa_r must be [nr][nz] and kappa_z [nr][nz+1]")
    out = _vp()
    _check(lib().axipcg_op_create_faces(nr, nz, lr, lz, bc_z, _hp(kappa_r), _hp(kappa_z), _hp(q),
                                        kbar, qbar, _stream(stream), ctypes.byref(out)),
           "op_create_faces")
    return Op(out.value)


def op_destroy(op: Op):
    op.close()


def apply_A(op: Op, x, y, stream=None):
    _check(lib().axipcg_apply_A(op.handle, _dev(x, "x"), _dev(y, "y"), _stream(stream)), "apply_A")


def rhs_from_f(op: Op, f, b, stream=None):
    _check(lib().axipcg_rhs_from_f(op.handle, _dev(f, "f"), _dev(b, "b"), _stream(stream)), "rhs_from_f")


def precond_apply(op: Op, r, z, prec=PREC_FP32, stream=None):
    _check(lib().axipcg_precond_apply(op.handle, _dev(r, "r"), _dev(z, "z"), prec, _stream(stream)),
           "precond_apply")


def op_set_fused(op: Op, enable: bool):
    _check(lib().axipcg_op_set_fused(op.handle, int(bool(enable))), "op_set_fused")


def op_set_strips(op: Op, rows):
    """rows: False/0 off, True/1 on (default height), 4 or 8 rows per strip."""
    _check(lib().axipcg_op_set_strips(op.handle, int(rows)), "op_set_strips")


def op_strips_info(op: Op, prec=PREC_FP32):
    """(active, strips) of the strip-partitioned preconditioner for prec."""
    act, strips = _i(), _i()
    _check(lib().axipcg_op_strips_info(op.handle, prec, ctypes.byref(act), ctypes.byref(strips)), "op_strips_info")
    return bool(act.value), strips.value


FUSED_APPLY, FUSED_PCG = 0, 1


def op_fused_info(op: Op, kind=FUSED_APPLY, want_errors=False):
    """(active, strips, barrier_errors or None) of the single-launch form for
    standalone FP32 applies (kind 0) or FP32 PCG iterations (kind 1);
    want_errors synchronises the device."""
    act, strips, errs = _i(), _i(), _i()
    _check(lib().axipcg_op_fused_info(op.handle, kind, ctypes.byref(act), ctypes.byref(strips),
                                      ctypes.byref(errs) if want_errors else None), "op_fused_info")
    return bool(act.value), strips.value, (errs.value if want_errors else None)


def residual_norm(op: Op, b, x, stream=None):
    out = np.zeros(2)
    _check(lib().axipcg_residual_norm(op.handle, _dev(b, "b"), _dev(x, "x"), _hp(out), _stream(stream)),
           "residual_norm")
    return float(out[0]), float(out[1])


def pcg_solve(op: Op, b, x, rtol=1e-10, maxit=1000, prec=PREC_FP32, flags=0, stream=None,
              allow_notconv=True) -> dict:
    st = Stats()
    code = lib().axipcg_pcg_solve(op.handle, _dev(b, "b"), _dev(x, "x"), rtol, maxit, prec, flags,
                                  ctypes.byref(st), _stream(stream))
    _check(code, "pcg_solve", allow=(OK, ENOTCONV) if allow_notconv else (OK,))
    d = st.as_dict()
    d["code"] = code
    return d


def op_bounds(op: Op):
    g1, g2 = _d(), _d()
    _check(lib().axipcg_op_bounds(op.handle, ctypes.byref(g1), ctypes.byref(g2)), "op_bounds")
    return g1.value, g2.value


def op_bounds_lanczos(op: Op, b, steps=20, prec=PREC_FP64, stream=None):
    """Extreme Ritz values of B^{-1} A from `steps` PCG steps on A x = b:
    (gamma1, gamma2, steps done)."""
    g1, g2, k = _d(), _d(), _i()
    _check(lib().axipcg_op_bounds_lanczos(op.handle, _dev(b, "b"), int(steps), prec, ctypes.byref(g1),
                                          ctypes.byref(g2), ctypes.byref(k), _stream(stream)),
           "op_bounds_lanczos")
    return g1.value, g2.value, k.value


def cheb_solve(op: Op, b, x, gamma1=0.0, gamma2=0.0, rtol=1e-10, maxit=1000, prec=PREC_FP32, stream=None,
               allow_notconv=True) -> dict:
    st = Stats()
    code = lib().axipcg_cheb_solve(op.handle, _dev(b, "b"), _dev(x, "x"), gamma1, gamma2, rtol, maxit, prec,
                                   ctypes.byref(st), _stream(stream))
    _check(code, "cheb_solve", allow=(OK, ENOTCONV) if allow_notconv else (OK,))
    d = st.as_dict()
    d["code"] = code
    return d


def batch_solve(ops, bs, xs, rtol=1e-10, maxit=1000, prec=PREC_FP32, flags=0, stream=None,
                allow_notconv=True):
    n = len(ops)
    if not (len(bs) == len(xs) == n):
        raise ValueError("ops, bs and xs must have the same length")
    h = (_vp * n)(*[o.handle.value for o in ops])
    bp = (_vp * n)(*[_dev(t, "b").value for t in bs])
    xp = (_vp * n)(*[_dev(t, "x").value for t in xs])
    st = (Stats * n)()
    code = lib().axipcg_batch_solve(n, h, bp, xp, rtol, maxit, prec, flags, st, _stream(stream))
    _check(code, "batch_solve", allow=(OK, ENOTCONV) if allow_notconv else (OK,))
    return code, [s.as_dict() for s in st]


def batch_cheb_solve(ops, bs, xs, gamma1=None, gamma2=None, rtol=1e-10, maxit=1000, prec=PREC_FP32, flags=0,
                     stream=None, allow_notconv=True):
    """The Chebyshev form for every member of a batch; gamma1, gamma2: a
    bound per member (None: each member's own energy bounds)."""
    n = len(ops)
    if not (len(bs) == len(xs) == n):
        raise ValueError("ops, bs and xs must have the same length")
    h = (_vp * n)(*[o.handle.value for o in ops])
    bp = (_vp * n)(*[_dev(t, "b").value for t in bs])
    xp = (_vp * n)(*[_dev(t, "x").value for t in xs])
    g1 = None if gamma1 is None else (_d * n)(*[float(v) for v in gamma1])
    g2 = None if gamma2 is None else (_d * n)(*[float(v) for v in gamma2])
    st = (Stats * n)()
    code = lib().axipcg_batch_cheb_solve(n, h, bp, xp, g1, g2, rtol, maxit, prec, flags, st, _stream(stream))
    _check(code, "batch_cheb_solve", allow=(OK, ENOTCONV) if allow_notconv else (OK,))
    return code, [s.as_dict() for s in st]


def laguerre_coeffs(n: int, eta: float, f_samples, t_max: float, stream=None) -> np.ndarray:
    f = _host(f_samples)
    g = np.zeros(n)
    _check(lib().axipcg_laguerre_coeffs(n, eta, f.size, t_max, _hp(f), _hp(g), _stream(stream)),
           "laguerre_coeffs")
    return g


def laguerre_rhs(op: Op, g_m: float, src_i: int, src_k: int, S1, S2, b, u_prev=None, coef=None,
                 stream=None):
    _check(lib().axipcg_laguerre_rhs(op.handle, g_m, src_i, src_k, _opt_dev(coef, "coef"),
                                     _opt_dev(u_prev, "u_prev"), _dev(S1, "S1"), _dev(S2, "S2"),
                                     _dev(b, "b"), _stream(stream)), "laguerre_rhs")


def laguerre_coeffs_alpha(n: int, alpha: int, eta: float, f_samples, t_max: float, stream=None) -> np.ndarray:
    f = _host(f_samples)
    g = np.zeros(n)
    _check(lib().axipcg_laguerre_coeffs_alpha(n, alpha, eta, len(f), t_max, _hp(f), _hp(g), _stream(stream)),
           "laguerre_coeffs_alpha")
    return g


def laguerre_coeffs_alpha_noalloc(n: int, alpha: int, eta: float, f_samples, t_max: float,
                                  stream=None) -> np.ndarray:
    f = _host(f_samples)
    g = np.zeros(n)
    _check(lib().axipcg_laguerre_coeffs_alpha_noalloc(n, alpha, eta, len(f), t_max, _hp(f), _hp(g),
                                                      _stream(stream)), "laguerre_coeffs_alpha_noalloc")
    return g


def laguerre_rhs_alpha(op: Op, m: int, alpha: int, g_m: float, src_i: int, src_k: int, S1, S2, b, u_prev=None,
                       coef=None, stream=None):
    _check(lib().axipcg_laguerre_rhs_alpha(op.handle, m, alpha, g_m, src_i, src_k, _opt_dev(coef, "coef"),
                                           _opt_dev(u_prev, "u_prev"), _dev(S1, "S1"), _dev(S2, "S2"),
                                           _dev(b, "b"), _stream(stream)), "laguerre_rhs_alpha")


def _dev_any(t, name, dtype):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous device tensor of {dtype}")
    return _vp(t.data_ptr())


def gather(op: Op, u, idx, out, stream=None):
    """out[j] = u.flatten()[idx[j]] (idx: int64 device tensor; NaN where out of range)."""
    import torch
    n = idx.numel()
    if out.numel() != n:
        raise ValueError("out and idx must have the same length")
    _check(lib().axipcg_gather(op.handle, _dev(u, "u"), _dev_any(idx, "idx", torch.int64), n,
                               _dev(out, "out"), _stream(stream)), "gather")


def laguerre_synth(alpha: int, eta: float, Q, nt: int, t_max: float, traces, stream=None):
    """traces[r][j] = sum_m Q[m][r] phi_m(t_j) (Q [n][nrec], traces [nrec][nt], device float64)."""
    n, nrec = Q.shape
    if tuple(traces.shape) != (nrec, nt):
        raise ValueError("traces must be [nrec][nt]")
    _check(lib().axipcg_laguerre_synth(n, alpha, eta, nrec, _dev(Q, "Q"), nt, t_max, _dev(traces, "traces"),
                                       _stream(stream)), "laguerre_synth")


def guess_extrap(op: Op, b, u1, u2, x, stream=None, want_info=False):
    """Best of u1 and 2 u1 - u2 by residual into x; returns (residual norms
    [extrapolation, previous], choice) when want_info (which synchronises)."""
    res = np.zeros(2)
    choice = _i()
    _check(lib().axipcg_guess_extrap(op.handle, _dev(b, "b"), _dev(u1, "u1"), _dev(u2, "u2"), _dev(x, "x"),
                                     _hp(res) if want_info else None,
                                     ctypes.byref(choice) if want_info else None, _stream(stream)),
           "guess_extrap")
    return (res, choice.value) if want_info else None


def guess_poly(op: Op, b, hist: list, x, stream=None, want_info=False):
    """Polynomial extrapolation of order 0 .. len(hist) - 1 through hist =
    [u_{m-1}, u_{m-2}, ...] (1 to 7 arrays) with the smallest residual into
    x; returns (residual norms by order, chosen order) when want_info (which
    synchronises)."""
    k = len(hist)
    res = np.zeros(max(k, 1))
    choice = _i()
    ptrs = (_vp * max(k, 1))(*[_dev(t, "hist") for t in hist])
    _check(lib().axipcg_guess_poly(op.handle, _dev(b, "b"), ptrs, k, _dev(x, "x"), _hp(res) if want_info else None,
                                   ctypes.byref(choice) if want_info else None, _stream(stream)), "guess_poly")
    return (res, choice.value) if want_info else None


def _fp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def nn_num_params() -> int:
    return int(lib().axipcg_nn_num_params())


class Net:
    """Owning wrapper of an axipcg_nn_t handle (learned initial guess)."""

    def __init__(self, handle: int, nr: int, nz: int):
        self.handle = _vp(handle)
        _live.add(self)
        self.nr, self.nz = nr, nz

    def close(self):
        if self.handle is not None and self.handle.value:
            lib().axipcg_nn_destroy(self.handle)
        self.handle = None
        _live.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the exit hook has already released it (or
        # the runtime is going away): touch nothing (the check is bound at
        # definition, since module globals may already be cleared then)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def nn_create(nr: int, nz: int, params) -> Net:
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != nn_num_params():
        raise ValueError(f"expected {nn_num_params()} parameters, got {p.size}")
    out = _vp()
    _check(lib().axipcg_nn_create(nr, nz, _fp(p), ctypes.byref(out)), "nn_create")
    return Net(out.value, nr, nz)


def nn_destroy(net: Net):
    net.close()


def nn_get_params(net: Net):
    """Return (params, grads) as host float32 arrays."""
    p = np.zeros(nn_num_params(), dtype=np.float32)
    g = np.zeros(nn_num_params(), dtype=np.float32)
    _check(lib().axipcg_nn_get_params(net.handle, _fp(p), _fp(g)), "nn_get_params")
    return p, g


def nn_set_params(net: Net, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != nn_num_params():
        raise ValueError(f"expected {nn_num_params()} parameters, got {p.size}")
    _check(lib().axipcg_nn_set_params(net.handle, _fp(p)), "nn_set_params")


def nn_forward(net: Net, u1, u2, b, kappa, guess, stream=None):
    _check(lib().axipcg_nn_forward(net.handle, _dev(u1, "u1"), _dev(u2, "u2"), _dev(b, "b"),
                                   _dev(kappa, "kappa"), _dev(guess, "guess"), _stream(stream)), "nn_forward")


def nn_backward(op: Op, net: Net, u1, u2, u_target, stream=None, want_loss=True):
    loss = np.zeros(1)
    _check(lib().axipcg_nn_backward(op.handle, net.handle, _dev(u1, "u1"), _dev(u2, "u2"),
                                    _dev(u_target, "u_target"), _hp(loss) if want_loss else None,
                                    _stream(stream)), "nn_backward")
    return float(loss[0]) if want_loss else None


def nn_backward_poly(op: Op, net: Net, hist: list, u_target, stream=None, want_loss=True):
    """nn_backward for any base order: hist as read by the last nn_guess_poly."""
    loss = np.zeros(1)
    k = len(hist)
    ptrs = (_vp * max(k, 1))(*[_dev(t, "hist") for t in hist])
    _check(lib().axipcg_nn_backward_poly(op.handle, net.handle, ptrs, k, _dev(u_target, "u_target"),
                                         _hp(loss) if want_loss else None, _stream(stream)), "nn_backward_poly")
    return float(loss[0]) if want_loss else None


def nn_set_base(net: Net, order: int):
    """Order of the polynomial extrapolation the network corrects (1..6)."""
    _check(lib().axipcg_nn_set_base(net.handle, int(order)), "nn_set_base")


def nn_get_base(net: Net) -> int:
    return int(lib().axipcg_nn_get_base(net.handle))


def nn_adam(net: Net, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().axipcg_nn_adam(net.handle, lr, beta1, beta2, eps, _stream(stream)), "nn_adam")


GUESS_PREV, GUESS_EXTRAP, GUESS_NN = 0, 1, 2


def nn_guess(op: Op, net: Net, b, u1, u2, kappa, x, stream=None, want_info=True):
    """Guarded guess into x; returns (residual norms [network, extrapolation,
    previous], choice) when want_info (which synchronises), else None."""
    phi = np.zeros(3)
    choice = _i()
    _check(lib().axipcg_nn_guess(op.handle, net.handle, _dev(b, "b"), _dev(u1, "u1"), _dev(u2, "u2"),
                                 _dev(kappa, "kappa"), _dev(x, "x"), _hp(phi) if want_info else None,
                                 ctypes.byref(choice) if want_info else None, _stream(stream)), "nn_guess")
    return (phi, choice.value) if want_info else None


def nn_guess_poly(op: Op, net: Net, b, hist: list, kappa, x, stream=None, want_info=True):
    """The learned guess among the polynomial extrapolations through hist
    (2 to 7 arrays); returns (residual norms [orders..., network], choice:
    the order, or len(hist) for the network) when want_info (which
    synchronises), else None."""
    k = len(hist)
    phi = np.zeros(k + 1)
    choice = _i()
    ptrs = (_vp * max(k, 1))(*[_dev(t, "hist") for t in hist])
    _check(lib().axipcg_nn_guess_poly(op.handle, net.handle, _dev(b, "b"), ptrs, k, _dev(kappa, "kappa"),
                                      _dev(x, "x"), _hp(phi) if want_info else None,
                                      ctypes.byref(choice) if want_info else None, _stream(stream)),
           "nn_guess_poly")
    return (phi, choice.value) if want_info else None


# initial-guess modes of series_step / series_run; the polynomial ones read
# POLY_HISTORY earlier harmonics and exist in series_run only
SERIES_GUESS = {"zero": 0, "prev": 1, "extrap": 2, "nn": 3, "poly": 4, "nn_poly": 5}
POLY_HISTORY = 7


def history_len(guess: str) -> int:
    """Earlier harmonics a guess mode reads."""
    return POLY_HISTORY if guess in ("poly", "nn_poly") else 2


def series_step(op: Op, m: int, g_m: float, src_i: int, src_k: int, S1, S2, b, u1, u2, x, guess: str,
                solver: str = "pcg", net=None, kappa=None, coef=None, rtol=1e-10, maxit=1000, prec=PREC_FP32,
                stream=None, allow_notconv=True) -> dict:
    """Harmonic m of a Laguerre series in one call: right-hand side into b,
    initial guess into x, then the solve (PCG or Chebyshev)."""
    st = Stats()
    code = lib().axipcg_series_step(op.handle, net.handle if net is not None else None, m, g_m, src_i, src_k,
                                    _opt_dev(coef, "coef"), _dev(S1, "S1"), _dev(S2, "S2"), _dev(b, "b"),
                                    _dev(u1, "u1"), _dev(u2, "u2"), _opt_dev(kappa, "kappa"), _dev(x, "x"),
                                    SERIES_GUESS[guess], {"pcg": 0, "cheb": 1}[solver], rtol, maxit, prec,
                                    ctypes.byref(st), _stream(stream))
    _check(code, "series_step", allow=(OK, ENOTCONV) if allow_notconv else (OK,))
    d = st.as_dict()
    d["code"] = code
    return d


def series_run(op: Op, m0: int, g, src_i: int, src_k: int, S1, S2, b, u: list, guess: str,
               solver: str = "pcg", net=None, kappa=None, coef=None, rtol=1e-10, maxit=1000, prec=PREC_FP32,
               stream=None, allow_notconv=True):
    """Harmonics m0 .. m0 + len(g) - 1 in one call (see series_step).  u is a
    list of device arrays [u_{m0-1}, u_{m0-2}, ..., work]: three, or eight for
    the polynomial guesses; it is rotated in place so that afterwards u[0]
    holds the last solution, u[1] the one before, and so on.  Returns (code,
    per-harmonic stats dicts)."""
    gv = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    count = int(gv.size)
    nu = history_len(guess) + 1
    if len(u) != nu:
        raise ValueError(f"guess {guess!r} needs {nu} arrays in u")
    ptrs = (_vp * nu)(*[_dev(t, "u") for t in u])
    by_ptr = {t.data_ptr(): t for t in u}
    st = (Stats * max(count, 1))()
    done = _i()
    code = lib().axipcg_series_run(op.handle, net.handle if net is not None else None, m0, count,
                                   gv.ctypes.data_as(_dp), src_i, src_k, _opt_dev(coef, "coef"), _dev(S1, "S1"),
                                   _dev(S2, "S2"), _dev(b, "b"), ptrs, _opt_dev(kappa, "kappa"), SERIES_GUESS[guess],
                                   {"pcg": 0, "cheb": 1}[solver], rtol, maxit, prec, st, ctypes.byref(done),
                                   _stream(stream))
    u[:] = [by_ptr[ptrs[j]] for j in range(nu)]
    _check(code, "series_run", allow=(OK, ENOTCONV) if allow_notconv else (OK,))
    return code, [st[j].as_dict() for j in range(done.value)]


def series_run_alpha(op: Op, m0: int, alpha: int, g, src_i: int, src_k: int, coef, S1, S2, b, u: list, rec_idx, Q,
                     guess: str, solver: str = "pcg", rtol=1e-10, maxit=1000, prec=PREC_FP32, stream=None,
                     allow_notconv=True):
    """The paper's pipeline over harmonics m0 .. m0 + len(g) - 1 in one call:
    right-hand side with alpha, zero or previous guess, solve, receiver
    samples into Q[m] (Q device [>= m0 + len(g)][n_rec], rec_idx int64 device
    or None).  u is [u_{m0-1}, work], or [u_{m0-1}, ..., u_{m0-7}, work] for
    guess 'poly', rotated in place after each harmonic.  Returns (code,
    per-harmonic stats dicts)."""
    import torch
    if guess not in ("zero", "prev", "poly"):
        raise ValueError("guess must be 'zero', 'prev' or 'poly'")
    nu = (POLY_HISTORY if guess == "poly" else 1) + 1
    if len(u) != nu:
        raise ValueError(f"guess {guess!r} needs {nu} arrays in u")
    gv = np.ascontiguousarray(np.asarray(g, dtype=np.float64))
    count = int(gv.size)
    n_rec = 0 if rec_idx is None else int(rec_idx.numel())
    if n_rec:
        if Q.dim() != 2 or Q.shape[1] != n_rec or Q.shape[0] < m0 + count:
            raise ValueError("Q must be [>= m0 + count][n_rec]")
    ptrs = (_vp * nu)(*[_dev(t, "u") for t in u])
    by_ptr = {t.data_ptr(): t for t in u}
    st = (Stats * max(count, 1))()
    done = _i()
    code = lib().axipcg_series_run_alpha(op.handle, m0, count, alpha, gv.ctypes.data_as(_dp), src_i, src_k,
                                         _opt_dev(coef, "coef"), _dev(S1, "S1"), _dev(S2, "S2"), _dev(b, "b"), ptrs,
                                         _dev_any(rec_idx, "rec_idx", torch.int64) if n_rec else None, n_rec,
                                         _dev(Q, "Q") if n_rec else None, SERIES_GUESS[guess],
                                         {"pcg": 0, "cheb": 1}[solver], rtol, maxit, prec, st, ctypes.byref(done),
                                         _stream(stream))
    u[:] = [by_ptr[ptrs[j]] for j in range(nu)]
    _check(code, "series_run_alpha", allow=(OK, ENOTCONV) if allow_notconv else (OK,))
    return code, [st[j].as_dict() for j in range(done.value)]


def profile_select(op: Op, kernel: int, every: int = 1):
    _check(lib().axipcg_profile_select(op.handle, kernel, every), "profile_select")


def profile_read(op: Op, reset: bool = False):
    ms = ctypes.c_double()
    n = ctypes.c_longlong()
    _check(lib().axipcg_profile_read(op.handle, ctypes.byref(ms), ctypes.byref(n), int(reset)), "profile_read")
    return ms.value, n.value


def strerror(code: int) -> str:
    return lib().axipcg_strerror(code).decode()


def last_error() -> str:
    return lib().axipcg_last_error().decode()
