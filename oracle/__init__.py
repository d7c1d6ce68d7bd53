"""Plain FP64 CPU oracle: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_1002_3094_amd``)
never imports it, and the two share no code: the only common dependency is the
seeded input generator module ``synth``.

The numerical work is in ``oracle.c`` (built into ``liboracle.so`` by
``oracle/build.py``); this module marshals numpy arrays and holds the Laguerre
series driver, written as a plain loop over harmonics with the direct sum of
the paper's eq. (35).

Parity notes: every function is pinned by ``tests/test_oracle_*.py`` against
the mathematics (dense assembly, closed forms, library routines, brute force).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# AXIPCG_ORACLE_LIB selects another build of oracle.c (the sanitized one of
# build.build_sanitized)
_LIB_PATH = os.environ.get("AXIPCG_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

Z_DIRICHLET = 0
Z_NEUMANN = 1
GRID_CELLS = 0   # cell-centred grid (h = l / N), boundaries on faces
# the paper's r-grid of §2.1 (h_r = l_r / (N_1 - 1/2), the last r-node on r = l_r
# carrying u = 0); z stays cell-centred, the grid on which the cosine basis of
# eq. (38) is exact (with h_z = l_z / (N_2 - 1/2) the Neumann wall would sit half
# a step beyond l_z)
GRID_NODES = 1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i, d = ctypes.c_int, ctypes.c_double
    sig = {
        "orc_num_threads": ([], i),
        "orc_face_kappa": ([i, i, _dp, _dp, _dp], None),
        "orc_coeffs": ([i, i, d, d, i, i, _dp, _dp, _dp, _dp, _dp, _dp], None),
        "orc_apply": ([i, i, _dp, _dp, _dp, _dp, _dp], None),
        "orc_rhs": ([i, i, d, d, i, _dp, _dp], None),
        "orc_dot": ([i, i, _dp, _dp], d),
        "orc_fft": ([i, _dp, _dp], None),
        "orc_ztrans_fwd": ([i, i, _dp, _dp], None),
        "orc_ztrans_inv": ([i, i, _dp, _dp], None),
        "orc_mode_eig": ([i, d, i, i, _dp], None),
        "orc_thomas": ([i, _dp, _dp, _dp, _dp, _dp], None),
        "orc_precond": ([i, i, d, d, i, i, d, d, _dp, _dp], None),
        "orc_pcg": ([i, i, d, d, i, i, _dp, _dp, _dp, d, d, _dp, _dp, d, i, _ip, _dp], i),
        "orc_laguerre_coeffs": ([i, d, i, d, _dp, _dp], None),
        "orc_laguerre_functions": ([i, d, i, _dp, _dp], None),
        "orc_laguerre_psi": ([i, i, d, i, _dp, _dp], None),
        "orc_laguerre_coeffs_a": ([i, i, d, i, d, _dp, _dp], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().orc_num_threads()


# --------------------------------------------------------------------------
# Operator of the scheme, §2.1 eqs. (4)-(6)
# --------------------------------------------------------------------------
@dataclass
class Operator:
    nr: int
    nz: int
    lr: float
    lz: float
    bc_z: int
    cr: np.ndarray      # [nr][nz]   r-face conductances (outer face doubled)
    cz: np.ndarray      # [nr][nz+1] z-face conductances
    w: np.ndarray       # [nr][nz]   r q
    kbar: float         # preconditioner constants, §4.2 eq. (37)
    qbar: float
    grid: int = 0       # GRID_CELLS or GRID_NODES (the paper's grid of §2.1)

    @property
    def hr(self):
        return self.lr / (self.nr + 0.5) if self.grid == GRID_NODES else self.lr / self.nr

    @property
    def hz(self):
        return self.lz / self.nz   # both grids: see GRID_NODES

    @property
    def r(self):
        return (np.arange(self.nr) + 0.5) * self.hr


def face_kappa(kappa: np.ndarray):
    nr, nz = kappa.shape
    kc = _c(kappa)
    kr = np.empty((nr, nz))
    kz = np.empty((nr, nz + 1))
    _load().orc_face_kappa(nr, nz, _p(kc), _p(kr), _p(kz))
    return kr, kz


def operator_from_faces(kr, kz, q, lr=1.0, lz=1.0, bc_z=Z_DIRICHLET, kbar=None, qbar=None,
                        grid=GRID_CELLS) -> Operator:
    """The scheme from kappa at the faces.  ``grid`` = GRID_NODES is the
    paper's r-grid of §2.1 (nodes at (i - 1/2) h_r with h_r = l_r/(N_1 - 1/2),
    the last r-node on the boundary r = l_r carrying u = 0, so nr = N_1 - 1
    unknown rows) with z cell-centred, paired, as in the paper, with Neumann
    z."""
    kr, kz, q = _c(kr), _c(kz), _c(q)
    nr, nz = q.shape
    assert kr.shape == (nr, nz) and kz.shape == (nr, nz + 1)
    assert grid == GRID_CELLS or bc_z == Z_NEUMANN, "the node grid is defined with Neumann z"
    cr = np.empty((nr, nz))
    cz = np.empty((nr, nz + 1))
    w = np.empty((nr, nz))
    _load().orc_coeffs(nr, nz, float(lr), float(lz), int(bc_z), int(grid), _p(kr), _p(kz), _p(q), _p(cr), _p(cz),
                       _p(w))
    if kbar is None:
        kbar = float(kr.mean())
    if qbar is None:
        qbar = float(q.mean())
    return Operator(nr, nz, float(lr), float(lz), int(bc_z), cr, cz, w, float(kbar), float(qbar), int(grid))


def operator_from_cells(kappa, q, lr=1.0, lz=1.0, bc_z=Z_DIRICHLET, kbar=None, qbar=None,
                        grid=GRID_CELLS) -> Operator:
    """Operator from kappa and q at the unknowns (cell centres, or the
    paper's nodes with ``grid`` = GRID_NODES).  Preconditioner constants
    default to the arithmetic means of the values (the paper's footnote to
    eq. (37) uses the mid-range (min+max)/2; CG is invariant to scaling B, so
    this choice only changes iteration counts)."""
    kappa = _c(kappa)
    kr, kz = face_kappa(kappa)
    if kbar is None:
        kbar = float(kappa.mean())
    if qbar is None:
        qbar = float(np.asarray(q).mean())
    return operator_from_faces(kr, kz, q, lr, lz, bc_z, kbar, qbar, grid)


def apply(op: Operator, x) -> np.ndarray:
    x = _c(x)
    y = np.empty_like(x)
    _load().orc_apply(op.nr, op.nz, _p(op.cr), _p(op.cz), _p(op.w), _p(x), _p(y))
    return y


def rhs(op: Operator, f) -> np.ndarray:
    """phi = r f, eq. (6)."""
    f = _c(f)
    b = np.empty_like(f)
    _load().orc_rhs(op.nr, op.nz, op.lr, op.lz, op.grid, _p(f), _p(b))
    return b


def dot(a, b) -> float:
    a, b = _c(a), _c(b)
    if a.ndim == 1:
        a = a[None, :]
        b = b[None, :]
    return _load().orc_dot(a.shape[0], a.shape[1], _p(a), _p(b))


# --------------------------------------------------------------------------
# Transforms, §4.2 eq. (38)
# --------------------------------------------------------------------------
def fft(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    re, im = _c(x.real), _c(x.imag)
    _load().orc_fft(len(x), _p(re), _p(im))
    return re + 1j * im


def ztrans_fwd(x, bc_z=Z_DIRICHLET) -> np.ndarray:
    """Row-wise orthonormal forward z-transform of a [.., nz] array."""
    x = _c(x)
    flat = x.reshape(-1, x.shape[-1])
    out = np.empty_like(flat)
    lib = _load()
    for i in range(flat.shape[0]):
        lib.orc_ztrans_fwd(flat.shape[1], int(bc_z), _p(_c(flat[i])), out[i:].ctypes.data_as(_dp))
    return out.reshape(x.shape)


def ztrans_inv(X, bc_z=Z_DIRICHLET) -> np.ndarray:
    X = _c(X)
    flat = X.reshape(-1, X.shape[-1])
    out = np.empty_like(flat)
    lib = _load()
    for i in range(flat.shape[0]):
        lib.orc_ztrans_inv(flat.shape[1], int(bc_z), _p(_c(flat[i])), out[i:].ctypes.data_as(_dp))
    return out.reshape(X.shape)


def mode_eig(nz, lz=1.0, bc_z=Z_DIRICHLET, grid=GRID_CELLS) -> np.ndarray:
    mu = np.empty(nz)
    _load().orc_mode_eig(nz, float(lz), int(bc_z), int(grid), _p(mu))
    return mu


def thomas(a, b, c, f) -> np.ndarray:
    a, b, c, f = _c(a), _c(b), _c(c), _c(f)
    x = np.empty_like(f)
    _load().orc_thomas(len(f), _p(a), _p(b), _p(c), _p(f), _p(x))
    return x


def precond(op: Operator, r) -> np.ndarray:
    """B^{-1} r, §4.2 eqs. (36)-(39)."""
    r = _c(r)
    z = np.empty_like(r)
    _load().orc_precond(op.nr, op.nz, op.lr, op.lz, op.bc_z, op.grid, op.kbar, op.qbar, _p(r), _p(z))
    return z


def pcg(op: Operator, b, x0=None, rtol=1e-13, maxit=500):
    """PCG (§2.2, eq. (8) with CG parameters).  Returns (x, status, iters, relres)."""
    b = _c(b)
    x = np.zeros_like(b) if x0 is None else _c(x0).copy()
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    st = _load().orc_pcg(op.nr, op.nz, op.lr, op.lz, op.bc_z, op.grid, _p(op.cr), _p(op.cz), _p(op.w),
                         op.kbar, op.qbar, _p(b), _p(x), float(rtol), int(maxit),
                         ctypes.byref(it), ctypes.byref(rel))
    return x, int(st), int(it.value), float(rel.value)


def solve_reference(op: Operator, b, x0=None, rtol=1e-13, maxit=500):
    """Reference solution for parity: PCG run to rtol (default 1e-13) or to
    maxit, whichever comes first."""
    x, st, it, rel = pcg(op, b, x0, rtol, maxit)
    return x


# --------------------------------------------------------------------------
# Laguerre series, §4.1 eqs. (34)-(35) with alpha = 0
# --------------------------------------------------------------------------
def laguerre_coeffs(n: int, eta: float, ft, t_max: float) -> np.ndarray:
    ft = _c(ft)
    g = np.empty(n)
    _load().orc_laguerre_coeffs(int(n), float(eta), len(ft), float(t_max), _p(ft), _p(g))
    return g


def laguerre_functions(n: int, eta: float, t) -> np.ndarray:
    t = _c(t)
    out = np.empty((n, len(t)))
    _load().orc_laguerre_functions(int(n), float(eta), len(t), _p(t), _p(out))
    return out


def laguerre_psi(n: int, alpha: int, eta: float, t) -> np.ndarray:
    """Projection kernel of the generalized transform (§4.1 eq. (34)):
    psi_m(t) = sqrt(eta m!/(m+alpha)!) e^{-eta t/2} L^alpha_m(eta t), [n][len(t)]."""
    t = _c(t)
    out = np.empty((n, len(t)))
    _load().orc_laguerre_psi(int(n), int(alpha), float(eta), len(t), _p(t), _p(out))
    return out


def laguerre_synthesis(n: int, alpha: int, eta: float, t) -> np.ndarray:
    """Synthesis functions phi_m(t) = (eta t)^alpha psi_m(t) of eq. (34):
    u(t) = sum_m Q_m phi_m(t).  [n][len(t)]."""
    t = _c(t)
    return laguerre_psi(n, alpha, eta, t) * (eta * t)[None, :] ** alpha


def laguerre_coeffs_a(n: int, alpha: int, eta: float, ft, t_max: float) -> np.ndarray:
    """f_m = int f psi_m dt (composite Simpson on uniform samples of [0, t_max])."""
    ft = _c(ft)
    g = np.empty(n)
    _load().orc_laguerre_coeffs_a(int(n), int(alpha), float(eta), len(ft), float(t_max), _p(ft), _p(g))
    return g


def laguerre_weights(n: int, alpha: int):
    """c_m = sqrt(m!/(m+alpha)!) and d_k = sqrt((k+alpha)!/k!) of eq. (35)."""
    from math import lgamma, exp
    c = np.array([exp(0.5 * (lgamma(m + 1) - lgamma(m + alpha + 1))) for m in range(n)])
    return c, 1.0 / c


def laguerre_chain_a(op: Operator, coef, g, alpha: int, src_i: int, src_k: int, n_harm: int,
                     rtol=1e-13, maxit=500, guess="zero"):
    """Harmonics of eq. (35) with general alpha:
        A Q_m = r (g_m delta_h - coef * c_m * sum_{k<m} (m - k) d_k Q_k),
    coef = eta^2 / rho^2 per cell; the sum is evaluated directly."""
    us, stats = [], []
    r = op.r[:, None]
    c, dd = laguerre_weights(n_harm, alpha)
    delta = point_delta_rhs(op, src_i, src_k)
    for m in range(n_harm):
        s = np.zeros((op.nr, op.nz))
        for k in range(m):
            s += (m - k) * dd[k] * us[k]
        b = g[m] * delta - r * coef * c[m] * s
        x0 = us[-1] if (guess == "prev" and us) else None
        x, st, it, rel = pcg(op, b, x0, rtol, maxit)
        us.append(x)
        stats.append((st, it, rel))
    return us, stats


def point_delta_rhs(op: Operator, src_i: int, src_k: int) -> np.ndarray:
    """r-weighted discrete delta: b = 1/(h_r h_z) in the source cell, so that
    sum(b) h_r h_z = 1 (the 1/(2 pi) of the 3-D delta is a dropped scale)."""
    b = np.zeros((op.nr, op.nz))
    b[src_i, src_k] = 1.0 / (op.hr * op.hz)
    return b


def laguerre_chain(op: Operator, kappa, g, eta: float, src_i: int, src_k: int,
                   n_harm: int, rtol=1e-13, maxit=500, guess="prev"):
    """Harmonics u_0..u_{n_harm-1} of eq. (35) with alpha = 0 and rho^2 read as
    c^2 = kappa:
        A u_m = r f_m,  f_m = g_m delta_h - (eta^2 / c^2) * sum_{k<m} (m-k) u_k.
    The sum is evaluated directly over the stored harmonics."""
    us = []
    r = op.r[:, None]
    coef = eta * eta / np.asarray(kappa)
    delta = point_delta_rhs(op, src_i, src_k)
    stats = []
    for m in range(n_harm):
        s = np.zeros((op.nr, op.nz))
        for k in range(m):
            s += (m - k) * us[k]
        b = g[m] * delta - r * coef * s
        x0 = us[-1] if (guess == "prev" and us) else None
        x, st, it, rel = pcg(op, b, x0, rtol, maxit)
        us.append(x)
        stats.append((st, it, rel))
    return us, stats


def energy_bounds(op: Operator):
    """Energy-equivalence constants of eq. (10) for B = the same scheme with
    kbar, qbar in place of kappa, q (§4.2 eqs. (36)-(37)): both quadratic forms
    are sums over faces of conductance * (difference)^2 plus sums over cells of
    w * u^2, so gamma1 / gamma2 are the smallest / largest ratio of matching
    terms (faces and cells where B's term is non-zero)."""
    B = operator_from_cells(np.full((op.nr, op.nz), op.kbar), np.full((op.nr, op.nz), op.qbar),
                            op.lr, op.lz, op.bc_z, op.kbar, op.qbar, op.grid)
    ratios = []
    for a, b in ((op.cr, B.cr), (op.cz, B.cz), (op.w, B.w)):
        m = b > 0
        if m.any():
            ratios.append(a[m] / b[m])
    allr = np.concatenate([x.ravel() for x in ratios])
    return float(allr.min()), float(allr.max())


def lanczos_tridiagonal(op: Operator, b, steps: int):
    """The Lanczos matrix T_k of B^{-1} A (symmetric in the B inner product)
    taken out of k steps of PCG from x = 0 on A x = b (§2.2 eq. (8) with the
    conjugate-gradient parameters alpha_j = r_j.z_j / p_j.A p_j and
    beta_j = r_{j+1}.z_{j+1} / r_j.z_j): the Lanczos vectors are the
    normalised residuals, and
        T[j][j]   = 1 / alpha_j + beta_{j-1} / alpha_{j-1}   (no second term for j = 0),
        T[j][j+1] = sqrt(beta_j) / alpha_j.
    Stops early when r.z vanishes.  Returns (diagonal, off-diagonal)."""
    r = _c(b).copy()
    z = precond(op, r)
    p = z.copy()
    rho = dot(r, z)
    alphas, betas = [], []
    for _ in range(steps):
        if not rho > 0.0:
            break
        q = apply(op, p)
        alpha = rho / dot(p, q)
        r -= alpha * q
        z = precond(op, r)
        rho_new = dot(r, z)
        alphas.append(alpha)
        betas.append(rho_new / rho)
        p = z + betas[-1] * p
        rho = rho_new
    m = len(alphas)
    d = np.array([1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0) for j in range(m)])
    e = np.array([math.sqrt(max(betas[j], 0.0)) / alphas[j] for j in range(m - 1)])
    return d, e


def lanczos_bounds(op: Operator, b, steps: int):
    """The smallest and largest eigenvalues of the Lanczos matrix of
    lanczos_tridiagonal (Ritz values of B^{-1} A: inside its spectrum, the
    extreme ones approaching its ends as the steps grow)."""
    d, e = lanczos_tridiagonal(op, b, steps)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def cheb_alpha(m: int, rho2: float) -> float:
    """alpha_m of the Chebyshev parameters of eq. (8): alpha_1 = 1,
    alpha_2 = 2 / (2 - rho0^2), alpha_{k+1} = 4 / (4 - rho0^2 alpha_k)."""
    if m == 1:
        return 1.0
    a = 2.0 / (2.0 - rho2)
    for _ in range(2, m):
        a = 4.0 / (4.0 - rho2 * a)
    return a


def cheb(op: Operator, b, x0=None, gamma1=None, gamma2=None, rtol=1e-13, maxit=500, iters=None):
    """The two-step iteration of §2.2 eq. (8),
        B (ybar - y_k) / tau + A y_k = f,   y_{k+1} = alpha_{k+1} ybar + (1 - alpha_{k+1}) y_{k-1},
    with the Chebyshev parameters for the bounds gamma1, gamma2 of eq. (10):
    tau = 2 / (gamma1 + gamma2), rho0 = (1 - xi) / (1 + xi), xi = gamma1 / gamma2
    (alpha_1 = 1, so y_{-1} does not enter).  Stops when ||f - A y_k|| / ||f||
    <= rtol, or after exactly `iters` steps when given.  Returns
    (y, status, iterations, relres) with status 0 converged, 1 maxit."""
    if gamma1 is None or gamma2 is None:
        gamma1, gamma2 = energy_bounds(op)
    f = _c(b)
    y = np.zeros_like(f) if x0 is None else _c(x0).copy()
    y_prev = y.copy()
    tau = 2.0 / (gamma1 + gamma2)
    xi = gamma1 / gamma2
    rho2 = ((1.0 - xi) / (1.0 + xi)) ** 2
    fn = np.linalg.norm(f)
    if fn == 0.0:
        return np.zeros_like(f), 0, 0, 0.0
    k = 0
    limit = maxit if iters is None else iters
    while True:
        res = f - apply(op, y)
        rel = np.linalg.norm(res) / fn
        if (iters is None and rel <= rtol) or k >= limit:
            break
        ybar = y + tau * precond(op, res)
        a = cheb_alpha(k + 1, rho2)
        y, y_prev = a * ybar + (1.0 - a) * y_prev, y
        k += 1
    status = 0 if rel <= rtol else 1
    return y, status, k, rel
