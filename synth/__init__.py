"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: coefficient fields sampled at cell
centres, source fields, point-source cell indices and samples of the source
time pulse.  It holds none of the solver's arithmetic (no operator, no
transform, no Laguerre projection), so the CPU oracle and the HIP path can both
consume it without sharing code.

Grid convention used to sample fields (cell-centred): for ``n`` cells over
``[0, l]`` the centres are ``(i + 1/2) * l / n``.

Media recipes follow the structural traits of the paper's acoustic workloads
(§4.1, eq. (30); §4.3: a layered medium of moderate contrast with a point
source on the axis); the paper's own media (fault model, Marmousi) are not
reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import ndimage

__all__ = [
    "Problem",
    "cell_centres",
    "medium_smooth_small",
    "medium_layered",
    "medium_batch_member",
    "gaussian_source",
    "ricker_source",
    "point_source_cell",
    "ricker_pulse_samples",
    "problem_small",
    "problem_layered",
    "problem_batch_member",
    "laguerre_series_inputs",
    "gauss_sine_pulse_samples",
    "medium_fault",
    "medium_fault_smooth",
    "node_coords",
    "paper_series_inputs",
]


def cell_centres(n: int, length: float) -> np.ndarray:
    """Cell-centre coordinates ``(i + 1/2) * length / n`` for ``i < n``."""
    return (np.arange(n, dtype=np.float64) + 0.5) * (length / n)


@dataclasses.dataclass
class Problem:
    """One elliptic problem: grid, coefficient fields and a source field.

    Arrays are ``[nr][nz]`` row-major float64 with z contiguous.
    ``f`` is the right-hand side of the continuous equation (not r-weighted).
    """

    nr: int
    nz: int
    lr: float
    lz: float
    kappa: np.ndarray
    q: np.ndarray
    f: np.ndarray
    bc_z: int = 0  # 0: Dirichlet at z = 0, lz; 1: Neumann
    seed: int = 0
    name: str = ""


def node_coords(n: int, length: float, boundary_unknown: bool) -> np.ndarray:
    """Unknown positions of the paper's node grid (§2.1): nodes at
    (i - 1/2) h, i = 1..N, with h = length / (N - 1/2), the last node on the
    boundary.  ``boundary_unknown`` False (r, Dirichlet at the boundary
    node): the n unknowns are the first N - 1 = n nodes, h = length/(n + 1/2);
    True (z, Neumann): all n = N nodes, h = length/(n - 1/2)."""
    h = length / (n + 0.5) if not boundary_unknown else length / (n - 0.5)
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def _unit_std(g: np.ndarray) -> np.ndarray:
    g = g - g.mean()
    s = g.std()
    return g / s if s > 0 else g


def medium_smooth_small(n: int = 64, seed: int = 0):
    """Smooth variable kappa on [0,1]^2 with constant q = 0.1.

    kappa = 1 + 0.5 sin(2 pi r) cos(2 pi z) + 0.2 * box3x3(U(0,1)); the 3x3 box
    filter replicates edge cells.
    """
    rng = np.random.default_rng(seed)
    r = cell_centres(n, 1.0)[:, None]
    z = cell_centres(n, 1.0)[None, :]
    noise = ndimage.uniform_filter(rng.uniform(0.0, 1.0, size=(n, n)), size=3, mode="nearest")
    kappa = 1.0 + 0.5 * np.sin(2 * np.pi * r) * np.cos(2 * np.pi * z) + 0.2 * noise
    q = np.full((n, n), 0.1)
    return np.ascontiguousarray(kappa), q


def medium_layered(nr: int, nz: int, seed: int = 0, eta: float = 10.0, lz: float = 1.0):
    """Layered medium: 5 equal z-layers with values U[1,4], times a smooth
    lognormal perturbation exp(0.1 g), g a Gaussian-filtered N(0,1) field
    (sigma = N/64 cells per axis) rescaled to unit std.  q = (eta^2/4)/kappa,
    i.e. the Laguerre damping term with c^2 = kappa.
    """
    rng = np.random.default_rng(seed)
    layer_vals = rng.uniform(1.0, 4.0, size=5)
    z = cell_centres(nz, lz)
    layer = np.minimum((z / lz * 5).astype(int), 4)
    base = np.broadcast_to(layer_vals[layer][None, :], (nr, nz))
    g = rng.standard_normal((nr, nz))
    g = ndimage.gaussian_filter(g, sigma=(nr / 64.0, nz / 64.0), mode="reflect")
    g = _unit_std(g)
    kappa = base * np.exp(0.1 * g)
    q = (eta * eta / 4.0) / kappa
    return np.ascontiguousarray(kappa), np.ascontiguousarray(q)


def medium_batch_member(p: int):
    """Member ``p`` of the uneven batch: Nr, Nz ~ U{256,512,1024} independently;
    kappa = Gaussian-filtered N(0,1) (sigma = N/16 per axis) min-max rescaled
    to [1,4]; q the same recipe rescaled to [0,1].  Seed 1000 + p.
    """
    rng = np.random.default_rng(1000 + p)
    nr = int(rng.choice([256, 512, 1024]))
    nz = int(rng.choice([256, 512, 1024]))

    def smooth(lo, hi):
        g = ndimage.gaussian_filter(rng.standard_normal((nr, nz)), sigma=(nr / 16.0, nz / 16.0), mode="reflect")
        g = (g - g.min()) / (g.max() - g.min())
        return lo + (hi - lo) * g

    kappa = smooth(1.0, 4.0)
    q = smooth(0.0, 1.0)
    r0 = rng.uniform(0.0, 0.8)
    z0 = rng.uniform(0.2, 0.8)
    return nr, nz, np.ascontiguousarray(kappa), np.ascontiguousarray(q), (r0, z0)


def gaussian_source(nr, nz, lr, lz, r0, z0, sigma):
    """Unnormalised Gaussian exp(-((r-r0)^2 + (z-z0)^2) / (2 sigma^2))."""
    r = cell_centres(nr, lr)[:, None]
    z = cell_centres(nz, lz)[None, :]
    return np.exp(-((r - r0) ** 2 + (z - z0) ** 2) / (2 * sigma * sigma))


def ricker_source(nr, nz, lr, lz, z0, sigma):
    """Spatial Ricker wavelet on the axis: (1 - d^2/s^2) exp(-d^2/(2 s^2)),
    d^2 = r^2 + (z - z0)^2."""
    r = cell_centres(nr, lr)[:, None]
    z = cell_centres(nz, lz)[None, :]
    d2 = r * r + (z - z0) ** 2
    return (1.0 - d2 / (sigma * sigma)) * np.exp(-d2 / (2 * sigma * sigma))


def point_source_cell(nz: int, lz: float, z0: float) -> int:
    """Index of the cell centre nearest to z0 (ties go to the lower index)."""
    zc = cell_centres(nz, lz)
    d = np.abs(zc - z0)
    return int(np.argmin(d))  # argmin returns the first (lower) index on ties


def ricker_pulse_samples(nt: int = 8001, t_max: float = 0.2, f0: float = 25.0, t0: float = 0.1):
    """Ricker time pulse (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2)
    sampled uniformly on [0, t_max] (nt points, both ends included)."""
    t = np.linspace(0.0, t_max, nt)
    a = (math.pi * f0 * (t - t0)) ** 2
    return t, (1.0 - 2.0 * a) * np.exp(-a)


def problem_small(seed: int = 0, n: int = 64) -> Problem:
    """64x64 plain problem on [0,1]^2: smooth kappa, q = 0.1, Gaussian source
    at (0, 0.5) with sigma 0.05, Dirichlet in z."""
    kappa, q = medium_smooth_small(n, seed)
    f = gaussian_source(n, n, 1.0, 1.0, 0.0, 0.5, 0.05)
    return Problem(n, n, 1.0, 1.0, kappa, q, np.ascontiguousarray(f), 0, seed, f"smooth{n}")


def problem_layered(nr: int = 1024, nz: int = 1024, seed: int = 0, eta: float = 10.0) -> Problem:
    """Layered medium with a spatial Ricker source at (0, 0.3), sigma 0.01."""
    kappa, q = medium_layered(nr, nz, seed, eta)
    f = ricker_source(nr, nz, 1.0, 1.0, 0.3, 0.01)
    return Problem(nr, nz, 1.0, 1.0, kappa, q, np.ascontiguousarray(f), 0, seed, f"layered{nr}x{nz}")


def problem_batch_member(p: int) -> Problem:
    nr, nz, kappa, q, (r0, z0) = medium_batch_member(p)
    f = gaussian_source(nr, nz, 1.0, 1.0, r0, z0, 0.02)
    return Problem(nr, nz, 1.0, 1.0, kappa, q, np.ascontiguousarray(f), 0, 1000 + p, f"batch{p}")


def laguerre_series_inputs(nr: int, nz: int, seed: int = 0, eta: float = 10.0, z0: float = 0.3):
    """Inputs of one Laguerre series: layered medium, the source cell on the
    axis nearest to (0, z0), and the Ricker time pulse samples."""
    kappa, q = medium_layered(nr, nz, seed, eta)
    k0 = point_source_cell(nz, 1.0, z0)
    t, ft = ricker_pulse_samples()
    return dict(nr=nr, nz=nz, lr=1.0, lz=1.0, kappa=kappa, q=q, src_i=0, src_k=k0,
                eta=eta, t=t, ft=ft, seed=seed)


def nn_example(nr: int, nz: int, seed: int = 0):
    """Smooth random fields shaped like the learned guess's inputs.

    u1, u2, ut play u_{m-1}, u_{m-2} and the solved u_m (correlated, O(1)
    amplitude), b a right-hand side with a localised bump and kappa a medium
    in [1, 4].  Plain random data: no step of the method is computed here.
    """
    rng = np.random.default_rng(seed)

    def smooth(scale):
        g = ndimage.gaussian_filter(rng.standard_normal((nr, nz)), sigma=max(1.0, min(nr, nz) / 8), mode="wrap")
        return scale * _unit_std(g)

    base = smooth(1.0)
    u1 = base + 0.3 * smooth(1.0)
    u2 = base + 0.3 * smooth(1.0)
    ut = base + 0.3 * smooth(1.0)
    b = smooth(0.2)
    b[nr // 3, nz // 2] += 5.0
    kappa = 2.5 + 1.5 * np.tanh(smooth(1.0))
    return {"u1": u1, "u2": u2, "ut": ut, "b": b, "kappa": kappa}


def gauss_sine_pulse_samples(nt: int = 4001, t_max: float = 0.4, f0: float = 30.0, t0: float = 0.2,
                             gamma: float = 4.0):
    """The source time function of the paper's experiment (§4.3 eq. (40)),
    exp(-(2 pi f0 (t-t0))^2 / gamma^2) sin(2 pi f0 (t-t0)) with f0 = 30 Hz,
    t0 = 0.2 s, gamma = 4, sampled uniformly on [0, t_max] (both ends)."""
    t = np.linspace(0.0, t_max, nt)
    a = 2.0 * math.pi * f0 * (t - t0)
    return t, np.exp(-a * a / (gamma * gamma)) * np.sin(a)


def medium_fault(nr: int, nz: int, lr: float = 2.0, lz: float = 2.0, seed: int = 0):
    """Stand-in for the paper's "geological fault" model (whose figure is not
    available): wave speed 2.0 km/s above and 3.5 km/s below an interface at
    depth 0.6 km for r < 0.8 km and 0.9 km beyond (a vertical throw of
    0.3 km), times a smooth 5% lognormal perturbation (Gaussian-filtered
    N(0,1), sigma = N/32 cells, unit std), the interface smoothed over two
    cells.  Returns V [nr][nz] (the coefficient of the operator, read as
    kappa)."""
    rng = np.random.default_rng(seed)
    r = cell_centres(nr, lr)[:, None]
    z = cell_centres(nz, lz)[None, :]
    depth = np.where(r < 0.8, 0.6, 0.9)
    v = np.where(z < depth, 2.0, 3.5)
    v = ndimage.gaussian_filter(v, sigma=2.0, mode="nearest")
    g = _unit_std(ndimage.gaussian_filter(rng.standard_normal((nr, nz)), sigma=(nr / 32.0, nz / 32.0),
                                          mode="reflect"))
    return np.ascontiguousarray(v * np.exp(0.05 * g))


def medium_fault_smooth(r, z, seed: int = 0):
    """The fault stand-in as a function of position (so that grids of every
    size sample the same medium, for refinement studies): 2.0 km/s above and
    3.5 km/s below an interface at depth 0.6 km for r < 0.8 km and 0.9 km
    beyond, both steps tanh-smoothed over 20 m, times exp(0.05 g) with g a sum
    of six seeded plane waves (wavelengths 0.3-2 km) scaled to unit variance.
    r, z broadcastable arrays (km); returns V."""
    rng = np.random.default_rng(seed)
    step = lambda x: 0.5 * (1.0 + np.tanh(x / 0.02))  # noqa: E731
    depth = 0.6 + 0.3 * step(r - 0.8)
    v = 2.0 + 1.5 * step(z - depth)
    kr = rng.uniform(0.5, 3.0, 6)
    kz = rng.uniform(0.5, 3.0, 6)
    ph = rng.uniform(0.0, 2.0 * math.pi, 6)
    g = sum(np.sin(2.0 * math.pi * (kr[j] * r + kz[j] * z) + ph[j]) for j in range(6)) / math.sqrt(3.0)
    return v * np.exp(0.05 * g)


def paper_series_inputs(nr: int, nz: int, seed: int = 0, eta: float = 300.0, alpha: int = 5, n_rec: int = 16,
                        lr: float = 2.0, lz: float = 2.0, grid: str = "cells"):
    """Inputs of the paper's Laguerre experiment (§4.3): the fault stand-in
    (kappa = V), density rho = 1 so that q = eta^2/4 and the history
    coefficient is eta^2 (eq. (35)), Neumann in z (free surface, eq. (32)), the
    point source at the origin (cell (0, 0)), the pulse of eq. (40), alpha = 5,
    eta (the paper's h) = 300, and n_rec receivers on the surface row k = 0 at
    r = (j + 1/2) lr / (2 n_rec) (flat indices i * nz).

    ``grid`` "nodes": the paper's r-grid (§2.1; bc_z carries the node-grid
    flag 0x100; z cell-centred) with the medium sampled from
    ``medium_fault_smooth`` at the unknowns, so that every grid size sees the
    same medium; "cells" (default):
    the cell-centred grid with the grid-sampled ``medium_fault``."""
    if grid == "nodes":
        r = node_coords(nr, lr, False)[:, None]
        z = cell_centres(nz, lz)[None, :]
        kappa = np.ascontiguousarray(medium_fault_smooth(r, z, seed) * np.ones((nr, nz)))
    else:
        kappa = medium_fault(nr, nz, lr, lz, seed)
    q = np.full((nr, nz), eta * eta / 4.0)
    coef = np.full((nr, nz), eta * eta)
    t, ft = gauss_sine_pulse_samples()
    ri = np.minimum(((np.arange(n_rec) + 0.5) * nr / (2 * n_rec)).astype(np.int64), nr - 1)
    return dict(nr=nr, nz=nz, lr=lr, lz=lz, kappa=kappa, q=q, coef=coef, bc_z=1 | (0x100 if grid == "nodes" else 0),
                src_i=0, src_k=0, eta=eta, alpha=alpha, t=t, ft=ft, rec_idx=ri * nz, seed=seed, grid=grid)
