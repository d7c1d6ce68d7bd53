"""Laguerre series driver (§4.1, eqs. (34)-(35), alpha = 0).

Harmonics are solved in order m = 0, 1, ...: the right-hand side of m needs
the sum of all earlier solutions, kept on the device as two running sums
(``axipcg_laguerre_rhs``), and each PCG run (§2.2) starts from a guess:

* ``"zero"``  -- x0 = 0, as in the paper's experiments;
* ``"prev"``  -- x0 = u_{m-1};
* ``"extrap"`` -- whichever of u_{m-1} and 2 u_{m-1} - u_{m-2} has the smaller
  residual (``axipcg_guess_extrap``);
* ``"nn"``    -- the learned guess with its guard (``axipcg_nn_guess``: the
  one of u_{m-1}, 2 u_{m-1} - u_{m-2} and the network's correction of the
  latter with the smallest residual), optionally trained online: after harmonic m is
  solved, one backward pass against u_m and one Adam step.

Every numerical step runs in the HIP library; this module only sequences the
calls and owns the device buffers.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

from . import axipcg as ax


@dataclass
class SeriesStats:
    iters: list = field(default_factory=list)
    status: list = field(default_factory=list)
    choice: list = field(default_factory=list)      # guard's pick: 0 prev, 1 extrap, 2 network
    resid: list = field(default_factory=list)       # guard's |b - A x| per candidate
    loss: list = field(default_factory=list)        # training loss per harmonic (when training)
    gpu_ms: float = 0.0


class LaguerreSeries:
    """Device state of one series: running sums, right-hand side, the last
    seven solutions (``hist[0]`` = u_{m-1}, the guesses read two or all seven)
    and the current one.  ``kappa`` (host [nr][nz]) feeds the learned guess.
    One series keeps to one guess mode."""

    def __init__(self, op: "ax.Op", g, src_i: int, src_k: int, kappa=None, coef=None):
        import torch
        self.torch = torch
        self.op, self.g = op, [float(v) for v in g]
        self.src_i, self.src_k = int(src_i), int(src_k)
        shape = (op.nr, op.nz)
        z = lambda: torch.zeros(shape, dtype=torch.float64, device="cuda")  # noqa: E731
        self.S1, self.S2, self.b = z(), z(), z()
        self.hist = [z() for _ in range(ax.POLY_HISTORY)]
        self.u = z()
        self.coef = coef
        self.kappa = None if kappa is None else torch.as_tensor(kappa, dtype=torch.float64).cuda().contiguous()
        self.m = 0

    @property
    def u1(self):
        return self.hist[0]

    @property
    def u2(self):
        return self.hist[1]

    def _rotate(self):
        """The solved harmonic becomes u_{m-1}; the oldest array is the next work array."""
        self.hist, self.u = [self.u] + self.hist[:-1], self.hist[-1]

    def reset(self):
        for t in (self.S1, self.S2, self.b, self.u, *self.hist):
            t.zero_()
        self.m = 0

    def step(self, guess: str, prec: int, rtol: float, maxit: int, stats: SeriesStats,
             net=None, lr: float | None = None, want_info: bool = False, solver: str = "pcg"):
        """Solve harmonic self.m (PCG, or the Chebyshev iteration of eq. (8)
        with the operator's own bounds); afterwards self.u1 holds u_m."""
        m = self.m
        nn_mode = guess in ("nn", "nn_poly")
        if nn_mode and (net is None or self.kappa is None):
            raise ValueError("nn guess needs a network and kappa")
        if not want_info and lr is None and guess not in ("poly", "nn_poly"):
            # the whole harmonic in one library call (no host round trips
            # between the right-hand side, the guess and the solve)
            st = ax.series_step(self.op, m, self.g[m], self.src_i, self.src_k, self.S1, self.S2, self.b,
                                self.u1, self.u2, self.u, guess, solver=solver, net=net,
                                kappa=self.kappa if nn_mode else None, coef=self.coef, rtol=rtol,
                                maxit=maxit, prec=prec)
            stats.iters.append(st["iters"])
            stats.status.append(st["code"])
            self._rotate()
            self.m += 1
            return
        ax.laguerre_rhs(self.op, self.g[m], self.src_i, self.src_k, self.S1, self.S2, self.b,
                        u_prev=(self.u1 if m > 0 else None), coef=self.coef)
        if guess == "zero":
            self.u.zero_()
        elif guess == "prev":
            self.u.copy_(self.u1)
        elif guess == "extrap":
            r = ax.guess_extrap(self.op, self.b, self.u1, self.u2, self.u, want_info=want_info)
            if r is not None:
                stats.resid.append(r[0])
                stats.choice.append(r[1])
        elif guess == "nn":
            r = ax.nn_guess(self.op, net, self.b, self.u1, self.u2, self.kappa, self.u, want_info=want_info)
            if r is not None:
                stats.resid.append(r[0])
                stats.choice.append(r[1])
        elif guess == "poly":
            r = ax.guess_poly(self.op, self.b, self.hist, self.u, want_info=want_info)
            if r is not None:
                stats.resid.append(r[0])
                stats.choice.append(r[1])
        elif guess == "nn_poly":
            r = ax.nn_guess_poly(self.op, net, self.b, self.hist, self.kappa, self.u, want_info=want_info)
            if r is not None:
                stats.resid.append(r[0])
                stats.choice.append(r[1])
        else:
            raise ValueError(f"unknown guess {guess!r}")
        if solver == "cheb":
            st = ax.cheb_solve(self.op, self.b, self.u, rtol=rtol, maxit=maxit, prec=prec)
        else:
            st = ax.pcg_solve(self.op, self.b, self.u, rtol=rtol, maxit=maxit, prec=prec)
        stats.iters.append(st["iters"])
        stats.status.append(st["code"])
        if nn_mode and lr is not None:
            if guess == "nn_poly":
                stats.loss.append(ax.nn_backward_poly(self.op, net, self.hist, self.u, want_loss=want_info))
            else:
                stats.loss.append(ax.nn_backward(self.op, net, self.u1, self.u2, self.u, want_loss=want_info))
            ax.nn_adam(net, lr=lr)
        self._rotate()
        self.m += 1

    def run_harmonics(self, n: int, guess: str, prec: int, rtol: float, maxit: int, stats: SeriesStats,
                      net=None, solver: str = "pcg"):
        """Solve the next n harmonics in one library call (series_run: no
        return to Python between harmonics); afterwards self.u1 holds the
        last solution."""
        if n <= 0:
            return
        if self.m + n > len(self.g):
            raise ValueError("not enough Laguerre coefficients")
        nn_mode = guess in ("nn", "nn_poly")
        if nn_mode and (net is None or self.kappa is None):
            raise ValueError("nn guess needs a network and kappa")
        nh = ax.history_len(guess)
        u = self.hist[:nh] + [self.u]
        code, sts = ax.series_run(self.op, self.m, self.g[self.m:self.m + n], self.src_i, self.src_k, self.S1,
                                  self.S2, self.b, u, guess, solver=solver, net=net,
                                  kappa=self.kappa if nn_mode else None, coef=self.coef, rtol=rtol,
                                  maxit=maxit, prec=prec)
        stats.iters.extend(st["iters"] for st in sts)
        stats.status.extend(st["status"] for st in sts)
        self.hist[:nh], self.u = u[:nh], u[nh]
        self.m += len(sts)

    def run(self, n: int, guess: str, prec: int, rtol: float = 1e-10, maxit: int = 1000, net=None,
            lr: float | None = None, want_info: bool = False, solver: str = "pcg") -> SeriesStats:
        """Solve the next n harmonics, timed with events on the current stream."""
        torch = self.torch
        stats = SeriesStats()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if not want_info and lr is None:
            self.run_harmonics(n, guess, prec, rtol, maxit, stats, net=net, solver=solver)
        else:
            for _ in range(n):
                self.step(guess, prec, rtol, maxit, stats, net=net, lr=lr, want_info=want_info, solver=solver)
        e1.record(stream)
        torch.cuda.synchronize()
        stats.gpu_ms = e0.elapsed_time(e1)
        return stats


class PaperSeries:
    """The paper's experiment (§4.3): the harmonics of eq. (35) with integer
    alpha (alpha = 5, eta = h = 300 there), a zero or previous-harmonic
    initial guess, the receiver samples of every harmonic, and the time
    traces synthesised from them (eq. (34)).  ``coef`` (device or host
    [nr][nz]) is eta^2/rho^2; ``rec_idx`` flat receiver indices.  The guess
    'poly' (the extrapolation guard) reads the last seven harmonics."""

    def __init__(self, op: "ax.Op", g, alpha: int, eta: float, src_i: int, src_k: int, coef, rec_idx):
        import torch
        self.torch = torch
        self.op, self.g, self.alpha, self.eta = op, [float(v) for v in g], int(alpha), float(eta)
        self.src_i, self.src_k = int(src_i), int(src_k)
        shape = (op.nr, op.nz)
        z = lambda: torch.zeros(shape, dtype=torch.float64, device="cuda")  # noqa: E731
        self.S1, self.S2, self.b, self.u = z(), z(), z(), z()
        self.hist = [z() for _ in range(ax.POLY_HISTORY)]
        self.coef = torch.as_tensor(coef, dtype=torch.float64).cuda().contiguous()
        self.rec_idx = torch.as_tensor(rec_idx, dtype=torch.int64).cuda().contiguous()
        self.Q = torch.zeros((len(self.g), self.rec_idx.numel()), dtype=torch.float64, device="cuda")
        self.m = 0

    @property
    def u1(self):
        return self.hist[0]

    def step(self, guess: str, prec: int, rtol: float, maxit: int, stats: SeriesStats, solver: str = "pcg"):
        m = self.m
        ax.laguerre_rhs_alpha(self.op, m, self.alpha, self.g[m], self.src_i, self.src_k, self.S1, self.S2, self.b,
                              u_prev=(self.u1 if m > 0 else None), coef=self.coef)
        if guess == "zero":
            self.u.zero_()
        elif guess == "prev":
            self.u.copy_(self.u1)
        elif guess == "poly":
            ax.guess_poly(self.op, self.b, self.hist, self.u)
        else:
            raise ValueError(f"unknown guess {guess!r}")
        if solver == "cheb":
            st = ax.cheb_solve(self.op, self.b, self.u, rtol=rtol, maxit=maxit, prec=prec)
        else:
            st = ax.pcg_solve(self.op, self.b, self.u, rtol=rtol, maxit=maxit, prec=prec)
        stats.iters.append(st["iters"])
        stats.status.append(st["code"])
        ax.gather(self.op, self.u, self.rec_idx, self.Q[m])
        self.hist, self.u = [self.u] + self.hist[:-1], self.hist[-1]
        self.m += 1

    def run_harmonics(self, n: int, guess: str, prec: int, rtol: float, maxit: int, stats: SeriesStats,
                      solver: str = "pcg"):
        """The next n harmonics in one library call (series_run_alpha)."""
        if n <= 0:
            return
        if self.m + n > len(self.g):
            raise ValueError("not enough Laguerre coefficients")
        nh = ax.POLY_HISTORY if guess == "poly" else 1
        u = self.hist[:nh] + [self.u]
        code, sts = ax.series_run_alpha(self.op, self.m, self.alpha, self.g[self.m:self.m + n], self.src_i,
                                        self.src_k, self.coef, self.S1, self.S2, self.b, u, self.rec_idx, self.Q,
                                        guess, solver=solver, rtol=rtol, maxit=maxit, prec=prec)
        stats.iters.extend(st["iters"] for st in sts)
        stats.status.extend(st["status"] for st in sts)
        self.hist[:nh], self.u = u[:nh], u[nh]
        self.m += len(sts)

    def run(self, n: int, guess: str, prec: int, rtol: float = 1e-10, maxit: int = 1000,
            solver: str = "pcg") -> SeriesStats:
        torch = self.torch
        stats = SeriesStats()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        self.run_harmonics(n, guess, prec, rtol, maxit, stats, solver=solver)
        e1.record()
        torch.cuda.synchronize()
        stats.gpu_ms = e0.elapsed_time(e1)
        return stats

    def traces(self, nt: int, t_max: float):
        """[n_rec][nt] receiver traces u(t_j) from the harmonics solved so far."""
        out = self.torch.empty((self.rec_idx.numel(), nt), dtype=self.torch.float64, device="cuda")
        ax.laguerre_synth(self.alpha, self.eta, self.Q[:self.m].contiguous(), nt, t_max, out)
        return out


def train_online(net, problems, n_harm: int, prec: int, lr: float = 1e-3, rtol: float = 1e-10,
                 maxit: int = 1000, guess: str = "nn"):
    """Train the learned guess on the series of each problem in turn, in the
    guess mode it will serve ("nn", or "nn_poly" for a base order above 1).

    ``problems`` yields (op, g, src_i, src_k, kappa).  Returns (seconds,
    per-problem mean iterations, last losses)."""
    t0 = time.perf_counter()
    iters, losses = [], []
    for op, g, si, sk, kappa in problems:
        s = LaguerreSeries(op, g, si, sk, kappa=kappa)
        st = s.run(n_harm, guess, prec, rtol=rtol, maxit=maxit, net=net, lr=lr, want_info=True)
        iters.append(sum(st.iters) / len(st.iters))
        losses.append(st.loss[-1] if st.loss else None)
    return time.perf_counter() - t0, iters, losses


# layer shapes of the learned guess (cin, cout) and its flat parameter layout:
# per layer W[t][ci][co] then bias[co]
NN_LAYERS = ((4, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1))


def nn_init_params(seed: int, last_zero: bool = True):
    """He-normal weights and zero biases (float32); with a zero last layer the
    network starts as the previous-harmonic guess."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    for l, (ci, co) in enumerate(NN_LAYERS):
        w = rng.standard_normal(9 * ci * co) * np.sqrt(2.0 / (9 * ci))
        if l == len(NN_LAYERS) - 1 and last_zero:
            w[:] = 0.0
        parts += [w, np.zeros(co)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == ax.nn_num_params()
    return p
