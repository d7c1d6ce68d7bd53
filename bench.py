#!/usr/bin/env python3
"""Benchmark: Laguerre harmonics solved per second on a 1024^2 grid.

One step = one harmonic of the Laguerre series (§4.1 eq. (35)): the
right-hand side from the running history sums, then PCG to ||r||/||b|| <=
1e-10 with the FP32 separation-of-variables preconditioner and FP64 outer
iteration, warm-started from the previous harmonic.  The medium is the
layered synthetic recipe (5 z-layers, smooth lognormal perturbation, q =
(eta^2/4)/kappa, eta = 10) on a held-out seed; the source is a point source on
the axis at z = 0.3 with a 25 Hz Ricker time pulse.  Inputs are resident in
HBM before the timed region.  Accuracy (error <= 1e-8 against the FP64
oracle) is asserted by the GPU test suite, not here.

Prints one JSON line (see the design doc for the fields).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Laguerre harmonics solved/sec at 1e-8 rel err (1024² grid); precond GB/s vs peak"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per grid point of each PCG kernel class with the FP32
# preconditioner (FP64 = 8 B, FP32 = 4 B per value).
BYTES_PER_POINT = {
    "spmv": 56,      # read z, p_old, D, CR, CZ; write p, q
    "zfwd": 52,      # read x, r, p, q; write x, r, spectral (f32)
    "tridiag": 8,    # read + write spectral (f32)
    "zinv": 20,      # read spectral (f32), r; write z
}
PRECOND_BYTES_PER_POINT = 32  # r (8) -> spectral (4+4) -> spectral (4+4) -> z (8)
KERNEL_IDS = {"spmv": 0, "zfwd": 1, "tridiag": 2, "zinv": 3}
KERNEL_SYMBOLS = {"spmv": "k_pcg_spmv", "zfwd": "k_zfwd", "tridiag": "k_tridiag", "zinv": "k_zinv"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed harmonics")
    ap.add_argument("--warmup", type=int, default=5, help="untimed harmonics before the timed ones")
    ap.add_argument("--nr", type=int, default=1024)
    ap.add_argument("--nz", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=101)
    ap.add_argument("--prec", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--guess", choices=["prev", "zero"], default="prev")
    ap.add_argument("--roofline-kernel", choices=list(KERNEL_IDS), default="spmv")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem uneven batch")
    return ap.parse_args()


def source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1002_3094_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, launch_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload; None if absent or taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_sha") != source_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(inp, prec_rtol, budget_s, n_max=16):
    """The FP64 oracle's own Laguerre chain on the host cores, for a bounded
    prefix of the same series (time-bounded)."""
    import oracle
    op = oracle.operator_from_cells(inp["kappa"], inp["q"])
    g = oracle.laguerre_coeffs(n_max, inp["eta"], inp["ft"], inp["t"][-1])
    r = op.r[:, None]
    coef = inp["eta"] ** 2 / inp["kappa"]
    us = []
    t0 = time.perf_counter()
    done = 0
    for m in range(n_max):
        s = np.zeros_like(inp["kappa"])
        for k in range(m):
            s += (m - k) * us[k]
        b = g[m] * oracle.point_delta_rhs(op, inp["src_i"], inp["src_k"]) - r * coef * s
        x, st, it, rel = oracle.pcg(op, b, us[-1] if us else None, prec_rtol, 1000)
        us.append(x)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "harmonics/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {done} harmonics of the same {inp['nr']}x{inp['nz']} chain, FP64 oracle "
                      f"(4N-embedding FFT transforms, Thomas r-solves, PCG to 1e-10), {el:.1f} s"}


def batch_measure(ax, torch, prec, reps=3):
    """64 independent uneven problems (N_r, N_z ~ U{256,512,1024}, seeds
    1000+p): one batched solve versus the same problems solved one by one."""
    import synth
    probs = [synth.problem_batch_member(p) for p in range(64)]
    ops, bs, xs = [], [], []
    for pr in probs:
        op = ax.op_create(pr.kappa, pr.q)
        b = torch.empty((pr.nr, pr.nz), dtype=torch.float64, device="cuda")
        ax.rhs_from_f(op, torch.from_numpy(pr.f).cuda(), b)
        ops.append(op)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    ax.batch_solve(ops, bs, xs, 1e-10, 1000, prec)      # warm-up
    times, iters = [], []
    for _ in range(reps):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, st = ax.batch_solve(ops, bs, xs, 1e-10, 1000, prec)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        iters = [s["iters"] for s in st]
        assert code == ax.OK
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for op, b, x in zip(ops, bs, xs):
        ax.pcg_solve(op, b, x, 1e-10, 1000, prec)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    pts = sum(p.nr * p.nz for p in probs)
    for op in ops:
        op.close()
    t_b = min(times)
    return {"workload": "batch_64_uneven_256-1024", "points": pts, "solves_per_s": round(64 / t_b, 1),
            "ms_per_batch": round(t_b * 1e3, 3), "sequential_solves_per_s": round(64 / t_seq, 1),
            "iters_min_max": [min(iters), max(iters)]}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the multi-GPU r-strip "
              "decomposition is a design in DESIGN.md, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1002_3094_amd import axipcg as ax

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    prec = ax.PREC_FP32 if a.prec == "fp32" else ax.PREC_FP64
    rtol = 1e-10
    inp = synth.laguerre_series_inputs(a.nr, a.nz, seed=a.seed)
    workload = f"laguerre_{a.nr}x{a.nz}"
    n_harm = a.warmup + a.steps

    t_setup = time.perf_counter()
    op = ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    g = ax.laguerre_coeffs(n_harm, inp["eta"], inp["ft"], inp["t"][-1])
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup

    shape = (a.nr, a.nz)
    S1 = torch.zeros(shape, dtype=torch.float64, device=dev)
    S2 = torch.zeros(shape, dtype=torch.float64, device=dev)
    b = torch.zeros(shape, dtype=torch.float64, device=dev)
    u = torch.zeros(shape, dtype=torch.float64, device=dev)
    iters = []
    statuses = []

    def harmonic(m):
        # S1 += u_{m-1}; S2 += S1; b_m; then u is overwritten in place by u_m
        ax.laguerre_rhs(op, float(g[m]), inp["src_i"], inp["src_k"], S1, S2, b, u_prev=(u if m > 0 else None))
        if a.guess == "zero":
            u.zero_()
        st = ax.pcg_solve(op, b, u, rtol=rtol, maxit=1000, prec=prec)
        iters.append(st["iters"])
        statuses.append(st["code"])

    for m in range(a.warmup):
        harmonic(m)
    torch.cuda.synchronize()

    ax.profile_select(op, KERNEL_IDS[a.roofline_kernel])
    ax.profile_read(op, reset=True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for m in range(a.warmup, n_harm):
        harmonic(m)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    k_ms, k_n = ax.profile_read(op, reset=True)
    ax.profile_select(op, ax.KERNEL_NONE)
    timed_iters = iters[a.warmup:]
    assert all(s == ax.OK for s in statuses), statuses

    n_pts = a.nr * a.nz
    elapsed_s = max(wall, gpu_ms / 1e3)
    value = a.steps / elapsed_s

    # roofline of the dominant kernel: algorithmic bytes per launch / mean duration
    k_avg_s = (k_ms / 1e3) / max(k_n, 1)
    k_bytes = BYTES_PER_POINT[a.roofline_kernel] * n_pts
    achieved = k_bytes / k_avg_s / 1e9
    traffic = measured_traffic(a.roofline_kernel, workload, k_bytes)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_SYMBOLS[a.roofline_kernel], "launches": k_n,
                "mean_us": round(k_avg_s * 1e6, 2), "bytes_per_launch": k_bytes}

    # preconditioner applies (3 launches: transform, r-solves, inverse), standalone
    r = torch.randn(shape, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    for _ in range(3):
        ax.precond_apply(op, r, z, prec)
    n_pc = 50
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    p0.record(stream)
    for _ in range(n_pc):
        ax.precond_apply(op, r, z, prec)
    p1.record(stream)
    torch.cuda.synchronize()
    pc_s = p0.elapsed_time(p1) / 1e3 / n_pc
    pc_gbs = PRECOND_BYTES_PER_POINT * n_pts / pc_s / 1e9

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "harmonics/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed_s * 1e3 / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if prec == ax.PREC_FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "nr": a.nr, "nz": a.nz, "medium": "layered", "seed": a.seed,
                   "eta": inp["eta"], "harmonics_timed": a.steps, "preconditioner": a.prec,
                   "guess": a.guess, "rtol": rtol},
        "roofline": roofline,
        "precond": {"applies_per_s": round(1.0 / pc_s, 1), "gbs": round(pc_gbs, 1),
                    "frac_of_peak": round(pc_gbs / HBM_PEAK_GBS, 4), "bytes_per_point": PRECOND_BYTES_PER_POINT,
                    "mean_us": round(pc_s * 1e6, 2)},
        "iters_per_harmonic": round(float(np.mean(timed_iters)), 2),
        "us_per_iteration": round(elapsed_s * 1e6 / max(1, sum(timed_iters)), 2),
        "setup_s": round(t_setup, 3),
    }
    if not a.no_batch:
        out["batch"] = batch_measure(ax, torch, prec)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, rtol, a.cpu_seconds)
    op.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
