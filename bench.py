#!/usr/bin/env python3
"""Benchmark: Laguerre harmonics solved per second on a 1024^2 grid.

One step = one harmonic of the Laguerre series (§4.1 eq. (35)): the
right-hand side from the running history sums, an initial guess, then PCG to
||r||/||b|| <= 1e-10 with the separation-of-variables preconditioner.  The
medium is the layered synthetic recipe (5 z-layers, smooth lognormal
perturbation, q = (eta^2/4)/kappa, eta = 10) on a held-out seed; the source
is a point source on the axis at z = 0.3 with a 25 Hz Ricker time pulse.
Inputs are resident in HBM before the timed region.

Modes (each a fresh series of warmup + steps harmonics on the same medium):
  A  FP64 preconditioner, previous-harmonic guess (the plain method)
  B  FP32 preconditioner, previous-harmonic guess
  X  FP32 preconditioner, best of u_{m-1} and the extrapolation by residual
  Z  FP32 preconditioner, zero guess (the paper's choice)
  Y  FP32 preconditioner, extrapolation guard, Chebyshev iteration of eq. (8)
     (the operator's own bounds; no dot products)
  C  FP32 preconditioner, learned guess with its guard (headline), the network
     trained beforehand (untimed) on harmonics of eight other media
The first harmonics of the headline mode are checked against the FP64 oracle
chain that the CPU-baseline leg computes on the same inputs, and harmonics
across the timed range (the last one included) against the oracle's solve of
the same right-hand side, with the iterations PCG needs to first reach an
error of 1e-8 there (untimed).  A fixed 400-harmonic comparison of B, X and C
on the two held-out media (seeds 101, 102) follows.

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
BYTES_PER_POINT = {   # one PCG iteration, FP32 preconditioner in 4-row strips
    "spmv": 56,      # read z, p_old, D, CR, CZ; write p, q
    "zfwd": 53,      # read x, r, p, q; write x, r, 3/4 of f' (f32), E1 and G0 (2 f32 per strip and mode)
    "tridiag": 3,    # read E1, G0; write X (f32 per strip and mode)
    "zinv": 21,      # read 3/4 of f', X of the strip and the one before, r; write z
}
PRECOND_BYTES_PER_POINT = 32  # r (8) -> spectral (4+4) -> spectral (4+4) -> z (8)
PRECOND_BYTES_PER_POINT_FP64 = 48  # r (8) -> spectral (8+8) -> spectral (8+8) -> z (8)
KERNEL_IDS = {"spmv": 0, "zfwd": 1, "tridiag": 2, "zinv": 3}
PROFILE_EVERY = 8   # time one launch in 8 of the roofline kernel inside the timed loop
KERNEL_SYMBOLS = {"spmv": "k_pcg_spmv", "zfwd": "k_strip_fwd", "tridiag": "k_strip_reduced", "zinv": "k_strip_inv"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400, help="timed harmonics")
    ap.add_argument("--warmup", type=int, default=5, help="untimed harmonics before the timed ones")
    ap.add_argument("--nr", type=int, default=1024)
    ap.add_argument("--nz", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=101)
    ap.add_argument("--modes", default="A,B,L,X,Z,Y,W,C", help="comma-separated modes to run")
    ap.add_argument("--headline", default="C", help="mode whose throughput is the value")
    ap.add_argument("--train-seeds", default="1,2,3,4,5,6,7,8")
    ap.add_argument("--train-harmonics", type=int, default=200)
    ap.add_argument("--nn-base", type=int, default=6,
                    help="order of the extrapolation the network corrects (1..6)")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--roofline-kernel", choices=list(KERNEL_IDS), default="spmv")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem uneven batch")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-experiment pipeline record")
    ap.add_argument("--no-large", action="store_true", help="skip the 2048^2 series record")
    ap.add_argument("--large-harmonics", type=int, default=100, help="timed harmonics of the 2048^2 record")
    ap.add_argument("--no-held-out", action="store_true",
                    help="skip the fixed-length comparison on the two held-out media")
    ap.add_argument("--held-out-harmonics", type=int, default=400,
                    help="timed harmonics per mode and medium of the held-out comparison")
    ap.add_argument("--no-xl", action="store_true", help="skip the 4096^2 series record")
    ap.add_argument("--xl-harmonics", type=int, default=20, help="timed harmonics of the 4096^2 record")
    ap.add_argument("--paper-harmonics", type=int, default=2000,
                    help="harmonics of the paper-experiment records (the paper's n = 2000)")
    ap.add_argument("--no-refinement", action="store_true",
                    help="skip the paper experiment's grid-refinement record (256^2 .. 2048^2)")
    ap.add_argument("--strips", type=int, default=1, choices=[0, 1, 4, 8],
                    help="preconditioner form of the solves: strips of 4 or 8 rows, 1 = the library's "
                         "default, 0 = the per-mode r-solve over whole lines")
    ap.add_argument("--fused", type=int, default=0, choices=[0, 1],
                    help="1: the single-launch preconditioner for FP32 applies and PCG iterations")
    ap.add_argument("--precond-variants", default="",
                    help="with --precond-only: comma list of variant keys (e.g. fp32_strips8); default all")
    ap.add_argument("--precond-only", type=int, default=0, metavar="N",
                    help="only time standalone preconditioner applies on an N x N layered medium (FP32 "
                         "then FP64, --steps applies each) and print their rates; the run to profile "
                         "the preconditioner's kernels")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 64 MiB tensor five times (the known-size kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a --pmc run)")
    ap.add_argument("--ingest-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn the counter CSVs of two rocprofv3 --pmc runs of this script (with "
                         "--copy-calibration) into profiles/traffic_<kernel>_<workload>.json and exit")
    return ap.parse_args()


def _block(text, start):
    """The text of the declaration that begins with `start` up to its closing
    brace at column 0 (or its first line, for one-line declarations)."""
    a = text.index(start)
    line_end = text.index("\n", a)
    if text[a:line_end].rstrip().endswith(";") or text[a:line_end].rstrip().endswith("}"):
        return text[a:line_end]
    return text[a:text.index("\n}", a) + 2]


def source_sha():
    """Hash of the source text the roofline kernel (the PCG SpMV) is built
    from: its tile body and stencil helpers (spmv.h), its kernel wrapper and
    launch size in pcg.hip, and the state, slot layout and reduction helpers
    it uses from common.h."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1002_3094_amd", "csrc")
    hdr = open(os.path.join(csrc, "spmv.h")).read()
    h.update(hdr[hdr.index("struct Pair {"):hdr.index("// Chebyshev step of eq. (8) in increment form")].encode())
    pcg = open(os.path.join(csrc, "pcg.hip")).read()
    h.update(pcg[pcg.index("template <bool PR, int RW>\n__global__"):pcg.index("// Chebyshev step of eq. (8)")].encode())
    com = open(os.path.join(csrc, "common.h")).read()
    for start in ("struct PcgState {", "enum Slot {", "constexpr int MAX_PARTIALS",
                  "__device__ inline double block_sum(", "struct TotalLoads {", "__device__ inline void total_issue(",
                  "__device__ inline double total_finish(", "__device__ inline double block_total(",
                  "__device__ inline int xcd_swizzle("):
        h.update(_block(com, start).encode())
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


COPY_BYTES = 64 << 20


def ingest_traffic(a, fetch_csv, write_csv):
    """HBM (data-fabric) bytes per launch of the roofline kernel from two
    rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
    scaled by what the same counter reads for the calibration copy of
    COPY_BYTES.  Launches past the stop test (which return at once) are left
    out: only dispatches above a tenth of the kernel's largest count are
    averaged."""
    import csv

    def per_kernel(path):
        out = {}
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"]
            out.setdefault(name, []).append(float(r["Counter_Value"]))
        return out

    def copy_kib(d):
        # the calibration copies are the largest copy dispatches of the run
        vals = [v for n, vs in d.items() if "copybuffer" in n.lower() for v in vs]
        big = [v for v in vals if v > 0.95 * max(vals)]
        return sum(big) / len(big)

    def kernel_kib(d, symbol):
        vals = [v for n, vs in d.items() if symbol in n for v in vs]
        big = [v for v in vals if v > 0.1 * max(vals)]
        return sum(big) / len(big), len(big)

    f, w = per_kernel(fetch_csv), per_kernel(write_csv)
    fscale = COPY_BYTES / (copy_kib(f) * 1024)
    wscale = COPY_BYTES / (copy_kib(w) * 1024)
    sym = KERNEL_SYMBOLS[a.roofline_kernel]
    fk, nf = kernel_kib(f, sym)
    wk, nw = kernel_kib(w, sym)
    rec = {"kernel": sym, "workload": f"laguerre_{a.nr}x{a.nz}", "source_sha": source_sha(),
           "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4),
           "fetch_bytes_per_launch": round(fk * 1024 * fscale), "write_bytes_per_launch": round(wk * 1024 * wscale),
           "dispatches": [nf, nw]}
    rec["hbm_bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    rec["algorithmic_bytes_per_launch"] = BYTES_PER_POINT[a.roofline_kernel] * a.nr * a.nz
    path = os.path.join(ROOT, "profiles", f"traffic_{a.roofline_kernel}_{rec['workload']}.json")
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec))


def cpu_baseline(inp, prec_rtol, budget_s, n_max=16):
    """The FP64 oracle's own Laguerre chain on the host cores, for a bounded
    prefix of the same series (time-bounded).  Returns (record, harmonics)."""
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
    return ({"value": done / el, "unit": "harmonics/s", "cores": oracle.num_threads(), "kind": "oracle",
             "sample": f"first {done} harmonics of the same {inp['nr']}x{inp['nz']} chain, FP64 oracle "
                       f"(4N-embedding FFT transforms, Thomas r-solves, PCG to 1e-10), {el:.1f} s"}, us)


def large_measure(ax, torch, n, n_harm, seed):
    """The Laguerre chain of the layered medium on an n x n grid (the
    paper-scale series): FP32 and FP64 preconditioners with the previous
    harmonic as guess, the SpMV's HIP-event duration in the FP32 run, and
    standalone preconditioner applies."""
    import synth
    from paper_1002_3094_amd import series
    inp = synth.laguerre_series_inputs(n, n, seed=seed)
    op = ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    g = ax.laguerre_coeffs(n_harm + 3, inp["eta"], inp["ft"], inp["t"][-1])
    rec = {"workload": f"laguerre_{n}x{n}", "harmonics": n_harm, "guess": "prev", "rtol": 1e-10}
    for name, prec in (("fp64", ax.PREC_FP64), ("fp32", ax.PREC_FP32)):
        s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"])
        s.run(3, "prev", prec)
        if prec == ax.PREC_FP32:
            ax.profile_select(op, KERNEL_IDS["spmv"], PROFILE_EVERY)
            ax.profile_read(op, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.run(n_harm, "prev", prec)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert all(c == ax.OK for c in st.status), st.status
        rec[name] = {"harmonics_per_s": round(n_harm / el, 2), "iters_per_harmonic": round(float(np.mean(st.iters)), 3),
                     "us_per_iteration": round(el * 1e6 / max(1, sum(st.iters)), 2)}
        if prec == ax.PREC_FP32:
            k_ms, k_n = ax.profile_read(op, reset=True)
            ax.profile_select(op, ax.KERNEL_NONE)
            k_s = (k_ms / 1e3) / max(k_n, 1)
            gbs = BYTES_PER_POINT["spmv"] * n * n / k_s / 1e9
            rec["spmv"] = {"mean_us": round(k_s * 1e6, 2), "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                           "launches": k_n}
    rec["speedup_fp32_vs_fp64"] = round(rec["fp32"]["harmonics_per_s"] / rec["fp64"]["harmonics_per_s"], 3)
    # the same series from the order 0-6 extrapolation guard instead of u_{m-1}
    s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"])
    s.run(3, "poly", ax.PREC_FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.run(n_harm, "poly", ax.PREC_FP32)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert all(c == ax.OK for c in st.status), st.status
    rec["fp32_poly_guard"] = {"harmonics_per_s": round(n_harm / el, 2),
                              "iters_per_harmonic": round(float(np.mean(st.iters)), 3),
                              "us_per_iteration": round(el * 1e6 / max(1, sum(st.iters)), 2)}
    r = torch.randn((n, n), dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for name, prec in (("fp64", ax.PREC_FP64), ("fp32", ax.PREC_FP32)):
        for _ in range(3):
            ax.precond_apply(op, r, z, prec)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(50):
            ax.precond_apply(op, r, z, prec)
        e1.record()
        torch.cuda.synchronize()
        pc_s = e0.elapsed_time(e1) / 1e3 / 50
        bpp = PRECOND_BYTES_PER_POINT if prec == ax.PREC_FP32 else PRECOND_BYTES_PER_POINT_FP64
        gbs = bpp * n * n / pc_s / 1e9
        rec[f"precond_{name}"] = {"applies_per_s": round(1.0 / pc_s, 1), "mean_us": round(pc_s * 1e6, 2),
                                  "bytes_per_point": bpp, "gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
    op.close()
    return rec


def precond_measure(ax, torch, n, reps, seed=101, precs=("fp32", "fp64"), only=None):
    """Standalone preconditioner applies z = B^{-1} r on the n x n layered
    medium, timed with HIP events on the current stream over `reps` applies
    after three untimed ones (`only`: the variant keys to run, else all)."""
    import synth
    inp = synth.laguerre_series_inputs(n, n, seed=seed)
    op = ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    r = torch.randn((n, n), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(seed))
    z = torch.empty_like(r)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    rec = {"workload": f"precond_{n}x{n}"}
    variants = [(name, rows, False) for name in precs for rows in (4, 8, 0)] + [("fp32", 4, True)]
    for name, rows, one in variants:
        prec = ax.PREC_FP32 if name == "fp32" else ax.PREC_FP64
        key = f"{name}_single_launch" if one else (f"{name}_strips{rows}" if rows else f"{name}_per_mode")
        if only and key not in only:
            continue
        ax.op_set_strips(op, rows)
        ax.op_set_fused(op, one)
        if rows and not ax.op_strips_info(op, prec)[0]:
            continue
        if one and not ax.op_fused_info(op, ax.FUSED_APPLY)[0]:
            continue
        for _ in range(3):
            ax.precond_apply(op, r, z, prec)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            ax.precond_apply(op, r, z, prec)
        e1.record(stream)
        torch.cuda.synchronize()
        pc_s = e0.elapsed_time(e1) / 1e3 / reps
        bpp = PRECOND_BYTES_PER_POINT if prec == ax.PREC_FP32 else PRECOND_BYTES_PER_POINT_FP64
        gbs = bpp * n * n / pc_s / 1e9
        rec[key] = {"applies_per_s": round(1.0 / pc_s, 1), "mean_us": round(pc_s * 1e6, 2), "bytes_per_point": bpp,
                    "gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                    "min_bytes_per_point": 16, "gbs_at_min_bytes": round(16 * n * n / pc_s / 1e9, 1)}
        print(f"[precond] {n}x{n} {key}: {pc_s * 1e6:.2f} us per apply ({reps} applies)", flush=True)
    ax.op_set_strips(op, 1)
    ax.op_set_fused(op, False)
    op.close()
    return rec


def paper_measure(ax, torch, n_harm):
    """The paper's experiment (§4.3) at 1024^2 on its node grid in r: the
    fault stand-in, Neumann in z, alpha = 5, h = 300, the pulse of eq. (40),
    FP32 preconditioner; a zero initial guess (the paper's), the previous
    harmonic, and the polynomial extrapolation guard; receiver traces
    synthesised from the harmonics."""
    import synth
    from paper_1002_3094_amd import series
    inp = synth.paper_series_inputs(1024, 1024, seed=101, grid="nodes")
    op = ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"], bc_z=inp["bc_z"])
    g = ax.laguerre_coeffs_alpha(n_harm, inp["alpha"], inp["eta"], inp["ft"], inp["t"][-1])
    rec = {"workload": "laguerre_paper_1024x1024_alpha5_h300", "grid": "paper nodes in r (h_r = l/(N - 1/2))",
           "harmonics": n_harm, "alpha": inp["alpha"], "eta": inp["eta"], "bc_z": "neumann",
           "receivers": int(len(inp["rec_idx"]))}
    for guess in ("zero", "prev", "poly"):
        s = series.PaperSeries(op, g, inp["alpha"], inp["eta"], inp["src_i"], inp["src_k"], inp["coef"],
                               inp["rec_idx"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.run(n_harm, guess, ax.PREC_FP32)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        assert all(c == ax.OK for c in st.status), st.status
        rec[guess] = {"harmonics_per_s": round(n_harm / el, 2), "iters_per_harmonic": round(float(np.mean(st.iters)), 2),
                      "preconditioner_inversions": int(sum(st.iters)),
                      "us_per_iteration": round(el * 1e6 / max(1, sum(st.iters)), 2)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = s.traces(1001, 0.8)
    torch.cuda.synchronize()
    rec["traces_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
    rec["trace_peak"] = float(tr.abs().max().item())
    op.close()
    return rec


def paper_refinement(ax, torch, n_harm, grids=(256, 512, 1024, 2048), length=1.0, r_star=0.25, t_star=0.4):
    """Table 2 of §4.3 on the stand-in: the paper's experiment (node grid in
    r, zero guesses, FP32 preconditioner, n_harm harmonics) on N^2 grids of
    the same medium over a length x length km domain (1 km: 17 to 136 nodes
    per 67 m wavelength of the 30 Hz pulse in the 2 km/s layer, the paper's
    range being 35 to 280); the wave field u(t*, r*, z) along the vertical slice
    r = r* (linear interpolation between the two bracketing r-nodes, then in
    z onto the coarsest grid's z points), each grid's relative L2 error
    against the finest, their ratio per halving, and the preconditioner
    inversions (PCG iterations) per harmonic of each grid."""
    import synth
    from paper_1002_3094_amd import series
    slices, iters = {}, {}
    z_ref = None
    for n in grids:
        inp = synth.paper_series_inputs(n, n, seed=101, grid="nodes", lr=length, lz=length)
        hr = inp["lr"] / (n + 0.5)
        i0 = int(r_star / hr - 0.5)
        w1 = (r_star - (i0 + 0.5) * hr) / hr
        idx = np.concatenate([i0 * n + np.arange(n), (i0 + 1) * n + np.arange(n)]).astype(np.int64)
        op = ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"], bc_z=inp["bc_z"])
        g = ax.laguerre_coeffs_alpha(n_harm, inp["alpha"], inp["eta"], inp["ft"], inp["t"][-1])
        s = series.PaperSeries(op, g, inp["alpha"], inp["eta"], inp["src_i"], inp["src_k"], inp["coef"], idx)
        st = s.run(n_harm, "zero", ax.PREC_FP32)
        assert all(c == ax.OK for c in st.status), st.status
        u = s.traces(2, t_star)[:, 1].cpu().numpy()          # u(t*) at the receivers
        col = (1.0 - w1) * u[:n] + w1 * u[n:]
        z = synth.cell_centres(n, inp["lz"])
        if z_ref is None:
            z_ref = z
        slices[n] = np.interp(z_ref, z, col)
        iters[n] = float(np.mean(st.iters))
        op.close()
    fine = slices[grids[-1]]
    errs = [float(np.linalg.norm(slices[n] - fine) / np.linalg.norm(fine)) for n in grids[:-1]]
    return {"workload": "laguerre_paper_refinement", "grids": list(grids), "harmonics": n_harm,
            "domain_km": [length, length], "slice": {"r_km": r_star, "t_s": t_star}, "iters_per_harmonic": [round(iters[n], 3) for n in grids],
            "rel_err_vs_finest": [round(e, 6) for e in errs],
            "error_ratio_per_halving": [round(e0 / e1, 3) for e0, e1 in zip(errs, errs[1:])]}


def held_out_measure(ax, torch, a, net, seeds=(101, 102), modes=("B", "X", "C")):
    """The learned guess evaluated as trained: a fixed number of harmonics
    (400 by default, whatever --steps is) on each held-out medium, for the
    plain previous-harmonic guess (B), the extrapolation guard without the
    network (X) and the network with its guard (C), each timed after 5 warmup
    harmonics; the guard's picks from an untimed replay of the C series."""
    import synth
    from paper_1002_3094_amd import series
    n = a.held_out_harmonics
    rec = {"workload": f"laguerre_{a.nr}x{a.nz}_held_out", "harmonics": n, "warmup": 5, "rtol": 1e-10,
           "seeds": {}}
    for seed in seeds:
        inp = synth.laguerre_series_inputs(a.nr, a.nz, seed=seed)
        r = {}
        with ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"]) as op:
            g = ax.laguerre_coeffs(n + 5, inp["eta"], inp["ft"], inp["t"][-1])
            for mode in modes:
                prec_name, guess, solver = MODES[mode]
                if guess in ("nn", "nn_poly") and net is None:
                    continue
                prec = ax.PREC_FP32 if prec_name == "fp32" else ax.PREC_FP64
                s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
                s.run(5, guess, prec, net=net, solver=solver)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = s.run(n, guess, prec, net=net, solver=solver)
                torch.cuda.synchronize()
                el = max(time.perf_counter() - t0, st.gpu_ms / 1e3)
                assert all(c == ax.OK for c in st.status), st.status
                r[mode] = {"guess": guess, "harmonics_per_s": round(n / el, 2),
                           "iters_per_harmonic": round(float(np.mean(st.iters)), 3)}
                if guess == "nn_poly":
                    s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
                    st = s.run(n + 5, guess, prec, net=net, want_info=True, solver=solver)
                    k = ax.history_len(guess) + 1
                    r[mode]["guard_picks_by_candidate"] = np.bincount(st.choice, minlength=k).tolist()
        if "B" in r:
            for mode in r:
                r[mode]["iters_vs_B"] = round(r[mode]["iters_per_harmonic"] / r["B"]["iters_per_harmonic"], 3)
        rec["seeds"][str(seed)] = r
    return rec


def batch_measure(ax, torch, prec, reps=3):
    """64 independent uneven problems (N_r, N_z ~ U{256,512,1024}, seeds
    1000+p): one batched solve with a launch per phase, the same solve in one
    cooperative launch, the batched Chebyshev form, and the problems solved
    one by one."""
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

    def timed(flags):
        ax.batch_solve(ops, bs, xs, 1e-10, 1000, prec, flags)      # warm-up
        times, iters = [], []
        for _ in range(reps):
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            code, st = ax.batch_solve(ops, bs, xs, 1e-10, 1000, prec, flags)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            iters = [s["iters"] for s in st]
            assert code == ax.OK
        return min(times), iters

    t_b, iters = timed(0)
    t_s, iters_s = timed(ax.FLAG_SINGLE_LAUNCH)
    # the Chebyshev form of eq. (8), each member with its own bounds; these
    # media have cells with q = 0, where eq. (10) bounds B^-1 A from below
    # only for a B without the q term, so both forms run on such operators
    ops0 = [ax.op_create(pr.kappa, pr.q, qbar=0.0) for pr in probs]

    def timed_on(fn):
        fn()      # warm-up
        best, its = None, []
        for _ in range(reps):
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            code, st = fn()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            best = el if best is None else min(best, el)
            its = [s["iters"] for s in st]
            assert code == ax.OK
        return best, its

    t_c, iters_c = timed_on(lambda: ax.batch_cheb_solve(ops0, bs, xs, rtol=1e-10, maxit=1000, prec=prec))
    t_c0, iters_c0 = timed_on(lambda: ax.batch_solve(ops0, bs, xs, 1e-10, 1000, prec))
    for op in ops0:
        op.close()
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
    return {"workload": "batch_64_uneven_256-1024", "points": pts, "solves_per_s": round(64 / t_b, 1),
            "ms_per_batch": round(t_b * 1e3, 3), "sequential_solves_per_s": round(64 / t_seq, 1),
            "iters_min_max": [min(iters), max(iters)],
            "single_launch": {"solves_per_s": round(64 / t_s, 1), "ms_per_batch": round(t_s * 1e3, 3),
                              "iters_min_max": [min(iters_s), max(iters_s)]},
            "chebyshev": {"preconditioner": "kbar only (qbar = 0)",
                          "solves_per_s": round(64 / t_c, 1), "ms_per_batch": round(t_c * 1e3, 3),
                          "iters_min_max": [min(iters_c), max(iters_c)],
                          "pcg_same_operators": {"solves_per_s": round(64 / t_c0, 1),
                                                 "iters_min_max": [min(iters_c0), max(iters_c0)]}}}


def per_step_parity(ax, series, op, g, inp, a, net, last_b, last_u):
    """Per-step parity of the headline chain: at harmonics spread over the
    timed range, and at the last timed one, the oracle solves A u = b_m from
    the GPU's own right-hand side b_m to a relative residual of 1e-13 and
    u_m must match it to 1e-8.  The last timed harmonic is checked on the b_m
    and u_m the timed run itself left behind; the others come from an untimed
    replay of the same series in chunks, which reproduces the timed run
    bit for bit (checked on the last harmonic)."""
    import oracle
    prec_name, guess, solver = MODES[a.headline]
    prec = ax.PREC_FP32 if prec_name == "fp32" else ax.PREC_FP64
    oop = oracle.operator_from_cells(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    n_harm = a.warmup + a.steps
    marks = sorted({a.warmup + (a.steps * q) // 4 for q in (1, 2, 3)} | {n_harm - 1})
    s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
    st = series.SeriesStats()
    cases, reach = [], []
    for m in marks:
        if m + 1 > s.m:
            s.run_harmonics(m + 1 - s.m, guess, prec, 1e-10, 1000, st, net=net, solver=solver)
        ref = oracle.solve_reference(oop, s.b.cpu().numpy(), rtol=1e-13, maxit=1000)
        reach.append(first_reach(ax, op, s, ref, prec, guess, net, st.iters[-1]))
        cases.append((m, s.b.cpu().numpy(), s.u1.cpu().numpy(), ref))
    replay_equal = bool(np.array_equal(cases[-1][1], last_b) and np.array_equal(cases[-1][2], last_u))
    cases[-1] = (n_harm - 1, last_b, last_u, cases[-1][3])
    errs = [float(np.linalg.norm(u - ref) / max(np.linalg.norm(ref), 1e-300)) for _, _, u, ref in cases]
    return {"harmonics": [c[0] for c in cases], "rel_err": errs, "max_rel_err": max(errs),
            "oracle_rtol": 1e-13, "last_timed_harmonic": n_harm - 1, "replay_bitwise_equal_to_timed": replay_equal,
            "iterations_to_1e-8_error": reach}


def first_reach(ax, op, s, ref, prec, guess, net, iters_stop, kmax=80):
    """Untimed diagnostic at the harmonic m the series `s` has just solved:
    PCG restarted from the harmonic's initial guess, stopped after k = 1, 2,
    ... iterations, until its iterate's error against the oracle's solution
    `ref` of the same A u = b_m falls to 1e-8 relative.  Done for the
    previous-harmonic guess u_{m-1} and for the guess of the mode itself
    (recomputed from the history the step started from); reported next to
    the iterations the 1e-10 residual test took."""
    torch = s.torch
    b = s.b
    nh = ax.history_len(guess)
    hist = s.hist[1:nh] + [s.u]   # u_{m-1}, u_{m-2}, ... as the step saw them
    nref = max(np.linalg.norm(ref), 1e-300)
    out = {"harmonic": s.m - 1, "iters_at_1e-10_residual": int(iters_stop)}
    for name in dict.fromkeys(("prev", guess)):
        x0 = torch.empty_like(b)
        if name == "prev":
            x0.copy_(hist[0])
        elif name == "zero":
            x0.zero_()
        elif name == "extrap":
            ax.guess_extrap(op, b, hist[0], hist[1], x0)
        elif name == "poly":
            ax.guess_poly(op, b, hist, x0)
        elif name == "nn_poly":
            ax.nn_guess_poly(op, net, b, hist, s.kappa, x0)
        elif name == "nn":
            ax.nn_guess(op, net, b, hist[0], hist[1], s.kappa, x0)
        else:
            raise ValueError(name)
        x = torch.empty_like(b)
        err0 = float(np.linalg.norm(x0.cpu().numpy() - ref) / nref)
        reached = 0 if err0 <= 1e-8 else None
        for k in range(1, kmax + 1):
            if reached is not None:
                break
            x.copy_(x0)
            ax.pcg_solve(op, b, x, rtol=1e-30, maxit=k, prec=prec)
            if np.linalg.norm(x.cpu().numpy() - ref) / nref <= 1e-8:
                reached = k
        out[name] = {"guess_rel_err": err0, "iters": reached}
    return out


MODES = {   # (preconditioner, guess, solver)
    "A": ("fp64", "prev", "pcg"),
    "B": ("fp32", "prev", "pcg"),
    "L": ("fp32", "extrap", "pcg"),
    "X": ("fp32", "poly", "pcg"),
    "Z": ("fp32", "zero", "pcg"),
    "Y": ("fp32", "poly", "cheb"),
    "C": ("fp32", "nn_poly", "pcg"),
    "W": ("fp32", "nn_poly", "cheb"),
}
NN_FLOP_PER_POINT = 2 * 9 * (4 * 32 + 4 * 32 * 32 + 32 * 1)   # 76 608: six 3x3 convolutions
BF16_PEAK_TFLOPS = 2500.0


def train_network(ax, torch, synth, series, a):
    """Online training on the series of each training medium (untimed)."""
    net = ax.nn_create(a.nr, a.nz, series.nn_init_params(0))
    ax.nn_set_base(net, a.nn_base)
    mode = "nn" if a.nn_base == 1 else "nn_poly"
    seeds = [int(v) for v in a.train_seeds.split(",") if v]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, losses = [], []
    for seed in seeds:
        inp = synth.laguerre_series_inputs(a.nr, a.nz, seed=seed)
        with ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"]) as op:
            g = ax.laguerre_coeffs(a.train_harmonics, inp["eta"], inp["ft"], inp["t"][-1])
            s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
            st = s.run(a.train_harmonics, mode, ax.PREC_FP32, net=net, lr=a.lr, want_info=True)
            iters.append(float(np.mean(st.iters)))
            losses.append(float(np.mean(st.loss[-20:])))
    torch.cuda.synchronize()
    return net, {"seeds": seeds, "harmonics_per_seed": a.train_harmonics, "base_order": a.nn_base, "mode": mode,
                 "seconds": round(time.perf_counter() - t0, 2),
                 "final_loss_per_seed": [round(v, 5) for v in losses]}


def main():
    a = parse()
    if a.ingest_traffic:
        ingest_traffic(a, *a.ingest_traffic)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); splitting the grid into "
              "r-strips across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1002_3094_amd import axipcg as ax
    from paper_1002_3094_amd import series

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if a.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
    if a.precond_only:
        only = [v for v in a.precond_variants.split(",") if v] if a.precond_variants else None
        print(json.dumps(precond_measure(ax, torch, a.precond_only, a.steps, only=only)), flush=True)
        return
    modes = [m for m in a.modes.split(",") if m]
    if a.headline not in modes:
        modes.append(a.headline)
    rtol = 1e-10
    inp = synth.laguerre_series_inputs(a.nr, a.nz, seed=a.seed)
    workload = f"laguerre_{a.nr}x{a.nz}"
    n_harm = a.warmup + a.steps

    t_setup = time.perf_counter()
    op = ax.op_create(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
    if a.strips != 1:
        ax.op_set_strips(op, a.strips)
    if a.fused:
        ax.op_set_fused(op, True)
    g = ax.laguerre_coeffs(n_harm, inp["eta"], inp["ft"], inp["t"][-1])
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup

    net, training = (None, None)
    if any(MODES[m][1] in ("nn", "nn_poly") for m in modes):
        net, training = train_network(ax, torch, synth, series, a)

    results = {}
    roofline = None
    stream = torch.cuda.current_stream()
    for mode in modes:
        prec_name, guess, solver = MODES[mode]
        prec = ax.PREC_FP32 if prec_name == "fp32" else ax.PREC_FP64
        s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        warm = s.run(a.warmup, guess, prec, rtol=rtol, net=net, solver=solver)
        assert all(c == ax.OK for c in warm.status), warm.status
        head = mode == a.headline
        if head:
            ax.profile_select(op, KERNEL_IDS[a.roofline_kernel], PROFILE_EVERY)
            ax.profile_read(op, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.run(a.steps, guess, prec, rtol=rtol, net=net, solver=solver)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert all(c == ax.OK for c in st.status), st.status
        elapsed = max(wall, st.gpu_ms / 1e3)
        if head:
            # the last timed harmonic as the timed run left it (copied after the clock stopped)
            last_b, last_u = s.b.cpu().numpy(), s.u1.cpu().numpy()
        results[mode] = {"precond": prec_name, "guess": guess, "solver": solver,
                         "harmonics_per_s": round(a.steps / elapsed, 2),
                         "ms_per_harmonic": round(elapsed * 1e3 / a.steps, 4),
                         "iters_per_harmonic": round(float(np.mean(st.iters)), 3),
                         "us_per_iteration": round(elapsed * 1e6 / max(1, sum(st.iters)), 2)}
        if head:
            k_ms, k_n = ax.profile_read(op, reset=True)
            ax.profile_select(op, ax.KERNEL_NONE)
            n_pts = a.nr * a.nz
            k_avg_s = (k_ms / 1e3) / max(k_n, 1)
            k_bytes = BYTES_PER_POINT[a.roofline_kernel] * n_pts
            achieved = k_bytes / k_avg_s / 1e9
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(a.roofline_kernel, workload, k_bytes),
                        "kernel": KERNEL_SYMBOLS[a.roofline_kernel], "launches": k_n,
                        "mean_us": round(k_avg_s * 1e6, 2), "bytes_per_launch": k_bytes}
            head_elapsed = elapsed
    # the guard's picks in the headline run (untimed replay of the same series)
    if a.headline in ("C", "X"):
        s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st = s.run(n_harm, MODES[a.headline][1], ax.PREC_FP32, rtol=rtol, net=net, want_info=True,
                   solver=MODES[a.headline][2])
        k = ax.history_len(MODES[a.headline][1]) + (1 if MODES[a.headline][1] in ("nn", "nn_poly") else 0)
        results[a.headline]["guard_picks_by_candidate"] = np.bincount(st.choice, minlength=k).tolist()

    n_pts = a.nr * a.nz
    # preconditioner applies (3 launches: transform, r-solves, inverse), standalone
    prec_head = ax.PREC_FP32 if MODES[a.headline][0] == "fp32" else ax.PREC_FP64
    r = torch.randn((a.nr, a.nz), dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    for _ in range(3):
        ax.precond_apply(op, r, z, prec_head)
    n_pc = 50
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    p0.record(stream)
    for _ in range(n_pc):
        ax.precond_apply(op, r, z, prec_head)
    p1.record(stream)
    torch.cuda.synchronize()
    pc_s = p0.elapsed_time(p1) / 1e3 / n_pc
    pc_gbs = PRECOND_BYTES_PER_POINT * n_pts / pc_s / 1e9

    nn_rec = None
    if net is not None:
        s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        s.run(3, "prev", ax.PREC_FP32, rtol=rtol)
        gx = torch.empty_like(s.u)
        ax.nn_set_base(net, 1)      # the unguarded two-array forward; the same network pass
        for _ in range(3):
            ax.nn_forward(net, s.u1, s.u2, s.b, s.kappa, gx)
        n_nn = 20
        torch.cuda.synchronize()
        p0.record(stream)
        for _ in range(n_nn):
            ax.nn_forward(net, s.u1, s.u2, s.b, s.kappa, gx)
        p1.record(stream)
        torch.cuda.synchronize()
        f_s = p0.elapsed_time(p1) / 1e3 / n_nn
        ax.nn_set_base(net, a.nn_base)
        tfl = NN_FLOP_PER_POINT * n_pts / f_s / 1e12
        nn_rec = {"forward_ms": round(f_s * 1e3, 4), "tflops": round(tfl, 1), "peak_tflops": BF16_PEAK_TFLOPS,
                  "frac": round(tfl / BF16_PEAK_TFLOPS, 4), "flop_per_point": NN_FLOP_PER_POINT,
                  "training": training}

    prec_name, guess, solver = MODES[a.headline]
    out = {
        "metric": METRIC,
        "value": results[a.headline]["harmonics_per_s"],
        "unit": "harmonics/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(head_elapsed * 1e3 / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32+bf16" if guess in ("nn", "nn_poly") else ("f64+f32" if prec_name == "fp32" else "f64"),
        "data": "synthetic",
        "config": {"workload": workload, "nr": a.nr, "nz": a.nz, "medium": "layered", "seed": a.seed,
                   "eta": inp["eta"], "harmonics_timed": a.steps, "mode": a.headline, "preconditioner": prec_name,
                   "guess": guess, "rtol": rtol},
        "roofline": roofline,
        "modes": results,
        "precond": {"applies_per_s": round(1.0 / pc_s, 1), "gbs": round(pc_gbs, 1),
                    "frac_of_peak": round(pc_gbs / HBM_PEAK_GBS, 4), "bytes_per_point": PRECOND_BYTES_PER_POINT,
                    "mean_us": round(pc_s * 1e6, 2), "prec": MODES[a.headline][0]},
        "nn": nn_rec,
        "setup_s": round(t_setup, 3),
    }
    if "A" in results:
        out["speedup_vs_plain_fp64"] = round(results[a.headline]["harmonics_per_s"] / results["A"]["harmonics_per_s"], 3)
    if not a.no_held_out:
        out["held_out"] = held_out_measure(ax, torch, a, net)
    if not a.no_batch:
        out["batch"] = batch_measure(ax, torch, ax.PREC_FP32)
    if not a.no_paper:
        out["paper_pipeline"] = paper_measure(ax, torch, a.paper_harmonics)
        if not a.no_refinement:
            out["paper_refinement"] = paper_refinement(ax, torch, a.paper_harmonics)
    if not a.no_large:
        out["series_2048"] = large_measure(ax, torch, 2048, a.large_harmonics, a.seed)
    if not a.no_xl:
        # rows of 4096: the block-wide transforms and the per-mode r-solve;
        # a working set of about 3 GB, far beyond the 256 MB Infinity Cache
        out["series_4096"] = large_measure(ax, torch, 4096, a.xl_harmonics, a.seed)
    if not a.no_cpu_baseline:
        rec, us = cpu_baseline(inp, rtol, a.cpu_seconds)
        out["cpu_baseline"] = rec
        # accuracy of the headline mode on the harmonics the oracle reached
        s = series.LaguerreSeries(op, g, inp["src_i"], inp["src_k"], kappa=inp["kappa"])
        st = series.SeriesStats()
        errs = []
        for uo in us:
            s.step(guess, ax.PREC_FP32 if prec_name == "fp32" else ax.PREC_FP64, rtol, 1000, st, net=net,
                   solver=solver)
            ug = s.u1.cpu().numpy()
            errs.append(float(np.linalg.norm(ug - uo) / max(np.linalg.norm(uo), 1e-300)))
        out["accuracy"] = {"chain_prefix": {"harmonics_checked": len(errs),
                                            "max_rel_err_vs_oracle_chain": max(errs) if errs else None},
                           "per_step": per_step_parity(ax, series, op, g, inp, a, net, last_b, last_u),
                           "tolerance": 1e-8}
        assert out["accuracy"]["per_step"]["max_rel_err"] <= 1e-8, out["accuracy"]
    if net is not None:
        net.close()
    op.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
