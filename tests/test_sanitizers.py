"""Host-code sanitizer runs on the CPU: AddressSanitizer and
UndefinedBehaviorSanitizer (aborting on the first report) over

* the oracle (oracle.c built by gcc with both sanitizers), exercised through
  its Python wrapper on small grids: operator assembly on both grids and both
  z-boundaries, the transforms and FFT, the preconditioner, PCG, Chebyshev,
  the Laguerre coefficients and a short harmonic chain;
* the library's host code (every source built host-only by hipcc with both
  sanitizers, no device code): the boundary's argument checks of
  tests/test_abi.py, which run without a GPU.

Each runs in a child process with the matching ASan runtime preloaded, the
library chosen by AXIPCG_ORACLE_LIB / AXIPCG_LIB.  Sanitizer GPU builds do
not exist on this target; the device code is covered by the parity tests.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_SCRIPT = r"""
import numpy as np
import oracle as orc
import synth
rng = np.random.default_rng(0)
for grid in (orc.GRID_CELLS, orc.GRID_NODES):
    for bc in (orc.Z_DIRICHLET, orc.Z_NEUMANN):
        if grid == orc.GRID_NODES and bc != orc.Z_NEUMANN:
            continue
        nr, nz = 12, 16
        kappa, q = synth.medium_layered(nr, nz, 3)
        op = orc.operator_from_cells(kappa, q, bc_z=bc, grid=grid)
        x = rng.standard_normal((nr, nz))
        y = orc.apply(op, x)
        z = orc.precond(op, y)
        b = orc.rhs(op, rng.standard_normal((nr, nz)))
        u, status, it, _ = orc.pcg(op, b, rtol=1e-12, maxit=400)
        assert status == 0, status
        g1, g2 = orc.energy_bounds(op)
        uc = orc.cheb(op, b, gamma1=g1, gamma2=g2, rtol=1e-10, maxit=400)
X = orc.ztrans_fwd(rng.standard_normal((3, 32)), orc.Z_NEUMANN)
orc.ztrans_inv(X, orc.Z_NEUMANN)
orc.fft(rng.standard_normal(64) + 0j)
inp = synth.laguerre_series_inputs(16, 16, seed=1)
op = orc.operator_from_cells(inp["kappa"], inp["q"], lr=inp["lr"], lz=inp["lz"])
g = orc.laguerre_coeffs(4, inp["eta"], inp["ft"], inp["t"][-1])
orc.laguerre_chain(op, inp["kappa"], g, inp["eta"], inp["src_i"], inp["src_k"], 4, rtol=1e-12)
print("oracle under sanitizers: ok")
"""


def _run(cmd, env):
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert p.returncode == 0, out[-4000:]
    return out


def _gcc_asan():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("gcc's ASan runtime is not installed")
    return os.path.realpath(path)


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle import build as ob
    lib = ob.build_sanitized(str(tmp_path))
    env = dict(os.environ, LD_PRELOAD=_gcc_asan(), AXIPCG_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0", OMP_NUM_THREADS="2", PYTHONPATH=ROOT)
    out = _run([sys.executable, "-c", ORACLE_SCRIPT], env)
    assert "oracle under sanitizers: ok" in out


def test_boundary_host_code_under_asan_ubsan(tmp_path):
    from paper_1002_3094_amd import build as pb
    try:
        rt = pb.san_runtime()
    except FileNotFoundError:
        pytest.skip("clang's ASan runtime is not installed")
    lib = pb.build_host_sanitized(str(tmp_path))
    env = dict(os.environ, LD_PRELOAD=rt, AXIPCG_LIB=lib, ASAN_OPTIONS="detect_leaks=0", PYTHONPATH=ROOT)
    out = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                os.path.join("tests", "test_abi.py")], env)
    assert " passed" in out
