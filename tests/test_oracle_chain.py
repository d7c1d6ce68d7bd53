"""Pin of the oracle's Laguerre series driver (§4.1 eq. (35), alpha = 0)
against an independent chain built on a sparse direct solver."""
import numpy as np
import scipy.sparse.linalg as spla

import synth
from tests import _assembly


def test_chain_matches_sparse_direct_chain(orc):
    inp = synth.laguerre_series_inputs(12, 16, seed=3)
    kappa, q, eta = inp["kappa"], inp["q"], inp["eta"]
    nr, nz = kappa.shape
    op = orc.operator_from_cells(kappa, q)
    g = orc.laguerre_coeffs(8, eta, inp["ft"], inp["t"][-1])
    us, stats = orc.laguerre_chain(op, kappa, g, eta, inp["src_i"], inp["src_k"], 8, rtol=1e-13)

    kr, kz = orc.face_kappa(kappa)
    A = _assembly.assemble(kr, kz, q).tocsc()
    lu = spla.splu(A)
    hr, hz = 1.0 / nr, 1.0 / nz
    r = (np.arange(nr) + 0.5) * hr
    ref = []
    for m in range(8):
        # the running-sum form S1_m = sum_{k<m} u_k, S2_m = S2_{m-1} + S1_m
        # equals sum_{k<m} (m-k) u_k; it is used here so that the two chains
        # do not share the way the history term is formed.
        if m == 0:
            S1 = np.zeros((nr, nz))
            S2 = np.zeros((nr, nz))
        else:
            S1 = S1 + ref[-1]
            S2 = S2 + S1
        f = -(eta * eta / kappa) * S2
        f[inp["src_i"], inp["src_k"]] += g[m] / (r[inp["src_i"]] * hr * hz)
        ref.append(lu.solve((r[:, None] * f).ravel()).reshape(nr, nz))
    for m in range(8):
        assert stats[m][0] == 0
        assert np.linalg.norm(us[m] - ref[m]) <= 1e-11 * np.linalg.norm(ref[m]), m
