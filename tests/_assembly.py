"""Independent sparse assembly of the scheme's matrix for pinning the oracle.

The matrix is built from the energy (quadratic-form) representation of the
finite-volume scheme of §2.1 eqs. (4)-(6):

    y^T A y = sum_{interior faces f} C_f (y_a - y_b)^2
            + sum_{Dirichlet boundary faces f} C_f y_c^2  +  sum_c w_c y_c^2,

i.e. A = G^T diag(C) G + diag(w) with G the face-difference (incidence) matrix.
This is a different formulation from the oracle's per-cell flux loop, so a
wrong index, a missing boundary term or a transposed coefficient in either one
shows up as a mismatch.
"""
import numpy as np
import scipy.sparse as sp


def steps(nr, nz, lr, lz, grid=0, z_nodes=False):
    """Grid steps: cells h = l / N; the paper's r-nodes (grid 1)
    h_r = l_r / (N_1 - 1/2) with N_1 = nr + 1 (the boundary node on r = lr is
    not an unknown), z cell-centred -- or, with z_nodes, the literal
    h_z = l_z / (N_2 - 1/2) of the paper's z-grid."""
    hr = lr / (nr + 0.5) if grid == 1 else lr / nr
    hz = lz / (nz - 0.5) if z_nodes else lz / nz
    return hr, hz


def conductances(kr, kz, q, lr, lz, bc_z, grid=0):
    nr, nz = q.shape
    hr, hz = steps(nr, nz, lr, lz, grid)
    r = (np.arange(nr) + 0.5) * hr
    rho = (np.arange(nr) + 1.0) * hr
    cr = rho[:, None] * kr / hr**2          # face i+1/2 ; i = nr-1 is r = lr
    cz = r[:, None] * kz / hz**2            # face k-1/2 ; k = 0..nz
    w = r[:, None] * q
    return cr, cz, w


def assemble(kr, kz, q, lr=1.0, lz=1.0, bc_z=0, grid=0):
    """Sparse CSR matrix of the r-weighted operator, unknowns ordered i*nz + k.
    On the node grid (grid 1) the outer r-face term couples the last unknown
    to the boundary node's value 0 one full step away: C y^2, not 2 C y^2."""
    nr, nz = q.shape
    cr, cz, w = conductances(kr, kz, q, lr, lz, bc_z, grid)
    idx = lambda i, k: i * nz + k
    rows, cols, vals = [], [], []
    faces_a, faces_b, faces_c = [], [], []
    # interior r-faces
    for i in range(nr - 1):
        for k in range(nz):
            faces_a.append(idx(i, k)); faces_b.append(idx(i + 1, k)); faces_c.append(cr[i, k])
    # interior z-faces
    for i in range(nr):
        for k in range(1, nz):
            faces_a.append(idx(i, k - 1)); faces_b.append(idx(i, k)); faces_c.append(cz[i, k])
    nf = len(faces_c)
    G = sp.csr_matrix((np.r_[np.ones(nf), -np.ones(nf)],
                       (np.r_[np.arange(nf), np.arange(nf)], np.r_[faces_a, faces_b])),
                      shape=(nf, nr * nz))
    A = G.T @ sp.diags(np.asarray(faces_c)) @ G
    diag = w.ravel().copy()
    # Dirichlet outer r-face: half-cell flux to the boundary value 0 -> 2 C
    # (cells), full-step flux to the boundary node -> C (nodes)
    diag[[idx(nr - 1, k) for k in range(nz)]] += (1.0 if grid == 1 else 2.0) * cr[nr - 1, :]
    if bc_z == 0:
        diag[[idx(i, 0) for i in range(nr)]] += 2.0 * cz[:, 0]
        diag[[idx(i, nz - 1) for i in range(nr)]] += 2.0 * cz[:, nz]
    return (A + sp.diags(diag)).tocsr()


def energy(kr, kz, q, y, lr=1.0, lz=1.0, bc_z=0):
    nr, nz = q.shape
    cr, cz, w = conductances(kr, kz, q, lr, lz, bc_z)
    e = np.sum(cr[:-1] * (y[:-1] - y[1:]) ** 2) + np.sum(cz[:, 1:nz] * (y[:, :-1] - y[:, 1:]) ** 2)
    e += np.sum(2 * cr[-1] * y[-1] ** 2) + np.sum(w * y * y)
    if bc_z == 0:
        e += np.sum(2 * cz[:, 0] * y[:, 0] ** 2) + np.sum(2 * cz[:, nz] * y[:, -1] ** 2)
    return e
