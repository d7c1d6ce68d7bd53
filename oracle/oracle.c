/*
 * Plain FP64 CPU oracle for the axisymmetric variable-coefficient PCG solver.
 *
 * TEST INFRASTRUCTURE ONLY: this library is called by the tests, by the
 * package's smoke check and by the benchmark's CPU-baseline leg.  The product
 * (the HIP library) never links, loads or calls it, and the two share no code.
 *
 * Paper: A.V. Terekhov, "High performance parallel algorithm for solving
 * elliptic equations with non-separable variables" (arXiv:1002.3094).
 * Section and equation numbers below are the paper's.
 *
 * Everything is written for clarity, not speed: the z-transform is evaluated
 * through a length-4N complex FFT of an odd/even extension (a direct way of
 * evaluating the sums of eq. (38)), the r-solves use the textbook Thomas
 * algorithm, and PCG is the two-term recurrence form of the three-level scheme
 * of eq. (8) with conjugate-gradient parameters.  OpenMP only splits
 * independent rows / modes; every reduction is summed in a fixed order so the
 * result does not depend on the thread count.
 *
 * Grid (cell-centred reading of §2.1): h_r = lr/nr, r_i = (i+1/2) h_r,
 * h_z = lz/nz, z_k = (k+1/2) h_z.  The r-face between cells i and i+1 sits at
 * radius rho_{i+1/2} = (i+1) h_r; face i = nr-1 is the outer boundary r = lr.
 * Arrays are [nr][nz] row-major (z contiguous) unless stated.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_Z_DIRICHLET 0
#define ORC_Z_NEUMANN 1
#define ORC_GRID_CELLS 0
#define ORC_GRID_NODES 1

/* Grid steps (§2.1).  Cells (the default reading): h_r = l_r / N_r,
 * h_z = l_z / N_z, unknowns at cell centres (i + 1/2) h, boundaries on faces.
 * Nodes (the paper's r-grid): nodes at (i - 1/2) h_r, i = 1..N_1, with
 * h_r = l_r / (N_1 - 1/2), so the last node lies on r = l_r and carries the
 * Dirichlet value; the nr = N_1 - 1 unknown rows give h_r = l_r/(nr + 1/2).
 * In z the node grid keeps h_z = l_z / N_z: the paper's cosine basis
 * (eq. (38)) and its one-sided boundary flux are exact for a Neumann wall at
 * N_2 h_z, and with h_z = l_z/(N_2 - 1/2) that wall would sit half a step
 * beyond z = l_z (first order; a test shows it). */
static void orc_steps(int nr, int nz, double lr, double lz, int grid, double *hr, double *hz)
{
    if (grid == ORC_GRID_NODES) {
        *hr = lr / (nr + 0.5);
        *hz = lz / nz;
    } else {
        *hr = lr / nr;
        *hz = lz / nz;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Coefficients of the finite-volume scheme, §2.1 eqs. (4)-(6).             */
/* ------------------------------------------------------------------------ */

/* kappa at faces from cell-centre values.  The paper samples kappa at the
 * face points (r_i + h/2, z_k) and (r_i, z_k + h/2), eq. (6); for a field
 * given at cell centres the face value is the mean of the two adjacent cells
 * (linear interpolation to the face point); on a boundary face the adjacent
 * cell's value is used.
 *   kr[i][k], i = 0..nr-1  : face between cells i and i+1 (i = nr-1: r = lr)
 *   kz[i][k], k = 0..nz    : face below cell k ([nr][nz+1]; k = 0 and k = nz
 *                            are the boundary faces z = 0 and z = lz)        */
void orc_face_kappa(int nr, int nz, const double *kc, double *kr, double *kz)
{
    for (int i = 0; i < nr; ++i)
        for (int k = 0; k < nz; ++k)
            kr[(size_t)i * nz + k] = (i < nr - 1)
                ? 0.5 * (kc[(size_t)i * nz + k] + kc[(size_t)(i + 1) * nz + k])
                : kc[(size_t)i * nz + k];
    for (int i = 0; i < nr; ++i)
        for (int k = 0; k <= nz; ++k) {
            double v;
            if (k == 0) v = kc[(size_t)i * nz];
            else if (k == nz) v = kc[(size_t)i * nz + nz - 1];
            else v = 0.5 * (kc[(size_t)i * nz + k - 1] + kc[(size_t)i * nz + k]);
            kz[(size_t)i * (nz + 1) + k] = v;
        }
}

/* Face conductances of the r-weighted scheme (eq. (6): a1 = rbar kappa,
 * a2 = r kappa, w = r q), divided by the squared step (orc_steps) so that
 *   (A y)_c = sum over the faces f of cell c of C_f (y_c - y_nb(f)) + w_c y_c.
 *   cr[i][k]  conductance of r-face i+1/2 : rho_{i+1/2} kappa / h_r^2;
 *             the outer face r = lr (Dirichlet, eq. (2)) is doubled, its
 *             neighbour value being the ghost -y (zero on the face).
 *             The axis face rho_{-1/2} = 0 carries no flux (r kappa u_r = 0).
 *   cz[i][k]  conductance of z-face k-1/2 ([nr][nz+1]) : r_i kappa / h_z^2;
 *             boundary faces are doubled for Dirichlet z and zero for
 *             Neumann z (the paper's d u/dz = 0, eq. (2)).
 *   w[i][k]   = r_i q.                                                       */
void orc_coeffs(int nr, int nz, double lr, double lz, int bcz, int grid,
                const double *kr, const double *kz, const double *q,
                double *cr, double *cz, double *w)
{
    double hr, hz;
    orc_steps(nr, nz, lr, lz, grid, &hr, &hz);
    for (int i = 0; i < nr; ++i) {
        const double ri = (i + 0.5) * hr;
        const double rho = (i + 1) * hr;
        /* cells: the outer face lies half a step from the last unknown (ghost
         * -y, doubled); nodes: the boundary node carrying u = 0 is a full step
         * away, so the face keeps its plain conductance */
        const double bnd_r = (i == nr - 1 && grid == ORC_GRID_CELLS) ? 2.0 : 1.0;
        for (int k = 0; k < nz; ++k) {
            cr[(size_t)i * nz + k] = bnd_r * rho * kr[(size_t)i * nz + k] / (hr * hr);
            w[(size_t)i * nz + k] = ri * q[(size_t)i * nz + k];
        }
        for (int k = 0; k <= nz; ++k) {
            double s = 1.0;
            if (k == 0 || k == nz) s = (bcz == ORC_Z_DIRICHLET) ? 2.0 : 0.0;
            cz[(size_t)i * (nz + 1) + k] = s * ri * kz[(size_t)i * (nz + 1) + k] / (hz * hz);
        }
    }
}

/* y = A x, the SPD form -(Lambda_r + Lambda_z) + w of eq. (4), written as the
 * sum of face fluxes around each cell. */
void orc_apply(int nr, int nz, const double *cr, const double *cz, const double *w,
               const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; ++i) {
        for (int k = 0; k < nz; ++k) {
            const size_t c = (size_t)i * nz + k;
            const double xc = x[c];
            double acc = w[c] * xc;
            /* r-face i+1/2 */
            if (i < nr - 1) acc += cr[c] * (xc - x[c + nz]);
            else acc += cr[c] * xc;                 /* ghost value 0 beyond r = lr */
            /* r-face i-1/2 (none on the axis) */
            if (i > 0) acc += cr[c - nz] * (xc - x[c - nz]);
            /* z-faces k-1/2 and k+1/2 */
            const double *czr = cz + (size_t)i * (nz + 1);
            if (k > 0) acc += czr[k] * (xc - x[c - 1]);
            else acc += czr[0] * xc;
            if (k < nz - 1) acc += czr[k + 1] * (xc - x[c + 1]);
            else acc += czr[nz] * xc;
            y[c] = acc;
        }
    }
}

/* Right-hand side of the scheme: phi = r f (eq. (6)). */
void orc_rhs(int nr, int nz, double lr, double lz, int grid, const double *f, double *b)
{
    double hr, hz;
    orc_steps(nr, nz, lr, lz, grid, &hr, &hz);
    for (int i = 0; i < nr; ++i)
        for (int k = 0; k < nz; ++k)
            b[(size_t)i * nz + k] = (i + 0.5) * hr * f[(size_t)i * nz + k];
}

/* Deterministic dot product: per-row sums, then rows in order. */
double orc_dot(int nr, int nz, const double *a, const double *b)
{
    double *rows = (double *)malloc(sizeof(double) * nr);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; ++i) {
        double s = 0.0;
        for (int k = 0; k < nz; ++k) s += a[(size_t)i * nz + k] * b[(size_t)i * nz + k];
        rows[i] = s;
    }
    double s = 0.0;
    for (int i = 0; i < nr; ++i) s += rows[i];
    free(rows);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Textbook iterative radix-2 complex FFT (forward, e^{-2 pi i jk/n}).        */
/* ------------------------------------------------------------------------ */
void orc_fft(int n, double *re, double *im)
{
    /* bit-reversal permutation */
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len >> 1;
        for (int j = 0; j < half; ++j) {
            const double ang = -2.0 * M_PI * j / len;
            const double wr = cos(ang), wi = sin(ang);
            for (int s = 0; s < n; s += len) {
                const int a = s + j, b = a + half;
                const double tr = re[b] * wr - im[b] * wi;
                const double ti = re[b] * wi + im[b] * wr;
                re[b] = re[a] - tr; im[b] = im[a] - ti;
                re[a] += tr; im[a] += ti;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Orthonormal z-transforms, §4.2 eq. (38).                                   */
/*  Neumann z (the paper's case): basis sqrt(2/N) cos(pi l (k+1/2)/N),        */
/*    l = 0..N-1, with the l = 0 function scaled by 1/sqrt(2).  Output index  */
/*    j = l.                                                                  */
/*  Dirichlet z: basis sqrt(2/N) sin(pi l (k+1/2)/N), l = 1..N, with the      */
/*    l = N function scaled by 1/sqrt(2).  Output index j = l - 1.            */
/* Both sums are evaluated through one length-4N FFT of an extension of x:    */
/*  v[2k+1] = x_k, v[4N-2k-1] = +/- x_k (even for cos, odd for sin), zero     */
/*  elsewhere, so that FFT(v)_l = 2 sum x_k cos(theta) (even) or              */
/*  -2i sum x_k sin(theta) (odd), theta = pi l (2k+1)/(2N).                   */
/* ------------------------------------------------------------------------ */
void orc_ztrans_fwd(int n, int bcz, const double *x, double *X)
{
    const int m = 4 * n;
    double *re = (double *)calloc((size_t)m, sizeof(double));
    double *im = (double *)calloc((size_t)m, sizeof(double));
    const double sgn = (bcz == ORC_Z_DIRICHLET) ? -1.0 : 1.0;
    for (int k = 0; k < n; ++k) {
        re[2 * k + 1] = x[k];
        re[m - 2 * k - 1] = sgn * x[k];
    }
    orc_fft(m, re, im);
    const double nrm = sqrt(2.0 / n);
    if (bcz == ORC_Z_DIRICHLET) {
        for (int l = 1; l <= n; ++l) {
            const double s = (l == n) ? 1.0 / sqrt(2.0) : 1.0;
            X[l - 1] = nrm * s * (-0.5 * im[l]);
        }
    } else {
        for (int l = 0; l < n; ++l) {
            const double s = (l == 0) ? 1.0 / sqrt(2.0) : 1.0;
            X[l] = nrm * s * (0.5 * re[l]);
        }
    }
    free(re); free(im);
}

/* Inverse (= transpose) of orc_ztrans_fwd: x_k = sum_j S_{jk} X_j.  With
 * u_l = s_l X_l placed at index l of a length-4N sequence, FFT(u) evaluated
 * at 2k+1 gives sum u_l e^{-i theta}: the real part is the cosine sum and
 * minus the imaginary part is the sine sum. */
void orc_ztrans_inv(int n, int bcz, const double *X, double *x)
{
    const int m = 4 * n;
    double *re = (double *)calloc((size_t)m, sizeof(double));
    double *im = (double *)calloc((size_t)m, sizeof(double));
    if (bcz == ORC_Z_DIRICHLET) {
        for (int l = 1; l <= n; ++l) re[l] = ((l == n) ? 1.0 / sqrt(2.0) : 1.0) * X[l - 1];
    } else {
        for (int l = 0; l < n; ++l) re[l] = ((l == 0) ? 1.0 / sqrt(2.0) : 1.0) * X[l];
    }
    orc_fft(m, re, im);
    const double nrm = sqrt(2.0 / n);
    for (int k = 0; k < n; ++k)
        x[k] = nrm * ((bcz == ORC_Z_DIRICHLET) ? -im[2 * k + 1] : re[2 * k + 1]);
    free(re); free(im);
}

/* Eigenvalues of the z second difference for the basis above (eq. (39)):
 * mu_j = (4/h_z^2) sin^2(pi l / (2N)) with l = j+1 (Dirichlet) or l = j
 * (Neumann).  They enter the r-problem of mode j as + r_i kbar mu_j in the SPD
 * sign convention (the paper's "+4 a2/h^2 sin^2" term inside Lambda_r + ... - d
 * has the opposite sign of the eigenvalue of Lambda_z; this oracle takes the
 * eigenvalue of the operator itself). */
void orc_mode_eig(int nz, double lz, int bcz, int grid, double *mu)
{
    const double hz = lz / nz;   /* both grids (orc_steps) */
    (void)grid;
    for (int j = 0; j < nz; ++j) {
        const int l = (bcz == ORC_Z_DIRICHLET) ? j + 1 : j;
        const double s = sin(M_PI * l / (2.0 * nz));
        mu[j] = 4.0 / (hz * hz) * s * s;
    }
}

/* Thomas algorithm: a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = f[i]. */
void orc_thomas(int n, const double *a, const double *b, const double *c,
                const double *f, double *x)
{
    double *cp = (double *)malloc(sizeof(double) * n);
    double *fp = (double *)malloc(sizeof(double) * n);
    cp[0] = c[0] / b[0];
    fp[0] = f[0] / b[0];
    for (int i = 1; i < n; ++i) {
        const double den = b[i] - a[i] * cp[i - 1];
        cp[i] = (i < n - 1) ? c[i] / den : 0.0;
        fp[i] = (f[i] - a[i] * fp[i - 1]) / den;
    }
    x[n - 1] = fp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = fp[i] - cp[i] * x[i + 1];
    free(cp); free(fp);
}

/* ------------------------------------------------------------------------ */
/* Preconditioner B^{-1} r, §4.2 eqs. (36)-(39): B is the scheme's operator   */
/* with kappa = kbar and q = qbar everywhere.  Separation of variables:       */
/* transform each r-row along z (eq. (38)), solve one tridiagonal system in r */
/* per z-mode (eq. (39)), transform back.                                     */
/* ------------------------------------------------------------------------ */
void orc_precond(int nr, int nz, double lr, double lz, int bcz, int grid, double kbar, double qbar,
                 const double *r, double *z)
{
    double hr, hz;
    orc_steps(nr, nz, lr, lz, grid, &hr, &hz);
    double *spec = (double *)malloc(sizeof(double) * (size_t)nr * nz);
    double *mu = (double *)malloc(sizeof(double) * nz);
    orc_mode_eig(nz, lz, bcz, grid, mu);

    /* step 1: forward transform of each row */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; ++i)
        orc_ztrans_fwd(nz, bcz, r + (size_t)i * nz, spec + (size_t)i * nz);

    /* step 2: one r-tridiagonal system per mode */
#pragma omp parallel
    {
        double *a = (double *)malloc(sizeof(double) * nr);
        double *b = (double *)malloc(sizeof(double) * nr);
        double *c = (double *)malloc(sizeof(double) * nr);
        double *f = (double *)malloc(sizeof(double) * nr);
        double *y = (double *)malloc(sizeof(double) * nr);
#pragma omp for schedule(static)
        for (int j = 0; j < nz; ++j) {
            for (int i = 0; i < nr; ++i) {
                const double ri = (i + 0.5) * hr;
                const double cup = (i + 1) * hr * kbar / (hr * hr) *
                                   ((i == nr - 1 && grid == ORC_GRID_CELLS) ? 2.0 : 1.0);
                const double cdn = (i > 0) ? i * hr * kbar / (hr * hr) : 0.0;
                a[i] = -cdn;
                c[i] = (i < nr - 1) ? -cup : 0.0;
                b[i] = cup + cdn + ri * (kbar * mu[j] + qbar);
                f[i] = spec[(size_t)i * nz + j];
            }
            orc_thomas(nr, a, b, c, f, y);
            for (int i = 0; i < nr; ++i) spec[(size_t)i * nz + j] = y[i];
        }
        free(a); free(b); free(c); free(f); free(y);
    }

    /* step 3: inverse transform of each row */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; ++i)
        orc_ztrans_inv(nz, bcz, spec + (size_t)i * nz, z + (size_t)i * nz);

    free(spec); free(mu);
}

/* ------------------------------------------------------------------------ */
/* PCG, §2.2: the implicit three-level scheme of eq. (8) with the parameters  */
/* of the conjugate-gradient method, in its standard two-term form.  Stops    */
/* when ||r_k|| / ||b|| <= rtol (the stop test of §4.3) with r_k the          */
/* recursively updated residual.  x holds the initial guess on entry.         */
/* Returns 0 on convergence, 1 if maxit was reached, -1 on breakdown.         */
/* ------------------------------------------------------------------------ */
int orc_pcg(int nr, int nz, double lr, double lz, int bcz, int grid,
            const double *cr, const double *cz, const double *w,
            double kbar, double qbar, const double *b, double *x,
            double rtol, int maxit, int *iters, double *relres)
{
    const size_t n = (size_t)nr * nz;
    double *r = (double *)malloc(sizeof(double) * n);
    double *zv = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    int status = 1, it = 0;

    orc_apply(nr, nz, cr, cz, w, x, q);
    for (size_t c = 0; c < n; ++c) r[c] = b[c] - q[c];
    const double bn = sqrt(orc_dot(nr, nz, b, b));
    double rn = sqrt(orc_dot(nr, nz, r, r));
    if (bn == 0.0) {
        memset(x, 0, sizeof(double) * n);
        *iters = 0; *relres = 0.0;
        free(r); free(zv); free(p); free(q);
        return 0;
    }
    orc_precond(nr, nz, lr, lz, bcz, grid, kbar, qbar, r, zv);
    memcpy(p, zv, sizeof(double) * n);
    double rho = orc_dot(nr, nz, r, zv);
    while (rn / bn > rtol && it < maxit) {
        orc_apply(nr, nz, cr, cz, w, p, q);
        const double pq = orc_dot(nr, nz, p, q);
        if (!(pq > 0.0)) { status = -1; break; }
        const double alpha = rho / pq;
        for (size_t c = 0; c < n; ++c) { x[c] += alpha * p[c]; r[c] -= alpha * q[c]; }
        rn = sqrt(orc_dot(nr, nz, r, r));
        ++it;
        if (rn / bn <= rtol) break;
        orc_precond(nr, nz, lr, lz, bcz, grid, kbar, qbar, r, zv);
        const double rho1 = orc_dot(nr, nz, r, zv);
        const double beta = rho1 / rho;
        rho = rho1;
        for (size_t c = 0; c < n; ++c) p[c] = zv[c] + beta * p[c];
    }
    if (status != -1) status = (rn / bn <= rtol) ? 0 : 1;
    *iters = it;
    *relres = rn / bn;
    free(r); free(zv); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Laguerre coefficients of the source pulse, §4.1 eqs. (34)-(35) with        */
/* alpha = 0: g_m = int_0^T f(t) l_m(t) dt, l_m(t) = sqrt(eta) e^{-eta t/2}   */
/* L_m(eta t), where L_m is the Laguerre polynomial from the three-term       */
/* recurrence (k+1) L_{k+1} = (2k+1-x) L_k - k L_{k-1}.  The integral over the */
/* nt uniform samples on [0, T] (nt odd) is composite Simpson.                */
/* ------------------------------------------------------------------------ */
void orc_laguerre_coeffs(int n, double eta, int nt, double tmax, const double *f, double *g)
{
    const double dt = tmax / (nt - 1);
    for (int m = 0; m < n; ++m) g[m] = 0.0;
    double *lk = (double *)malloc(sizeof(double) * n);
    for (int j = 0; j < nt; ++j) {
        const double wgt = (j == 0 || j == nt - 1) ? 1.0 : ((j % 2) ? 4.0 : 2.0);
        const double t = j * dt, xx = eta * t;
        double lm1 = 0.0, l0 = 1.0;
        for (int m = 0; m < n; ++m) {
            lk[m] = l0;
            const double l1 = ((2.0 * m + 1.0 - xx) * l0 - m * lm1) / (m + 1.0);
            lm1 = l0; l0 = l1;
        }
        const double env = sqrt(eta) * exp(-0.5 * xx) * f[j] * wgt * dt / 3.0;
        for (int m = 0; m < n; ++m) g[m] += env * lk[m];
    }
    free(lk);
}

/* Laguerre function values l_m(t_j) (for the transform pins). */
void orc_laguerre_functions(int n, double eta, int nt, const double *t, double *out /* [n][nt] */)
{
    for (int j = 0; j < nt; ++j) {
        const double xx = eta * t[j];
        double lm1 = 0.0, l0 = 1.0;
        const double env = sqrt(eta) * exp(-0.5 * xx);
        for (int m = 0; m < n; ++m) {
            out[(size_t)m * nt + j] = env * l0;
            const double l1 = ((2.0 * m + 1.0 - xx) * l0 - m * lm1) / (m + 1.0);
            lm1 = l0; l0 = l1;
        }
    }
}

/* Generalized transform of §4.1 eq. (34) with integer alpha >= 0: the
 * projection kernel psi_m(t) = sqrt(eta m!/(m+alpha)!) e^{-eta t/2} L^alpha_m(eta t),
 * with L^alpha_m from its three-term recurrence
 *   (m+1) L_{m+1} = (2m + 1 + alpha - x) L_m - (m + alpha) L_{m-1},
 * so that Q_m = int u(t) psi_m(t) dt and u(t) = sum_m Q_m (eta t)^alpha psi_m(t).
 * out: [n][nt]. */
void orc_laguerre_psi(int n, int alpha, double eta, int nt, const double *t, double *out)
{
    for (int j = 0; j < nt; ++j) {
        const double x = eta * t[j];
        const double env = exp(-0.5 * x);
        double lm1 = 0.0, l0 = 1.0;
        for (int m = 0; m < n; ++m) {
            const double nrm = exp(0.5 * (log(eta) + lgamma(m + 1.0) - lgamma(m + alpha + 1.0)));
            out[(size_t)m * nt + j] = nrm * env * l0;
            const double l1 = ((2.0 * m + 1.0 + alpha - x) * l0 - (m + alpha) * lm1) / (m + 1.0);
            lm1 = l0;
            l0 = l1;
        }
    }
}

/* f_m = int f(t) psi_m(t) dt over the uniform samples of [0, tmax] (composite
 * Simpson; nt odd). */
void orc_laguerre_coeffs_a(int n, int alpha, double eta, int nt, double tmax, const double *f, double *g)
{
    const double dt = tmax / (nt - 1);
    double *tt = (double *)malloc(sizeof(double) * nt);
    double *psi = (double *)malloc(sizeof(double) * (size_t)n * nt);
    for (int j = 0; j < nt; ++j) tt[j] = j * dt;
    orc_laguerre_psi(n, alpha, eta, nt, tt, psi);
    for (int m = 0; m < n; ++m) {
        double acc = 0.0;
        for (int j = 0; j < nt; ++j) {
            const double wgt = (j == 0 || j == nt - 1) ? 1.0 : ((j % 2) ? 4.0 : 2.0);
            acc += wgt * f[j] * psi[(size_t)m * nt + j];
        }
        g[m] = acc * dt / 3.0;
    }
    free(psi);
    free(tt);
}
