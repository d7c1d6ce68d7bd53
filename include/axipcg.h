/*
 * axipcg — preconditioned conjugate gradients for the axisymmetric
 * variable-coefficient elliptic operator, on one AMD Instinct MI355X (gfx950).
 *
 * Method: A.V. Terekhov, "High performance parallel algorithm for solving
 * elliptic equations with non-separable variables" (arXiv:1002.3094).
 * Section and equation numbers below are the paper's.
 *
 * Problem (§2.1 eq. (2)):
 *     (1/r) d/dr (r kappa du/dr) + d/dz (kappa du/dz) - q u = -f
 * on [0, lr] x [0, lz], with r kappa du/dr = 0 on the axis, u = 0 at r = lr,
 * and either u = 0 (Dirichlet) or du/dz = 0 (Neumann, the paper's choice) at
 * z = 0 and z = lz.  kappa > 0, q >= 0 (eq. (3)).
 *
 * Discretisation (eqs. (4)-(6), cell-centred reading): nr x nz cells,
 * h_r = lr/nr, h_z = lz/nz, r_i = (i+1/2) h_r.  The discrete operator A is the
 * r-weighted finite-volume scheme, symmetric positive definite (eq. (7)); the
 * discrete right-hand side is b = r f.  Boundary faces with u = 0 use the
 * half-cell flux (doubled face conductance).
 *
 * Preconditioner (§4.2 eqs. (36)-(39)): B = A with kappa = kbar and q = qbar
 * everywhere, inverted by separation of variables: an orthonormal sine
 * (Dirichlet) or cosine (Neumann) transform along z, one tridiagonal solve in r
 * per z-mode, the inverse transform.
 *
 * Conventions for every entry point:
 *  - Grid arrays are [nr][nz] row-major, z contiguous, 0-based, IEEE double
 *    unless stated.  "device" pointers are HIP device memory of the calling
 *    process' current device (e.g. torch tensors); "host" pointers are host
 *    memory.  The caller owns every array it passes; the library never keeps
 *    a caller pointer after the call returns.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    stream-ordered: device outputs are valid once the stream reaches the
 *    call's position; entry points that return host values synchronise the
 *    stream before returning.
 *  - An operator handle owns its device buffers and workspace.  It must not be
 *    used from two streams (or two host threads) at the same time.
 *  - Arguments are validated before any device work; on failure the call
 *    returns AXIPCG_EINVAL (or another negative code), writes no output, and
 *    axipcg_last_error() describes the problem.  C++ exceptions never cross
 *    this interface.
 */
#ifndef AXIPCG_H
#define AXIPCG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct axipcg_op *axipcg_op_t;

/* Status codes.  AXIPCG_ENOTCONV is positive: the call completed and its
 * outputs hold the last iterate. */
enum {
    AXIPCG_OK = 0,
    AXIPCG_ENOTCONV = 1,
    AXIPCG_EINVAL = -1,
    AXIPCG_ENOMEM = -2,
    AXIPCG_EDEVICE = -3,
    AXIPCG_EBREAKDOWN = -4
};

enum { AXIPCG_Z_DIRICHLET = 0, AXIPCG_Z_NEUMANN = 1 };

/* Grid flag, OR-ed into bc_z of op_create / op_create_faces.  Without it the
 * grid is cell-centred: h_r = lr/nr, h_z = lz/nz, r_i = (i+1/2) h_r, and the
 * boundaries lie on cell faces (the Dirichlet face at r = lr half a step from
 * the last unknown, its conductance doubled).  With it the r-grid is the
 * paper's (§2.1): nodes at (i - 1/2) h_r, i = 1..N_1, h_r = lr/(N_1 - 1/2),
 * so the last node lies on r = lr and carries u = 0; the nr = N_1 - 1 unknown
 * rows give h_r = lr/(nr + 1/2), and the coupling to the boundary node keeps
 * its plain conductance.  z stays cell-centred (h_z = lz/nz): the paper's
 * cosine basis of eq. (38) with its one-sided boundary flux is exact for a
 * Neumann wall at N_2 h_z, which h_z = lz/(N_2 - 1/2) would put half a step
 * beyond z = lz (first order).  The flag requires AXIPCG_Z_NEUMANN, the
 * paper's z condition. */
enum { AXIPCG_GRID_NODES = 0x100 };

/* Arithmetic of the preconditioner.  The outer PCG vectors, dot products,
 * residual recurrence and stop test are FP64 in both cases. */
enum { AXIPCG_PREC_FP64 = 0, AXIPCG_PREC_FP32 = 1 };

/* pcg_solve flags (and batch_solve's) */
enum {
    AXIPCG_FLAG_TRUE_RESIDUAL = 1u,  /* also compute ||b - A x|| / ||b|| at exit */
    AXIPCG_FLAG_POLAK_RIBIERE = 2u,  /* beta = r.(z - z_old) / rho_old (flexible CG) */
    AXIPCG_FLAG_SINGLE_LAUNCH = 4u   /* batch_solve only: the whole solve in one launch */
};

typedef struct {
    int iters;          /* PCG iterations performed */
    int status;         /* AXIPCG_OK, AXIPCG_ENOTCONV or AXIPCG_EBREAKDOWN */
    double relres_rec;  /* ||r_k|| / ||b|| from the recurrence */
    double relres_true; /* ||b - A x|| / ||b|| if requested, else -1 */
} axipcg_stats;

/* ---- operator setup (§2.1 eqs. (4)-(6); §4.2 eqs. (36)-(37)) ---------------
 * Build the operator from cell-centre kappa and q (host arrays [nr][nz]).
 * Face values of kappa are the mean of the two adjacent cells (the boundary
 * face takes its cell's value).  kbar <= 0 selects the mean of kappa, qbar < 0
 * the mean of q (the paper's footnote to eq. (37) uses the mid-range; PCG is
 * invariant to scaling B, so this only changes iteration counts).
 * Limits: 2 <= nr <= 4096; nz a power of two with 2 <= nz <= 4096 (rows of
 * 4096 take the block-wide transforms and the per-mode r-solve); lr, lz > 0;
 * kappa > 0 and q >= 0, all finite.  Allocates ~ (10 * 8) bytes per cell of
 * device memory.  *out receives the handle. */
int axipcg_op_create(int nr, int nz, double lr, double lz, int bc_z,
                     const double *kappa, const double *q,
                     double kbar, double qbar, void *stream, axipcg_op_t *out);

/* Same, with kappa given directly at the faces (host arrays):
 * kappa_r [nr][nz] at (rho_{i+1/2}, z_k), i = nr-1 being the face r = lr;
 * kappa_z [nr][nz+1] at (r_i, k h_z), k = 0 and k = nz the faces z = 0, lz.
 * kbar must be > 0 and qbar >= 0 (no default). */
int axipcg_op_create_faces(int nr, int nz, double lr, double lz, int bc_z,
                           const double *kappa_r, const double *kappa_z, const double *q,
                           double kbar, double qbar, void *stream, axipcg_op_t *out);

/* Release the handle and its device memory (NULL-safe).  Synchronises the
 * stream the handle was created on. */
void axipcg_op_destroy(axipcg_op_t op);

/* Sizes and preconditioner constants of a handle (any pointer may be NULL). */
int axipcg_op_info(axipcg_op_t op, int *nr, int *nz, double *kbar, double *qbar);

/* ---- operator application (§2.1 eq. (4)) ---------------------------------
 * y = A x; x, y device [nr][nz]; x and y must not overlap. */
int axipcg_apply_A(axipcg_op_t op, const double *x, double *y, void *stream);

/* b = r f (eq. (6)); f, b device [nr][nz]; may alias. */
int axipcg_rhs_from_f(axipcg_op_t op, const double *f, double *b, void *stream);

/* ---- preconditioner (§4.2 eqs. (36)-(39)) --------------------------------
 * z = B^{-1} r; r, z device [nr][nz] (must not overlap).  prec selects the
 * arithmetic of the transforms and r-solves (AXIPCG_PREC_FP32 reads r as
 * double, computes in float, writes z as double). */
int axipcg_precond_apply(axipcg_op_t op, const double *r, double *z, int prec, void *stream);

/* ---- strip-partitioned preconditioner (default where it applies) --------
 * precond_apply and the solves run the preconditioner as three launches over
 * strips of R consecutive r-rows (the partition idea of §3, eqs. (18)-(22),
 * with the strips as the parts): (1) the z-transform of each strip's rows and
 * the elimination of its interior rows in terms of the strips' last rows, (2)
 * per z-mode the tridiagonal system of those last rows (nr/R unknowns), (3)
 * the strips' interior rows and the inverse transform.  It applies when nz is
 * 256..2048 (FP32) or 256..1024 (FP64) and nr is a multiple of R with
 * nr/R <= 1024; otherwise, or when set_strips disables it for the handle, the
 * per-mode r-solve of eq. (39) over the whole line runs instead.  Both
 * compute the same B^{-1} r up to rounding.  set_strips takes 0 (off), 1 (on,
 * the default height R = 4), 4 or 8; other values return AXIPCG_EINVAL.
 * Standalone FP32 applies of rows of length 2048 use strips of 8 rows
 * (faster there), and the solves' FP32 launches at that length use strips of
 * 4 whatever the height (their in-loop kernels need the registers of 4-wave
 * workgroups); strips_info reports the solves' strips.
 * strips_info reports whether the strip form is used for `prec` and its
 * strip count (host pointers, may be NULL). */
int axipcg_op_set_strips(axipcg_op_t op, int enable);
int axipcg_op_strips_info(axipcg_op_t op, int prec, int *active, int *strips);

/* ---- single-launch preconditioner (opt-in) -------------------------------
 * The strip form in one cooperative launch: the three phases separated by
 * two grid barriers, the strips' forward-eliminated spectra kept in LDS
 * between the phases (only three values per strip and mode cross
 * workgroups), for FP32.  set_fused(op, 1) enables it for the handle's
 * standalone FP32 applies (strips of 8 rows for nz = 2048, else 4) and for
 * the iterations of its FP32 PCG solves (strips of 4; the x, r update, the
 * stop test and the r.z partials in the same launch, after the SpMV), where
 * every strip's workgroup fits the chip at once and nz is 256..2048; the
 * three launches run otherwise.  Barriers are numbered from a per-handle
 * launch counter, and every wait is bounded: a barrier that gives up fills
 * the strip's output with NaN, marks a PCG solve broken down and sets the
 * handle's error word.  fused_info(op, kind, ...) reports for kind
 * AXIPCG_FUSED_APPLY (0) or AXIPCG_FUSED_PCG (1) whether the single launch
 * is used and its strip count, and (synchronising the device) whether a
 * barrier ever gave up (host pointers, may be NULL). */
enum { AXIPCG_FUSED_APPLY = 0, AXIPCG_FUSED_PCG = 1 };
int axipcg_op_set_fused(axipcg_op_t op, int enable);
int axipcg_op_fused_info(axipcg_op_t op, int kind, int *active, int *strips, int *barrier_errors);

/* out_host[0] = ||b - A x||_2, out_host[1] = ||b||_2 (host double[2]).
 * b, x device.  Synchronises the stream. */
int axipcg_residual_norm(axipcg_op_t op, const double *b, const double *x,
                         double *out_host, void *stream);

/* ---- PCG (§2.2 eq. (8) with conjugate-gradient parameters) -----------------
 * Solve A x = b.  x (device) holds the initial guess on entry and the last
 * iterate on return; b device.  Stops when ||r_k|| / ||b|| <= rtol, r_k the
 * recursively updated residual (§4.3 stop test), or after maxit iterations.
 * st (host, may be NULL) receives the statistics.  Returns AXIPCG_OK,
 * AXIPCG_ENOTCONV (maxit reached) or AXIPCG_EBREAKDOWN (p.Ap <= 0 or a
 * non-finite scalar; x holds the last iterate).  b = 0 gives x = 0.
 * Synchronises the stream (the iteration count is decided on the device and
 * read back in chunks).  rtol > 0, 1 <= maxit <= 100000. */
int axipcg_pcg_solve(axipcg_op_t op, const double *b, double *x, double rtol, int maxit,
                     int prec, unsigned flags, axipcg_stats *st, void *stream);

/* ---- Chebyshev iteration (§2.2 eq. (8) with Chebyshev parameters) ---------
 * The two-step scheme of eq. (8) with tau = 2 / (gamma1 + gamma2) and
 * alpha_1 = 1, alpha_2 = 2 / (2 - rho0^2), alpha_{k+1} = 4 / (4 - rho0^2
 * alpha_k), rho0 = (1 - xi) / (1 + xi), xi = gamma1 / gamma2, where
 * gamma1 <= (Au,u)/(Bu,u) <= gamma2 (eq. (10)).  Run in increment form
 * (d_k = (alpha_{k+1} - 1) d_{k-1} + alpha_{k+1} tau B^{-1} r_k,
 * x += d_k, r -= A d_k): no dot products except ||r||^2 for the stop test
 * ||r_k|| / ||b|| <= rtol.  gamma1 = gamma2 = 0 takes the operator's own
 * bounds (op_bounds); bounds that do not contain the spectrum may diverge
 * (reported as AXIPCG_ENOTCONV or AXIPCG_EBREAKDOWN).  x: initial guess in,
 * solution out (device).  Synchronises the stream; uses the handle's PCG
 * workspace. */
int axipcg_cheb_solve(axipcg_op_t op, const double *b, double *x, double gamma1, double gamma2,
                      double rtol, int maxit, int prec, axipcg_stats *st, void *stream);
/* The operator's energy-equivalence bounds of eq. (10) for its B: the extreme
 * ratios kappa_face / kbar over faces with non-zero conductance and q / qbar
 * over cells (when qbar > 0).  gamma1 is 0 when some q is 0 and qbar > 0. */
int axipcg_op_bounds(axipcg_op_t op, double *gamma1, double *gamma2);

/* Lanczos estimates of the spectrum of B^{-1} A taken out of `steps` PCG
 * steps (§2.2 eq. (8) with conjugate-gradient parameters) from x = 0 on
 * A x = b: the extreme eigenvalues of the Lanczos matrix (diagonal
 * 1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j).
 * They lie inside the spectrum and approach its ends as the steps grow, so
 * gamma1 suits the Chebyshev form as its lower parameter where eq. (10) gives
 * none (components below it are still damped), with eq. (10)'s gamma2 as the
 * upper one.  b: device [nr][nz], non-zero; steps in [1, 1000]; prec as for
 * pcg_solve; gamma1, gamma2, steps_done (the steps completed; fewer when the
 * residual vanishes): host pointers, each may be NULL.  Uses the handle's
 * work vectors (not b).  Synchronises the stream after every step. */
int axipcg_op_bounds_lanczos(axipcg_op_t op, const double *b, int steps, int prec, double *gamma1,
                             double *gamma2, int *steps_done, void *stream);

/* ---- batched PCG over independent problems (§2.2 eq. (8) for each) ---------
 * Solve A_p x_p = b_p for p < n at once; ops[p] are distinct handles (each
 * problem uses its handle's workspace), b[p] and x[p] device pointers of that
 * handle's size (host arrays of n pointers).  Every PCG phase is one launch
 * over the whole batch, so the launch count per iteration does not grow with
 * n; each problem stops on its own test.  st (host, may be NULL) receives n
 * statistics.  Returns the worst status (AXIPCG_EBREAKDOWN, then
 * AXIPCG_ENOTCONV, else AXIPCG_OK).  Members need nr <= 1024 and 4 <= nz <= 2048; all
 * handles must live on the current device.  Synchronises the stream.
 *
 * flags as for pcg_solve, plus AXIPCG_FLAG_SINGLE_LAUNCH: the whole solve,
 * start to stop, in one cooperative launch whose resident workgroups take the
 * same phases in turn with grid barriers between them (the host reads the
 * states once, at the end).  The same operations in the same order as the
 * launch-per-phase form (results equal up to the compiler's fused
 * multiply-adds).  Members need nz <= 1024 and the device cooperative launches
 * (else AXIPCG_EINVAL); AXIPCG_EDEVICE if a grid barrier gives up (every
 * wait is bounded). */
int axipcg_batch_solve(int n, const axipcg_op_t *ops, const double *const *b, double *const *x,
                       double rtol, int maxit, int prec, unsigned flags, axipcg_stats *st, void *stream);

/* The Chebyshev form of eq. (8) (as axipcg_cheb_solve) for every problem of
 * a batch, one launch per phase over the whole batch, with no inner products
 * but ||r||^2 for the stop test.  gamma1, gamma2: host arrays of n bounds
 * 0 < gamma1[p] <= gamma2[p] of the spectrum of B^{-1} A_p; NULL, or both
 * entries <= 0, takes member p's own energy-equivalence bounds (eq. (10),
 * which need gamma1 > 0: every q > 0 or qbar = 0).  ops, b, x, st, the member
 * limits and the return value as for axipcg_batch_solve; flags: 0 or
 * AXIPCG_FLAG_TRUE_RESIDUAL.  Each member's p0 work buffer holds its
 * increment.  Synchronises the stream. */
int axipcg_batch_cheb_solve(int n, const axipcg_op_t *ops, const double *const *b, double *const *x,
                            const double *gamma1, const double *gamma2, double rtol, int maxit, int prec,
                            unsigned flags, axipcg_stats *st, void *stream);

/* ---- Laguerre series (§4.1 eqs. (34)-(35), alpha = 0) ----------------------
 * g_m = int_0^{t_max} f(t) l_m(t) dt, l_m(t) = sqrt(eta) e^{-eta t/2} L_m(eta t),
 * for m < n, from nt >= 3 uniform samples f_host[j] = f(j t_max/(nt-1)) (host).
 * The integral is the trapezoid rule (exact to machine precision for pulses
 * that vanish smoothly at both ends).  g_host: host double[n]. */
int axipcg_laguerre_coeffs(int n, double eta, int nt, double t_max,
                           const double *f_host, double *g_host, void *stream);

/* Right-hand side of harmonic m (eq. (35)):
 *     b = r * (g_m delta_h - c * sum_{k<m} (m-k) u_k)
 * kept as two running sums (device [nr][nz], caller-owned, zero before m = 0):
 *     S1 += u_prev (skipped when u_prev is NULL, i.e. m = 0);  S2 += S1;
 *     b = r g_m delta_h - r c S2.
 * delta_h is the discrete point source at cell (src_i, src_k): r delta_h =
 * 1/(h_r h_z) there and 0 elsewhere.  c is `coef` (device [nr][nz], e.g.
 * eta^2/c^2) or, when coef is NULL, 4 q: the paper's damping and history
 * coefficients are h^2/(4 rho^2) and h^2/rho^2.  u_prev may not alias S1, S2
 * or b. */
int axipcg_laguerre_rhs(axipcg_op_t op, double g_m, int src_i, int src_k,
                        const double *coef, const double *u_prev,
                        double *S1, double *S2, double *b, void *stream);

/* ---- Laguerre series with integer alpha >= 0 (§4.1 eqs. (34)-(35)) --------
 * The transform of eq. (34): Q_m = int u(t) psi_m(t) dt and
 * u(t) = sum_m Q_m phi_m(t), with psi_m(t) = sqrt(eta m!/(m+alpha)!)
 * e^{-eta t/2} L^alpha_m(eta t) and phi_m(t) = (eta t)^alpha psi_m(t)
 * (alpha = 0 gives the functions of axipcg_laguerre_coeffs).
 *
 * f_m = int_0^{t_max} f psi_m dt for m < n from nt >= 3 uniform host samples
 * (trapezoid rule), into g_host (host double[n]); 0 <= alpha <= 64. */
int axipcg_laguerre_coeffs_alpha(int n, int alpha, double eta, int nt, double t_max,
                                 const double *f_host, double *g_host, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same as
 * axipcg_laguerre_coeffs_alpha and the same kernel, with the staged samples
 * and coefficients in a fixed device array of the library (1 MiB per device,
 * held until the process ends) instead of per-call hipMalloc'd buffers.  It
 * calls no hipMalloc, hipFree or other allocating routine.  Limit:
 * nt + n <= 131072, else AXIPCG_EINVAL.  Synchronises `stream` before
 * returning.  Every call on one device shares that array: calls that overlap
 * on one device (two host threads, or two streams) race. */
int axipcg_laguerre_coeffs_alpha_noalloc(int n, int alpha, double eta, int nt, double t_max,
                                         const double *f_host, double *g_host, void *stream);
/* Right-hand side of harmonic m of eq. (35) with alpha:
 *     b = r * (f_m delta_h - c * c_m * sum_{k<m} (m-k) d_k u_k),
 *     c_m = sqrt(m!/(m+alpha)!),  d_k = sqrt((k+alpha)!/k!),
 * through the running sums S1 += d_{m-1} u_prev, S2 += S1 (device, zero
 * before m = 0).  u_prev is u_{m-1}: NULL exactly when m = 0.  c, delta_h,
 * coef and aliasing rules as for axipcg_laguerre_rhs. */
int axipcg_laguerre_rhs_alpha(axipcg_op_t op, int m, int alpha, double g_m, int src_i, int src_k,
                              const double *coef, const double *u_prev, double *S1, double *S2,
                              double *b, void *stream);
/* out[j] = u[idx[j]] for j < n (receiver samples of a harmonic; u, idx, out
 * device, idx flat indices into the op's [nr][nz] grid, 1 <= n <= 65536; an
 * index outside the grid yields NaN). */
int axipcg_gather(axipcg_op_t op, const double *u, const long long *idx, int n, double *out, void *stream);
/* Time traces from harmonics (eq. (34)): traces[r][j] = sum_{m<n} Q[m][r]
 * phi_m(t_j), t_j = j t_max/(nt-1); Q device [n][nrec], traces device
 * [nrec][nt]. */
int axipcg_laguerre_synth(int n, int alpha, double eta, int nrec, const double *Q, int nt, double t_max,
                          double *traces, void *stream);

/* ---- initial guess from earlier harmonics (§4.1: the harmonics are solved in
 * order, so u_{m-1} = u1 and u_{m-2} = u2 are known when harmonic m starts) ----
 * Writes to x whichever of u1 and the linear extrapolation 2 u1 - u2 has the
 * smaller residual |b - A x| (the extrapolation only when strictly smaller).
 * Device [nr][nz] arrays of op's size; x may alias u1 or u2, not b.
 * resid_host (host double[2]: extrapolation, u1) and choice_host (0 u1,
 * 1 extrapolation) may be NULL; when either is given the call synchronises
 * the stream.  Uses the handle's workspace: do not overlap with a solve on
 * the same handle. */
int axipcg_guess_extrap(axipcg_op_t op, const double *b, const double *u1, const double *u2, double *x,
                        double *resid_host, int *choice_host, void *stream);
/* The same guard over K = 1..7 earlier harmonics hist[j] = u_{m-1-j} (host
 * array of device [nr][nz] arrays): candidate p < K is the polynomial
 * extrapolation of order p through u_{m-1}, ..., u_{m-1-p},
 *     x_p = sum_{i <= p} (-1)^i C(p+1, i+1) u_{m-1-i}
 * (u_{m-1}; 2u_{m-1} - u_{m-2}; 3u_{m-1} - 3u_{m-2} + u_{m-3}; ...), taken in
 * order, a higher order replacing the choice only when its residual is
 * strictly smaller.  resid_host (host double[K], order p at p) and
 * choice_host (the order) may be NULL; when either is given the call
 * synchronises the stream.  x may alias a history array, not b.  Uses the
 * handle's workspace like guess_extrap. */
int axipcg_guess_poly(axipcg_op_t op, const double *b, const double *const *hist, int K, double *x,
                      double *resid_host, int *choice_host, void *stream);

/* ---- learned initial guess (extension; §4.1's harmonics are solved in order,
 * so u_{m-1} and u_{m-2} are known when harmonic m starts) ---------------------
 * A 6-layer 3x3 convolutional network, 32 channels wide, ReLU between layers,
 * zero padding, BF16 weights and activations with FP32 accumulation.  Inputs
 * (device [nr][nz] doubles): u1 = u_{m-1}, u2 = u_{m-2}, b = right-hand side
 * of harmonic m, kappa per cell.  With s = RMS(u1) and s_b = RMS(b) (1 where
 * zero) the channels are u1/s, u2/s, b/s_b, (kappa - 2.5)/1.5, and the guess
 * is x_P + s * out, x_P the polynomial extrapolation of the handle's base
 * order P (guess_poly's candidate P; P = 1, the default, is the linear
 * 2 u1 - u2), so a network whose last layer is zero returns x_P.  Parameters (host float[axipcg_nn_num_params()]):
 * for each layer l = 0..5, W_l[t][ci][co] (t = 3 (di+1) + (dk+1) over the
 * 3x3 window in (r, z), ci < cin_l, co < cout_l; cin = 4,32,32,32,32,32,
 * cout = 32,...,32,1) then bias_l[co].  The handle owns device copies, the
 * activations of the last forward and the Adam moments; sizes: nr in
 * [1, 8192], nz a multiple of 64 in [64, 8192].  Calls on one handle must not
 * overlap. */
typedef struct axipcg_nn *axipcg_nn_t;
int axipcg_nn_num_params(void);
int axipcg_nn_create(int nr, int nz, const float *params, axipcg_nn_t *out);
void axipcg_nn_destroy(axipcg_nn_t nn);
/* Copy parameters and/or the last gradients to host float arrays (either may
 * be NULL).  Synchronises the device. */
int axipcg_nn_get_params(axipcg_nn_t nn, float *params, float *grads);
/* Replace the parameters (finite values only); Adam moments are kept. */
int axipcg_nn_set_params(axipcg_nn_t nn, const float *params);
/* The base order P in [1, 6] (default 1).  With P > 1 the base reads
 * u_{m-1}, ..., u_{m-1-P}, so only the history-form calls take the network
 * (nn_guess_poly and series_step / series_run with AXIPCG_GUESS_NN_POLY with
 * K > P arrays, nn_backward_poly); nn_forward, nn_guess, nn_backward and
 * AXIPCG_GUESS_NN then return AXIPCG_EINVAL.  nn_get_base returns P (or
 * AXIPCG_EINVAL for a NULL handle). */
int axipcg_nn_set_base(axipcg_nn_t nn, int order);
int axipcg_nn_get_base(axipcg_nn_t nn);
/* guess = 2 u1 - u2 + s * net(u1, u2, b, kappa), unguarded (device
 * [nr][nz]; guess may alias u1 or u2, not b or kappa); base order 1 only. */
int axipcg_nn_forward(axipcg_nn_t nn, const double *u1, const double *u2, const double *b,
                      const double *kappa, double *guess, void *stream);
/* Training loss of the last forward (or nn_guess) against the solved
 * harmonic u_target: with e = 2 u1 - u2 + s * out - u_target,
 *     L = e^T A e / (s^2 nr nz)   (the energy norm of the guess error),
 * A the operator of op (same sizes), and its gradient w.r.t. every parameter
 * (kept on the device; nn_get_params reads it).  u1 and u2 must be the
 * forward's.  loss_host (may be NULL) receives L and then the call
 * synchronises the stream. */
int axipcg_nn_backward(axipcg_op_t op, axipcg_nn_t nn, const double *u1, const double *u2,
                       const double *u_target, double *loss_host, void *stream);
/* The same for any base order: e = x_P + s * out - u_target with x_P formed
 * from hist[0..P] (host array of K > P device arrays, hist[0] = u_{m-1},
 * hist[1] = u_{m-2} as read by the last nn_guess_poly, unchanged since). */
int axipcg_nn_backward_poly(axipcg_op_t op, axipcg_nn_t nn, const double *const *hist, int K,
                            const double *u_target, double *loss_host, void *stream);
/* One Adam step with the last gradients (bias-corrected moments, step count
 * kept by the handle). */
int axipcg_nn_adam(axipcg_nn_t nn, double lr, double beta1, double beta2, double eps, void *stream);
/* Guarded guess for PCG: runs the network, then writes to x the candidate
 * among u1, 2 u1 - u2 and the network guess with the smallest residual
 * |b - A x| (a later candidate must be strictly smaller; a NaN never wins).
 * x may alias u1 or u2, not b or kappa.  resid_host (host double[3]: network,
 * extrapolation, u1) and choice_host (0 u1, 1 extrapolation, 2 network) may
 * be NULL; when either is given the call synchronises the stream. */
int axipcg_nn_guess(axipcg_op_t op, axipcg_nn_t nn, const double *b, const double *u1, const double *u2,
                    const double *kappa, double *x, double *resid_host, int *choice_host, void *stream);
/* The learned guess among the polynomial extrapolations of guess_poly:
 * the network reads hist[0] = u_{m-1} and hist[1] = u_{m-2} (K = P+1..7 for
 * base order P) and its candidate (x_P plus its correction) comes after
 * the K extrapolations.  resid_host (host double[K + 1]: orders 0..K-1, then
 * the network) and choice_host (the order, or K for the network) may be
 * NULL; when either is given the call synchronises the stream.  x may alias a
 * history array, not b or kappa. */
int axipcg_nn_guess_poly(axipcg_op_t op, axipcg_nn_t nn, const double *b, const double *const *hist, int K,
                         const double *kappa, double *x, double *resid_host, int *choice_host, void *stream);

/* ---- one harmonic of a Laguerre series (§4.1 eqs. (34)-(35); §2.2 eq. (8)) --
 * The calls a series makes for harmonic m, queued back to back so that the
 * device never waits for the host between them: b = the right-hand side of
 * harmonic m (laguerre_rhs, u_prev = u1 when m > 0), the initial guess into x
 * (guess: AXIPCG_GUESS_ZERO, _PREV = u1, _EXTRAP = guess_extrap,
 * _NN = nn_guess with nn and kappa), then the solve (solver 0: pcg_solve with
 * flags 0; 1: cheb_solve with the operator's own bounds).  The only host wait
 * is the solve's own state read.  Arguments, ownership and errors are those
 * of the individual calls (nn and kappa may be NULL unless guess is _NN); x
 * must not alias b, S1, S2, u1 or u2.  st (host, may be NULL) receives the
 * solve's statistics; the return value is the solve's status. */
enum {
    AXIPCG_GUESS_ZERO = 0,
    AXIPCG_GUESS_PREV = 1,
    AXIPCG_GUESS_EXTRAP = 2,
    AXIPCG_GUESS_NN = 3,
    AXIPCG_GUESS_POLY = 4,     /* guess_poly over AXIPCG_POLY_HISTORY harmonics (series_run only) */
    AXIPCG_GUESS_NN_POLY = 5,  /* nn_guess_poly over as many (series_run only) */
    AXIPCG_POLY_HISTORY = 7
};
int axipcg_series_step(axipcg_op_t op, axipcg_nn_t nn, int m, double g_m, int src_i, int src_k,
                       const double *coef, double *S1, double *S2, double *b, const double *u1,
                       const double *u2, const double *kappa, double *x, int guess, int solver,
                       double rtol, int maxit, int prec, axipcg_stats *st, void *stream);
/* Harmonics m0, m0 + 1, ..., m0 + count - 1 of the same series in one call,
 * each as series_step, with no return to the caller between them.  g (host,
 * count values): g_{m0}, g_{m0+1}, ....  u (host array of three distinct
 * device [nr][nz] arrays): {u_{m0-1}, u_{m0-2}, work} on entry (at m0 = 0
 * the first two only feed the initial guess: zero them); each harmonic solves
 * into the work array and the three pointers rotate, so that on return u[0]
 * holds u_{m0+count-1}, u[1] u_{m0+count-2} and u[2] is free.  st (host,
 * count entries, may be NULL) receives each solve's statistics; done (host,
 * may be NULL) the number of harmonics completed.  With the polynomial
 * guesses (AXIPCG_GUESS_POLY, _NN_POLY) u holds AXIPCG_POLY_HISTORY + 1 = eight
 * arrays, {u_{m0-1}, ..., u_{m0-7}, work}, rotated the same way (u[0] the
 * last solution, u[1] the one before, ...).  A harmonic that does not
 * converge is kept and the run goes on (the return value is then
 * AXIPCG_ENOTCONV); a breakdown or any other error stops the run at that
 * harmonic with its code, leaving u as it was before it. */
int axipcg_series_run(axipcg_op_t op, axipcg_nn_t nn, int m0, int count, const double *g, int src_i, int src_k,
                      const double *coef, double *S1, double *S2, double *b, double **u, const double *kappa,
                      int guess, int solver, double rtol, int maxit, int prec, axipcg_stats *st, int *done,
                      void *stream);
/* The paper's experiment (§4.3) over harmonics m0 .. m0 + count - 1 in one
 * call: for each, the right-hand side of eq. (35) with alpha
 * (laguerre_rhs_alpha, u_prev = u[0] when m > 0), a zero
 * (AXIPCG_GUESS_ZERO), previous-harmonic (AXIPCG_GUESS_PREV) or polynomial
 * extrapolation (AXIPCG_GUESS_POLY, as guess_poly over the last
 * AXIPCG_POLY_HISTORY harmonics) initial guess in the work array, the solve
 * (solver 0 PCG, 1 Chebyshev with the operator's
 * bounds), and the receiver samples Q[m][r] = u_m[rec_idx[r]] (axipcg_gather;
 * Q device [m0 + count][n_rec] at least, rec_idx device; n_rec = 0 skips
 * them).  g (host): g_{m0} ... .  u (host array of distinct device
 * arrays): {u_{m0-1}, work} on entry, or {u_{m0-1}, ..., u_{m0-7}, work} for
 * AXIPCG_GUESS_POLY, rotated after each harmonic as in series_run, so that on
 * return u[0] holds the last solution.  st, done and the error behaviour as
 * for axipcg_series_run. */
int axipcg_series_run_alpha(axipcg_op_t op, int m0, int count, int alpha, const double *g, int src_i, int src_k,
                            const double *coef, double *S1, double *S2, double *b, double **u,
                            const long long *rec_idx, int n_rec, double *Q, int guess, int solver, double rtol,
                            int maxit, int prec, axipcg_stats *st, int *done, void *stream);

/* ---- per-kernel timing (tracing aid) ----------------------------------------
 * Select one kernel class of the PCG iteration; pcg_solve then brackets one
 * launch in `every` (>= 1) of that class with a pair of HIP events on the
 * caller's stream -- sampling keeps the events' own cost out of a timed loop
 * -- and, once the solve has synchronised, adds the elapsed times of the
 * bracketed launches that did work (iterations before the stop test fired).
 * AXIPCG_KERNEL_NONE turns the timing off (the default).  profile_read
 * returns the accumulated time and launch count (host pointers, may be NULL)
 * and clears them if reset. */
enum {
    AXIPCG_KERNEL_NONE = -1,
    AXIPCG_KERNEL_SPMV = 0,    /* p update, q = A p, p.q           */
    AXIPCG_KERNEL_ZFWD = 1,    /* x, r update, ||r||^2, transform  */
    AXIPCG_KERNEL_TRIDIAG = 2, /* r-solves, one per z-mode         */
    AXIPCG_KERNEL_ZINV = 3     /* inverse transform, r.z           */
};
int axipcg_profile_select(axipcg_op_t op, int kernel, int every);
int axipcg_profile_read(axipcg_op_t op, double *total_ms, long long *launches, int reset);

/* ---- errors ---------------------------------------------------------------- */
const char *axipcg_strerror(int code);
/* Message of the last failing call on this host thread ("" if none). */
const char *axipcg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AXIPCG_H */
