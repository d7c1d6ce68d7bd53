// One harmonic of a Laguerre series (§4.1 eqs. (34)-(35)) as one library
// call: right-hand side, initial guess and solve are queued back to back on
// the caller's stream, so the device does not idle while the host returns
// between them; and a run of harmonics as one call, so that the caller's own
// per-harmonic overhead is not paid between them either.  Composed of the
// public entry points; no arithmetic here.
#include "axipcg.h"
#include "kernels.h"

using namespace axipcg;

namespace {

// sync_end = false: return once the host has seen the solve's outcome, with
// the tail of its last chunk possibly still queued (see pcg_solve_entry).
// Number of earlier harmonics a guess mode reads.
int history_of(int guess)
{
    return (guess == AXIPCG_GUESS_POLY || guess == AXIPCG_GUESS_NN_POLY) ? AXIPCG_POLY_HISTORY : 2;
}

// hist[j] = u_{m-1-j}, nh = history_of(guess) arrays.
// ah (may be NULL): the cache of A hist[j] for the polynomial guesses (see
// guess_poly_cached).
int series_step_impl(axipcg_op_t hop, axipcg_nn_t nn, int m, double g_m, int src_i, int src_k, const double *coef,
                     double *S1, double *S2, double *b, const double *const *hist, int nh, const double *kappa,
                     double *x, int guess, int solver, double rtol, int maxit, int prec, axipcg_stats *st,
                     void *stream, bool sync_end, double *const *ah = nullptr)
{
    const double *u1 = hist[0], *u2 = hist[1];
    int code = guarded([&] {
        AXI_REQUIRE(hop && S1 && S2 && b && x, "NULL argument");
        for (int j = 0; j < nh; ++j) AXI_REQUIRE(hist[j] != nullptr, "NULL argument");
        AXI_REQUIRE(m >= 0, "m must be >= 0");
        AXI_REQUIRE(guess >= AXIPCG_GUESS_ZERO && guess <= AXIPCG_GUESS_NN_POLY, "unknown guess mode");
        AXI_REQUIRE(nh == history_of(guess), "polynomial guesses need axipcg_series_run");
        AXI_REQUIRE(solver == 0 || solver == 1, "unknown solver");
        AXI_REQUIRE((guess != AXIPCG_GUESS_NN && guess != AXIPCG_GUESS_NN_POLY) || (nn && kappa),
                    "the learned guess needs nn and kappa");
        AXI_REQUIRE(x != b && x != S1 && x != S2, "x aliases another array");
        for (int j = 0; j < nh; ++j) AXI_REQUIRE(x != hist[j], "x aliases another array");
        return AXIPCG_OK;
    });
    if (code != AXIPCG_OK) return code;
    code = axipcg_laguerre_rhs(hop, g_m, src_i, src_k, coef, m > 0 ? u1 : nullptr, S1, S2, b, stream);
    if (code != AXIPCG_OK) return code;
    const Operator *op = reinterpret_cast<const Operator *>(hop);
    const size_t bytes = (size_t)op->nr * op->nz * sizeof(double);
    switch (guess) {
    case AXIPCG_GUESS_ZERO:
        code = guarded([&] {
            AXI_CHECK_HIP(hipMemsetAsync(x, 0, bytes, (hipStream_t)stream));
            return AXIPCG_OK;
        });
        break;
    case AXIPCG_GUESS_PREV:
        code = guarded([&] {
            AXI_CHECK_HIP(hipMemcpyAsync(x, u1, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
            return AXIPCG_OK;
        });
        break;
    case AXIPCG_GUESS_EXTRAP:
        code = axipcg_guess_extrap(hop, b, u1, u2, x, nullptr, nullptr, stream);
        break;
    case AXIPCG_GUESS_NN:
        code = axipcg_nn_guess(hop, nn, b, u1, u2, kappa, x, nullptr, nullptr, stream);
        break;
    case AXIPCG_GUESS_POLY:
        if (ah)
            code = guarded([&] {
                guess_poly_cached(*reinterpret_cast<Operator *>(hop), nullptr, b, hist, nh, ah, nullptr, x,
                                  (hipStream_t)stream);
                return AXIPCG_OK;
            });
        else
            code = axipcg_guess_poly(hop, b, hist, nh, x, nullptr, nullptr, stream);
        break;
    default:
        if (ah)
            code = guarded([&] {
                guess_poly_cached(*reinterpret_cast<Operator *>(hop), nn, b, hist, nh, ah, kappa, x,
                                  (hipStream_t)stream);
                return AXIPCG_OK;
            });
        else
            code = axipcg_nn_guess_poly(hop, nn, b, hist, nh, kappa, x, nullptr, nullptr, stream);
        break;
    }
    if (code != AXIPCG_OK) return code;
    if (solver == 1) return cheb_solve_entry(hop, b, x, 0.0, 0.0, rtol, maxit, prec, st, stream, sync_end);
    return pcg_solve_entry(hop, b, x, rtol, maxit, prec, 0u, st, stream, sync_end);
}

}  // namespace

extern "C" int axipcg_series_step(axipcg_op_t hop, axipcg_nn_t nn, int m, double g_m, int src_i, int src_k,
                                  const double *coef, double *S1, double *S2, double *b, const double *u1,
                                  const double *u2, const double *kappa, double *x, int guess, int solver,
                                  double rtol, int maxit, int prec, axipcg_stats *st, void *stream)
{
    const double *hist[2] = {u1, u2};
    return series_step_impl(hop, nn, m, g_m, src_i, src_k, coef, S1, S2, b, hist, 2, kappa, x, guess, solver, rtol,
                            maxit, prec, st, stream, true);
}

extern "C" int axipcg_series_run(axipcg_op_t hop, axipcg_nn_t nn, int m0, int count, const double *g, int src_i,
                                 int src_k, const double *coef, double *S1, double *S2, double *b, double **u,
                                 const double *kappa, int guess, int solver, double rtol, int maxit, int prec,
                                 axipcg_stats *st, int *done, void *stream)
{
    if (done) *done = 0;
    const int nh = history_of(guess);
    int code = guarded([&] {
        AXI_REQUIRE(m0 >= 0 && count >= 0, "m0 and count must be >= 0");
        AXI_REQUIRE(count == 0 || g != nullptr, "g is NULL");
        AXI_REQUIRE(u != nullptr, "u is NULL");
        for (int j = 0; j <= nh; ++j) {
            AXI_REQUIRE(u[j] != nullptr, "u must hold the history arrays and a work array");
            for (int i = 0; i < j; ++i) AXI_REQUIRE(u[i] != u[j], "the u arrays must be distinct");
        }
        return AXIPCG_OK;
    });
    if (code != AXIPCG_OK) return code;
    // the polynomial guesses keep A u of the history arrays (one application
    // of A per harmonic instead of nh): filled here for u[1..nh-1], rotated
    // with u, u[0]'s written by each harmonic's guard
    double *ah[AXIPCG_POLY_HISTORY + 1] = {};
    const bool poly = (guess == AXIPCG_GUESS_POLY || guess == AXIPCG_GUESS_NN_POLY) && count > 0;
    if (poly) {
        code = guarded([&] {
            Operator *op = reinterpret_cast<Operator *>(hop);
            AXI_REQUIRE(op != nullptr, "NULL argument");
            const size_t n = (size_t)op->nr * op->nz;
            if (!op->au_cache)
                AXI_CHECK_HIP(hipMalloc((void **)&op->au_cache, sizeof(double) * n * AXIPCG_POLY_HISTORY));
            for (int i = 0; i < nh; ++i) ah[i] = op->au_cache + (size_t)i * n;
            for (int i = 1; i < nh; ++i) apply_a_pairs(*op, u[i], ah[i], (hipStream_t)stream);
            return AXIPCG_OK;
        });
        if (code != AXIPCG_OK) return code;
    }
    // between harmonics the host does not wait for the stream to drain: the
    // next right-hand side is queued behind the tail of the previous solve
    int worst = AXIPCG_OK;
    for (int j = 0; j < count; ++j) {
        code = series_step_impl(hop, nn, m0 + j, g[j], src_i, src_k, coef, S1, S2, b, u, nh, kappa, u[nh], guess,
                                solver, rtol, maxit, prec, st ? st + j : nullptr, stream, false, poly ? ah : nullptr);
        if (code < 0) {              // the failed harmonic's buffers keep their roles
            (void)hipStreamSynchronize((hipStream_t)stream);
            return code;
        }
        if (code == AXIPCG_ENOTCONV) worst = AXIPCG_ENOTCONV;
        double *w = u[nh - 1];       // the oldest harmonic becomes the next work array
        for (int i = nh - 1; i > 0; --i) u[i] = u[i - 1];
        u[0] = u[nh];
        u[nh] = w;
        if (poly) {                  // A u moves with u; the new u[0]'s is computed next
            double *wa = ah[nh - 1];
            for (int i = nh - 1; i > 0; --i) ah[i] = ah[i - 1];
            ah[0] = wa;
        }
        if (done) *done = j + 1;
    }
    code = guarded([&] {
        AXI_CHECK_HIP(hipStreamSynchronize((hipStream_t)stream));
        return AXIPCG_OK;
    });
    return code != AXIPCG_OK ? code : worst;
}

extern "C" int axipcg_series_run_alpha(axipcg_op_t hop, int m0, int count, int alpha, const double *g, int src_i,
                                       int src_k, const double *coef, double *S1, double *S2, double *b,
                                       double **u, const long long *rec_idx, int n_rec, double *Q, int guess,
                                       int solver, double rtol, int maxit, int prec, axipcg_stats *st, int *done,
                                       void *stream)
{
    if (done) *done = 0;
    const bool poly = guess == AXIPCG_GUESS_POLY;
    const int nh = poly ? AXIPCG_POLY_HISTORY : 1;   // earlier harmonics kept; u[nh] is the work array
    int code = guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(hop);
        AXI_REQUIRE(op != nullptr, "NULL operator");
        AXI_REQUIRE(m0 >= 0 && count >= 0, "m0 and count must be >= 0");
        AXI_REQUIRE(count == 0 || g != nullptr, "g is NULL");
        AXI_REQUIRE(guess == AXIPCG_GUESS_ZERO || guess == AXIPCG_GUESS_PREV || poly,
                    "guess must be zero, prev or poly");
        AXI_REQUIRE(u != nullptr, "u is NULL");
        for (int a = 0; a <= nh; ++a) {
            AXI_REQUIRE(u[a] != nullptr, "u must hold the history arrays and a work array");
            AXI_REQUIRE(u[a] != b && u[a] != S1 && u[a] != S2, "u aliases b, S1 or S2");
            for (int c = 0; c < a; ++c) AXI_REQUIRE(u[c] != u[a], "the u arrays must be distinct");
        }
        AXI_REQUIRE(solver == 0 || solver == 1, "unknown solver");
        AXI_REQUIRE(n_rec == 0 || (rec_idx && Q), "receivers need rec_idx and Q");
        return AXIPCG_OK;
    });
    if (code != AXIPCG_OK) return code;
    Operator *op = reinterpret_cast<Operator *>(hop);
    const size_t bytes = (size_t)op->nr * op->nz * sizeof(double);
    hipStream_t s = (hipStream_t)stream;
    double *ah[AXIPCG_POLY_HISTORY + 1] = {};
    if (poly && count > 0) {         // the cache of A u, as in series_run
        code = guarded([&] {
            const size_t n = (size_t)op->nr * op->nz;
            if (!op->au_cache)
                AXI_CHECK_HIP(hipMalloc((void **)&op->au_cache, sizeof(double) * n * AXIPCG_POLY_HISTORY));
            for (int i = 0; i < nh; ++i) ah[i] = op->au_cache + (size_t)i * n;
            for (int i = 1; i < nh; ++i) apply_a_pairs(*op, u[i], ah[i], s);
            return AXIPCG_OK;
        });
        if (code != AXIPCG_OK) return code;
    }
    int worst = AXIPCG_OK;
    for (int j = 0; j < count; ++j) {
        const int m = m0 + j;
        double *u1 = u[0], *x = u[nh];
        code = axipcg_laguerre_rhs_alpha(hop, m, alpha, g[j], src_i, src_k, coef, m > 0 ? u1 : nullptr, S1, S2, b,
                                         stream);
        if (code == AXIPCG_OK)
            code = guarded([&] {
                if (guess == AXIPCG_GUESS_ZERO) AXI_CHECK_HIP(hipMemsetAsync(x, 0, bytes, s));
                else if (guess == AXIPCG_GUESS_PREV)
                    AXI_CHECK_HIP(hipMemcpyAsync(x, u1, bytes, hipMemcpyDeviceToDevice, s));
                else
                    guess_poly_cached(*op, nullptr, b, u, nh, ah, nullptr, x, s);
                return AXIPCG_OK;
            });
        if (code == AXIPCG_OK || code == AXIPCG_ENOTCONV)
            code = solver == 1
                       ? cheb_solve_entry(hop, b, x, 0.0, 0.0, rtol, maxit, prec, st ? st + j : nullptr, stream, false)
                       : pcg_solve_entry(hop, b, x, rtol, maxit, prec, 0u, st ? st + j : nullptr, stream, false);
        if (code >= 0 && n_rec > 0) {
            const int gc = axipcg_gather(hop, x, rec_idx, n_rec, Q + (size_t)m * n_rec, stream);
            if (gc != AXIPCG_OK) code = gc;
        }
        if (code < 0) {              // the failed harmonic's buffers keep their roles
            (void)hipStreamSynchronize(s);
            return code;
        }
        if (code == AXIPCG_ENOTCONV) worst = AXIPCG_ENOTCONV;
        double *w = u[nh - 1];       // rotate as in series_run
        for (int i = nh - 1; i > 0; --i) u[i] = u[i - 1];
        u[0] = u[nh];
        u[nh] = w;
        if (poly) {
            double *wa = ah[nh - 1];
            for (int i = nh - 1; i > 0; --i) ah[i] = ah[i - 1];
            ah[0] = wa;
        }
        if (done) *done = j + 1;
    }
    code = guarded([&] {
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        return AXIPCG_OK;
    });
    return code != AXIPCG_OK ? code : worst;
}
