// Host-side launchers shared between the library's translation units.
#pragma once

#include "common.h"

namespace axipcg {

// Forward z-transform of every r-row (§4.2 eq. (38)).
//  plain: spec = S rin
//  fused PCG step (iteration after SpMV): x += alpha p, r -= alpha q,
//    ||r||^2 reduced into state->rr (iteration counter and stop test updated
//    by the last block), then spec = S r.
struct ZfwdArgs {
    const double *rin = nullptr;           // plain mode input
    double *x = nullptr, *r = nullptr;     // fused mode
    const double *p = nullptr, *q = nullptr;
    PcgState *state = nullptr;             // fused: gate + scalars
    bool fused = false;
};
void launch_zfwd(const Operator &op, int prec, const ZfwdArgs &a, hipStream_t s);

// One r-tridiagonal solve per z-mode, in place on op.spec (§4.2 eq. (39)).
void launch_tridiag(const Operator &op, int prec, const PcgState *gate, hipStream_t s);

// Inverse z-transform of every row: zout = S^T spec.
//  mode 0: plain;  mode 1: PCG step, rho' = r.z reduced, beta and rho
//  updated by the last block (Polak-Ribiere if state->flags asks);
//  mode 2: PCG start, rho = r.z, beta = 0.
struct ZinvArgs {
    double *zout = nullptr;
    const double *r = nullptr;
    PcgState *state = nullptr;
    int mode = 0;
};
void launch_zinv(const Operator &op, int prec, const ZinvArgs &a, hipStream_t s);

// z = B^{-1} r with three launches (forward, r-solves, inverse).
void precond_apply_impl(const Operator &op, const double *r, double *z, int prec, hipStream_t s);

// Flattened grid geometry for pointwise kernels.
inline unsigned pointwise_blocks(size_t n, int threads = 256)
{
    size_t b = (n + threads - 1) / threads;
    if (b > (size_t)MAX_PARTIALS) b = MAX_PARTIALS;
    return (unsigned)b;
}

}  // namespace axipcg
