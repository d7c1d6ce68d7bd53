// Lanczos estimates of the spectrum of B^{-1} A out of a few PCG steps (§2.2
// eq. (8) with conjugate-gradient parameters), for the Chebyshev form's
// parameters where the energy bounds of eq. (10) give no positive lower bound
// (media with cells where q = 0 while the preconditioner keeps a q term).
//
// The steps run from x = 0 on A x = b with the handle's work vectors, driven
// from the host (each step reads its two inner products back): alpha_j =
// r_j.z_j / p_j.A p_j, beta_j = r_{j+1}.z_{j+1} / r_j.z_j.  The Lanczos matrix
// of B^{-1} A in the B inner product (its vectors are the normalised
// residuals) is then
//     T[j][j]   = 1 / alpha_j + beta_{j-1} / alpha_{j-1},
//     T[j][j+1] = sqrt(beta_j) / alpha_j,
// and its extreme eigenvalues, found by bisection on Sturm counts, are Ritz
// values: inside the spectrum of B^{-1} A, approaching its ends as the steps
// grow.  Inner products are deterministic (fixed-order partial sums).
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.h"

namespace axipcg {
namespace {

constexpr int LZ_BLOCKS = 512;

struct LzBuf {
    double *p = nullptr;
    ~LzBuf() { if (p) (void)hipFree(p); }
};

// One partial of a.b per workgroup (grid-stride order), then their sum.
__global__ void __launch_bounds__(256) k_lz_dot(const double *__restrict__ a, const double *__restrict__ b, size_t n,
                                                double *__restrict__ part)
{
    __shared__ double red[8];
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        s += a[e] * b[e];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_lz_fin(const double *__restrict__ part, int nb, double *__restrict__ out)
{
    __shared__ double red[8];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) *out = t;
}

// r -= alpha q
__global__ void __launch_bounds__(256) k_lz_axpy(double *__restrict__ r, const double *__restrict__ q, double alpha,
                                                 size_t n)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        r[e] -= alpha * q[e];
}

// p = z + beta p
__global__ void __launch_bounds__(256) k_lz_xpay(double *__restrict__ p, const double *__restrict__ z, double beta,
                                                 size_t n)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        p[e] = z[e] + beta * p[e];
}

double dot_host(const double *a, const double *b, size_t n, double *buf, hipStream_t s)
{
    hipLaunchKernelGGL(k_lz_dot, dim3(LZ_BLOCKS), dim3(256), 0, s, a, b, n, buf);
    AXI_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_lz_fin, dim3(1), dim3(256), 0, s, buf, LZ_BLOCKS, buf + LZ_BLOCKS);
    AXI_CHECK_HIP(hipGetLastError());
    double v = 0.0;
    AXI_CHECK_HIP(hipMemcpyAsync(&v, buf + LZ_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
    AXI_CHECK_HIP(hipStreamSynchronize(s));
    return v;
}

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x (Sturm
// count of the LDL^T pivots).
int sturm_below(const std::vector<double> &d, const std::vector<double> &e, double x)
{
    int c = 0;
    double q = 1.0;
    for (size_t j = 0; j < d.size(); ++j) {
        const double e2 = j > 0 ? e[j - 1] * e[j - 1] : 0.0;
        q = d[j] - x - (j > 0 ? e2 / q : 0.0);
        if (q == 0.0) q = -1e-300;   // x on an eigenvalue of the leading block: count it below
        if (q < 0.0) ++c;
    }
    return c;
}

// The k-th smallest eigenvalue (k = 1 .. m) by bisection inside the
// Gershgorin interval.
double tri_eig(const std::vector<double> &d, const std::vector<double> &e, int k)
{
    double lo = d[0], hi = d[0];
    for (size_t j = 0; j < d.size(); ++j) {
        const double rad = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < d.size() ? std::fabs(e[j]) : 0.0);
        lo = std::min(lo, d[j] - rad);
        hi = std::max(hi, d[j] + rad);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_below(d, e, mid) >= k) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

int lanczos_impl(Operator &op, const double *b, int steps, int prec, double *g1, double *g2, int *done,
                 hipStream_t s)
{
    const size_t n = (size_t)op.nr * op.nz;
    double *r = op.r, *z = op.z, *p = op.p0, *q = op.q;
    LzBuf buf;
    AXI_CHECK_HIP(hipMalloc(&buf.p, sizeof(double) * (LZ_BLOCKS + 1)));
    const unsigned blocks = pointwise_blocks(n);
    AXI_CHECK_HIP(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    precond_apply_impl(op, r, z, prec, s);
    AXI_CHECK_HIP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    double rho = dot_host(r, z, n, buf.p, s);
    AXI_REQUIRE(std::isfinite(rho) && rho > 0.0, "b must be non-zero and finite (b.B^-1 b > 0)");
    std::vector<double> alpha, beta;
    for (int j = 0; j < steps && rho > 0.0; ++j) {
        apply_a_pairs(op, p, q, s);
        const double pq = dot_host(p, q, n, buf.p, s);
        if (!(pq > 0.0) || !std::isfinite(pq)) break;   // breakdown: keep the steps so far
        const double a = rho / pq;
        hipLaunchKernelGGL(k_lz_axpy, dim3(blocks), dim3(256), 0, s, r, q, a, n);
        AXI_CHECK_HIP(hipGetLastError());
        precond_apply_impl(op, r, z, prec, s);
        const double rho_new = dot_host(r, z, n, buf.p, s);
        alpha.push_back(a);
        beta.push_back(std::isfinite(rho_new) && rho_new > 0.0 ? rho_new / rho : 0.0);
        hipLaunchKernelGGL(k_lz_xpay, dim3(blocks), dim3(256), 0, s, p, z, beta.back(), n);
        AXI_CHECK_HIP(hipGetLastError());
        rho = rho_new;
    }
    AXI_REQUIRE(!alpha.empty(), "no PCG step completed (p.A p <= 0)");
    const size_t m = alpha.size();
    std::vector<double> d(m), e(m > 0 ? m - 1 : 0);
    for (size_t j = 0; j < m; ++j) d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    for (size_t j = 0; j + 1 < m; ++j) e[j] = std::sqrt(beta[j]) / alpha[j];
    if (g1) *g1 = tri_eig(d, e, 1);
    if (g2) *g2 = tri_eig(d, e, (int)m);
    if (done) *done = (int)m;
    return AXIPCG_OK;
}

}  // namespace
}  // namespace axipcg

using namespace axipcg;

extern "C" int axipcg_op_bounds_lanczos(axipcg_op_t h, const double *b, int steps, int prec, double *gamma1,
                                        double *gamma2, int *steps_done, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op && b, "NULL argument");
        AXI_REQUIRE(steps >= 1 && steps <= 1000, "steps must be in [1, 1000]");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        return lanczos_impl(*op, b, steps, prec, gamma1, gamma2, steps_done, (hipStream_t)stream);
    });
}
