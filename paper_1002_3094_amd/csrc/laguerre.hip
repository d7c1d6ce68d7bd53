// Laguerre series helpers (§4.1 eqs. (34)-(35), alpha = 0).
#include <cmath>

#include "kernels.h"

namespace axipcg {
namespace {

// g_m = int f(t) sqrt(eta) e^{-eta t/2} L_m(eta t) dt by the trapezoid rule on
// the uniform samples; workgroup m evaluates L_m at every node through the
// three-term recurrence (k+1) L_{k+1} = (2k+1-x) L_k - k L_{k-1}.
__global__ void __launch_bounds__(256)
k_laguerre_coeffs(const double *__restrict__ f, int nt, double dt, double eta, double *__restrict__ g)
{
    __shared__ double red[8];
    const int m = blockIdx.x;
    double acc = 0.0;
    for (int j = threadIdx.x; j < nt; j += blockDim.x) {
        const double xx = eta * (j * dt);
        double lm1 = 0.0, l0 = 1.0;
        for (int k = 0; k < m; ++k) {
            const double l1 = ((2.0 * k + 1.0 - xx) * l0 - k * lm1) / (k + 1.0);
            lm1 = l0;
            l0 = l1;
        }
        const double wgt = (j == 0 || j == nt - 1) ? 0.5 * dt : dt;
        acc += wgt * f[j] * sqrt(eta) * exp(-0.5 * xx) * l0;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) g[m] = s;
}

// S1 += u_prev; S2 += S1; b = r (g delta - c S2), c = coef or 4 q.
__global__ void __launch_bounds__(256)
k_laguerre_rhs(const double *__restrict__ u_prev, double *__restrict__ S1, double *__restrict__ S2,
               double *__restrict__ b, const double *__restrict__ coef, const double *__restrict__ W,
               const double *__restrict__ rw, int nr, int nz, int si, int sk, double src)
{
    const size_t n = (size_t)nr * nz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double s1 = S1[e];
        if (u_prev) {
            s1 += u_prev[e];
            S1[e] = s1;
        }
        const double s2 = S2[e] + s1;
        S2[e] = s2;
        const int i = (int)(e / nz);
        const double cr = coef ? coef[e] * rw[i] : 4.0 * W[e];
        double v = -cr * s2;
        if (e == (size_t)si * nz + sk) v += src;
        b[e] = v;
    }
}

}  // namespace
}  // namespace axipcg

using namespace axipcg;

extern "C" int axipcg_laguerre_coeffs(int n, double eta, int nt, double t_max, const double *f_host,
                                      double *g_host, void *stream)
{
    return guarded([&] {
        AXI_REQUIRE(n >= 1 && n <= 100000, "n must be in [1, 100000]");
        AXI_REQUIRE(nt >= 3, "nt must be >= 3");
        AXI_REQUIRE(std::isfinite(eta) && eta > 0 && std::isfinite(t_max) && t_max > 0, "eta, t_max must be > 0");
        AXI_REQUIRE(f_host && g_host, "NULL argument");
        for (int j = 0; j < nt; ++j) AXI_REQUIRE(std::isfinite(f_host[j]), "f has non-finite values");
        hipStream_t s = (hipStream_t)stream;
        double *d_f = nullptr, *d_g = nullptr;
        struct Tmp {
            double **a, **b;
            ~Tmp() { if (*a) (void)hipFree(*a); if (*b) (void)hipFree(*b); }
        } tmp{&d_f, &d_g};
        AXI_CHECK_HIP(hipMalloc((void **)&d_f, sizeof(double) * nt));
        AXI_CHECK_HIP(hipMalloc((void **)&d_g, sizeof(double) * n));
        AXI_CHECK_HIP(hipMemcpyAsync(d_f, f_host, sizeof(double) * nt, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_laguerre_coeffs, dim3(n), dim3(256), 0, s, d_f, nt, t_max / (nt - 1), eta, d_g);
        AXI_CHECK_HIP(hipGetLastError());
        AXI_CHECK_HIP(hipMemcpyAsync(g_host, d_g, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        return AXIPCG_OK;
    });
}

extern "C" int axipcg_laguerre_rhs(axipcg_op_t h, double g_m, int src_i, int src_k, const double *coef,
                                   const double *u_prev, double *S1, double *S2, double *b, void *stream)
{
    return guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(h);
        AXI_REQUIRE(op && S1 && S2 && b, "NULL argument");
        AXI_REQUIRE(std::isfinite(g_m), "g_m must be finite");
        AXI_REQUIRE(src_i >= 0 && src_i < op->nr && src_k >= 0 && src_k < op->nz, "source cell out of range");
        AXI_REQUIRE(S1 != S2 && S1 != b && S2 != b, "S1, S2 and b must be distinct");
        AXI_REQUIRE(!u_prev || (u_prev != S1 && u_prev != S2 && u_prev != b), "u_prev aliases an output");
        const size_t n = (size_t)op->nr * op->nz;
        const double src = g_m / (op->hr * op->hz);
        hipLaunchKernelGGL(k_laguerre_rhs, dim3(pointwise_blocks(n)), dim3(256), 0, (hipStream_t)stream, u_prev, S1,
                           S2, b, coef, op->W, op->rw64, op->nr, op->nz, src_i, src_k, src);
        AXI_CHECK_HIP(hipGetLastError());
        return AXIPCG_OK;
    });
}
