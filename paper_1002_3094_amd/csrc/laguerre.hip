// Laguerre series helpers (§4.1 eqs. (34)-(35)): coefficients of the source
// pulse, right-hand sides of the harmonics (alpha = 0 and general integer
// alpha), receiver samples and the synthesis of time traces.
#include <cmath>
#include <mutex>

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

// S1 += du u_prev; S2 += S1; b = r (g delta - c cs S2), c = coef or 4 q.
// (alpha = 0: du = cs = 1, and the products are exact.)
__global__ void __launch_bounds__(256)
k_laguerre_rhs(const double *__restrict__ u_prev, double *__restrict__ S1, double *__restrict__ S2,
               double *__restrict__ b, const double *__restrict__ coef, const double *__restrict__ W,
               const double *__restrict__ rw, int nr, int nz, int si, int sk, double src, double du, double cs)
{
    const size_t n = (size_t)nr * nz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double s1 = S1[e];
        if (u_prev) {
            s1 += du * u_prev[e];
            S1[e] = s1;
        }
        const double s2 = S2[e] + s1;
        S2[e] = s2;
        const int i = (int)(e / nz);
        const double cr = coef ? coef[e] * rw[i] : 4.0 * W[e];
        double v = -cr * (cs * s2);
        if (e == (size_t)si * nz + sk) v += src;
        b[e] = v;
    }
}

// Normalised generalized Laguerre functions by their recurrence:
// ell_m(x) = sqrt(eta) rt_m e^{-x/2} L^alpha_m(x), rt_m = sqrt(m!/(m+alpha)!),
// stepped as (m+1) ell_{m+1} = (2m+1+alpha-x) ell_m s1 - (m+alpha) ell_{m-1} s2
// with s1 = rt_{m+1}/rt_m, s2 = rt_{m+1}/rt_{m-1} (no factorial is formed).
struct LagStep {
    double a = 0.0, b;   // ell_{m-1}, ell_m
    int m = 0;
    __device__ LagStep(double x, double eta, int alpha)
    {
        double r0 = 1.0;   // rt_0 = 1/sqrt(alpha!)
        for (int k = 2; k <= alpha; ++k) r0 /= sqrt((double)k);
        b = sqrt(eta) * r0 * exp(-0.5 * x);
    }
    __device__ void next(double x, int alpha)
    {
        const double m1 = m + 1.0;
        const double s1 = sqrt(m1 / (m1 + alpha));
        const double s2 = (m > 0) ? s1 * sqrt(m / (m + (double)alpha)) : 0.0;
        const double c = ((2.0 * m + 1.0 + alpha - x) * b * s1 - (m + alpha) * a * s2) / m1;
        a = b;
        b = c;
        ++m;
    }
};

// f_m = int f(t) psi_m(t) dt, psi_m(t) = ell_m(eta t) (the projection kernel of
// eq. (34)), by the trapezoid rule; workgroup m steps the recurrence to m at
// every sample.
__global__ void __launch_bounds__(256)
k_laguerre_coeffs_a(const double *__restrict__ f, int nt, double dt, double eta, int alpha, double *__restrict__ g)
{
    __shared__ double red[8];
    const int m = blockIdx.x;
    double acc = 0.0;
    for (int j = threadIdx.x; j < nt; j += blockDim.x) {
        const double x = eta * (j * dt);
        LagStep l(x, eta, alpha);
        for (int k = 0; k < m; ++k) l.next(x, alpha);
        const double wgt = (j == 0 || j == nt - 1) ? 0.5 * dt : dt;
        acc += wgt * f[j] * l.b;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) g[m] = s;
}

// out[j] = u[idx[j]] for the receivers (NaN for an index outside the grid)
__global__ void __launch_bounds__(64)
k_gather(const double *__restrict__ u, const long long *__restrict__ idx, int n, long long total,
         double *__restrict__ out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const long long q = idx[j];
    out[j] = (q >= 0 && q < total) ? u[q] : __builtin_nan("");
}

// traces[r][j] = sum_m Q[m][r] phi_m(t_j), phi_m(t) = (eta t)^alpha psi_m(t)
// (eq. (34)); one thread per time sample runs the recurrence over m.
__global__ void __launch_bounds__(256)
k_laguerre_synth(const double *__restrict__ Q, int n, int nrec, int nt, double dt, double eta, int alpha,
                 double *__restrict__ traces)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nt) return;
    const double x = eta * (j * dt);
    double xa = 1.0;
    for (int k = 0; k < alpha; ++k) xa *= x;
    constexpr int RB = 16;   // receivers per pass
    for (int r0 = 0; r0 < nrec; r0 += RB) {
        double acc[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[q] = 0.0;
        LagStep l(x, eta, alpha);
        for (int m = 0; m < n; ++m) {
            const double ph = xa * l.b;
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (r0 + q < nrec) acc[q] += Q[(size_t)m * nrec + r0 + q] * ph;
            if (m + 1 < n) l.next(x, alpha);
        }
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (r0 + q < nrec) traces[(size_t)(r0 + q) * nt + j] = acc[q];
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
                           S2, b, coef, op->W, op->rw64, op->nr, op->nz, src_i, src_k, src, 1.0, 1.0);
        AXI_CHECK_HIP(hipGetLastError());
        return AXIPCG_OK;
    });
}

// sqrt((k + alpha)! / k!) in FP64 through lgamma (k, alpha >= 0)
static double lag_ratio(int k, int alpha)
{
    return std::exp(0.5 * (std::lgamma(k + alpha + 1.0) - std::lgamma(k + 1.0)));
}

extern "C" int axipcg_laguerre_coeffs_alpha(int n, int alpha, double eta, int nt, double t_max, const double *f_host,
                                            double *g_host, void *stream)
{
    return guarded([&] {
        AXI_REQUIRE(n >= 1 && n <= 100000, "n must be in [1, 100000]");
        AXI_REQUIRE(alpha >= 0 && alpha <= 64, "alpha must be in [0, 64]");
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
        hipLaunchKernelGGL(k_laguerre_coeffs_a, dim3(n), dim3(256), 0, s, d_f, nt, t_max / (nt - 1), eta, alpha, d_g);
        AXI_CHECK_HIP(hipGetLastError());
        AXI_CHECK_HIP(hipMemcpyAsync(g_host, d_g, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        return AXIPCG_OK;
    });
}

// ---- allocation-free variant of axipcg_laguerre_coeffs_alpha ---------------
// The staged pulse samples and the coefficients live in one file-scope device
// array instead of two hipMalloc'd buffers.  Each device holds its own copy;
// host code reaches it only through the address hipGetSymbolAddress returns
// for that device (the array's name in host code is a stand-in, not a device
// address).
namespace {

constexpr size_t NOALLOC_DOUBLES = size_t(1) << 17;   // 1 MiB per device: nt + n <= 131072
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

std::mutex g_scratch_mu;
double *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Address of `scratch` on the current device, looked up once per device.
double *scratch_on_current_device()
{
    int dev = -1;
    AXI_CHECK_HIP(hipGetDevice(&dev));
    AXI_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        AXI_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        AXI_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int axipcg_laguerre_coeffs_alpha_noalloc(int n, int alpha, double eta, int nt, double t_max,
                                                    const double *f_host, double *g_host, void *stream)
{
    return guarded([&] {
        AXI_REQUIRE(n >= 1 && n <= 100000, "n must be in [1, 100000]");
        AXI_REQUIRE(alpha >= 0 && alpha <= 64, "alpha must be in [0, 64]");
        AXI_REQUIRE(nt >= 3, "nt must be >= 3");
        AXI_REQUIRE((size_t)nt + (size_t)n <= NOALLOC_DOUBLES,
                    "nt + n exceeds the 131072 doubles of the allocation-free scratch");
        AXI_REQUIRE(std::isfinite(eta) && eta > 0 && std::isfinite(t_max) && t_max > 0, "eta, t_max must be > 0");
        AXI_REQUIRE(f_host && g_host, "NULL argument");
        for (int j = 0; j < nt; ++j) AXI_REQUIRE(std::isfinite(f_host[j]), "f has non-finite values");
        hipStream_t s = (hipStream_t)stream;
        double *d_f = scratch_on_current_device();
        double *d_g = d_f + nt;
        AXI_CHECK_HIP(hipMemcpyAsync(d_f, f_host, sizeof(double) * nt, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_laguerre_coeffs_a, dim3(n), dim3(256), 0, s, d_f, nt, t_max / (nt - 1), eta, alpha, d_g);
        AXI_CHECK_HIP(hipGetLastError());
        AXI_CHECK_HIP(hipMemcpyAsync(g_host, d_g, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        return AXIPCG_OK;
    });
}

extern "C" int axipcg_laguerre_rhs_alpha(axipcg_op_t h, int m, int alpha, double g_m, int src_i, int src_k,
                                         const double *coef, const double *u_prev, double *S1, double *S2, double *b,
                                         void *stream)
{
    return guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(h);
        AXI_REQUIRE(op && S1 && S2 && b, "NULL argument");
        AXI_REQUIRE(m >= 0 && alpha >= 0 && alpha <= 64, "need m >= 0 and alpha in [0, 64]");
        AXI_REQUIRE((m == 0) == (u_prev == nullptr), "u_prev is NULL exactly when m = 0");
        AXI_REQUIRE(std::isfinite(g_m), "g_m must be finite");
        AXI_REQUIRE(src_i >= 0 && src_i < op->nr && src_k >= 0 && src_k < op->nz, "source cell out of range");
        AXI_REQUIRE(S1 != S2 && S1 != b && S2 != b, "S1, S2 and b must be distinct");
        AXI_REQUIRE(!u_prev || (u_prev != S1 && u_prev != S2 && u_prev != b), "u_prev aliases an output");
        const size_t n = (size_t)op->nr * op->nz;
        const double src = g_m / (op->hr * op->hz);
        const double du = (m > 0) ? lag_ratio(m - 1, alpha) : 0.0;   // d_{m-1}
        const double cs = 1.0 / lag_ratio(m, alpha);                  // c_m
        hipLaunchKernelGGL(k_laguerre_rhs, dim3(pointwise_blocks(n)), dim3(256), 0, (hipStream_t)stream, u_prev, S1,
                           S2, b, coef, op->W, op->rw64, op->nr, op->nz, src_i, src_k, src, du, cs);
        AXI_CHECK_HIP(hipGetLastError());
        return AXIPCG_OK;
    });
}

extern "C" int axipcg_gather(axipcg_op_t h, const double *u, const long long *idx, int n, double *out, void *stream)
{
    return guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(h);
        AXI_REQUIRE(op && u && idx && out, "NULL argument");
        AXI_REQUIRE(n >= 1 && n <= 65536, "n must be in [1, 65536]");
        hipLaunchKernelGGL(k_gather, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, u, idx, n,
                           (long long)op->nr * op->nz, out);
        AXI_CHECK_HIP(hipGetLastError());
        return AXIPCG_OK;
    });
}

extern "C" int axipcg_laguerre_synth(int n, int alpha, double eta, int nrec, const double *Q, int nt, double t_max,
                                     double *traces, void *stream)
{
    return guarded([&] {
        AXI_REQUIRE(n >= 1 && n <= 100000 && nrec >= 1 && nrec <= 4096, "need 1 <= n <= 100000, 1 <= nrec <= 4096");
        AXI_REQUIRE(alpha >= 0 && alpha <= 64, "alpha must be in [0, 64]");
        AXI_REQUIRE(nt >= 2 && std::isfinite(eta) && eta > 0 && std::isfinite(t_max) && t_max > 0,
                    "need nt >= 2 and eta, t_max > 0");
        AXI_REQUIRE(Q && traces, "NULL argument");
        hipLaunchKernelGGL(k_laguerre_synth, dim3((nt + 255) / 256), dim3(256), 0, (hipStream_t)stream, Q, n, nrec,
                           nt, t_max / (nt - 1), eta, alpha, traces);
        AXI_CHECK_HIP(hipGetLastError());
        return AXIPCG_OK;
    });
}
