// Operator setup (§2.1 eqs. (4)-(6); §4.2 eqs. (36)-(37)), operator
// application and residual norms.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"

namespace axipcg {

namespace {

// kappa at the faces from cell values: the mean of the two adjacent cells,
// the adjacent cell's value on a boundary face.
__global__ void k_face_kappa(const double *__restrict__ kc, double *__restrict__ kr,
                             double *__restrict__ kz, int nr, int nz)
{
    const size_t n = (size_t)nr * nz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nz), k = (int)(e - (size_t)i * nz);
        kr[e] = (i < nr - 1) ? 0.5 * (kc[e] + kc[e + nz]) : kc[e];
        double *kzr = kz + (size_t)i * (nz + 1);
        kzr[k] = (k == 0) ? kc[e] : 0.5 * (kc[e - 1] + kc[e]);
        if (k == nz - 1) kzr[nz] = kc[e];
    }
}

// Scheme coefficients: conductance of a face = (face radius) kappa / h^2;
// faces with u = 0 on the boundary are doubled (half-cell flux), Neumann
// faces carry none, the axis face has radius 0.
__global__ void k_coeffs(const double *__restrict__ kr, const double *__restrict__ kz,
                         const double *__restrict__ q, double *__restrict__ D, double *__restrict__ CR,
                         double *__restrict__ CZ, double *__restrict__ W, int nr, int nz, double hr,
                         double hz, double zb, double rb)
{
    const size_t n = (size_t)nr * nz;
    const double ihr2 = 1.0 / (hr * hr), ihz2 = 1.0 / (hz * hz);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nz), k = (int)(e - (size_t)i * nz);
        const double ri = (i + 0.5) * hr;
        const double up = (i + 1) * hr * kr[e] * ihr2 * (i == nr - 1 ? rb : 1.0);
        const double dn = (i > 0) ? i * hr * kr[e - nz] * ihr2 : 0.0;
        const double *kzr = kz + (size_t)i * (nz + 1);
        const double zd = ri * kzr[k] * ihz2 * (k == 0 ? zb : 1.0);
        const double zu = ri * kzr[k + 1] * ihz2 * (k == nz - 1 ? zb : 1.0);
        const double w = ri * q[e];
        D[e] = up + dn + zd + zu + w;
        CR[e] = (i < nr - 1) ? up : 0.0;
        CZ[e] = (k < nz - 1) ? zu : 0.0;
        W[e] = w;
    }
}

// Deterministic sums of two fields: one partial pair per workgroup (fixed
// grid-stride order), then one workgroup adds the partials in index order.
__global__ void __launch_bounds__(256)
k_sum2_part(const double *__restrict__ a, const double *__restrict__ b, size_t n, double *__restrict__ part)
{
    __shared__ double red[16];
    double sa = 0.0, sb = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        sa += a[e];
        sb += b[e];
    }
    const double ta = block_sum(sa, red);
    const double tb = block_sum(sb, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = ta;
        part[2 * blockIdx.x + 1] = tb;
    }
}

__global__ void __launch_bounds__(1024) k_sum2_fin(const double *__restrict__ part, int nb, double *__restrict__ out)
{
    __shared__ double red[16];
    double sa = 0.0, sb = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        sa += part[2 * i];
        sb += part[2 * i + 1];
    }
    const double ta = block_sum(sa, red);
    const double tb = block_sum(sb, red);
    if (threadIdx.x == 0) {
        out[0] = ta;
        out[1] = tb;
    }
}

// r-line arrays and mode eigenvalues of the preconditioner, FFT tables.
__global__ void k_tables(Operator op, double kbar, double qbar, double rb)
{
    const int nr = op.nr, N = op.nz;
    const double hr = op.hr, hz = op.hz;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nthr = gridDim.x * blockDim.x;
    for (int i = tid; i < nr; i += nthr) {
        const double cbi = (i < nr - 1) ? (i + 1) * hr * kbar / (hr * hr) : 0.0;
        const double up = (i < nr - 1) ? cbi : rb * nr * hr * kbar / (hr * hr);
        const double dn = (i > 0) ? i * hr * kbar / (hr * hr) : 0.0;
        const double ri = (i + 0.5) * hr;
        op.cb64[i] = cbi;
        op.db64[i] = up + dn;
        op.rw64[i] = ri;
        op.cb32[i] = (float)cbi;
        op.db32[i] = (float)(up + dn);
        op.rw32[i] = (float)ri;
    }
    for (int j = tid; j < N; j += nthr) {
        // mode j <-> l = j+1 (sine) or l = j (cosine); mu = (4/hz^2) sin^2(pi l / 2N)
        const int l = (op.bc_z == AXIPCG_Z_DIRICHLET) ? j + 1 : j;
        const double sn = sinpi((double)l / (2.0 * N));
        const double mu = 4.0 / (hz * hz) * sn * sn;
        const double lam = kbar * mu + qbar;
        op.lam64[j] = lam;
        op.lam32[j] = (float)lam;
        const double c = cospi(2.0 * j / N), s = -sinpi(2.0 * j / N);
        op.tw64[j] = make_double2(c, s);
        op.tw32[j] = make_float2((float)c, (float)s);
        const double c2 = cospi(j / (2.0 * N)), s2 = -sinpi(j / (2.0 * N));
        op.pt64[j] = make_double2(c2, s2);
        op.pt32[j] = make_float2((float)c2, (float)s2);
    }
}

// y = A x (5-point stencil with the precomputed diagonal).
__global__ void __launch_bounds__(256)
k_apply(const double *__restrict__ x, double *__restrict__ y, const double *__restrict__ D,
        const double *__restrict__ CR, const double *__restrict__ CZ, int nr, int nz)
{
    const size_t n = (size_t)nr * nz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nz), k = (int)(e - (size_t)i * nz);
        double v = D[e] * x[e];
        if (i + 1 < nr) v -= CR[e] * x[e + nz];
        if (i > 0) v -= CR[e - nz] * x[e - nz];
        if (k + 1 < nz) v -= CZ[e] * x[e + 1];
        if (k > 0) v -= CZ[e - 1] * x[e - 1];
        y[e] = v;
    }
}

__global__ void k_rhs(const double *__restrict__ f, double *__restrict__ b, const double *__restrict__ rw,
                      int nr, int nz)
{
    const size_t n = (size_t)nr * nz;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        b[e] = rw[e / nz] * f[e];
}

// Partial sums of ||b - A x||^2 and ||b||^2, one pair per workgroup.
__global__ void __launch_bounds__(256)
k_resid(const double *__restrict__ b, const double *__restrict__ x, const double *__restrict__ D,
        const double *__restrict__ CR, const double *__restrict__ CZ, int nr, int nz, double *partials)
{
    __shared__ double red[8];
    const size_t n = (size_t)nr * nz;
    double s_r = 0.0, s_b = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nz), k = (int)(e - (size_t)i * nz);
        double v = D[e] * x[e];
        if (i + 1 < nr) v -= CR[e] * x[e + nz];
        if (i > 0) v -= CR[e - nz] * x[e - nz];
        if (k + 1 < nz) v -= CZ[e] * x[e + 1];
        if (k > 0) v -= CZ[e - 1] * x[e - 1];
        const double d = b[e] - v;
        s_r += d * d;
        s_b += b[e] * b[e];
    }
    const double tb = block_sum(s_b, red);
    const double tr = block_sum(s_r, red);
    if (threadIdx.x == 0) {
        partials[SLOT_PQ * MAX_PARTIALS + blockIdx.x] = tr;
        partials[SLOT_MISC * MAX_PARTIALS + blockIdx.x] = tb;
    }
}

__global__ void __launch_bounds__(256)
k_resid_finish(const double *__restrict__ partials, int n, double *out)
{
    __shared__ double red[8];
    const double rt = block_total(partials + SLOT_PQ * MAX_PARTIALS, n, red);
    const double bt = block_total(partials + SLOT_MISC * MAX_PARTIALS, n, red);
    if (threadIdx.x == 0) {
        out[0] = rt;
        out[1] = bt;
    }
}

template <typename P>
void dmalloc(P **p, size_t count)
{
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, count * sizeof(P));
    if (e != hipSuccess) throw Error{AXIPCG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    *p = static_cast<P *>(v);
}

void free_op(Operator *op)
{
    if (!op) return;
    void *ptrs[] = {op->D, op->CR, op->CZ, op->W, op->cb64, op->db64, op->rw64, op->lam64, op->cb32,
                    op->db32, op->rw32, op->lam32, op->tw64, op->pt64, op->tw32, op->pt32, op->r,
                    op->z, op->p0, op->p1, op->q, op->spec, op->partials, op->state, op->dscal,
                    op->pf_bar, op->pf_err, op->strip_red};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (hipEvent_t e : op->prof_events) (void)hipEventDestroy(e);
    if (op->state_host) (void)hipHostFree(op->state_host);
    if (op->scratch_host) (void)hipHostFree(op->scratch_host);
    if (op->mirror_host) (void)hipHostFree(op->mirror_host);
    if (op->au_cache) (void)hipFree(op->au_cache);
    delete op;
}

bool all_finite(const double *a, size_t n) {
    for (size_t e = 0; e < n; ++e)
        if (!std::isfinite(a[e])) return false;
    return true;
}

Operator *create_impl(int nr, int nz, double lr, double lz, int bc_z, const double *kappa_cells,
                      const double *kappa_r, const double *kappa_z, const double *q, double kbar,
                      double qbar, hipStream_t s)
{
    AXI_REQUIRE(nr >= 2 && nr <= 4096, "nr must be in [2, 4096]");
    AXI_REQUIRE(is_pow2(nz) && nz >= 2 && nz <= 4096, "nz must be a power of two in [2, 4096]");
    AXI_REQUIRE(std::isfinite(lr) && lr > 0 && std::isfinite(lz) && lz > 0, "lr and lz must be positive");
    const bool nodes = (bc_z & AXIPCG_GRID_NODES) != 0;
    bc_z &= ~AXIPCG_GRID_NODES;
    AXI_REQUIRE(bc_z == AXIPCG_Z_DIRICHLET || bc_z == AXIPCG_Z_NEUMANN,
                "bc_z must be 0 or 1 (optionally with AXIPCG_GRID_NODES)");
    AXI_REQUIRE(!nodes || bc_z == AXIPCG_Z_NEUMANN, "the node grid is defined with Neumann z");
    AXI_REQUIRE(q != nullptr, "q is NULL");
    const size_t n = (size_t)nr * nz;
    AXI_REQUIRE(all_finite(q, n), "q has non-finite values");
    for (size_t e = 0; e < n; ++e) AXI_REQUIRE(q[e] >= 0.0, "q must be >= 0");
    if (kappa_cells) {
        AXI_REQUIRE(all_finite(kappa_cells, n), "kappa has non-finite values");
        for (size_t e = 0; e < n; ++e) AXI_REQUIRE(kappa_cells[e] > 0.0, "kappa must be > 0");
        AXI_REQUIRE(std::isfinite(kbar) && std::isfinite(qbar), "kbar/qbar must be finite");
    } else {
        AXI_REQUIRE(kappa_r && kappa_z, "face kappa is NULL");
        AXI_REQUIRE(all_finite(kappa_r, n) && all_finite(kappa_z, (size_t)nr * (nz + 1)),
                    "face kappa has non-finite values");
        for (size_t e = 0; e < n; ++e) AXI_REQUIRE(kappa_r[e] > 0.0, "kappa_r must be > 0");
        for (size_t e = 0; e < (size_t)nr * (nz + 1); ++e) AXI_REQUIRE(kappa_z[e] > 0.0, "kappa_z must be > 0");
        AXI_REQUIRE(std::isfinite(kbar) && kbar > 0 && std::isfinite(qbar) && qbar >= 0,
                    "face form needs kbar > 0 and qbar >= 0");
    }
    const int nr_tri_max = 64 * 64;
    AXI_REQUIRE(nr <= nr_tri_max, "nr too large");

    Operator *op = new (std::nothrow) Operator();
    if (!op) throw Error{AXIPCG_ENOMEM, "host allocation failed"};
    try {
        op->nr = nr; op->nz = nz; op->bc_z = bc_z; op->lr = lr; op->lz = lz;
        op->nodes = nodes;
        op->hr = nodes ? lr / (nr + 0.5) : lr / nr;
        op->hz = lz / nz;   // z is cell-centred on both grids
        op->create_stream = s;
        AXI_CHECK_HIP(hipGetDevice(&op->device));
        dmalloc(&op->D, n); dmalloc(&op->CR, n); dmalloc(&op->CZ, n); dmalloc(&op->W, n);
        dmalloc(&op->cb64, nr); dmalloc(&op->db64, nr); dmalloc(&op->rw64, nr); dmalloc(&op->lam64, nz);
        dmalloc(&op->cb32, nr); dmalloc(&op->db32, nr); dmalloc(&op->rw32, nr); dmalloc(&op->lam32, nz);
        dmalloc(&op->tw64, nz); dmalloc(&op->pt64, nz); dmalloc(&op->tw32, nz); dmalloc(&op->pt32, nz);
        dmalloc(&op->r, n); dmalloc(&op->z, n); dmalloc(&op->p0, n); dmalloc(&op->p1, n); dmalloc(&op->q, n);
        dmalloc((double **)&op->spec, n);
        dmalloc(&op->partials, (size_t)PARTIAL_ROWS * MAX_PARTIALS);
        dmalloc(&op->state, 1);
        dmalloc(&op->dscal, 24);
        if (const size_t sb = strip_red_bytes(nr, nz))
            AXI_CHECK_HIP(hipMalloc(&op->strip_red, sb));
        AXI_CHECK_HIP(hipMalloc((void **)&op->pf_bar, (1 + 1024) * sizeof(unsigned)));
        AXI_CHECK_HIP(hipMalloc((void **)&op->pf_err, sizeof(int)));
        AXI_CHECK_HIP(hipMemsetAsync(op->pf_bar, 0, (1 + 1024) * sizeof(unsigned), s));
        AXI_CHECK_HIP(hipMemsetAsync(op->pf_err, 0, sizeof(int), s));
        AXI_CHECK_HIP(hipHostMalloc((void **)&op->state_host, sizeof(PcgState), hipHostMallocDefault));
        AXI_CHECK_HIP(hipHostMalloc((void **)&op->scratch_host, 16 * sizeof(double), hipHostMallocDefault));
        AXI_CHECK_HIP(hipHostMalloc((void **)&op->mirror_host, sizeof(HostMirror),
                                    hipHostMallocCoherent | hipHostMallocMapped));
        *op->mirror_host = HostMirror{};
        AXI_CHECK_HIP(hipHostGetDevicePointer((void **)&op->mirror_dev, op->mirror_host, 0));
        AXI_CHECK_HIP(hipMemsetAsync(op->partials, 0, sizeof(double) * PARTIAL_ROWS * MAX_PARTIALS, s));
        AXI_CHECK_HIP(hipMemsetAsync(op->p0, 0, sizeof(double) * n, s));
        AXI_CHECK_HIP(hipMemsetAsync(op->p1, 0, sizeof(double) * n, s));
        AXI_CHECK_HIP(hipMemsetAsync(op->state, 0, sizeof(PcgState), s));

        // temporaries: kappa at faces and q on the device
        double *d_kr = nullptr, *d_kz = nullptr, *d_q = nullptr, *d_kc = nullptr, *d_kq = nullptr;
        struct Tmp {
            double **p[5];
            ~Tmp() { for (auto pp : p) if (*pp) (void)hipFree(*pp); }
        } tmp{{&d_kr, &d_kz, &d_q, &d_kc, &d_kq}};
        const unsigned blocks = pointwise_blocks(n);
        dmalloc(&d_kr, n); dmalloc(&d_kz, (size_t)nr * (nz + 1)); dmalloc(&d_q, n);
        dmalloc(&d_kq, 2 + 2 * (size_t)blocks);   // the two sums, then the partials
        AXI_CHECK_HIP(hipMemcpyAsync(d_q, q, n * sizeof(double), hipMemcpyHostToDevice, s));
        if (kappa_cells) {
            dmalloc(&d_kc, n);
            AXI_CHECK_HIP(hipMemcpyAsync(d_kc, kappa_cells, n * sizeof(double), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_face_kappa, dim3(blocks), dim3(256), 0, s, d_kc, d_kr, d_kz, nr, nz);
            AXI_CHECK_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_sum2_part, dim3(blocks), dim3(256), 0, s, d_kc, d_q, n, d_kq + 2);
            AXI_CHECK_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_sum2_fin, dim3(1), dim3(1024), 0, s, d_kq + 2, (int)blocks, d_kq);
            AXI_CHECK_HIP(hipGetLastError());
        } else {
            AXI_CHECK_HIP(hipMemcpyAsync(d_kr, kappa_r, n * sizeof(double), hipMemcpyHostToDevice, s));
            AXI_CHECK_HIP(hipMemcpyAsync(d_kz, kappa_z, (size_t)nr * (nz + 1) * sizeof(double),
                                         hipMemcpyHostToDevice, s));
            AXI_CHECK_HIP(hipMemsetAsync(d_kq, 0, 2 * sizeof(double), s));
        }
        hipLaunchKernelGGL(k_coeffs, dim3(blocks), dim3(256), 0, s, d_kr, d_kz, d_q, op->D, op->CR, op->CZ, op->W,
                           nr, nz, op->hr, op->hz, bc_z == AXIPCG_Z_DIRICHLET ? 2.0 : 0.0, nodes ? 1.0 : 2.0);
        AXI_CHECK_HIP(hipGetLastError());
        // means of kappa and q (cells) unless given
        AXI_CHECK_HIP(hipMemcpyAsync(op->scratch_host, d_kq, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        const double kb = kbar > 0 ? kbar : op->scratch_host[0] / (double)n;
        const double qb = qbar >= 0 ? qbar : op->scratch_host[1] / (double)n;
        op->kbar = kb;
        op->qbar = qb;
        // energy-equivalence bounds of eq. (10) for B (kbar, qbar): both
        // quadratic forms are sums of face terms (conductance x squared
        // difference) and cell terms (r q u^2), so gamma1 / gamma2 are the
        // extreme ratios of matching terms where B's is non-zero
        {
            double g1 = INFINITY, g2 = 0.0;
            auto acc = [&](double v) {
                g1 = v < g1 ? v : g1;
                g2 = v > g2 ? v : g2;
            };
            const bool dir = bc_z == AXIPCG_Z_DIRICHLET;
            for (int i = 0; i < nr; ++i)
                for (int k = 0; k < nz; ++k) {
                    const size_t e = (size_t)i * nz + k;
                    if (kappa_cells) {
                        const double kc = kappa_cells[e];
                        acc((i + 1 < nr ? 0.5 * (kc + kappa_cells[e + nz]) : kc) / kb);   // r-face i+1/2
                        if (k + 1 < nz) acc(0.5 * (kc + kappa_cells[e + 1]) / kb);        // z-face k+1/2
                        if (dir && (k == 0 || k == nz - 1)) acc(kc / kb);                 // Dirichlet z-faces
                    } else {
                        acc(kappa_r[e] / kb);
                        const size_t f = (size_t)i * (nz + 1) + k;
                        if (k > 0) acc(kappa_z[f] / kb);
                        if (dir && k == 0) acc(kappa_z[f] / kb);
                        if (dir && k == nz - 1) acc(kappa_z[f + 1] / kb);
                    }
                    if (qb > 0) acc(q[e] / qb);
                }
            op->gamma1 = g1;
            op->gamma2 = g2;
        }
        const int tb = (nr > nz ? nr : nz);
        hipLaunchKernelGGL(k_tables, dim3((tb + 255) / 256), dim3(256), 0, s, *op, kb, qb, nodes ? 1.0 : 2.0);
        AXI_CHECK_HIP(hipGetLastError());
        AXI_CHECK_HIP(hipStreamSynchronize(s));
    } catch (...) {
        free_op(op);
        throw;
    }
    return op;
}

}  // namespace

namespace {
thread_local std::string g_last_error;
}
void set_last_error(const std::string &msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }
const char *last_error_cstr() { return g_last_error.c_str(); }

void apply_impl(const Operator &op, const double *x, double *y, hipStream_t s)
{
    const size_t n = (size_t)op.nr * op.nz;
    hipLaunchKernelGGL(k_apply, dim3(pointwise_blocks(n)), dim3(256), 0, s, x, y, op.D, op.CR, op.CZ, op.nr, op.nz);
    AXI_CHECK_HIP(hipGetLastError());
}

void resid_impl(const Operator &op, const double *b, const double *x, double *out_dev, hipStream_t s)
{
    const size_t n = (size_t)op.nr * op.nz;
    const unsigned nb = pointwise_blocks(n);
    hipLaunchKernelGGL(k_resid, dim3(nb), dim3(256), 0, s, b, x, op.D, op.CR, op.CZ, op.nr, op.nz, op.partials);
    AXI_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_resid_finish, dim3(1), dim3(256), 0, s, op.partials, (int)nb, out_dev);
    AXI_CHECK_HIP(hipGetLastError());
}

}  // namespace axipcg

using namespace axipcg;

extern "C" {

int axipcg_op_create(int nr, int nz, double lr, double lz, int bc_z, const double *kappa, const double *q,
                     double kbar, double qbar, void *stream, axipcg_op_t *out)
{
    return guarded([&] {
        AXI_REQUIRE(out != nullptr, "out is NULL");
        AXI_REQUIRE(kappa != nullptr, "kappa is NULL");
        Operator *op = create_impl(nr, nz, lr, lz, bc_z, kappa, nullptr, nullptr, q, kbar, qbar,
                                   (hipStream_t)stream);
        *out = reinterpret_cast<axipcg_op_t>(op);
        return AXIPCG_OK;
    });
}

int axipcg_op_create_faces(int nr, int nz, double lr, double lz, int bc_z, const double *kappa_r,
                           const double *kappa_z, const double *q, double kbar, double qbar, void *stream,
                           axipcg_op_t *out)
{
    return guarded([&] {
        AXI_REQUIRE(out != nullptr, "out is NULL");
        Operator *op = create_impl(nr, nz, lr, lz, bc_z, nullptr, kappa_r, kappa_z, q, kbar, qbar,
                                   (hipStream_t)stream);
        *out = reinterpret_cast<axipcg_op_t>(op);
        return AXIPCG_OK;
    });
}

void axipcg_op_destroy(axipcg_op_t h)
{
    Operator *op = reinterpret_cast<Operator *>(h);
    if (!op) return;
    (void)hipStreamSynchronize(op->create_stream);
    free_op(op);
}

int axipcg_op_info(axipcg_op_t h, int *nr, int *nz, double *kbar, double *qbar)
{
    return guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        if (nr) *nr = op->nr;
        if (nz) *nz = op->nz;
        if (kbar) *kbar = op->kbar;
        if (qbar) *qbar = op->qbar;
        return AXIPCG_OK;
    });
}

int axipcg_apply_A(axipcg_op_t h, const double *x, double *y, void *stream)
{
    return guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(h);
        AXI_REQUIRE(op && x && y, "NULL argument");
        AXI_REQUIRE(x != y, "x and y must not alias");
        apply_impl(*op, x, y, (hipStream_t)stream);
        return AXIPCG_OK;
    });
}

int axipcg_rhs_from_f(axipcg_op_t h, const double *f, double *b, void *stream)
{
    return guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(h);
        AXI_REQUIRE(op && f && b, "NULL argument");
        const size_t n = (size_t)op->nr * op->nz;
        hipLaunchKernelGGL(k_rhs, dim3(pointwise_blocks(n)), dim3(256), 0, (hipStream_t)stream, f, b, op->rw64,
                           op->nr, op->nz);
        AXI_CHECK_HIP(hipGetLastError());
        return AXIPCG_OK;
    });
}

int axipcg_precond_apply(axipcg_op_t h, const double *r, double *z, int prec, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op && r && z, "NULL argument");
        AXI_REQUIRE(r != z, "r and z must not alias");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        if (op->fused_enabled && prec == AXIPCG_PREC_FP32 && pfused_plan(*op, 0))
            pfused_apply(*op, r, z, (hipStream_t)stream);
        else precond_apply_impl(*op, r, z, prec, (hipStream_t)stream);
        return AXIPCG_OK;
    });
}

int axipcg_op_bounds(axipcg_op_t h, double *gamma1, double *gamma2)
{
    return guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        if (gamma1) *gamma1 = op->gamma1;
        if (gamma2) *gamma2 = op->gamma2;
        return AXIPCG_OK;
    });
}

int axipcg_op_set_fused(axipcg_op_t h, int enable)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        op->fused_enabled = enable != 0;
        return AXIPCG_OK;
    });
}

int axipcg_op_set_strips(axipcg_op_t h, int enable)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        AXI_REQUIRE(enable == 0 || enable == 1 || enable == 4 || enable == 8,
                    "strip height must be 0 (off), 1 (default), 4 or 8");
        op->strip_rows = enable == 1 ? 4 : enable;
        return AXIPCG_OK;
    });
}

int axipcg_op_strips_info(axipcg_op_t h, int prec, int *active, int *strips)
{
    return guarded([&] {
        const Operator *op = reinterpret_cast<const Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        AXI_REQUIRE(prec == AXIPCG_PREC_FP32 || prec == AXIPCG_PREC_FP64, "prec must be 0 or 1");
        const int rows = strip_solve_rows(*op, prec);
        const bool ok = rows > 0 && strip_usable(*op, prec, rows);
        if (active) *active = ok ? 1 : 0;
        if (strips) *strips = ok ? op->nr / rows : 0;
        return AXIPCG_OK;
    });
}

int axipcg_op_fused_info(axipcg_op_t h, int kind, int *active, int *strips, int *barrier_errors)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op != nullptr, "op is NULL");
        AXI_REQUIRE(kind == AXIPCG_FUSED_APPLY || kind == AXIPCG_FUSED_PCG, "kind must be 0 or 1");
        const bool ok = op->fused_enabled && pfused_plan(*op, kind);
        if (active) *active = ok ? 1 : 0;
        if (strips) *strips = ok ? op->pf[kind].G : 0;
        if (barrier_errors) {
            int e = 0;
            AXI_CHECK_HIP(hipDeviceSynchronize());
            AXI_CHECK_HIP(hipMemcpy(&e, op->pf_err, sizeof(int), hipMemcpyDeviceToHost));
            *barrier_errors = e;
        }
        return AXIPCG_OK;
    });
}

int axipcg_residual_norm(axipcg_op_t h, const double *b, const double *x, double *out_host, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(h);
        AXI_REQUIRE(op && b && x && out_host, "NULL argument");
        hipStream_t s = (hipStream_t)stream;
        double *dev = op->dscal;
        resid_impl(*op, b, x, dev, s);
        AXI_CHECK_HIP(hipMemcpyAsync(op->scratch_host, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        AXI_CHECK_HIP(hipStreamSynchronize(s));
        out_host[0] = std::sqrt(op->scratch_host[0]);
        out_host[1] = std::sqrt(op->scratch_host[1]);
        return AXIPCG_OK;
    });
}

const char *axipcg_strerror(int code)
{
    switch (code) {
    case AXIPCG_OK: return "success";
    case AXIPCG_ENOTCONV: return "not converged within maxit";
    case AXIPCG_EINVAL: return "invalid argument";
    case AXIPCG_ENOMEM: return "out of memory";
    case AXIPCG_EDEVICE: return "device error";
    case AXIPCG_EBREAKDOWN: return "iteration breakdown (non-positive or non-finite scalar)";
    default: return "unknown status";
    }
}

const char *axipcg_last_error(void) { return last_error_cstr(); }

}  // extern "C"
