// Preconditioner B^{-1} of §4.2 (eqs. (36)-(39)) on gfx950: the launches of
// the z-transforms (one wave per row, or block-wide) and of the partitioned
// r-tridiagonal solver, for one operator and for a batch, with their plans
// (rows per workgroup, LDS, twiddle placement).  The device bodies are in
// xform.h and wxform.h.
#include "xform.h"

namespace axipcg {

namespace {

// (512 threads for N = 4096, 256 or fewer below)
template <typename T, int BC, bool FUSED, bool TWLDS, int ROWS>
__global__ void __launch_bounds__(512)
k_zfwd(const double *__restrict__ rin, double *__restrict__ x, double *__restrict__ r,
       const double *__restrict__ p, const double *__restrict__ q, PcgState *st,
       double *__restrict__ partials, int n_pq,
       T *__restrict__ spec, const typename vec2_of<T>::type *__restrict__ tw,
       const typename vec2_of<T>::type *__restrict__ pt, int nr, int N)
{
    zfwd_body<T, BC, FUSED, TWLDS, ROWS>(rin, x, r, p, q, st, partials, n_pq, spec, tw, pt, nr, N, blockIdx.x);
}

template <typename T, int BC, int MODE, bool TWLDS, int ROWS>
__global__ void __launch_bounds__(512)
k_zinv(const T *__restrict__ spec, double *__restrict__ zout, const double *__restrict__ r,
       const PcgState *st, double *__restrict__ partials, bool pr,
       const typename vec2_of<T>::type *__restrict__ tw,
       const typename vec2_of<T>::type *__restrict__ pt, int nr, int N, double *__restrict__ dinc, double tau,
       double rho2)
{
    zinv_body<T, BC, MODE, TWLDS, ROWS>(spec, zout, r, st, partials, pr, tw, pt, nr, N, blockIdx.x, dinc, tau, rho2);
}

template <typename T, int BC, bool FUSED, int R2>
__global__ void __launch_bounds__(256)
k_zfwd_w(const double *__restrict__ rin, double *__restrict__ x, double *__restrict__ r,
         const double *__restrict__ p, const double *__restrict__ q, PcgState *st,
         double *__restrict__ partials, int n_pq, T *__restrict__ spec,
         const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
         int nr)
{
    constexpr int WR = wave_rows<T, R2>();
    const int row = blockIdx.x * WR + (threadIdx.x >> 6);
    RowStore<T> out{spec + (size_t)(row < nr ? row : 0) * wfft::Geo<R2>::N};
    zfwd_w_body<T, BC, FUSED, R2>(rin, x, r, p, q, st, partials, n_pq, tw, pt, nr, row, blockIdx.x, out);
}

template <typename T, int BC, int MODE, int R2>
__global__ void __launch_bounds__(256)
k_zinv_w(const T *__restrict__ spec, double *__restrict__ zout, const double *__restrict__ r,
         const PcgState *st, double *__restrict__ partials, bool pr,
         const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
         int nr, double *__restrict__ dinc, double tau, double rho2)
{
    constexpr int WR = wave_rows<T, R2>();
    const int row = blockIdx.x * WR + (threadIdx.x >> 6);
    RowLoad<T> in{spec + (size_t)(row < nr ? row : nr - 1) * wfft::Geo<R2>::N};
    zinv_w_body<T, BC, MODE, R2>(in, zout, r, st, partials, pr, tw, pt, nr, dinc, tau, rho2, row, blockIdx.x);
}

// Threads of an r-solve workgroup (one wave per mode): up to eight FP32 modes
// on lines of 2048 rows and more (32-byte row pieces), else up to four.
template <typename T, int LMAX>
constexpr int tri_threads() { return (sizeof(T) == 4 && LMAX >= 32) ? 512 : 256; }

template <typename T, int LMAX, bool UNI>
__global__ void __launch_bounds__((tri_threads<T, LMAX>()))
k_tridiag(T *__restrict__ spec, const T *__restrict__ cb_g, const T *__restrict__ db_g,
          const T *__restrict__ rw_g, const T *__restrict__ lam, PcgState *st,
          const double *__restrict__ partials, TriGate g, int nr, int nz, int M, int S, int pitch, int Lp)
{
    tridiag_body<T, LMAX, UNI>(spec, cb_g, db_g, rw_g, lam, st, partials, g, nr, nz, M, S, pitch, Lp, blockIdx.x);
}

// ---- batched launches ----------------------------------------------------

// The batched transforms run one launch per transform plan; `d` holds the
// problems of that plan, with tr_start counted within the launch.  One work
// item (xform.h) per workgroup.
template <typename T, int KIND, bool TWLDS>
__global__ void __launch_bounds__(256) k_b_zfwd(const ProbDesc *__restrict__ d, int n, int parity)
{
    b_zfwd_item<T, KIND == BZ_PCG, TWLDS, false, KIND == BZ_CHEB>(d, n, blockIdx.x, parity);
}

template <typename T, int MODE, bool TWLDS>
__global__ void __launch_bounds__(256) k_b_zinv(const ProbDesc *__restrict__ d, int n, bool pr)
{
    b_zinv_item<T, MODE, TWLDS>(d, n, blockIdx.x, pr);
}

// Two waves per SIMD for the FP32 plans up to rows of 1024 points: the fused
// 1024-point forward needs 259 registers when left unbounded (one wave per
// SIMD) and fits 256 without spilling; the larger plans would spill.
template <typename T, int R2>
constexpr int bzw_waves() { return (sizeof(T) == 4 && R2 <= 8) ? 2 : 1; }

template <typename T, int KIND, int R2>
__global__ void __launch_bounds__(256, (bzw_waves<T, R2>())) k_b_zfwd_w(const ProbDesc *__restrict__ d, int n, int parity)
{
    b_zfwd_w_item<T, KIND == BZ_PCG, R2, false, KIND == BZ_CHEB>(d, n, blockIdx.x, parity);
}

template <typename T, int MODE, int R2>
__global__ void __launch_bounds__(256) k_b_zinv_w(const ProbDesc *__restrict__ d, int n, bool pr)
{
    b_zinv_w_item<T, MODE, R2>(d, n, blockIdx.x, pr);
}

template <typename T>
__global__ void __launch_bounds__(256) k_b_tridiag(const ProbDesc *__restrict__ d, int n, TriGate g, int M)
{
    b_tridiag_item<T>(d, n, g, M, blockIdx.x);
}

template <typename T>
struct Tables {
    const typename vec2_of<T>::type *tw, *pt;
    const T *cb, *db, *rw, *lam;
};
template <typename T> Tables<T> tables(const Operator &op);
template <> Tables<float> tables<float>(const Operator &op)
{
    return {op.tw32, op.pt32, op.cb32, op.db32, op.rw32, op.lam32};
}
template <> Tables<double> tables<double>(const Operator &op)
{
    return {op.tw64, op.pt64, op.cb64, op.db64, op.rw64, op.lam64};
}

// LDS of a transform workgroup: two data buffers, plus the twiddle table when
// the total stays within 64 KiB.
template <typename T>
bool twiddles_in_lds(int N) { return 3 * (size_t)N * sizeof(cx<T>) <= 65536; }
template <typename T>
size_t transform_lds(int N) { return (twiddles_in_lds<T>(N) ? 3 : 2) * (size_t)N * sizeof(cx<T>); }

// Rows per transform workgroup: two (pipelined) for the FP64 transforms, and
// for the FP32 ones of rows of 4096 points, when that still leaves at least
// 256 workgroups, else one.  (Measured at 1024^2: two rows take the FP64
// forward transform from 28 to 25 us but slow the FP32 ones, whose FFT is too
// short to hide a second row's loads behind while the grid loses half its
// workgroups; at 4096^2 the FP32 apply goes from 528 to 503 us with two.)
inline int transform_rows(int nr, int nz, int prec)
{
    return ((prec == AXIPCG_PREC_FP64 || nz >= 4096) && nr % 2 == 0 && nr >= 512) ? 2 : 1;
}

// Dynamic LDS above the default 64 KiB (FP64 rows of 4096) needs the
// kernel's attribute, set once per kernel.
inline void allow_transform_lds(const void *fn, size_t bytes, bool &done)
{
    if (done || bytes <= 65536) return;
    AXI_CHECK_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done = true;
}

template <typename T, int BC, bool TWL, int ROWS>
void zfwd_ttr(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    const int N = op.nz;
    const auto tb = tables<T>(op);
    const size_t shm = transform_lds<T>(N);
    const int thr = fft_threads(N);
    const dim3 grid(op.nr / ROWS);
    static bool lds_set[2] = {false, false};
    allow_transform_lds(reinterpret_cast<const void *>(&k_zfwd<T, BC, true, TWL, ROWS>), shm, lds_set[0]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zfwd<T, BC, false, TWL, ROWS>), shm, lds_set[1]);
    if (a.fused)
        hipLaunchKernelGGL((k_zfwd<T, BC, true, TWL, ROWS>), grid, dim3(thr), shm, s, nullptr, a.x, a.r, a.p, a.q,
                           a.state, op.partials, a.n_pq, (T *)op.spec, tb.tw, tb.pt, op.nr, N);
    else
        hipLaunchKernelGGL((k_zfwd<T, BC, false, TWL, ROWS>), grid, dim3(thr), shm, s, a.rin, nullptr, nullptr,
                           nullptr, nullptr, a.state, op.partials, 0, (T *)op.spec, tb.tw, tb.pt, op.nr, N);
    AXI_CHECK_HIP(hipGetLastError());
}

// Rows per workgroup of the one-wave transforms for length N, 0 when N has
// no one-wave plan (then the block-wide Stockham kernels run).
template <typename T>
int wave_plan_rows(int N)
{
    switch (N) {
    case 256: return wave_rows<T, 2>();
    case 512: return wave_rows<T, 4>();
    case 1024: return wave_rows<T, 8>();
    case 2048: return sizeof(T) == 4 ? wave_rows<T, 16>() : 0;   // FP64 at 2048 would spill
    default: return 0;
    }
}

template <typename T, int BC, int R2>
void zfwd_wave(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    constexpr int WR = wave_rows<T, R2>();
    const auto tb = tables<T>(op);
    const dim3 grid((op.nr + WR - 1) / WR), block(64 * WR);
    const size_t shm = (size_t)WR * wfft::Geo<R2>::LB * sizeof(cx<T>);
    if (a.fused)
        hipLaunchKernelGGL((k_zfwd_w<T, BC, true, R2>), grid, block, shm, s, nullptr, a.x, a.r, a.p, a.q, a.state,
                           op.partials, a.n_pq, (T *)op.spec, tb.tw, tb.pt, op.nr);
    else
        hipLaunchKernelGGL((k_zfwd_w<T, BC, false, R2>), grid, block, shm, s, a.rin, nullptr, nullptr, nullptr,
                           nullptr, a.state, op.partials, 0, (T *)op.spec, tb.tw, tb.pt, op.nr);
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int BC>
void zfwd_t(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    switch (op.nz) {
    case 256: return zfwd_wave<T, BC, 2>(op, a, s);
    case 512: return zfwd_wave<T, BC, 4>(op, a, s);
    case 1024: return zfwd_wave<T, BC, 8>(op, a, s);
    case 2048:
        if constexpr (sizeof(T) == 4) return zfwd_wave<T, BC, 16>(op, a, s);
        break;
    default: break;
    }
    const bool twl = twiddles_in_lds<T>(op.nz);
    if (transform_rows(op.nr, op.nz, sizeof(T) == 8 ? AXIPCG_PREC_FP64 : AXIPCG_PREC_FP32) == 2) {
        if (twl) zfwd_ttr<T, BC, true, 2>(op, a, s);
        else zfwd_ttr<T, BC, false, 2>(op, a, s);
    } else {
        if (twl) zfwd_ttr<T, BC, true, 1>(op, a, s);
        else zfwd_ttr<T, BC, false, 1>(op, a, s);
    }
}

template <typename T, int BC, bool TWL, int ROWS>
void zinv_ttr(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    const int N = op.nz;
    const auto tb = tables<T>(op);
    const size_t shm = transform_lds<T>(N);
    const int thr = fft_threads(N);
    const dim3 grid(op.nr / ROWS);
    static bool lds_set[5] = {false, false, false, false, false};
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 0, TWL, ROWS>), shm, lds_set[0]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 1, TWL, ROWS>), shm, lds_set[1]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 2, TWL, ROWS>), shm, lds_set[2]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 3, TWL, ROWS>), shm, lds_set[3]);
    allow_transform_lds(reinterpret_cast<const void *>(&k_zinv<T, BC, 4, TWL, ROWS>), shm, lds_set[4]);
    switch (a.mode) {
    case 0:
        hipLaunchKernelGGL((k_zinv<T, BC, 0, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, a.zout,
                           nullptr, nullptr, op.partials, false, tb.tw, tb.pt, op.nr, N, nullptr, 0.0, 0.0);
        break;
    case 1:
        hipLaunchKernelGGL((k_zinv<T, BC, 1, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, a.zout,
                           a.r, a.state, op.partials, a.pr, tb.tw, tb.pt, op.nr, N, nullptr, 0.0, 0.0);
        break;
    case 2:
        hipLaunchKernelGGL((k_zinv<T, BC, 2, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, a.zout,
                           a.r, a.state, op.partials, false, tb.tw, tb.pt, op.nr, N, nullptr, 0.0, 0.0);
        break;
    case 3:
        hipLaunchKernelGGL((k_zinv<T, BC, 3, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, nullptr,
                           nullptr, a.state, op.partials, false, tb.tw, tb.pt, op.nr, N, a.d, a.tau, a.rho2);
        break;
    default:
        hipLaunchKernelGGL((k_zinv<T, BC, 4, TWL, ROWS>), grid, dim3(thr), shm, s, (const T *)op.spec, nullptr,
                           nullptr, a.state, op.partials, false, tb.tw, tb.pt, op.nr, N, a.d, a.tau, a.rho2);
        break;
    }
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int BC, int R2>
void zinv_wave(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    constexpr int WR = wave_rows<T, R2>();
    const auto tb = tables<T>(op);
    const dim3 grid((op.nr + WR - 1) / WR), block(64 * WR);
    const size_t shm = (size_t)WR * wfft::Geo<R2>::LB * sizeof(cx<T>);
    const T *spec = (const T *)op.spec;
    switch (a.mode) {
    case 0:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 0, R2>), grid, block, shm, s, spec, a.zout, nullptr, nullptr,
                           op.partials, false, tb.tw, tb.pt, op.nr, nullptr, 0.0, 0.0);
        break;
    case 1:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 1, R2>), grid, block, shm, s, spec, a.zout, a.r, a.state, op.partials,
                           a.pr, tb.tw, tb.pt, op.nr, nullptr, 0.0, 0.0);
        break;
    case 2:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 2, R2>), grid, block, shm, s, spec, a.zout, a.r, a.state, op.partials,
                           false, tb.tw, tb.pt, op.nr, nullptr, 0.0, 0.0);
        break;
    case 3:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 3, R2>), grid, block, shm, s, spec, nullptr, nullptr, a.state,
                           op.partials, false, tb.tw, tb.pt, op.nr, a.d, a.tau, a.rho2);
        break;
    default:
        hipLaunchKernelGGL((k_zinv_w<T, BC, 4, R2>), grid, block, shm, s, spec, nullptr, nullptr, a.state,
                           op.partials, false, tb.tw, tb.pt, op.nr, a.d, a.tau, a.rho2);
        break;
    }
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int BC>
void zinv_t(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    switch (op.nz) {
    case 256: return zinv_wave<T, BC, 2>(op, a, s);
    case 512: return zinv_wave<T, BC, 4>(op, a, s);
    case 1024: return zinv_wave<T, BC, 8>(op, a, s);
    case 2048:
        if constexpr (sizeof(T) == 4) return zinv_wave<T, BC, 16>(op, a, s);
        break;
    default: break;
    }
    const bool twl = twiddles_in_lds<T>(op.nz);
    if (transform_rows(op.nr, op.nz, sizeof(T) == 8 ? AXIPCG_PREC_FP64 : AXIPCG_PREC_FP32) == 2) {
        if (twl) zinv_ttr<T, BC, true, 2>(op, a, s);
        else zinv_ttr<T, BC, false, 2>(op, a, s);
    } else {
        if (twl) zinv_ttr<T, BC, true, 1>(op, a, s);
        else zinv_ttr<T, BC, false, 1>(op, a, s);
    }
}

// LDS of an r-solve workgroup (its [M][N_r] tile, padded): up to 136 KiB, so
// that lines of 4096 rows keep eight FP32 or four FP64 modes per workgroup,
// 32 bytes of each row (the kernels' attribute raised on first use).
constexpr size_t TRI_LDS_MAX = 136 * 1024;

struct TriGeom {
    int M, S, L, Lp, pitch;
    size_t shm;
};

template <typename T>
TriGeom tri_geom(int nr, int nz)
{
    TriGeom g;
    g.S = nr / 2 < 64 ? nr / 2 : 64;
    g.L = (nr + g.S - 1) / g.S;
    g.Lp = nr / g.S;
    g.pitch = nr + nr / g.Lp + 1;
    // one 16-byte vector of modes per row; two on lines of 2048 rows and more,
    // whose tiles written back 16 bytes per row left partly written lines
    // (1.35x the FP32 tile's bytes at 4096 rows, 1.7x in FP64)
    g.M = (g.L >= 32 ? 32 : 16) / (int)sizeof(T);
    auto lds = [&](int M) { return (size_t)M * g.pitch * sizeof(T); };
    while (g.M > 1 && (lds(g.M) > TRI_LDS_MAX || nz % g.M != 0)) g.M >>= 1;
    g.shm = lds(g.M);
    return g;
}

template <typename T>
void tridiag_t(const Operator &op, const TriGate &gate, hipStream_t s)
{
    const TriGeom g = tri_geom<T>(op.nr, op.nz);
    const auto tb = tables<T>(op);
    const dim3 grid(op.nz / g.M), block(64 * g.M);
    T *spec = (T *)op.spec;
#define AXI_TRI(LM, U)                                                                                   \
    do {                                                                                                 \
        static bool lds_set = false;                                                                     \
        if (g.shm > 65536 && !lds_set) {                                                                 \
            AXI_CHECK_HIP(hipFuncSetAttribute((const void *)k_tridiag<T, LM, U>,                          \
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)TRI_LDS_MAX)); \
            lds_set = true;                                                                              \
        }                                                                                                \
        hipLaunchKernelGGL((k_tridiag<T, LM, U>), grid, block, g.shm, s, spec, tb.cb, tb.db, tb.rw, tb.lam, \
                           gate.state, op.partials, gate, op.nr, op.nz, g.M, g.S, g.pitch, g.Lp);          \
    } while (0)
    const bool uni = (op.nr % g.S) == 0;
    if (uni && g.L == 2) AXI_TRI(2, true);
    else if (uni && g.L == 4) AXI_TRI(4, true);
    else if (uni && g.L == 8) AXI_TRI(8, true);
    else if (uni && g.L == 16) AXI_TRI(16, true);
    else if (uni && g.L == 32) AXI_TRI(32, true);
    else if (uni && g.L == 64) AXI_TRI(64, true);
    else if (g.L <= 4) AXI_TRI(4, false);
    else if (g.L <= 8) AXI_TRI(8, false);
    else if (g.L <= 16) AXI_TRI(16, false);
    else if (g.L <= 32) AXI_TRI(32, false);
    else if (g.L <= 64) AXI_TRI(64, false);
    else throw Error{AXIPCG_EINVAL, "nr too large for the r-solver"};
#undef AXI_TRI
    AXI_CHECK_HIP(hipGetLastError());
}

}  // namespace

// Strip height of the solves' launches: the handle's, except that 8-row
// strips at FP32 rows of 2048 (whose PCG-form kernels would spill registers
// in 8-wave workgroups) run as 4-row strips.
int strip_solve_rows(const Operator &op, int prec)
{
    return (op.strip_rows == 8 && prec == AXIPCG_PREC_FP32 && op.nz == 2048) ? 4 : op.strip_rows;
}

int transform_blocks(const Operator &op, int prec)
{
    if (strip_usable(op, prec, strip_solve_rows(op, prec))) return op.nr / strip_solve_rows(op, prec);
    const int wr = (prec == AXIPCG_PREC_FP32) ? wave_plan_rows<float>(op.nz) : wave_plan_rows<double>(op.nz);
    if (wr > 0) return (op.nr + wr - 1) / wr;
    return op.nr / transform_rows(op.nr, op.nz, prec);
}

// ---- batched launchers -------------------------------------------------------
void batch_tri_geom(int nr, int prec, int M, int *S, int *L, int *Lp, int *pitch, size_t *shm)
{
    *S = nr / 2 < 64 ? nr / 2 : 64;
    *L = (nr + *S - 1) / *S;
    *Lp = nr / *S;
    *pitch = nr + nr / *Lp + 1;
    const size_t el = (prec == AXIPCG_PREC_FP32) ? sizeof(float) : sizeof(double);
    *shm = (size_t)M * *pitch * el;
}

template <typename T>
size_t plan_lds_t(const BatchPlan &pl, bool *twl)
{
    *twl = false;
    switch (pl.r2) {
    case 2: return (size_t)wave_rows<T, 2>() * wfft::Geo<2>::LB * sizeof(cx<T>);
    case 4: return (size_t)wave_rows<T, 4>() * wfft::Geo<4>::LB * sizeof(cx<T>);
    case 8: return (size_t)wave_rows<T, 8>() * wfft::Geo<8>::LB * sizeof(cx<T>);
    case 16: return (size_t)wave_rows<T, 16>() * wfft::Geo<16>::LB * sizeof(cx<T>);
    default:
        *twl = twiddles_in_lds<T>(pl.nz_max);
        return transform_lds<T>(pl.nz_max);
    }
}

size_t batch_plan_lds(const BatchPlan &pl, int prec, bool *twl)
{
    return prec == AXIPCG_PREC_FP32 ? plan_lds_t<float>(pl, twl) : plan_lds_t<double>(pl, twl);
}

int batch_transform_plan(int nz, int prec, int *rows_per_wg)
{
    const int wr = (prec == AXIPCG_PREC_FP32) ? wave_plan_rows<float>(nz) : wave_plan_rows<double>(nz);
    *rows_per_wg = wr > 0 ? wr : 1;
    return wr > 0 ? nz / 128 : 0;
}

template <typename T, int R2>
void b_zfwd_wave(const ProbDesc *d, const BatchPlan &pl, int kind, int parity, hipStream_t s)
{
    constexpr int WR = wave_rows<T, R2>();
    const size_t shm = (size_t)WR * wfft::Geo<R2>::LB * sizeof(cx<T>);
#define AXI_BZW(K) hipLaunchKernelGGL((k_b_zfwd_w<T, K, R2>), dim3(pl.blocks), dim3(64 * WR), shm, s, d + pl.off, pl.n, parity)
    if (kind == BZ_PCG) AXI_BZW(BZ_PCG);
    else if (kind == BZ_CHEB) AXI_BZW(BZ_CHEB);
    else AXI_BZW(BZ_START);
#undef AXI_BZW
}

template <typename T, int R2>
void b_zinv_wave(const ProbDesc *d, const BatchPlan &pl, int mode, bool pr, hipStream_t s)
{
    constexpr int WR = wave_rows<T, R2>();
    const size_t shm = (size_t)WR * wfft::Geo<R2>::LB * sizeof(cx<T>);
#define AXI_BIW(MD) hipLaunchKernelGGL((k_b_zinv_w<T, MD, R2>), dim3(pl.blocks), dim3(64 * WR), shm, s, d + pl.off, pl.n, pr)
    switch (mode) {
    case 1: AXI_BIW(1); break;
    case 2: AXI_BIW(2); break;
    case 3: AXI_BIW(3); break;
    default: AXI_BIW(4);
    }
#undef AXI_BIW
}

template <typename T>
void b_zfwd_t(const ProbDesc *d, const BatchPlan &pl, int kind, int parity, hipStream_t s)
{
    switch (pl.r2) {
    case 2: b_zfwd_wave<T, 2>(d, pl, kind, parity, s); break;
    case 4: b_zfwd_wave<T, 4>(d, pl, kind, parity, s); break;
    case 8: b_zfwd_wave<T, 8>(d, pl, kind, parity, s); break;
    case 16:
        if constexpr (sizeof(T) == 4) b_zfwd_wave<T, 16>(d, pl, kind, parity, s);
        else AXI_REQUIRE(false, "no one-wave FP64 plan for N = 2048");
        break;
    default: {
        const size_t shm = transform_lds<T>(pl.nz_max);
        const dim3 grid(pl.blocks), block(256);
        const ProbDesc *dp = d + pl.off;
#define AXI_BZF(K, TW) hipLaunchKernelGGL((k_b_zfwd<T, K, TW>), grid, block, shm, s, dp, pl.n, parity)
        if (twiddles_in_lds<T>(pl.nz_max)) {
            if (kind == BZ_PCG) AXI_BZF(BZ_PCG, true);
            else if (kind == BZ_CHEB) AXI_BZF(BZ_CHEB, true);
            else AXI_BZF(BZ_START, true);
        } else {
            if (kind == BZ_PCG) AXI_BZF(BZ_PCG, false);
            else if (kind == BZ_CHEB) AXI_BZF(BZ_CHEB, false);
            else AXI_BZF(BZ_START, false);
        }
#undef AXI_BZF
    }
    }
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T>
void b_zinv_t(const ProbDesc *d, const BatchPlan &pl, int mode, bool pr, hipStream_t s)
{
    switch (pl.r2) {
    case 2: b_zinv_wave<T, 2>(d, pl, mode, pr, s); break;
    case 4: b_zinv_wave<T, 4>(d, pl, mode, pr, s); break;
    case 8: b_zinv_wave<T, 8>(d, pl, mode, pr, s); break;
    case 16:
        if constexpr (sizeof(T) == 4) b_zinv_wave<T, 16>(d, pl, mode, pr, s);
        else AXI_REQUIRE(false, "no one-wave FP64 plan for N = 2048");
        break;
    default: {
        const size_t shm = transform_lds<T>(pl.nz_max);
        const bool twl = twiddles_in_lds<T>(pl.nz_max);
        const dim3 grid(pl.blocks), block(256);
        const ProbDesc *dp = d + pl.off;
#define AXI_BZI(MD, TW) hipLaunchKernelGGL((k_b_zinv<T, MD, TW>), grid, block, shm, s, dp, pl.n, pr)
#define AXI_BZI2(MD) do { if (twl) AXI_BZI(MD, true); else AXI_BZI(MD, false); } while (0)
        switch (mode) {
        case 1: AXI_BZI2(1); break;
        case 2: AXI_BZI2(2); break;
        case 3: AXI_BZI2(3); break;
        default: AXI_BZI2(4);
        }
#undef AXI_BZI2
#undef AXI_BZI
    }
    }
    AXI_CHECK_HIP(hipGetLastError());
}

void launch_b_zfwd(const ProbDesc *d, const BatchPlan &pl, int prec, int kind, int parity, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) b_zfwd_t<float>(d, pl, kind, parity, s);
    else b_zfwd_t<double>(d, pl, kind, parity, s);
}

void launch_b_zinv(const ProbDesc *d, const BatchPlan &pl, int prec, int mode, bool pr, hipStream_t s)
{
    AXI_REQUIRE(mode >= 1 && mode <= 4, "batched inverse transform mode must be 1..4");
    if (prec == AXIPCG_PREC_FP32) b_zinv_t<float>(d, pl, mode, pr, s);
    else b_zinv_t<double>(d, pl, mode, pr, s);
}

void launch_b_tridiag(const ProbDesc *d, int n, int blocks, int prec, const TriGate &g, int M, size_t shm,
                      hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32)
        hipLaunchKernelGGL(k_b_tridiag<float>, dim3(blocks), dim3(64 * M), shm, s, d, n, g, M);
    else
        hipLaunchKernelGGL(k_b_tridiag<double>, dim3(blocks), dim3(64 * M), shm, s, d, n, g, M);
    AXI_CHECK_HIP(hipGetLastError());
}

void launch_zfwd(const Operator &op, int prec, const ZfwdArgs &a, hipStream_t s)
{
    if (strip_usable(op, prec, strip_solve_rows(op, prec))) return strip_fwd(op, prec, strip_solve_rows(op, prec), a, s);
    if (prec == AXIPCG_PREC_FP32) {
        if (op.bc_z == DIR) zfwd_t<float, DIR>(op, a, s);
        else zfwd_t<float, AXIPCG_Z_NEUMANN>(op, a, s);
    } else {
        if (op.bc_z == DIR) zfwd_t<double, DIR>(op, a, s);
        else zfwd_t<double, AXIPCG_Z_NEUMANN>(op, a, s);
    }
}

void launch_zinv(const Operator &op, int prec, const ZinvArgs &a, hipStream_t s)
{
    if (strip_usable(op, prec, strip_solve_rows(op, prec))) return strip_inv(op, prec, strip_solve_rows(op, prec), a, s);
    if (prec == AXIPCG_PREC_FP32) {
        if (op.bc_z == DIR) zinv_t<float, DIR>(op, a, s);
        else zinv_t<float, AXIPCG_Z_NEUMANN>(op, a, s);
    } else {
        if (op.bc_z == DIR) zinv_t<double, DIR>(op, a, s);
        else zinv_t<double, AXIPCG_Z_NEUMANN>(op, a, s);
    }
}

void launch_tridiag(const Operator &op, int prec, const TriGate &g, hipStream_t s)
{
    if (strip_usable(op, prec, strip_solve_rows(op, prec)))
        return strip_reduced(op, prec, strip_solve_rows(op, prec), g, s);
    if (prec == AXIPCG_PREC_FP32) tridiag_t<float>(op, g, s);
    else tridiag_t<double>(op, g, s);
}

// Standalone applies of FP32 rows of length 2048 use strips of 8 rows when
// strips are on (their transform kernels fit the registers of 8-wave
// workgroups without the PCG vectors, and the reduced system halves); the
// solves keep strip_solve_rows.
void precond_apply_impl(const Operator &op, const double *r, double *z, int prec, hipStream_t s)
{
    int rows = strip_solve_rows(op, prec);
    if (rows == 4 && prec == AXIPCG_PREC_FP32 && op.nz == 2048 && strip_usable(op, prec, 8)) rows = 8;
    if (rows > 0 && strip_usable(op, prec, rows)) {
        ZfwdArgs fa;
        fa.rin = r;
        strip_fwd(op, prec, rows, fa, s);
        strip_reduced(op, prec, rows, TriGate{}, s);
        ZinvArgs ia;
        ia.zout = z;
        strip_inv(op, prec, rows, ia, s);
        return;
    }
    ZfwdArgs fa;
    fa.rin = r;
    launch_zfwd(op, prec, fa, s);
    launch_tridiag(op, prec, TriGate{}, s);
    ZinvArgs ia;
    ia.zout = z;
    launch_zinv(op, prec, ia, s);
}

}  // namespace axipcg
