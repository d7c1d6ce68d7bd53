// Strip-partitioned preconditioner z = B^{-1} r (§4.2 eqs. (36)-(39)) with
// the partition idea of §3: the grid is cut into strips of R consecutive
// r-rows, one workgroup each, the interior of every strip is eliminated in
// terms of the strips' boundary rows (the "preparatory" solutions of
// eqs. (18)-(22)), and only one reduced equation per strip and z-mode crosses
// workgroups.  Three launches:
//
//  K1 (forward + local elimination): each wave z-transforms one row of the
//     strip into the workgroup's LDS tile; then, per mode, the strip's
//     interior rows are swept forward (Thomas) and the forward-eliminated
//     data f' is written back row by row, together with two values per
//     (strip, mode) that the reduced equations need (E1, G0 below).
//  K2 (reduced systems): per mode, the tridiagonal system in the strips'
//     last rows X_s (G = nr / R unknowns), solved by one wavefront (segments
//     per lane, parallel cyclic reduction across lanes).  In PCG mode it
//     first runs the stop test.
//  K3 (back substitution + inverse): each strip rebuilds its interior rows
//     from f', X_{s-1} and X_s in the LDS tile, and each wave inverse-
//     transforms one row to z.
//
// Every global access is along z (whole rows), so no kernel gathers or
// scatters the strided [nr][modes] tiles a per-mode r-solve needs; the
// spectral data crosses HBM once each way as f' (4 + 4 bytes per point in
// FP32), and the reduced data is 3 values per strip and mode.
//
// Notation for strip s (rows i0 = s R + t, t < R; n = R - 1 interior rows,
// interface row j = i0 + n), mode l with lam = kbar mu_l + qbar:
//   row equation  -cb[i-1] y[i-1] + (db[i] + rw[i] lam) y[i] - cb[i] y[i+1] = f[i];
//   interior sweep  den_t = D_t - L_t c'_{t-1},  c'_t = cb[i0+t] / den_t,
//                   f'_t = (f_t + L_t f'_{t-1}) / den_t,
//                   v'_t = (t = 0 ? cb[i0-1] : L_t v'_{t-1}) / den_t,
//     with L_t = cb[i0+t-1] (t >= 1), so that
//                   y_t = f'_t + v'_t X_{s-1} + c'_t y_{t+1},  y_n = X_s;
//   back to the first interior row: y_0 = G0 + v_0 X_{s-1} + w_0 X_s and
//   y_{n-1} = f'_{n-1} + v'_{n-1} X_{s-1} + c'_{n-1} X_s;
//   reduced equation of strip s (the interface row with both neighbours
//   eliminated):
//     a_s = -cb[j-1] v'_{n-1},  b_s = D_j - cb[j-1] c'_{n-1} - cb[j] v_0(s+1),
//     c_s = -cb[j] w_0(s+1),    e_s = E1_s + cb[j] G0_{s+1},
//     E1_s = f_j + cb[j-1] f'_{n-1}.
// The coefficient-only quantities (c', v', v_0, w_0) are recomputed where
// needed from the O(nr) r-line arrays instead of being stored.
#include "strip.h"

namespace axipcg {
namespace {

template <typename T, int BC, bool FUSED, int R2, int R>
__global__ void __launch_bounds__(64 * R)
k_strip_fwd(const double *__restrict__ rin, double *__restrict__ x, double *__restrict__ r,
            const double *__restrict__ p, const double *__restrict__ q, PcgState *st, double *__restrict__ partials,
            int n_pq, T *__restrict__ fprime, T *__restrict__ red_e, T *__restrict__ red_g,
            const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
            Lines<T> ln, int nr)
{
    extern __shared__ char smem_raw[];
    strip_phase1<T, BC, FUSED, R2, R>(rin, x, r, p, q, st, partials, n_pq, fprime, red_e, red_g, tw, pt, ln, nr,
                                      blockIdx.x, reinterpret_cast<T *>(smem_raw));
}

// MT modes per workgroup (one wave each)
template <typename T, int R, int LMAX, int MT>
__global__ void __launch_bounds__(64 * MT)
k_strip_reduced(const T *__restrict__ red_e, const T *__restrict__ red_g, T *__restrict__ red_x, Lines<T> ln,
                PcgState *st, const double *__restrict__ partials, TriGate g, int nr, int N, int G)
{
    __shared__ double red[RED_SLOTS];
    extern __shared__ char smem_raw[];
    T *base = reinterpret_cast<T *>(smem_raw);
    const int l0 = xcd_swizzle(blockIdx.x, N / MT) * MT;
    constexpr bool VEC = MT % (16 / (int)sizeof(T)) == 0;   // 16-byte staging loads
    GatePre pre;
    if (g.mode == 1) gate_issue(st, partials, g, pre);
    strip_stage2<T, VEC>(red_e, red_g, ln, nr, N, G, l0, MT, base);
    if (g.mode != 0 && tridiag_gate(st, partials, g, red, blockIdx.x, g.mode == 1 ? &pre : nullptr) != ST_RUN)
        return;
    __syncthreads();
    strip_solve2<T, R, LMAX, VEC>(red_x, ln, nr, N, G, l0, MT, base);
}

template <typename T, int BC, int MODE, int R2, int R>
__global__ void __launch_bounds__(64 * R)
k_strip_inv(const T *__restrict__ fprime, const T *__restrict__ red_x, double *__restrict__ zout,
            const double *__restrict__ r, const PcgState *st, double *__restrict__ partials, bool pr,
            const typename vec2_of<T>::type *__restrict__ tw, const typename vec2_of<T>::type *__restrict__ pt,
            Lines<T> ln, int nr, double *__restrict__ dinc, double tau, double rho2)
{
    extern __shared__ char smem_raw[];
    strip_phase3<T, BC, MODE, R2, R>(fprime, red_x, zout, r, st, partials, pr, tw, pt, ln, nr, dinc, tau, rho2,
                                     blockIdx.x, reinterpret_cast<T *>(smem_raw));
}

template <typename T>
Lines<T> lines_of(const Operator &op);
template <>
Lines<float> lines_of<float>(const Operator &op) { return {op.cb32, op.db32, op.rw32, op.lam32}; }
template <>
Lines<double> lines_of<double>(const Operator &op) { return {op.cb64, op.db64, op.rw64, op.lam64}; }

template <typename T>
const typename vec2_of<T>::type *tw_of(const Operator &op);
template <>
const float2 *tw_of<float>(const Operator &op) { return op.tw32; }
template <>
const double2 *tw_of<double>(const Operator &op) { return op.tw64; }
template <typename T>
const typename vec2_of<T>::type *pt_of(const Operator &op);
template <>
const float2 *pt_of<float>(const Operator &op) { return op.pt32; }
template <>
const double2 *pt_of<double>(const Operator &op) { return op.pt64; }

template <typename T>
struct RedBufs {
    T *e, *g, *x;
};
template <typename T>
RedBufs<T> red_bufs(const Operator &op, int R)
{
    T *b = static_cast<T *>(op.strip_red);
    const size_t gn = (size_t)(op.nr / R) * op.nz;
    return {b, b + gn, b + 2 * gn};
}

// modes per reduced-system workgroup: 32 bytes of each strip's row
template <typename T>
constexpr int red_mt() { return 32 / (int)sizeof(T); }
// Modes per workgroup for nr rows in G strips: red_mt, halved (down to 2)
// only while the LDS stage would not fit (FP64 with 1024 strips).  Fewer
// modes per workgroup than red_mt made PCG iterations slower at 1024^2.
template <typename T>
int red_mt_for(int nr, int G)
{
    int mt = red_mt<T>();
    while (mt > 2 && strip_red_lds<T>(nr, G, mt) > 160 * 1024) mt /= 2;
    return mt;
}

// Dynamic LDS above the default 64 KiB needs the kernel's attribute, set
// once per kernel.
void allow_lds(const void *fn, size_t bytes, bool &done)
{
    if (done || bytes <= 65536) return;
    AXI_CHECK_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done = true;
}

template <typename T, int BC, int R2, int R>
void fwd_r(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    const RedBufs<T> rb = red_bufs<T>(op, R);
    const dim3 grid(op.nr / R), block(64 * R);
    const size_t shm = (size_t)R * wfft::Geo<R2>::LB * sizeof(cx<T>);
    if (a.fused)
        hipLaunchKernelGGL((k_strip_fwd<T, BC, true, R2, R>), grid, block, shm, s, nullptr, a.x, a.r, a.p, a.q,
                           a.state, op.partials, a.n_pq, (T *)op.spec, rb.e, rb.g, tw_of<T>(op), pt_of<T>(op),
                           lines_of<T>(op), op.nr);
    else
        hipLaunchKernelGGL((k_strip_fwd<T, BC, false, R2, R>), grid, block, shm, s, a.rin, nullptr, nullptr,
                           nullptr, nullptr, a.state, op.partials, 0, (T *)op.spec, rb.e, rb.g, tw_of<T>(op),
                           pt_of<T>(op), lines_of<T>(op), op.nr);
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int BC, int R2, int R>
void inv_r(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    const RedBufs<T> rb = red_bufs<T>(op, R);
    const dim3 grid(op.nr / R), block(64 * R);
    const size_t shm = (size_t)R * wfft::Geo<R2>::LB * sizeof(cx<T>);
    const T *fp = (const T *)op.spec;
    const auto tw = tw_of<T>(op);
    const auto pt = pt_of<T>(op);
    const Lines<T> ln = lines_of<T>(op);
#define AXI_SINV(MD, Z, RR, ST, PR, D)                                                                           \
    hipLaunchKernelGGL((k_strip_inv<T, BC, MD, R2, R>), grid, block, shm, s, fp, rb.x, Z, RR, ST, op.partials,  \
                       PR, tw, pt, ln, op.nr, D, a.tau, a.rho2)
    switch (a.mode) {
    case 0: AXI_SINV(0, a.zout, nullptr, nullptr, false, nullptr); break;
    case 1: AXI_SINV(1, a.zout, a.r, a.state, a.pr, nullptr); break;
    case 2: AXI_SINV(2, a.zout, a.r, a.state, false, nullptr); break;
    case 3: AXI_SINV(3, nullptr, nullptr, a.state, false, a.d); break;
    default: AXI_SINV(4, nullptr, nullptr, a.state, false, a.d); break;
    }
#undef AXI_SINV
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int R, int LM, int MT>
void red_launch_mt(const Operator &op, const TriGate &g, hipStream_t s)
{
    const RedBufs<T> rb = red_bufs<T>(op, R);
    const int G = op.nr / R;
    const size_t shm = strip_red_lds<T>(op.nr, G, MT);
    static bool lds_set = false;
    allow_lds(reinterpret_cast<const void *>(&k_strip_reduced<T, R, LM, MT>), shm, lds_set);
    hipLaunchKernelGGL((k_strip_reduced<T, R, LM, MT>), dim3(op.nz / MT), dim3(64 * MT), shm, s, rb.e, rb.g, rb.x,
                       lines_of<T>(op), g.state, op.partials, g, op.nr, op.nz, G);
    AXI_CHECK_HIP(hipGetLastError());
}

template <typename T, int R, int LM>
void red_launch(const Operator &op, const TriGate &g, hipStream_t s)
{
    const int mt = red_mt_for<T>(op.nr, op.nr / R);
    if (mt >= 8) red_launch_mt<T, R, LM, (red_mt<T>() >= 8 ? 8 : 2)>(op, g, s);
    else if (mt >= 4) red_launch_mt<T, R, LM, 4>(op, g, s);
    else red_launch_mt<T, R, LM, 2>(op, g, s);
}

template <typename T, int R>
void red_r(const Operator &op, const TriGate &g, hipStream_t s)
{
    const int per = (op.nr / R + 63) / 64;
    if (per <= 1) red_launch<T, R, 1>(op, g, s);
    else if (per <= 2) red_launch<T, R, 2>(op, g, s);
    else if (per <= 4) red_launch<T, R, 4>(op, g, s);
    else if (per <= 8) red_launch<T, R, 8>(op, g, s);
    else red_launch<T, R, 16>(op, g, s);
}

template <typename T>
int strip_r2(int nz)
{
    switch (nz) {
    case 256: return 2;
    case 512: return 4;
    case 1024: return 8;
    case 2048: return sizeof(T) == 4 ? 16 : 0;   // FP64 at 2048 would spill
    default: return 0;
    }
}

template <typename T, int BC, int R>
void fwd_rb(const Operator &op, const ZfwdArgs &a, hipStream_t s)
{
    switch (op.nz) {
    case 256: fwd_r<T, BC, 2, R>(op, a, s); break;
    case 512: fwd_r<T, BC, 4, R>(op, a, s); break;
    case 1024: fwd_r<T, BC, 8, R>(op, a, s); break;
    default:
        if constexpr (sizeof(T) == 4) fwd_r<T, BC, 16, R>(op, a, s);
        break;
    }
}

template <typename T, int BC, int R>
void inv_rb(const Operator &op, const ZinvArgs &a, hipStream_t s)
{
    switch (op.nz) {
    case 256: inv_r<T, BC, 2, R>(op, a, s); break;
    case 512: inv_r<T, BC, 4, R>(op, a, s); break;
    case 1024: inv_r<T, BC, 8, R>(op, a, s); break;
    default:
        if constexpr (sizeof(T) == 4) inv_r<T, BC, 16, R>(op, a, s);
        break;
    }
}

template <typename T>
void fwd_t(const Operator &op, int rows, const ZfwdArgs &a, hipStream_t s)
{
    const bool dir = op.bc_z == DIR;
    if (rows == 8) {
        if (dir) fwd_rb<T, DIR, 8>(op, a, s);
        else fwd_rb<T, AXIPCG_Z_NEUMANN, 8>(op, a, s);
    } else {
        if (dir) fwd_rb<T, DIR, 4>(op, a, s);
        else fwd_rb<T, AXIPCG_Z_NEUMANN, 4>(op, a, s);
    }
}

template <typename T>
void inv_t(const Operator &op, int rows, const ZinvArgs &a, hipStream_t s)
{
    const bool dir = op.bc_z == DIR;
    if (rows == 8) {
        if (dir) inv_rb<T, DIR, 8>(op, a, s);
        else inv_rb<T, AXIPCG_Z_NEUMANN, 8>(op, a, s);
    } else {
        if (dir) inv_rb<T, DIR, 4>(op, a, s);
        else inv_rb<T, AXIPCG_Z_NEUMANN, 4>(op, a, s);
    }
}

template <typename T>
bool usable_t(const Operator &op, int R)
{
    if (R != 4 && R != 8) return false;
    if (strip_r2<T>(op.nz) == 0 || op.nr % R != 0) return false;
    const int G = op.nr / R;
    return G >= 1 && G <= 1024 && strip_red_lds<T>(op.nr, G, red_mt_for<T>(op.nr, G)) <= 160 * 1024;
}

}  // namespace

// The strip path serves an operator and precision with strips of `rows`
// rows (4 or 8) when the one-wave transforms cover nz, the rows split into
// such strips and the reduced system fits one wavefront's registers (at most
// 1024 strips) and its workgroup's LDS.
bool strip_usable(const Operator &op, int prec, int rows)
{
    if (!op.strip_red) return false;
    return prec == AXIPCG_PREC_FP32 ? usable_t<float>(op, rows) : usable_t<double>(op, rows);
}

// Reduced data for strips of 4 rows (the larger of the two heights' needs).
size_t strip_red_bytes(int nr, int nz)
{
    return (nr % 4 == 0) ? 3 * (size_t)(nr / 4) * nz * sizeof(double) : 0;
}

void strip_fwd(const Operator &op, int prec, int rows, const ZfwdArgs &a, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) fwd_t<float>(op, rows, a, s);
    else fwd_t<double>(op, rows, a, s);
}

void strip_reduced(const Operator &op, int prec, int rows, const TriGate &g, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) {
        if (rows == 8) red_r<float, 8>(op, g, s);
        else red_r<float, 4>(op, g, s);
    } else {
        if (rows == 8) red_r<double, 8>(op, g, s);
        else red_r<double, 4>(op, g, s);
    }
}

void strip_inv(const Operator &op, int prec, int rows, const ZinvArgs &a, hipStream_t s)
{
    if (prec == AXIPCG_PREC_FP32) inv_t<float>(op, rows, a, s);
    else inv_t<double>(op, rows, a, s);
}

}  // namespace axipcg
