// Single-pass preconditioner z = B^{-1} r on gfx950 (§4.2 eqs. (36)-(39)),
// one cooperative launch instead of three.
//
// The grid is G workgroups, all resident (one per CU), workgroup s owning R =
// nr / G consecutive r-rows (a strip, as in the paper's decomposition of the
// grid into strips of rows, §4.3).  Three phases separated by grid barriers:
//
//  1. Forward z-transform of the strip's rows into LDS.  For every z-mode l,
//     the strip's interior rows are eliminated against the strip's first and
//     last rows (the partition idea of §3: the interior of each part is solved
//     in terms of its boundary values, eqs. (18)-(22)); what remains are two
//     equations per strip and mode, in the unknowns top_s = y(first row) and
//     bot_s = y(last row), coupled to the neighbouring strips.  They are
//     written to global memory.
//  2. The reduced system of mode l (tridiagonal, 2G unknowns ordered top_0,
//     bot_0, top_1, ...) is solved by one wavefront (segments per lane,
//     parallel cyclic reduction across lanes); workgroup w takes modes
//     [w N / G, (w + 1) N / G).
//  3. Each strip reads its top_s and bot_s, solves its interior rows (Thomas),
//     and inverse-transforms its rows into z.
//
// Only the 2 G equations and unknowns per mode cross the grid; the strip's
// spectral data stays in LDS between the phases.
//
// Measured on MI355X at 1024^2 this form is slower than the three launches
// (one workgroup per CU cannot hide the latency of its rows' FFTs the way
// four independent workgroups per CU do, and each grid barrier costs several
// microseconds), so it is opt-in (axipcg_op_set_fused).  Grid barriers are an
// arrival counter and a generation word with agent-scope release/acquire, and
// a bounded wait: a barrier that does not complete within the spin limit
// sets an error flag and the kernel returns (z is then filled with NaN).
#include <cmath>

#include "fft.h"
#include "kernels.h"

namespace axipcg {
namespace {

constexpr int PF_THREADS = 256;
constexpr unsigned long long PF_SPIN_LIMIT = 1ull << 20;

template <typename T> __device__ inline T pf_rcp(T x);
template <> __device__ inline float pf_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double pf_rcp<double>(double x) { return 1.0 / x; }

template <typename T> struct Eq4 { T a, b, c, e; };

// Grid barrier without a contended counter.  bar[0] is the number of
// completed barriers (the generation), bar[1 + s] the last generation
// workgroup s has reached.  Each workgroup releases its stores at agent scope
// (every wave: the L2s of the XCDs are not coherent with each other
// otherwise) and posts its flag; workgroup 0 waits for all flags (one thread
// per flag), acquires, and publishes the new generation; everyone else waits
// for it and acquires.  Every wait is bounded: on giving up the barrier
// returns false.
__device__ inline bool spin_until(const unsigned *w, unsigned target)
{
    unsigned long long n = 0;
    // relaxed polls (no cache invalidation per poll); the acquire follows
    while ((int)(__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
        if (++n > PF_SPIN_LIMIT) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

__device__ inline bool grid_barrier(unsigned *bar, unsigned nblk, unsigned &gen, int *flag_lds)
{
    const unsigned target = gen + 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (threadIdx.x == 0) *flag_lds = 1;
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&bar[1 + blockIdx.x], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (blockIdx.x == 0) {
        for (unsigned t = threadIdx.x; t < nblk; t += blockDim.x)
            if (!spin_until(&bar[1 + t], target)) *flag_lds = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&bar[0], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        if (!spin_until(&bar[0], target)) *flag_lds = 0;
    }
    gen = target;
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *flag_lds != 0;
}

// Orthonormal forward transform of one row by the 256 threads of group
// (local index lt): values rv[j] of k = lt + 256 j, result in `out` (LDS).
// Every group of the block calls this together (block-wide barriers).
template <typename T, int BC>
__device__ inline void fwd_row(const double (&rv)[8], T *__restrict__ out, cx<T> *a, cx<T> *b,
                               const typename vec2_of<T>::type *twp, const typename vec2_of<T>::type *pt, int N,
                               int lt, bool on)
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = lt + j * PF_THREADS;
        if (!on) break;
        if (k < N) {
            T v = (T)rv[j];
            int n;
            if ((k & 1) == 0) {
                n = k >> 1;
            } else {
                n = N - 1 - (k >> 1);
                if (BC == AXIPCG_Z_DIRICHLET) v = -v;
            }
            a[n] = {v, (T)0};
        }
    }
    __syncthreads();
    const cx<T> *Vr = fft_stockham_part<T>(a, b, N, twp, lt, PF_THREADS);
    const T nrm = (T)sqrt(2.0 / N);
    const T half = (T)0.70710678118654752440;
    for (int j = lt; on && j < N; j += PF_THREADS) {
        const int m = (BC == AXIPCG_Z_DIRICHLET) ? N - 1 - j : j;
        const cx<T> w = ld_tw<T>(pt, m);
        const T Y = Vr[m].x * w.x - Vr[m].y * w.y;
        const bool edge = (BC == AXIPCG_Z_DIRICHLET) ? (j == N - 1) : (j == 0);
        out[j] = nrm * (edge ? half : (T)1) * Y;
    }
    __syncthreads();
}

// Inverse of fwd_row: spectral row `in` (LDS) -> zv[j] of k = lt + 256 j.
template <typename T, int BC>
__device__ inline void inv_row(const T *__restrict__ in, double (&zv)[8], cx<T> *a, cx<T> *b,
                               const typename vec2_of<T>::type *twp, const typename vec2_of<T>::type *pt, int N,
                               int lt, bool on)
{
    const T isc = (T)sqrt(0.5 * N);
    const T sq2 = (T)1.41421356237309504880;
    auto Y = [&](int m) -> T {
        const int j = (BC == AXIPCG_Z_DIRICHLET) ? N - 1 - m : m;
        const bool edge = (BC == AXIPCG_Z_DIRICHLET) ? (j == N - 1) : (j == 0);
        return in[j] * isc * (edge ? sq2 : (T)1);
    };
    for (int m = lt; on && m < N; m += PF_THREADS) {
        const T ym = Y(m);
        const T yn = (m == 0) ? (T)0 : Y(N - m);
        const cx<T> w = ld_tw<T>(pt, m);
        a[m] = {w.x * ym - w.y * yn, w.x * yn + w.y * ym};
    }
    __syncthreads();
    const cx<T> *res = fft_stockham_part<T>(a, b, N, twp, lt, PF_THREADS);
    const T invN = (T)1 / (T)N;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = lt + j * PF_THREADS;
        if (on && k < N) {
            const int n = (k & 1) ? N - 1 - (k >> 1) : (k >> 1);
            T v = res[n].x * invN;
            if (BC == AXIPCG_Z_DIRICHLET && (k & 1)) v = -v;
            zv[j] = (double)v;
        }
    }
    __syncthreads();
}

// Reduced system of one mode, n2 = 2G rows (a_k y_{k-1} + b_k y_k + c_k y_{k+1}
// = e_k, a_0 = c_{n2-1} = 0), solved by one wavefront: lane s owns rows
// [s L2, (s+1) L2); its interior rows are eliminated against the interface
// rows (the lane's last row and the previous lane's), the S interface
// unknowns are found by parallel cyclic reduction, then the interior rows.
template <typename T, int L2>
__device__ inline void wave_tridiag(const Eq4<T> *__restrict__ eq, T *__restrict__ sol, int S)
{
    const int lane = threadIdx.x & 63;
    const bool active = lane < S;
    const int lo = lane * L2;
    T a[L2], bb[L2], c[L2], e[L2];
#pragma unroll
    for (int t = 0; t < L2; ++t) {
        if (active) {
            const Eq4<T> q = eq[lo + t];
            a[t] = q.a;
            bb[t] = q.b;
            c[t] = q.c;
            e[t] = q.e;
        } else {
            a[t] = 0;
            bb[t] = 1;
            c[t] = 0;
            e[t] = 0;
        }
    }
    // interior rows t = 0 .. L2-2: y_t = G_t + V_t x_{s-1} + W_t x_s
    T cp[L2], gp[L2], vp[L2], wp[L2];
    T cprev = 0, gprev = 0, vprev = 0, wprev = 0;
#pragma unroll
    for (int t = 0; t < L2 - 1; ++t) {
        const T sub = (t > 0) ? a[t] : (T)0;
        const T inv = pf_rcp<T>(bb[t] - sub * cprev);
        cprev = (t < L2 - 2) ? c[t] * inv : (T)0;
        gprev = (e[t] - sub * gprev) * inv;
        vprev = ((t == 0 ? -a[t] : (T)0) - sub * vprev) * inv;
        wprev = ((t == L2 - 2 ? -c[t] : (T)0) - sub * wprev) * inv;
        cp[t] = cprev;
        gp[t] = gprev;
        vp[t] = vprev;
        wp[t] = wprev;
    }
    T G[L2], V[L2], W[L2];
    G[L2 - 2] = gp[L2 - 2];
    V[L2 - 2] = vp[L2 - 2];
    W[L2 - 2] = wp[L2 - 2];
#pragma unroll
    for (int t = L2 - 3; t >= 0; --t) {
        G[t] = gp[t] - cp[t] * G[t + 1];
        V[t] = vp[t] - cp[t] * V[t + 1];
        W[t] = wp[t] - cp[t] * W[t + 1];
    }
    // interface row of this lane (t = L2-1), using the next lane's first interior row
    const T Gn = __shfl_down(G[0], 1, 64);
    const T Vn = __shfl_down(V[0], 1, 64);
    const T Wn = __shfl_down(W[0], 1, 64);
    const bool has_right = active && lane + 1 < S;
    const T aR = a[L2 - 1], bR = bb[L2 - 1], cR = has_right ? c[L2 - 1] : (T)0;
    T ra = 0, rb = 1, rc = 0, re = 0;
    if (active) {
        ra = aR * V[L2 - 2];
        rb = bR + aR * W[L2 - 2] + (has_right ? cR * Vn : (T)0);
        rc = has_right ? cR * Wn : (T)0;
        re = e[L2 - 1] - aR * G[L2 - 2] - (has_right ? cR * Gn : (T)0);
    }
    for (int k = 1; k < S; k <<= 1) {
        const T am = __shfl_up(ra, k, 64), bm = __shfl_up(rb, k, 64);
        const T cm = __shfl_up(rc, k, 64), em = __shfl_up(re, k, 64);
        const T ap = __shfl_down(ra, k, 64), bp = __shfl_down(rb, k, 64);
        const T cq = __shfl_down(rc, k, 64), ep = __shfl_down(re, k, 64);
        const bool hm = lane >= k, hp = lane + k < S;
        const T al = hm ? -ra * pf_rcp<T>(bm) : (T)0;
        const T ga = hp ? -rc * pf_rcp<T>(bp) : (T)0;
        const T na = hm ? al * am : (T)0;
        const T nc = hp ? ga * cq : (T)0;
        const T nb = rb + (hm ? al * cm : (T)0) + (hp ? ga * ap : (T)0);
        const T ne = re + (hm ? al * em : (T)0) + (hp ? ga * ep : (T)0);
        if (active) {
            ra = na;
            rb = nb;
            rc = nc;
            re = ne;
        }
    }
    const T xs = active ? re / rb : (T)0;
    T xm = __shfl_up(xs, 1, 64);
    if (lane == 0) xm = 0;
    if (active) {
#pragma unroll
        for (int t = 0; t < L2 - 1; ++t) sol[lo + t] = G[t] + V[t] * xm + W[t] * xs;
        sol[lo + L2 - 1] = xs;
    }
}

struct PfArgs {
    const double *rin;
    double *zout;
    int nr, N, G;
    unsigned *bar;
    int *err;
};

template <typename T>
struct PfTables {
    const typename vec2_of<T>::type *tw, *pt;
    const T *cb, *db, *rw, *lam;
    Eq4<T> *eq;   // [N][2G]
    T *sol;       // [N][2G]
};

// R rows per strip; L2 = 2G / min(64, G) reduced rows per lane; the block is
// RP groups of 256 threads, each group transforming one row of the strip at a
// time (RP rows at once).
template <typename T, int BC, int R, int L2, bool TWL, int RP>
__global__ void __launch_bounds__(256 * RP) k_pfused(PfArgs A, PfTables<T> P)
{
    using V2 = typename vec2_of<T>::type;
    constexpr int NT = 256 * RP;
    extern __shared__ char smem_raw[];
    __shared__ int flag;
    const int N = A.N, G = A.G, n2 = 2 * G;
    const int grp = threadIdx.x >> 8, lt = threadIdx.x & 255;
    T *spec = reinterpret_cast<T *>(smem_raw);                                   // [R][N]
    cx<T> *fa = reinterpret_cast<cx<T> *>(spec + (size_t)R * N) + (size_t)grp * 2 * N;
    cx<T> *fb = fa + N;
    V2 *twl = reinterpret_cast<V2 *>(reinterpret_cast<cx<T> *>(spec + (size_t)R * N) + (size_t)RP * 2 * N);
    const V2 *twp = P.tw;
    if (TWL) {
        for (int k = threadIdx.x; k < N; k += NT) twl[k] = P.tw[k];
        twp = twl;
    }
    unsigned gen = __hip_atomic_load(&A.bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int s = blockIdx.x;
    const int i0 = s * R;

    // ---- phase 1: transforms, strip elimination, reduced equations ----
#pragma unroll 1
    for (int t0 = 0; t0 < R; t0 += RP) {
        const int t = t0 + grp;
        const bool on = t < R;
        double rv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = lt + j * PF_THREADS;
            if (on && k < N) rv[j] = A.rin[(size_t)(i0 + t) * N + k];
        }
        fwd_row<T, BC>(rv, spec + (size_t)(on ? t : 0) * N, fa, fb, twp, P.pt, N, lt, on);
    }
    T cbv[R], dbv[R], rwv[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        cbv[t] = P.cb[i0 + t];
        dbv[t] = P.db[i0 + t];
        rwv[t] = P.rw[i0 + t];
    }
    const T cbm1 = i0 > 0 ? P.cb[i0 - 1] : (T)0;
    for (int j = threadIdx.x; j < N; j += NT) {
        const T lm = P.lam[j];
        T D[R], f[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            D[t] = dbv[t] + rwv[t] * lm;
            f[t] = spec[(size_t)t * N + j];
        }
        Eq4<T> top, bot;
        if constexpr (R > 2) {
            // interior rows 1..R-2 with three right-hand sides: data, top, bottom
            T cp[R], gp[R], ap[R], bp[R];
            T cprev = 0, gprev = 0, aprev = 0, bprev = 0;
#pragma unroll
            for (int t = 1; t <= R - 2; ++t) {
                const T sub = (t > 1) ? -cbv[t - 1] : (T)0;
                const T inv = pf_rcp<T>(D[t] - sub * cprev);
                cprev = (t < R - 2) ? -cbv[t] * inv : (T)0;
                gprev = (f[t] - sub * gprev) * inv;
                aprev = ((t == 1 ? cbv[0] : (T)0) - sub * aprev) * inv;
                bprev = ((t == R - 2 ? cbv[R - 2] : (T)0) - sub * bprev) * inv;
                cp[t] = cprev;
                gp[t] = gprev;
                ap[t] = aprev;
                bp[t] = bprev;
            }
            T g1 = gp[R - 2], a1 = ap[R - 2], b1 = bp[R - 2];   // back-substitute to row 1
            const T gL = g1, aL = a1, bL = b1;                  // row R-2
#pragma unroll
            for (int t = R - 3; t >= 1; --t) {
                g1 = gp[t] - cp[t] * g1;
                a1 = ap[t] - cp[t] * a1;
                b1 = bp[t] - cp[t] * b1;
            }
            top = {-cbm1, D[0] - cbv[0] * a1, -cbv[0] * b1, f[0] + cbv[0] * g1};
            bot = {-cbv[R - 2] * aL, D[R - 1] - cbv[R - 2] * bL, -cbv[R - 1], f[R - 1] + cbv[R - 2] * gL};
        } else {
            top = {-cbm1, D[0], -cbv[0], f[0]};
            bot = {-cbv[0], D[1], -cbv[1], f[1]};
        }
        P.eq[(size_t)j * n2 + 2 * s] = top;
        P.eq[(size_t)j * n2 + 2 * s + 1] = bot;
    }
    bool ok = grid_barrier(A.bar, (unsigned)G, gen, &flag);

    // ---- phase 2: reduced systems of this workgroup's modes ----
    if (ok) {
        const int mpw = N / G;
        const int wv = threadIdx.x >> 6;
        const int S = G < 64 ? G : 64;
        for (int u = wv; u < mpw; u += NT / 64) {
            const int j = s * mpw + u;
            wave_tridiag<T, L2>(P.eq + (size_t)j * n2, P.sol + (size_t)j * n2, S);
        }
        ok = grid_barrier(A.bar, (unsigned)G, gen, &flag);
    }
    if (!ok) {
        if (threadIdx.x == 0) __hip_atomic_store(A.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int t = 0; t < R; ++t)
            for (int k = threadIdx.x; k < N; k += NT) A.zout[(size_t)(i0 + t) * N + k] = __builtin_nan("");
        return;
    }

    // ---- phase 3: interior rows from top/bot, inverse transforms ----
    for (int j = threadIdx.x; j < N; j += NT) {
        const T top = P.sol[(size_t)j * n2 + 2 * s];
        const T bot = P.sol[(size_t)j * n2 + 2 * s + 1];
        spec[j] = top;
        spec[(size_t)(R - 1) * N + j] = bot;
        if constexpr (R > 2) {
            const T lm = P.lam[j];
            T cp[R], dp[R];
            T cprev = 0, dprev = 0;
#pragma unroll
            for (int t = 1; t <= R - 2; ++t) {
                const T D = dbv[t] + rwv[t] * lm;
                const T sub = (t > 1) ? -cbv[t - 1] : (T)0;
                const T inv = pf_rcp<T>(D - sub * cprev);
                T rhs = spec[(size_t)t * N + j];
                if (t == 1) rhs += cbv[0] * top;
                if (t == R - 2) rhs += cbv[R - 2] * bot;
                cprev = (t < R - 2) ? -cbv[t] * inv : (T)0;
                dprev = (rhs - sub * dprev) * inv;
                cp[t] = cprev;
                dp[t] = dprev;
            }
            T y = dp[R - 2];
            spec[(size_t)(R - 2) * N + j] = y;
#pragma unroll
            for (int t = R - 3; t >= 1; --t) {
                y = dp[t] - cp[t] * y;
                spec[(size_t)t * N + j] = y;
            }
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int t0 = 0; t0 < R; t0 += RP) {
        const int t = t0 + grp;
        const bool on = t < R;
        double zv[8];
        inv_row<T, BC>(spec + (size_t)(on ? t : 0) * N, zv, fa, fb, twp, P.pt, N, lt, on);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = lt + j * PF_THREADS;
            if (on && k < N) A.zout[(size_t)(i0 + t) * N + k] = zv[j];
        }
    }
}

template <typename T>
bool pf_twl(int N) { return (size_t)N * sizeof(cx<T>) <= 16384; }

template <typename T>
size_t pf_lds(int R, int RP, int N)
{
    return (size_t)R * N * sizeof(T) + (2 * (size_t)RP + (pf_twl<T>(N) ? 1 : 0)) * (size_t)N * sizeof(cx<T>);
}

template <typename T, int BC, int R, int L2, int RP>
void *pf_kernel(int N)
{
    if (pf_twl<T>(N)) return reinterpret_cast<void *>(&k_pfused<T, BC, R, L2, true, RP>);
    return reinterpret_cast<void *>(&k_pfused<T, BC, R, L2, false, RP>);
}

template <typename T, int BC, int R, int RP>
void *pf_kernel_l2(int L2, int N)
{
    switch (L2) {
    case 2: return pf_kernel<T, BC, R, 2, RP>(N);
    case 4: return pf_kernel<T, BC, R, 4, RP>(N);
    case 8: return pf_kernel<T, BC, R, 8, RP>(N);
    default: return nullptr;
    }
}

template <typename T, int BC, int R>
void *pf_kernel_rp(int RP, int L2, int N)
{
    switch (RP) {
    case 1: return pf_kernel_l2<T, BC, R, 1>(L2, N);
    case 2: return pf_kernel_l2<T, BC, R, 2>(L2, N);
    default: return nullptr;
    }
}

template <typename T, int BC>
void *pf_kernel_r(int R, int RP, int L2, int N)
{
    switch (R) {
    case 2: return pf_kernel_rp<T, BC, 2>(RP, L2, N);
    case 4: return pf_kernel_rp<T, BC, 4>(RP, L2, N);
    case 8: return pf_kernel_rp<T, BC, 8>(RP, L2, N);
    case 16: return pf_kernel_rp<T, BC, 16>(RP, L2, N);
    default: return nullptr;
    }
}

template <typename T>
void *pf_select(int bc, int R, int RP, int L2, int N)
{
    return bc == AXIPCG_Z_DIRICHLET ? pf_kernel_r<T, AXIPCG_Z_DIRICHLET>(R, RP, L2, N)
                                    : pf_kernel_r<T, AXIPCG_Z_NEUMANN>(R, RP, L2, N);
}

}  // namespace

// Plan the single-pass preconditioner for this operator and precision, or
// return false when its geometry or residency does not hold (the three-launch
// path is then used): G a power of two dividing nr and nz with R = nr / G in
// {2, 4, 8, 16}, 2G / min(64, G) in {2, 4, 8}, the strip in LDS, and all G
// workgroups resident at once.
bool pfused_plan(Operator &op, int prec)
{
    PfPlan &pl = op.pf[prec == AXIPCG_PREC_FP32 ? 1 : 0];
    if (pl.state != 0) return pl.state > 0;
    pl.state = -1;
    int dev = 0, cus = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    const int N = op.nz, nr = op.nr;
    for (int G = 256; G >= 16; G >>= 1) {
        if (G > cus || nr % G != 0 || N % G != 0) continue;
        const int R = nr / G;
        const int L2 = 2 * G / (G < 64 ? G : 64);
        if (R != 2 && R != 4 && R != 8 && R != 16) continue;
        if (L2 != 2 && L2 != 4 && L2 != 8) continue;
        // rows transformed at once: two when they fit in LDS (four groups of
        // 256 threads leave too few registers and spill)
        int RP = R < 2 ? R : 2;
        auto lds = [&](int rp) { return prec == AXIPCG_PREC_FP32 ? pf_lds<float>(R, rp, N) : pf_lds<double>(R, rp, N); };
        while (RP > 1 && lds(RP) > 150 * 1024) RP >>= 1;
        const size_t shm = lds(RP);
        if (shm > 150 * 1024) continue;
        void *fn = prec == AXIPCG_PREC_FP32 ? pf_select<float>(op.bc_z, R, RP, L2, N)
                                           : pf_select<double>(op.bc_z, R, RP, L2, N);
        if (!fn) continue;
        if (shm > 65536 &&
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess)
            continue;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256 * RP, shm) != hipSuccess) continue;
        if ((long)per_cu * cus < G) continue;
        const size_t el = prec == AXIPCG_PREC_FP32 ? sizeof(float) : sizeof(double);
        if (!op.pf_work) {
            // reduced equations and unknowns, sized for the larger (FP64) element
            const size_t bytes = (size_t)N * 2 * G * 5 * sizeof(double);
            if (hipMalloc(&op.pf_work, bytes) != hipSuccess) return false;
            op.pf_work_bytes = bytes;
        }
        if ((size_t)N * 2 * G * 5 * el > op.pf_work_bytes) continue;
        pl.G = G;
        pl.RP = RP;
        pl.R = R;
        pl.L2 = L2;
        pl.shm = shm;
        pl.fn = fn;
        pl.state = 1;
        return true;
    }
    return false;
}

template <typename T>
static PfTables<T> pf_tables(const Operator &op, int G);
template <>
PfTables<float> pf_tables<float>(const Operator &op, int G)
{
    Eq4<float> *eq = reinterpret_cast<Eq4<float> *>(op.pf_work);
    float *sol = reinterpret_cast<float *>(eq + (size_t)op.nz * 2 * G);
    return {op.tw32, op.pt32, op.cb32, op.db32, op.rw32, op.lam32, eq, sol};
}
template <>
PfTables<double> pf_tables<double>(const Operator &op, int G)
{
    Eq4<double> *eq = reinterpret_cast<Eq4<double> *>(op.pf_work);
    double *sol = reinterpret_cast<double *>(eq + (size_t)op.nz * 2 * G);
    return {op.tw64, op.pt64, op.cb64, op.db64, op.rw64, op.lam64, eq, sol};
}

void pfused_apply(const Operator &op, const double *r, double *z, int prec, hipStream_t s)
{
    const PfPlan &pl = op.pf[prec == AXIPCG_PREC_FP32 ? 1 : 0];
    PfArgs a{r, z, op.nr, op.nz, pl.G, op.pf_bar, op.pf_err};
    if (prec == AXIPCG_PREC_FP32) {
        PfTables<float> t = pf_tables<float>(op, pl.G);
        void *args[] = {&a, &t};
        AXI_CHECK_HIP(hipLaunchCooperativeKernel(pl.fn, dim3(pl.G), dim3(256 * pl.RP), args, (unsigned)pl.shm, s));
    } else {
        PfTables<double> t = pf_tables<double>(op, pl.G);
        void *args[] = {&a, &t};
        AXI_CHECK_HIP(hipLaunchCooperativeKernel(pl.fn, dim3(pl.G), dim3(256 * pl.RP), args, (unsigned)pl.shm, s));
    }
}

}  // namespace axipcg
