// Single-launch form of the strip-partitioned preconditioner z = B^{-1} r
// (§4.2 eqs. (36)-(39), with the partition idea of §3): the three phases of
// strip.h in one cooperative launch, separated by two grid barriers.  The
// grid is the G = nr / R strips, all resident; the strip's forward-
// eliminated data f' stays in its workgroup's LDS from phase 1 to phase 3,
// so the spectral round trip through HBM of the three-launch form (4 + 4
// bytes per point in FP32) disappears and only the reduced data (E1, G0,
// X: three values per strip and mode) crosses workgroups:
//
//  phase 1  transform of the strip's rows, forward sweep of its interior
//           rows per mode (f' in LDS), E1 and G0 to global memory
//  barrier
//  phase 2  [PCG: the stop test, every workgroup reaching the same verdict]
//           reduced systems of the modes [s mpw, (s + 1) mpw), X to global
//  barrier
//  phase 3  back substitution from X_{s-1}, X_s; inverse transform to z
//
// Used for FP32 standalone applies (plain transform) and for the PCG
// iteration (the x, r update fused into phase 1, ||r||^2 and r.z partials as
// in the three launches), when the strips fit the chip at once.
//
// Grid barriers (gridbar.h).  Barrier numbers come from a per-handle launch
// counter (2 epoch + 1 and 2 epoch + 2).  A barrier that does not complete
// within the spin limit sets the error word, fills the strip's output with
// NaN and (in PCG mode) marks the solve broken down, and the kernel returns.
#include "gridbar.h"
#include "strip.h"

namespace axipcg {
namespace {


template <typename T>
struct OneArgs {
    // phase 1: plain (rin) or the PCG step (x, r, p, q, p.q partials)
    const double *rin;
    double *x, *r;
    const double *p, *q;
    PcgState *st;
    double *partials;
    int n_pq;
    T *red_e, *red_g, *red_x;
    TriGate g;             // phase 2: stop test (mode 1) or none (mode 0)
    double *zout;          // phase 3
    const typename vec2_of<T>::type *tw, *pt;
    Lines<T> ln;
    int nr, G, mpw;
    unsigned *bar;
    int *err;
    unsigned epoch;
};

// KIND 0: standalone apply (plain transform, no gate, z out);
// KIND 1: PCG iteration (x, r update, stop test, z and r.z partials).
template <typename T, int BC, int KIND, int R2, int R>
__global__ void __launch_bounds__(64 * R) k_strip_one(OneArgs<T> A)
{
    constexpr bool PCG = KIND == 1;
    constexpr int LMAX = 8;
    using Gm = wfft::Geo<R2>;
    constexpr int N = Gm::N, PITCH = 2 * Gm::LB;
    __shared__ double red[RED_SLOTS];
    __shared__ int flag;
    extern __shared__ char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    T *base2 = tile + R * PITCH;
    const int s = blockIdx.x;
    auto fail = [&]() {
        if (threadIdx.x == 0) {
            __hip_atomic_store(A.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (PCG) A.st->done = ST_BREAK;
        }
        for (int e = threadIdx.x; e < R * N; e += blockDim.x) A.zout[(size_t)s * R * N + e] = __builtin_nan("");
    };
    // every workgroup reaches the same verdict (the stop flag and p.q are
    // read or summed identically), so either all continue or all return
    if (!strip_phase1<T, BC, PCG, R2, R>(A.rin, A.x, A.r, A.p, A.q, A.st, A.partials, A.n_pq, nullptr, A.red_e,
                                         A.red_g, A.tw, A.pt, A.ln, A.nr, s, tile))
        return;
    if (!grid_sync(A.bar, A.G, 2u * A.epoch + 1u, &flag)) return fail();
    if (PCG && tridiag_gate(A.st, A.partials, A.g, red, s) != ST_RUN) return;
    const int l0 = s * A.mpw, cnt = N - l0 < A.mpw ? N - l0 : A.mpw;
    if (cnt > 0) {
        strip_stage2<T, false>(A.red_e, A.red_g, A.ln, A.nr, N, A.G, l0, cnt, base2);
        __syncthreads();
        strip_solve2<T, R, LMAX, false>(A.red_x, A.ln, A.nr, N, A.G, l0, cnt, base2);
    }
    if (!grid_sync(A.bar, A.G, 2u * A.epoch + 2u, &flag)) return fail();
    strip_phase3<T, BC, PCG ? 1 : 0, R2, R>(nullptr, A.red_x, A.zout, A.r, A.st, A.partials, false, A.tw, A.pt,
                                            A.ln, A.nr, nullptr, 0.0, 0.0, s, tile);
}

template <int BC, int KIND, int R2>
void *one_kernel_r(int R)
{
    if (R == 8) return reinterpret_cast<void *>(&k_strip_one<float, BC, KIND, R2, 8>);
    return reinterpret_cast<void *>(&k_strip_one<float, BC, KIND, R2, 4>);
}

template <int BC, int KIND>
void *one_kernel(int nz, int R)
{
    switch (nz) {
    case 256: return one_kernel_r<BC, KIND, 2>(R);
    case 512: return one_kernel_r<BC, KIND, 4>(R);
    case 1024: return one_kernel_r<BC, KIND, 8>(R);
    case 2048: return one_kernel_r<BC, KIND, 16>(R);
    default: return nullptr;
    }
}

int r2_of(int nz) { return nz / 128; }

}  // namespace

// Plan of the single launch for `kind` (0 standalone apply, 1 PCG
// iteration) in FP32: the strip height (8 for standalone applies of rows of
// 2048, else 4, the height of the three-launch strips of the same handle),
// and a check that every strip's workgroup is resident at once.
bool pfused_plan(Operator &op, int kind)
{
    PfPlan &pl = op.pf[kind];
    if (pl.state != 0) return pl.state > 0;
    pl.state = -1;
    if (!op.strip_red) return false;
    const int N = op.nz, nr = op.nr;
    if (N < 256 || N > 2048 || op.strip_rows != 4) return false;
    const int R = (kind == 0 && N == 2048 && nr % 8 == 0) ? 8 : 4;
    if (nr % R != 0) return false;
    const int G = nr / R;
    if (G < 1 || G > 512) return false;
    int dev = 0, cus = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    const int mpw = (N + G - 1) / G;
    const size_t shm = (size_t)R * (r2_of(N) * 72) * sizeof(cx<float>) + strip_red_lds<float>(nr, G, mpw);
    if (shm > 160 * 1024) return false;
    void *fn = nullptr;
    if (op.bc_z == DIR) fn = kind == 0 ? one_kernel<DIR, 0>(N, R) : one_kernel<DIR, 1>(N, R);
    else fn = kind == 0 ? one_kernel<AXIPCG_Z_NEUMANN, 0>(N, R) : one_kernel<AXIPCG_Z_NEUMANN, 1>(N, R);
    if (!fn) return false;
    if (shm > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) != hipSuccess)
        return false;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * R, shm) != hipSuccess) return false;
    if ((long)per_cu * cus < G) return false;
    pl.G = G;
    pl.R = R;
    pl.L2 = mpw;
    pl.shm = shm;
    pl.fn = fn;
    pl.state = 1;
    return true;
}

static OneArgs<float> one_args(Operator &op, const PfPlan &pl)
{
    OneArgs<float> a{};
    float *b = static_cast<float *>(op.strip_red);
    const size_t gn = (size_t)pl.G * op.nz;
    a.red_e = b;
    a.red_g = b + gn;
    a.red_x = b + 2 * gn;
    a.tw = op.tw32;
    a.pt = op.pt32;
    a.ln = {op.cb32, op.db32, op.rw32, op.lam32};
    a.nr = op.nr;
    a.G = pl.G;
    a.mpw = pl.L2;
    a.bar = op.pf_bar;
    a.err = op.pf_err;
    a.epoch = ++op.pf_epoch;
    return a;
}

void pfused_apply(Operator &op, const double *r, double *z, hipStream_t s)
{
    const PfPlan &pl = op.pf[0];
    OneArgs<float> a = one_args(op, pl);
    a.rin = r;
    a.zout = z;
    void *args[] = {&a};
    AXI_CHECK_HIP(hipLaunchCooperativeKernel(pl.fn, dim3(pl.G), dim3(64 * pl.R), args, (unsigned)pl.shm, s));
}

void pfused_pcg_step(Operator &op, const ZfwdArgs &fa, const TriGate &g, const ZinvArgs &ia, hipStream_t s)
{
    const PfPlan &pl = op.pf[1];
    OneArgs<float> a = one_args(op, pl);
    a.x = fa.x;
    a.r = fa.r;
    a.p = fa.p;
    a.q = fa.q;
    a.st = fa.state;
    a.partials = op.partials;
    a.n_pq = fa.n_pq;
    a.g = g;
    a.zout = ia.zout;
    void *args[] = {&a};
    AXI_CHECK_HIP(hipLaunchCooperativeKernel(pl.fn, dim3(pl.G), dim3(64 * pl.R), args, (unsigned)pl.shm, s));
}

}  // namespace axipcg
