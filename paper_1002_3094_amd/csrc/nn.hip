// Learned initial guess for the Laguerre series (an extension beyond the
// paper; PCG of §2.2 still decides the answer).
//
// A 6-layer 3x3 convolutional network, 32 channels wide, maps four input
// channels of harmonic m -- u_{m-1}/s, u_{m-2}/s, b_m/s_b and (kappa-2.5)/1.5,
// s = RMS(u_{m-1}), s_b = RMS(b_m) -- to a correction c, and the guess is
// x_P + s c: the network corrects the polynomial extrapolation in m of the
// handle's base order P (P = 1, the default: 2 u_{m-1} - u_{m-2}; P up to 6
// through u_{m-1}, ..., u_{m-1-P}), which is formed in FP64 outside it, so
// the network's own rounding noise scales with the correction only.  ReLU after every layer but the
// last, zero "same" padding.  Weights and activations are BF16, products are
// accumulated in FP32 by MFMA (v_mfma_f32_16x16x16_bf16); training keeps FP32
// master weights with Adam.
//
// Training minimises the energy norm of the guess error, (g - u)^T A (g - u),
// the norm of CG's error bound; unlike an L2 loss it weighs the grid-scale
// roughness a pointwise network produces, and unlike a residual loss (A^2
// weighting) its gradients stay dominated by the learnable smooth part.  The
// guard picks, among u_{m-1}, the extrapolation and the network guess, the
// one with the smallest residual |b - A x|: PCG's stop test measures that
// norm, and with a spectrally equivalent preconditioner the iterations a
// start needs follow it.
//
// Every convolution is an implicit GEMM over 16-pixel tiles of one grid row:
// M = pixels, N = output channels, K = 9 taps x input channels.  A wave holds
// all of its layer's B fragments in registers and sweeps tiles.  The data
// gradient is the same kernel with flipped, transposed weights and the ReLU
// mask of the layer below fused into its epilogue.  The weight gradient is a
// GEMM over pixels (M = output channels, N = input channels, K = pixels) fed
// from channel-major tiles staged in LDS, with per-workgroup partials summed
// in a fixed order.
#include <cmath>
#include <vector>

#include "kernels.h"

namespace axipcg {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;

constexpr int NL = 6;
constexpr int NPARAM = 38465;
__host__ __device__ constexpr int cin_of(int l) { return l == 0 ? 4 : 32; }
__host__ __device__ constexpr int cout_of(int l) { return l == NL - 1 ? 1 : 32; }
__host__ __device__ constexpr int cinp_of(int l) { return l == 0 ? 16 : 32; }     // padded for MFMA K
__host__ __device__ constexpr int coutp_of(int l) { return l == NL - 1 ? 16 : 32; }
// offset of layer l's parameters: W[t][ci][co] (9 cin cout values) then b[co]
__host__ __device__ constexpr int param_off(int l)
{
    int o = 0;
    for (int j = 0; j < l; ++j) o += 9 * cin_of(j) * cout_of(j) + cout_of(j);
    return o;
}
static_assert(param_off(NL) == NPARAM, "parameter count");

__host__ __device__ inline bf16 to_bf16(float f)
{
    unsigned u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    return (bf16)(u >> 16);
}
__device__ inline float from_bf16(bf16 h) { return __uint_as_float((unsigned)h << 16); }

struct Net {
    int nr = 0, nz = 0, device = 0;
    float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
    long long adam_t = 0;
    bf16 *wf_fwd[NL] = {}, *wf_bwd[NL] = {};
    float *bias_p[NL] = {};
    bf16 *act[NL] = {};          // act[0]: packed input (16 ch); act[l]: output of layer l-1 (32 ch)
    float *out = nullptr;        // last layer (1 channel, FP32)
    bf16 *dpre[2] = {};          // gradient w.r.t. a layer's pre-activation (<= 32 ch)
    float *wpart = nullptr;      // weight-gradient partials [WG_BLOCKS][9*32*32 + 32]
    double *scal = nullptr;      // [0] s, [1] s_b, [2] loss, [3] residual of guess, [4] residual of u1
    double *red = nullptr;       // [GMAX + 1][MAX_PARTIALS] partial sums
    double *res_host = nullptr;  // pinned
    int base = 1;                // order of the extrapolation the network corrects
};

constexpr int WG_BLOCKS = 1024;
constexpr int WG_SEG = 64;   // pixels per staged segment of the weight gradient

// ---- input normalisation -----------------------------------------------------
__global__ void __launch_bounds__(256)
k_nn_norms(const double *__restrict__ u1, const double *__restrict__ b, size_t n, double *red)
{
    __shared__ double sm[8];
    double s1 = 0.0, s2 = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        s1 += u1[e] * u1[e];
        s2 += b[e] * b[e];
    }
    const double t1 = block_sum(s1, sm);
    const double t2 = block_sum(s2, sm);
    if (threadIdx.x == 0) {
        red[blockIdx.x] = t1;
        red[MAX_PARTIALS + blockIdx.x] = t2;
    }
}

// (a one-workgroup launch: folding these sums into every workgroup of the
// packing kernel made it slower than the two launches together)
__global__ void __launch_bounds__(256) k_nn_norms_fin(const double *red, int nb, size_t n, double *scal)
{
    __shared__ double sm[8];
    const double t1 = block_total(red, nb, sm);
    const double t2 = block_total(red + MAX_PARTIALS, nb, sm);
    if (threadIdx.x == 0) {
        const double s = sqrt(t1 / (double)n), sb = sqrt(t2 / (double)n);
        scal[0] = s > 0 ? s : 1.0;
        scal[1] = sb > 0 ? sb : 1.0;
    }
}

__global__ void __launch_bounds__(256)
k_nn_pack(const double *__restrict__ u1, const double *__restrict__ u2, const double *__restrict__ b,
          const double *__restrict__ kap, bf16 *__restrict__ act0, size_t n, const double *scal)
{
    const double is = 1.0 / scal[0], ib = 1.0 / scal[1];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        bf16x4 v;
        v[0] = (short)to_bf16((float)(u1[e] * is));
        v[1] = (short)to_bf16((float)(u2[e] * is));
        v[2] = (short)to_bf16((float)(b[e] * ib));
        v[3] = (short)to_bf16((float)((kap[e] - 2.5) / 1.5));
        *reinterpret_cast<bf16x4 *>(act0 + e * 4) = v;
    }
}

// ---- 3x3 convolution (forward, or data gradient with flipped weights) --------
// Activations are [pixels][C] BF16 with C = 16 or 32 (natural channel order).
// A 32-input-channel convolution uses v_mfma_f32_16x16x32_bf16 (one K-block
// per tap: lane (m, kq) holds channels 8 kq .. 8 kq + 7 of pixel m, one
// 16-byte load); a 16-channel input uses v_mfma_f32_16x16x16_bf16 (channels
// 4 kq .. 4 kq + 3).
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 mbf16x8 __attribute__((ext_vector_type(8)));

template <int CINP>
struct FragT;
template <>
struct FragT<32> { typedef bf16x8 type; };
template <>
struct FragT<16> { typedef bf16x4 type; };

__device__ inline f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mbf16x8, a), __builtin_bit_cast(mbf16x8, b),
                                                   c, 0, 0, 0);
}
__device__ inline f32x4 mfma(const bf16x4 &a, const bf16x4 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// A-operand fragments of input row `row` for the z-offsets dk = -1, 0, +1 of
// the 16-pixel strip starting at column k0 (lane m holds pixel k0 + m).  Out
// of the grid the fragment is zero (the load itself stays in bounds).
template <int CINP>
__device__ inline void load_row(typename FragT<CINP>::type (&f)[3], const bf16 *__restrict__ in, int row, int nr,
                                int nz, int k0, int m, int kq)
{
    typedef typename FragT<CINP>::type Frag;
    constexpr int LANE_OFF = CINP / 4;
    const bool row_ok = row >= 0 && row < nr;
    const int rr = row_ok ? row : 0;
#pragma unroll
    for (int dk = 0; dk < 3; ++dk) {
        const int col = k0 + m + dk - 1;
        const bool ok = row_ok && col >= 0 && col < nz;
        const int cc = ok ? col : 0;
        const Frag v = *reinterpret_cast<const Frag *>(in + ((size_t)rr * nz + cc) * CINP + kq * LANE_OFF);
        f[dk] = ok ? v : Frag{};
    }
}

template <int CINP, int NB>
__device__ inline void conv_taps(f32x4 (&acc)[NB], const typename FragT<CINP>::type (&r)[3],
                                 const typename FragT<CINP>::type (&w)[9][NB], int di)
{
#pragma unroll
    for (int dk = 0; dk < 3; ++dk)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma(r[dk], w[di * 3 + dk][nb], acc[nb]);
}

// Epilogue of a hidden layer for one 16-pixel tile: bias is already in acc
// (D layout: lane (m, kq) holds pixels 4 kq + j of channels 16 nb + m);
// ReLU, BF16, transpose through the wave's own LDS slice, then coalesced
// 16-byte stores ([pixels][32]), with the ReLU mask of the layer below
// applied when MASK.  Only this wave touches the slice and a wave's LDS
// operations complete in issue order, so a compiler fence orders the write,
// the read and the next tile's write.
template <bool RELU, bool MASK>
__device__ inline void store_hidden(const f32x4 (&acc)[2], bf16 *ep, bf16 *__restrict__ out,
                                    const bf16 *__restrict__ mask, size_t pix0, int lane)
{
    const int m = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float v = acc[nb][j];
            if (RELU) v = v > 0.f ? v : 0.f;
            ep[(4 * kq + j) * 32 + nb * 16 + m] = to_bf16(v);
        }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int lp = lane >> 2, q = lane & 3;
    bf16x8 v = *reinterpret_cast<const bf16x8 *>(&ep[lp * 32 + q * 8]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const size_t g = (pix0 + lp) * 32 + q * 8;
    if (MASK) {
        const bf16x8 mk = *reinterpret_cast<const bf16x8 *>(mask + g);
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (!(mk[e] > 0)) v[e] = 0;   // a BF16 value is positive iff its bits are, as int16
    }
    *reinterpret_cast<bf16x8 *>(out + g) = v;
}

// Input layer (4 channels) as im2col: K = tap * 4 + channel over the nine
// taps, padded to three K-blocks of 16; lane (m, kq) of K-block kb loads the
// four channels of pixel m at tap 4 kb + kq (zero past tap 8 or outside the
// grid).  Six v_mfma_f32_16x16x16_bf16 per 16-pixel tile instead of 18 with
// the channels padded to 16.  wf: [3 kb][2 nb][64 lanes] fragments.
__global__ void __launch_bounds__(256)
k_conv_in(const bf16 *__restrict__ in, bf16 *__restrict__ out, const bf16x4 *__restrict__ wf,
          const float *__restrict__ bias, int nr, int nz, int rows_per_band)
{
    __shared__ bf16 ep[4][16 * 32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int groups = nz >> 6;
    const int band = blockIdx.x / groups, grp = blockIdx.x - band * groups;
    const int k0 = (grp * 4 + wv) * 16;
    const int i0 = band * rows_per_band;
    const int i1 = min(nr, i0 + rows_per_band);
    bf16x4 w[3][2];
#pragma unroll
    for (int kb = 0; kb < 3; ++kb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) w[kb][nb] = wf[(kb * 2 + nb) * 64 + lane];
    const float b0 = bias[m], b1 = bias[16 + m];
    // fragment of K-block kb for output row i (row i + 1's are loaded while row i computes)
    auto load = [&](bf16x4 (&a)[3], int i) {
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) {
            const int t = 4 * kb + kq;
            const int ii = i + t / 3 - 1, kk = k0 + m + t % 3 - 1;
            const bool ok = t < 9 && ii >= 0 && ii < nr && kk >= 0 && kk < nz;
            const bf16x4 v = *reinterpret_cast<const bf16x4 *>(in + (ok ? (size_t)ii * nz + kk : 0) * 4);
            a[kb] = ok ? v : bf16x4{0, 0, 0, 0};
        }
    };
    bf16x4 cur[3], nxt[3];
    load(cur, i0);
    for (int i = i0; i < i1; ++i) {
        if (i + 1 < i1) load(nxt, i + 1);
        f32x4 acc[2] = {f32x4{b0, b0, b0, b0}, f32x4{b1, b1, b1, b1}};
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) {
            acc[0] = mfma(cur[kb], w[kb][0], acc[0]);
            acc[1] = mfma(cur[kb], w[kb][1], acc[1]);
        }
        store_hidden<true, false>(acc, ep[wv], out, nullptr, (size_t)i * nz + k0, lane);
#pragma unroll
        for (int kb = 0; kb < 3; ++kb) cur[kb] = nxt[kb];
    }
}

// One workgroup = 4 waves on 4 adjacent 16-pixel strips of one band of rows.
// Each wave streams down its strip keeping input rows i-1, i, i+1 (and the
// prefetched i+2) in registers, so every input row is read once per strip.
// in: [pixels][CINP]; out: [pixels][32] BF16 or, LAST, FP32 channel 0; wf: B
// fragments [9][COUTP/16][64 lanes]; MASK zeroes outputs where mask (same
// layout as out) is not positive.
template <int CINP, int COUTP, bool RELU, bool MASK, bool LAST>
__global__ void __launch_bounds__(256)
k_conv3(const bf16 *__restrict__ in, void *__restrict__ outp, const typename FragT<CINP>::type *__restrict__ wf,
        const float *__restrict__ bias, const bf16 *__restrict__ mask, int nr, int nz, int rows_per_band)
{
    typedef typename FragT<CINP>::type Frag;
    constexpr int NB = COUTP / 16;
    static_assert(LAST || COUTP == 32, "hidden outputs have 32 channels");
    __shared__ bf16 ep[4][16 * 32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int groups = nz >> 6;
    const int band = blockIdx.x / groups, grp = blockIdx.x - band * groups;
    const int k0 = (grp * 4 + wv) * 16;
    const int i0 = band * rows_per_band;
    const int i1 = min(nr, i0 + rows_per_band);

    Frag w[9][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) w[t][nb] = wf[(t * NB + nb) * 64 + lane];
    float bl[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) bl[nb] = bias ? bias[nb * 16 + m] : 0.f;

    auto row_out = [&](int i, const Frag(&ra)[3], const Frag(&rb)[3], const Frag(&rc)[3]) {
        f32x4 acc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = f32x4{bl[nb], bl[nb], bl[nb], bl[nb]};
        conv_taps<CINP, NB>(acc, ra, w, 0);
        conv_taps<CINP, NB>(acc, rb, w, 1);
        conv_taps<CINP, NB>(acc, rc, w, 2);
        const size_t pix0 = (size_t)i * nz + k0;
        if constexpr (LAST) {
            // D layout: lane holds pixels 4 kq + j of channel 16 nb + m
            if (m == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) static_cast<float *>(outp)[pix0 + 4 * kq + j] = acc[0][j];
            }
        } else {
            store_hidden<RELU, MASK>(acc, ep[wv], static_cast<bf16 *>(outp), mask, pix0, lane);
        }
    };

    // a ring of five input rows: output row i needs rows i-1..i+1 while rows
    // i+2 and i+3 are in flight
    Frag S0[3], S1[3], S2[3], S3[3], S4[3];
    load_row<CINP>(S0, in, i0 - 1, nr, nz, k0, m, kq);
    load_row<CINP>(S1, in, i0, nr, nz, k0, m, kq);
    load_row<CINP>(S2, in, i0 + 1, nr, nz, k0, m, kq);
    load_row<CINP>(S3, in, i0 + 2, nr, nz, k0, m, kq);
    for (int i = i0; i < i1; i += 5) {
        load_row<CINP>(S4, in, i + 3, nr, nz, k0, m, kq);
        row_out(i, S0, S1, S2);
        if (i + 1 >= i1) break;
        load_row<CINP>(S0, in, i + 4, nr, nz, k0, m, kq);
        row_out(i + 1, S1, S2, S3);
        if (i + 2 >= i1) break;
        load_row<CINP>(S1, in, i + 5, nr, nz, k0, m, kq);
        row_out(i + 2, S2, S3, S4);
        if (i + 3 >= i1) break;
        load_row<CINP>(S2, in, i + 6, nr, nz, k0, m, kq);
        row_out(i + 3, S3, S4, S0);
        if (i + 4 >= i1) break;
        load_row<CINP>(S3, in, i + 7, nr, nz, k0, m, kq);
        row_out(i + 4, S4, S0, S1);
    }
}

// ---- history of earlier harmonics and the extrapolation weights -------------
// History u_{m-1}, ..., u_{m-K} (K <= GMAX); row p of kExtrap holds the
// weights of the order-p polynomial extrapolation through the last p + 1
// harmonics, (-1)^i C(p+1, i+1) for u_{m-1-i}.
constexpr int GMAX = 7;
static_assert(GMAX <= PARTIAL_ROWS, "the guard's partial rows");
struct Hist {
    const double *u[GMAX];
};
__device__ constexpr double kExtrap[GMAX][GMAX] = {
    {1, 0, 0, 0, 0, 0, 0},           {2, -1, 0, 0, 0, 0, 0},         {3, -3, 1, 0, 0, 0, 0},
    {4, -6, 4, -1, 0, 0, 0},         {5, -10, 10, -5, 1, 0, 0},      {6, -15, 20, -15, 6, -1, 0},
    {7, -21, 35, -35, 21, -7, 1}};

// ---- loss: energy norm of the guess error ----------------------------------------
// e = x_P + s out - u_target, y = A e (A symmetric), L = e.y / (s^2 P);
// dL/dout = 2 y / (s P), written as the BF16 gradient seed (channel 0 of 16).
// x_P, the base, from the history h: sum_{j <= P} kExtrap[P][j] h_j.
__device__ inline double guess_err(const float *out, const Hist &h, int order, const double *ut, double s,
                                   size_t q)
{
    double x = 0.0;
#pragma unroll
    for (int j = 0; j < GMAX; ++j)
        if (j <= order) x += kExtrap[order][j] * h.u[j][q];
    return x + s * (double)out[q] - ut[q];
}

__global__ void __launch_bounds__(256)
k_nn_energy_seed(const float *__restrict__ out, Hist h, int order, const double *__restrict__ ut,
                 const double *__restrict__ D, const double *__restrict__ CR, const double *__restrict__ CZ, int nr,
                 int nz, bf16 *__restrict__ dpre, const double *scal, double *red)
{
    __shared__ double sm[8];
    const size_t n = (size_t)nr * nz;
    const double s = scal[0];
    const double g = 2.0 / (s * (double)n);
    double acc = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / nz), k = (int)(e - (size_t)i * nz);
        const double ee = guess_err(out, h, order, ut, s, e);
        double y = D[e] * ee;
        if (i + 1 < nr) y -= CR[e] * guess_err(out, h, order, ut, s, e + nz);
        if (i > 0) y -= CR[e - nz] * guess_err(out, h, order, ut, s, e - nz);
        if (k + 1 < nz) y -= CZ[e] * guess_err(out, h, order, ut, s, e + 1);
        if (k > 0) y -= CZ[e - 1] * guess_err(out, h, order, ut, s, e - 1);
        acc += ee * y;
        alignas(16) bf16 v[16] = {};
        v[0] = to_bf16((float)(g * y));
        uint4 *dst = reinterpret_cast<uint4 *>(dpre + e * 16);
        dst[0] = *reinterpret_cast<const uint4 *>(&v[0]);
        dst[1] = *reinterpret_cast<const uint4 *>(&v[8]);
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) red[2 * MAX_PARTIALS + blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_nn_loss_fin(const double *red, int nb, size_t n, double *scal)
{
    __shared__ double sm[8];
    const double t = block_total(red + 2 * MAX_PARTIALS, nb, sm);
    if (threadIdx.x == 0) scal[2] = t / (scal[0] * scal[0] * (double)n);
}

// ---- weight gradient ------------------------------------------------------------
// dW[t][ci][co] = sum_p x[p + off_t][ci] g[p][co] and db[co] = sum_p g[p][co],
// a GEMM over pixels per tap (M = co, N = ci, K = pixels) with
// v_mfma_f32_16x16x32_bf16.  A workgroup stages one 64-pixel segment of a
// row at a time in LDS, channel-major so that a lane's eight consecutive
// pixels are one aligned 16-byte read: g of the row, and x of rows i-1..i+1
// in three copies shifted by the z-offset of the tap.  Each wave owns one
// (co-block, ci-block) pair and a share of the taps; per-workgroup partials
// [block][t][co][ci] (+ bias) are summed in a fixed order afterwards.  x has
// CMEM channels in memory (4 for the input layer), padded to CINP in LDS.
constexpr int WG_PITCH = WG_SEG + 8;   // LDS row pitch (elements): staggers banks, keeps 16-byte alignment

template <int CINP, int COUTP, int CMEM>
__global__ void __launch_bounds__(256)
k_wgrad(const bf16 *__restrict__ act, const bf16 *__restrict__ dpre, float *__restrict__ wpart, int nr, int nz)
{
    constexpr int NBO = COUTP / 16, NBI = CINP / 16, NPAIR = NBO * NBI;
    constexpr int PARTS = 4 / NPAIR;                 // waves sharing a pair split the taps
    constexpr int TPW = (9 + PARTS - 1) / PARTS;     // taps per wave
    __shared__ __attribute__((aligned(16))) bf16 xs[3][3][CINP][WG_PITCH];
    __shared__ __attribute__((aligned(16))) bf16 gs[COUTP][WG_PITCH];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int pair = wv % NPAIR, part = wv / NPAIR;
    const int ob = pair / NBI, ib = pair - ob * NBI;
    const int t0 = part * TPW;
    f32x4 acc[TPW];
#pragma unroll
    for (int u = 0; u < TPW; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;
    const int segs_per_row = nz / WG_SEG;
    const int nseg = nr * segs_per_row;
    for (int sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const int i = sg / segs_per_row, k0 = (sg - i * segs_per_row) * WG_SEG;
        __syncthreads();
        // g of row i: task (co, octet), eight 2-byte loads (lanes on consecutive co coalesce)
        for (int e = threadIdx.x; e < COUTP * 8; e += blockDim.x) {
            const int co = e % COUTP, o = e / COUTP;
            bf16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (short)dpre[((size_t)i * nz + k0 + 8 * o + j) * COUTP + co];
            *reinterpret_cast<bf16x8 *>(&gs[co][8 * o]) = v;
        }
        // x of rows i-1..i+1: task (ci, octet, row) loads ten pixels and
        // writes the three z-shifted octets
        for (int e = threadIdx.x; e < 3 * 8 * CINP; e += blockDim.x) {
            const int ci = e % CINP, o = (e / CINP) % 8, r = e / (8 * CINP);
            const int ii = i + r - 1;
            short v[10];
#pragma unroll
            for (int j = 0; j < 10; ++j) {
                const int kk = k0 + 8 * o + j - 1;
                const bool ok = ci < CMEM && ii >= 0 && ii < nr && kk >= 0 && kk < nz;
                v[j] = ok ? (short)act[((size_t)ii * nz + kk) * CMEM + ci] : (short)0;
            }
#pragma unroll
            for (int dk = 0; dk < 3; ++dk) {
                bf16x8 w;
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = v[j + dk];
                *reinterpret_cast<bf16x8 *>(&xs[r][dk][ci][8 * o]) = w;
            }
        }
        __syncthreads();
        if (threadIdx.x < COUTP) {
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const bf16x8 v = *reinterpret_cast<const bf16x8 *>(&gs[threadIdx.x][8 * o]);
#pragma unroll
                for (int j = 0; j < 8; ++j) dbias += from_bf16((bf16)v[j]);
            }
        }
#pragma unroll
        for (int ks = 0; ks < WG_SEG / 32; ++ks) {
            const int q = ks * 32 + kq * 8;
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&gs[ob * 16 + m][q]);
#pragma unroll
            for (int u = 0; u < TPW; ++u) {
                const int t = t0 + u;
                if (t < 9) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&xs[t / 3][t % 3][ib * 16 + m][q]);
                    acc[u] = mfma(a, b, acc[u]);
                }
            }
        }
    }
    // D[co][ci]: lane holds co = 16 ob + 4 kq + j, ci = 16 ib + m
    float *wp = wpart + (size_t)blockIdx.x * (9 * 32 * 32 + 32);
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
        const int t = t0 + u;
        if (t < 9) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int co = ob * 16 + 4 * kq + j, ci = ib * 16 + m;
                wp[(t * COUTP + co) * CINP + ci] = acc[u][j];
            }
        }
    }
    if (threadIdx.x < COUTP) wp[9 * 32 * 32 + threadIdx.x] = dbias;
}

// grads (master layout) = sum of the partials over workgroups in a fixed
// order: 32 parameters per workgroup, eight threads per parameter striding
// over the partials, then the eight sums in order.
template <int CINP, int COUTP>
__global__ void __launch_bounds__(256)
k_wgrad_reduce(const float *__restrict__ wpart, int nblk, float *__restrict__ grads, int cin, int cout)
{
    __shared__ double sm[8][32];
    const int nw = 9 * cin * cout;
    const int pl = threadIdx.x & 31, part = threadIdx.x >> 5;
    const int e = blockIdx.x * 32 + pl;
    int src = -1;
    if (e < nw) {
        const int t = e / (cin * cout), rem = e - t * cin * cout;
        const int ci = rem / cout, co = rem - ci * cout;
        src = (t * COUTP + co) * CINP + ci;
    } else if (e < nw + cout) {
        src = 9 * 32 * 32 + (e - nw);
    }
    double acc = 0.0;
    if (src >= 0)
        for (int b = part; b < nblk; b += 8) acc += wpart[(size_t)b * (9 * 32 * 32 + 32) + src];
    sm[part][pl] = acc;
    __syncthreads();
    if (part == 0 && src >= 0) {
        double t = 0.0;
        for (int j = 0; j < 8; ++j) t += sm[j][pl];
        grads[e] = (float)t;
    }
}

// ---- Adam on the FP32 master weights ---------------------------------------------
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const float gv = g[e];
        const float a = b1 * m1[e] + (1.f - b1) * gv;
        const float v = b2 * m2[e] + (1.f - b2) * gv * gv;
        m1[e] = a;
        m2[e] = v;
        p[e] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
    }
}

// ---- master weights -> BF16 MFMA fragments ----------------------------------------
// Fragment (t, nb, lane, item) of a convolution with C input channels
// (K = C per tap; 8 items per lane when C = 32, 4 when C = 16):
//   B[k = (C/4) (lane/16) + item][n = 16 nb + lane%16].
// Forward: k = ci, n = co of W[t]; data gradient (flipped, transposed):
// k = co, n = ci of W[8 - t].
template <int L>
__global__ void k_pack_weights(const float *__restrict__ params, bf16 *__restrict__ wf, bf16 *__restrict__ wb,
                               float *__restrict__ bias_p)
{
    constexpr int CI = cin_of(L), CO = cout_of(L), CIP = cinp_of(L), COP = coutp_of(L);
    const float *W = params + param_off(L);
    const float *bias = W + 9 * CI * CO;
    if constexpr (L == 0) {
        // input layer, im2col: fragment (kb, nb, lane, item) holds
        // W[t = 4 kb + lane/16][ci = item][co = 16 nb + lane%16] (0 past tap 8)
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 3 * 2 * 64 * 4; e += gridDim.x * blockDim.x) {
            const int item = e & 3, lane = (e >> 2) & 63, frag = e >> 8;
            const int nb = frag & 1, kb = frag >> 1;
            const int t = 4 * kb + (lane >> 4), co = 16 * nb + (lane & 15);
            wf[e] = to_bf16(t < 9 ? W[(t * CI + item) * CO + co] : 0.f);
        }
        for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < COP; c += gridDim.x * blockDim.x) bias_p[c] = bias[c];
        return;
    }
    const int nf = 9 * CIP * COP;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += gridDim.x * blockDim.x) {
        // forward: K = CIP, N = COP
        {
            constexpr int IT = CIP / 4;
            const int item = e % IT, lane = (e / IT) % 64, frag = e / (IT * 64);
            const int nb = frag % (COP / 16), t = frag / (COP / 16);
            const int ci = IT * (lane >> 4) + item, co = 16 * nb + (lane & 15);
            wf[e] = to_bf16((ci < CI && co < CO) ? W[(t * CI + ci) * CO + co] : 0.f);
        }
        // data gradient: K = COP (its input channels), N = CIP
        if (wb) {
            constexpr int IT = COP / 4;
            const int item = e % IT, lane = (e / IT) % 64, frag = e / (IT * 64);
            const int nb = frag % (CIP / 16), t = frag / (CIP / 16);
            const int co = IT * (lane >> 4) + item, ci = 16 * nb + (lane & 15);
            wb[e] = to_bf16((ci < CI && co < CO) ? W[((8 - t) * CI + ci) * CO + co] : 0.f);
        }
    }
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < COP; c += gridDim.x * blockDim.x)
        bias_p[c] = c < CO ? bias[c] : 0.f;
}

// guess = 2 u1 - u2 + s * out
__global__ void __launch_bounds__(256)
k_nn_unpack(const double *u1, const double *u2, const float *__restrict__ out, double *g, size_t n,
            const double *scal)
{
    const double s = scal[0];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        g[e] = 2.0 * u1[e] - u2[e] + s * (double)out[e];
}

// ---- guard -------------------------------------------------------------------------
// ---- the guard: candidate initial guesses ranked by residual ----------------
// History u_{m-1}, ..., u_{m-K} (K <= GMAX).  Candidate p < K is the
// polynomial extrapolation of order p through the last p + 1 harmonics,
//     x_p = sum_{i <= p} (-1)^i C(p+1, i+1) u_{m-1-i}
// (u_{m-1}; 2 u_{m-1} - u_{m-2}; 3 u_{m-1} - 3 u_{m-2} + u_{m-3}; ...), and
// with a network candidate K the learned guess x_P + s out (its correction
// sits on the extrapolation of the handle's base order P).  PCG's stop test measures |b - A x|, and
// with a spectrally equivalent preconditioner the iterations a start needs
// follow it, so the guard ranks the candidates by that norm.

__device__ inline double2 ld_pair(const double *p) { return *reinterpret_cast<const double2 *>(p); }
__device__ inline double2 ld_pair(const float *p)
{
    const float2 v = *reinterpret_cast<const float2 *>(p);
    return double2{(double)v.x, (double)v.y};
}

// f + |r|^2 without contraction into fused multiply-adds, so that equal
// residuals give bit-equal sums whichever candidate they belong to (ties then
// keep the lower-order candidate)
__device__ inline double add_sq(double f, double2 r)
{
    return __dadd_rn(f, __dadd_rn(__dmul_rn(r.x, r.x), __dmul_rn(r.y, r.y)));
}

// (A v) at the element pair (k, k + 1) of row i, k even (d, cz: the pair's
// diagonal and z-couplings, already loaded)
template <typename V>
__device__ inline double2 apply_pair(const V *__restrict__ v, double2 d, double2 cz, const double *__restrict__ CR,
                                     const double *__restrict__ CZ, size_t e, int i, int k, int nr, int nz)
{
    // no fused multiply-adds: A u computed here, cached, or in another kernel
    // is the same to the last bit
#pragma clang fp contract(off)
    const double2 c = ld_pair(v + e);
    double2 a{d.x * c.x, d.y * c.y};
    if (i + 1 < nr) {
        const double2 cr = ld_pair(CR + e), vn = ld_pair(v + e + nz);
        a.x -= cr.x * vn.x;
        a.y -= cr.y * vn.y;
    }
    if (i > 0) {
        const double2 cr = ld_pair(CR + e - nz), vn = ld_pair(v + e - nz);
        a.x -= cr.x * vn.x;
        a.y -= cr.y * vn.y;
    }
    a.x -= cz.x * c.y;   // (k, k+1) inside the pair, k-1 and k+2 outside
    a.y -= cz.x * c.x;
    if (k + 2 < nz) a.y -= cz.y * (double)v[e + 2];
    if (k > 0) a.x -= CZ[e - 1] * (double)v[e - 1];
    return a;
}

// Partial sums of |b - A x_p|^2 for every candidate: red[p][MAX_PARTIALS],
// p < K the extrapolations, p = K the network.  Workgroups take whole rows,
// the rows of one XCD contiguous (their neighbour rows then come from that
// XCD's L2); each thread the element pairs (k, k + 1), k even.  A x_p is
// formed from the A u_j, so each history array is read once.  CACHED: A u_j
// for j >= 1 is read from ah.u[j] (computed for an earlier harmonic), and
// A u_0 is computed and also stored in ah0 for the next one.
template <int K, bool NET, bool CACHED>
__global__ void __launch_bounds__(256)
k_guess_hist(const double *__restrict__ b, Hist h, Hist ah, double *__restrict__ ah0,
             const float *__restrict__ out, int nbase, const double *__restrict__ D, const double *__restrict__ CR,
             const double *__restrict__ CZ, int nr, int nz, const double *scal, double *red)
{
#pragma clang fp contract(off)
    static_assert(K >= 1 && K <= GMAX && (!NET || K >= 2), "history length");
    __shared__ double sm[8];
    const double s = NET ? scal[0] : 0.0;
    double f[K + 1];
#pragma unroll
    for (int p = 0; p <= K; ++p) f[p] = 0.0;
    for (int blk = blockIdx.x; blk < nr; blk += gridDim.x) {
        const int i = xcd_swizzle(blk, nr);
        for (int k = 2 * threadIdx.x; k < nz; k += 512) {
            const size_t e = (size_t)i * nz + k;
            const double2 d = ld_pair(D + e), cz = ld_pair(CZ + e), bv = ld_pair(b + e);
            double2 au[K];
            au[0] = apply_pair(h.u[0], d, cz, CR, CZ, e, i, k, nr, nz);
            if (CACHED) *reinterpret_cast<double2 *>(ah0 + e) = au[0];
#pragma unroll
            for (int j = 1; j < K; ++j)
                au[j] = CACHED ? ld_pair(ah.u[j] + e) : apply_pair(h.u[j], d, cz, CR, CZ, e, i, k, nr, nz);
            double2 r1{0.0, 0.0};
#pragma unroll
            for (int p = 0; p < K; ++p) {
                double2 a{0.0, 0.0};
#pragma unroll
                for (int q = 0; q <= p; ++q) {
                    a.x += kExtrap[p][q] * au[q].x;
                    a.y += kExtrap[p][q] * au[q].y;
                }
                const double2 r{bv.x - a.x, bv.y - a.y};
                if (p == nbase) r1 = r;
                f[p] = add_sq(f[p], r);
            }
            if (NET) {
                // the network's candidate is x_P + s out (P = nbase): its
                // residual is r_P - s A out
                const double2 ao = apply_pair(out, d, cz, CR, CZ, e, i, k, nr, nz);
                f[K] = add_sq(f[K], double2{r1.x - s * ao.x, r1.y - s * ao.y});
            }
        }
    }
#pragma unroll
    for (int p = 0; p <= K; ++p) {
        if (p == K && !NET) break;
        const double t = block_sum(f[p], sm);
        if (threadIdx.x == 0) red[(size_t)p * MAX_PARTIALS + blockIdx.x] = t;
    }
}

// Block sums of R rows of partials (row stride MAX_PARTIALS), every row's
// loads in flight together (one row after another waits R round trips);
// each row in the same fixed order, so equal rows give equal sums.  The
// result is valid in thread 0.
template <int R>
__device__ inline void block_totals(const double *__restrict__ parts, int n, double (&out)[R], double *sm)
{
    const int nt = blockDim.x;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int base = 0; base < n; base += 4 * nt) {
        double v[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = base + (int)threadIdx.x + j * nt;
                v[r][j] = (i < n) ? parts[(size_t)r * MAX_PARTIALS + i] : 0.0;
            }
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] += (v[r][0] + v[r][1]) + (v[r][2] + v[r][3]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) out[r] = block_sum(acc[r], sm);
}

// The residual norms res[p] (p <= K; res[K] NaN without a network) and the
// choice res[K + 1]: the candidates in the order x_0, x_1, ..., network, a
// later one replacing the choice only when its residual is strictly smaller
// (a NaN never does).  One workgroup.
template <int K, bool NET>
__global__ void __launch_bounds__(256) k_guess_fin(const double *red, int nb, double *res)
{
    __shared__ double sm[8];
    constexpr int R = NET ? K + 1 : K;
    double t[R];
    block_totals<R>(red, nb, t, sm);
    double f[K + 1];
#pragma unroll
    for (int p = 0; p < K; ++p) f[p] = sqrt(t[p]);
    f[K] = NET ? sqrt(t[R - 1]) : __builtin_nan("");
    int c = 0;
    double best = f[0];
#pragma unroll
    for (int p = 1; p <= K; ++p)
        if ((p < K || NET) && f[p] < best) {
            c = p;
            best = f[p];
        }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int p = 0; p <= K; ++p) res[p] = f[p];
        res[K + 1] = (double)c;
    }
}

// x = the chosen candidate; x may alias a history array (element-wise read
// before write).
template <int K, bool NET>
__global__ void __launch_bounds__(256)
k_guess_pick(Hist h, const float *__restrict__ out, int nbase, double *x, size_t n, const double *res,
             const double *scal)
{
    const int c = (int)res[K + 1];
    const double s = NET ? scal[0] : 0.0;
    const int order = c < K ? c : nbase;   // the network's candidate sits on x_nbase
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        double u[K];
#pragma unroll
        for (int q = 0; q < K; ++q) u[q] = q <= order ? h.u[q][e] : 0.0;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (q <= order) v += kExtrap[order][q] * u[q];
        if (NET && c == K) v += s * (double)out[e];
        x[e] = v;
    }
}

// ---- host helpers -------------------------------------------------------------------
template <typename P>
void nalloc(P **p, size_t count)
{
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, count * sizeof(P));
    if (e != hipSuccess) throw Error{AXIPCG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    *p = static_cast<P *>(v);
}

void free_net(Net *n)
{
    if (!n) return;
    std::vector<void *> ptrs = {n->params, n->grads, n->m1, n->m2, n->out, n->dpre[0], n->dpre[1], n->wpart,
                                n->scal, n->red};
    for (int l = 0; l < NL; ++l) {
        ptrs.push_back(n->wf_fwd[l]);
        ptrs.push_back(n->wf_bwd[l]);
        ptrs.push_back(n->bias_p[l]);
        ptrs.push_back(n->act[l]);
    }
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (n->res_host) (void)hipHostFree(n->res_host);
    delete n;
}

unsigned pw_blocks(size_t n) { return pointwise_blocks(n); }
// grid of a reduction kernel: at most 1024 partial sums for its one-block finish
unsigned red_blocks(size_t n)
{
    const unsigned b = pointwise_blocks(n);
    return b < 1024 ? b : 1024;
}

// grid of the guard's residual kernel: whole rows per workgroup, at most 1024
// partial sums
unsigned guard_blocks(int nr) { return nr < 1024 ? (unsigned)nr : 1024u; }

// y = A v with the guard's own stencil arithmetic (fills the cache of A u).
__global__ void __launch_bounds__(256)
k_apply_pairs(const double *__restrict__ v, double *__restrict__ y, const double *__restrict__ D,
              const double *__restrict__ CR, const double *__restrict__ CZ, int nr, int nz)
{
    for (int blk = blockIdx.x; blk < nr; blk += gridDim.x) {
        const int i = xcd_swizzle(blk, nr);
        for (int k = 2 * threadIdx.x; k < nz; k += 512) {
            const size_t e = (size_t)i * nz + k;
            *reinterpret_cast<double2 *>(y + e) =
                apply_pair(v, ld_pair(D + e), ld_pair(CZ + e), CR, CZ, e, i, k, nr, nz);
        }
    }
}

template <int K, bool NET>
void guard_k(const Operator &op, const double *b, const Hist &h, const float *out, int nbase, const double *scal,
             double *red, double *x, double *res, hipStream_t s, const Hist *ah, double *ah0)
{
    const size_t np = (size_t)op.nr * op.nz;
    const unsigned pb = guard_blocks(op.nr);
    if (ah)
        hipLaunchKernelGGL((k_guess_hist<K, NET, true>), dim3(pb), dim3(256), 0, s, b, h, *ah, ah0, out, nbase, op.D, op.CR,
                           op.CZ, op.nr, op.nz, scal, red);
    else
        hipLaunchKernelGGL((k_guess_hist<K, NET, false>), dim3(pb), dim3(256), 0, s, b, h, h, nullptr, out, nbase, op.D,
                           op.CR, op.CZ, op.nr, op.nz, scal, red);
    hipLaunchKernelGGL((k_guess_fin<K, NET>), dim3(1), dim3(256), 0, s, red, (int)pb, res);
    hipLaunchKernelGGL((k_guess_pick<K, NET>), dim3(pw_blocks(np)), dim3(256), 0, s, h, out, nbase, x, np, res, scal);
    AXI_CHECK_HIP(hipGetLastError());
}

// Guard over the history h (K arrays) and, with out, the network candidate
// x_nbase + s out (nbase < K): partial sums in red (K + 1 rows), norms and
// choice in res (K + 2 values).  With ah: A h.u[j] for j >= 1 cached there,
// A h.u[0] stored into ah0.
void run_guard(const Operator &op, const double *b, const Hist &h, int K, const float *out, int nbase,
               const double *scal, double *red, double *x, double *res, hipStream_t s, const Hist *ah = nullptr,
               double *ah0 = nullptr)
{
    if (out) AXI_REQUIRE(nbase >= 1 && nbase < K, "the network's base order needs more history arrays");
#define AXI_G(KK, NN) return guard_k<KK, NN>(op, b, h, out, nbase, scal, red, x, res, s, ah, ah0)
    if (out) {
        switch (K) {
        case 2: AXI_G(2, true);
        case 3: AXI_G(3, true);
        case 4: AXI_G(4, true);
        case 5: AXI_G(5, true);
        case 6: AXI_G(6, true);
        case 7: AXI_G(7, true);
        default: break;
        }
    } else {
        switch (K) {
        case 1: AXI_G(1, false);
        case 2: AXI_G(2, false);
        case 3: AXI_G(3, false);
        case 4: AXI_G(4, false);
        case 5: AXI_G(5, false);
        case 6: AXI_G(6, false);
        case 7: AXI_G(7, false);
        default: break;
        }
    }
#undef AXI_G
    throw Error{AXIPCG_EINVAL, "history length out of range"};
}

// The history arrays of a guard call (host array of K device pointers).
Hist make_hist(const double *const *hist, int K, const double *x, const double *b, const double *kappa)
{
    AXI_REQUIRE(hist != nullptr, "hist is NULL");
    AXI_REQUIRE(K >= 1 && K <= GMAX, "history length must be in [1, 7]");
    Hist h{};
    for (int j = 0; j < K; ++j) {
        AXI_REQUIRE(hist[j] != nullptr, "NULL history array");
        AXI_REQUIRE(hist[j] != b && hist[j] != kappa, "a history array aliases b or kappa");
        h.u[j] = hist[j];
    }
    AXI_REQUIRE(x != b && x != kappa, "x aliases b or kappa");
    return h;
}

void pack_all(Net &n, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_weights<0>, dim3(16), dim3(256), 0, s, n.params, n.wf_fwd[0], nullptr, n.bias_p[0]);
    hipLaunchKernelGGL(k_pack_weights<1>, dim3(64), dim3(256), 0, s, n.params, n.wf_fwd[1], n.wf_bwd[1], n.bias_p[1]);
    hipLaunchKernelGGL(k_pack_weights<2>, dim3(64), dim3(256), 0, s, n.params, n.wf_fwd[2], n.wf_bwd[2], n.bias_p[2]);
    hipLaunchKernelGGL(k_pack_weights<3>, dim3(64), dim3(256), 0, s, n.params, n.wf_fwd[3], n.wf_bwd[3], n.bias_p[3]);
    hipLaunchKernelGGL(k_pack_weights<4>, dim3(64), dim3(256), 0, s, n.params, n.wf_fwd[4], n.wf_bwd[4], n.bias_p[4]);
    hipLaunchKernelGGL(k_pack_weights<5>, dim3(32), dim3(256), 0, s, n.params, n.wf_fwd[5], n.wf_bwd[5], n.bias_p[5]);
    AXI_CHECK_HIP(hipGetLastError());
}

// Rows per band of a convolution launch: about `waves` waves over the nz/16
// strips (2048 = one round at two waves per SIMD on 1024 SIMDs for the
// register-heavy 32-channel kernels), at least 4 rows so the halo rows stay a
// small overhead.
int conv_rows(int nr, int nz, long waves = 2048)
{
    const long strips = nz / 16;
    long r = ((long)nr * strips + waves - 1) / waves;
    if (r < 4) r = 4;
    return (int)r;
}

unsigned conv_blocks(int nr, int nz, int rows)
{
    return (unsigned)(((nr + rows - 1) / rows) * (nz / 64));
}

void forward_impl(Net &n, const double *u1, const double *u2, const double *b, const double *kap, hipStream_t s)
{
    const size_t np = (size_t)n.nr * n.nz;
    const unsigned rb = red_blocks(np);
    hipLaunchKernelGGL(k_nn_norms, dim3(rb), dim3(256), 0, s, u1, b, np, n.red);
    hipLaunchKernelGGL(k_nn_norms_fin, dim3(1), dim3(256), 0, s, n.red, (int)rb, np, n.scal);
    hipLaunchKernelGGL(k_nn_pack, dim3(pw_blocks(np)), dim3(256), 0, s, u1, u2, b, kap, n.act[0], np, n.scal);
    const int rows = conv_rows(n.nr, n.nz);
    const dim3 cg(conv_blocks(n.nr, n.nz, rows)), cb(256);
    const int rows_in = conv_rows(n.nr, n.nz, 8192);
    hipLaunchKernelGGL(k_conv_in, dim3(conv_blocks(n.nr, n.nz, rows_in)), cb, 0, s, n.act[0], n.act[1],
                       (const bf16x4 *)n.wf_fwd[0], n.bias_p[0], n.nr, n.nz, rows_in);
    for (int l = 1; l < NL - 1; ++l)
        hipLaunchKernelGGL((k_conv3<32, 32, true, false, false>), cg, cb, 0, s, n.act[l], (void *)n.act[l + 1],
                           (const bf16x8 *)n.wf_fwd[l], n.bias_p[l], nullptr, n.nr, n.nz, rows);
    hipLaunchKernelGGL((k_conv3<32, 16, false, false, true>), cg, cb, 0, s, n.act[NL - 1], (void *)n.out,
                       (const bf16x8 *)n.wf_fwd[NL - 1], n.bias_p[NL - 1], nullptr, n.nr, n.nz, rows);
    AXI_CHECK_HIP(hipGetLastError());
}

// h: the forward's history (at least base + 1 arrays)
void backward_impl(Net &n, const Operator &op, const Hist &h, const double *ut, hipStream_t s)
{
    const size_t np = (size_t)n.nr * n.nz;
    const unsigned pb = red_blocks(np);
    hipLaunchKernelGGL(k_nn_energy_seed, dim3(pb), dim3(256), 0, s, n.out, h, n.base, ut, op.D, op.CR, op.CZ, n.nr,
                       n.nz, n.dpre[0], n.scal, n.red);
    hipLaunchKernelGGL(k_nn_loss_fin, dim3(1), dim3(256), 0, s, n.red, (int)pb, np, n.scal);
    const int rows = conv_rows(n.nr, n.nz);
    const dim3 cg(conv_blocks(n.nr, n.nz, rows)), cb(256);
    const int nseg = (int)(np / WG_SEG);
    const int wgb = nseg < WG_BLOCKS ? nseg : WG_BLOCKS;
    int cur = 0;
    for (int l = NL - 1; l >= 0; --l) {
        float *g = n.grads + param_off(l);
        const int rb = (9 * cin_of(l) * cout_of(l) + cout_of(l) + 31) / 32;
        // weight gradient of layer l from act[l] and dpre[cur]
        if (l == 0) {
            hipLaunchKernelGGL((k_wgrad<16, 32, 4>), dim3(wgb), dim3(256), 0, s, n.act[0], n.dpre[cur], n.wpart, n.nr, n.nz);
            hipLaunchKernelGGL((k_wgrad_reduce<16, 32>), dim3(rb), dim3(256), 0, s, n.wpart, wgb, g, cin_of(l), cout_of(l));
        } else if (l == NL - 1) {
            hipLaunchKernelGGL((k_wgrad<32, 16, 32>), dim3(wgb), dim3(256), 0, s, n.act[l], n.dpre[cur], n.wpart, n.nr, n.nz);
            hipLaunchKernelGGL((k_wgrad_reduce<32, 16>), dim3(rb), dim3(256), 0, s, n.wpart, wgb, g, cin_of(l), cout_of(l));
        } else {
            hipLaunchKernelGGL((k_wgrad<32, 32, 32>), dim3(wgb), dim3(256), 0, s, n.act[l], n.dpre[cur], n.wpart, n.nr, n.nz);
            hipLaunchKernelGGL((k_wgrad_reduce<32, 32>), dim3(rb), dim3(256), 0, s, n.wpart, wgb, g, cin_of(l), cout_of(l));
        }
        // data gradient into layer l-1's pre-activation (masked by its ReLU output act[l])
        if (l >= 1) {
            if (l == NL - 1)
                hipLaunchKernelGGL((k_conv3<16, 32, false, true, false>), cg, cb, 0, s, n.dpre[cur], (void *)n.dpre[1 - cur],
                                   (const bf16x4 *)n.wf_bwd[l], nullptr, n.act[l], n.nr, n.nz, rows);
            else
                hipLaunchKernelGGL((k_conv3<32, 32, false, true, false>), cg, cb, 0, s, n.dpre[cur], (void *)n.dpre[1 - cur],
                                   (const bf16x8 *)n.wf_bwd[l], nullptr, n.act[l], n.nr, n.nz, rows);
            cur = 1 - cur;
        }
    }
    AXI_CHECK_HIP(hipGetLastError());
}

Net *create_impl_nn(int nr, int nz, const float *params)
{
    Net *n = new (std::nothrow) Net();
    if (!n) throw Error{AXIPCG_ENOMEM, "host allocation failed"};
    try {
        n->nr = nr;
        n->nz = nz;
        AXI_CHECK_HIP(hipGetDevice(&n->device));
        const size_t np = (size_t)nr * nz;
        nalloc(&n->params, NPARAM);
        nalloc(&n->grads, NPARAM);
        nalloc(&n->m1, NPARAM);
        nalloc(&n->m2, NPARAM);
        for (int l = 0; l < NL; ++l) {
            nalloc(&n->wf_fwd[l], (size_t)9 * cinp_of(l) * coutp_of(l));
            if (l >= 1) nalloc(&n->wf_bwd[l], (size_t)9 * cinp_of(l) * coutp_of(l));
            nalloc(&n->bias_p[l], (size_t)coutp_of(l));
            nalloc(&n->act[l], np * (size_t)(l == 0 ? cin_of(0) : cinp_of(l)));
        }
        nalloc(&n->out, np);
        nalloc(&n->dpre[0], np * 32);
        nalloc(&n->dpre[1], np * 32);
        nalloc(&n->wpart, (size_t)WG_BLOCKS * (9 * 32 * 32 + 32));
        nalloc(&n->scal, 16);
        nalloc(&n->red, (GMAX + 1) * (size_t)MAX_PARTIALS);
        AXI_CHECK_HIP(hipHostMalloc((void **)&n->res_host, 16 * sizeof(double), hipHostMallocDefault));
        AXI_CHECK_HIP(hipMemcpy(n->params, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
        AXI_CHECK_HIP(hipMemset(n->grads, 0, sizeof(float) * NPARAM));
        AXI_CHECK_HIP(hipMemset(n->m1, 0, sizeof(float) * NPARAM));
        AXI_CHECK_HIP(hipMemset(n->m2, 0, sizeof(float) * NPARAM));
        pack_all(*n, nullptr);
        AXI_CHECK_HIP(hipDeviceSynchronize());
    } catch (...) {
        free_net(n);
        throw;
    }
    return n;
}

}  // namespace

void apply_a_pairs(const Operator &op, const double *v, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_apply_pairs, dim3(guard_blocks(op.nr)), dim3(256), 0, s, v, y, op.D, op.CR, op.CZ, op.nr,
                       op.nz);
    AXI_CHECK_HIP(hipGetLastError());
}

void guess_poly_cached(Operator &op, axipcg_nn_t nn, const double *b, const double *const *hist, int K,
                       double *const *ah, const double *kappa, double *x, hipStream_t s)
{
    const Hist hh = make_hist(hist, K, x, b, kappa);
    Hist ahh{};
    for (int j = 0; j < K; ++j) {
        AXI_REQUIRE(ah && ah[j], "NULL cache array");
        ahh.u[j] = ah[j];
    }
    if (nn) {
        Net *n = reinterpret_cast<Net *>(nn);
        AXI_REQUIRE(K > n->base && kappa, "the learned guess needs base order + 1 history arrays and kappa");
        AXI_REQUIRE(op.nr == n->nr && op.nz == n->nz, "operator and network sizes differ");
        forward_impl(*n, hist[0], hist[1], b, kappa, s);
        run_guard(op, b, hh, K, n->out, n->base, n->scal, n->red, x, n->scal + 3, s, &ahh, ah[0]);
    } else {
        run_guard(op, b, hh, K, nullptr, 0, nullptr, op.partials, x, op.dscal + 8, s, &ahh, ah[0]);
    }
}

}  // namespace axipcg

using namespace axipcg;

extern "C" {

int axipcg_nn_num_params(void) { return NPARAM; }

int axipcg_nn_create(int nr, int nz, const float *params, axipcg_nn_t *out)
{
    return guarded([&] {
        AXI_REQUIRE(out && params, "NULL argument");
        AXI_REQUIRE(nr >= 1 && nr <= 8192, "nr must be in [1, 8192]");
        AXI_REQUIRE(nz >= 64 && nz <= 8192 && nz % 64 == 0, "nz must be a multiple of 64 in [64, 8192]");
        for (int e = 0; e < NPARAM; ++e) AXI_REQUIRE(std::isfinite(params[e]), "non-finite parameter");
        *out = reinterpret_cast<axipcg_nn_t>(create_impl_nn(nr, nz, params));
        return AXIPCG_OK;
    });
}

void axipcg_nn_destroy(axipcg_nn_t h)
{
    Net *n = reinterpret_cast<Net *>(h);
    if (!n) return;
    (void)hipDeviceSynchronize();
    free_net(n);
}

int axipcg_nn_get_params(axipcg_nn_t h, float *params, float *grads)
{
    return guarded([&] {
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(n != nullptr, "NULL network");
        AXI_CHECK_HIP(hipDeviceSynchronize());
        if (params) AXI_CHECK_HIP(hipMemcpy(params, n->params, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
        if (grads) AXI_CHECK_HIP(hipMemcpy(grads, n->grads, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
        return AXIPCG_OK;
    });
}

int axipcg_nn_set_params(axipcg_nn_t h, const float *params)
{
    return guarded([&] {
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(n && params, "NULL argument");
        for (int e = 0; e < NPARAM; ++e) AXI_REQUIRE(std::isfinite(params[e]), "non-finite parameter");
        AXI_CHECK_HIP(hipDeviceSynchronize());
        AXI_CHECK_HIP(hipMemcpy(n->params, params, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
        pack_all(*n, nullptr);
        AXI_CHECK_HIP(hipDeviceSynchronize());
        return AXIPCG_OK;
    });
}

int axipcg_nn_forward(axipcg_nn_t h, const double *u1, const double *u2, const double *b, const double *kappa,
                      double *guess, void *stream)
{
    return guarded([&] {
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(n && u1 && u2 && b && kappa && guess, "NULL argument");
        AXI_REQUIRE(n->base == 1, "the network's base order needs the history form (nn_guess_poly)");
        hipStream_t s = (hipStream_t)stream;
        forward_impl(*n, u1, u2, b, kappa, s);
        const size_t np = (size_t)n->nr * n->nz;
        hipLaunchKernelGGL(k_nn_unpack, dim3(pw_blocks(np)), dim3(256), 0, s, u1, u2, n->out, guess, np, n->scal);
        AXI_CHECK_HIP(hipGetLastError());
        return AXIPCG_OK;
    });
}

int axipcg_nn_backward(axipcg_op_t hop, axipcg_nn_t h, const double *u1, const double *u2, const double *u_target,
                       double *loss_host, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(hop);
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(op && n && u1 && u2 && u_target, "NULL argument");
        AXI_REQUIRE(op->nr == n->nr && op->nz == n->nz, "operator and network sizes differ");
        AXI_REQUIRE(n->base == 1, "the network's base order needs the history form (nn_backward_poly)");
        hipStream_t s = (hipStream_t)stream;
        const double *hist[2] = {u1, u2};
        backward_impl(*n, *op, make_hist(hist, 2, u_target, nullptr, nullptr), u_target, s);
        if (loss_host) {
            AXI_CHECK_HIP(hipMemcpyAsync(n->res_host, n->scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
            AXI_CHECK_HIP(hipStreamSynchronize(s));
            *loss_host = n->res_host[0];
        }
        return AXIPCG_OK;
    });
}

int axipcg_nn_adam(axipcg_nn_t h, double lr, double beta1, double beta2, double eps, void *stream)
{
    return guarded([&] {
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(n != nullptr, "NULL network");
        AXI_REQUIRE(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0, "bad Adam constants");
        hipStream_t s = (hipStream_t)stream;
        n->adam_t += 1;
        const float c1 = (float)(1.0 - std::pow(beta1, (double)n->adam_t));
        const float c2 = (float)(1.0 - std::pow(beta2, (double)n->adam_t));
        hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, n->params, n->grads, n->m1, n->m2,
                           NPARAM, (float)lr, (float)beta1, (float)beta2, (float)eps, c1, c2);
        AXI_CHECK_HIP(hipGetLastError());
        pack_all(*n, s);
        return AXIPCG_OK;
    });
}

int axipcg_nn_set_base(axipcg_nn_t h, int order)
{
    return guarded([&] {
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(n != nullptr, "NULL network");
        AXI_REQUIRE(order >= 1 && order <= GMAX - 1, "base order must be in [1, 6]");
        n->base = order;
        return AXIPCG_OK;
    });
}

int axipcg_nn_get_base(axipcg_nn_t h)
{
    const Net *n = reinterpret_cast<const Net *>(h);
    return n ? n->base : AXIPCG_EINVAL;
}

int axipcg_nn_backward_poly(axipcg_op_t hop, axipcg_nn_t h, const double *const *hist, int K,
                            const double *u_target, double *loss_host, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(hop);
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(op && n && u_target, "NULL argument");
        AXI_REQUIRE(op->nr == n->nr && op->nz == n->nz, "operator and network sizes differ");
        AXI_REQUIRE(K > n->base, "the base order needs base + 1 history arrays");
        const Hist hh = make_hist(hist, K, u_target, nullptr, nullptr);
        hipStream_t s = (hipStream_t)stream;
        backward_impl(*n, *op, hh, u_target, s);
        if (loss_host) {
            AXI_CHECK_HIP(hipMemcpyAsync(n->res_host, n->scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
            AXI_CHECK_HIP(hipStreamSynchronize(s));
            *loss_host = n->res_host[0];
        }
        return AXIPCG_OK;
    });
}

int axipcg_nn_guess(axipcg_op_t hop, axipcg_nn_t h, const double *b, const double *u1, const double *u2,
                    const double *kappa, double *x, double *resid_host, int *choice_host, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(hop);
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(op && n && b && u1 && u2 && kappa && x, "NULL argument");
        AXI_REQUIRE(op->nr == n->nr && op->nz == n->nz, "operator and network sizes differ");
        AXI_REQUIRE(x != b && x != kappa, "x aliases b or kappa");
        AXI_REQUIRE(n->base == 1, "the network's base order needs the history form (nn_guess_poly)");
        hipStream_t s = (hipStream_t)stream;
        forward_impl(*n, u1, u2, b, kappa, s);
        const double *hist[2] = {u1, u2};
        // res: u1, extrapolation, network, choice (0 u1, 1 extrapolation, 2 network)
        double *res = n->scal + 3;
        run_guard(*op, b, make_hist(hist, 2, x, b, kappa), 2, n->out, 1, n->scal, n->red, x, res, s);
        if (resid_host || choice_host) {
            AXI_CHECK_HIP(hipMemcpyAsync(n->res_host, res, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
            AXI_CHECK_HIP(hipStreamSynchronize(s));
            if (resid_host) {
                resid_host[0] = n->res_host[2];
                resid_host[1] = n->res_host[1];
                resid_host[2] = n->res_host[0];
            }
            if (choice_host) *choice_host = (int)n->res_host[3];
        }
        return AXIPCG_OK;
    });
}

int axipcg_nn_guess_poly(axipcg_op_t hop, axipcg_nn_t h, const double *b, const double *const *hist, int K,
                         const double *kappa, double *x, double *resid_host, int *choice_host, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(hop);
        Net *n = reinterpret_cast<Net *>(h);
        AXI_REQUIRE(op && n && b && kappa && x, "NULL argument");
        AXI_REQUIRE(op->nr == n->nr && op->nz == n->nz, "operator and network sizes differ");
        AXI_REQUIRE(K > n->base, "the learned guess needs base order + 1 history arrays");
        const Hist hh = make_hist(hist, K, x, b, kappa);
        hipStream_t s = (hipStream_t)stream;
        forward_impl(*n, hist[0], hist[1], b, kappa, s);
        double *res = n->scal + 3;
        run_guard(*op, b, hh, K, n->out, n->base, n->scal, n->red, x, res, s);
        if (resid_host || choice_host) {
            AXI_CHECK_HIP(hipMemcpyAsync(n->res_host, res, (K + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
            AXI_CHECK_HIP(hipStreamSynchronize(s));
            if (resid_host)
                for (int p = 0; p <= K; ++p) resid_host[p] = n->res_host[p];
            if (choice_host) *choice_host = (int)n->res_host[K + 1];
        }
        return AXIPCG_OK;
    });
}

int axipcg_guess_extrap(axipcg_op_t hop, const double *b, const double *u1, const double *u2, double *x,
                        double *resid_host, int *choice_host, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(hop);
        AXI_REQUIRE(op && b && u1 && u2 && x, "NULL argument");
        hipStream_t s = (hipStream_t)stream;
        const double *hist[2] = {u1, u2};
        // the reductions use the handle's partial-sum rows 0..1 and scalars 8..11,
        // which a solve only reads after writing them itself; res: u1,
        // extrapolation, (no network), choice
        double *res = op->dscal + 8;
        run_guard(*op, b, make_hist(hist, 2, x, b, nullptr), 2, nullptr, 0, nullptr, op->partials, x, res, s);
        if (resid_host || choice_host) {
            AXI_CHECK_HIP(hipMemcpyAsync(op->scratch_host, res, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
            AXI_CHECK_HIP(hipStreamSynchronize(s));
            if (resid_host) {
                resid_host[0] = op->scratch_host[1];
                resid_host[1] = op->scratch_host[0];
            }
            if (choice_host) *choice_host = (int)op->scratch_host[3];
        }
        return AXIPCG_OK;
    });
}

int axipcg_guess_poly(axipcg_op_t hop, const double *b, const double *const *hist, int K, double *x,
                      double *resid_host, int *choice_host, void *stream)
{
    return guarded([&] {
        Operator *op = reinterpret_cast<Operator *>(hop);
        AXI_REQUIRE(op && b && x, "NULL argument");
        const Hist hh = make_hist(hist, K, x, b, nullptr);
        hipStream_t s = (hipStream_t)stream;
        // partial-sum rows 0..K-1 and scalars 8..8+K+1 of the handle (see guess_extrap)
        double *res = op->dscal + 8;
        run_guard(*op, b, hh, K, nullptr, 0, nullptr, op->partials, x, res, s);
        if (resid_host || choice_host) {
            AXI_CHECK_HIP(hipMemcpyAsync(op->scratch_host, res, (K + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
            AXI_CHECK_HIP(hipStreamSynchronize(s));
            if (resid_host)
                for (int p = 0; p < K; ++p) resid_host[p] = op->scratch_host[p];
            if (choice_host) *choice_host = (int)op->scratch_host[K + 1];
        }
        return AXIPCG_OK;
    });
}

}  // extern "C"
