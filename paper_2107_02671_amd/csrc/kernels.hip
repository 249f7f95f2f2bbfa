// HIP kernels of the NNFFT (Algorithm 2.2) for gfx950.
//
// Stage map of one exec:
//   spread   step 1, (2.12): g_l = (1/N1) sum_k f_k phi_1(l/N1 - v*_k)
//   fft      steps 2-3: g_hat_l = g_l / phi_hat_2(l), h_s = (1/N2) DFT; the
//            merge of the spreading partials, the division by phi_hat_2 and
//            both scale factors 1/N1, 1/N2 are fused into the FFT load
//   interp   step 4 + output: y_j = sum_s h_s phi_2(x_j/sigma1 - s/N2)
//            / phi_hat_1(N x_j)
//
// Work decomposition (both node sides): the plan sorts the nodes of each
// block of consecutive caller indices into cell bins; a work item is up to Q
// sorted points of one bin; a workgroup ("chunk") takes up to blockDim items
// of one block covering at most blockDim consecutive bins.
//
// FP32 path.  A point at offset x in [0, 1) of bin c puts the weight
// omega((r - m + 1 - x)/m) on cell c - m + 1 + r (r < 2m).  Each of these 2m
// functions of t = 2x - 1 is a degree-kDeg Chebyshev series with
// coefficients C[r][k] (fitted in FP64 at plan time), so the contribution of
// all points of one bin to tap r is sum_k C[r][k] mu_k with the bin moments
// mu_k = sum_p f_p T_k(t_p).  Spreading therefore accumulates kDeg + 1
// complex moments per point instead of evaluating 2m windows, and the 2m taps
// are formed once per bin.  Interpolation is the transpose: per bin
// H_k = sum_r C[r][k] h_{c-m+1+r}, per point y = sum_k H_k T_k(t).
// Grid cells are accumulated with error-free two-sum transformations
// (hi + lo pairs) from the per-item moments up to the merge in the FFT load.
//
// FP64 path (the plain comparator): the same decomposition, windows evaluated
// exactly per tap with exp/sqrt in FP64, plain FP64 sums.
#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>

#include "internal.h"
#include "../../include/nnfft.h"

namespace nnfft {

// Launches `kernel`; with a timing record, through hipExtLaunchKernelGGL
// with the record's next event pair attached to the dispatch.
template <typename K, typename... Args>
static void launch_k(KernelTimes *kt, int kid, K kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                     Args... args)
{
    if (kt != nullptr && kt->n < kMaxTimedKernels) {
        hipExtLaunchKernelGGL(kernel, grid, block, lds, s, kt->start[kt->n], kt->stop[kt->n], 0, args...);
        kt->kid[kt->n++] = kid;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    }
}

const char *kernel_name(int kid)
{
    static const char *const names[KID_COUNT] = {"k_spread32", "k_spread64", "k_fft_single", "k_fft_stageA",
                                                 "k_fft_stageB", "k_interp32", "k_interp64", "k_sinc_mid", "k_premerge"};
    return kid >= 0 && kid < KID_COUNT ? names[kid] : "?";
}

int kernel_stage(int kid)
{
    switch (kid) {
    case KID_SPREAD32:
    case KID_SPREAD64: return 0;
    case KID_INTERP32:
    case KID_INTERP64: return 2;
    default: return 1;
    }
}

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cxmk(T a, T b)
{
    cx<T> r;
    r.re = a;
    r.im = b;
    return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return cxmk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return cxmk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return cxmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cx<T> scal(cx<T> a, T s) { return cxmk(a.re * s, a.im * s); }
// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return cxmk(a.im, -a.re); }

// Error-free sum: s + e == a + b exactly (Knuth's two-sum).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}
// (hi, lo) += x with the rounding error of hi + x kept in lo
__device__ __forceinline__ void comp_add(float &hi, float &lo, float x)
{
    float s, e;
    two_sum(hi, x, s, e);
    hi = s;
    lo += e;
}

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (__syncthreads also waits for those).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Partial windows of the spreading step.  A plane stores its cells in slot
// order slot(c) = (c mod T) P + c div T (T: the first four-step factor n1 of
// the plan's FFT, or 1; P = ceil(G1 / T)), so that the cells one four-step
// column reads (one residue mod n1) are contiguous.  Chunk.part_off < 0:
// the window lies in plane -part_off - 1; else it is the overflow window at
// partial index part_off (cells contiguous).
__device__ __forceinline__ int cell_slot(int c, int T, int P)
{
    if (T == 1) return c;
    if ((T & (T - 1)) == 0) {   // power of two (the usual four-step factor): shifts
        const int sh = __builtin_ctz((unsigned)T);
        return (c & (T - 1)) * P + (c >> sh);
    }
    return (c % T) * P + c / T;
}

__device__ __forceinline__ int window_index(const Chunk &ch, int wc, int m, int T, int P)
{
    if (ch.part_off >= 0) return ch.part_off + wc;
    return (-ch.part_off - 1) * (T * P) + cell_slot(ch.bin_lo - m + 1 + wc, T, P);
}

// sinh window of Example 2.1 in FP64:
//   sinh(beta s)/sinh(beta) = (e^{beta(s-1)} - e^{-beta(s+1)}) / (1 - e^{-2 beta});
// the second term is e^{-2 beta s} times the first and is below FP64 rounding
// (e^{-40} < 5e-18) once 2 beta s > 40, where it is skipped
__device__ __forceinline__ double omega64(double u, double beta, double inv_den)
{
    const double q = (1.0 - u) * (1.0 + u);
    if (!(q > 0.0)) return 0.0;
    const double s = sqrt(q);
    double v = exp(beta * (s - 1.0));
    if (2.0 * beta * s <= 40.0) v -= exp(-beta * (s + 1.0));
    return v * inv_den;
}

// Chebyshev series sum_k c_k T_k(t) by Clenshaw's recurrence, FP64
__device__ __forceinline__ double cheb64(const double *__restrict__ c, int deg, double t)
{
    double b1 = 0.0, b2 = 0.0;
    const double t2 = t + t;
    for (int k = deg; k >= 1; --k) {
        const double b0 = fma(t2, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(t, b1, c[0] - b2);
}

// Weight of tap r (0 <= r < 2m) of a point at offset x in [0, 1) of its cell
// in the FP64 kernels: omega(u) with u = (r - m + 1 - x) / m (the caller may
// pass -u: every window is even), for the window families of Example 2.1:
//   sinh       exp form above;
//   B-spline   tap r is one polynomial piece of degree 2m - 1 in x, stored as
//              its exact Chebyshev series in 2x - 1 (T: [2m][2m]);
//   algebraic  (1 - u^2)^(beta - 1/2) = q^(beta - 1) sqrt(q), beta = 3m integer;
//   Kaiser-Bessel  (I_0(beta sqrt(q)) - 1) / (I_0(beta) - 1) = sum_k T[k] q^(k+1),
//              q = 1 - u^2, by Horner's rule (nser positive terms).
template <int WIN>
__device__ __forceinline__ double tap64(const double *__restrict__ T, int r, int m, double x, double u, double beta,
                                        double inv_den, int nser)
{
    if constexpr (WIN == NNFFT_WINDOW_BSPLINE) return cheb64(T + r * 2 * m, 2 * m - 1, fma(2.0, x, -1.0));
    if constexpr (WIN == NNFFT_WINDOW_KAISER_BESSEL) {
        const double q = (1.0 - u) * (1.0 + u);
        if (!(q > 0.0)) return 0.0;
        double acc = T[nser - 1];
        for (int k = nser - 2; k >= 0; --k) acc = fma(acc, q, T[k]);
        return acc * q;
    }
    if constexpr (WIN == NNFFT_WINDOW_ALGEBRAIC) {
        const double q = (1.0 - u) * (1.0 + u);
        if (!(q > 0.0)) return 0.0;
        double p = 1.0, b = q;
        for (int e = (int)beta - 1; e > 0; e >>= 1) {
            if (e & 1) p *= b;
            b *= b;
        }
        return p * sqrt(q);
    }
    return omega64(u, beta, inv_den);
}

// 1/phi_hat_1(N* x_j) from its FP64 Chebyshev series in t = 8 x^2 - 1, with
// x_j reconstructed in FP64 from the bin label and the cell offset.
template <int CD>
__device__ __forceinline__ double inv_phi1_fixed(const double *__restrict__ c, double u_to_x, int lab,
                                                 double fr)
{
    const double x = ((double)lab + fr) * u_to_x;
    const double t = fma(8.0 * x, x, -1.0);
    const double t2 = t + t;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = CD; k >= 1; --k) {
        const double b0 = fma(t2, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(t, b1, c[0] - b2);
}

// Coefficient k of the spreading input, times w[k] when weights are given
// (the fast sinc transform's quadrature weights, step 2 of its Algorithm 6.1,
// folded into the load: the same products in the same precision as a
// separate scaling pass, in FP64 and rounded once).
// Output s (a label, |s| <= N2/2) of the length-N2 transform whose second
// four-step stage is folded into the interpolation: with k = s mod N2 =
// k2 + n2 k1, h_s = sum_{j1 < n1} Y[k2 n1 + j1] exp(-2 pi i j1 k1 / n1), Y the
// first stage's output (its row k2 is contiguous).
// The sum is evaluated by Horner's rule in w = exp(-2 pi i k1 / n1) (one
// twiddle; the row is read with 16-byte loads).
template <typename T, int N1>
__device__ __forceinline__ cx<T> folded_row(const cx<T> *__restrict__ row, cx<T> w)
{
    cx<T> y[N1];
    if constexpr (sizeof(T) == 4) {
        const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll
        for (int j = 0; j < N1 / 2; ++j) {
            const float4 v = r4[j];
            y[2 * j] = cxmk(v.x, v.y);
            y[2 * j + 1] = cxmk(v.z, v.w);
        }
    } else {
#pragma unroll
        for (int j = 0; j < N1; ++j) y[j] = row[j];
    }
    cx<T> acc = y[N1 - 1];
#pragma unroll
    for (int j = N1 - 2; j >= 0; --j) acc = cmul(acc, w) + y[j];
    return acc;
}

// The same sum from a row already loaded as 8 float4 (FP32, n1 = 16)
__device__ __forceinline__ cx<float> horner16(const float4 (&r4)[8], cx<float> w)
{
    cx<float> acc = cxmk(r4[7].z, r4[7].w);
    acc = cmul(acc, w) + cxmk(r4[7].x, r4[7].y);
#pragma unroll
    for (int j = 6; j >= 0; --j) {
        acc = cmul(acc, w) + cxmk(r4[j].z, r4[j].w);
        acc = cmul(acc, w) + cxmk(r4[j].x, r4[j].y);
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ cx<T> folded_output(const InterpArgs &A, int s)
{
    const int n1 = A.fusedB, n2 = A.fn2, N2 = A.N2;
    const int k = s < 0 ? s + N2 : s;
    const int k1 = k / n2, k2 = k - k1 * n2;
    const cx<T> *__restrict__ row = reinterpret_cast<const cx<T> *>(A.Y) + (size_t)k2 * n1;
    const cx<T> w = reinterpret_cast<const cx<T> *>(A.twB)[k1];
    if (n1 == 16) return folded_row<T, 16>(row, w);
    cx<T> acc = row[n1 - 1];
    for (int j = n1 - 2; j >= 0; --j) acc = cmul(acc, w) + row[j];
    return acc;
}

__device__ __forceinline__ cx<float> coef32(const cx<float> *__restrict__ f, const double *__restrict__ w, int k)
{
    const cx<float> v = f[k];
    if (w == nullptr) return v;
    const double s = w[k];
    return cxmk((float)((double)v.re * s), (float)((double)v.im * s));
}

__device__ __forceinline__ cx<double> coef64(const cx<double> *__restrict__ f, const double *__restrict__ w, int k)
{
    const cx<double> v = f[k];
    return w == nullptr ? v : scal(v, w[k]);
}

// ===========================================================================
// Spreading, FP32 path
// ===========================================================================
// FP32 spreading and interpolation run four wavefronts per 64-item chunk: each
// wave takes a quarter of every item's points, so a CU holds four times as
// many waves as chunks and hides the latency of the loads and of the
// dependent FMA chains.
constexpr int kWaves32 = 4;
constexpr int kThreads32 = kWaves32 * kItemsPerWg;
constexpr int kRowsPerWave = 8;   // record rows a wave loads in one batch
// Interpolation of items of at most 4 kWaves32 = 16 points (at most 4 rows
// per wave) loads 4 rows per batch: every load is a row the wave uses.  (The
// same change in spreading measured 0.3 us slower, so spreading keeps 8.)
constexpr int kRowsShort = 4;
constexpr int kSerialRun = 8;     // bins of up to this many items in a chunk are summed in order

// Record row for the j-th load of a wave that owns rows [row0, row0 + rpw):
// loads past its share repeat its last row (same addresses, no extra lines).
__device__ __forceinline__ int wave_row(int row0, int j, int rpw, int rows)
{
    return min(row0 + min(j, rpw - 1), rows - 1);
}

// LDS arrays are indexed [moment or tap][item or bin] so that the lanes of a
// wave (consecutive items or bins) touch consecutive 8-byte words: no bank
// conflicts in any phase.
template <int TM>   // TM >= 2 m, a multiple of kWaves32
struct Spread32Cells {
    static_assert(TM % kWaves32 == 0, "taps are split evenly over the waves");
    cx<float> sbin[TM][kItemsPerWg];               // 2m taps of each bin (B2, C)
    double cre[kWaves32][kItemsPerWg + TM];        // wave w's FP64 sum of taps r = w mod 4 of each cell (C)
    double cim[kWaves32][kItemsPerWg + TM];
};
template <int TM>
struct Spread32Lds {
    union {
        cx<float> mom[kWaves32][kDeg + 1][kItemsPerWg];   // each wave's share of the item moments (A, B1)
        Spread32Cells<TM> cs;                             // (B2, C)
    };
    cx<float> bmom[kDeg + 1][kItemsPerWg];                // moments of each bin
    float C[TM * (kDeg + 1)];                         // tap coefficients
    int ibin[kItemsPerWg];
    int runS[kItemsPerWg];
    int runE[kItemsPerWg];
};

// Copies the [2m][kDeg + 1] tap coefficients into LDS.
__device__ __forceinline__ void stage_taps(float *dst, const float *__restrict__ src, int tm)
{
    for (int i = threadIdx.x; i < tm * (kDeg + 1); i += blockDim.x) dst[i] = src[i];
}

// Chebyshev moments mu_k += f * T_k(y), k = 0..kDeg
__device__ __forceinline__ void add_moments(float *mr, float *mi, cx<float> fv, float y)
{
    constexpr int D = kDeg;
    const float y2 = y + y;
    float T0 = 1.f, T1 = y;
    mr[0] += fv.re;
    mi[0] += fv.im;
    mr[1] = fmaf(fv.re, y, mr[1]);
    mi[1] = fmaf(fv.im, y, mi[1]);
#pragma unroll
    for (int k = 2; k <= D; ++k) {
        const float T2 = fmaf(y2, T1, -T0);
        mr[k] = fmaf(fv.re, T2, mr[k]);
        mi[k] = fmaf(fv.im, T2, mi[k]);
        T0 = T1;
        T1 = T2;
    }
}

// One chunk of up to 64 items (4 waves, lane t = item t):
//  A: wave w accumulates the Chebyshev moments of its rows of each item
//     (record loads and coefficient gathers first, then the arithmetic);
//  B1: thread (w, bin) forms the bin moments M_k, k = w, w + 4, w + 8: the
//     item moment is the plain sum of the four wave shares, items of a bin are
//     added with two-sum;
//  B2: thread (w, bin) forms taps r = w, w + 4, ...: sum_k C[r][k] M_k;
//  C: window cell c (grid cell bin_lo - m + 1 + c) = sum over r of tap r of
//     bin c - r in FP64, stored as the FP32 pair (hi.re, hi.im, lo.re, lo.im).
// (All of a workgroup's loads are issued before any arithmetic; the kernel
// is VALU- and latency-bound, one chunk per workgroup with all chunks
// resident at once: a persistent variant that prefetched the next chunk
// during the LDS phases measured 2.4x slower.)

// per-thread registers of a chunk's loads: this wave's record rows of item
// t, the item, and the gathered coefficients of the rows that hold points
struct Spread32Regs {
    PtRec r[kRowsPerWave];
    cx<float> fv[kRowsPerWave];
    Item it;
};

__device__ __forceinline__ void spread32_load_records(const SpreadArgs &A, int g, Spread32Regs &R)
{
    const int t = threadIdx.x & (kItemsPerWg - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kItemsPerWg);
    const int rows = A.rows, rpw = (rows + kWaves32 - 1) / kWaves32, row0 = w * rpw;
    const PtRec *__restrict__ rec = A.rec32 + (size_t)g * rows * kItemsPerWg + t;
    // every row load is issued unconditionally (rows past the wave's share
    // repeat its last row: same lines): under a branch per row the compiler
    // completes each load before issuing the next
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j) R.r[j] = rec[wave_row(row0, j, rpw, rows) * kItemsPerWg];
    R.it = A.items[g * kItemsPerWg + t];
}

// rows past an item's end repeat its last record and are not gathered
__device__ __forceinline__ void spread32_gather(const SpreadArgs &A, const cx<float> *__restrict__ f,
                                                Spread32Regs &R)
{
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kItemsPerWg);
    const int rows = A.rows, rpw = (rows + kWaves32 - 1) / kWaves32, row0 = w * rpw;
#pragma unroll
    for (int j = 0; j < kRowsPerWave; ++j)
        R.fv[j] = (j < rpw && row0 + j < R.it.n) ? coef32(f, A.wts, R.r[j].perm) : cxmk(0.f, 0.f);
}

// Phase A arithmetic: this wave's item moments into LDS (and the item's bin);
// the run bounds of the bins are cleared.  Rows past the first batch of
// kRowsPerWave (items longer than 4 kRowsPerWave points) are loaded here.
template <int TM>
__device__ __forceinline__ void spread32_moments(const SpreadArgs &A, const cx<float> *__restrict__ f, int g,
                                                 const Chunk &ch, Spread32Regs &R, Spread32Lds<TM> &L)
{
    constexpr int D = kDeg;
    const int t = threadIdx.x & (kItemsPerWg - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kItemsPerWg);
    const int rows = A.rows, rpw = (rows + kWaves32 - 1) / kWaves32, row0 = w * rpw;
    const PtRec *__restrict__ rec = A.rec32 + (size_t)g * rows * kItemsPerWg + t;
    if (w == 0 && t < ch.nbin) {   // empty run unless an item of the bin sets it
        L.runS[t] = 0;
        L.runE[t] = 0;
    }
    float mr[D + 1], mi[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) mr[k] = mi[k] = 0.f;
    const int nq = min(rpw, R.it.n - row0);   // this wave's points of the item
    for (int j0 = 0; j0 < nq; j0 += kRowsPerWave) {
        if (j0 > 0) {
#pragma unroll
            for (int j = 0; j < kRowsPerWave; ++j) R.r[j] = rec[wave_row(row0, j0 + j, rpw, rows) * kItemsPerWg];
#pragma unroll
            for (int j = 0; j < kRowsPerWave; ++j)
                R.fv[j] = (j0 + j < nq) ? coef32(f, A.wts, R.r[j].perm) : cxmk(0.f, 0.f);
        }
#pragma unroll
        for (int j = 0; j < kRowsPerWave; ++j)
            if (j0 + j < nq) add_moments(mr, mi, R.fv[j], fmaf(2.f, R.r[j].frac, -1.f));
    }
#pragma unroll
    for (int k = 0; k <= D; ++k) L.mom[w][k][t] = cxmk(mr[k], mi[k]);
    if (w == 0 && R.it.n > 0) L.ibin[t] = R.it.bin - ch.bin_lo;
}

// Phases B1, B2, C: bin moments, taps, window cells (the tap coefficients
// are in L.C).  Barriers order LDS only, so loads issued before stay in
// flight.
template <int TM>
__device__ __forceinline__ void spread32_cells(const SpreadArgs &A, const Chunk &ch, int run, Spread32Lds<TM> &L)
{
    constexpr int D = kDeg;
    const int t = threadIdx.x & (kItemsPerWg - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kItemsPerWg);
    const int m = A.m, tm = 2 * m;
    lds_barrier();
    if (w == 0 && t < ch.nitem) {
        const int b = L.ibin[t];
        if (t == 0 || L.ibin[t - 1] != b) L.runS[b] = t;
        if (t == ch.nitem - 1 || L.ibin[t + 1] != b) L.runE[b] = t + 1;
    }
    lds_barrier();
    constexpr int KW = (D + kWaves32) / kWaves32;   // moments per wave (3; the last one only on wave 0)
    if (run <= kSerialRun) {
        // short runs: thread (w, bin) adds the bin's items in order
        if (t < ch.nbin) {
            const int s = L.runS[t], e = L.runE[t];   // s = e for a bin without items
            float hr[KW], hi[KW], lr[KW], li[KW];
#pragma unroll
            for (int j = 0; j < KW; ++j) hr[j] = hi[j] = lr[j] = li[j] = 0.f;
            for (int i = s; i < e; ++i) {
#pragma unroll
                for (int j = 0; j < KW; ++j) {
                    const int k = min(w + kWaves32 * j, D);
                    cx<float> v = L.mom[0][k][i];
#pragma unroll
                    for (int ww = 1; ww < kWaves32; ++ww) {
                        v.re += L.mom[ww][k][i].re;
                        v.im += L.mom[ww][k][i].im;
                    }
                    comp_add(hr[j], lr[j], v.re);
                    comp_add(hi[j], li[j], v.im);
                }
            }
#pragma unroll
            for (int j = 0; j < KW; ++j)
                if (w + kWaves32 * j <= D) L.bmom[w + kWaves32 * j][t] = cxmk(hr[j] + lr[j], hi[j] + li[j]);
        }
    } else {
        // long runs (crowded cells): a tree over each run.  Thread (w, item)
        // owns moments k = w + 4 j of its item: the item total (plain sum of
        // the wave shares, as above) becomes the pair (mom[0], mom[1]) =
        // (hi, lo); in round d the item at run offset r = 0 mod 2d adds the
        // pair at r + d with two-sum; the run's first item ends with the sum.
        if (t < ch.nitem) {
#pragma unroll
            for (int j = 0; j < KW; ++j) {
                const int k = w + kWaves32 * j;
                if (k <= D) {
                    cx<float> v = L.mom[0][k][t];
#pragma unroll
                    for (int ww = 1; ww < kWaves32; ++ww) {
                        v.re += L.mom[ww][k][t].re;
                        v.im += L.mom[ww][k][t].im;
                    }
                    L.mom[0][k][t] = v;
                    L.mom[1][k][t] = cxmk(0.f, 0.f);
                }
            }
        }
        lds_barrier();
        const int bt = (t < ch.nitem) ? L.ibin[t] : 0;
        const int r = t - L.runS[bt], len = L.runE[bt] - L.runS[bt];
        for (int d = 1; d < run; d <<= 1) {
            if (t < ch.nitem && (r & (2 * d - 1)) == 0 && r + d < len) {
#pragma unroll
                for (int j = 0; j < KW; ++j) {
                    const int k = w + kWaves32 * j;
                    if (k <= D) {
                        cx<float> h = L.mom[0][k][t], l = L.mom[1][k][t];
                        const cx<float> h2 = L.mom[0][k][t + d], l2 = L.mom[1][k][t + d];
                        float sr, er, si, ei;
                        two_sum(h.re, h2.re, sr, er);
                        two_sum(h.im, h2.im, si, ei);
                        L.mom[0][k][t] = cxmk(sr, si);
                        L.mom[1][k][t] = cxmk(l.re + l2.re + er, l.im + l2.im + ei);
                    }
                }
            }
            lds_barrier();
        }
        if (t < ch.nbin) {
            const int s0 = L.runS[t], e0 = L.runE[t];
#pragma unroll
            for (int j = 0; j < KW; ++j) {
                const int k = w + kWaves32 * j;
                if (k <= D) {
                    cx<float> v = cxmk(0.f, 0.f);
                    if (s0 < e0) {
                        const cx<float> h = L.mom[0][k][s0], l = L.mom[1][k][s0];
                        v = cxmk(h.re + l.re, h.im + l.im);
                    }
                    L.bmom[k][t] = v;
                }
            }
        }
    }
    lds_barrier();
    if (t < ch.nbin) {
        float Mr[D + 1], Mi[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            const cx<float> v = L.bmom[k][t];
            Mr[k] = v.re;
            Mi[k] = v.im;
        }
        for (int r0 = w; r0 < tm; r0 += kWaves32) {
            const float *c = L.C + r0 * (D + 1);
            float ar = 0.f, ai = 0.f;
#pragma unroll
            for (int k = 0; k <= D; ++k) {
                ar = fmaf(c[k], Mr[k], ar);
                ai = fmaf(c[k], Mi[k], ai);
            }
            L.cs.sbin[r0][t] = cxmk(ar, ai);
        }
    }
    lds_barrier();
    // C1: wave w adds taps r = w, w + 4, ... of every cell in FP64
    const int W = ch.nbin + tm - 1;   // <= kItemsPerWg + TM - 1
    for (int wc = t; wc < W; wc += kItemsPerWg) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int j = 0; j < TM / kWaves32; ++j) {
            const int rr = w + kWaves32 * j, b = wc - rr;
            const cx<float> v = L.cs.sbin[rr][min(max(b, 0), ch.nbin - 1)];
            if (rr < tm && b >= 0 && b < ch.nbin) {
                sr += (double)v.re;
                si += (double)v.im;
            }
        }
        L.cs.cre[w][wc] = sr;
        L.cs.cim[w][wc] = si;
    }
    lds_barrier();
    // C2: the cell's four partial sums added in FP64 (exact for FP32 taps of
    // similar size, far below FP32 rounding otherwise), then split into the
    // (hi, lo) FP32 pair the merge adds with two-sum
    float4 *part = reinterpret_cast<float4 *>(A.partial);
    for (int wc = threadIdx.x; wc < W; wc += blockDim.x) {
        const double sr = ((L.cs.cre[0][wc] + L.cs.cre[1][wc]) + L.cs.cre[2][wc]) + L.cs.cre[3][wc];
        const double si = ((L.cs.cim[0][wc] + L.cs.cim[1][wc]) + L.cs.cim[2][wc]) + L.cs.cim[3][wc];
        const float hr = (float)sr, hi = (float)si;
        part[window_index(ch, wc, m, A.slotT, A.slotP)] =
            make_float4(hr, hi, (float)(sr - (double)hr), (float)(si - (double)hi));
    }
}

// One chunk, one workgroup (the batched kernel's body)
template <int TM>
__device__ void spread32_slot(const SpreadArgs &A, const cx<float> *__restrict__ f, int g, Spread32Lds<TM> &L)
{
    Spread32Regs R;
    spread32_load_records(A, g, R);
    spread32_gather(A, f, R);
    const Chunk ch = A.chunks[g];
    if (ch.nitem == 0) return;
    stage_taps(L.C, A.C, 2 * A.m);   // read after the barriers below
    spread32_moments<TM>(A, f, g, ch, R, L);
    // the chunk's longest bin run, from its first item (lane 0 of every wave)
    const int run = __builtin_amdgcn_readfirstlane(R.it.maxrun);
    spread32_cells<TM>(A, ch, run, L);
}

// One workgroup per launch slot (slot g runs on XCD g mod 8).  At least 6
// waves per SIMD for short windows: then 1536 workgroups are resident at once.
template <int TM>
__global__ __launch_bounds__(kThreads32, TM <= 16 ? 6 : 4) void k_spread32(SpreadArgs A,
                                                                        const cx<float> *__restrict__ f)
{
    __shared__ Spread32Lds<TM> L;
    spread32_slot<TM>(A, f, blockIdx.x, L);
}

// ===========================================================================
// Spreading, FP64 plain path (items of up to Q64 points)
// ===========================================================================
constexpr int Q64 = 8;
constexpr int kWaves64 = 4;                          // waves per FP64 workgroup
constexpr int kThreads64 = kWaves64 * kItemsPerWg;

// LDS of the FP64 spreading kernel, sized at launch for the plan's 2m taps and
// item size (dynamic shared memory), so that short windows and small items
// leave room for more workgroups per CU.
struct Spread64Lds {
    cx<double> *sitem;   // [2m][64]: tap r of item t at r * 64 + t
    cx<double> *pv;      // [rows][64]: coefficient of point q of item t at q * 64 + t
    double *pf;          // [rows][64]: its cell offset
    int *ibin, *runS, *runE;
};

__device__ __forceinline__ Spread64Lds spread64_lds(int tm, int rows)
{
    extern __shared__ __align__(16) char smem[];
    Spread64Lds L;
    L.sitem = reinterpret_cast<cx<double> *>(smem);
    L.pv = L.sitem + (size_t)tm * kItemsPerWg;
    L.pf = reinterpret_cast<double *>(L.pv + (size_t)rows * kItemsPerWg);
    int *ip = reinterpret_cast<int *>(L.pf + (size_t)rows * kItemsPerWg);
    L.ibin = ip;
    L.runS = ip + kItemsPerWg;
    L.runE = ip + 2 * kItemsPerWg;
    return L;
}

static size_t lds64_bytes(int tm, int rows)
{
    return ((size_t)tm + rows) * kItemsPerWg * sizeof(cx<double>) + (size_t)rows * kItemsPerWg * sizeof(double) +
           3 * kItemsPerWg * sizeof(int);
}

// Four waves per chunk: lane t of every wave holds item t.  Wave w loads the
// points q = w, w + 4 of the item (each point once) into LDS; then wave w
// forms the taps r = w, w + 4, ... of the item over all its points
// (disjoint outputs, no reduction).
template <int WIN>
__device__ void spread64_slot(const SpreadArgs &A, const cx<double> *__restrict__ f, int g, Spread64Lds &L)
{
    constexpr int QW = Q64 / kWaves64;   // points of an item one wave loads
    const int t = threadIdx.x & (kItemsPerWg - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kItemsPerWg);
    const Item it = A.items[g * kItemsPerWg + t];
    const Chunk ch = A.chunks[g];
    if (ch.nitem == 0) return;
    const int m = A.m, tm = 2 * m, rows = A.rows;   // rows <= Q64
    if (wv == 0 && t < ch.nbin) {
        L.runS[t] = -1;
        L.runE[t] = 0;
    }
    {
        int pm[QW];
        double xl[QW];
        cx<double> fl[QW];
#pragma unroll
        for (int j = 0; j < QW; ++j) {
            const int q = wv + kWaves64 * j;
            const int p = it.p0 + (q < it.n ? q : 0);
            pm[j] = (q < it.n) ? A.perm[p] : -1;
            xl[j] = (q < it.n) ? A.frac64[p] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < QW; ++j) fl[j] = pm[j] >= 0 ? coef64(f, A.wts, pm[j]) : cxmk(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < QW; ++j) {
            const int q = wv + kWaves64 * j;
            if (q < rows) {
                L.pv[q * kItemsPerWg + t] = fl[j];
                L.pf[q * kItemsPerWg + t] = xl[j];
            }
        }
    }
    __syncthreads();
    if (it.n > 0) {
        // the points are read from LDS per tap (it.n <= rows), not held in
        // registers: the kernel then fits twice the waves per SIMD
        const double inv_m = 1.0 / (double)m;
        for (int r = wv; r < tm; r += kWaves64) {
            double ar = 0.0, ai = 0.0;
            for (int q = 0; q < it.n; ++q) {
                const double xq = L.pf[q * kItemsPerWg + t];
                const cx<double> fq = L.pv[q * kItemsPerWg + t];
                const double w = tap64<WIN>(A.T64, r, m, xq, ((double)(r - m + 1) - xq) * inv_m, A.beta,
                                            A.inv_den, A.nser);
                ar = fma(fq.re, w, ar);
                ai = fma(fq.im, w, ai);
            }
            L.sitem[r * kItemsPerWg + t] = cxmk(ar, ai);
        }
        if (wv == 0) L.ibin[t] = it.bin - ch.bin_lo;
    }
    __syncthreads();
    if (wv == 0 && t < ch.nitem) {
        const int b = L.ibin[t];
        if (t == 0 || L.ibin[t - 1] != b) L.runS[b] = t;
        if (t == ch.nitem - 1 || L.ibin[t + 1] != b) L.runE[b] = t + 1;
    }
    __syncthreads();
    const int W = ch.nbin + tm - 1;
    double2 *part = reinterpret_cast<double2 *>(A.partial);
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        const int blo = max(0, w - tm + 1), bhi = min(ch.nbin - 1, w);
        double ar = 0.0, ai = 0.0;
        for (int b = blo; b <= bhi; ++b) {
            const int s = L.runS[b];
            if (s < 0) continue;
            const int e = L.runE[b];
            for (int i = s; i < e; ++i) {
                const cx<double> v = L.sitem[(w - b) * kItemsPerWg + i];
                ar += v.re;
                ai += v.im;
            }
        }
        part[window_index(ch, w, m, A.slotT, A.slotP)] = make_double2(ar, ai);
    }
}

// WIN: the plan's window family (one instantiation per family keeps the
// sinh kernel's registers at what the sinh taps need)
template <int WIN>
__global__ __launch_bounds__(kThreads64) void k_spread64(SpreadArgs A, const cx<double> *__restrict__ f)
{
    Spread64Lds L = spread64_lds(2 * A.m, A.rows);
    spread64_slot<WIN>(A, f, blockIdx.x, L);
}

// ===========================================================================
// Interpolation
// ===========================================================================
// Four waves per chunk of 64 items (lane t = item t).  The item's bin
// coefficients H_k = sum_r C[r][k] h_{c - m + 1 + r} (the transpose of the
// spreading taps) are formed by wave w for k = w, w + 4, w + 8 and shared in
// LDS; then wave w evaluates y_j = (sum_k H_k T_k(t_j)) / phi_hat_1(N* x_j)
// for its rows of the item's points.
struct Interp32Lds {
    cx<float> H[kDeg + 1][kItemsPerWg];
    cx<float> hw[kItemsPerWg + 2 * kMaxM - 1];   // the chunk's h_s window
    float C[2 * kMaxM * (kDeg + 1)];             // tap series [2m][kDeg + 1]
};

template <int CD, int RB>
__device__ __forceinline__ void interp32_slot(const InterpArgs &A, cx<float> *__restrict__ y, int g,
                                              Interp32Lds &L)
{
    constexpr int D = kDeg;
    // the wave index, known to the compiler as wave-uniform (scalar branches)
    const int t = threadIdx.x & (kItemsPerWg - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kItemsPerWg);
    const int rows = A.rows, rpw = (rows + kWaves32 - 1) / kWaves32, row0 = w * rpw;
    const Chunk ch = A.chunks[g];   // one scalar load; its window loads go out first
    if (ch.nitem == 0) return;
    const int m = A.m, tm = 2 * m;
    // the h_s the chunk's items read (labels bin_lo - m + 1 .. bin_lo + nbin + m - 1
    // after the offset) and the tap series, staged in LDS; the record rows and
    // the item follow in the same round of loads
    // (nwin < 64 + 2m <= kThreads32; the series has up to 2 kThreads32 entries)
    // Loads in the order they are needed (the memory counter completes them
    // in issue order): the window values' data, the tap series and the item,
    // then the record rows (unconditional, as in spreading), which stay in
    // flight across the LDS barrier below.  A folded window value is formed
    // from its row only after the record rows are issued.
    const int nwin = ch.nbin + tm - 1, nc = tm * (D + 1);
    // (the FP32 fold has n1 = 16; the loads of both forms go to registers
    // of their own, so that neither waits for the other's)
    const int sw = ch.bin_lo - A.ip_off - m + 1 + min((int)threadIdx.x, nwin - 1);   // label of window value
    float4 wrow[8];
    cx<float> wtw, hv;
    if (A.fusedB) {
        const int k = sw < 0 ? sw + A.N2 : sw;
        const int k1 = k / A.fn2, k2 = k - k1 * A.fn2;
        const float4 *row = reinterpret_cast<const float4 *>(reinterpret_cast<const cx<float> *>(A.Y) + (size_t)k2 * 16);
#pragma unroll
        for (int j = 0; j < 8; ++j) wrow[j] = row[j];
        wtw = reinterpret_cast<const cx<float> *>(A.twB)[k1];
    } else {
        hv = reinterpret_cast<const cx<float> *>(A.hlin)[sw + A.h_off];
    }
    const float c0 = A.C[min((int)threadIdx.x, nc - 1)];
    const float c1 = A.C[min((int)threadIdx.x + kThreads32, nc - 1)];
    const Item it = A.items[g * kItemsPerWg + t];
    const PtRec *__restrict__ rec = A.rec32 + (size_t)g * rows * kItemsPerWg + t;
    PtRec r[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) r[j] = rec[wave_row(row0, j, rpw, rows) * kItemsPerWg];
    cx<float> hw0;
    if (A.fusedB) hw0 = horner16(wrow, wtw);
    else hw0 = hv;
    const int lab = it.bin - A.ip_off;
    if (threadIdx.x < nwin) L.hw[threadIdx.x] = hw0;
    if (threadIdx.x < nc) L.C[threadIdx.x] = c0;
    if (threadIdx.x + kThreads32 < nc) L.C[threadIdx.x + kThreads32] = c1;
    lds_barrier();   // the record rows stay in flight
    if (it.n > 0) {
        const cx<float> *h = L.hw + (it.bin - ch.bin_lo);
        constexpr int KW = (D + kWaves32) / kWaves32;   // moments per wave (3)
        float ar[KW], ai[KW];
#pragma unroll
        for (int j = 0; j < KW; ++j) ar[j] = ai[j] = 0.f;
        // straight-line body: moments past D (only j = KW - 1 on some waves)
        // read a valid coefficient and are dropped below
#pragma unroll 4
        for (int rr = 0; rr < tm; ++rr) {
            const cx<float> hv = h[rr];
#pragma unroll
            for (int j = 0; j < KW; ++j) {
                const float c = L.C[rr * (D + 1) + min(w + kWaves32 * j, D)];
                ar[j] = fmaf(c, hv.re, ar[j]);
                ai[j] = fmaf(c, hv.im, ai[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            const int k = w + kWaves32 * j;
            if (k <= D) L.H[k][t] = cxmk(ar[j], ai[j]);
        }
    }
    lds_barrier();
    if (it.n > 0) {
        float Hr[D + 1], Hi[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            const cx<float> v = L.H[k][t];
            Hr[k] = v.re;
            Hi[k] = v.im;
        }
        double c[CD + 1];
#pragma unroll
        for (int k = 0; k <= CD; ++k) c[k] = A.corr[k];
        const int nq = min(rpw, it.n - row0);
        for (int j0 = 0; j0 < nq; j0 += RB) {
            if (j0 > 0) {
#pragma unroll
                for (int j = 0; j < RB; ++j) r[j] = rec[wave_row(row0, j0 + j, rpw, rows) * kItemsPerWg];
            }
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                if (j0 + j < nq) {
                    const float yv = fmaf(2.f, r[j].frac, -1.f);
                    const float y2 = yv + yv;
                    float T0 = 1.f, T1 = yv;
                    float sr = fmaf(Hr[1], yv, Hr[0]);
                    float si = fmaf(Hi[1], yv, Hi[0]);
#pragma unroll
                    for (int k = 2; k <= D; ++k) {
                        const float T2 = fmaf(y2, T1, -T0);
                        sr = fmaf(Hr[k], T2, sr);
                        si = fmaf(Hi[k], T2, si);
                        T0 = T1;
                        T1 = T2;
                    }
                    const double corr = inv_phi1_fixed<CD>(c, A.u_to_x, lab, (double)r[j].frac);
                    y[r[j].perm] = cxmk((float)((double)sr * corr), (float)((double)si * corr));
                }
            }
        }
    }
}

// CD: degree of the 1/phi_hat_1 series as evaluated (the plan's series
// zero-padded to CD; leading zero terms leave the result bit for bit unchanged);
// RB: record rows per load batch
template <int CD, int RB>
__global__ __launch_bounds__(kThreads32) void k_interp32(InterpArgs A, cx<float> *__restrict__ y)
{
    __shared__ Interp32Lds L;
    interp32_slot<CD, RB>(A, y, blockIdx.x, L);
}

struct Interp64Lds {
    cx<double> *hw;   // the chunk's window: h at labels bin_lo - ip_off - m + 1 + i
};

__device__ __forceinline__ Interp64Lds interp64_lds()
{
    extern __shared__ __align__(16) char smem[];
    Interp64Lds L;
    L.hw = reinterpret_cast<cx<double> *>(smem);
    return L;
}

// the window holds nbin + 2m - 1 < 64 + 2m values
static size_t interp64_lds_bytes(int tm)
{
    return ((size_t)kItemsPerWg + tm) * sizeof(cx<double>);
}

// Four waves per chunk: lane t of every wave holds item t; wave w computes
// the points p0 + w, p0 + w + 4, ... of the item.  The chunk's h window
// (< 64 + 2m values) is staged in LDS with one round of loads.
template <int WIN>
__device__ void interp64_slot(const InterpArgs &A, cx<double> *__restrict__ y, int g, Interp64Lds &L)
{
    const int t = threadIdx.x & (kItemsPerWg - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kItemsPerWg);
    const Chunk ch = A.chunks[g];
    if (ch.nitem == 0) return;
    const int m = A.m, tm = 2 * m;
    const int nwin = ch.nbin + tm - 1;   // < 64 + 2m <= kThreads64
    cx<double> hv0 = cxmk(0.0, 0.0);
    if (threadIdx.x < nwin) {
        const int s = ch.bin_lo - A.ip_off - m + 1 + threadIdx.x;   // label of window value
        hv0 = A.fusedB ? folded_output<double>(A, s) : reinterpret_cast<const cx<double> *>(A.hlin)[s + A.h_off];
    }
    const Item it = A.items[g * kItemsPerWg + t];
    if (threadIdx.x < nwin) L.hw[threadIdx.x] = hv0;
    __syncthreads();
    if (it.n > 0) {
        const int b = it.bin - ch.bin_lo;
        const int lab = ch.bin_lo + b - A.ip_off;
        const double inv_m = 1.0 / (double)m;
        for (int p = it.p0 + wv; p < it.p0 + it.n; p += kWaves64) {
            const double fr = A.frac64[p];
            double sr = 0.0, si = 0.0;
            for (int r = 0; r < tm; ++r) {
                const double w = tap64<WIN>(A.T64, r, m, fr, (fr + (double)(m - 1 - r)) * inv_m, A.beta,
                                            A.inv_den, A.nser);
                const cx<double> hv = L.hw[b + r];
                sr = fma(hv.re, w, sr);
                si = fma(hv.im, w, si);
            }
            const double x = ((double)lab + fr) * A.u_to_x;
            const double corr = cheb64(A.corr, A.corr_deg, fma(8.0 * x, x, -1.0));
            y[A.perm[p]] = cxmk(sr * corr, si * corr);
        }
    }
}

template <int WIN>
__global__ __launch_bounds__(kThreads64) void k_interp64(InterpArgs A, cx<double> *__restrict__ y)
{
    Interp64Lds L = interp64_lds();
    interp64_slot<WIN>(A, y, blockIdx.x, L);
}

static void launch_spread64(const SpreadArgs &A, const void *f, hipStream_t s, KernelTimes *kt = nullptr)
{
    const cx<double> *in = reinterpret_cast<const cx<double> *>(f);
    const size_t lds = lds64_bytes(2 * A.m, A.rows);
    switch (A.window) {
    case NNFFT_WINDOW_BSPLINE:
        launch_k(kt, KID_SPREAD64, k_spread64<NNFFT_WINDOW_BSPLINE>, dim3(A.ngrid), dim3(kThreads64), lds, s, A, in);
        break;
    case NNFFT_WINDOW_ALGEBRAIC:
        launch_k(kt, KID_SPREAD64, k_spread64<NNFFT_WINDOW_ALGEBRAIC>, dim3(A.ngrid), dim3(kThreads64), lds, s, A, in);
        break;
    case NNFFT_WINDOW_KAISER_BESSEL:
        launch_k(kt, KID_SPREAD64, k_spread64<NNFFT_WINDOW_KAISER_BESSEL>, dim3(A.ngrid), dim3(kThreads64), lds, s,
                 A, in);
        break;
    default:
        launch_k(kt, KID_SPREAD64, k_spread64<NNFFT_WINDOW_SINH>, dim3(A.ngrid), dim3(kThreads64), lds, s, A, in);
        break;
    }
}

static void launch_interp64(const InterpArgs &A, void *y, hipStream_t s, KernelTimes *kt = nullptr)
{
    cx<double> *out = reinterpret_cast<cx<double> *>(y);
    const size_t lds = interp64_lds_bytes(2 * A.m);
    switch (A.window) {
    case NNFFT_WINDOW_BSPLINE:
        launch_k(kt, KID_INTERP64, k_interp64<NNFFT_WINDOW_BSPLINE>, dim3(A.ngrid), dim3(kThreads64), lds, s, A,
                 out);
        break;
    case NNFFT_WINDOW_ALGEBRAIC:
        launch_k(kt, KID_INTERP64, k_interp64<NNFFT_WINDOW_ALGEBRAIC>, dim3(A.ngrid), dim3(kThreads64), lds, s, A,
                 out);
        break;
    case NNFFT_WINDOW_KAISER_BESSEL:
        launch_k(kt, KID_INTERP64, k_interp64<NNFFT_WINDOW_KAISER_BESSEL>, dim3(A.ngrid), dim3(kThreads64), lds, s,
                 A, out);
        break;
    default:
        launch_k(kt, KID_INTERP64, k_interp64<NNFFT_WINDOW_SINH>, dim3(A.ngrid), dim3(kThreads64), lds, s, A,
                 out);
        break;
    }
}

// ===========================================================================
// FFT (steps 2-3)
// ===========================================================================

// Adds the partial sums of the grid cell at slot `slot` (its window planes,
// then the overflow windows through their index lists) to the two-sum pairs.
__device__ __forceinline__ void merge_cell32(const FftArgs &A, int slot, float &hr, float &hi, float &lr, float &li)
{
    const float4 *part = reinterpret_cast<const float4 *>(A.partial);
    const int e0 = A.merge_off[slot], e1 = A.merge_off[slot + 1];
    // the planes: fixed offsets s T P + slot, all loads in flight together
    const int np = A.nplanes, ps = A.slotT * A.slotP;
    {
        float4 v[kMaxPlanes];
#pragma unroll
        for (int q = 0; q < kMaxPlanes; ++q) v[q] = part[(size_t)min(q, np - 1) * ps + slot];
#pragma unroll
        for (int q = 0; q < kMaxPlanes; ++q) {
            if (q < np) {
                comp_add(hr, lr, v[q].x);
                comp_add(hi, li, v[q].y);
                lr += v[q].z;
                li += v[q].w;
            }
        }
    }
    // overflow windows: eight entries at a time
    for (int e = e0; e < e1; e += 8) {
        int idx[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) idx[q] = A.merge_idx[(e + q < e1) ? e + q : e0];
        float4 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = part[idx[q]];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (e + q < e1) {
                comp_add(hr, lr, v[q].x);
                comp_add(hi, li, v[q].y);
                lr += v[q].z;
                li += v[q].w;
            }
        }
    }
}

__device__ __forceinline__ void merge_cell64(const FftArgs &A, int slot, double &ar, double &ai)
{
    const double2 *part = reinterpret_cast<const double2 *>(A.partial);
    const int e1 = A.merge_off[slot + 1];
    const int np = A.nplanes, ps = A.slotT * A.slotP;
    {
        double2 v[kMaxPlanes];
#pragma unroll
        for (int q = 0; q < kMaxPlanes; ++q) v[q] = part[(size_t)min(q, np - 1) * ps + slot];
#pragma unroll
        for (int q = 0; q < kMaxPlanes; ++q) {
            if (q < np) {
                ar += v[q].x;
                ai += v[q].y;
            }
        }
    }
    // overflow windows: eight entries at a time
    const int e0 = A.merge_off[slot];
    for (int e = e0; e < e1; e += 8) {
        int idx[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) idx[q] = A.merge_idx[(e + q < e1) ? e + q : e0];
        double2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = part[idx[q]];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (e + q < e1) {
                ar += v[q].x;
                ai += v[q].y;
            }
        }
    }
}

// Pre-merge of long merge lists: one thread per segment, its entries added in
// list order with the merge's own arithmetic (two-sum pairs in FP32, plain
// sums in FP64), eight loads in flight at a time.
template <typename T>
__global__ __launch_bounds__(256) void k_premerge(PreMergeArgs A)
{
    const int sg = blockIdx.x * 256 + threadIdx.x;
    if (sg >= A.nseg) return;
    const int e0 = A.seg[2 * sg], e1 = e0 + A.seg[2 * sg + 1];
    if constexpr (sizeof(T) == 4) {
        float4 *part = reinterpret_cast<float4 *>(A.partial);
        float hr = 0.f, hi = 0.f, lr = 0.f, li = 0.f;
        for (int e = e0; e < e1; e += 8) {
            int idx[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) idx[q] = A.idx[(e + q < e1) ? e + q : e0];
            float4 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = part[idx[q]];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (e + q < e1) {
                    comp_add(hr, lr, v[q].x);
                    comp_add(hi, li, v[q].y);
                    lr += v[q].z;
                    li += v[q].w;
                }
            }
        }
        part[A.base + sg] = make_float4(hr, hi, lr, li);
    } else {
        double2 *part = reinterpret_cast<double2 *>(A.partial);
        double ar = 0.0, ai = 0.0;
        for (int e = e0; e < e1; e += 8) {
            int idx[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) idx[q] = A.idx[(e + q < e1) ? e + q : e0];
            double2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = part[idx[q]];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (e + q < e1) {
                    ar += v[q].x;
                    ai += v[q].y;
                }
            }
        }
        part[A.base + sg] = make_double2(ar, ai);
    }
}

// FFT input element q (index mod N2):
//  mode 0 (NNFFT steps 1-2): merged step-1 cell of label l = q or q - N2 (zero
//    outside I_{G1}) times 1 / (N1 N2 phi_hat_2(l)) (table in slot order);
//  mode 1 (NFFT): coefficient f_k, k = l in I_N, times 1 / (n phi_hat(k));
//  mode 2 (adjoint NFFT): conjugate of the sum of the cells of labels l, l + n,
//    l - n in the linear grid (the 1-periodic fold of the spread values);
//  mode 3 (fast sinc transform, second plan): the value the middle operator
//    wrote for label l (zero outside I_{G1}; already deconvolved).
__device__ __forceinline__ cx<float> fft_input32(const FftArgs &A, int q)
{
    const int lab = (q < A.N2 / 2) ? q : q - A.N2;
    if (A.mode == 3) {
        if (lab < -A.G1 / 2 || lab >= A.G1 / 2) return cxmk(0.f, 0.f);
        return reinterpret_cast<const cx<float> *>(A.dense_in)[lab + A.G1 / 2];
    }
    if (A.mode == 1) {
        if (lab < -A.Nout / 2 || lab >= A.Nout / 2) return cxmk(0.f, 0.f);
        const cx<float> v = reinterpret_cast<const cx<float> *>(A.dense_in)[lab + A.Nout / 2];
        const double sc = A.deconv[lab + A.Nout / 2];
        return cxmk((float)((double)v.re * sc), (float)((double)v.im * sc));
    }
    float hr = 0.f, hi = 0.f, lr = 0.f, li = 0.f;
    if (A.mode == 2) {
#pragma unroll
        for (int r = -1; r <= 1; ++r) {
            const int cell = lab + r * A.N2 + A.G1 / 2;
            if (cell >= 0 && cell < A.G1) merge_cell32(A, cell_slot(cell, A.slotT, A.slotP), hr, hi, lr, li);
        }
        return cxmk(hr + lr, -(hi + li));
    }
    if (lab < -A.G1 / 2 || lab >= A.G1 / 2) return cxmk(0.f, 0.f);
    const int slot = cell_slot(lab + A.G1 / 2, A.slotT, A.slotP);
    const double sc = A.deconv[slot];   // issued with the plane loads
    merge_cell32(A, slot, hr, hi, lr, li);
    return cxmk((float)((double)(hr + lr) * sc), (float)((double)(hi + li) * sc));
}

__device__ __forceinline__ cx<double> fft_input64(const FftArgs &A, int q)
{
    const int lab = (q < A.N2 / 2) ? q : q - A.N2;
    if (A.mode == 3) {
        if (lab < -A.G1 / 2 || lab >= A.G1 / 2) return cxmk(0.0, 0.0);
        return reinterpret_cast<const cx<double> *>(A.dense_in)[lab + A.G1 / 2];
    }
    if (A.mode == 1) {
        if (lab < -A.Nout / 2 || lab >= A.Nout / 2) return cxmk(0.0, 0.0);
        const cx<double> v = reinterpret_cast<const cx<double> *>(A.dense_in)[lab + A.Nout / 2];
        return scal(v, A.deconv[lab + A.Nout / 2]);
    }
    double ar = 0.0, ai = 0.0;
    if (A.mode == 2) {
#pragma unroll
        for (int r = -1; r <= 1; ++r) {
            const int cell = lab + r * A.N2 + A.G1 / 2;
            if (cell >= 0 && cell < A.G1) merge_cell64(A, cell_slot(cell, A.slotT, A.slotP), ar, ai);
        }
        return cxmk(ar, -ai);
    }
    if (lab < -A.G1 / 2 || lab >= A.G1 / 2) return cxmk(0.0, 0.0);
    const int slot = cell_slot(lab + A.G1 / 2, A.slotT, A.slotP);
    const double sc = A.deconv[slot];
    merge_cell64(A, slot, ar, ai);
    return cxmk(ar * sc, ai * sc);
}

template <typename T>
__device__ __forceinline__ cx<T> fft_input(const FftArgs &A, int q);
template <>
__device__ __forceinline__ cx<float> fft_input<float>(const FftArgs &A, int q) { return fft_input32(A, q); }
template <>
__device__ __forceinline__ cx<double> fft_input<double>(const FftArgs &A, int q) { return fft_input64(A, q); }

// forward DFT of size R in registers: X_q = sum_r a_r exp(-2 pi i r q / R)
template <typename T, int R>
struct Dft;

template <typename T>
struct Dft<T, 2> {
    __device__ static void run(cx<T> *a)
    {
        const cx<T> t = a[0];
        a[0] = t + a[1];
        a[1] = t - a[1];
    }
};
template <typename T>
struct Dft<T, 4> {
    __device__ static void run(cx<T> *a)
    {
        const cx<T> s0 = a[0] + a[2], d0 = a[0] - a[2];
        const cx<T> s1 = a[1] + a[3], d1 = a[1] - a[3];
        a[0] = s0 + s1;
        a[2] = s0 - s1;
        a[1] = d0 + mul_mi(d1);
        a[3] = d0 - mul_mi(d1);
    }
};
template <typename T>
struct Dft<T, 8> {
    __device__ static void run(cx<T> *a)
    {
        cx<T> e[4] = {a[0], a[2], a[4], a[6]};
        cx<T> o[4] = {a[1], a[3], a[5], a[7]};
        Dft<T, 4>::run(e);
        Dft<T, 4>::run(o);
        const T h = (T)0.70710678118654752440084436210484904;
        const cx<T> w1 = cxmk(h, -h), w3 = cxmk(-h, -h);
        const cx<T> t0 = o[0], t1 = cmul(o[1], w1), t2 = mul_mi(o[2]), t3 = cmul(o[3], w3);
        a[0] = e[0] + t0;
        a[4] = e[0] - t0;
        a[1] = e[1] + t1;
        a[5] = e[1] - t1;
        a[2] = e[2] + t2;
        a[6] = e[2] - t2;
        a[3] = e[3] + t3;
        a[7] = e[3] - t3;
    }
};
template <typename T>
struct Dft<T, 3> {
    __device__ static void run(cx<T> *a)
    {
        const T c = (T)-0.5, s = (T)0.86602540378443864676372317075293618;
        const cx<T> t1 = a[1] + a[2];
        const cx<T> t2 = a[0] + scal(t1, c);
        const cx<T> t3 = scal(a[1] - a[2], s);
        a[0] = a[0] + t1;
        a[1] = t2 + mul_mi(t3);
        a[2] = t2 - mul_mi(t3);
    }
};
template <typename T>
struct Dft<T, 5> {
    __device__ static void run(cx<T> *a)
    {
        // cos/sin of 2 pi k / 5, k = 1, 2
        const T c1 = (T)0.30901699437494742410229341718281906;
        const T c2 = (T)-0.80901699437494742410229341718281906;
        const T s1 = (T)0.95105651629515357211643933337938214;
        const T s2 = (T)0.58778525229247312916870595463907277;
        const cx<T> p1 = a[1] + a[4], m1 = a[1] - a[4];
        const cx<T> p2 = a[2] + a[3], m2 = a[2] - a[3];
        const cx<T> b1 = a[0] + scal(p1, c1) + scal(p2, c2);
        const cx<T> b2 = a[0] + scal(p1, c2) + scal(p2, c1);
        // -i (s1 m1 + s2 m2) and -i (s2 m1 - s1 m2)
        const cx<T> d1 = mul_mi(scal(m1, s1) + scal(m2, s2));
        const cx<T> d2 = mul_mi(scal(m1, s2) - scal(m2, s1));
        a[0] = a[0] + p1 + p2;
        a[1] = b1 + d1;
        a[4] = b1 - d1;
        a[2] = b2 + d2;
        a[3] = b2 - d2;
    }
};

// One Stockham pass of radix R on B transforms of length Lsub held in LDS
// (src[b * Lsub + j]) into dst.  Twiddle exp(-2 pi i e / Lsub) = tw[e * tstride]
// (an LDS table of the sub-transform length, tstride = 1).
template <typename T, int R>
__device__ void stockham_pass(const cx<T> *src, cx<T> *dst, int Lsub, int B, int Ns,
                              const cx<T> *__restrict__ tw, int tstride)
{
    const int nbf = Lsub / R;
    const int total = nbf * B;
    const int tws = (Lsub / (Ns * R)) * tstride;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int b = idx / nbf;
        const int j = idx - b * nbf;
        const cx<T> *in = src + b * Lsub;
        cx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = in[j + r * nbf];
        const int k = j % Ns;
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) a[r] = cmul(a[r], tw[k * r * tws]);
        }
        Dft<T, R>::run(a);
        const int o = (j / Ns) * Ns * R + k;
        cx<T> *out = dst + b * Lsub;
#pragma unroll
        for (int r = 0; r < R; ++r) out[o + r * Ns] = a[r];
    }
}

// The same pass with the length, radix and stride known at compile time (the
// index arithmetic reduces to shifts and masks).
template <typename T, int L, int R, int Ns>
__device__ __forceinline__ void stockham_pass_fixed(const cx<T> *src, cx<T> *dst, int B, const cx<T> *__restrict__ tw)
{
    constexpr int nbf = L / R;
    constexpr int tws = L / (Ns * R);
    const int total = nbf * B;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int b = idx / nbf;
        const int j = idx - b * nbf;
        const cx<T> *in = src + b * L;
        cx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = in[j + r * nbf];
        const int k = j % Ns;
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) a[r] = cmul(a[r], tw[k * r * tws]);
        }
        Dft<T, R>::run(a);
        const int o = (j / Ns) * Ns * R + k;
        cx<T> *out = dst + b * L;
#pragma unroll
        for (int r = 0; r < R; ++r) out[o + r * Ns] = a[r];
    }
}

// Passes of radices R, Rest... ping-ponging between the two buffers; the
// result is in the second buffer after an odd number of passes.
template <typename T, int L, int Ns, int R, int... Rest>
__device__ __forceinline__ void stockham_fixed(cx<T> *src, cx<T> *dst, int B, const cx<T> *__restrict__ tw)
{
    stockham_pass_fixed<T, L, R, Ns>(src, dst, B, tw);
    __syncthreads();
    if constexpr (sizeof...(Rest) > 0) stockham_fixed<T, L, Ns * R, Rest...>(dst, src, B, tw);
}

// Transforms the B length-Lsub sequences in buf[0] in place (result ends up in
// buf[0] or buf[1]; the returned pointer tells which).  Power-of-two lengths
// 64..4096 take fixed radix-4/8 plans (radix 16 measured slower: its
// butterfly is a long serial chain per lane); other lengths the plan's
// radix list.
template <typename T>
__device__ cx<T> *stockham(cx<T> *buf0, cx<T> *buf1, int Lsub, int B, const int8_t *rad, int npass,
                           const cx<T> *__restrict__ tw, int tstride)
{
    if (tstride == 1) {
        int odd = -1;   // passes of the fixed plan modulo 2
        switch (Lsub) {
        case 64: stockham_fixed<T, 64, 1, 8, 8>(buf0, buf1, B, tw); odd = 0; break;
        case 128: stockham_fixed<T, 128, 1, 4, 4, 8>(buf0, buf1, B, tw); odd = 1; break;
        case 256: stockham_fixed<T, 256, 1, 4, 8, 8>(buf0, buf1, B, tw); odd = 1; break;
        case 512: stockham_fixed<T, 512, 1, 8, 8, 8>(buf0, buf1, B, tw); odd = 1; break;
        case 1024: stockham_fixed<T, 1024, 1, 4, 4, 8, 8>(buf0, buf1, B, tw); odd = 0; break;
        case 2048: stockham_fixed<T, 2048, 1, 4, 8, 8, 8>(buf0, buf1, B, tw); odd = 0; break;
        case 4096: stockham_fixed<T, 4096, 1, 8, 8, 8, 8>(buf0, buf1, B, tw); odd = 0; break;
        default: break;
        }
        if (odd >= 0) return odd ? buf1 : buf0;
    }
    cx<T> *src = buf0, *dst = buf1;
    int Ns = 1;
    for (int ps = 0; ps < npass; ++ps) {
        const int R = rad[ps];
        switch (R) {
        case 8: stockham_pass<T, 8>(src, dst, Lsub, B, Ns, tw, tstride); break;
        case 4: stockham_pass<T, 4>(src, dst, Lsub, B, Ns, tw, tstride); break;
        case 2: stockham_pass<T, 2>(src, dst, Lsub, B, Ns, tw, tstride); break;
        case 5: stockham_pass<T, 5>(src, dst, Lsub, B, Ns, tw, tstride); break;
        default: stockham_pass<T, 3>(src, dst, Lsub, B, Ns, tw, tstride); break;
        }
        __syncthreads();
        cx<T> *tmp = src;
        src = dst;
        dst = tmp;
        Ns *= R;
    }
    return src;
}

// write output k (index mod N2) of the length-N2 transform into hlin if consumed
template <typename T>
__device__ __forceinline__ void fft_store(const FftArgs &A, int k, cx<T> v)
{
    const int half = A.N2 / 2;
    const int s = (k < half) ? k : k - A.N2;
    if (A.mode == 2) {
        // adjoint NFFT: h_k = conj(X_k) / (n phi_hat(k)) for k in I_N, dense output
        if (s >= -A.Nout / 2 && s < A.Nout / 2) {
            const double sc = A.deconv[s + A.Nout / 2];
            reinterpret_cast<cx<T> *>(A.dense_out)[s + A.Nout / 2] =
                cxmk((T)((double)v.re * sc), (T)(-(double)v.im * sc));
        }
        return;
    }
    // labels s, s + N2, s - N2 that the interpolation reads (|label| <= S),
    // stored at label + h_off: the 1-periodic extension of the transform
    cx<T> *h = reinterpret_cast<cx<T> *>(A.hlin);
    if (s >= -A.S && s <= A.S) h[s + A.h_off] = v;
    if (s + A.N2 <= A.S) h[s + A.N2 + A.h_off] = v;
    if (s - A.N2 >= -A.S) h[s - A.N2 + A.h_off] = v;
}

// LDS of an FFT workgroup, sized at launch (dynamic shared memory) for the
// plan's sub-transforms: two ping-pong buffers, the sub-transform twiddles and
// (stage A) the four-step twiddles, `vals` complex values each.
template <typename T>
struct FftLds {
    cx<T> *buf[2];
    cx<T> *tw;
    cx<T> *otw;
};

// complex values per array: the whole transform (one workgroup) or the
// largest batch of sub-transforms of the two four-step stages
__host__ __device__ __forceinline__ int fft_vals(const FftArgs &A)
{
    return A.n1 == 1 ? A.N2 : max(A.batchA * A.n2, A.batchB * A.n1);
}

template <typename T>
__device__ __forceinline__ FftLds<T> fft_lds(const FftArgs &A)
{
    extern __shared__ __align__(16) char smem[];
    cx<T> *p = reinterpret_cast<cx<T> *>(smem);
    const int v = fft_vals(A);
    FftLds<T> L;
    L.buf[0] = p;
    L.buf[1] = p + v;
    L.tw = p + 2 * v;
    L.otw = p + 3 * v;
    return L;
}

template <typename T>
static size_t fft_lds_bytes(const FftArgs &A)
{
    return 4 * (size_t)fft_vals(A) * sizeof(cx<T>);
}

// Column block handled by local workgroup w of a launch of 8 ceil(ng / 8)
// workgroups: XCD x = w mod 8 takes the contiguous blocks [x per, (x + 1) per),
// so neighbouring columns, which share cache lines of the strided loads and
// stores, meet in one L2.  Blocks >= ng are idle.
__device__ __forceinline__ int xcd_block(int w, int ng)
{
    const int per = (ng + 7) / 8;
    return (w & 7) * per + (w >> 3);
}

// Whole transform in one workgroup (N2 <= 1024)
template <typename T>
__device__ void fft_single_body(const FftArgs &A, FftLds<T> &L)
{
    const int N2 = A.N2;
    const cx<T> *gtw = reinterpret_cast<const cx<T> *>(A.tw);
    // data and twiddles in one round of loads; all passes then run from LDS
    for (int q = threadIdx.x; q < N2; q += blockDim.x) {
        const cx<T> t = gtw[q];
        const cx<T> xv = fft_input<T>(A, q);
        L.tw[q] = t;
        L.buf[0][q] = xv;
    }
    __syncthreads();
    cx<T> *res = stockham<T>(L.buf[0], L.buf[1], N2, 1, A.radA, A.npassA, L.tw, 1);
    for (int k = threadIdx.x; k < N2; k += blockDim.x) fft_store<T>(A, k, res[k]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_fft_single(FftArgs A)
{
    FftLds<T> L = fft_lds<T>(A);
    fft_single_body<T>(A, L);
}

// Four-step stage A: for columns j1, length-n2 transforms over j2 of
// x[j1 + n1 j2], times exp(-2 pi i j1 k2 / N2), stored to Y[k2 n1 + j1] (so
// that stage B reads its columns contiguously).
template <typename T>
__device__ void fft_stageA_body(const FftArgs &A, int w, FftLds<T> &L)
{
    const int n1 = A.n1, n2 = A.n2, B = A.batchA;
    const int ng = (n1 + B - 1) / B;
    const int blk = xcd_block(w, ng);
    if (blk >= ng) return;
    const int j1_0 = blk * B;
    const int nb = min(B, n1 - j1_0);
    const cx<T> *twA = reinterpret_cast<const cx<T> *>(A.twA);
    const cx<T> *tw4 = reinterpret_cast<const cx<T> *>(A.tw4);
    // one round of loads: the merged input, the length-n2 twiddles and the
    // four-step twiddles exp(-2 pi i j1 k2 / N2) of these columns (tables
    // [n2] and [n1][n2], read contiguously)
    // (every global load of an element is issued before its LDS stores, so
    // the loads of one element travel together)
    for (int idx = threadIdx.x; idx < nb * n2; idx += blockDim.x) {
        const int j2 = idx / nb, bl = idx - j2 * nb;
        const cx<T> ta = twA[min(idx, n2 - 1)];
        const cx<T> t4 = tw4[(size_t)j1_0 * n2 + idx];
        const cx<T> xv = fft_input<T>(A, j1_0 + bl + n1 * j2);
        if (idx < n2) L.tw[idx] = ta;
        L.otw[idx] = t4;
        L.buf[0][bl * n2 + j2] = xv;
    }
    __syncthreads();
    cx<T> *res = stockham<T>(L.buf[0], L.buf[1], n2, nb, A.radA, A.npassA, L.tw, 1);
    cx<T> *Y = reinterpret_cast<cx<T> *>(A.Y);
    for (int idx = threadIdx.x; idx < nb * n2; idx += blockDim.x) {
        const int bl = idx / n2, k2 = idx - bl * n2;
        const int j1 = j1_0 + bl;
        Y[(size_t)k2 * n1 + j1] = cmul(res[idx], L.otw[idx]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fft_stageA(FftArgs A)
{
    FftLds<T> L = fft_lds<T>(A);
    fft_stageA_body<T>(A, blockIdx.x, L);
}

// Four-step stage B: for columns k2, length-n1 transforms over j1 of
// Y[k2 n1 + j1]; output k1 is X[k2 + n2 k1].
template <typename T>
__device__ void fft_stageB_body(const FftArgs &A, int w, FftLds<T> &L)
{
    const int n1 = A.n1, n2 = A.n2, B = A.batchB;
    const int ng = (n2 + B - 1) / B;
    const int blk = xcd_block(w, ng);
    if (blk >= ng) return;
    const int k2_0 = blk * B;
    const int nb = min(B, n2 - k2_0);
    const cx<T> *Y = reinterpret_cast<const cx<T> *>(A.Y);
    const cx<T> *twB = reinterpret_cast<const cx<T> *>(A.twB);
    for (int idx = threadIdx.x; idx < nb * n1; idx += blockDim.x) {
        const cx<T> tb = twB[min(idx, n1 - 1)];
        const cx<T> yv = Y[(size_t)k2_0 * n1 + idx];   // column bl = idx / n1, j1 = idx mod n1
        if (idx < n1) L.tw[idx] = tb;
        L.buf[0][idx] = yv;
    }
    __syncthreads();
    cx<T> *res = stockham<T>(L.buf[0], L.buf[1], n1, nb, A.radB, A.npassB, L.tw, 1);
    for (int idx = threadIdx.x; idx < nb * n1; idx += blockDim.x) {
        const int bl = idx / n1, k1 = idx - bl * n1;
        fft_store<T>(A, k2_0 + bl + n2 * k1, res[bl * n1 + k1]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fft_stageB(FftArgs A)
{
    FftLds<T> L = fft_lds<T>(A);
    fft_stageB_body<T>(A, blockIdx.x, L);
}

// ===========================================================================
// Fast sinc transform: the middle operator (Algorithm 6.1 steps 1-3 between
// the two FFTs, composed on the host into the band K)
// ===========================================================================
// h_s of the first plan, as its interpolation reads it
template <typename T>
__device__ __forceinline__ cx<T> plan_output(const InterpArgs &A, int s)
{
    return A.fusedB ? folded_output<T>(A, s) : reinterpret_cast<const cx<T> *>(A.hlin)[s + A.h_off];
}

// One workgroup per kSincMidRows rows: each thread's first kMidK band
// coefficients are loaded first (coalesced over the rows, kept in
// registers), then the labels the workgroup's rows read are staged in LDS;
// the band is accumulated in FP64.
constexpr int kMidK = 32;
template <typename T>
__global__ __launch_bounds__(kSincMidRows) void k_sinc_mid(SincMidArgs A)
{
    extern __shared__ __align__(16) char smem[];
    cx<T> *hw = reinterpret_cast<cx<T> *>(smem);
    const int g = blockIdx.x;
    const int row = g * kSincMidRows + threadIdx.x;
    const int rr = min(row, A.G1 - 1);   // rows past the end read a valid row and store nothing
    double kr[kMidK];
#pragma unroll
    for (int b = 0; b < kMidK; ++b) kr[b] = A.K[(size_t)min(b, A.Wb - 1) * A.G1 + rr];
    const int lo = A.lo[rr];
    const int base = A.base[g], span = A.span[g];
    for (int i = threadIdx.x; i < span; i += kSincMidRows) {
        const int sl = base + i;
        hw[i] = (sl >= -A.S && sl <= A.S) ? plan_output<T>(A.h, sl) : cxmk((T)0, (T)0);
    }
    __syncthreads();
    if (row >= A.G1) return;
    const cx<T> *hr = hw + (lo - base);
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int b = 0; b < kMidK; ++b) {
        if (b < A.Wb) {
            const cx<T> v = hr[b];
            re = fma(kr[b], (double)v.re, re);
            im = fma(kr[b], (double)v.im, im);
        }
    }
    for (int b = kMidK; b < A.Wb; ++b) {   // bands wider than kMidK
        const double k = A.K[(size_t)b * A.G1 + row];
        const cx<T> v = hr[b];
        re = fma(k, (double)v.re, re);
        im = fma(k, (double)v.im, im);
    }
    reinterpret_cast<cx<T> *>(A.out)[row] = cxmk((T)re, (T)im);
}

// ===========================================================================
// Batched kernels: one launch per stage for up to kMaxBatch plans of one
// precision.  Each workgroup finds its plan in the table and runs the same
// slot / column code as the plan's own launch, so results are bitwise equal.
// ===========================================================================
__device__ __forceinline__ int batch_plan(const BatchTable &T, int g)
{
    int p = 0;
    while (p + 1 < T.n && T.start[p + 1] <= g) ++p;
    return p;
}

template <int TM>
__global__ __launch_bounds__(kThreads32, TM <= 16 ? 6 : 4) void k_spread32_batch(BatchTable T)
{
    __shared__ Spread32Lds<TM> L;
    const int p = batch_plan(T, blockIdx.x);
    const SpreadArgs A = T.desc[p]->sp;
    const int g = blockIdx.x - T.start[p];
    if (g >= A.ngrid) return;
    spread32_slot<TM>(A, static_cast<const cx<float> *>(T.in[p]), g, L);
}

__global__ __launch_bounds__(kThreads64) void k_spread64_batch(BatchTable T)
{
    const int p = batch_plan(T, blockIdx.x);
    const SpreadArgs A = T.desc[p]->sp;
    Spread64Lds L = spread64_lds(2 * A.m, A.rows);
    const int g = blockIdx.x - T.start[p];
    if (g >= A.ngrid) return;
    const cx<double> *in = static_cast<const cx<double> *>(T.in[p]);
    if (A.window == NNFFT_WINDOW_BSPLINE)
        spread64_slot<NNFFT_WINDOW_BSPLINE>(A, in, g, L);
    else if (A.window == NNFFT_WINDOW_ALGEBRAIC)
        spread64_slot<NNFFT_WINDOW_ALGEBRAIC>(A, in, g, L);
    else if (A.window == NNFFT_WINDOW_KAISER_BESSEL)
        spread64_slot<NNFFT_WINDOW_KAISER_BESSEL>(A, in, g, L);
    else
        spread64_slot<NNFFT_WINDOW_SINH>(A, in, g, L);
}

template <int CD>
__global__ __launch_bounds__(kThreads32) void k_interp32_batch(BatchTable T)
{
    __shared__ Interp32Lds L;
    const int p = batch_plan(T, blockIdx.x);
    const InterpArgs A = T.desc[p]->ip;
    const int g = blockIdx.x - T.start[p];
    if (g >= A.ngrid) return;
    interp32_slot<CD, kRowsPerWave>(A, static_cast<cx<float> *>(T.out[p]), g, L);
}

__global__ __launch_bounds__(kThreads64) void k_interp64_batch(BatchTable T)
{
    const int p = batch_plan(T, blockIdx.x);
    const InterpArgs A = T.desc[p]->ip;
    Interp64Lds L = interp64_lds();
    const int g = blockIdx.x - T.start[p];
    if (g >= A.ngrid) return;
    cx<double> *out = static_cast<cx<double> *>(T.out[p]);
    if (A.window == NNFFT_WINDOW_BSPLINE)
        interp64_slot<NNFFT_WINDOW_BSPLINE>(A, out, g, L);
    else if (A.window == NNFFT_WINDOW_ALGEBRAIC)
        interp64_slot<NNFFT_WINDOW_ALGEBRAIC>(A, out, g, L);
    else if (A.window == NNFFT_WINDOW_KAISER_BESSEL)
        interp64_slot<NNFFT_WINDOW_KAISER_BESSEL>(A, out, g, L);
    else
        interp64_slot<NNFFT_WINDOW_SINH>(A, out, g, L);
}

// stage A of four-step plans and the whole transform of one-workgroup plans
template <typename T>
__global__ __launch_bounds__(256) void k_fftA_batch(BatchTable Tb)
{
    const int p = batch_plan(Tb, blockIdx.x);
    const FftArgs &A = Tb.desc[p]->fft;
    FftLds<T> L = fft_lds<T>(A);
    const int w = blockIdx.x - Tb.start[p];
    if (A.n1 == 1) {
        if (w == 0) fft_single_body<T>(A, L);
    } else {
        fft_stageA_body<T>(A, w, L);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fftB_batch(BatchTable Tb)
{
    const int p = batch_plan(Tb, blockIdx.x);
    const FftArgs &A = Tb.desc[p]->fft;
    FftLds<T> L = fft_lds<T>(A);
    fft_stageB_body<T>(A, blockIdx.x - Tb.start[p], L);
}

// ===========================================================================
// Launchers
// ===========================================================================
// workgroups of a four-step stage: column blocks rounded up to a multiple of 8
static int fft_groups(int ncol, int batch)
{
    return ((ncol + batch - 1) / batch + 7) / 8 * 8;
}

template <typename T>
static void launch_fft(const FftArgs &A, hipStream_t s, KernelTimes *kt = nullptr)
{
    const uint32_t lds = (uint32_t)fft_lds_bytes<T>(A);
    if (A.n1 == 1) {
        launch_k(kt, KID_FFT_SINGLE, k_fft_single<T>, dim3(1), dim3(A.threadsA), lds, s, A);
    } else {
        const int gA = fft_groups(A.n1, A.batchA), gB = fft_groups(A.n2, A.batchB);
        launch_k(kt, KID_FFT_A, k_fft_stageA<T>, dim3(gA), dim3(A.threadsA), lds, s, A);
        if (!A.fusedB) launch_k(kt, KID_FFT_B, k_fft_stageB<T>, dim3(gB), dim3(A.threadsB), lds, s, A);
    }
}

// k_interp32 variants: correction degree CD in {8, 10, 12, 16, 24, 32}, RB
// record rows per load batch
template <int RB>
static void launch_interp32_rb(int cd, int grid, hipStream_t s, const InterpArgs &A, cx<float> *y,
                               KernelTimes *kt)
{
    const dim3 g(grid), b(kThreads32);
    switch (cd) {
    case 8: launch_k(kt, KID_INTERP32, k_interp32<8, RB>, g, b, 0, s, A, y); break;
    case 10: launch_k(kt, KID_INTERP32, k_interp32<10, RB>, g, b, 0, s, A, y); break;
    case 12: launch_k(kt, KID_INTERP32, k_interp32<12, RB>, g, b, 0, s, A, y); break;
    case 16: launch_k(kt, KID_INTERP32, k_interp32<16, RB>, g, b, 0, s, A, y); break;
    case 24: launch_k(kt, KID_INTERP32, k_interp32<24, RB>, g, b, 0, s, A, y); break;
    default: launch_k(kt, KID_INTERP32, k_interp32<32, RB>, g, b, 0, s, A, y); break;
    }
}

static void launch_interp32(int cd, int grid, hipStream_t s, const InterpArgs &A, cx<float> *y,
                            KernelTimes *kt = nullptr)
{
    if (A.rows <= kRowsShort * kWaves32)
        launch_interp32_rb<kRowsShort>(cd, grid, s, A, y, kt);
    else
        launch_interp32_rb<kRowsPerWave>(cd, grid, s, A, y, kt);
}

static void launch_interp32_batch(int cd, int grid, hipStream_t s, const BatchTable &T)
{
    switch (cd) {
    case 8: hipLaunchKernelGGL((k_interp32_batch<8>), dim3(grid), dim3(kThreads32), 0, s, T); break;
    case 10: hipLaunchKernelGGL((k_interp32_batch<10>), dim3(grid), dim3(kThreads32), 0, s, T); break;
    case 12: hipLaunchKernelGGL((k_interp32_batch<12>), dim3(grid), dim3(kThreads32), 0, s, T); break;
    case 16: hipLaunchKernelGGL((k_interp32_batch<16>), dim3(grid), dim3(kThreads32), 0, s, T); break;
    case 24: hipLaunchKernelGGL((k_interp32_batch<24>), dim3(grid), dim3(kThreads32), 0, s, T); break;
    default: hipLaunchKernelGGL((k_interp32_batch<32>), dim3(grid), dim3(kThreads32), 0, s, T); break;
    }
}

// k_spread32 variants: tap rows TM in {12, 16, 32}, the smallest >= 2m
static void launch_spread32(const SpreadArgs &A, int grid, const cx<float> *f, hipStream_t s,
                            KernelTimes *kt = nullptr)
{
    const dim3 g(grid), b(kThreads32);
    if (2 * A.m <= 12)
        launch_k(kt, KID_SPREAD32, k_spread32<12>, g, b, 0, s, A, f);
    else if (2 * A.m <= 16)
        launch_k(kt, KID_SPREAD32, k_spread32<16>, g, b, 0, s, A, f);
    else
        launch_k(kt, KID_SPREAD32, k_spread32<32>, g, b, 0, s, A, f);
}

// evaluated degree of the 1/phi_hat_1 series: the smallest variant >= deg
static int corr_variant(int deg)
{
    return deg <= 8 ? 8 : deg <= 10 ? 10 : deg <= 12 ? 12 : deg <= 16 ? 16 : deg <= 24 ? 24 : 32;
}


// the pre-merge of long merge lists, between the spreading and the FFT
template <typename T>
static void launch_premerge(const PreMergeArgs &M, hipStream_t s, KernelTimes *kt = nullptr)
{
    if (M.nseg > 0) launch_k(kt, KID_PREMERGE, k_premerge<T>, dim3((M.nseg + 255) / 256), dim3(256), 0, s, M);
}

hipError_t launch_exec(const PlanDev &P, const void *f, void *y, hipStream_t s, KernelTimes *kt)
{
    if (kt) kt->n = 0;
    if (P.prec == NNFFT_FP32_COMP) {
        const cx<float> *fin = reinterpret_cast<const cx<float> *>(f);
        const int gs = P.sp.ngrid, gi = P.ip.ngrid;
        launch_spread32(P.sp, gs, fin, s, kt);
        launch_premerge<float>(P.pm, s, kt);
        launch_fft<float>(P.fft, s, kt);
        launch_interp32(corr_variant(P.ip.corr_deg), gi, s, P.ip, reinterpret_cast<cx<float> *>(y), kt);
    } else {
        launch_spread64(P.sp, f, s, kt);
        launch_premerge<double>(P.pm, s, kt);
        launch_fft<double>(P.fft, s, kt);
        launch_interp64(P.ip, y, s, kt);
    }
    return hipGetLastError();
}

hipError_t launch_sinc_middle(const PlanDev &P1, const SincMidArgs &M, const PlanDev &P2, const void *c, void *h,
                              hipStream_t s)
{
    FftArgs F = P2.fft;
    F.mode = 3;
    F.dense_in = M.out;
    if (P1.prec == NNFFT_FP32_COMP) {
        launch_spread32(P1.sp, P1.sp.ngrid, reinterpret_cast<const cx<float> *>(c), s);
        launch_premerge<float>(P1.pm, s);
        launch_fft<float>(P1.fft, s);
        hipLaunchKernelGGL(k_sinc_mid<float>, dim3(M.nwg), dim3(kSincMidRows), (size_t)M.span_max * sizeof(cx<float>),
                           s, M);
        launch_fft<float>(F, s);
        launch_interp32(corr_variant(P2.ip.corr_deg), P2.ip.ngrid, s, P2.ip, reinterpret_cast<cx<float> *>(h));
    } else {
        launch_spread64(P1.sp, c, s, nullptr);
        launch_premerge<double>(P1.pm, s);
        launch_fft<double>(P1.fft, s);
        hipLaunchKernelGGL(k_sinc_mid<double>, dim3(M.nwg), dim3(kSincMidRows),
                           (size_t)M.span_max * sizeof(cx<double>), s, M);
        launch_fft<double>(F, s);
        launch_interp64(P2.ip, h, s, nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_exec_batch(int n, const PlanDev *const *host, const PlanDev *const *dev,
                             const void *const *f, void *const *y, hipStream_t s)
{
    auto rnd8 = [](int x) { return (x + 7) / 8 * 8; };
    for (int b0 = 0; b0 < n; b0 += kMaxBatch) {
        const int nb = std::min(kMaxBatch, n - b0);
        BatchTable Tsp{}, Tip{}, TA{}, TB{};
        int ssp = 0, sip = 0, sA = 0, sB = 0, thrA = 64, thrB = 64;
        int tm_sp = 2, tm_ip = 2;   // largest 2m of the group (FP32 variant, FP64 LDS size)
        int rows_sp = 1;            // largest item size of the group (FP64 LDS size)
        size_t fft_bytes = 0;       // largest FFT LDS of the group
        int corr_deg = 0;
        for (int i = 0; i < nb; ++i) {
            const PlanDev &P = *host[b0 + i];
            for (BatchTable *T : {&Tsp, &Tip, &TA, &TB}) {
                T->desc[i] = dev[b0 + i];
                T->in[i] = f[b0 + i];
                T->out[i] = y[b0 + i];
            }
            Tsp.start[i] = ssp;
            ssp += rnd8(P.sp.ngrid);
            Tip.start[i] = sip;
            sip += rnd8(P.ip.ngrid);
            TA.start[i] = sA;
            TB.start[i] = sB;
            if (P.fft.n1 == 1) {
                sA += 8;
                thrA = std::max(thrA, P.fft.threadsA);
            } else {
                sA += fft_groups(P.fft.n1, P.fft.batchA);
                if (!P.fft.fusedB) sB += fft_groups(P.fft.n2, P.fft.batchB);
                thrA = std::max(thrA, P.fft.threadsA);
                thrB = std::max(thrB, P.fft.threadsB);
            }
            tm_sp = std::max(tm_sp, 2 * P.sp.m);
            rows_sp = std::max(rows_sp, P.sp.rows);
            fft_bytes = std::max(fft_bytes, P.prec == NNFFT_FP32_COMP ? fft_lds_bytes<float>(P.fft)
                                                                      : fft_lds_bytes<double>(P.fft));
            tm_ip = std::max(tm_ip, 2 * P.ip.m);
            corr_deg = std::max(corr_deg, P.ip.corr_deg);
        }
        Tsp.start[nb] = ssp;
        Tip.start[nb] = sip;
        TA.start[nb] = sA;
        TB.start[nb] = sB;
        Tsp.n = Tip.n = TA.n = TB.n = nb;
        if (host[b0]->prec == NNFFT_FP32_COMP) {
            if (tm_sp > 16)
                hipLaunchKernelGGL((k_spread32_batch<32>), dim3(ssp), dim3(kThreads32), 0, s, Tsp);
            else if (tm_sp > 12)
                hipLaunchKernelGGL((k_spread32_batch<16>), dim3(ssp), dim3(kThreads32), 0, s, Tsp);
            else
                hipLaunchKernelGGL((k_spread32_batch<12>), dim3(ssp), dim3(kThreads32), 0, s, Tsp);
            for (int i = 0; i < nb; ++i) launch_premerge<float>(host[b0 + i]->pm, s);   // plans that need it
            hipLaunchKernelGGL((k_fftA_batch<float>), dim3(sA), dim3(thrA), fft_bytes, s, TA);
            if (sB > 0) hipLaunchKernelGGL((k_fftB_batch<float>), dim3(sB), dim3(thrB), fft_bytes, s, TB);
            launch_interp32_batch(corr_variant(corr_deg), sip, s, Tip);
        } else {
            hipLaunchKernelGGL(k_spread64_batch, dim3(ssp), dim3(kThreads64), lds64_bytes(tm_sp, rows_sp), s,
                               Tsp);
            for (int i = 0; i < nb; ++i) launch_premerge<double>(host[b0 + i]->pm, s);
            hipLaunchKernelGGL((k_fftA_batch<double>), dim3(sA), dim3(thrA), fft_bytes, s, TA);
            if (sB > 0) hipLaunchKernelGGL((k_fftB_batch<double>), dim3(sB), dim3(thrB), fft_bytes, s, TB);
            hipLaunchKernelGGL(k_interp64_batch, dim3(sip), dim3(kThreads64), interp64_lds_bytes(tm_ip), s,
                               Tip);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// NFFT with equispaced frequencies: forward = FFT (deconvolved coefficients
// in the load) + interpolation; adjoint = spreading + FFT (periodic fold and
// conjugation in the load, conjugation and deconvolution in the store).
hipError_t launch_nfft(const PlanDev &P, bool adjoint, const void *in, void *out, hipStream_t s)
{
    FftArgs F = P.fft;
    if (!adjoint) {
        F.mode = 1;
        F.dense_in = in;
    } else {
        F.mode = 2;
        F.dense_out = out;
    }
    if (P.prec == NNFFT_FP32_COMP) {
        if (adjoint) {
            const cx<float> *yin = reinterpret_cast<const cx<float> *>(in);
            launch_spread32(P.sp, P.sp.ngrid, yin, s);
            launch_premerge<float>(P.pm, s);
            launch_fft<float>(F, s);
        } else {
            launch_fft<float>(F, s);
            launch_interp32(corr_variant(P.ip.corr_deg), P.ip.ngrid, s, P.ip, reinterpret_cast<cx<float> *>(out));
        }
    } else {
        if (adjoint) {
            launch_spread64(P.sp, in, s);
            launch_premerge<double>(P.pm, s);
            launch_fft<double>(F, s);
        } else {
            launch_fft<double>(F, s);
            launch_interp64(P.ip, out, s);
        }
    }
    return hipGetLastError();
}

// ===========================================================================
// Algorithm 6.1 step 2: alpha_j = w_j g~_j with FP64 weights
// ===========================================================================
__global__ void k_scale32(const double *__restrict__ w, const cx<float> *src, cx<float> *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const cx<float> v = src[i];
        dst[i] = cxmk((float)((double)v.re * w[i]), (float)((double)v.im * w[i]));
    }
}
__global__ void k_scale64(const double *__restrict__ w, const cx<double> *src, cx<double> *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = scal(src[i], w[i]);
}

// ===========================================================================
// Exec without allocation: working memory in a static device array
// ===========================================================================
// One array per device (the runtime places a copy on every GPU the library
// runs on; it lives until the process ends).  Host code never passes the
// array's name to a kernel: in host code it is a stand-in, and its device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}   // namespace

// Device address of the current device's array (null on failure).
static void *static_scratch_ptr()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

__global__ void k_zero16(float4 *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t static_scratch_need(const ExecScratch &sz)
{
    return align256(sz.part_bytes) + align256(sz.y_bytes) + align256(sz.hlin_bytes);
}

hipError_t launch_exec_static(const PlanDev &P, const ExecScratch &sz, const void *f, void *y, hipStream_t s)
{
    if (static_scratch_need(sz) > kStaticScratchBytes) return hipErrorInvalidValue;
    unsigned char *base = static_cast<unsigned char *>(static_scratch_ptr());
    if (base == nullptr) return hipErrorInvalidSymbol;
    PlanDev D = P;
    void *part = base;
    void *Y = base + align256(sz.part_bytes);
    void *hlin = base + align256(sz.part_bytes) + align256(sz.y_bytes);
    D.sp.partial = part;
    D.fft.partial = part;
    D.pm.partial = part;
    D.fft.Y = Y;
    D.fft.hlin = hlin;
    D.ip.hlin = hlin;
    if (D.ip.fusedB) D.ip.Y = Y;
    // the array keeps the previous call's contents: plane cells that no
    // window of this plan writes must read as zero (a fill kernel, so the
    // call stays capturable in a graph)
    const int64_t n16 = (int64_t)(sz.plane_bytes / 16);
    if (n16 > 0) {
        const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 2048);
        hipLaunchKernelGGL(k_zero16, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<float4 *>(part), n16);
    }
    return launch_exec(D, f, y, s, nullptr);
}

hipError_t launch_scale_by_weights(int prec, const double *w, const void *src, void *dst, int64_t n,
                                   hipStream_t s)
{
    const int nt = 256;
    const int64_t g = (n + nt - 1) / nt;
    if (prec == NNFFT_FP32_COMP)
        hipLaunchKernelGGL(k_scale32, dim3((unsigned)g), dim3(nt), 0, s, w,
                           reinterpret_cast<const cx<float> *>(src), reinterpret_cast<cx<float> *>(dst), n);
    else
        hipLaunchKernelGGL(k_scale64, dim3((unsigned)g), dim3(nt), 0, s, w,
                           reinterpret_cast<const cx<double> *>(src), reinterpret_cast<cx<double> *>(dst), n);
    return hipGetLastError();
}

}  // namespace nnfft
