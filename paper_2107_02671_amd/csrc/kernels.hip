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
#include "internal.h"
#include "../../include/nnfft.h"

namespace nnfft {

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

// sinh window of Example 2.1 in FP64:
//   sinh(beta s)/sinh(beta) = (e^{beta(s-1)} - e^{-beta(s+1)}) / (1 - e^{-2 beta})
__device__ __forceinline__ double omega64(double u, double beta, double inv_den)
{
    const double q = (1.0 - u) * (1.0 + u);
    if (!(q > 0.0)) return 0.0;
    const double s = sqrt(q);
    return (exp(beta * (s - 1.0)) - exp(-beta * (s + 1.0))) * inv_den;
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

// 1/phi_hat_1(N* x_j) for the bin label `lab` and offset `fr` of a node
__device__ __forceinline__ double inv_phi1(const PlanDesc &P, int lab, double fr)
{
    const double x = ((double)lab + fr) * P.u_to_x;
    return cheb64(P.corr, P.corr_deg, fma(8.0 * x, x, -1.0));
}

// ===========================================================================
// Spreading, FP32 path
// ===========================================================================
template <int TM>   // TM >= 2 m1
struct Spread32Lds {
    cx<float> mom[256 * (kDeg + 1)];
    cx<float> sbin[256 * TM];
    int ibin[256];
    int runS[256];
    int runE[256];
};

template <int TM>
__device__ void spread32_wg(const PlanDesc &P, int cid, const cx<float> *__restrict__ f,
                            Spread32Lds<TM> &L)
{
    constexpr int D = kDeg;
    const Chunk ch = P.sp.chunks[cid];
    const int m = P.m1, tm = 2 * m;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int b = t; b < ch.nbin; b += nt) {
        L.runS[b] = -1;
        L.runE[b] = 0;
    }
    // Phase A: Chebyshev moments of each item
    if (t < ch.nitem) {
        const Item it = P.sp.items[ch.item0 + t];
        float mr[D + 1], mi[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) mr[k] = mi[k] = 0.f;
        for (int p = it.p0; p < it.p0 + it.n; ++p) {
            const float y = fmaf(2.f, P.sp.frac32[p], -1.f);
            const cx<float> fv = f[P.sp.perm[p]];
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
#pragma unroll
        for (int k = 0; k <= D; ++k) L.mom[t * (D + 1) + k] = cxmk(mr[k], mi[k]);
        L.ibin[t] = it.bin - ch.bin_lo;
    }
    __syncthreads();
    if (t < ch.nitem) {
        const int b = L.ibin[t];
        if (t == 0 || L.ibin[t - 1] != b) L.runS[b] = t;
        if (t == ch.nitem - 1 || L.ibin[t + 1] != b) L.runE[b] = t + 1;
    }
    __syncthreads();
    // Phase B: per bin, compensated sum of its items' moments, then the 2m taps
    for (int b = t; b < ch.nbin; b += nt) {
        cx<float> *out = L.sbin + b * TM;
        const int s = L.runS[b];
        if (s < 0) {
            for (int r = 0; r < tm; ++r) out[r] = cxmk(0.f, 0.f);
            continue;
        }
        const int e = L.runE[b];
        float hr[D + 1], hi[D + 1], lr[D + 1], li[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            const cx<float> v = L.mom[s * (D + 1) + k];
            hr[k] = v.re;
            hi[k] = v.im;
            lr[k] = li[k] = 0.f;
        }
        for (int i = s + 1; i < e; ++i) {
#pragma unroll
            for (int k = 0; k <= D; ++k) {
                const cx<float> v = L.mom[i * (D + 1) + k];
                comp_add(hr[k], lr[k], v.re);
                comp_add(hi[k], li[k], v.im);
            }
        }
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            hr[k] += lr[k];
            hi[k] += li[k];
        }
        for (int r = 0; r < tm; ++r) {
            const float *c = P.C1 + r * (D + 1);
            float ar = 0.f, ai = 0.f;
#pragma unroll
            for (int k = 0; k <= D; ++k) {
                ar = fmaf(c[k], hr[k], ar);
                ai = fmaf(c[k], hi[k], ai);
            }
            out[r] = cxmk(ar, ai);
        }
    }
    __syncthreads();
    // Phase C: window cell w (cell bin_lo - m + 1 + w) collects tap w - b of
    // bin b; compensated, stored as (hi.re, hi.im, lo.re, lo.im)
    const int W = ch.nbin + tm - 1;
    float4 *part = reinterpret_cast<float4 *>(P.partial) + ch.part_off;
    for (int w = t; w < W; w += nt) {
        const int blo = max(0, w - tm + 1), bhi = min(ch.nbin - 1, w);
        float hr = 0.f, hi = 0.f, lr = 0.f, li = 0.f;
        for (int b = blo; b <= bhi; ++b) {
            const cx<float> v = L.sbin[b * TM + (w - b)];
            comp_add(hr, lr, v.re);
            comp_add(hi, li, v.im);
        }
        part[w] = make_float4(hr, hi, lr, li);
    }
}

template <int TM>
__global__ __launch_bounds__(256) void k_spread32(PlanDesc P, const cx<float> *__restrict__ f)
{
    __shared__ Spread32Lds<TM> L;
    const int cid = P.sp.sched[blockIdx.x];
    if (cid < 0) return;
    spread32_wg<TM>(P, cid, f, L);
}

// ===========================================================================
// Spreading, FP64 plain path (64 threads, items of up to Q64 points)
// ===========================================================================
constexpr int Q64 = 8;

struct Spread64Lds {
    cx<double> sitem[64 * 2 * kMaxM];
    int ibin[64];
    int runS[64];
    int runE[64];
};

__device__ void spread64_wg(const PlanDesc &P, int cid, const cx<double> *__restrict__ f,
                            Spread64Lds &L)
{
    const Chunk ch = P.sp.chunks[cid];
    const int m = P.m1, tm = 2 * m;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int b = t; b < ch.nbin; b += nt) {
        L.runS[b] = -1;
        L.runE[b] = 0;
    }
    if (t < ch.nitem) {
        const Item it = P.sp.items[ch.item0 + t];
        double xf[Q64];
        cx<double> fv[Q64];
#pragma unroll
        for (int q = 0; q < Q64; ++q) {
            if (q < it.n) {
                const int p = it.p0 + q;
                xf[q] = P.sp.frac64[p];
                fv[q] = f[P.sp.perm[p]];
            } else {
                xf[q] = 0.0;
                fv[q] = cxmk(0.0, 0.0);
            }
        }
        const double inv_m = 1.0 / (double)m;
        for (int r = 0; r < tm; ++r) {
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int q = 0; q < Q64; ++q) {
                if (q < it.n) {
                    const double w = omega64(((double)(r - m + 1) - xf[q]) * inv_m, P.beta1, P.inv_den1);
                    ar = fma(fv[q].re, w, ar);
                    ai = fma(fv[q].im, w, ai);
                }
            }
            L.sitem[t * tm + r] = cxmk(ar, ai);
        }
        L.ibin[t] = it.bin - ch.bin_lo;
    }
    __syncthreads();
    if (t < ch.nitem) {
        const int b = L.ibin[t];
        if (t == 0 || L.ibin[t - 1] != b) L.runS[b] = t;
        if (t == ch.nitem - 1 || L.ibin[t + 1] != b) L.runE[b] = t + 1;
    }
    __syncthreads();
    const int W = ch.nbin + tm - 1;
    double2 *part = reinterpret_cast<double2 *>(P.partial) + ch.part_off;
    for (int w = t; w < W; w += nt) {
        const int blo = max(0, w - tm + 1), bhi = min(ch.nbin - 1, w);
        double ar = 0.0, ai = 0.0;
        for (int b = blo; b <= bhi; ++b) {
            const int s = L.runS[b];
            if (s < 0) continue;
            const int e = L.runE[b];
            for (int i = s; i < e; ++i) {
                const cx<double> v = L.sitem[i * tm + (w - b)];
                ar += v.re;
                ai += v.im;
            }
        }
        part[w] = make_double2(ar, ai);
    }
}

__global__ __launch_bounds__(64) void k_spread64(PlanDesc P, const cx<double> *__restrict__ f)
{
    __shared__ Spread64Lds L;
    const int cid = P.sp.sched[blockIdx.x];
    if (cid < 0) return;
    spread64_wg(P, cid, f, L);
}

// ===========================================================================
// Interpolation
// ===========================================================================
struct Interp32Lds {
    cx<float> Hb[256 * (kDeg + 1)];
    int ibin[256];
    int used[256];
};

__device__ void interp32_wg(const PlanDesc &P, int cid, cx<float> *__restrict__ y, Interp32Lds &L)
{
    constexpr int D = kDeg;
    const Chunk ch = P.ip.chunks[cid];
    const int m = P.m2, tm = 2 * m;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int b = t; b < ch.nbin; b += nt) L.used[b] = 0;
    __syncthreads();
    Item it;
    it.n = 0;
    if (t < ch.nitem) {
        it = P.ip.items[ch.item0 + t];
        const int b = it.bin - ch.bin_lo;
        L.ibin[t] = b;
        L.used[b] = 1;
    }
    __syncthreads();
    // Phase B: per used bin, H_k = sum_r C2[r][k] h_{c - m + 1 + r}
    const cx<float> *h = reinterpret_cast<const cx<float> *>(P.hlin);
    for (int b = t; b < ch.nbin; b += nt) {
        if (!L.used[b]) continue;
        const int lab = ch.bin_lo + b - P.ip_off;
        const int s0 = lab - m + 1 + P.N2 / 2;
        float Hr[D + 1], Hi[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) Hr[k] = Hi[k] = 0.f;
        for (int r = 0; r < tm; ++r) {
            const cx<float> hv = h[s0 + r];
            const float *c = P.C2 + r * (D + 1);
#pragma unroll
            for (int k = 0; k <= D; ++k) {
                Hr[k] = fmaf(c[k], hv.re, Hr[k]);
                Hi[k] = fmaf(c[k], hv.im, Hi[k]);
            }
        }
#pragma unroll
        for (int k = 0; k <= D; ++k) L.Hb[b * (D + 1) + k] = cxmk(Hr[k], Hi[k]);
    }
    __syncthreads();
    // Phase C: per point, y = (sum_k H_k T_k(t)) / phi_hat_1(N* x)
    if (t < ch.nitem) {
        const int b = L.ibin[t];
        const int lab = ch.bin_lo + b - P.ip_off;
        float Hr[D + 1], Hi[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            const cx<float> v = L.Hb[b * (D + 1) + k];
            Hr[k] = v.re;
            Hi[k] = v.im;
        }
        for (int p = it.p0; p < it.p0 + it.n; ++p) {
            const float fr = P.ip.frac32[p];
            const float yv = fmaf(2.f, fr, -1.f);
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
            const double corr = inv_phi1(P, lab, (double)fr);
            y[P.ip.perm[p]] = cxmk((float)((double)sr * corr), (float)((double)si * corr));
        }
    }
}

__global__ __launch_bounds__(256) void k_interp32(PlanDesc P, cx<float> *__restrict__ y)
{
    __shared__ Interp32Lds L;
    const int cid = P.ip.sched[blockIdx.x];
    if (cid < 0) return;
    interp32_wg(P, cid, y, L);
}

struct Interp64Lds {
    cx<double> hw[64 * 2 * kMaxM];
    int ibin[64];
    int used[64];
};

__device__ void interp64_wg(const PlanDesc &P, int cid, cx<double> *__restrict__ y, Interp64Lds &L)
{
    const Chunk ch = P.ip.chunks[cid];
    const int m = P.m2, tm = 2 * m;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int b = t; b < ch.nbin; b += nt) L.used[b] = 0;
    __syncthreads();
    Item it;
    it.n = 0;
    if (t < ch.nitem) {
        it = P.ip.items[ch.item0 + t];
        const int b = it.bin - ch.bin_lo;
        L.ibin[t] = b;
        L.used[b] = 1;
    }
    __syncthreads();
    const cx<double> *h = reinterpret_cast<const cx<double> *>(P.hlin);
    for (int b = t; b < ch.nbin; b += nt) {
        if (!L.used[b]) continue;
        const int lab = ch.bin_lo + b - P.ip_off;
        const int s0 = lab - m + 1 + P.N2 / 2;
        for (int r = 0; r < tm; ++r) L.hw[b * tm + r] = h[s0 + r];
    }
    __syncthreads();
    if (t < ch.nitem) {
        const int b = L.ibin[t];
        const int lab = ch.bin_lo + b - P.ip_off;
        const double inv_m = 1.0 / (double)m;
        for (int p = it.p0; p < it.p0 + it.n; ++p) {
            const double fr = P.ip.frac64[p];
            double sr = 0.0, si = 0.0;
            for (int r = 0; r < tm; ++r) {
                const double w = omega64((fr + (double)(m - 1 - r)) * inv_m, P.beta2, P.inv_den2);
                const cx<double> hv = L.hw[b * tm + r];
                sr = fma(hv.re, w, sr);
                si = fma(hv.im, w, si);
            }
            const double corr = inv_phi1(P, lab, fr);
            y[P.ip.perm[p]] = cxmk(sr * corr, si * corr);
        }
    }
}

__global__ __launch_bounds__(64) void k_interp64(PlanDesc P, cx<double> *__restrict__ y)
{
    __shared__ Interp64Lds L;
    const int cid = P.ip.sched[blockIdx.x];
    if (cid < 0) return;
    interp64_wg(P, cid, y, L);
}

// ===========================================================================
// FFT (steps 2-3)
// ===========================================================================
constexpr int kFftVals = 4096;   // complex values per FFT workgroup

// FFT input element q (index mod N2) = merged, deconvolved step-1 output:
// label l = q (q < N2/2) or q - N2; zero outside I_{G1}.
__device__ __forceinline__ cx<float> fft_input32(const PlanDesc &P, int q)
{
    const int lab = (q < P.N2 / 2) ? q : q - P.N2;
    if (lab < -P.G1 / 2 || lab >= P.G1 / 2) return cxmk(0.f, 0.f);
    const int cell = lab + P.G1 / 2;
    const float4 *part = reinterpret_cast<const float4 *>(P.partial);
    float hr = 0.f, hi = 0.f, lr = 0.f, li = 0.f;
    const int e1 = P.merge_off[cell + 1];
    for (int e = P.merge_off[cell]; e < e1; ++e) {
        const float4 v = part[P.merge_idx[e]];
        comp_add(hr, lr, v.x);
        comp_add(hi, li, v.y);
        lr += v.z;
        li += v.w;
    }
    const double sc = P.deconv[cell];
    return cxmk((float)((double)(hr + lr) * sc), (float)((double)(hi + li) * sc));
}

__device__ __forceinline__ cx<double> fft_input64(const PlanDesc &P, int q)
{
    const int lab = (q < P.N2 / 2) ? q : q - P.N2;
    if (lab < -P.G1 / 2 || lab >= P.G1 / 2) return cxmk(0.0, 0.0);
    const int cell = lab + P.G1 / 2;
    const double2 *part = reinterpret_cast<const double2 *>(P.partial);
    double ar = 0.0, ai = 0.0;
    const int e1 = P.merge_off[cell + 1];
    for (int e = P.merge_off[cell]; e < e1; ++e) {
        const double2 v = part[P.merge_idx[e]];
        ar += v.x;
        ai += v.y;
    }
    const double sc = P.deconv[cell];
    return cxmk(ar * sc, ai * sc);
}

template <typename T>
__device__ __forceinline__ cx<T> fft_input(const PlanDesc &P, int q);
template <>
__device__ __forceinline__ cx<float> fft_input<float>(const PlanDesc &P, int q) { return fft_input32(P, q); }
template <>
__device__ __forceinline__ cx<double> fft_input<double>(const PlanDesc &P, int q) { return fft_input64(P, q); }

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
// (src[b * Lsub + j]) into dst.  Twiddle exp(-2 pi i e / Lsub) = tw[e * tstride].
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

// Transforms the B length-Lsub sequences in buf[0] in place (result ends up in
// buf[0] or buf[1]; the returned pointer tells which).
template <typename T>
__device__ cx<T> *stockham(cx<T> *buf0, cx<T> *buf1, int Lsub, int B, const int *rad, int npass,
                           const cx<T> *__restrict__ tw, int tstride)
{
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
__device__ __forceinline__ void fft_store(const PlanDesc &P, int k, cx<T> v)
{
    cx<T> *h = reinterpret_cast<cx<T> *>(P.hlin);
    const int half = P.N2 / 2;
    const int s = (k < half) ? k : k - P.N2;
    const int S = P.fft.S;
    if (s >= -S && s <= S) h[s + half] = v;
    if (k == half && half <= S) h[P.N2] = v;   // label +N2/2 equals label -N2/2
}

template <typename T>
struct FftLds {
    cx<T> buf[2][kFftVals];
};

// Whole transform in one workgroup (N2 <= kFftVals)
template <typename T>
__global__ __launch_bounds__(256) void k_fft_single(PlanDesc P)
{
    __shared__ FftLds<T> L;
    const int N2 = P.N2;
    for (int q = threadIdx.x; q < N2; q += blockDim.x) L.buf[0][q] = fft_input<T>(P, q);
    __syncthreads();
    const cx<T> *tw = reinterpret_cast<const cx<T> *>(P.tw);
    cx<T> *res = stockham<T>(L.buf[0], L.buf[1], N2, 1, P.fft.radA, P.fft.npassA, tw, 1);
    for (int k = threadIdx.x; k < N2; k += blockDim.x) fft_store<T>(P, k, res[k]);
}

// Four-step stage A: for columns j1, length-n2 transforms over j2 of
// x[j1 + n1 j2], times exp(-2 pi i j1 k2 / N2), stored to Y[j1 n2 + k2].
template <typename T>
__global__ __launch_bounds__(256) void k_fft_stageA(PlanDesc P)
{
    __shared__ FftLds<T> L;
    const int n1 = P.fft.n1, n2 = P.fft.n2, B = P.fft.batchA;
    const int j1_0 = blockIdx.x * B;
    const int nb = min(B, n1 - j1_0);
    for (int idx = threadIdx.x; idx < nb * n2; idx += blockDim.x) {
        const int j2 = idx / nb, bl = idx - j2 * nb;
        L.buf[0][bl * n2 + j2] = fft_input<T>(P, j1_0 + bl + n1 * j2);
    }
    __syncthreads();
    const cx<T> *tw = reinterpret_cast<const cx<T> *>(P.tw);
    cx<T> *res = stockham<T>(L.buf[0], L.buf[1], n2, nb, P.fft.radA, P.fft.npassA, tw, n1);
    cx<T> *Y = reinterpret_cast<cx<T> *>(P.Y);
    for (int idx = threadIdx.x; idx < nb * n2; idx += blockDim.x) {
        const int bl = idx / n2, k2 = idx - bl * n2;
        const int j1 = j1_0 + bl;
        Y[(size_t)j1 * n2 + k2] = cmul(res[bl * n2 + k2], tw[j1 * k2]);
    }
}

// Four-step stage B: for columns k2, length-n1 transforms over j1 of
// Y[j1 n2 + k2]; output k1 is X[k2 + n2 k1].
template <typename T>
__global__ __launch_bounds__(256) void k_fft_stageB(PlanDesc P)
{
    __shared__ FftLds<T> L;
    const int n1 = P.fft.n1, n2 = P.fft.n2, B = P.fft.batchB;
    const int k2_0 = blockIdx.x * B;
    const int nb = min(B, n2 - k2_0);
    const cx<T> *Y = reinterpret_cast<const cx<T> *>(P.Y);
    for (int idx = threadIdx.x; idx < nb * n1; idx += blockDim.x) {
        const int j1 = idx / nb, bl = idx - j1 * nb;
        L.buf[0][bl * n1 + j1] = Y[(size_t)j1 * n2 + k2_0 + bl];
    }
    __syncthreads();
    const cx<T> *tw = reinterpret_cast<const cx<T> *>(P.tw);
    cx<T> *res = stockham<T>(L.buf[0], L.buf[1], n1, nb, P.fft.radB, P.fft.npassB, tw, n2);
    for (int idx = threadIdx.x; idx < nb * n1; idx += blockDim.x) {
        const int bl = idx / n1, k1 = idx - bl * n1;
        fft_store<T>(P, k2_0 + bl + n2 * k1, res[bl * n1 + k1]);
    }
}

// ===========================================================================
// Launchers
// ===========================================================================
template <typename T>
static void launch_fft(const PlanDesc &P, hipStream_t s)
{
    if (P.fft.n1 == 1) {
        hipLaunchKernelGGL((k_fft_single<T>), dim3(1), dim3(kFftThreads), 0, s, P);
    } else {
        const int gA = (P.fft.n1 + P.fft.batchA - 1) / P.fft.batchA;
        const int gB = (P.fft.n2 + P.fft.batchB - 1) / P.fft.batchB;
        hipLaunchKernelGGL((k_fft_stageA<T>), dim3(gA), dim3(kFftThreads), 0, s, P);
        hipLaunchKernelGGL((k_fft_stageB<T>), dim3(gB), dim3(kFftThreads), 0, s, P);
    }
}

hipError_t launch_exec(const PlanDesc &P, const void *f, void *y, hipStream_t s)
{
    if (P.prec == NNFFT_FP32_COMP) {
        const cx<float> *fin = reinterpret_cast<const cx<float> *>(f);
        if (2 * P.m1 <= 16)
            hipLaunchKernelGGL((k_spread32<16>), dim3(P.sp.ngrid), dim3(P.items_per_wg), 0, s, P, fin);
        else
            hipLaunchKernelGGL((k_spread32<32>), dim3(P.sp.ngrid), dim3(P.items_per_wg), 0, s, P, fin);
        launch_fft<float>(P, s);
        hipLaunchKernelGGL(k_interp32, dim3(P.ip.ngrid), dim3(P.items_per_wg), 0, s, P,
                           reinterpret_cast<cx<float> *>(y));
    } else {
        hipLaunchKernelGGL(k_spread64, dim3(P.sp.ngrid), dim3(P.items_per_wg), 0, s, P,
                           reinterpret_cast<const cx<double> *>(f));
        launch_fft<double>(P, s);
        hipLaunchKernelGGL(k_interp64, dim3(P.ip.ngrid), dim3(P.items_per_wg), 0, s, P,
                           reinterpret_cast<cx<double> *>(y));
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
