// Internal declarations shared by the host plan code and the HIP kernels of
// the NNFFT library.  Not part of the public C ABI (include/nnfft.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace nnfft {

// Degree of the Chebyshev series that represent each window tap on the FP32
// path (Sec. 2, Algorithm 2.2 step 0 (ii)/(iii): the tap values
// phi_1(l/N1 - v_k) and phi_2(x_j/sigma1 - s/N2) as functions of the
// fractional grid offset).
constexpr int kDeg = 8;
constexpr int kMaxM = 16;           // largest truncation parameter m
constexpr int kMaxCorrDeg = 48;     // largest degree of the 1/phi_hat_1 series
constexpr int kMaxPasses = 20;      // radix passes of one sub-transform
constexpr int kFftThreads = 256;    // threads of every FFT workgroup
constexpr int kFftLds = 16384;      // complex values held in LDS by one FFT workgroup (FP32)

// One work item: up to Q consecutive sorted points of one cell bin.
struct Item {
    int32_t bin;   // bin (cell) storage index
    int32_t p0;    // first sorted point
    int32_t n;     // number of points
    int32_t pad;
};

// One workgroup's share: consecutive items of one node block, bins
// [bin_lo, bin_lo + nbin), nbin <= items per workgroup.
struct Chunk {
    int32_t item0;
    int32_t nitem;
    int32_t bin_lo;
    int32_t nbin;
    int32_t part_off;   // spreading side: first partial cell of this chunk
    int32_t pad0, pad1, pad2;
};

// Node records of one side (spreading: v_k; interpolation: x_j).
struct SideDesc {
    const Item *items;
    const Chunk *chunks;
    const int32_t *sched;     // workgroup -> chunk id (-1: idle), XCD-aware order
    const int32_t *perm;      // sorted position -> caller's index
    const float *frac32;      // fractional offset in the cell (FP32 path)
    const double *frac64;     // fractional offset in the cell (FP64 path)
    int32_t ngrid;            // workgroups of the launch
    int32_t nchunks;
};

struct FftDesc {
    int32_t N2;               // transform length
    int32_t n1, n2;           // N2 = n1 * n2; n1 == 1: one workgroup does it all
    int32_t npassA, npassB;   // passes of the length-n2 and length-n1 transforms
    int32_t radA[kMaxPasses]; // radices of the length-n2 transform (or of N2)
    int32_t radB[kMaxPasses]; // radices of the length-n1 transform
    int32_t batchA, batchB;   // sub-transforms per workgroup in stage A / B
    int32_t S;                // outputs with |s| <= S are consumed by step 4
    int32_t pad;
};

// Everything the kernels of one plan read.  Passed by value as a kernel
// argument (single plan) or stored in device memory (batched launches).
struct PlanDesc {
    int32_t prec;             // nnfft_precision
    int32_t m1, m2;
    int32_t G1, N2;
    int32_t corr_deg;         // degree of the 1/phi_hat_1 Chebyshev series
    int32_t ip_off;           // interpolation bin storage index = floor(u) + ip_off
    int32_t items_per_wg;     // threads of spreading / interpolation workgroups
    double beta1, beta2;
    double inv_den1, inv_den2;   // 1 / (1 - exp(-2 beta_j)), exact sinh ratio
    double u_to_x;               // x_j = u_j * u_to_x, u_j = N2 N* x_j / N1
    SideDesc sp, ip;
    const float *C1;          // FP32: [2 m1][kDeg + 1] tap coefficients, spreading
    const float *C2;          // FP32: [2 m2][kDeg + 1] tap coefficients, interpolation
    const double *corr;       // [corr_deg + 1] series of 1/phi_hat_1 in t = 8 x^2 - 1
    const double *deconv;     // [G1] 1 / (N1 N2 phi_hat_2(l)), l = cell - G1/2
    const int32_t *merge_off; // [G1 + 1] CSR over grid cells of partial indices
    const int32_t *merge_idx;
    const void *tw;           // [N2] exp(-2 pi i q / N2) (float2 or double2)
    void *partial;            // spreading partials (float4 hi/lo or double2)
    void *X;                  // [N2] FFT input / stage-B output staging
    void *Y;                  // [N2] four-step intermediate
    void *hlin;               // [N2 + 1] h_s at index s + N2/2, consumed part only
    FftDesc fft;
};

// Kernel launchers (kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_exec(const PlanDesc &P, const void *f, void *y, hipStream_t s);
hipError_t launch_exec_batch(int n, const PlanDesc *const *descs, const PlanDesc *d_descs,
                             const void *const *f, void *const *y, hipStream_t s);

}  // namespace nnfft
