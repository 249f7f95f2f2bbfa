// Internal declarations shared by the host plan code and the HIP kernels of
// the NNFFT library.  Not part of the public C ABI (include/nnfft.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace nnfft {

// Degree of the Chebyshev series that represent each window tap on the FP32
// path (Algorithm 2.2 step 0 (ii)/(iii): the tap values phi_1(l/N1 - v_k)
// and phi_2(x_j/sigma1 - s/N2) as functions of the fractional grid offset).
constexpr int kDeg = 8;
constexpr int kMaxM = 16;           // largest truncation parameter m
constexpr int kMaxCorrDeg = 48;     // largest degree of the 1/phi_hat_1 series
constexpr int kCorr32 = 32;         // FP32 path: the series is zero-padded to this degree
constexpr int kMaxPasses = 20;      // radix passes of one sub-transform
constexpr int kItemsPerWg = 64;     // items (= threads) of a spreading / interpolation workgroup
constexpr int kMaxPlanes = 16;      // colours of spreading windows with fixed offsets

// One work item: up to Q consecutive sorted points of one cell bin.
struct Item {
    int32_t bin;      // bin (cell) storage index
    int32_t p0;       // first sorted point
    int32_t n;        // number of points (0: padding item)
    int32_t maxrun;   // first item of a chunk: the most items of one bin in the
                      // chunk (the spreading kernels choose how to sum a bin
                      // by it); 0 elsewhere
};

// One workgroup's share: up to 64 consecutive items of one node block with
// bins in [bin_lo, bin_lo + nbin), nbin <= 64.  Its items are stored at
// items[64 g .. 64 g + 63] for launch slot g (padding items have n = 0).
struct Chunk {
    int32_t nitem;
    int32_t bin_lo;
    int32_t nbin;
    int32_t part_off;   // spreading side: < 0: the window is in plane -part_off - 1 (cells
                        // in slot order); >= 0: overflow window at this partial index
};

// FP32 point record: the caller's index and the fractional offset of the
// node in its cell, read with one 8-byte load.  Records are stored per launch
// slot transposed, `rows` rows per slot: point q of item t of slot g is at
// (g rows + q) 64 + t, so a wavefront's load of one row is contiguous and its
// address does not depend on any other load (rows q >= n of an item repeat
// its last record).
struct alignas(8) PtRec {
    int32_t perm;
    float frac;
};

// Step 1 (spreading) arguments of one plan.
struct SpreadArgs {
    const Item *items;        // [ngrid * 64]
    const Chunk *chunks;      // [ngrid], launch order (XCD-aware); nitem = 0: idle
    const PtRec *rec32;       // FP32 path records
    const int32_t *perm;      // FP64 path: caller's index
    const double *frac64;     // FP64 path: offset in the cell
    const double *wts;        // null, or [M] weights the coefficients are multiplied
                              // by as they are loaded (set per exec)
    const float *C;           // FP32 path: [2m][kDeg + 1] tap coefficients
    const double *T64;        // FP64 path, B-spline windows: [2m][2m] exact tap series;
                              // Kaiser-Bessel windows: [nser] power series in 1 - u^2
    void *partial;            // chunk windows: float4 (hi, lo) or double2
    double beta, inv_den;     // FP64 path window: beta, 1 / (1 - exp(-2 beta)) (sinh)
    int32_t m, ngrid;
    int32_t rows;             // FP32 path: record rows per slot (max points per item)
    int32_t window;           // nnfft_window
    int32_t slotT, slotP;     // plane cell c at slot (c mod T) P + c div T
    int32_t nser;             // FP64 path, Kaiser-Bessel windows: terms of T64
};

// Steps 2-3 (merge, 1/phi_hat_2, FFT) arguments of one plan.
struct FftArgs {
    const void *partial;      // nplanes planes of G1 cells, then overflow windows
    const int32_t *merge_off; // [G1 + 1] CSR over grid cells of overflow partial indices
    const int32_t *merge_idx;
    const double *deconv;     // NNFFT: [G1] 1 / (N1 N2 phi_hat_2(l)), l = cell - G1/2;
                              // NFFT: [N] 1 / (n phi_hat(k)), k + N/2
    const void *tw;           // [N2] exp(-2 pi i q / N2) (float2 or double2)
    const void *twA;          // four-step: [n2] exp(-2 pi i k / n2)
    const void *twB;          // four-step: [n1] exp(-2 pi i k / n1)
    const void *tw4;          // four-step: [n1][n2] exp(-2 pi i j1 k2 / N2)
    void *Y;                  // [N2] four-step intermediate
    void *hlin;               // [2 S + 1] h_s at index s + h_off for |s| <= S
    const void *dense_in;     // mode 1: the NFFT coefficients f_k; mode 3: the inputs at
                              // labels l in I_G1, index l + G1/2 (set per exec)
    void *dense_out;          // mode 2: the adjoint NFFT output h_k (set per exec)
    int32_t N2, G1;
    int32_t n1, n2;           // N2 = n1 * n2; n1 == 1: one workgroup does it all
    int32_t batchA, batchB;   // sub-transforms per workgroup in stage A / B
    int32_t threadsA, threadsB;
    int32_t S;                // outputs with |s| <= S are consumed by step 4
    int32_t h_off;            // hlin index of label 0
    int32_t mode;             // 0 NNFFT, 1 NFFT, 2 adjoint NFFT, 3 dense NNFFT input (see fft_input32)
    int32_t Nout;             // NFFT: number of frequencies N
    int32_t npassA, npassB;
    int32_t fusedB;           // 1: no stage B launch, interpolation folds it in
    int32_t nplanes;          // planes of spreading windows summed for every cell
    int32_t slotT, slotP;     // plane cell c at slot (c mod T) P + c div T
    int8_t radA[kMaxPasses];  // radices of the length-n2 transform (or of N2)
    int8_t radB[kMaxPasses];  // radices of the length-n1 transform
};

// Step 4 + output (interpolation, 1/phi_hat_1) arguments of one plan.
struct InterpArgs {
    const Item *items;        // [ngrid * 64]
    const Chunk *chunks;      // [ngrid]
    const PtRec *rec32;
    const int32_t *perm;
    const double *frac64;
    const float *C;           // FP32 path: [2m][kDeg + 1] tap coefficients
    const double *T64;        // FP64 path, B-spline windows: [2m][2m] exact tap series;
                              // Kaiser-Bessel windows: [nser] power series in 1 - u^2
    const double *corr;       // series of 1/phi_hat_1 in t = 8 x^2 - 1 (FP32: kCorr32 + 1 terms)
    const void *hlin;
    // second four-step stage folded into the window load (fusedB > 0): h_s =
    // sum_{j1 < n1} Y[k2 n1 + j1] exp(-2 pi i j1 k1 / n1), k = s mod N2 =
    // k2 + n2 k1, with Y the first stage's output and twB its [n1] twiddles
    const void *Y;
    const void *twB;
    int32_t fusedB, fn2;      // n1 (0: read hlin) and n2 of the fold
    double beta, inv_den;
    double u_to_x;            // x_j = u_j * u_to_x, u_j = N2 N* x_j / N1
    int32_t m, ngrid;
    int32_t N2, ip_off;       // bin storage index = floor(u_j) + ip_off
    int32_t corr_deg;
    int32_t rows;             // FP32 path: record rows per slot
    int32_t h_off;            // hlin index of label 0
    int32_t window;           // nnfft_window
    int32_t nser;             // FP64 path, Kaiser-Bessel windows: terms of T64
};

// Pre-merge of long merge lists (crowded cells covered by many overflow
// windows): segment s sums the partial cells idx[seg[2 s] ..][0 .. seg[2 s + 1])
// of one grid cell into partial cell base + s, which the cell's merge list
// names instead, so no FFT thread walks a long list.
struct PreMergeArgs {
    void *partial;            // the plan's partial cells (the spreading output)
    const int32_t *seg;       // [2 nseg]: first index in idx, count
    const int32_t *idx;
    int32_t nseg, base;
};

struct PlanDev {
    int32_t prec;             // nnfft_precision
    int32_t pad0, pad1;
    SpreadArgs sp;
    FftArgs fft;
    InterpArgs ip;
    PreMergeArgs pm;          // nseg = 0: none
};

// The middle operator of a fast sinc transform (the first plan's
// interpolation, the quadrature weights and the second plan's spreading as
// one banded map from the first FFT's outputs to the second FFT's inputs):
// row r (label r - G1/2) is out[r] = sum_{b < Wb} K[b][r] h_{lo[r] + b};
// workgroup g (rows kSincMidRows g ..) stages h at labels
// [base[g], base[g] + span[g]) in LDS (labels with |s| > S read as zero).
constexpr int kSincMidRows = 128;   // rows (= threads) per workgroup of the middle kernel
struct SincMidArgs {
    InterpArgs h;             // the first plan's access to its FFT outputs
    const double *K;          // [Wb][G1]
    const int32_t *lo;        // [G1]
    const int32_t *base;      // [nwg]
    const int32_t *span;      // [nwg]
    void *out;                // [G1] complex of the plan's precision
    int32_t G1, Wb, S, span_max, nwg;
};

// Batched launches: up to kMaxBatch plans of one precision per launch.  The
// table travels as the kernel argument; workgroups [start[p], start[p + 1])
// belong to plan p (start[p] is a multiple of 8, so a plan's local workgroup
// index has the same XCD residue as in a launch of its own).
constexpr int kMaxBatch = 32;
struct BatchTable {
    const PlanDev *desc[kMaxBatch];   // device copies of the plans' descriptors
    const void *in[kMaxBatch];        // f of each plan
    void *out[kMaxBatch];             // y of each plan
    int32_t start[kMaxBatch + 1];
    int32_t n;
};

// Kernel timing of one exec: every kernel of the exec is launched with a
// pair of events attached to its dispatch (hipExtLaunchKernel), so their
// elapsed time is the kernel's own execution on the device, without the
// gaps between kernels.  Filled in launch order.
constexpr int kMaxTimedKernels = 6;
enum KernelId : int32_t {
    KID_SPREAD32 = 0, KID_SPREAD64, KID_FFT_SINGLE, KID_FFT_A, KID_FFT_B, KID_INTERP32, KID_INTERP64, KID_SINC_MID,
    KID_PREMERGE, KID_COUNT
};
struct KernelTimes {
    hipEvent_t start[kMaxTimedKernels] = {}, stop[kMaxTimedKernels] = {};
    int32_t kid[kMaxTimedKernels] = {};
    int32_t n = 0;
};
const char *kernel_name(int kid);
int kernel_stage(int kid);   // 0 spreading, 1 FFT, 2 interpolation

// Kernel launchers (kernels.hip).  kt: null, or the event pairs of this exec.
hipError_t launch_exec(const PlanDev &P, const void *f, void *y, hipStream_t s, KernelTimes *kt);
// NFFT plans: forward (in = f_k, out = y_j) or adjoint (in = y_j, out = h_k)
hipError_t launch_nfft(const PlanDev &P, bool adjoint, const void *in, void *out, hipStream_t s);
// n plans of one precision: host descriptors (sizes) and their device copies
hipError_t launch_exec_batch(int n, const PlanDev *const *host, const PlanDev *const *dev,
                             const void *const *f, void *const *y, hipStream_t s);
hipError_t launch_scale_by_weights(int prec, const double *w, const void *src, void *dst, int64_t n,
                                   hipStream_t s);
// Fast sinc transform with its middle operator: spreading and FFT of P1 from
// c, the middle operator M, FFT of P2 from M.out and its interpolation to h.
hipError_t launch_sinc_middle(const PlanDev &P1, const SincMidArgs &M, const PlanDev &P2, const void *c, void *h,
                              hipStream_t s);

// Node preparation on the device (plan_device.hip): the key of node k of a
// side is (block << bbits) | bin; device_sort_nodes checks the domain (flag
// bit 0: a node outside [-1/2, 1/2] or NaN; bit 1: a bin outside [0, nbins)),
// adds the bin counts of every block to counts[block * nbins + bin] (zeroed
// by the caller) and sorts the caller indices stably by key into
// *sorted_idx (inside tmp, device_sort_tmp_bytes(M) bytes).
bool device_sort_fits(int64_t M, int64_t nbins, int64_t block);
size_t device_sort_tmp_bytes(int64_t M);
hipError_t device_sort_nodes(const double *x, int64_t M, double scale, int64_t off, int64_t nbins, int64_t block,
                             int32_t *counts, int32_t *flag, void *tmp, int32_t **sorted_idx, hipStream_t s);
// Both sides of a plan in one sort: side i's keys get i as the bit above the
// wider side's key bits, so the sorted order is side 0's (by its keys), then
// side 1's; the indices of each side count from 0 (*sorted_b = *sorted_a +
// a.M).  tmp: device_sort_tmp_bytes(a.M + b.M) bytes; counts and flag per
// side as for device_sort_nodes.
struct SortSide {
    const double *x;
    int64_t M;
    double scale;
    int64_t off, nbins, block;
    int32_t *counts, *flag;
};
bool device_sort_pair_fits(const SortSide &a, const SortSide &b);
hipError_t device_sort_node_pair(const SortSide &a, const SortSide &b, void *tmp, int32_t **sorted_a,
                                 int32_t **sorted_b, hipStream_t s);
// The records of the sorted points: FP64 caller index and cell offset, or
// FP32 (index, offset) records in sorted order.
hipError_t device_sorted_records(const double *x, const int32_t *sorted_idx, int64_t M, double scale, bool fp32,
                                 int32_t *perm, double *frac64, PtRec *rec32, hipStream_t s);
// The FP32 records in per-slot transposed blocks directly from the sorted
// indices: point q of item t of launch slot g at (g rows + q) 64 + t, rows
// past an item's end repeating its last record, empty items zero.
hipError_t device_transposed_records(const double *x, const int32_t *sorted_idx, double scale, const Item *launch_items,
                                     int64_t nslot, int rows, PtRec *trec32, hipStream_t s);
hipError_t device_gather(const double *x, const int64_t *idx, int64_t n, double *out, hipStream_t s);
// Both sides of a plan in one launch each: the records (FP32: transposed
// slot blocks into trec; FP64: perm and frac in sorted order) and the
// density samples.
struct RecSide {
    const double *x;
    const int32_t *idx;
    double scale;
    int64_t M;            // FP64: points
    const Item *items;    // FP32: launch slots' items
    int64_t nslot;
    int32_t rows;
    PtRec *trec;
    int32_t *perm;
    double *frac;
};
hipError_t device_records_pair(bool fp32, const RecSide &a, const RecSide &b, hipStream_t s);
hipError_t device_gather_pair(const double *x0, const int64_t *idx0, int64_t n0, double *out0, const double *x1,
                              const int64_t *idx1, int64_t n1, double *out1, hipStream_t s);

// Per-exec working memory of a plan (window planes and overflow windows, the
// four-step intermediate, the consumed FFT outputs), in bytes; the planes
// (the first plane_bytes of the window area) hold cells no window writes,
// which must read as zero.
struct ExecScratch {
    size_t part_bytes, plane_bytes, y_bytes, hlin_bytes;
};
// Largest working memory that nnfft_exec_noalloc takes from the library's
// static device array.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
// Bytes of the static array a plan needs (each part 256-byte aligned).
size_t static_scratch_need(const ExecScratch &sz);
// nnfft_exec with the working memory in the static device array of the
// current device (the plan's own scratch is not touched).  Returns
// hipErrorInvalidValue if the plan needs more than kStaticScratchBytes.
hipError_t launch_exec_static(const PlanDev &P, const ExecScratch &sz, const void *f, void *y, hipStream_t s);

}  // namespace nnfft
