// Host-side plan construction shared by the plan, autotuning and serving
// entry points (Algorithm 2.2 step 0 and the node preprocessing).  Not part
// of the public C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/nnfft.h"
#include "internal.h"

namespace nnfft {

// A failed HIP call inside plan construction (thrown by the plan code,
// turned into NNFFT_ERR_DEVICE at the C ABI).
struct HipError {
    hipError_t err;
    const char *what;
};

// Records the message for nnfft_last_error (thread-local) and returns st.
nnfft_status fail(nnfft_status st, const std::string &msg);

// Layout knobs of one node side: what the autotuner chooses.
struct Layout {
    int64_t block = 0;   // points per node block (consecutive caller indices)
    int Q = 0;           // max points per work item
};

// The tuned layout for M nodes if the table has one, else the rule.
// spreading: the layout of a spreading side (the rule takes larger node
// blocks there above 2^20 points; interpolation sides keep 2^17).
Layout choose_layout(int64_t M, bool fp32, bool spreading = true);
Layout rule_layout(int64_t M, bool fp32, bool spreading = true);
Layout choose_layout_nodes(const std::vector<double> &nodes, double scale, bool fp32, bool spreading);
void set_tuned_layout(bool fp32, int64_t M, const Layout &L);
bool get_tuned_layout(bool fp32, int64_t M, Layout &L);
void clear_tuned_layouts();
// Clamps a requested layout to what the kernels implement.
Layout sanitize_layout(Layout L, int64_t M, bool fp32);

// An allocator whose resize leaves new elements default-initialized (no
// zeroing), for buffers of trivial types the planner writes in full.
template <typename T>
struct UninitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = UninitAlloc<U>;
    };
    UninitAlloc() = default;
    template <typename U>
    UninitAlloc(const UninitAlloc<U> &) noexcept {}
    template <typename U>
    void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value)
    {
        ::new (static_cast<void *>(p)) U;
    }
    template <typename U, typename... Args>
    void construct(U *p, Args &&...args)
    {
        ::new (static_cast<void *>(p)) U(std::forward<Args>(args)...);
    }
};
using ItemBuf = std::vector<Item, UninitAlloc<Item>>;

// Node layout of one side, built on the host.
struct SideHost {
    std::vector<int32_t> perm;          // FP64: caller's index of each sorted point
    std::vector<PtRec> rec32;           // FP32: (index, offset) of each sorted point
    std::vector<double> frac64;         // FP64: offset of each sorted point
    std::vector<Chunk> chunks;
    std::vector<int32_t> chunk_block;
    std::vector<int32_t> chunk_item0;   // first item of each chunk in its block's items
    std::vector<Chunk> launch;          // chunks in launch order, empty ones pad
    ItemBuf launch_items;               // 64 items per launch slot, n = 0 pads
    std::vector<PtRec> trec32;          // FP32: records in per-slot transposed blocks
    int64_t part_cells = 0;             // spreading side: plane cells + overflow cells
    int64_t ovf_cells = 0;              // spreading side: cells of the overflow windows
    int32_t nplanes = 0;                // spreading side: colours of the windows
    int64_t nblocks = 0;
    int32_t rows = 0;                   // FP32: record rows per slot (the item size)
    bool dev = false;                   // records sorted and written on the device
    int64_t npts = 0;                   // points of the side
};

// Items and chunks of one node block (host schedule of a side).
struct BlockOut {
    ItemBuf items;
    std::vector<Chunk> chunks;
    std::vector<int32_t> item0;   // first item of each chunk, within the block
    bool ok = true;
};
void block_schedule(const int32_t *cnt, int64_t nbins, int64_t k0, int Q, BlockOut &o);
// (the blocks' items are consumed: copied into the launch slots and freed)
bool finish_side(std::vector<BlockOut> &outs, int m, SideHost &S, std::string &err);

// FFT factorization chosen at plan time (copied into FftArgs).
struct FftPlan {
    int32_t N2 = 0, n1 = 0, n2 = 0, npassA = 0, npassB = 0;
    int radA[kMaxPasses] = {}, radB[kMaxPasses] = {};
    int32_t batchA = 0, batchB = 0, threadsA = 0, threadsB = 0, S = 0;
    bool fusedB = false;   // stage B folded into the interpolation's window load
};

// Everything of one plan that is computed on the host, and the size of the
// single device block it needs.
struct HostPlan {
    nnfft_info_t info{};
    bool fp32 = false;
    Layout lay1{}, lay2{};
    SideHost sp, ip;
    std::vector<float> C1, C2;         // FP32: window tap series of both sides
    std::vector<double> T1, T2;        // FP64 B-spline windows: exact tap series of both sides
    std::vector<double> corr;          // series of 1/phi_hat_1
    std::vector<double> deconv;        // 1 / (N1 N2 phi_hat_2(l))
    std::vector<double> tw64;          // FFT twiddles
    std::vector<float> tw32;
    std::vector<double> twA, twB, tw4; // four-step tables (values of the plan's precision)
    int32_t slotT = 1, slotP = 0;      // plane cell c at slot (c mod T) P + c div T
    std::vector<int32_t> moff, midx;   // merge lists of the spreading windows
    std::vector<int32_t> pm_seg, pm_idx;   // pre-merge segments of long lists (PreMergeArgs)
    int64_t pm_base = 0, pm_cells = 0;     // their output cells: partial cells pm_base ..
    FftPlan fd{};
    int kind = 0;                      // 0 NNFFT, 1 NFFT with equispaced frequencies
    int64_t hlin_len = 0;              // FFT outputs kept for the interpolation
    int32_t h_off = 0;                 // their index of label 0
    size_t total_bytes = 0;            // device bytes of the plan (one block)
    size_t upload_bytes = 0;           // of which uploaded from the host image
};

// Provider of the plan's device block.
struct DevMem {
    void *(*alloc)(void *ctx, size_t bytes);   // null on failure
    void (*release)(void *ctx, void *p);
    void *ctx;
};
const DevMem &hip_mem();                       // hipMalloc / hipFree

}  // namespace nnfft

// Public handles (opaque in nnfft.h).
struct nnfft_plan_s {
    int kind = 0;                      // 0 NNFFT (nnfft_plan), 1 NFFT (nfft_plan)
    nnfft_info_t info{};
    nnfft::PlanDev desc{};
    nnfft::PlanDev *ddesc = nullptr;   // device copy of desc (batched launches)
    void *base = nullptr;              // the plan's device block
    nnfft::DevMem mem{};
    nnfft::ExecScratch scratch{};      // sizes of the per-exec working memory
    size_t upload_bytes = 0;           // tables, schedule and records at the block's start
    std::vector<nnfft::KernelTimes> prof;   // kernel event pairs of each profiled exec
    int prof_max = 0, prof_used = 0;

    void drop_events();
    ~nnfft_plan_s();
};

struct sinc_plan_s {
    nnfft_plan_t p1 = nullptr, p2 = nullptr;
    double *w = nullptr;      // [n_nodes] quadrature weights (FP64, device)
    void *g = nullptr;        // [n_nodes] complex intermediate
    void *wg_base = nullptr;  // device block of w and g (and of the middle operator)
    nnfft::SincMidArgs mid{}; // the middle operator (has_mid)
    bool has_mid = false;     // built at plan time
    bool use_mid = false;     // sinc_exec runs it (sinc_set_middle)
    nnfft::DevMem mem{};
    int64_t n_nodes = 0;
    int64_t L1 = 0, L2 = 0;   // input and output lengths
    int32_t prec = 0;
    bool step1_nfft = false;  // step 1 is an NFFT (a_k equispaced), step 3 an adjoint
    bool step3_nfft = false;  // NFFT (b_l = l / N): the special cases of Sec. 6
    ~sinc_plan_s();
};

namespace nnfft {

// Validations, tables and node layouts of Algorithm 2.2 step 0 from host
// copies of the nodes.  lay1 / lay2: null = choose_layout.
nnfft_status plan_host(HostPlan &H, int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2,
                       int m1, int m2, nnfft_precision prec, const std::vector<double> &v,
                       const std::vector<double> &x, const Layout *lay1 = nullptr,
                       const Layout *lay2 = nullptr, int window = NNFFT_WINDOW_SINH);

// NFFT with equispaced frequencies k in I_N at nodes x[M] (host copies):
// the same layout machinery with one node set on both sides.
nnfft_status nfft_plan_host(HostPlan &H, int64_t N, int64_t M, double sigma, int m, nnfft_precision prec,
                            const std::vector<double> &x);

// The records of a side whose nodes were sorted on the device: the nodes,
// the sorted caller indices and the grid scale.
struct DevSideRecords {
    const double *x = nullptr;
    const int32_t *sorted = nullptr;
    double scale = 0.0;
};
struct DevRecords {
    DevSideRecords sp, ip;
};

// Allocates H.total_bytes from mem, uploads (one copy, synchronizes s) and
// returns the handle, which releases the block to mem when destroyed.  With
// dev, the sides marked dev get their records written on the device.
nnfft_status plan_create(const HostPlan &H, const DevMem &mem, hipStream_t s, nnfft_plan_t *out,
                         const DevRecords *dev = nullptr);

// Device and pinned host memory of the node preparation, reused across plans
// (grown on demand, freed with the object).
struct NodePrepScratch {
    void *dev = nullptr;
    size_t dev_bytes = 0;
    void *pin = nullptr;
    size_t pin_bytes = 0;
    NodePrepScratch() = default;
    NodePrepScratch(const NodePrepScratch &) = delete;
    NodePrepScratch &operator=(const NodePrepScratch &) = delete;
    ~NodePrepScratch();
    bool reserve(size_t dev_need, size_t pin_need);
};

// Host plan of an NNFFT with device nodes v[M1], x[M2]: node order on the
// device, schedule and tables on the host; R (pointing into T) feeds
// plan_create, which must run before T is reused.  *host: the sort keys do
// not fit 32 bits, nothing was done, plan on the host instead.
nnfft_status plan_device_nodes(HostPlan &H, DevRecords &R, NodePrepScratch &T, int64_t N, int64_t M1, int64_t M2,
                               double sigma1, double sigma2, int m1, int m2, nnfft_precision prec, int window,
                               const double *v, const double *x, hipStream_t s, bool *host);

// FNV-1a hash of a byte range (layout digests).
uint64_t fnv1a64(const void *p, size_t n);

// Fast sinc transform (Algorithm 6.1) on the host: quadrature and both plans.
// The middle of Algorithm 6.1 as one operator: the first plan's
// interpolation at x_j = z_j / 2 with its 1/phi_hat_1 factors, the weights and
// the second plan's spreading from v_j = -z_j / 2 with its 1/phi_hat_2
// deconvolution are linear in the first FFT's outputs h_s and depend on the
// quadrature and the plan parameters only:
//   u_l = sum_s K[l][s] h_s,  l in I_G1 (the second FFT's input at label l),
//   K[l][s] = d(l) sum_j omega_1((l - t_j) / m1) w_j / phi_hat_1(N* x_j)
//                       omega_2((u_j - s) / m2),
// t_j = N1 N v_j / N*, u_j = N2 N* x_j / N1, d(l) = 1 / (N1 N2 phi_hat_2(l)).
// Row l (index l + G1/2) has its nonzero entries at labels s in
// [lo[l], lo[l] + Wb); workgroup g (rows 256 g ..) reads the labels
// [base[g], base[g] + span[g]).
struct SincMiddle {
    int32_t Wb = 0, span_max = 0, S = 0;
    std::vector<double> K;                   // [Wb][G1]
    std::vector<int32_t> lo, base, span;     // [G1], [nwg], [nwg]
};

struct SincHostPlan {
    HostPlan h1, h2;
    std::vector<double> w;
    SincMiddle mid;           // built when mid_ok
    bool mid_ok = false;
    int64_t n_nodes = 0;
    int64_t L1 = 0, L2 = 0;
    int32_t prec = 0;
    bool step1_nfft = false, step3_nfft = false;
    size_t wg_bytes = 0;
    size_t total_bytes = 0;   // both plans plus weights and intermediate
};
nnfft_status sinc_host(SincHostPlan &S, int64_t N, int64_t L1, int64_t L2, sinc_quad quad, int64_t n_quad,
                       double sigma1, double sigma2, int m1, int m2, nnfft_precision prec,
                       const std::vector<double> &a, const std::vector<double> &b, bool middle = false);
nnfft_status sinc_create(const SincHostPlan &S, const DevMem &mem, hipStream_t s, sinc_plan_t *out);

// Verifies the layout invariants the kernels rely on (no device work).
nnfft_status check_plan(const HostPlan &H, const std::vector<double> &v, const std::vector<double> &x);

// Device-to-host copy of n FP64 nodes (synchronizes s).
nnfft_status copy_nodes(const double *d, int64_t n, std::vector<double> &h, hipStream_t s);

}  // namespace nnfft
