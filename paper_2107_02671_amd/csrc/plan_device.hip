// Node preparation of Algorithm 2.2 step 0 on the device: the (cell, offset)
// split of every node in FP64, the domain check, the bin counts of every node
// block and the stable sort of the nodes by (block, bin), and the sorted and
// per-slot transposed point records the exec kernels read.
//
// A side's nodes x[M] (FP64, device) have grid coordinates t_k = scale x_k,
// cell c_k = floor(t_k) and offset t_k - c_k in [0, 1); bin = c_k + off in
// [0, nbins).  Node block b holds the caller indices [b B, (b + 1) B).  The
// sort key of node k is (block << bbits) | bin, so a stable sort of the
// indices by key is the per-block stable counting sort by bin: the host
// builds the items and chunks from the counts alone, and the positions of
// the points agree with the host layout exactly.
//
// Stable sort: least-significant-digit radix sort, 8-bit digits, over the
// key bits in use.  Each pass: per-tile digit histograms (tile = 1024
// elements), an exclusive scan of each digit's row over the tiles (one
// workgroup per digit) with the row totals, and a scatter that starts each
// digit at the prefix of the totals plus its row scan and ranks the
// elements of a tile in index order (ballot match within a wavefront,
// per-wave counts in LDS across wavefronts).  The bin counts are then read
// off the sorted keys: the length of each key's run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.h"

namespace nnfft {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;                            // elements per thread and tile
constexpr int kTile = kSortThreads * kSortItems;          // 1024
constexpr int kRadix = 256;
constexpr int kSortWaves = kSortThreads / 64;

// cell of t by truncation stepped down for negative non-integers: the exact
// floor for |t| <= 2^52 (the host layout uses the same expression)
__device__ __forceinline__ double cell_floor(double t)
{
    const double tr = (double)(long long)t;
    return tr > t ? tr - 1.0 : tr;
}

// keys[k] = keyor | (block << bbits) | bin, vals[k] = k; flag bit 0: a node
// outside [-1/2, 1/2] (or NaN), bit 1: a bin outside [0, nbins) (then the key
// uses bin 0 and the plan is refused)
__device__ __forceinline__ void node_key(const double *__restrict__ x, int64_t k, double scale, int64_t off,
                                         int64_t nbins, int64_t block, int bbits, uint32_t keyor,
                                         uint32_t *__restrict__ key, int32_t *__restrict__ val,
                                         int32_t *__restrict__ flag)
{
#pragma clang fp contract(off)
    const double v = x[k];
    int fl = 0;
    if (!(fabs(v) <= 0.5)) fl |= 1;
    const double t = scale * v;
    int64_t bin = 0;
    if (fl == 0) {
        bin = (int64_t)cell_floor(t) + off;
        if (bin < 0 || bin >= nbins) fl |= 2;
    }
    if (fl != 0) {
        atomicOr(flag, fl);
        bin = 0;
    }
    const int64_t blk = k / block;
    *key = keyor | ((uint32_t)blk << bbits) | (uint32_t)bin;
    *val = (int32_t)k;
}

__global__ void k_node_keys(const double *__restrict__ x, int64_t M, double scale, int64_t off, int64_t nbins,
                            int64_t block, int bbits, uint32_t keyor, uint32_t *__restrict__ keys,
                            int32_t *__restrict__ vals, int32_t *__restrict__ flag)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < M; k += (int64_t)gridDim.x * blockDim.x)
        node_key(x, k, scale, off, nbins, block, bbits, keyor, keys + k, vals + k, flag);
}

// the keys of both sides of a plan in one launch: side 1's at [a.M, a.M + b.M)
struct KeySide {
    const double *x;
    int64_t M;
    double scale;
    int64_t off, nbins, block;
    int bbits;
    uint32_t keyor;
    int32_t *flag;
};

__global__ void k_node_keys_pair(KeySide a, KeySide b, uint32_t *__restrict__ keys, int32_t *__restrict__ vals)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.M + b.M;
         p += (int64_t)gridDim.x * blockDim.x) {
        if (p < a.M)
            node_key(a.x, p, a.scale, a.off, a.nbins, a.block, a.bbits, a.keyor, keys + p, vals + p, a.flag);
        else
            node_key(b.x, p - a.M, b.scale, b.off, b.nbins, b.block, b.bbits, b.keyor, keys + p, vals + p, b.flag);
    }
}

// Bin counts from the sorted keys: counts[block * nbins + bin] = length of
// the key's run.  Run starts store their position, run ends (a later
// launch) replace it by the length.
__global__ void k_run_starts(const uint32_t *__restrict__ keys, int64_t M, int bbits, int64_t nbins,
                             int32_t *__restrict__ counts)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = keys[p];
        if (p == 0 || keys[p - 1] != k)
            counts[(int64_t)(k >> bbits) * nbins + (k & ((1u << bbits) - 1u))] = (int32_t)p;
    }
}

__global__ void k_run_ends(const uint32_t *__restrict__ keys, int64_t M, int bbits, int64_t nbins,
                           int32_t *__restrict__ counts)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = keys[p];
        if (p == M - 1 || keys[p + 1] != k) {
            int32_t *c = &counts[(int64_t)(k >> bbits) * nbins + (k & ((1u << bbits) - 1u))];
            *c = (int32_t)(p + 1) - *c;
        }
    }
}

// Both sides sorted together: side i's keys carry i at bit kb above its own
// (block << bbits_i) | bin; the count of a run goes to that side's array.
struct RunPair {
    int32_t *counts[2];
    int64_t nbins[2];
    int bbits[2];
    int kb;
};

__device__ __forceinline__ int32_t *pair_cell(const RunPair &R, uint32_t k)
{
    const bool one = (k >> R.kb) != 0u;
    const uint32_t rest = k & ((1u << R.kb) - 1u);
    const int bb = one ? R.bbits[1] : R.bbits[0];
    int32_t *const c = one ? R.counts[1] : R.counts[0];
    return c + (int64_t)(rest >> bb) * (one ? R.nbins[1] : R.nbins[0]) + (rest & ((1u << bb) - 1u));
}

// the run lengths in one pass: the run's first position subtracts its
// index, its last adds its index + 1 (integer adds: the order of the two
// does not matter; counts zeroed by the caller)
__global__ void k_run_counts_pair(const uint32_t *__restrict__ keys, int64_t M, RunPair R)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = keys[p];
        const bool first = p == 0 || keys[p - 1] != k, last = p == M - 1 || keys[p + 1] != k;
        if (first || last) {
            int32_t *c = pair_cell(R, k);
            if (first) atomicAdd(c, -(int32_t)p);
            if (last) atomicAdd(c, (int32_t)(p + 1));
        }
    }
}

// digit histogram of each tile: hist[d * ntiles + tile]
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                             int64_t ntiles, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t cnt[kRadix];
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t e = base + (int64_t)r * kSortThreads + tid;
        if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * ntiles + blockIdx.x] = cnt[tid];
}

// exclusive scan of each digit's row hist[d * ntiles .. (d + 1) * ntiles) in
// place (workgroup d), the row total to tot[d]: segments of 256 x 16
// entries, each thread summing 16 consecutive ones, the thread sums scanned in
// LDS, a carry between segments
__global__ __launch_bounds__(kSortThreads) void k_radix_scan_rows(uint32_t *__restrict__ hist, int64_t ntiles,
                                                                  uint32_t *__restrict__ tot)
{
    __shared__ uint32_t sums[kSortThreads];
    const int tid = threadIdx.x;
    uint32_t *row = hist + (int64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int64_t seg = 0; seg < ntiles; seg += kSortThreads * 16) {
        const int64_t a = seg + (int64_t)tid * 16;
        uint32_t v[16];
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            v[i] = (a + i < ntiles) ? row[a + i] : 0u;
            s += v[i];
        }
        sums[tid] = s;
        __syncthreads();
        for (int d = 1; d < kSortThreads; d <<= 1) {   // inclusive scan of the thread sums
            const uint32_t add = tid >= d ? sums[tid - d] : 0u;
            __syncthreads();
            sums[tid] += add;
            __syncthreads();
        }
        uint32_t run = carry + (tid > 0 ? sums[tid - 1] : 0u);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (a + i < ntiles) row[a + i] = run;
            run += v[i];
        }
        carry += sums[kSortThreads - 1];
        __syncthreads();
    }
    if (tid == 0) tot[blockIdx.x] = carry;
}

// stable scatter of one tile: elements are ranked in index order (round r,
// then thread order) among the tile's elements of the same digit
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                                const int32_t *__restrict__ vin, int64_t n,
                                                                int shift, int64_t ntiles,
                                                                const uint32_t *__restrict__ offs,
                                                                const uint32_t *__restrict__ tot,
                                                                uint32_t *__restrict__ kout,
                                                                int32_t *__restrict__ vout)
{
    __shared__ uint32_t base_d[kRadix];           // tile's first output position of each digit
    __shared__ uint32_t wcnt[kSortWaves][kRadix];  // elements of each digit in each wave, this round
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // digit starts: exclusive scan of the digit totals (in wcnt[0] as scratch)
    wcnt[0][tid] = tot[tid];
    __syncthreads();
    for (int d = 1; d < kRadix; d <<= 1) {
        const uint32_t add = tid >= d ? wcnt[0][tid - d] : 0u;
        __syncthreads();
        wcnt[0][tid] += add;
        __syncthreads();
    }
    base_d[tid] = (tid > 0 ? wcnt[0][tid - 1] : 0u) + offs[(int64_t)tid * ntiles + blockIdx.x];
    __syncthreads();
    for (int w = 0; w < kSortWaves; ++w) wcnt[w][tid] = 0;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));   // lanes below this one
    const int64_t tbase = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kSortItems; ++r) {
        __syncthreads();   // base_d and wcnt settled (previous round's updates)
        const int64_t e = tbase + (int64_t)r * kSortThreads + tid;
        const bool valid = e < n;
        uint32_t key = 0;
        int32_t val = 0;
        if (valid) {
            key = kin[e];
            val = vin[e];
        }
        const uint32_t d = (key >> shift) & (kRadix - 1);
        // lanes of this wave holding the same digit
        uint64_t mask = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bb = __ballot(on);
            mask &= on ? bb : ~bb;
        }
        const int rank_w = __popcll(mask & lt);
        if (valid && rank_w == 0) wcnt[wave][d] = (uint32_t)__popcll(mask);
        __syncthreads();
        if (valid) {
            uint32_t pos = base_d[d] + (uint32_t)rank_w;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        // thread tid advances digit tid past this round and clears its counts
        uint32_t add = 0;
        for (int w = 0; w < kSortWaves; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        base_d[tid] += add;
    }
}

// sorted records: p-th point of the sorted order is node k = idx[p]
// the FP64 cell offset of node k: the product and the difference rounded
// separately, as on the host (a fused multiply-subtract would give another
// offset)
__device__ __forceinline__ double node_offset(const double *__restrict__ x, int32_t k, double scale)
{
#pragma clang fp contract(off)
    const double t = scale * x[k];
    return t - cell_floor(t);
}

// the FP32 record of sorted point p
__device__ __forceinline__ PtRec node_rec32(const double *__restrict__ x, const int32_t *__restrict__ idx, int64_t p,
                                            double scale)
{
    const int32_t k = idx[p];
    float f = (float)node_offset(x, k, scale);
    if (!(f < 1.0f)) f = 0.99999994f;   // keep the offset inside [0, 1)
    PtRec r;
    r.perm = k;
    r.frac = f;
    return r;
}

__global__ void k_sorted_records(const double *__restrict__ x, const int32_t *__restrict__ idx, int64_t M,
                                 double scale, int fp32, int32_t *__restrict__ perm, double *__restrict__ frac64,
                                 PtRec *__restrict__ rec32)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M; p += (int64_t)gridDim.x * blockDim.x) {
        if (fp32) {
            rec32[p] = node_rec32(x, idx, p, scale);
        } else {
            const int32_t k = idx[p];
            perm[p] = k;
            frac64[p] = node_offset(x, k, scale);
        }
    }
}

// FP32 records in per-slot transposed blocks, formed directly from the
// sorted indices: point q of item t of slot g at (g rows + q) 64 + t holds
// the record of its sorted point; rows past an item's end repeat its last
// record; empty items hold zeros
__device__ __forceinline__ void transposed_record(const double *__restrict__ x, const int32_t *__restrict__ idx,
                                                  double scale, const Item *__restrict__ items, int rows, int64_t i,
                                                  PtRec *__restrict__ out)
{
    const int t = (int)(i % kItemsPerWg);
    const int64_t gq = i / kItemsPerWg;
    const int64_t g = gq / rows, q = gq % rows;
    const Item it = items[g * kItemsPerWg + t];
    PtRec r;
    r.perm = 0;
    r.frac = 0.f;
    if (it.n > 0) r = node_rec32(x, idx, it.p0 + std::min<int64_t>(q, it.n - 1), scale);
    out[i] = r;
}

__global__ void k_transposed_records(const double *__restrict__ x, const int32_t *__restrict__ idx, double scale,
                                     const Item *__restrict__ items, int64_t nslot, int rows,
                                     PtRec *__restrict__ out)
{
    const int64_t total = nslot * rows * kItemsPerWg;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        transposed_record(x, idx, scale, items, rows, i, out);
}

// both sides' records in one launch (side b's entries after side a's)
__global__ void k_records_pair(RecSide a, RecSide b, int fp32)
{
    const int64_t na = fp32 ? a.nslot * a.rows * kItemsPerWg : a.M;
    const int64_t nb = fp32 ? b.nslot * b.rows * kItemsPerWg : b.M;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb;
         i += (int64_t)gridDim.x * blockDim.x) {
        const bool second = i >= na;
        const RecSide &S = second ? b : a;
        const int64_t j = second ? i - na : i;
        if (fp32) {
            transposed_record(S.x, S.idx, S.scale, S.items, S.rows, j, S.trec);
        } else {
            const int32_t k = S.idx[j];
            S.perm[j] = k;
            S.frac[j] = node_offset(S.x, k, S.scale);
        }
    }
}

__global__ void k_gather_pair(const double *__restrict__ x0, const int64_t *__restrict__ idx0, int64_t n0,
                              double *__restrict__ out0, const double *__restrict__ x1,
                              const int64_t *__restrict__ idx1, int64_t n1, double *__restrict__ out1)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0 + n1;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n0) out0[i] = x0[idx0[i]];
        else out1[i - n0] = x1[idx1[i - n0]];
    }
}

__global__ void k_gather(const double *__restrict__ x, const int64_t *__restrict__ idx, int64_t n,
                         double *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = x[idx[i]];
}

unsigned grid_for(int64_t n, int threads)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, 8192));
}

int bit_width(uint64_t v)
{
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

bool device_sort_fits(int64_t M, int64_t nbins, int64_t block)
{
    const int64_t nblocks = (M + block - 1) / block;
    const int bbits = std::max(1, bit_width((uint64_t)(nbins - 1)));
    return bbits + bit_width((uint64_t)(nblocks - 1)) <= 32 && M < ((int64_t)1 << 31);
}

size_t device_sort_tmp_bytes(int64_t M)
{
    const int64_t ntiles = (M + kTile - 1) / kTile;
    return 2 * al256((size_t)M * 4) + 2 * al256((size_t)M * 4) + al256((size_t)kRadix * ntiles * 4) +
           al256((size_t)kRadix * 4);
}

hipError_t device_sort_nodes(const double *x, int64_t M, double scale, int64_t off, int64_t nbins, int64_t block,
                             int32_t *counts, int32_t *flag, void *tmp, int32_t **sorted_idx, hipStream_t s)
{
    const int64_t nblocks = (M + block - 1) / block;
    const int bbits = std::max(1, bit_width((uint64_t)(nbins - 1)));
    const int kbits = bbits + bit_width((uint64_t)(nblocks - 1));
    const int64_t ntiles = (M + kTile - 1) / kTile;
    unsigned char *p = static_cast<unsigned char *>(tmp);
    uint32_t *keys[2];
    int32_t *vals[2];
    keys[0] = reinterpret_cast<uint32_t *>(p);
    p += al256((size_t)M * 4);
    keys[1] = reinterpret_cast<uint32_t *>(p);
    p += al256((size_t)M * 4);
    vals[0] = reinterpret_cast<int32_t *>(p);
    p += al256((size_t)M * 4);
    vals[1] = reinterpret_cast<int32_t *>(p);
    p += al256((size_t)M * 4);
    uint32_t *hist = reinterpret_cast<uint32_t *>(p);
    p += al256((size_t)kRadix * ntiles * 4);
    uint32_t *tot = reinterpret_cast<uint32_t *>(p);
    hipLaunchKernelGGL(k_node_keys, dim3(grid_for(M, 256)), dim3(256), 0, s, x, M, scale, off, nbins, block, bbits,
                       0u, keys[0], vals[0], flag);
    int cur = 0;
    for (int shift = 0; shift < kbits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, keys[cur], M, shift,
                           ntiles, hist);
        hipLaunchKernelGGL(k_radix_scan_rows, dim3(kRadix), dim3(kSortThreads), 0, s, hist, ntiles, tot);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, keys[cur], vals[cur],
                           M, shift, ntiles, hist, tot, keys[1 - cur], vals[1 - cur]);
        cur = 1 - cur;
    }
    hipLaunchKernelGGL(k_run_starts, dim3(grid_for(M, 256)), dim3(256), 0, s, keys[cur], M, bbits, nbins, counts);
    hipLaunchKernelGGL(k_run_ends, dim3(grid_for(M, 256)), dim3(256), 0, s, keys[cur], M, bbits, nbins, counts);
    *sorted_idx = vals[cur];
    return hipGetLastError();
}

static int key_bits(int64_t M, int64_t nbins, int64_t block, int *bbits)
{
    const int64_t nblocks = (M + block - 1) / block;
    *bbits = std::max(1, bit_width((uint64_t)(nbins - 1)));
    return *bbits + bit_width((uint64_t)(nblocks - 1));
}

bool device_sort_pair_fits(const SortSide &a, const SortSide &b)
{
    int ba, bb;
    const int kb = std::max(key_bits(a.M, a.nbins, a.block, &ba), key_bits(b.M, b.nbins, b.block, &bb));
    return kb + 1 <= 32 && a.M + b.M < ((int64_t)1 << 31);
}

hipError_t device_sort_node_pair(const SortSide &a, const SortSide &b, void *tmp, int32_t **sorted_a,
                                 int32_t **sorted_b, hipStream_t s)
{
    const SortSide *sd[2] = {&a, &b};
    RunPair R{};
    int kb = 0;
    for (int i = 0; i < 2; ++i) {
        kb = std::max(kb, key_bits(sd[i]->M, sd[i]->nbins, sd[i]->block, &R.bbits[i]));
        R.counts[i] = sd[i]->counts;
        R.nbins[i] = sd[i]->nbins;
    }
    R.kb = kb;
    const int kbits = kb + 1;
    const int64_t M = a.M + b.M;
    const int64_t ntiles = (M + kTile - 1) / kTile;
    unsigned char *p = static_cast<unsigned char *>(tmp);
    uint32_t *keys[2];
    int32_t *vals[2];
    keys[0] = reinterpret_cast<uint32_t *>(p);
    p += al256((size_t)M * 4);
    keys[1] = reinterpret_cast<uint32_t *>(p);
    p += al256((size_t)M * 4);
    vals[0] = reinterpret_cast<int32_t *>(p);
    p += al256((size_t)M * 4);
    vals[1] = reinterpret_cast<int32_t *>(p);
    p += al256((size_t)M * 4);
    uint32_t *hist = reinterpret_cast<uint32_t *>(p);
    p += al256((size_t)kRadix * ntiles * 4);
    uint32_t *tot = reinterpret_cast<uint32_t *>(p);
    KeySide ks[2];
    for (int i = 0; i < 2; ++i) {
        const SortSide &d = *sd[i];
        ks[i] = KeySide{d.x, d.M, d.scale, d.off, d.nbins, d.block, R.bbits[i], (uint32_t)i << kb, d.flag};
    }
    hipLaunchKernelGGL(k_node_keys_pair, dim3(grid_for(M, 256)), dim3(256), 0, s, ks[0], ks[1], keys[0], vals[0]);
    int cur = 0;
    for (int shift = 0; shift < kbits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, keys[cur], M, shift,
                           ntiles, hist);
        hipLaunchKernelGGL(k_radix_scan_rows, dim3(kRadix), dim3(kSortThreads), 0, s, hist, ntiles, tot);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kSortThreads), 0, s, keys[cur], vals[cur],
                           M, shift, ntiles, hist, tot, keys[1 - cur], vals[1 - cur]);
        cur = 1 - cur;
    }
    hipLaunchKernelGGL(k_run_counts_pair, dim3(grid_for(M, 256)), dim3(256), 0, s, keys[cur], M, R);
    *sorted_a = vals[cur];
    *sorted_b = vals[cur] + a.M;
    return hipGetLastError();
}

hipError_t device_sorted_records(const double *x, const int32_t *sorted_idx, int64_t M, double scale, bool fp32,
                                 int32_t *perm, double *frac64, PtRec *rec32, hipStream_t s)
{
    hipLaunchKernelGGL(k_sorted_records, dim3(grid_for(M, 256)), dim3(256), 0, s, x, sorted_idx, M, scale,
                       fp32 ? 1 : 0, perm, frac64, rec32);
    return hipGetLastError();
}

hipError_t device_transposed_records(const double *x, const int32_t *sorted_idx, double scale, const Item *launch_items,
                                     int64_t nslot, int rows, PtRec *trec32, hipStream_t s)
{
    const int64_t total = nslot * rows * kItemsPerWg;
    hipLaunchKernelGGL(k_transposed_records, dim3(grid_for(total, 256)), dim3(256), 0, s, x, sorted_idx, scale,
                       launch_items, nslot, rows, trec32);
    return hipGetLastError();
}

hipError_t device_records_pair(bool fp32, const RecSide &a, const RecSide &b, hipStream_t s)
{
    const int64_t n = fp32 ? (a.nslot * a.rows + b.nslot * b.rows) * kItemsPerWg : a.M + b.M;
    hipLaunchKernelGGL(k_records_pair, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, fp32 ? 1 : 0);
    return hipGetLastError();
}

hipError_t device_gather_pair(const double *x0, const int64_t *idx0, int64_t n0, double *out0, const double *x1,
                              const int64_t *idx1, int64_t n1, double *out1, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_pair, dim3(grid_for(n0 + n1, 256)), dim3(256), 0, s, x0, idx0, n0, out0, x1, idx1, n1,
                       out1);
    return hipGetLastError();
}

hipError_t device_gather(const double *x, const int64_t *idx, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256)), dim3(256), 0, s, x, idx, n, out);
    return hipGetLastError();
}

}  // namespace nnfft
