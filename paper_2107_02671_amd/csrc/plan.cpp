// NNFFT plans (Algorithm 2.2 step 0), the tuning table, the fast sinc
// transform plan (Algorithm 6.1) and the C ABI of include/nnfft.h.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/nnfft.h"
#include "host_math.h"
#include "internal.h"
#include "plan.h"

using namespace nnfft;

namespace {

thread_local std::string g_last_error;

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw HipError{e, what};
}

void *hip_alloc(void *, size_t bytes)
{
    void *p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}

void hip_release(void *, void *p)
{
    if (p) (void)hipFree(p);
}

// Tuning table: (precision, ceil(log2 M)) -> layout.
std::mutex g_tune_mu;
std::map<std::pair<int, int>, Layout> g_tune;

int size_class(int64_t M)
{
    int c = 0;
    while (((int64_t)1 << c) < M) ++c;
    return c;
}

}  // namespace

namespace nnfft {

const DevMem &hip_mem()
{
    static const DevMem m = {hip_alloc, hip_release, nullptr};
    return m;
}

nnfft_status fail(nnfft_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

// Rule measured on MI355X: one-wavefront workgroups of 64 items; items of up
// to Q points with Q growing with the node count (16 at 2^20 nodes, 32 at
// most on the FP32 path, 8 on the FP64 path) so that a launch keeps a few
// workgroups per CU; blocks of 2^17 nodes (FP32; 1 MB of c64 coefficients,
// well inside one XCD's 4 MB L2) or 2^16 (FP64), split into 8 when that keeps
// them >= 2^14 nodes so that every XCD has a block.
Layout rule_layout(int64_t M, bool fp32, bool spreading)
{
    Layout L;
    const int64_t target_wg = 4 * 256;
    const int64_t q = M / (kItemsPerWg * target_wg);
    int Q = 2;
    while (Q < q && Q < (fp32 ? 32 : 4)) Q *= 2;
    L.Q = Q;
    // 2^17 points per block (1 MB of FP32 coefficients per XCD's L2); above
    // 2^20 points a spreading side takes 2^18: fewer blocks mean fewer windows
    // per grid cell to merge (an interpolation side has no merge and keeps
    // its scattered stores local)
    const bool big = spreading && M > ((int64_t)1 << 20);
    const int64_t bmax = (int64_t)1 << (big ? 18 : 17);
    L.block = bmax;
    return sanitize_layout(L, M, fp32);
}

Layout sanitize_layout(Layout L, int64_t M, bool fp32)
{
    L.Q = std::max(1, std::min(L.Q, fp32 ? 64 : 8));   // the FP64 kernels hold 8 points per item
    const int64_t bmin = (int64_t)1 << 14;
    int64_t block = std::max<int64_t>(1, L.block);
    int64_t nblk = (M + block - 1) / block;
    if (nblk < 8 && M >= 8 * bmin) nblk = 8;
    if (nblk < 1) nblk = 1;
    L.block = std::max<int64_t>(1, (M + nblk - 1) / nblk);
    return L;
}

Layout choose_layout(int64_t M, bool fp32, bool spreading)
{
    Layout L;
    if (get_tuned_layout(fp32, M, L)) return sanitize_layout(L, M, fp32);
    return rule_layout(M, fp32, spreading);
}

// Indices of the density samples of a node set of M points laid out by L:
// strided samples (up to 4096) of up to four node blocks, in the order the
// item size rule reads them; none when the rule's items are already the
// largest.
std::vector<int64_t> density_sample_indices(int64_t M, const Layout &L, bool fp32)
{
    std::vector<int64_t> idx;
    const int qmax = fp32 ? 32 : 8;
    if (L.Q >= qmax) return idx;
    const int64_t nblk = (M + L.block - 1) / L.block;
    const int64_t nsb = std::min<int64_t>(nblk, 4);
    for (int64_t sb = 0; sb < nsb; ++sb) {
        const int64_t blk = sb * nblk / nsb;
        const int64_t k0 = blk * L.block, len = std::min(M, k0 + L.block) - k0;
        const int64_t S = std::min<int64_t>(len, 4096);
        if (S < 2) continue;
        for (int64_t i = 0; i < S; ++i) idx.push_back(k0 + i * len / S);
    }
    return idx;
}

// The item size rule for dense node sets, from the sampled node values (in
// density_sample_indices order): where a typical node's bin holds more than
// eight of the rule's items within its block, the item size is raised to the
// smallest power of two >= load / 1.5 (up to 32 on the FP32 path, 8 on the
// FP64 path), load = block x sum_b p_b^2 estimated from the samples of each
// block ((sum_b c_b^2 - S) / (S (S - 1)) over S sampled cells).  One thread
// sums the items of a bin, so dense cells cut into many short items
// serialize their chunk.
Layout raise_item_size(Layout L, int64_t M, double scale, bool fp32, const double *vals)
{
    const int qmax = fp32 ? 32 : 8;
    if (L.Q >= qmax) return L;
    const int64_t nblk = (M + L.block - 1) / L.block;
    const int64_t nsb = std::min<int64_t>(nblk, 4);
    double load = 0.0;
    int64_t used = 0, at = 0;
    std::vector<int64_t> cell;
    for (int64_t sb = 0; sb < nsb; ++sb) {
        const int64_t blk = sb * nblk / nsb;
        const int64_t k0 = blk * L.block, len = std::min(M, k0 + L.block) - k0;
        const int64_t S = std::min<int64_t>(len, 4096);
        if (S < 2) continue;
        cell.resize((size_t)S);
        int64_t cmin = INT64_MAX, cmax = INT64_MIN;
        for (int64_t i = 0; i < S; ++i) {
            const int64_t c = (int64_t)std::floor(scale * vals[at++]);
            cell[(size_t)i] = c;
            cmin = std::min(cmin, c);
            cmax = std::max(cmax, c);
        }
        // sum over the sampled cells of (samples in the cell)^2: counted in
        // an array over the cells' range (a sort where that range is wide);
        // the terms are integers, so the order of the sum does not matter
        double sumsq = 0.0;
        if (cmax - cmin < ((int64_t)1 << 20)) {
            std::vector<int32_t> cnt((size_t)(cmax - cmin + 1), 0);
            for (int64_t i = 0; i < S; ++i) ++cnt[(size_t)(cell[(size_t)i] - cmin)];
            for (const int32_t c : cnt) sumsq += (double)c * (double)c;
        } else {
            std::sort(cell.begin(), cell.end());
            for (int64_t i = 0; i < S;) {
                int64_t j = i;
                while (j < S && cell[(size_t)j] == cell[(size_t)i]) ++j;
                sumsq += (double)(j - i) * (double)(j - i);
                i = j;
            }
        }
        load += (double)len * (sumsq - (double)S) / ((double)S * (double)(S - 1));
        ++used;
    }
    if (used > 0) {
        load /= (double)used;
        // only where the rule's items would cut a typical bin into more than
        // eight pieces (the rule's item size already balances the launch
        // width against that loop for uniform nodes, at up to four pieces)
        if (load > 8.0 * L.Q)
            while (L.Q < qmax && L.Q < load / 1.5) L.Q *= 2;
    }
    return L;
}

// choose_layout for a given node set (grid coordinate t = scale * node); a
// tuned entry (timed on uniform nodes) takes the place of the rule and gets
// the same raise for dense node sets.
Layout choose_layout_nodes(const std::vector<double> &nodes, double scale, bool fp32, bool spreading)
{
    const int64_t M = (int64_t)nodes.size();
    const Layout L = choose_layout(M, fp32, spreading);
    const std::vector<int64_t> idx = density_sample_indices(M, L, fp32);
    std::vector<double> vals(idx.size());
    for (size_t i = 0; i < idx.size(); ++i) vals[i] = nodes[(size_t)idx[i]];
    return raise_item_size(L, M, scale, fp32, vals.data());
}

void set_tuned_layout(bool fp32, int64_t M, const Layout &L)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[{fp32 ? 1 : 0, size_class(M)}] = L;
}

bool get_tuned_layout(bool fp32, int64_t M, Layout &L)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find({fp32 ? 1 : 0, size_class(M)});
    if (it == g_tune.end()) return false;
    L = it->second;
    return true;
}

void clear_tuned_layouts()
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.clear();
}

namespace {

// Helper threads that plans may start, shared by every planning thread of the
// process: a plan takes what is free and runs the rest itself, so concurrent
// planners (the request server's) do not multiply the host's thread count.
constexpr int kHelperBudget = 8;
std::atomic<int> g_helpers_free{kHelperBudget};

struct HelperGrant {
    int n = 0;
    explicit HelperGrant(int want)
    {
        int cur = g_helpers_free.load(std::memory_order_relaxed);
        while (want > 0 && cur > 0) {
            const int got = std::min(want, cur);
            if (g_helpers_free.compare_exchange_weak(cur, cur - got)) {
                n = got;
                break;
            }
        }
    }
    ~HelperGrant()
    {
        if (n > 0) g_helpers_free.fetch_add(n);
    }
    HelperGrant(const HelperGrant &) = delete;
    HelperGrant &operator=(const HelperGrant &) = delete;
};

// Runs body(i, thread) for i in [0, n) on up to nthr threads (as many helpers
// as the budget grants): thread r takes the i with i mod nthr == r, the
// calling thread r = 0 and the residues of threads that could not be started.
// An exception of any body is rethrown here once every thread has finished.
template <typename Body>
void parallel_strided(int64_t n, int nthr, Body &&body)
{
    nthr = (int)std::max<int64_t>(1, std::min<int64_t>(nthr, n));
    const HelperGrant grant(nthr - 1);
    nthr = grant.n + 1;
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> xs((size_t)nthr);
    try {
        for (int r = 1; r < nthr; ++r)
            th.emplace_back([&, r] {
                try {
                    for (int64_t i = r; i < n; i += nthr) body(i, r);
                } catch (...) {
                    xs[(size_t)r] = std::current_exception();
                }
            });
    } catch (...) {   // fewer threads (none left or no memory for one): the rest runs here
    }
    const int started = (int)th.size() + 1;
    try {
        for (int64_t i = 0; i < n; ++i)
            if (i % nthr == 0 || i % nthr >= started) body(i, 0);
    } catch (...) {
        xs[0] = std::current_exception();
    }
    for (auto &t : th) t.join();
    for (auto &x : xs)
        if (x) std::rethrow_exception(x);
}

// Both sides on two threads once each holds this many points
constexpr int64_t kParallelSidePoints = (int64_t)1 << 15;
// Node blocks of one side on up to kBlockThreads threads once the side holds
// kParallelBlockPoints points (and the per-thread bin counts stay small)
constexpr int64_t kParallelBlockPoints = (int64_t)1 << 18;
constexpr int64_t kParallelBlockBins = (int64_t)1 << 21;
constexpr int kBlockThreads = 4;

}  // namespace

// Items and chunks of one node block (consecutive caller indices) from the
// block's bin counts cnt[0 .. nbins): the block's points sorted by bin start
// at sorted position k0; each bin run is split into ceil(n / Q) balanced
// items; a chunk takes consecutive items, at most kItemsPerWg of them, within
// kItemsPerWg bins.  Both the host and the device node layouts build their
// schedule here, so they agree item for item.
void block_schedule(const int32_t *cnt, int64_t nbins, int64_t k0, int Q, BlockOut &o)
{
    // items: one per bin of at most Q points, else the bin's points split
    // evenly.  The common case is written without a branch (an empty bin's
    // item is overwritten by the next one): bin counts are random, so
    // branches on them are mispredicted.
    int64_t npts = 0, nz = 0;
    for (int64_t b = 0; b < nbins; ++b) {
        npts += cnt[b];
        nz += cnt[b] != 0;
    }
    o.items.resize((size_t)(nz + npts / Q + 1));
    Item *it = o.items.data();
    int64_t k = 0;
    int32_t p = (int32_t)k0;
    for (int64_t b = 0; b < nbins; ++b) {
        const int32_t n = cnt[b];
        if (n <= Q) {
            it[k] = Item{(int32_t)b, p, n, 0};
            k += n != 0;
            p += n;
            continue;
        }
        const int32_t nit = (n + Q - 1) / Q;
        const int32_t base = n / nit, rem = n - base * nit;
        for (int32_t q = 0; q < nit; ++q) {
            const int32_t len = base + (q < rem ? 1 : 0);
            it[k++] = Item{(int32_t)b, p, len, 0};
            p += len;
        }
    }
    o.items.resize((size_t)k);
    o.chunks.reserve(o.items.size() / 16 + 1);
    o.item0.reserve(o.items.size() / 16 + 1);
    const size_t it1 = o.items.size();
    for (size_t ci = 0; ci < it1;) {
        const int32_t blo = o.items[ci].bin;
        size_t cj = ci;
        while (cj < it1 && (int)(cj - ci) < kItemsPerWg && o.items[cj].bin - blo < kItemsPerWg) ++cj;
        Chunk c{};
        c.nitem = (int32_t)(cj - ci);
        c.bin_lo = blo;
        c.nbin = o.items[cj - 1].bin - blo + 1;
        int32_t run = 1, maxrun = 1;
        for (size_t i = ci + 1; i < cj; ++i) {
            run = (o.items[i].bin == o.items[i - 1].bin) ? run + 1 : 1;
            maxrun = std::max(maxrun, run);
        }
        o.items[ci].maxrun = maxrun;
        o.chunks.push_back(c);
        o.item0.push_back((int32_t)ci);
        ci = cj;
    }
}

// Appends the blocks' items and chunks in block order, colours the spreading
// windows (m > 0) and lays out the launch slots (XCD-aware order, 64 items
// per slot).  The FP32 records of the slots are transposed separately.
bool finish_side(std::vector<BlockOut> &outs, int m, SideHost &S, std::string &err)
{
    {
        size_t nc = 0;
        for (const BlockOut &o : outs) {
            if (!o.ok) {
                err = "internal: node record outside the grid";
                return false;
            }
            nc += o.chunks.size();
        }
        // the items stay in their blocks' outputs until the launch slots are
        // filled (no concatenated copy)
        S.chunks.reserve(nc);
        S.chunk_block.reserve(nc);
        S.chunk_item0.reserve(nc);
        for (int64_t blk = 0; blk < (int64_t)outs.size(); ++blk) {
            BlockOut &o = outs[(size_t)blk];
            S.chunks.insert(S.chunks.end(), o.chunks.begin(), o.chunks.end());
            S.chunk_block.insert(S.chunk_block.end(), o.chunks.size(), (int32_t)blk);
            S.chunk_item0.insert(S.chunk_item0.end(), o.item0.begin(), o.item0.end());
        }
    }
    int64_t part = 0;
    // spreading windows: chunk c covers cells [bin_lo - m + 1, bin_lo + nbin + m).
    // Windows are coloured greedily in order of their first cell (interval
    // colouring: at most as many colours as windows overlap at one cell);
    // colour s writes into plane s (part_off = -s - 1), so a cell's partial
    // sums sit at fixed offsets in every plane.  Windows beyond kMaxPlanes
    // colours go to an overflow area merged through index lists (part_off =
    // offset in that area here; finalize_planes places the area).
    if (m > 0) {
        std::vector<int32_t> ord(S.chunks.size());
        for (size_t c = 0; c < ord.size(); ++c) ord[c] = (int32_t)c;
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int32_t a, int32_t b) { return S.chunks[a].bin_lo < S.chunks[b].bin_lo; });
        std::vector<int64_t> plane_end;   // first free cell of each colour
        int64_t ovf = 0;
        std::vector<int64_t> ovf_off(S.chunks.size(), -1);
        for (int32_t c : ord) {
            Chunk &ch = S.chunks[c];
            // cells lo .. hi - 1: nbin + 2 m - 1 of them
            const int64_t lo = (int64_t)ch.bin_lo - m + 1, hi = lo + ch.nbin + 2 * m - 1;
            int colour = -1;
            for (size_t k = 0; k < plane_end.size(); ++k)
                if (plane_end[k] <= lo) {
                    colour = (int)k;
                    break;
                }
            if (colour < 0 && (int)plane_end.size() < kMaxPlanes) {
                colour = (int)plane_end.size();
                plane_end.push_back(0);
            }
            if (colour >= 0) {
                plane_end[colour] = hi;
                ch.part_off = -(colour + 1);
            } else {
                ovf_off[c] = ovf;
                ovf += hi - lo;
            }
        }
        S.nplanes = (int32_t)plane_end.size();
        for (size_t c = 0; c < S.chunks.size(); ++c)
            if (ovf_off[c] >= 0) S.chunks[c].part_off = (int32_t)ovf_off[c];
        S.ovf_cells = ovf;
    }
    S.part_cells = part;
    // XCD-aware schedule: workgroup w runs on XCD w % 8 (round-robin dispatch),
    // so the chunks of block b go to slots with w % 8 == b % 8 and all
    // gathers/scatters of a block stay in one XCD's L2.
    const int nx = 8;
    std::vector<int32_t> order;   // launch slot -> chunk id (-1: empty)
    if (S.nblocks >= nx) {
        std::vector<std::vector<int32_t>> lists(nx);
        for (size_t c = 0; c < S.chunks.size(); ++c) lists[S.chunk_block[c] % nx].push_back((int32_t)c);
        size_t mx = 0;
        for (auto &l : lists) mx = std::max(mx, l.size());
        order.assign(mx * nx, -1);
        for (int x = 0; x < nx; ++x)
            for (size_t j = 0; j < lists[x].size(); ++j) order[j * nx + x] = lists[x][j];
    } else {
        order.resize(S.chunks.size());
        for (size_t c = 0; c < S.chunks.size(); ++c) order[c] = (int32_t)c;
    }
    const Chunk empty{0, 0, 0, 0};
    const Item pad_item{0, 0, 0, 0};
    S.launch.assign(order.size(), empty);
    S.launch_items.resize(order.size() * kItemsPerWg);   // every entry written below
    for (size_t g = 0; g < order.size(); ++g) {
        Item *dst = S.launch_items.data() + g * kItemsPerWg;
        int nitem = 0;
        if (order[g] >= 0) {
            const Chunk c = S.chunks[order[g]];
            const Item *src = outs[(size_t)S.chunk_block[order[g]]].items.data() + S.chunk_item0[order[g]];
            std::copy(src, src + c.nitem, dst);
            S.launch[g] = c;
            nitem = c.nitem;
        }
        std::fill(dst + nitem, dst + kItemsPerWg, pad_item);
    }
    for (BlockOut &o : outs) ItemBuf().swap(o.items);
    return true;
}

namespace {

// FP32 records: one transposed block of Q rows per launch slot, point q of
// item t of slot g at (g Q + q) 64 + t; rows past an item's end repeat its
// last record (same address, masked in the kernel), empty items hold zeros.
static bool transpose_records(SideHost &S, int64_t rows, std::string &err)
{
    const size_t nslot = S.launch.size();
    if ((int64_t)nslot * rows * kItemsPerWg >= ((int64_t)1 << 31)) {
        err = "too many padded records";
        return false;
    }
    S.trec32.assign((size_t)(nslot * rows * kItemsPerWg), PtRec{0, 0.f});
    for (size_t g = 0; g < nslot; ++g) {
        const Chunk &c = S.launch[g];
        // row by row, so the writes are sequential
        PtRec *blk = S.trec32.data() + (size_t)g * rows * kItemsPerWg;
        const Item *its = S.launch_items.data() + g * kItemsPerWg;
        for (int64_t q = 0; q < rows; ++q)
            for (int i = 0; i < c.nitem; ++i)
                blk[q * kItemsPerWg + i] = S.rec32[(size_t)(its[i].p0 + std::min<int64_t>(q, its[i].n - 1))];
    }
    return true;
}

// Builds the sorted records, items, chunks and schedule of one side on the
// host.  t_k = scale * node_k (grid units); bin = floor(t_k) + off in [0, nbins).
// Spreading side: `m` > 0 gives the chunk windows of 2m - 1 + nbin cells.
bool build_side(const std::vector<double> &nodes, double scale, int64_t off, int64_t nbins,
                const Layout &L, bool fp32, int m, SideHost &S, std::string &err)
{
    const int64_t M = (int64_t)nodes.size();
    if (!(std::fabs(scale) <= (double)((int64_t)1 << 26))) {
        err = "internal: grid scale out of range";
        return false;
    }
    // cell and offset of node k, formed again by each pass that needs them
    // (the same expression, so the same values) instead of held in arrays
    // (|t| <= 2^25 for nodes in [-1/2, 1/2], so truncation stepped down for
    // negative non-integers is the exact floor, without a library call)
    auto cell_of = [&](int64_t k, double *frac) {
        const double t = scale * nodes[k];
        const double tr = (double)(int64_t)t;
        const double c = tr > t ? tr - 1.0 : tr;
        *frac = t - c;
        return (int64_t)c + off;
    };
    S.perm.assign(M, 0);
    if (fp32) S.rec32.assign(M, PtRec{0, 0.f});
    else S.frac64.assign(M, 0.0);
    S.nblocks = (M + L.block - 1) / L.block;
    S.rows = L.Q;
    S.npts = M;
    // Each node block is sorted (stable counting sort by bin) and cut into
    // items and chunks on its own (writes to its own range of perm / records
    // and its own lists), on up to kBlockThreads threads for large sides; the
    // lists are then appended in block order, so the result does not depend
    // on the threads.
    std::vector<BlockOut> outs((size_t)S.nblocks);
    auto run_block = [&](int64_t blk, std::vector<int32_t> &cnt, std::vector<int64_t> &pos) {
        BlockOut &o = outs[(size_t)blk];
        const int64_t k0 = blk * L.block, k1 = std::min(M, k0 + L.block);
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int64_t k = k0; k < k1; ++k) {
            double fr;
            const int64_t b = cell_of(k, &fr);
            if (b < 0 || b >= nbins) {
                o.ok = false;
                return;
            }
            cnt[b]++;
        }
        block_schedule(cnt.data(), nbins, k0, L.Q, o);
        int64_t acc = k0;
        for (int64_t b = 0; b < nbins; ++b) {
            pos[b] = acc;
            acc += cnt[b];
        }
        for (int64_t k = k0; k < k1; ++k) {
            double fr;
            const int64_t b = cell_of(k, &fr);
            const int64_t p = pos[b]++;
            S.perm[p] = (int32_t)k;
            if (fp32) {
                float f = (float)fr;
                if (!(f < 1.0f)) f = 0.99999994f;   // keep the offset inside [0, 1)
                S.rec32[p] = PtRec{(int32_t)k, f};
            } else {
                S.frac64[p] = fr;
            }
        }
    };
    const int nthr = (M >= kParallelBlockPoints && nbins <= kParallelBlockBins) ? kBlockThreads : 1;
    std::vector<std::vector<int32_t>> cnts((size_t)nthr);   // bin counts of each thread
    std::vector<std::vector<int64_t>> poss((size_t)nthr);
    parallel_strided(S.nblocks, nthr, [&](int64_t blk, int r) {
        if (cnts[(size_t)r].empty()) {
            cnts[(size_t)r].resize((size_t)nbins);
            poss[(size_t)r].resize((size_t)nbins);
        }
        run_block(blk, cnts[(size_t)r], poss[(size_t)r]);
    });
    if (!finish_side(outs, m, S, err)) return false;
    if (fp32 && !transpose_records(S, L.Q, err)) return false;
    return true;
}

// Runs the two side builds, the second one on a thread of its own when
// `parallel` is set and the helper budget grants one (they share no state);
// the first failure's message goes to err and an exception of either build
// is rethrown here.
template <typename BuildA, typename BuildB>
bool build_both_sides(BuildA &&a, BuildB &&b, bool parallel, std::string &err)
{
    std::string ea, eb;
    bool okb = false;
    std::exception_ptr xb;
    const HelperGrant grant(parallel ? 1 : 0);
    std::thread tb;
    if (grant.n > 0) {
        try {
            tb = std::thread([&] {
                try {
                    okb = b(eb);
                } catch (...) {
                    xb = std::current_exception();
                }
            });
        } catch (const std::system_error &) {   // no thread available: build in turn
        }
    }
    bool oka = false;
    try {
        oka = a(ea);
    } catch (...) {
        if (tb.joinable()) tb.join();
        throw;
    }
    if (tb.joinable()) {
        tb.join();
        if (xb) std::rethrow_exception(xb);
    } else {
        okb = b(eb);
    }
    if (!oka || !okb) {
        err = oka ? eb : ea;
        return false;
    }
    return true;
}


// largest-square-ish factorization N2 = n1 * n2 with both parts <= limit
bool fft_factor(int64_t N2, int64_t limit, int64_t &n1, int64_t &n2)
{
    int64_t best = -1;
    double bestd = 1e300;
    for (int64_t d = 2; d <= N2 / 2; ++d) {
        if (N2 % d) continue;
        const int64_t e = N2 / d;
        if (d > limit || e > limit) continue;
        const double dist = std::fabs(std::log((double)d) - std::log((double)e));
        if (dist < bestd) {
            bestd = dist;
            best = d;
        }
    }
    if (best < 0) return false;
    n2 = best;
    n1 = N2 / best;
    return true;
}

}  // namespace

// Device block of a plan: every array at a 256-byte aligned offset, the
// uploaded tables first (one host-to-device copy), the scratch after them.
struct Carver {
    uintptr_t base;
    size_t off = 0;
    std::vector<char> *stage;   // host image of the uploaded part (null: sizing pass)
    explicit Carver(uintptr_t b, std::vector<char> *st) : base(b), stage(st) {}
    template <typename T, typename A>
    T *put(const std::vector<T, A> &v)
    {
        off = (off + 255) & ~(size_t)255;
        const size_t nb = std::max<size_t>(1, v.size()) * sizeof(T);
        if (stage) {
            if (stage->size() < off + nb) stage->resize(off + nb);
            if (!v.empty()) std::memcpy(stage->data() + off, v.data(), v.size() * sizeof(T));
        }
        T *p = reinterpret_cast<T *>(base + off);
        off += nb;
        return p;
    }
    // an array written on the device after the upload (no host image)
    template <typename T>
    T *reserve(size_t n)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = reinterpret_cast<T *>(base + off);
        off += std::max<size_t>(1, n) * sizeof(T);
        return p;
    }
    void *scratch(size_t nb)
    {
        off = (off + 255) & ~(size_t)255;
        void *p = reinterpret_cast<void *>(base + off);
        off += std::max<size_t>(nb, 16);
        return p;
    }
};

// Lays the plan out in its device block (base 0: sizing pass) and fills the
// kernel descriptors.  Returns the end of the uploaded part in *upload_end.
void layout_plan(const HostPlan &H, Carver &C, PlanDev &D, size_t *upload_end, PlanDev **ddesc,
                 size_t *dev_start = nullptr)
{
    const nnfft_info_t &P = H.info;
    const bool fp32 = H.fp32;
    D = PlanDev{};
    D.prec = P.precision;
    SpreadArgs &SA = D.sp;
    InterpArgs &IA = D.ip;
    FftArgs &FA = D.fft;
    SA.items = C.put(H.sp.launch_items);
    SA.chunks = C.put(H.sp.launch);
    SA.ngrid = (int32_t)H.sp.launch.size();
    SA.m = P.m1;
    SA.window = P.window;
    SA.beta = P.beta1;
    SA.inv_den = P.window == NNFFT_WINDOW_SINH ? 1.0 / (1.0 - std::exp(-2.0 * P.beta1)) : 0.0;
    IA.items = C.put(H.ip.launch_items);
    IA.chunks = C.put(H.ip.launch);
    IA.ngrid = (int32_t)H.ip.launch.size();
    IA.m = P.m2;
    IA.window = P.window;
    IA.beta = P.beta2;
    IA.inv_den = P.window == NNFFT_WINDOW_SINH ? 1.0 / (1.0 - std::exp(-2.0 * P.beta2)) : 0.0;
    IA.N2 = (int32_t)P.N2;
    IA.ip_off = (int32_t)(P.N2 / 2);
    IA.u_to_x = (double)P.N1 / ((double)P.N2 * (double)P.N_star);
    IA.corr = C.put(H.corr);
    IA.corr_deg = P.corr_degree;
    if (fp32) {
        SA.C = C.put(H.C1);
        IA.C = C.put(H.C2);
    } else {
        if (!H.T1.empty()) {
            SA.T64 = C.put(H.T1);
            IA.T64 = C.put(H.T2);
            SA.nser = (int32_t)H.T1.size();
            IA.nser = (int32_t)H.T2.size();
        }
    }
    FA.merge_off = C.put(H.moff);
    FA.merge_idx = C.put(H.midx);
    if (H.pm_cells > 0) {
        D.pm.seg = C.put(H.pm_seg);
        D.pm.idx = C.put(H.pm_idx);
        D.pm.nseg = (int32_t)H.pm_cells;
        D.pm.base = (int32_t)H.pm_base;
    }
    FA.deconv = C.put(H.deconv);
    if (fp32) FA.tw = C.put(H.tw32);
    else FA.tw = C.put(H.tw64);
    if (H.fd.n1 > 1) {
        if (fp32) {
            FA.twA = C.put(std::vector<float>(H.twA.begin(), H.twA.end()));
            FA.twB = C.put(std::vector<float>(H.twB.begin(), H.twB.end()));
            FA.tw4 = C.put(std::vector<float>(H.tw4.begin(), H.tw4.end()));
        } else {
            FA.twA = C.put(H.twA);
            FA.twB = C.put(H.twB);
            FA.tw4 = C.put(H.tw4);
        }
    }
    SA.slotT = FA.slotT = H.slotT;
    SA.slotP = FA.slotP = H.slotP;
    // the per-point records last: a plan whose nodes were sorted on the
    // device writes them there after the upload of everything before
    C.off = (C.off + 255) & ~(size_t)255;
    if (dev_start) *dev_start = C.off;
    auto side_records = [&](const SideHost &S, const PtRec **rec, const int32_t **perm, const double **frac) {
        if (fp32)
            *rec = S.dev ? C.reserve<PtRec>(S.launch.size() * (size_t)S.rows * kItemsPerWg) : C.put(S.trec32);
        else if (S.dev) {
            *perm = C.reserve<int32_t>((size_t)S.npts);
            *frac = C.reserve<double>((size_t)S.npts);
        } else {
            *perm = C.put(S.perm);
            *frac = C.put(S.frac64);
        }
    };
    side_records(H.sp, &SA.rec32, &SA.perm, &SA.frac64);
    side_records(H.ip, &IA.rec32, &IA.perm, &IA.frac64);
    *upload_end = C.off;
    const size_t csz = fp32 ? 8 : 16;
    SA.partial = C.scratch((size_t)H.sp.part_cells * 16);
    FA.partial = SA.partial;
    D.pm.partial = SA.partial;
    FA.Y = C.scratch((size_t)P.N2 * csz);
    FA.hlin = C.scratch((size_t)H.hlin_len * csz);
    IA.hlin = FA.hlin;
    FA.N2 = (int32_t)P.N2;
    FA.G1 = (int32_t)P.G1;
    FA.nplanes = H.sp.nplanes;
    FA.h_off = H.h_off;
    FA.mode = 0;
    FA.Nout = H.kind == 1 ? (int32_t)P.N : 0;
    IA.h_off = H.h_off;
    SA.rows = H.lay1.Q;
    IA.rows = H.lay2.Q;
    FA.n1 = H.fd.n1;
    FA.n2 = H.fd.n2;
    FA.batchA = H.fd.batchA;
    FA.batchB = H.fd.batchB;
    FA.threadsA = H.fd.threadsA;
    FA.threadsB = H.fd.threadsB;
    FA.S = H.fd.S;
    FA.npassA = H.fd.npassA;
    FA.npassB = H.fd.npassB;
    FA.fusedB = H.fd.fusedB ? 1 : 0;
    if (H.fd.fusedB) {
        IA.Y = FA.Y;
        IA.twB = FA.twB;
        IA.fusedB = H.fd.n1;
        IA.fn2 = H.fd.n2;
    }
    for (int i = 0; i < kMaxPasses; ++i) {
        FA.radA[i] = (int8_t)H.fd.radA[i];
        FA.radB[i] = (int8_t)H.fd.radB[i];
    }
    *ddesc = static_cast<PlanDev *>(C.scratch(sizeof(PlanDev)));   // the descriptor's device copy
}

// Merge lists of the overflow windows (those without a plane).
// Largest accepted error of the FP32 tap polynomials of one window: 5e-8, or
// 1e-3 of the window's own error term of Theorem 4.1,
// (24 m^1.5 + 10) exp(-2 pi m sqrt(1 - 1/sigma)), when that is larger (small
// m or sigma, where the transform's error dwarfs the polynomial's).
static double tap_fit_tolerance(int m, double sigma)
{
    const double term = (24.0 * std::pow((double)m, 1.5) + 10.0) *
                        std::exp(-2.0 * kPi * m * std::sqrt(1.0 - 1.0 / sigma));
    return std::max(5e-8, 1e-3 * term);
}

// Plane layout: cells in slot order with T = the first four-step factor n1
// of the FFT (1 for one-workgroup transforms), so a four-step column reads
// contiguous slots; the overflow area follows the planes.
static void finalize_planes(HostPlan &H, int64_t G1)
{
    H.slotT = H.fd.n1 > 1 ? H.fd.n1 : 1;
    H.slotP = (int32_t)((G1 + H.slotT - 1) / H.slotT);
    const int64_t ps = (int64_t)H.slotT * H.slotP;
    for (Chunk &c : H.sp.chunks)
        if (c.part_off >= 0) c.part_off = (int32_t)(H.sp.nplanes * ps + c.part_off);
    for (Chunk &c : H.sp.launch)   // the launch-order copies the kernels read
        if (c.nitem > 0 && c.part_off >= 0) c.part_off = (int32_t)(H.sp.nplanes * ps + c.part_off);
    H.sp.part_cells = H.sp.nplanes * ps + H.sp.ovf_cells;
}

static int64_t slot_of(const HostPlan &H, int64_t cell)
{
    return (cell % H.slotT) * H.slotP + cell / H.slotT;
}

constexpr int32_t kMergeDirect = 32;  // longest merge list the FFT load walks itself (rounds of 8 loads)
constexpr int32_t kMergeSplit = 8;    // segments a longer list is cut into (one round of loads)

static nnfft_status build_merge_lists(HostPlan &H, const nnfft_info_t &P, int m1)
{
    // merge lists of the overflow windows (those without a plane): for each
    // grid cell (by slot) the partial cells of the overflow chunks covering it
    const int64_t ns = (int64_t)H.slotT * H.slotP;
    H.moff.assign(ns + 1, 0);
    for (const Chunk &c : H.sp.chunks) {
        if (c.part_off < 0) continue;
        const int W = c.nbin + 2 * m1 - 1;
        for (int w = 0; w < W; ++w) {
            const int64_t cell = (int64_t)c.bin_lo - m1 + 1 + w;
            if (cell < 0 || cell >= P.G1) return fail(NNFFT_ERR_ARG, "internal: window outside the grid");
            H.moff[slot_of(H, cell) + 1]++;
        }
    }
    for (int64_t c = 0; c < ns; ++c) H.moff[c + 1] += H.moff[c];
    H.midx.resize(H.moff[ns]);
    {
        std::vector<int32_t> cur(H.moff.begin(), H.moff.end() - 1);
        for (const Chunk &c : H.sp.chunks) {
            if (c.part_off < 0) continue;
            const int W = c.nbin + 2 * m1 - 1;
            for (int w = 0; w < W; ++w) {
                const int64_t cell = (int64_t)c.bin_lo - m1 + 1 + w;
                H.midx[cur[slot_of(H, cell)]++] = c.part_off + w;
            }
        }
    }
    // lists longer than kMergeDirect entries: cut into segments of
    // L = ceil(n / kMergeSplit) entries, each pre-merged into a partial cell
    // of its own (after the existing ones), so such a list becomes at most
    // kMergeSplit entries (one round of loads in the FFT load).  Shorter
    // lists are walked by the FFT load itself: up to four rounds cost less
    // than the extra launch.
    H.pm_seg.clear();
    H.pm_idx.clear();
    H.pm_base = H.sp.part_cells;
    H.pm_cells = 0;
    bool longer = false;
    for (int64_t sl = 0; sl < ns && !longer; ++sl) longer = H.moff[sl + 1] - H.moff[sl] > kMergeDirect;
    if (longer) {
        std::vector<int32_t> off2(ns + 1, 0), idx2;
        idx2.reserve(H.midx.size());
        for (int64_t sl = 0; sl < ns; ++sl) {
            const int32_t e0 = H.moff[sl], n = H.moff[sl + 1] - e0;
            if (n <= kMergeDirect) {
                idx2.insert(idx2.end(), H.midx.begin() + e0, H.midx.begin() + e0 + n);
            } else {
                const int32_t L = (n + kMergeSplit - 1) / kMergeSplit;
                for (int32_t s0 = 0; s0 < n; s0 += L) {
                    const int32_t cnt = std::min(L, n - s0);
                    H.pm_seg.push_back((int32_t)H.pm_idx.size());
                    H.pm_seg.push_back(cnt);
                    H.pm_idx.insert(H.pm_idx.end(), H.midx.begin() + e0 + s0, H.midx.begin() + e0 + s0 + cnt);
                    idx2.push_back((int32_t)(H.pm_base + H.pm_cells));
                    ++H.pm_cells;
                }
            }
            off2[sl + 1] = (int32_t)idx2.size();
        }
        H.moff.swap(off2);
        H.midx.swap(idx2);
        H.sp.part_cells += H.pm_cells;
        if (H.sp.part_cells >= ((int64_t)1 << 31)) return fail(NNFFT_ERR_UNSUPPORTED, "too many partial cells");
    }
    return NNFFT_OK;
}

// Four-step twiddle tables from the plan's length-N2 table (same values):
// [n2] exp(-2 pi i k / n2), [n1] exp(-2 pi i k / n1), [n1][n2] exp(-2 pi i j1 k2 / N2).
static void fft_tables(HostPlan &H)
{
    if (H.fd.n1 <= 1) return;
    const int64_t n1 = H.fd.n1, n2 = H.fd.n2;
    auto tw = [&](int64_t q, int c) { return H.fp32 ? (double)H.tw32[2 * q + c] : H.tw64[2 * q + c]; };
    H.twA.resize(2 * n2);
    for (int64_t k = 0; k < n2; ++k)
        for (int c = 0; c < 2; ++c) H.twA[2 * k + c] = tw(k * n1, c);
    H.twB.resize(2 * n1);
    for (int64_t k = 0; k < n1; ++k)
        for (int c = 0; c < 2; ++c) H.twB[2 * k + c] = tw(k * n2, c);
    H.tw4.resize(2 * n1 * n2);
    for (int64_t j1 = 0; j1 < n1; ++j1)
        for (int64_t k2 = 0; k2 < n2; ++k2)
            for (int c = 0; c < 2; ++c) H.tw4[2 * (j1 * n2 + k2) + c] = tw(j1 * k2, c);
}

// FFT factorization of the length-N2 transform; outputs |s| <= S are stored.
// NNFFT plans with 1024 < N2 <= 4096 split N2 = 16 n2: stage A runs 16
// length-n2 transforms (n2 <= 256, one cell per thread) and the
// interpolation evaluates the 16-point second stage for the <= 64 + 2m
// outputs each of its workgroups reads, so the transform takes one launch.
// Longer transforms keep the two-launch split: 16 stage-A workgroups then
// merge too many window planes each (measured slower at N2 = 16384).
constexpr int kFusedN1 = 16;   // the FP32 interpolation folds rows of exactly 16 values
constexpr int64_t kFusedMaxN2 = 4096;

static nnfft_status plan_fft(HostPlan &H, const nnfft_info_t &P, bool fp32, int64_t S)
{
    // FFT factorization -----------------------------------------------------
    FftPlan &fd = H.fd;
    fd = FftPlan{};
    fd.N2 = (int32_t)P.N2;
    // one workgroup for short transforms; longer ones as two launches of
    // many workgroups (one or two columns each) so that the partial merge in
    // the first stage's load runs with enough workgroups in flight
    const int64_t single_max = 1024;
    const int kvals = fp32 ? 4096 : 2048;   // values per FFT workgroup (LDS)
    auto threads_for = [](int64_t vals) {
        int64_t t = (vals + 63) / 64 * 64;
        return (int32_t)std::max<int64_t>(64, std::min<int64_t>(256, t));
    };
    if (P.N2 <= single_max) {
        const std::vector<int> r = radix_passes(P.N2);
        if (r.empty() || (int)r.size() > kMaxPasses) return fail(NNFFT_ERR_UNSUPPORTED, "FFT length not 2,3,5-smooth");
        fd.n1 = 1;
        fd.n2 = (int32_t)P.N2;
        fd.npassA = (int32_t)r.size();
        std::copy(r.begin(), r.end(), fd.radA);
        fd.threadsA = 256;
    } else {
        int64_t n1, n2;
        const bool fuse = H.kind == 0 && P.N2 <= kFusedMaxN2 && P.N2 % kFusedN1 == 0;
        if (fuse) {
            n1 = kFusedN1;
            n2 = P.N2 / kFusedN1;
        } else if (!fft_factor(P.N2, kvals, n1, n2)) {
            return fail(NNFFT_ERR_UNSUPPORTED, "FFT length cannot be split");
        }
        fd.fusedB = fuse;
        const std::vector<int> rA = radix_passes(n2), rB = radix_passes(n1);
        if (rA.empty() || rB.empty() || (int)rA.size() > kMaxPasses || (int)rB.size() > kMaxPasses)
            return fail(NNFFT_ERR_UNSUPPORTED, "FFT length not 2,3,5-smooth");
        fd.n1 = (int32_t)n1;
        fd.n2 = (int32_t)n2;
        fd.npassA = (int32_t)rA.size();
        fd.npassB = (int32_t)rB.size();
        std::copy(rA.begin(), rA.end(), fd.radA);
        std::copy(rB.begin(), rB.end(), fd.radB);
        fd.batchA = fuse ? 1 : (int32_t)std::max<int64_t>(1, std::min<int64_t>(n1 / 128, kvals / n2));
        fd.batchB = (int32_t)std::max<int64_t>(1, std::min<int64_t>(n2 / 128, kvals / n1));
        fd.threadsA = threads_for((int64_t)fd.batchA * n2);
        fd.threadsB = threads_for((int64_t)fd.batchB * n1);
    }
    fd.S = (int32_t)S;

    return NNFFT_OK;
}

// Device block size and the layout figures of the info struct.
static void size_plan(HostPlan &H, const nnfft_info_t &P)
{
    PlanDev D, *dd = nullptr;
    Carver C(0, nullptr);
    size_t upload_end = 0;
    H.info = P;
    layout_plan(H, C, D, &upload_end, &dd);
    H.total_bytes = C.off;
    H.upload_bytes = upload_end;
    H.info.device_bytes = (int64_t)C.off;
    H.info.block_points = H.lay1.block;
    H.info.items_points = H.lay1.Q;
    H.info.spread_workgroups = D.sp.ngrid;
    H.info.interp_workgroups = D.ip.ngrid;
    H.info.fft_n1 = H.fd.n1;
    H.info.fft_n2 = H.fd.n2;
}

// Algorithm 2.2 step 0 without the nodes: parameters and their validation;
// H.info holds the parameters.
static nnfft_status plan_params(HostPlan &H, int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2,
                                int m1, int m2, nnfft_precision prec, int window)
{
    nnfft_info_t &P = H.info;
    P = nnfft_info_t{};
    nnfft_status st = derive_params(N, sigma1, sigma2, m1, m2, &P);
    if (st != NNFFT_OK) return fail(st, "invalid NNFFT parameters (N >= 1, m >= 2, sigma > 1, "
                                        "2 m1 < N1 and 2 m2 <= (1 - 1/sigma1) N2 are required)");
    // window family (Example 2.1): shape parameters and the sinh-only bound
    P.window = window;
    if (window == NNFFT_WINDOW_BSPLINE) {
        P.beta1 = P.beta2 = 0.0;
    } else if (window == NNFFT_WINDOW_ALGEBRAIC) {
        if (!(P.sigma1_eff > kPi / 3.0) || !(P.sigma2_eff > kPi / 3.0))
            return fail(NNFFT_ERR_ARG, "the algebraic window needs sigma > pi/3");
        P.beta1 = 3.0 * m1;
        P.beta2 = 3.0 * m2;
    } else if (window != NNFFT_WINDOW_SINH && window != NNFFT_WINDOW_KAISER_BESSEL) {
        return fail(NNFFT_ERR_ARG, "unknown window family");
    }
    if (window != NNFFT_WINDOW_SINH) {
        P.bound_thm41 = 0.0;
        P.thm41_applies = 0;
    }
    if (M1 < 1 || M2 < 1 || M1 > ((int64_t)1 << 30) || M2 > ((int64_t)1 << 30))
        return fail(NNFFT_ERR_ARG, "node counts must be in [1, 2^30]");
    if (prec != NNFFT_FP64_PLAIN && prec != NNFFT_FP32_COMP) return fail(NNFFT_ERR_ARG, "unknown precision");
    if (m1 > kMaxM || m2 > kMaxM) return fail(NNFFT_ERR_UNSUPPORTED, "m > 16 is not implemented");
    const bool fp32 = (prec == NNFFT_FP32_COMP);
    if (fp32 && (m1 < 4 || m2 < 4))
        return fail(NNFFT_ERR_UNSUPPORTED, "the FP32 path needs m >= 4 (its window polynomials "
                                           "cannot reach FP32 accuracy for smaller m)");
    if (P.N2 > ((int64_t)1 << 24) || P.G1 > ((int64_t)1 << 24) || (!fp32 && P.N2 > ((int64_t)1 << 22)))
        return fail(NNFFT_ERR_UNSUPPORTED, "FFT longer than 2^24 (FP32) or 2^22 (FP64)");

    P.M1 = M1;
    P.M2 = M2;
    P.precision = prec;
    H.fp32 = fp32;
    return NNFFT_OK;
}

// Tap series of a window: they depend on its family, m, beta and the degree
// only, so plans of every bandwidth share them (a short list, most recently
// used first).
struct TapSeries {
    int kind, m, deg;
    double beta;
    std::vector<double> c;
    double err;
};
constexpr size_t kTapCacheEntries = 32;
std::mutex g_taps_mu;
std::list<std::shared_ptr<const TapSeries>> g_taps;

static std::vector<double> window_taps_cached(const Window &w, int deg, double *max_err)
{
    {
        std::lock_guard<std::mutex> g(g_taps_mu);
        for (auto it = g_taps.begin(); it != g_taps.end(); ++it) {
            const TapSeries &t = **it;
            if (t.kind == w.kind && t.m == w.m && t.deg == deg && t.beta == w.beta) {
                *max_err = t.err;
                std::vector<double> c = t.c;
                g_taps.splice(g_taps.begin(), g_taps, it);
                return c;
            }
        }
    }
    auto t = std::make_shared<TapSeries>();
    t->kind = w.kind;
    t->m = w.m;
    t->deg = deg;
    t->beta = w.beta;
    t->c = fit_window_taps(w, deg, &t->err);
    *max_err = t->err;
    std::lock_guard<std::mutex> g(g_taps_mu);
    g_taps.push_front(t);
    if (g_taps.size() > kTapCacheEntries) g_taps.pop_back();
    return t->c;
}

// Twiddles exp(-2 pi i q / n) of an FFT length (shared by every plan of that
// length; a short list, most recently used first, bounded in entries and bytes).
constexpr size_t kTwCacheEntries = 128;
constexpr size_t kTwCacheBytes = (size_t)64 << 20;
std::mutex g_tw_mu;
std::list<std::pair<int64_t, std::shared_ptr<const std::vector<double>>>> g_tw;
size_t g_tw_bytes = 0;

static std::vector<double> twiddles_cached(int64_t n)
{
    {
        std::lock_guard<std::mutex> g(g_tw_mu);
        for (auto it = g_tw.begin(); it != g_tw.end(); ++it)
            if (it->first == n) {
                std::vector<double> t = *it->second;
                g_tw.splice(g_tw.begin(), g_tw, it);
                return t;
            }
    }
    auto t = std::make_shared<const std::vector<double>>(twiddles(n));
    const size_t bytes = t->size() * sizeof(double);
    if (bytes <= kTwCacheBytes / 8) {
        std::lock_guard<std::mutex> g(g_tw_mu);
        g_tw.emplace_front(n, t);
        g_tw_bytes += bytes;
        while (g_tw.size() > kTwCacheEntries || g_tw_bytes > kTwCacheBytes) {
            g_tw_bytes -= g_tw.back().second->size() * sizeof(double);
            g_tw.pop_back();
        }
    }
    return *t;
}

// The FP64 tables of a plan whose parameters plan_params set: window tap
// series, the 1/phi_hat_1 series, the phi_hat_2 deconvolution and the
// twiddles.  They depend on (N, sigma, m, precision, window) only and are
// kept in a small cache, so plans of repeated parameters skip them.
static nnfft_status plan_tables_compute(HostPlan &H)
{
    nnfft_info_t &P = H.info;
    const bool fp32 = H.fp32;
    const int m1 = P.m1, m2 = P.m2;
    const int window = P.window;
    // tables in FP64 -----------------------------------------------------
    double e1 = 0.0, e2 = 0.0;
    if (fp32) {
        const std::vector<double> c1 = window_taps_cached(make_window(P.window, m1, P.beta1), kDeg, &e1);
        const std::vector<double> c2 = window_taps_cached(make_window(P.window, m2, P.beta2), kDeg, &e2);
        P.window_degree = kDeg;
        P.window_fit_err = std::max(e1, e2);
        if (e1 > tap_fit_tolerance(m1, P.sigma1_eff) || e2 > tap_fit_tolerance(m2, P.sigma2_eff))
            return fail(NNFFT_ERR_UNSUPPORTED, "window polynomial misses FP32 accuracy for these sigma, m");
        H.C1.assign(c1.begin(), c1.end());
        H.C2.assign(c2.begin(), c2.end());
    } else if (window == NNFFT_WINDOW_BSPLINE) {
        // each tap is one polynomial piece of degree 2m - 1: its series is exact
        double t1 = 0.0, t2 = 0.0;
        H.T1 = window_taps_cached(make_window(window, m1, 0.0), 2 * m1 - 1, &t1);
        H.T2 = window_taps_cached(make_window(window, m2, 0.0), 2 * m2 - 1, &t2);
        if (std::max(t1, t2) > 1e-14)
            return fail(NNFFT_ERR_UNSUPPORTED, "B-spline tap series inexact");
    } else if (window == NNFFT_WINDOW_KAISER_BESSEL) {
        // the window's power series in 1 - u^2, evaluated per tap
        H.T1 = kaiser_bessel_series(P.beta1);
        H.T2 = kaiser_bessel_series(P.beta2);
    }
    double corr_err = 0.0;
    H.corr = fit_inverse_phi1(P, fp32 ? 1e-9 : 1e-14, fp32 ? kCorr32 : kMaxCorrDeg, &corr_err);
    P.corr_degree = (int32_t)H.corr.size() - 1;
    P.corr_fit_err = corr_err;
    if (corr_err > (fp32 ? 1e-8 : 1e-12))
        return fail(NNFFT_ERR_UNSUPPORTED, "1/phi_hat_1 series does not converge for this sigma1");
    if (fp32) H.corr.resize(kCorr32 + 1, 0.0);   // zero-padded to the unrolled length

    const Window w2 = make_window(P.window, m2, P.beta2);
    H.deconv.resize(P.G1);
    std::vector<double> hv((size_t)(P.G1 / 2 + 1)), ha(hv.size());
    for (int64_t c = 0; c <= P.G1 / 2; ++c) hv[(size_t)c] = m2 * (double)(P.G1 / 2 - c) / (double)P.N2;
    window_hat_many(w2, hv.data(), ha.data(), (int64_t)hv.size());
    for (int64_t c = 0; c <= P.G1 / 2; ++c) {   // phi_hat_2 is even: label -l shares the value of l
        const double phi2 = (double)m2 / (double)P.N2 * ha[(size_t)c];
        const double d = 1.0 / ((double)P.N1 * (double)P.N2 * phi2);
        H.deconv[c] = d;                                  // label -l
        if (c > 0 && P.G1 / 2 + (P.G1 / 2 - c) < P.G1) H.deconv[P.G1 / 2 + (P.G1 / 2 - c)] = d;   // label +l
    }
    H.tw64 = twiddles_cached(P.N2);
    if (fp32) {
        H.tw32.assign(H.tw64.begin(), H.tw64.end());
        H.tw64.clear();
    }
    return NNFFT_OK;
}

// Cache of the tables of recent parameter sets (least recently used out).
struct TableKey {
    int64_t N;
    double sigma1, sigma2;
    int m1, m2, prec, window;
    bool operator==(const TableKey &o) const
    {
        return N == o.N && sigma1 == o.sigma1 && sigma2 == o.sigma2 && m1 == o.m1 && m2 == o.m2 &&
               prec == o.prec && window == o.window;
    }
};
struct TableSet {
    TableKey key;
    int32_t window_degree, corr_degree;
    double window_fit_err, corr_fit_err;
    std::vector<float> C1, C2, tw32;
    std::vector<double> T1, T2, corr, deconv, tw64;
    size_t bytes = 0;
};
constexpr size_t kTableCacheEntries = 64;
constexpr size_t kTableCacheBytes = (size_t)256 << 20;
std::mutex g_tables_mu;
std::list<std::shared_ptr<const TableSet>> g_tables;   // most recent first
size_t g_tables_bytes = 0;

static nnfft_status plan_tables(HostPlan &H)
{
    const nnfft_info_t &P = H.info;
    const TableKey key{P.N, P.sigma1, P.sigma2, P.m1, P.m2, P.precision, P.window};
    std::shared_ptr<const TableSet> hit;
    {
        std::lock_guard<std::mutex> g(g_tables_mu);
        for (auto it = g_tables.begin(); it != g_tables.end(); ++it)
            if ((*it)->key == key) {
                hit = *it;
                g_tables.splice(g_tables.begin(), g_tables, it);
                break;
            }
    }
    if (hit) {
        H.info.window_degree = hit->window_degree;
        H.info.window_fit_err = hit->window_fit_err;
        H.info.corr_degree = hit->corr_degree;
        H.info.corr_fit_err = hit->corr_fit_err;
        H.C1 = hit->C1;
        H.C2 = hit->C2;
        H.T1 = hit->T1;
        H.T2 = hit->T2;
        H.corr = hit->corr;
        H.deconv = hit->deconv;
        H.tw64 = hit->tw64;
        H.tw32 = hit->tw32;
        return NNFFT_OK;
    }
    const nnfft_status st = plan_tables_compute(H);
    if (st != NNFFT_OK) return st;
    auto t = std::make_shared<TableSet>();
    t->key = key;
    t->window_degree = H.info.window_degree;
    t->window_fit_err = H.info.window_fit_err;
    t->corr_degree = H.info.corr_degree;
    t->corr_fit_err = H.info.corr_fit_err;
    t->C1 = H.C1;
    t->C2 = H.C2;
    t->T1 = H.T1;
    t->T2 = H.T2;
    t->corr = H.corr;
    t->deconv = H.deconv;
    t->tw64 = H.tw64;
    t->tw32 = H.tw32;
    t->bytes = 4 * (t->C1.size() + t->C2.size() + t->tw32.size()) +
               8 * (t->T1.size() + t->T2.size() + t->corr.size() + t->deconv.size() + t->tw64.size());
    if (t->bytes <= kTableCacheBytes / 4) {
        std::lock_guard<std::mutex> g(g_tables_mu);
        g_tables.push_front(t);
        g_tables_bytes += t->bytes;
        while (g_tables.size() > kTableCacheEntries || g_tables_bytes > kTableCacheBytes) {
            g_tables_bytes -= g_tables.back()->bytes;
            g_tables.pop_back();
        }
    }
    return NNFFT_OK;
}

// The rest of step 0 once both node sides are laid out: FFT factorization
// and tables, window planes, merge lists, sizes.
static nnfft_status plan_finish(HostPlan &H)
{
    const nnfft_info_t &P = H.info;
    const int m1 = P.m1, m2 = P.m2;
    const bool fp32 = H.fp32;
    nnfft_status st = NNFFT_OK;
    {
        const double U = (double)P.N2 * (double)P.N_star / (2.0 * (double)P.N1);
        const int64_t S = std::min<int64_t>((int64_t)std::ceil(U) + m2, P.N2 / 2);
        st = plan_fft(H, P, fp32, S);
        if (st != NNFFT_OK) return st;
    }
    fft_tables(H);
    finalize_planes(H, P.G1);
    if (H.sp.part_cells >= ((int64_t)1 << 31)) return fail(NNFFT_ERR_UNSUPPORTED, "too many partial cells");
    st = build_merge_lists(H, P, m1);
    if (st != NNFFT_OK) return st;
    {
        // the deconvolution table in slot order, as the FFT load reads it
        std::vector<double> d((size_t)H.slotT * H.slotP, 0.0);
        for (int64_t c = 0; c < P.G1; ++c) d[slot_of(H, c)] = H.deconv[c];
        H.deconv.swap(d);
    }
    H.hlin_len = P.N2 + 1;
    H.h_off = P.N2 / 2;
    size_plan(H, P);
    return NNFFT_OK;
}

nnfft_status plan_host(HostPlan &H, int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2,
                       int m1, int m2, nnfft_precision prec, const std::vector<double> &v,
                       const std::vector<double> &x, const Layout *lay1, const Layout *lay2, int window)
{
    nnfft_status st = plan_params(H, N, M1, M2, sigma1, sigma2, m1, m2, prec, window);
    if (st == NNFFT_OK) st = plan_tables(H);
    if (st != NNFFT_OK) return st;
    const nnfft_info_t &P = H.info;
    const bool fp32 = H.fp32;
    if ((int64_t)v.size() != M1 || (int64_t)x.size() != M2) return fail(NNFFT_ERR_ARG, "node array sizes");
    for (int64_t k = 0; k < M1; ++k)
        if (!(std::fabs(v[k]) <= 0.5)) return fail(NNFFT_ERR_DOMAIN, "frequency node outside [-1/2, 1/2]");
    for (int64_t j = 0; j < M2; ++j)
        if (!(std::fabs(x[j]) <= 0.5)) return fail(NNFFT_ERR_DOMAIN, "spatial node outside [-1/2, 1/2]");
    // node layouts ----------------------------------------------------------
    const double scale1 = (double)P.N1 * (double)N / (double)P.N_star;   // t_k = scale1 v_k
    const double scale2 = (double)P.N2 * (double)P.N_star / (double)P.N1; // u_j = scale2 x_j
    H.lay1 = lay1 ? sanitize_layout(*lay1, M1, fp32) : choose_layout_nodes(v, scale1, fp32, true);
    H.lay2 = lay2 ? sanitize_layout(*lay2, M2, fp32) : choose_layout_nodes(x, scale2, fp32, false);
    std::string err;
    // spreading: t_k = N1 v*_k = N1 N v_k / N*, bin = floor(t_k) + G1/2
    // interpolation: u_j = N2 N* x_j / N1, bin = floor(u_j) + N2/2
    if (!build_both_sides(
            [&](std::string &e) { return build_side(v, scale1, P.G1 / 2, P.G1, H.lay1, fp32, m1, H.sp, e); },
            [&](std::string &e) { return build_side(x, scale2, P.N2 / 2, P.N2 + 1, H.lay2, fp32, 0, H.ip, e); },
            std::min(M1, M2) >= kParallelSidePoints, err))
        return fail(NNFFT_ERR_ARG, err);
    // the sorted copies are only needed by the FP64 kernels
    if (fp32) {
        std::vector<int32_t>().swap(H.sp.perm);
        std::vector<int32_t>().swap(H.ip.perm);
    }
    std::vector<PtRec>().swap(H.sp.rec32);
    std::vector<PtRec>().swap(H.ip.rec32);
    return plan_finish(H);
}


nnfft_status nfft_plan_host(HostPlan &H, int64_t N, int64_t M, double sigma, int m, nnfft_precision prec,
                            const std::vector<double> &x)
{
    if (N < 2 || (N % 2)) return fail(NNFFT_ERR_ARG, "the NFFT needs an even N >= 2");
    if (M < 1 || M > ((int64_t)1 << 30)) return fail(NNFFT_ERR_ARG, "node count must be in [1, 2^30]");
    if (!(sigma > 1.0) || m < 2) return fail(NNFFT_ERR_ARG, "sigma > 1 and m >= 2 are required");
    if (prec != NNFFT_FP64_PLAIN && prec != NNFFT_FP32_COMP) return fail(NNFFT_ERR_ARG, "unknown precision");
    if ((int64_t)x.size() != M) return fail(NNFFT_ERR_ARG, "node array size");
    if (m > kMaxM) return fail(NNFFT_ERR_UNSUPPORTED, "m > 16 is not implemented");
    const bool fp32 = (prec == NNFFT_FP32_COMP);
    if (fp32 && m < 4)
        return fail(NNFFT_ERR_UNSUPPORTED, "the FP32 path needs m >= 4 (its window polynomials "
                                           "cannot reach FP32 accuracy for smaller m)");
    for (int64_t j = 0; j < M; ++j)
        if (!(std::fabs(x[j]) <= 0.5)) return fail(NNFFT_ERR_DOMAIN, "node outside [-1/2, 1/2]");
    // oversampled length: the smallest even 2,3,5-smooth integer >= sigma N
    int64_t n = (int64_t)std::ceil(sigma * (double)N - 1e-9);
    if (n % 2) ++n;
    while (radix_passes(n).empty()) n += 2;
    if (2 * m >= n) return fail(NNFFT_ERR_ARG, "2 m must be smaller than the oversampled length");
    if (n > ((int64_t)1 << (fp32 ? 24 : 22)))
        return fail(NNFFT_ERR_UNSUPPORTED, "FFT longer than 2^24 (FP32) or 2^22 (FP64)");

    nnfft_info_t P{};
    P.N = N;
    P.N_star = N;
    P.N1 = n;
    P.G1 = n + 2 * m + 2;   // linear spreading grid: labels [-G1/2, G1/2) hold every window
    P.N2 = n;
    P.M1 = M;
    P.M2 = M;
    P.m1 = P.m2 = m;
    P.precision = prec;
    P.sigma1 = P.sigma2 = sigma;
    P.sigma1_eff = P.sigma2_eff = (double)n / (double)N;
    P.a = (double)P.G1 / (double)n;
    P.beta1 = P.beta2 = 2.0 * kPi * m * (1.0 - (double)N / (2.0 * (double)n));
    P.thm41_applies = 0;
    H.kind = 1;
    H.fp32 = fp32;
    if (fp32) {
        double e = 0.0;
        const std::vector<double> c = window_taps_cached(make_window(NNFFT_WINDOW_SINH, m, P.beta1), kDeg, &e);
        P.window_degree = kDeg;
        P.window_fit_err = e;
        if (e > tap_fit_tolerance(m, P.sigma1_eff))
            return fail(NNFFT_ERR_UNSUPPORTED, "window polynomial misses FP32 accuracy for these sigma, m");
        H.C1.assign(c.begin(), c.end());
        H.C2 = H.C1;
    }
    // no correction after the interpolation: the series of the constant 1
    H.corr.assign(fp32 ? kCorr32 + 1 : 1, 0.0);
    H.corr[0] = 1.0;
    P.corr_degree = 0;
    P.corr_fit_err = 0.0;
    // 1 / (n phi_hat(k)) = 1 / (m omega_hat(m k / n)), k in I_N
    H.deconv.resize(N);
    for (int64_t k = -N / 2; k < N / 2; ++k)
        H.deconv[k + N / 2] = 1.0 / ((double)m * window_sinh_hat((double)m * (double)k / (double)n, P.beta1));
    H.tw64 = twiddles(n);
    if (fp32) {
        H.tw32.assign(H.tw64.begin(), H.tw64.end());
        H.tw64.clear();
    }
    H.lay1 = choose_layout_nodes(x, (double)n, fp32, true);
    H.lay2 = choose_layout_nodes(x, (double)n, fp32, false);
    std::string err;
    // spreading (adjoint): t_j = n x_j in the linear grid; interpolation (forward): u_j = n x_j
    if (!build_both_sides(
            [&](std::string &e) { return build_side(x, (double)n, P.G1 / 2, P.G1, H.lay1, fp32, m, H.sp, e); },
            [&](std::string &e) { return build_side(x, (double)n, n / 2, n + 1, H.lay2, fp32, 0, H.ip, e); },
            M >= kParallelSidePoints, err))
        return fail(NNFFT_ERR_ARG, err);
    if (fp32) {
        std::vector<int32_t>().swap(H.sp.perm);
        std::vector<int32_t>().swap(H.ip.perm);
    }
    std::vector<PtRec>().swap(H.sp.rec32);
    std::vector<PtRec>().swap(H.ip.rec32);
    // the interpolation reads labels |s| <= n/2 + m: the periodic extension
    nnfft_status st = plan_fft(H, P, fp32, n / 2 + m);
    if (st != NNFFT_OK) return st;
    fft_tables(H);
    finalize_planes(H, P.G1);
    if (H.sp.part_cells >= ((int64_t)1 << 31)) return fail(NNFFT_ERR_UNSUPPORTED, "too many partial cells");
    st = build_merge_lists(H, P, m);
    if (st != NNFFT_OK) return st;
    H.hlin_len = n + 2 * m + 1;
    H.h_off = (int32_t)(n / 2 + m);
    size_plan(H, P);
    return NNFFT_OK;
}

// Checks the invariants the kernels rely on: every point in exactly one
// item of at most Q points of one bin, chunks within 64 bins, FP32 record
// blocks matching the items, spreading windows inside the grid with no two
// windows of one plane sharing a cell, overflow windows disjoint and listed
// in the merge lists exactly once per cell.
nnfft_status check_plan(const HostPlan &H, const std::vector<double> &v, const std::vector<double> &x)
{
    const nnfft_info_t &P = H.info;
    auto side = [&](const SideHost &S, const Layout &L, int64_t M, int64_t nbins, int m, const char *name) {
        std::vector<char> seen(M, 0);
        const size_t rows = (size_t)L.Q;
        for (size_t g = 0; g < S.launch.size(); ++g) {
            const Chunk &c = S.launch[g];
            if (c.nitem < 0 || c.nitem > kItemsPerWg || c.nbin < 0 || c.nbin > kItemsPerWg)
                return std::string(name) + ": chunk size";
            for (int t = 0; t < kItemsPerWg; ++t) {
                const Item &it = S.launch_items[g * kItemsPerWg + t];
                if (t >= c.nitem) {
                    if (it.n != 0) return std::string(name) + ": padding item with points";
                    continue;
                }
                if (it.n < 1 || it.n > L.Q) return std::string(name) + ": item size";
                if (t == 0) {
                    int run = 1, maxrun = 1;
                    for (int u = 1; u < c.nitem; ++u) {
                        const int b0 = S.launch_items[g * kItemsPerWg + u - 1].bin;
                        run = (S.launch_items[g * kItemsPerWg + u].bin == b0) ? run + 1 : 1;
                        maxrun = std::max(maxrun, run);
                    }
                    if (it.maxrun != maxrun) return std::string(name) + ": chunk's longest bin run";
                } else if (it.maxrun != 0) {
                    return std::string(name) + ": run length outside a chunk's first item";
                }
                if (it.bin < c.bin_lo || it.bin >= c.bin_lo + c.nbin || it.bin >= nbins)
                    return std::string(name) + ": item bin outside its chunk";
                for (int q = 0; q < it.n; ++q) {
                    const int64_t k = H.fp32 ? S.trec32[(g * rows + q) * kItemsPerWg + t].perm
                                             : S.perm[(size_t)(it.p0 + q)];
                    if (k < 0 || k >= M || seen[k]) return std::string(name) + ": point listed twice or lost";
                    seen[k] = 1;
                }
                if (H.fp32)
                    for (size_t q = it.n; q < rows; ++q)
                        if (S.trec32[(g * rows + q) * kItemsPerWg + t].perm !=
                            S.trec32[(g * rows + it.n - 1) * kItemsPerWg + t].perm)
                            return std::string(name) + ": record padding";
            }
        }
        for (int64_t k = 0; k < M; ++k)
            if (!seen[k]) return std::string(name) + ": point not in any item";
        (void)m;
        return std::string();
    };
    std::string e;
    if (!build_both_sides(
            [&](std::string &r) {
                r = side(H.sp, H.lay1, P.M1, P.G1, P.m1, "spreading");
                return r.empty();
            },
            [&](std::string &r) {
                r = side(H.ip, H.lay2, P.M2, P.N2 + 1, P.m2, "interpolation");
                return r.empty();
            },
            std::min(P.M1, P.M2) >= kParallelSidePoints, e))
        return fail(NNFFT_ERR_ARG, "internal: " + e);
    (void)v;
    (void)x;
    // spreading windows
    const int64_t G1 = P.G1, W0 = 2 * (int64_t)P.m1 - 1;
    const int64_t T = H.slotT, Ps = H.slotP, ps = T * Ps;
    const int64_t plane_cells = (int64_t)H.sp.nplanes * ps;
    if (T < 1 || Ps * T < G1 || (H.fd.n1 > 1 && T != H.fd.n1) || (int64_t)H.moff.size() != ps + 1 ||
        (H.kind == 0 && (int64_t)H.deconv.size() != ps))
        return fail(NNFFT_ERR_ARG, "internal: slot layout of the planes");
    std::vector<int32_t> owner((size_t)H.sp.part_cells, -1), ovf_count(G1, 0);
    std::vector<int64_t> cell_of((size_t)H.sp.part_cells, -1);   // overflow partial cell -> grid cell
    for (size_t c = 0; c < H.sp.chunks.size(); ++c) {
        const Chunk &ch = H.sp.chunks[c];
        const int64_t lo = (int64_t)ch.bin_lo - P.m1 + 1, W = ch.nbin + W0;
        if (lo < 0 || lo + W > G1) return fail(NNFFT_ERR_ARG, "internal: window outside the grid");
        const bool in_plane = ch.part_off < 0;
        if (in_plane && -(int64_t)ch.part_off > H.sp.nplanes) return fail(NNFFT_ERR_ARG, "internal: no such plane");
        if (!in_plane && (ch.part_off < plane_cells || ch.part_off + W > H.sp.part_cells))
            return fail(NNFFT_ERR_ARG, "internal: window outside the partial buffer");
        for (int64_t w = 0; w < W; ++w) {
            const int64_t cell = lo + w;
            const int64_t idx = in_plane ? (-(int64_t)ch.part_off - 1) * ps + (cell % T) * Ps + cell / T
                                         : ch.part_off + w;
            if (idx < 0 || idx >= H.sp.part_cells) return fail(NNFFT_ERR_ARG, "internal: partial index out of range");
            if (owner[idx] >= 0) return fail(NNFFT_ERR_ARG, "internal: two windows share a partial cell");
            owner[idx] = (int32_t)c;
            if (!in_plane) {
                ovf_count[cell]++;
                cell_of[idx] = cell;
            }
        }
    }
    {
        // the launch-order copies carry the same windows
        std::vector<std::array<int32_t, 4>> a, b;
        for (const Chunk &ch : H.sp.chunks) a.push_back({ch.bin_lo, ch.nbin, ch.part_off, ch.nitem});
        for (const Chunk &ch : H.sp.launch)
            if (ch.nitem > 0) b.push_back({ch.bin_lo, ch.nbin, ch.part_off, ch.nitem});
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        if (a != b) return fail(NNFFT_ERR_ARG, "internal: launch chunks differ from the chunks");
    }
    // every overflow partial cell is merged exactly once, into its own grid
    // cell: directly from the cell's list, or through one pre-merge segment
    // named there (each segment named once)
    if ((int64_t)H.pm_seg.size() != 2 * H.pm_cells || H.pm_base + H.pm_cells != H.sp.part_cells)
        return fail(NNFFT_ERR_ARG, "internal: pre-merge segments");
    std::vector<char> merged((size_t)H.sp.part_cells, 0), seg_used((size_t)H.pm_cells, 0);
    auto take = [&](int64_t e2, int64_t cell) {
        if (e2 < plane_cells || e2 >= H.pm_base || owner[e2] < 0 || cell_of[e2] != cell || merged[e2]) return false;
        merged[e2] = 1;
        return true;
    };
    for (int64_t cell = 0; cell < G1; ++cell) {
        const int64_t sl = (cell % T) * Ps + cell / T;
        int64_t n = 0;
        for (int32_t e = H.moff[sl]; e < H.moff[sl + 1]; ++e) {
            const int64_t e2 = H.midx[e];
            if (e2 >= H.pm_base) {
                const int64_t sg = e2 - H.pm_base;
                if (sg >= H.pm_cells || seg_used[sg]) return fail(NNFFT_ERR_ARG, "internal: pre-merge segment reuse");
                seg_used[sg] = 1;
                const int32_t i0 = H.pm_seg[2 * sg], cnt = H.pm_seg[2 * sg + 1];
                if (i0 < 0 || cnt < 1 || (size_t)i0 + cnt > H.pm_idx.size())
                    return fail(NNFFT_ERR_ARG, "internal: pre-merge segment range");
                for (int32_t q = 0; q < cnt; ++q)
                    if (!take(H.pm_idx[i0 + q], cell))
                        return fail(NNFFT_ERR_ARG, "internal: pre-merge entry outside the cell's overflow windows");
                n += cnt;
            } else {
                if (!take(e2, cell)) return fail(NNFFT_ERR_ARG, "internal: merge list entry outside the overflow windows");
                ++n;
            }
        }
        if (n != ovf_count[cell]) return fail(NNFFT_ERR_ARG, "internal: merge list does not match the overflow windows");
        if (H.moff[sl + 1] - H.moff[sl] > kMergeDirect) return fail(NNFFT_ERR_ARG, "internal: merge list too long");
    }
    return NNFFT_OK;
}

uint64_t fnv1a64(const void *p, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

nnfft_status plan_create(const HostPlan &H, const DevMem &mem, hipStream_t s, nnfft_plan_t *out,
                         const DevRecords *dev)
{
    *out = nullptr;
    void *base = mem.alloc(mem.ctx, H.total_bytes);
    if (!base) return fail(NNFFT_ERR_NOMEM, "device memory for the plan (" + std::to_string(H.total_bytes) +
                                                " bytes) is not available");
    nnfft_plan_s *pl = new (std::nothrow) nnfft_plan_s();
    if (!pl) {
        mem.release(mem.ctx, base);
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
    pl->base = base;
    pl->mem = mem;
    pl->info = H.info;
    pl->kind = H.kind;
    {
        const size_t csz = H.fp32 ? 8 : 16;
        pl->scratch.part_bytes = (size_t)H.sp.part_cells * 16;
        pl->scratch.plane_bytes = (size_t)H.sp.nplanes * (size_t)H.slotT * (size_t)H.slotP * 16;
        pl->scratch.y_bytes = (size_t)H.info.N2 * csz;
        pl->scratch.hlin_bytes = (size_t)H.hlin_len * csz;
    }
    try {
        std::vector<char> stage;
        stage.reserve(H.upload_bytes);   // the image grows to this size (no reallocation)
        Carver C((uintptr_t)base, &stage);
        size_t upload_end = 0, dev_start = 0;
        layout_plan(H, C, pl->desc, &upload_end, &pl->ddesc, &dev_start);
        pl->upload_bytes = upload_end;
        const size_t up = dev ? dev_start : upload_end;   // device-written records follow dev_start
        if (stage.size() < up) stage.resize(up);
        hip_check(hipMemcpyAsync(base, stage.data(), up, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
        // plane cells that no window covers are read as zeros by every exec;
        // the planes follow the device-written records (layout_plan), so one
        // fill clears both where the records are written on the device
        const size_t part_off = (size_t)(static_cast<const char *>(pl->desc.sp.partial) - static_cast<char *>(base));
        const size_t part_end = part_off + (size_t)H.sp.part_cells * 16;
        if (dev) {
            // the gaps between the device-written arrays (alignment) read as
            // zeros, as in the host image; the record kernels fill the rest
            hip_check(hipMemsetAsync(static_cast<char *>(base) + dev_start, 0, part_end - dev_start, s),
                      "hipMemsetAsync");
            const PlanDev &D = pl->desc;
            auto rec_side = [&](const SideHost &S, const DevSideRecords &R, const Item *items, const PtRec *rec32,
                                const int32_t *perm, const double *frac) {
                return RecSide{R.x, R.sorted, R.scale, S.npts, items, (int64_t)S.launch.size(), S.rows,
                               const_cast<PtRec *>(rec32), const_cast<int32_t *>(perm), const_cast<double *>(frac)};
            };
            if (H.sp.dev && H.ip.dev) {   // both sides in one launch
                hip_check(device_records_pair(H.fp32, rec_side(H.sp, dev->sp, D.sp.items, D.sp.rec32, D.sp.perm,
                                                               D.sp.frac64),
                                              rec_side(H.ip, dev->ip, D.ip.items, D.ip.rec32, D.ip.perm, D.ip.frac64),
                                              s),
                          "records");
            } else {
                auto side = [&](const SideHost &S, const DevSideRecords &R, const Item *items, const PtRec *rec32,
                                const int32_t *perm, const double *frac) {
                    if (!S.dev) return;
                    if (H.fp32) {
                        hip_check(device_transposed_records(R.x, R.sorted, R.scale, items, (int64_t)S.launch.size(),
                                                            S.rows, const_cast<PtRec *>(rec32), s),
                                  "transposed records");
                    } else {
                        hip_check(device_sorted_records(R.x, R.sorted, S.npts, R.scale, false,
                                                        const_cast<int32_t *>(perm), const_cast<double *>(frac),
                                                        nullptr, s),
                                  "sorted records");
                    }
                };
                side(H.sp, dev->sp, D.sp.items, D.sp.rec32, D.sp.perm, D.sp.frac64);
                side(H.ip, dev->ip, D.ip.items, D.ip.rec32, D.ip.perm, D.ip.frac64);
            }
        }
        hip_check(hipMemcpyAsync(pl->ddesc, &pl->desc, sizeof(PlanDev), hipMemcpyHostToDevice, s),
                  "hipMemcpyAsync");
        if (!dev) hip_check(hipMemsetAsync(pl->desc.sp.partial, 0, (size_t)H.sp.part_cells * 16, s), "hipMemsetAsync");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    } catch (const HipError &e) {
        (void)hipStreamSynchronize(s);   // nothing queued may still write into the released block
        delete pl;
        return fail(NNFFT_ERR_DEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));
    } catch (const std::bad_alloc &) {
        (void)hipStreamSynchronize(s);
        delete pl;
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
    *out = pl;
    return NNFFT_OK;
}

NodePrepScratch::~NodePrepScratch()
{
    if (dev) (void)hipFree(dev);
    if (pin) (void)hipHostFree(pin);
}

bool NodePrepScratch::reserve(size_t dev_need, size_t pin_need)
{
    if (dev_need > dev_bytes) {
        if (dev) (void)hipFree(dev);
        dev = nullptr;
        dev_bytes = 0;
        if (hipMalloc(&dev, dev_need) != hipSuccess) {
            (void)hipGetLastError();
            dev = nullptr;
            return false;
        }
        dev_bytes = dev_need;
    }
    if (pin_need > pin_bytes) {
        if (pin) (void)hipHostFree(pin);
        pin = nullptr;
        pin_bytes = 0;
        if (hipHostMalloc(&pin, pin_need, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            pin = nullptr;
            return false;
        }
        pin_bytes = pin_need;
    }
    return true;
}

namespace {

// Node-sort scratch of nnfft_plan calls, kept between calls (a plan of up to
// 2^22 points per side fits the kept ones; larger ones are released after
// their plan): each call leases one, concurrent calls get their own.
// (The pool is never destroyed: its memory goes with the process, not with a
// static destructor that could run after the HIP runtime's own teardown.)
constexpr size_t kKeptScratchBytes = (size_t)256 << 20;
std::mutex g_scratch_mu;
std::vector<std::unique_ptr<NodePrepScratch>> &g_scratch_pool = *new std::vector<std::unique_ptr<NodePrepScratch>>();

struct ScratchLease {
    std::unique_ptr<NodePrepScratch> s;
    ScratchLease()
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (!g_scratch_pool.empty()) {
            s = std::move(g_scratch_pool.back());
            g_scratch_pool.pop_back();
        }
        if (!s) s.reset(new NodePrepScratch());
    }
    ~ScratchLease()
    {
        if (s->dev_bytes > kKeptScratchBytes) return;   // freed with s
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (g_scratch_pool.size() < 4) g_scratch_pool.push_back(std::move(s));
    }
    NodePrepScratch &operator*() { return *s; }
};

// One node side being prepared on the device: inputs, layout and its parts
// of the scratch memory.
struct DevSide {
    const double *x = nullptr;
    int64_t M = 0, off = 0, nbins = 0, nblocks = 0;
    double scale = 0.0;
    bool spreading = false;
    int m = 0;
    const char *what = "";
    Layout L;
    std::vector<int64_t> sidx;          // density sample indices
    size_t sort_b = 0, cnt_b = 0, smp_b = 0;
    // device
    void *sort_tmp = nullptr;
    int32_t *counts = nullptr, *flag = nullptr, *sorted = nullptr;
    int64_t *sidx_dev = nullptr;
    double *svals_dev = nullptr;
    // pinned host
    int32_t *counts_h = nullptr, *flag_h = nullptr;
    int64_t *sidx_h = nullptr;
    double *svals_h = nullptr;
};

size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

// Host plan of an NNFFT whose nodes are on the device.  Both node sides are
// ordered on the GPU (keys with the domain check, bin counts of the node
// blocks, the stable sort, density samples) while the host computes the
// tables; after one synchronization the host builds both sides' schedules
// from the counts alone (block_schedule, finish_side: the code of the host
// layout, so both agree exactly), on two threads.  plan_create then writes
// the point records on the device from R.  Sets *host and does nothing where
// the sort keys do not fit 32 bits.
nnfft_status plan_device_nodes(HostPlan &H, DevRecords &R, NodePrepScratch &T, int64_t N, int64_t M1, int64_t M2,
                               double sigma1, double sigma2, int m1, int m2, nnfft_precision prec, int window,
                               const double *v, const double *x, hipStream_t s, bool *host)
{
    *host = false;
    nnfft_status st = plan_params(H, N, M1, M2, sigma1, sigma2, m1, m2, prec, window);
    if (st != NNFFT_OK) return st;
    const nnfft_info_t &P = H.info;
    const bool fp32 = H.fp32;
    DevSide sd[2];
    sd[0].x = v;
    sd[0].M = M1;
    sd[0].scale = (double)P.N1 * (double)N / (double)P.N_star;   // t_k = N1 v*_k
    sd[0].off = P.G1 / 2;
    sd[0].nbins = P.G1;
    sd[0].spreading = true;
    sd[0].m = m1;
    sd[0].what = "frequency";
    sd[1].x = x;
    sd[1].M = M2;
    sd[1].scale = (double)P.N2 * (double)P.N_star / (double)P.N1;   // u_j = N2 N* x_j / N1
    sd[1].off = P.N2 / 2;
    sd[1].nbins = P.N2 + 1;
    sd[1].spreading = false;
    sd[1].m = 0;
    sd[1].what = "spatial";
    for (DevSide &d : sd) {
        d.L = choose_layout(d.M, fp32, d.spreading);
        if (!device_sort_fits(d.M, d.nbins, d.L.block) || !(std::fabs(d.scale) <= (double)((int64_t)1 << 26))) {
            *host = true;
            return NNFFT_OK;
        }
        d.nblocks = (d.M + d.L.block - 1) / d.L.block;
        d.sidx = density_sample_indices(d.M, d.L, fp32);
        d.sort_b = al256(device_sort_tmp_bytes(d.M));
        d.cnt_b = al256((size_t)d.nblocks * (size_t)d.nbins * 4);
        d.smp_b = al256(std::max<size_t>(1, d.sidx.size()) * 8);
    }
    auto sort_side = [&](DevSide &d) {
        return SortSide{d.x, d.M, d.scale, d.off, d.nbins, d.L.block, d.counts, d.flag};
    };
    // both sides in one sort where their keys fit 31 bits: one set of
    // launches and one read-back each for the counts and the samples.
    // Device: [sort scratch][counts 0][counts 1][flags][samples 0][samples 1]
    // [values 0][values 1]; pinned: the same from the counts on.
    const bool pair = device_sort_pair_fits(sort_side(sd[0]), sort_side(sd[1]));
    size_t dev_need = 0, pin_need = 0;
    if (pair) {
        const size_t tmp_b = al256(device_sort_tmp_bytes(sd[0].M + sd[1].M));
        pin_need = sd[0].cnt_b + sd[1].cnt_b + 256 + 2 * (sd[0].smp_b + sd[1].smp_b);
        dev_need = tmp_b + pin_need;
        if (!T.reserve(dev_need, pin_need))
            return fail(NNFFT_ERR_NOMEM, "memory for the node preparation is not available");
        unsigned char *pd = static_cast<unsigned char *>(T.dev), *ph = static_cast<unsigned char *>(T.pin);
        size_t o = 0;
        for (DevSide &d : sd) {
            d.sort_tmp = pd;   // shared by both sides' sort
            d.counts = reinterpret_cast<int32_t *>(pd + tmp_b + o);
            d.counts_h = reinterpret_cast<int32_t *>(ph + o);
            o += d.cnt_b;
        }
        for (int i = 0; i < 2; ++i) {
            sd[i].flag = reinterpret_cast<int32_t *>(pd + tmp_b + o) + i;
            sd[i].flag_h = reinterpret_cast<int32_t *>(ph + o) + i;
        }
        o += 256;
        for (DevSide &d : sd) {
            d.sidx_dev = reinterpret_cast<int64_t *>(pd + tmp_b + o);
            d.sidx_h = reinterpret_cast<int64_t *>(ph + o);
            o += d.smp_b;
        }
        for (DevSide &d : sd) {
            d.svals_dev = reinterpret_cast<double *>(pd + tmp_b + o);
            d.svals_h = reinterpret_cast<double *>(ph + o);
            o += d.smp_b;
        }
        for (DevSide &d : sd) std::copy(d.sidx.begin(), d.sidx.end(), d.sidx_h);
    } else {
        for (DevSide &d : sd) {
            dev_need += d.sort_b + d.cnt_b + 256 + 2 * d.smp_b;
            pin_need += d.cnt_b + 256 + 2 * d.smp_b;
        }
        if (!T.reserve(dev_need, pin_need))
            return fail(NNFFT_ERR_NOMEM, "memory for the node preparation is not available");
        unsigned char *pd = static_cast<unsigned char *>(T.dev), *ph = static_cast<unsigned char *>(T.pin);
        for (DevSide &d : sd) {
            d.sort_tmp = pd;
            d.counts = reinterpret_cast<int32_t *>(pd + d.sort_b);
            d.flag = reinterpret_cast<int32_t *>(pd + d.sort_b + d.cnt_b);
            d.sidx_dev = reinterpret_cast<int64_t *>(pd + d.sort_b + d.cnt_b + 256);
            d.svals_dev = reinterpret_cast<double *>(pd + d.sort_b + d.cnt_b + 256 + d.smp_b);
            pd += d.sort_b + d.cnt_b + 256 + 2 * d.smp_b;
            d.counts_h = reinterpret_cast<int32_t *>(ph);
            d.flag_h = reinterpret_cast<int32_t *>(ph + d.cnt_b);
            d.sidx_h = reinterpret_cast<int64_t *>(ph + d.cnt_b + 256);
            d.svals_h = reinterpret_cast<double *>(ph + d.cnt_b + 256 + d.smp_b);
            ph += d.cnt_b + 256 + 2 * d.smp_b;
            std::copy(d.sidx.begin(), d.sidx.end(), d.sidx_h);
        }
    }
    // device work of both sides, then the tables on the host meanwhile
    if (pair) {
        const size_t cnt_all = sd[0].cnt_b + sd[1].cnt_b + 256, smp_all = sd[0].smp_b + sd[1].smp_b;
        hip_check(hipMemsetAsync(sd[0].counts, 0, cnt_all, s), "hipMemsetAsync");
        hip_check(device_sort_node_pair(sort_side(sd[0]), sort_side(sd[1]), sd[0].sort_tmp, &sd[0].sorted,
                                        &sd[1].sorted, s),
                  "node sort");
        if (!sd[0].sidx.empty() || !sd[1].sidx.empty()) {
            hip_check(hipMemcpyAsync(sd[0].sidx_dev, sd[0].sidx_h, smp_all, hipMemcpyHostToDevice, s),
                      "hipMemcpyAsync");
            hip_check(device_gather_pair(sd[0].x, sd[0].sidx_dev, (int64_t)sd[0].sidx.size(), sd[0].svals_dev, sd[1].x,
                                         sd[1].sidx_dev, (int64_t)sd[1].sidx.size(), sd[1].svals_dev, s),
                      "density samples");
            hip_check(hipMemcpyAsync(sd[0].svals_h, sd[0].svals_dev, smp_all, hipMemcpyDeviceToHost, s),
                      "hipMemcpyAsync");
        }
        hip_check(hipMemcpyAsync(sd[0].counts_h, sd[0].counts, cnt_all, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    } else {
        for (DevSide &d : sd) {
            hip_check(hipMemsetAsync(d.counts, 0, d.cnt_b + 256, s), "hipMemsetAsync");
            hip_check(device_sort_nodes(d.x, d.M, d.scale, d.off, d.nbins, d.L.block, d.counts, d.flag, d.sort_tmp,
                                        &d.sorted, s),
                      "node sort");
            if (!d.sidx.empty()) {
                hip_check(hipMemcpyAsync(d.sidx_dev, d.sidx_h, d.sidx.size() * 8, hipMemcpyHostToDevice, s),
                          "hipMemcpyAsync");
                hip_check(device_gather(d.x, d.sidx_dev, (int64_t)d.sidx.size(), d.svals_dev, s), "density samples");
                hip_check(hipMemcpyAsync(d.svals_h, d.svals_dev, d.sidx.size() * 8, hipMemcpyDeviceToHost, s),
                          "hipMemcpyAsync");
            }
            hip_check(hipMemcpyAsync(d.counts_h, d.counts, d.cnt_b + 256, hipMemcpyDeviceToHost, s),
                      "hipMemcpyAsync");
        }
    }
    st = plan_tables(H);
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st != NNFFT_OK) return st;
    for (DevSide &d : sd) {
        if (*d.flag_h & 1) return fail(NNFFT_ERR_DOMAIN, std::string(d.what) + " node outside [-1/2, 1/2]");
        if (*d.flag_h & 2) return fail(NNFFT_ERR_ARG, "internal: node record outside the grid");
    }
    SideHost *S[2] = {&H.sp, &H.ip};
    Layout *Ls[2] = {&H.lay1, &H.lay2};
    auto schedule = [&](int i, std::string &err) {
        DevSide &d = sd[i];
        d.L = raise_item_size(d.L, d.M, d.scale, fp32, d.svals_h);
        *Ls[i] = d.L;
        SideHost &Sd = *S[i];
        Sd = SideHost{};
        Sd.nblocks = d.nblocks;
        Sd.rows = d.L.Q;
        Sd.npts = d.M;
        Sd.dev = true;
        std::vector<BlockOut> outs((size_t)d.nblocks);
        for (int64_t blk = 0; blk < d.nblocks; ++blk)
            block_schedule(d.counts_h + (size_t)blk * (size_t)d.nbins, d.nbins, blk * d.L.block, d.L.Q,
                           outs[(size_t)blk]);
        if (!finish_side(outs, d.m, Sd, err)) return false;
        if (fp32 && (int64_t)Sd.launch.size() * d.L.Q * kItemsPerWg >= ((int64_t)1 << 31)) {
            err = "too many padded records";
            return false;
        }
        return true;
    };
    std::string err;
    if (!build_both_sides([&](std::string &e) { return schedule(0, e); }, [&](std::string &e) { return schedule(1, e); },
                          std::min(M1, M2) >= kParallelSidePoints, err))
        return fail(NNFFT_ERR_ARG, err);
    st = plan_finish(H);
    if (st != NNFFT_OK) return st;
    R.sp = DevSideRecords{v, sd[0].sorted, sd[0].scale};
    R.ip = DevSideRecords{x, sd[1].sorted, sd[1].scale};
    return NNFFT_OK;
}

nnfft_status copy_nodes(const double *d, int64_t n, std::vector<double> &h, hipStream_t s)
{
    h.resize(n);
    if (n == 0) return NNFFT_OK;
    hipError_t e = hipMemcpyAsync(h.data(), d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("copying nodes: ") + hipGetErrorString(e));
    return NNFFT_OK;
}

// The middle operator of SincMiddle from the two host plans and the
// quadrature (z, w), in FP64 with the exact windows.  False (and nothing
// built) where it does not pay or does not fit: more than kMidMaxNodes
// quadrature nodes (host time grows with their number), a band wider than
// kMidMaxBand labels, or a workgroup window longer than kMidMaxSpan labels.
constexpr int64_t kMidMaxNodes = (int64_t)1 << 16;
constexpr int kMidMaxBand = 256;
constexpr int kMidMaxSpan = 4096;

// The quadrature rules of recent plans (the Gauss-Legendre rule costs
// O(n_quad^2) on the host), least recently used out.
static void quadrature_rule(sinc_quad quad, int64_t n, std::vector<double> &z, std::vector<double> &w)
{
    struct Rule {
        int quad;
        int64_t n;
        std::vector<double> z, w;
    };
    constexpr size_t kRules = 8;
    static std::mutex mu;
    static std::list<Rule> *cache = new std::list<Rule>();   // leaked: outlives static destructors
    {
        std::lock_guard<std::mutex> g(mu);
        for (auto it = cache->begin(); it != cache->end(); ++it)
            if (it->quad == (int)quad && it->n == n) {
                cache->splice(cache->begin(), *cache, it);
                z = it->z;
                w = it->w;
                return;
            }
    }
    if (quad == SINC_QUAD_GAUSS_LEGENDRE) gauss_legendre_rule(n, z, w);
    else clenshaw_curtis_rule(n, z, w);
    if (n > ((int64_t)1 << 16)) return;   // kept: rules of up to 2^16 nodes (1 MB)
    std::lock_guard<std::mutex> g(mu);
    cache->push_front(Rule{(int)quad, n, z, w});
    if (cache->size() > kRules) cache->pop_back();
}

// Device layout of the middle operator (after the weights and the
// intermediate): K, lo, base, span, out, each 256-byte aligned.
struct SincMidLayout {
    size_t K, lo, base, span, out, bytes;
};
static SincMidLayout sinc_middle_layout(const SincHostPlan &S)
{
    auto a256 = [](size_t x) { return (x + 255) / 256 * 256; };
    const SincMiddle &M = S.mid;
    const size_t csz = (S.prec == NNFFT_FP32_COMP) ? 8 : 16;
    SincMidLayout L;
    L.K = 0;
    L.lo = a256(M.K.size() * sizeof(double));
    L.base = L.lo + a256(M.lo.size() * sizeof(int32_t));
    L.span = L.base + a256(M.base.size() * sizeof(int32_t));
    L.out = L.span + a256(M.span.size() * sizeof(int32_t));
    L.bytes = L.out + a256(M.lo.size() * csz);
    return L;
}
static size_t sinc_middle_bytes(const SincHostPlan &S) { return sinc_middle_layout(S).bytes; }

static bool build_sinc_middle(SincHostPlan &S, const std::vector<double> &z)
{
    const nnfft_info_t &A = S.h1.info, &B = S.h2.info;
    const int64_t nn = (int64_t)z.size();
    if (nn > kMidMaxNodes || nn < 1) return false;
    const Window w_ip = make_window(A.window, A.m2, A.beta2);   // first plan: interpolation
    const Window w_c1 = make_window(A.window, A.m1, A.beta1);   // first plan: 1/phi_hat_1
    const Window w_sp = make_window(B.window, B.m1, B.beta1);   // second plan: spreading
    const Window w_d2 = make_window(B.window, B.m2, B.beta2);   // second plan: 1/phi_hat_2
    const int64_t G1 = B.G1, S_lab = S.h1.fd.S;
    const int ma = A.m2, mb = B.m1;
    // nodes: interpolation cell cu and spreading cell ct of each quadrature node
    std::vector<double> u(nn), t(nn);
    std::vector<int64_t> cu(nn), ct(nn);
    std::vector<int64_t> lo(G1, INT64_MAX), hi(G1, INT64_MIN);
    for (int64_t j = 0; j < nn; ++j) {
        const double x = 0.5 * z[j], v = -0.5 * z[j];
        u[j] = (double)A.N2 * (double)A.N_star * x / (double)A.N1;
        t[j] = (double)B.N1 * ((double)B.N * v / (double)B.N_star);
        cu[j] = (int64_t)std::floor(u[j]);
        ct[j] = (int64_t)std::floor(t[j]);
        if (cu[j] - ma + 1 < -S_lab || cu[j] + ma > S_lab) return false;
        for (int q = 0; q < 2 * mb; ++q) {
            const int64_t row = ct[j] - mb + 1 + q + G1 / 2;
            if (row < 0 || row >= G1) return false;
            lo[row] = std::min(lo[row], cu[j] - ma + 1);
            hi[row] = std::max(hi[row], cu[j] + ma);
        }
    }
    int64_t Wb = 1;
    for (int64_t r = 0; r < G1; ++r)
        if (hi[r] >= lo[r]) Wb = std::max(Wb, hi[r] - lo[r] + 1);
    if (Wb > kMidMaxBand) return false;
    // workgroup windows; rows without entries read the start of theirs
    const int64_t nwg = (G1 + kSincMidRows - 1) / kSincMidRows;
    SincMiddle &Mi = S.mid;
    Mi.base.assign(nwg, 0);
    Mi.span.assign(nwg, 0);
    Mi.lo.assign(G1, 0);
    int64_t span_max = 1;
    for (int64_t g = 0; g < nwg; ++g) {
        const int64_t r0 = g * kSincMidRows, r1 = std::min(G1, r0 + kSincMidRows);
        int64_t b0 = INT64_MAX;
        for (int64_t r = r0; r < r1; ++r)
            if (hi[r] >= lo[r]) b0 = std::min(b0, lo[r]);
        if (b0 == INT64_MAX) b0 = 0;
        int64_t end = b0 + 1;
        for (int64_t r = r0; r < r1; ++r) {
            const int64_t l0 = hi[r] >= lo[r] ? lo[r] : b0;
            Mi.lo[r] = (int32_t)l0;
            end = std::max(end, l0 + Wb);
        }
        Mi.base[g] = (int32_t)b0;
        Mi.span[g] = (int32_t)(end - b0);
        span_max = std::max(span_max, end - b0);
    }
    if (span_max > kMidMaxSpan) return false;
    // the band: sum over the nodes of spreading tap x weight / phi_hat_1 x
    // interpolation tap, then the deconvolution of each row
    std::vector<double> Kr((size_t)(G1 * Wb), 0.0);
    std::vector<double> tap_ip(2 * ma), tap_sp(2 * mb);
    for (int64_t j = 0; j < nn; ++j) {
        const double x = 0.5 * z[j];
        const double phi1 = (double)A.m1 / (double)A.N1 *
                            window_hat(w_c1, (double)A.m1 * (double)A.N_star * x / (double)A.N1);
        const double a = S.w[j] / phi1;
        for (int r = 0; r < 2 * ma; ++r)
            tap_ip[r] = window_value(w_ip, (u[j] - (double)(cu[j] - ma + 1 + r)) / ma);
        for (int q = 0; q < 2 * mb; ++q)
            tap_sp[q] = window_value(w_sp, ((double)(ct[j] - mb + 1 + q) - t[j]) / mb);
        for (int q = 0; q < 2 * mb; ++q) {
            const int64_t row = ct[j] - mb + 1 + q + G1 / 2;
            double *k = Kr.data() + row * Wb + (cu[j] - ma + 1 - Mi.lo[row]);
            const double aq = a * tap_sp[q];
            for (int r = 0; r < 2 * ma; ++r) k[r] += aq * tap_ip[r];
        }
    }
    Mi.K.assign((size_t)(G1 * Wb), 0.0);
    for (int64_t r = 0; r < G1; ++r) {
        const double l = (double)(r - G1 / 2);
        const double phi2 = (double)B.m2 / (double)B.N2 * window_hat(w_d2, (double)B.m2 * l / (double)B.N2);
        const double d = 1.0 / ((double)B.N1 * (double)B.N2 * phi2);
        for (int64_t b = 0; b < Wb; ++b) Mi.K[(size_t)(b * G1 + r)] = d * Kr[(size_t)(r * Wb + b)];
    }
    Mi.Wb = (int32_t)Wb;
    Mi.span_max = (int32_t)span_max;
    Mi.S = (int32_t)S_lab;
    return true;
}

nnfft_status sinc_host(SincHostPlan &S, int64_t N, int64_t L1, int64_t L2, sinc_quad quad, int64_t n_quad,
                       double sigma1, double sigma2, int m1, int m2, nnfft_precision prec,
                       const std::vector<double> &a, const std::vector<double> &b, bool middle)
{
    if (n_quad < 1 || n_quad > ((int64_t)1 << 24)) return fail(NNFFT_ERR_ARG, "n_quad out of range");
    if (quad != SINC_QUAD_GAUSS_LEGENDRE && quad != SINC_QUAD_CLENSHAW_CURTIS)
        return fail(NNFFT_ERR_ARG, "unknown quadrature rule");
    std::vector<double> z;
    quadrature_rule(quad, n_quad, z, S.w);
    const int64_t nn = (int64_t)z.size();
    std::vector<double> xs(nn), vs(nn);
    for (int64_t j = 0; j < nn; ++j) {
        xs[j] = 0.5 * z[j];    // step 1: spatial nodes z_j / 2
        vs[j] = -0.5 * z[j];   // step 3: frequencies -z_j / 2
    }
    // equispaced special cases (Sec. 6, after Algorithm 6.1): a_k = k / L1,
    // k in I_{L1} (and N <= L1), makes step 1 an NFFT with L1 frequencies at
    // the nodes N z_j / (2 L1); b_l = l / N, l in I_N, makes step 3 an adjoint
    // NFFT with N frequencies at the nodes z_j / 2.  Both use sigma1, m1.
    auto equispaced = [](const std::vector<double> &t, int64_t L) {
        if (L < 2 || (L % 2) || (int64_t)t.size() != L) return false;
        for (int64_t k = 0; k < L; ++k)
            if (t[k] != (double)(k - L / 2) / (double)L) return false;
        return true;
    };
    S.step1_nfft = equispaced(a, L1) && N <= L1;
    S.step3_nfft = L2 == N && equispaced(b, L2);
    nnfft_status st;
    if (S.step1_nfft) {
        std::vector<double> xn(nn);
        for (int64_t j = 0; j < nn; ++j) xn[j] = (double)N * z[j] / (2.0 * (double)L1);
        st = nfft_plan_host(S.h1, L1, nn, sigma1, m1, prec, xn);
    } else {
        st = plan_host(S.h1, N, L1, nn, sigma1, sigma2, m1, m2, prec, a, xs);
    }
    if (st == NNFFT_OK)
        st = S.step3_nfft ? nfft_plan_host(S.h2, N, nn, sigma1, m1, prec, xs)
                          : plan_host(S.h2, N, nn, L2, sigma1, sigma2, m1, m2, prec, vs, b);
    if (st != NNFFT_OK) return st;
    S.n_nodes = nn;
    S.L1 = L1;
    S.L2 = L2;
    S.prec = prec;
    const size_t csz = (prec == NNFFT_FP32_COMP) ? 8 : 16;
    S.wg_bytes = ((size_t)nn * sizeof(double) + 255) / 256 * 256 + (size_t)nn * csz;
    S.mid_ok = middle && !S.step1_nfft && !S.step3_nfft && build_sinc_middle(S, z);
    if (S.mid_ok) S.wg_bytes = (S.wg_bytes + 255) / 256 * 256 + sinc_middle_bytes(S);
    S.total_bytes = S.h1.total_bytes + S.h2.total_bytes + S.wg_bytes;
    return NNFFT_OK;
}

nnfft_status sinc_create(const SincHostPlan &S, const DevMem &mem, hipStream_t s, sinc_plan_t *out)
{
    *out = nullptr;
    sinc_plan_s *sp = new (std::nothrow) sinc_plan_s();
    if (!sp) return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    sp->mem = mem;
    sp->n_nodes = S.n_nodes;
    sp->L1 = S.L1;
    sp->L2 = S.L2;
    sp->prec = S.prec;
    sp->step1_nfft = S.step1_nfft;
    sp->step3_nfft = S.step3_nfft;
    nnfft_status st = plan_create(S.h1, mem, s, &sp->p1);
    if (st == NNFFT_OK) st = plan_create(S.h2, mem, s, &sp->p2);
    if (st != NNFFT_OK) {
        delete sp;
        return st;
    }
    sp->wg_base = mem.alloc(mem.ctx, S.wg_bytes);
    if (!sp->wg_base) {
        delete sp;
        return fail(NNFFT_ERR_NOMEM, "device memory for the quadrature weights is not available");
    }
    sp->w = static_cast<double *>(sp->wg_base);
    sp->g = static_cast<char *>(sp->wg_base) + ((size_t)S.n_nodes * sizeof(double) + 255) / 256 * 256;
    hipError_t e = hipMemcpyAsync(sp->w, S.w.data(), (size_t)S.n_nodes * sizeof(double), hipMemcpyHostToDevice, s);
    if (S.mid_ok) {
        const size_t csz = (S.prec == NNFFT_FP32_COMP) ? 8 : 16;
        const size_t off = ((size_t)S.n_nodes * sizeof(double) + 255) / 256 * 256 + (size_t)S.n_nodes * csz;
        char *mb = static_cast<char *>(sp->wg_base) + (off + 255) / 256 * 256;
        const SincMidLayout L = sinc_middle_layout(S);
        const SincMiddle &M = S.mid;
        SincMidArgs &A = sp->mid;
        A.h = sp->p1->desc.ip;
        A.K = reinterpret_cast<const double *>(mb + L.K);
        A.lo = reinterpret_cast<const int32_t *>(mb + L.lo);
        A.base = reinterpret_cast<const int32_t *>(mb + L.base);
        A.span = reinterpret_cast<const int32_t *>(mb + L.span);
        A.out = mb + L.out;
        A.G1 = (int32_t)M.lo.size();
        A.Wb = M.Wb;
        A.S = M.S;
        A.span_max = M.span_max;
        A.nwg = (int32_t)M.base.size();
        auto put = [&](size_t at, const void *src, size_t n) {
            if (e == hipSuccess && n > 0) e = hipMemcpyAsync(mb + at, src, n, hipMemcpyHostToDevice, s);
        };
        put(L.K, M.K.data(), M.K.size() * sizeof(double));
        put(L.lo, M.lo.data(), M.lo.size() * sizeof(int32_t));
        put(L.base, M.base.data(), M.base.size() * sizeof(int32_t));
        put(L.span, M.span.data(), M.span.size() * sizeof(int32_t));
        sp->has_mid = sp->use_mid = true;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete sp;
        return fail(NNFFT_ERR_DEVICE, hipGetErrorString(e));
    }
    *out = sp;
    return NNFFT_OK;
}

}  // namespace nnfft

void nnfft_plan_s::drop_events()
{
    for (nnfft::KernelTimes &k : prof)
        for (int i = 0; i < nnfft::kMaxTimedKernels; ++i) {
            if (k.start[i]) (void)hipEventDestroy(k.start[i]);
            if (k.stop[i]) (void)hipEventDestroy(k.stop[i]);
        }
    prof.clear();
    prof_max = prof_used = 0;
}

nnfft_plan_s::~nnfft_plan_s()
{
    drop_events();
    if (base) mem.release(mem.ctx, base);
}

sinc_plan_s::~sinc_plan_s()
{
    if (p1) nnfft_destroy(p1);
    if (p2) nnfft_destroy(p2);
    if (wg_base) mem.release(mem.ctx, wg_base);
}

// ---------------------------------------------------------------------------
extern "C" {

const char *nnfft_last_error(void) { return g_last_error.c_str(); }

const char *nnfft_version(void) { return "nnfft-mi355x 0.2 (gfx950)"; }

nnfft_status nnfft_derive_params(int64_t N, double sigma1, double sigma2, int m1, int m2,
                                 nnfft_info_t *out)
{
    if (!out) return fail(NNFFT_ERR_ARG, "null output");
    const nnfft_status st = derive_params(N, sigma1, sigma2, m1, m2, out);
    if (st != NNFFT_OK) return fail(st, "invalid NNFFT parameters (N >= 1, m >= 2, sigma > 1, "
                                        "2 m1 < N1 and 2 m2 <= (1 - 1/sigma1) N2 are required)");
    return NNFFT_OK;
}

nnfft_status nnfft_plan(nnfft_plan_t *out, int64_t N, int64_t M1, int64_t M2, double sigma1,
                        double sigma2, int m1, int m2, nnfft_precision prec, const double *v,
                        const double *x, void *stream)
{
    return nnfft_plan_window(out, N, M1, M2, sigma1, sigma2, m1, m2, prec, NNFFT_WINDOW_SINH, v, x, stream);
}

nnfft_status nnfft_plan_window(nnfft_plan_t *out, int64_t N, int64_t M1, int64_t M2, double sigma1,
                               double sigma2, int m1, int m2, nnfft_precision prec, nnfft_window window,
                               const double *v, const double *x, void *stream)
{
    if (!out) return fail(NNFFT_ERR_ARG, "null plan pointer");
    *out = nullptr;
    if (M1 < 1 || M2 < 1 || M1 > ((int64_t)1 << 30) || M2 > ((int64_t)1 << 30))
        return fail(NNFFT_ERR_ARG, "node counts must be in [1, 2^30]");
    if (prec != NNFFT_FP64_PLAIN && prec != NNFFT_FP32_COMP) return fail(NNFFT_ERR_ARG, "unknown precision");
    if (!v || !x) return fail(NNFFT_ERR_ARG, "null node array");
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        bool host = false;
        {
            ScratchLease T;
            HostPlan H;
            DevRecords R;
            nnfft_status st = plan_device_nodes(H, R, *T, N, M1, M2, sigma1, sigma2, m1, m2, prec, window, v, x, s,
                                                &host);
            if (!host) return st == NNFFT_OK ? plan_create(H, hip_mem(), s, out, &R) : st;
        }
        // sort keys wider than 32 bits: the node layout is built on the host
        std::vector<double> hv, hx;
        nnfft_status st = copy_nodes(v, M1, hv, s);
        if (st != NNFFT_OK) return st;
        st = copy_nodes(x, M2, hx, s);
        if (st != NNFFT_OK) return st;
        HostPlan H;
        st = plan_host(H, N, M1, M2, sigma1, sigma2, m1, m2, prec, hv, hx, nullptr, nullptr, window);
        if (st != NNFFT_OK) return st;
        return plan_create(H, hip_mem(), s, out);
    } catch (const HipError &e) {
        return fail(NNFFT_ERR_DEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status nnfft_plan_dry_run(int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2, int m1, int m2,
                                nnfft_precision prec, const double *v, const double *x, nnfft_info_t *out)
{
    return nnfft_plan_window_dry_run(N, M1, M2, sigma1, sigma2, m1, m2, prec, NNFFT_WINDOW_SINH, v, x, out);
}

nnfft_status nnfft_plan_window_dry_run(int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2, int m1,
                                       int m2, nnfft_precision prec, nnfft_window window, const double *v,
                                       const double *x, nnfft_info_t *out)
{
    if (!v || !x || !out) return fail(NNFFT_ERR_ARG, "null argument");
    if (M1 < 1 || M2 < 1 || M1 > ((int64_t)1 << 30) || M2 > ((int64_t)1 << 30))
        return fail(NNFFT_ERR_ARG, "node counts must be in [1, 2^30]");
    try {
        std::vector<double> hv(v, v + M1), hx(x, x + M2);
        HostPlan H;
        nnfft_status st = plan_host(H, N, M1, M2, sigma1, sigma2, m1, m2, prec, hv, hx, nullptr, nullptr, window);
        if (st != NNFFT_OK) return st;
        st = check_plan(H, hv, hx);
        if (st != NNFFT_OK) return st;
        *out = H.info;
        return NNFFT_OK;
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status nnfft_plan_window_dry_run_digest(int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2,
                                              int m1, int m2, nnfft_precision prec, nnfft_window window,
                                              const double *v, const double *x, uint64_t *digest)
{
    if (!v || !x || !digest) return fail(NNFFT_ERR_ARG, "null argument");
    if (M1 < 1 || M2 < 1 || M1 > ((int64_t)1 << 30) || M2 > ((int64_t)1 << 30))
        return fail(NNFFT_ERR_ARG, "node counts must be in [1, 2^30]");
    try {
        std::vector<double> hv(v, v + M1), hx(x, x + M2);
        HostPlan H;
        nnfft_status st = plan_host(H, N, M1, M2, sigma1, sigma2, m1, m2, prec, hv, hx, nullptr, nullptr, window);
        if (st != NNFFT_OK) return st;
        std::vector<char> stage;
        Carver C(0, &stage);
        PlanDev D;
        PlanDev *dd = nullptr;
        size_t upload_end = 0;
        layout_plan(H, C, D, &upload_end, &dd);
        stage.resize(upload_end);
        *digest = fnv1a64(stage.data(), stage.size());
        return NNFFT_OK;
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status nnfft_plan_digest(nnfft_plan_t p, uint64_t *digest)
{
    if (!p || !digest) return fail(NNFFT_ERR_ARG, "null argument");
    try {
        std::vector<char> img(p->upload_bytes);
        const hipError_t e = hipMemcpy(img.data(), p->base, img.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("copying the plan: ") + hipGetErrorString(e));
        *digest = fnv1a64(img.data(), img.size());
        return NNFFT_OK;
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status nfft_plan_dry_run(int64_t N, int64_t M, double sigma, int m, nnfft_precision prec, const double *x,
                               nnfft_info_t *out)
{
    if (!x || !out) return fail(NNFFT_ERR_ARG, "null argument");
    if (M < 1 || M > ((int64_t)1 << 30)) return fail(NNFFT_ERR_ARG, "node count must be in [1, 2^30]");
    try {
        std::vector<double> hx(x, x + M);
        HostPlan H;
        nnfft_status st = nfft_plan_host(H, N, M, sigma, m, prec, hx);
        if (st != NNFFT_OK) return st;
        st = check_plan(H, hx, hx);
        if (st != NNFFT_OK) return st;
        *out = H.info;
        return NNFFT_OK;
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status nnfft_exec(nnfft_plan_t p, const void *f, void *y, void *stream)
{
    if (!p || !f || !y) return fail(NNFFT_ERR_ARG, "null argument");
    if (p->kind != 0) return fail(NNFFT_ERR_ARG, "an NFFT plan: use nfft_exec or nfft_adjoint");
    KernelTimes *kt = nullptr;
    if (p->prof_used < p->prof_max) kt = &p->prof[(size_t)p->prof_used++];
    const hipError_t e = launch_exec(p->desc, f, y, static_cast<hipStream_t>(stream), kt);
    if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return NNFFT_OK;
}

nnfft_status nnfft_exec_noalloc(nnfft_plan_t p, const void *f, void *y, void *stream)
{
    if (!p || !f || !y) return fail(NNFFT_ERR_ARG, "null argument");
    if (p->kind != 0) return fail(NNFFT_ERR_ARG, "an NFFT plan: use nfft_exec or nfft_adjoint");
    const size_t need = static_scratch_need(p->scratch);
    if (need > kStaticScratchBytes)
        return fail(NNFFT_ERR_ARG, "nnfft_exec_noalloc: the plan needs " + std::to_string(need) +
                                       " bytes of working memory; the static scratch holds " +
                                       std::to_string(kStaticScratchBytes));
    const hipError_t e = launch_exec_static(p->desc, p->scratch, f, y, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return NNFFT_OK;
}

nnfft_status nnfft_exec_batch(int n, const nnfft_plan_t *plans, const void *const *f, void *const *y,
                              void *stream)
{
    if (n < 0 || (n > 0 && (!plans || !f || !y))) return fail(NNFFT_ERR_ARG, "null argument");
    try {
        std::vector<nnfft_plan_t> seen;
        seen.reserve(n);
        for (int i = 0; i < n; ++i) {
            if (!plans[i] || !f[i] || !y[i]) return fail(NNFFT_ERR_ARG, "null plan or array in the batch");
            if (plans[i]->kind != 0) return fail(NNFFT_ERR_ARG, "NFFT plans cannot be batched");
            seen.push_back(plans[i]);
        }
        std::sort(seen.begin(), seen.end());
        if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
            return fail(NNFFT_ERR_ARG, "a plan appears twice in the batch");
        // one group per precision, each in the callers' order
        for (int prec : {(int)NNFFT_FP32_COMP, (int)NNFFT_FP64_PLAIN}) {
            std::vector<const PlanDev *> host, dev;
            std::vector<const void *> fi;
            std::vector<void *> yi;
            for (int i = 0; i < n; ++i) {
                if (plans[i]->desc.prec != prec) continue;
                host.push_back(&plans[i]->desc);
                dev.push_back(plans[i]->ddesc);
                fi.push_back(f[i]);
                yi.push_back(y[i]);
            }
            if (host.empty()) continue;
            const hipError_t e = launch_exec_batch((int)host.size(), host.data(), dev.data(), fi.data(),
                                                   yi.data(), static_cast<hipStream_t>(stream));
            if (e != hipSuccess)
                return fail(NNFFT_ERR_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
        }
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
    return NNFFT_OK;
}

nnfft_status nnfft_info(nnfft_plan_t p, nnfft_info_t *out)
{
    if (!p || !out) return fail(NNFFT_ERR_ARG, "null argument");
    *out = p->info;
    return NNFFT_OK;
}

nnfft_status nnfft_profile_start(nnfft_plan_t p, int max_execs)
{
    if (!p || max_execs < 1) return fail(NNFFT_ERR_ARG, "bad argument");
    p->drop_events();
    try {
        p->prof.assign((size_t)max_execs, KernelTimes{});
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
    for (KernelTimes &k : p->prof)
        for (int i = 0; i < kMaxTimedKernels; ++i)
            if (hipEventCreate(&k.start[i]) != hipSuccess || hipEventCreate(&k.stop[i]) != hipSuccess) {
                p->drop_events();
                return fail(NNFFT_ERR_DEVICE, "hipEventCreate failed");
            }
    p->prof_max = max_execs;
    p->prof_used = 0;
    return NNFFT_OK;
}

// Reads the kernel times of the profiled execs (waits for the last one) and
// releases the events.  Every exec of a plan launches the same kernels.
static nnfft_status read_profile(nnfft_plan_t p, nnfft_kernel_time_t *kern, int kcap, int *nk, double *exec_ms,
                                 int ecap, int *nexecs)
{
    const int n = p->prof_used;
    const int nkern = n > 0 ? p->prof[0].n : 0;
    if (n > 0 && nkern > 0 && hipEventSynchronize(p->prof[(size_t)n - 1].stop[nkern - 1]) != hipSuccess) {
        p->drop_events();
        return fail(NNFFT_ERR_DEVICE, "hipEventSynchronize failed");
    }
    auto elapsed = [](hipEvent_t a, hipEvent_t b, double *ms) {
        float f = 0.f;
        if (hipEventElapsedTime(&f, a, b) != hipSuccess) return false;
        *ms = f;
        return true;
    };
    for (int k = 0; k < std::min(kcap, nkern); ++k) {
        nnfft_kernel_time_t &o = kern[k];
        o = nnfft_kernel_time_t{};
        std::snprintf(o.name, sizeof o.name, "%s", kernel_name(p->prof[0].kid[k]));
        o.stage = kernel_stage(p->prof[0].kid[k]);
        o.min_ms = 1e300;
        for (int i = 0; i < n; ++i) {
            double ms = 0.0;
            if (!elapsed(p->prof[(size_t)i].start[k], p->prof[(size_t)i].stop[k], &ms)) {
                p->drop_events();
                return fail(NNFFT_ERR_DEVICE, "hipEventElapsedTime failed");
            }
            o.avg_ms += ms / n;
            o.min_ms = std::min(o.min_ms, ms);
            o.max_ms = std::max(o.max_ms, ms);
        }
    }
    for (int i = 0; i < std::min(ecap, n); ++i)
        if (nkern == 0 || !elapsed(p->prof[(size_t)i].start[0], p->prof[(size_t)i].stop[nkern - 1], &exec_ms[i])) {
            p->drop_events();
            return fail(NNFFT_ERR_DEVICE, "hipEventElapsedTime failed");
        }
    if (nk) *nk = nkern;
    if (nexecs) *nexecs = n;
    p->drop_events();
    return NNFFT_OK;
}

nnfft_status nnfft_profile_stop(nnfft_plan_t p, double *stage_ms, int *nexecs)
{
    if (!p || !stage_ms) return fail(NNFFT_ERR_ARG, "bad argument");
    nnfft_kernel_time_t k[kMaxTimedKernels];
    int nk = 0;
    const nnfft_status st = read_profile(p, k, kMaxTimedKernels, &nk, nullptr, 0, nexecs);
    if (st != NNFFT_OK) return st;
    for (int s = 0; s < 3; ++s) stage_ms[s] = 0.0;
    for (int i = 0; i < nk; ++i) stage_ms[k[i].stage] += k[i].avg_ms;
    return NNFFT_OK;
}

nnfft_status nnfft_profile_kernels(nnfft_plan_t p, nnfft_kernel_time_t *kernels, int kcap, int *nkernels,
                                   double *exec_ms, int ecap, int *nexecs)
{
    if (!p || kcap < 0 || ecap < 0 || (kcap > 0 && !kernels) || (ecap > 0 && !exec_ms))
        return fail(NNFFT_ERR_ARG, "bad argument");
    return read_profile(p, kernels, kcap, nkernels, exec_ms, ecap, nexecs);
}

nnfft_status nnfft_destroy(nnfft_plan_t p)
{
    if (!p) return fail(NNFFT_ERR_ARG, "null plan");
    delete p;
    return NNFFT_OK;
}

// ---------------------------------------------------------------------------
// NFFT with equispaced frequencies
// ---------------------------------------------------------------------------
nnfft_status nfft_plan(nfft_plan_t *out, int64_t N, int64_t M, double sigma, int m, nnfft_precision prec,
                       const double *x, void *stream)
{
    if (!out) return fail(NNFFT_ERR_ARG, "null plan pointer");
    *out = nullptr;
    if (!x) return fail(NNFFT_ERR_ARG, "null node array");
    if (M < 1 || M > ((int64_t)1 << 30)) return fail(NNFFT_ERR_ARG, "node count must be in [1, 2^30]");
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<double> hx;
        nnfft_status st = copy_nodes(x, M, hx, s);
        if (st != NNFFT_OK) return st;
        HostPlan H;
        st = nfft_plan_host(H, N, M, sigma, m, prec, hx);
        if (st != NNFFT_OK) return st;
        return plan_create(H, hip_mem(), s, out);
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

static nnfft_status nfft_run(nfft_plan_t p, bool adjoint, const void *in, void *out, void *stream)
{
    if (!p || !in || !out) return fail(NNFFT_ERR_ARG, "null argument");
    if (p->kind != 1) return fail(NNFFT_ERR_ARG, "not an NFFT plan");
    const hipError_t e = launch_nfft(p->desc, adjoint, in, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return NNFFT_OK;
}

nnfft_status nfft_exec(nfft_plan_t p, const void *f, void *y, void *stream)
{
    return nfft_run(p, false, f, y, stream);
}

nnfft_status nfft_adjoint(nfft_plan_t p, const void *y, void *h, void *stream)
{
    return nfft_run(p, true, y, h, stream);
}

nnfft_status nfft_destroy(nfft_plan_t p)
{
    if (!p) return fail(NNFFT_ERR_ARG, "null plan");
    if (p->kind != 1) return fail(NNFFT_ERR_ARG, "not an NFFT plan");
    delete p;
    return NNFFT_OK;
}

// ---------------------------------------------------------------------------
// Tuning table
// ---------------------------------------------------------------------------
nnfft_status nnfft_set_tuning(nnfft_precision prec, int64_t M, const nnfft_tuning_t *t)
{
    if (!t || M < 1 || (prec != NNFFT_FP64_PLAIN && prec != NNFFT_FP32_COMP) || t->items_points < 1 ||
        t->block_points < 1)
        return fail(NNFFT_ERR_ARG, "bad tuning");
    Layout L;
    L.Q = t->items_points;
    L.block = t->block_points;
    set_tuned_layout(prec == NNFFT_FP32_COMP, M, L);
    return NNFFT_OK;
}

nnfft_status nnfft_get_tuning(nnfft_precision prec, int64_t M, nnfft_tuning_t *out)
{
    if (!out || M < 1 || (prec != NNFFT_FP64_PLAIN && prec != NNFFT_FP32_COMP))
        return fail(NNFFT_ERR_ARG, "bad argument");
    Layout L;
    const bool fp32 = prec == NNFFT_FP32_COMP;
    const bool tuned = get_tuned_layout(fp32, M, L);
    L = choose_layout(M, fp32);
    *out = nnfft_tuning_t{};
    out->items_points = L.Q;
    out->block_points = L.block;
    out->tuned = tuned ? 1 : 0;
    return NNFFT_OK;
}

nnfft_status nnfft_clear_tuning(void)
{
    clear_tuned_layouts();
    return NNFFT_OK;
}

// ---------------------------------------------------------------------------
// Fast sinc transform (Algorithm 6.1)
// ---------------------------------------------------------------------------
nnfft_status sinc_plan(sinc_plan_t *out, int64_t N, int64_t L1, int64_t L2, sinc_quad quad,
                       int64_t n_quad, double sigma1, double sigma2, int m1, int m2,
                       nnfft_precision prec, const double *a, const double *b, void *stream)
{
    if (!out) return fail(NNFFT_ERR_ARG, "null plan pointer");
    *out = nullptr;
    if (n_quad < 1 || n_quad > ((int64_t)1 << 24)) return fail(NNFFT_ERR_ARG, "n_quad out of range");
    if (quad != SINC_QUAD_GAUSS_LEGENDRE && quad != SINC_QUAD_CLENSHAW_CURTIS)
        return fail(NNFFT_ERR_ARG, "unknown quadrature rule");
    if (L1 < 1 || L2 < 1 || L1 > ((int64_t)1 << 30) || L2 > ((int64_t)1 << 30))
        return fail(NNFFT_ERR_ARG, "node counts must be in [1, 2^30]");
    if (!a || !b) return fail(NNFFT_ERR_ARG, "null node array");
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<double> ha, hb;
        nnfft_status st = copy_nodes(a, L1, ha, s);
        if (st != NNFFT_OK) return st;
        st = copy_nodes(b, L2, hb, s);
        if (st != NNFFT_OK) return st;
        SincHostPlan S;
        st = sinc_host(S, N, L1, L2, quad, n_quad, sigma1, sigma2, m1, m2, prec, ha, hb, true);
        if (st != NNFFT_OK) return st;
        return sinc_create(S, hip_mem(), s, out);
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status sinc_exec(sinc_plan_t p, const void *c, void *h, void *stream)
{
    if (!p || !c || !h) return fail(NNFFT_ERR_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->use_mid) {
        const hipError_t e = launch_sinc_middle(p->p1->desc, p->mid, p->p2->desc, c, h, s);
        if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
        return NNFFT_OK;
    }
    nnfft_status st = p->step1_nfft ? nfft_exec(p->p1, c, p->g, stream)        // step 1
                                    : nnfft_exec(p->p1, c, p->g, stream);
    if (st != NNFFT_OK) return st;
    // step 2 (alpha_j = w_j g_j) is folded into the coefficient loads of
    // step 3's spreading
    PlanDev D = p->p2->desc;
    D.sp.wts = p->w;
    const hipError_t e = p->step3_nfft ? launch_nfft(D, true, p->g, h, s)       // step 3
                                       : launch_exec(D, p->g, h, s, nullptr);
    if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(e));
    return NNFFT_OK;
}

nnfft_status nnfft_quadrature(sinc_quad quad, int64_t n_quad, double *z, double *w)
{
    if (n_quad < 1 || n_quad > ((int64_t)1 << 24) || !z || !w) return fail(NNFFT_ERR_ARG, "bad argument");
    if (quad != SINC_QUAD_GAUSS_LEGENDRE && quad != SINC_QUAD_CLENSHAW_CURTIS)
        return fail(NNFFT_ERR_ARG, "unknown quadrature rule");
    try {
        std::vector<double> zz, ww;
        quadrature_rule(quad, n_quad, zz, ww);
        std::copy(zz.begin(), zz.end(), z);
        std::copy(ww.begin(), ww.end(), w);
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
    return NNFFT_OK;
}

nnfft_status sinc_info(sinc_plan_t p, int which, nnfft_info_t *out)
{
    if (!p || !out || (which != 0 && which != 1)) return fail(NNFFT_ERR_ARG, "bad argument");
    *out = (which == 0 ? p->p1 : p->p2)->info;
    return NNFFT_OK;
}

nnfft_status sinc_sizes(sinc_plan_t p, int64_t *L1, int64_t *L2, int64_t *n_nodes, int32_t *nfft_steps)
{
    if (!p || !L1 || !L2 || !n_nodes || !nfft_steps) return fail(NNFFT_ERR_ARG, "bad argument");
    *L1 = p->L1;
    *L2 = p->L2;
    *n_nodes = p->n_nodes;
    *nfft_steps = (p->step1_nfft ? 1 : 0) | (p->step3_nfft ? 2 : 0);
    return NNFFT_OK;
}

nnfft_status sinc_middle(sinc_plan_t p, int on, int32_t *built, int32_t *active)
{
    if (!p) return fail(NNFFT_ERR_ARG, "null plan");
    if (on == 1 && !p->has_mid) return fail(NNFFT_ERR_UNSUPPORTED, "the plan has no middle operator");
    if (on == 0 || on == 1) p->use_mid = (on == 1);
    if (built) *built = p->has_mid ? 1 : 0;
    if (active) *active = p->use_mid ? 1 : 0;
    return NNFFT_OK;
}

nnfft_status sinc_middle_dry_run(int64_t N, sinc_quad quad, int64_t n_quad, double sigma1, double sigma2, int m1,
                                 int m2, nnfft_precision prec, double *K, int32_t *lo, int64_t cap, int64_t *G1,
                                 int32_t *Wb)
{
    if (!G1 || !Wb) return fail(NNFFT_ERR_ARG, "null argument");
    if (n_quad + (quad == SINC_QUAD_CLENSHAW_CURTIS ? 1 : 0) > kMidMaxNodes && n_quad <= ((int64_t)1 << 24) &&
        (quad == SINC_QUAD_GAUSS_LEGENDRE || quad == SINC_QUAD_CLENSHAW_CURTIS))
        return fail(NNFFT_ERR_UNSUPPORTED, "no middle operator for more than 2^16 quadrature nodes");
    try {
        // the operator does not depend on the nodes: one node on each side
        const std::vector<double> a(1, 0.0), b(1, 0.0);
        SincHostPlan S;
        nnfft_status st = sinc_host(S, N, 1, 1, quad, n_quad, sigma1, sigma2, m1, m2, prec, a, b, true);
        if (st != NNFFT_OK) return st;
        if (!S.mid_ok) return fail(NNFFT_ERR_UNSUPPORTED, "no middle operator for these parameters");
        const int64_t rows = (int64_t)S.mid.lo.size();
        *G1 = rows;
        *Wb = S.mid.Wb;
        if (K || lo) {
            if (!K || !lo || cap < rows * S.mid.Wb) return fail(NNFFT_ERR_ARG, "K / lo missing or too small");
            std::copy(S.mid.K.begin(), S.mid.K.end(), K);
            std::copy(S.mid.lo.begin(), S.mid.lo.end(), lo);
        }
        return NNFFT_OK;
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status sinc_destroy(sinc_plan_t p)
{
    if (!p) return fail(NNFFT_ERR_ARG, "null plan");
    delete p;
    return NNFFT_OK;
}

}  // extern "C"
