// NNFFT plans (Algorithm 2.2 step 0) and the C ABI of include/nnfft.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/nnfft.h"
#include "host_math.h"
#include "internal.h"

using namespace nnfft;

namespace {

thread_local std::string g_last_error;

nnfft_status fail(nnfft_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

struct HipError {
    hipError_t err;
    const char *what;
};

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) throw HipError{e, what};
}

// Node layout of one side, built on the host.
struct SideHost {
    std::vector<int32_t> perm;
    std::vector<PtRec> rec32;
    std::vector<double> frac64;
    std::vector<Item> items;
    std::vector<Chunk> chunks;
    std::vector<int32_t> chunk_block;
    std::vector<int32_t> chunk_item0;   // first item of each chunk
    std::vector<Chunk> launch;          // chunks in launch order, empty ones pad
    std::vector<Item> launch_items;     // 64 items per launch slot, n = 0 pads
    std::vector<PtRec> trec32;          // FP32: records in per-chunk transposed blocks
    int64_t part_cells = 0;
    int64_t nblocks = 0;
};

// Tunables chosen per plan (the "autotuner" table; see choose_layout).
struct Layout {
    int64_t block;      // points per node block
    int Q;              // max points per work item
    int IW;             // items per workgroup (= threads)
};

// Rule table measured on MI355X: one-wavefront workgroups of 64 items; items
// of up to Q points with Q growing with the node count (16 at 2^20 nodes,
// 32 at most on the FP32 path, 8 on the FP64 path) so that a launch keeps a
// few workgroups per CU;
// blocks of 2^17 nodes (1 MB of c64 coefficients, well inside one XCD's L2),
// split into 8 when that keeps them >= 2^14 nodes so every XCD has a block.
Layout choose_layout(int64_t M, bool fp32)
{
    Layout L;
    L.IW = kItemsPerWg;
    const int64_t cus = 256;
    const int64_t target_wg = 4 * cus;
    int64_t q = M / (L.IW * target_wg);
    int Q = 2;
    while (Q < q && Q < (fp32 ? 32 : 8)) Q *= 2;
    L.Q = Q;
    const int64_t bmax = fp32 ? (int64_t)1 << 17 : (int64_t)1 << 16;
    const int64_t bmin = (int64_t)1 << 14;
    int64_t nblk = (M + bmax - 1) / bmax;
    if (nblk < 8 && M >= 8 * bmin) nblk = 8;
    if (nblk < 1) nblk = 1;
    L.block = (M + nblk - 1) / nblk;
    // overrides for tuning sweeps
    if (const char *e = std::getenv("NNFFT_ITEM_POINTS")) L.Q = std::max(1, std::min(fp32 ? 64 : 8, atoi(e)));
    if (const char *e = std::getenv("NNFFT_BLOCK_POINTS")) L.block = std::max<int64_t>(1, atoll(e));
    return L;
}

// Builds the sorted records, items, chunks and schedule of one side.
// t_k = scale * node_k (grid units); bin = floor(t_k) + off in [0, nbins).
// Spreading side: `m` > 0 gives the chunk windows of 2m - 1 + nbin cells.
bool build_side(const std::vector<double> &nodes, double scale, int64_t off, int64_t nbins,
                const Layout &L, bool fp32, int m, SideHost &S, std::string &err)
{
    const int64_t M = (int64_t)nodes.size();
    std::vector<int32_t> bin(M);
    std::vector<double> fr(M);
    for (int64_t k = 0; k < M; ++k) {
        const double t = scale * nodes[k];
        const double c = std::floor(t);
        const int64_t b = (int64_t)c + off;
        if (b < 0 || b >= nbins) {
            err = "internal: node record outside the grid";
            return false;
        }
        bin[k] = (int32_t)b;
        fr[k] = t - c;
    }
    S.perm.assign(M, 0);
    if (fp32) S.rec32.assign(M, PtRec{0, 0.f});
    else S.frac64.assign(M, 0.0);
    std::vector<int32_t> sbin(M);
    std::vector<int64_t> cnt(nbins + 1);
    S.nblocks = (M + L.block - 1) / L.block;
    int64_t part = 0;
    for (int64_t blk = 0; blk < S.nblocks; ++blk) {
        const int64_t k0 = blk * L.block, k1 = std::min(M, k0 + L.block);
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int64_t k = k0; k < k1; ++k) cnt[bin[k] + 1]++;
        for (int64_t b = 0; b < nbins; ++b) cnt[b + 1] += cnt[b];
        // stable counting sort of the block by bin
        for (int64_t k = k0; k < k1; ++k) {
            const int64_t pos = k0 + cnt[bin[k]]++;
            S.perm[pos] = (int32_t)k;
            sbin[pos] = bin[k];
            if (fp32) {
                float f = (float)fr[k];
                if (!(f < 1.0f)) f = 0.99999994f;   // keep the offset inside [0, 1)
                S.rec32[pos] = PtRec{(int32_t)k, f};
            } else {
                S.frac64[pos] = fr[k];
            }
        }
        // items: balanced split of each bin run into ceil(n / Q) pieces
        const size_t it0 = S.items.size();
        for (int64_t i = k0; i < k1;) {
            int64_t j = i;
            while (j < k1 && sbin[j] == sbin[i]) ++j;
            const int64_t n = j - i;
            const int64_t nit = (n + L.Q - 1) / L.Q;
            const int64_t base = n / nit, rem = n % nit;
            int64_t p = i;
            for (int64_t q = 0; q < nit; ++q) {
                const int64_t len = base + (q < rem ? 1 : 0);
                S.items.push_back(Item{sbin[i], (int32_t)p, (int32_t)len, 0});
                p += len;
            }
            i = j;
        }
        // chunks: consecutive items, at most IW items and IW bins
        const size_t it1 = S.items.size();
        for (size_t ci = it0; ci < it1;) {
            const int32_t blo = S.items[ci].bin;
            size_t cj = ci;
            while (cj < it1 && (int)(cj - ci) < L.IW && S.items[cj].bin - blo < L.IW) ++cj;
            Chunk c{};
            c.nitem = (int32_t)(cj - ci);
            c.bin_lo = blo;
            c.nbin = S.items[cj - 1].bin - blo + 1;
            c.part_off = (int32_t)part;
            if (m > 0) part += c.nbin + 2 * m - 1;
            S.chunks.push_back(c);
            S.chunk_block.push_back((int32_t)blk);
            S.chunk_item0.push_back((int32_t)ci);
            ci = cj;
        }
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
    const Chunk empty{0, 0, 0, 0, 0, 0, 0, 0};
    const Item pad_item{0, 0, 0, 0};
    S.launch.assign(order.size(), empty);
    S.launch_items.assign(order.size() * kItemsPerWg, pad_item);
    int64_t roff = 0;
    for (size_t g = 0; g < order.size(); ++g) {
        if (order[g] < 0) continue;
        Chunk c = S.chunks[order[g]];
        const int32_t i0 = S.chunk_item0[order[g]];
        int qmax = 0;
        for (int i = 0; i < c.nitem; ++i) {
            S.launch_items[g * kItemsPerWg + i] = S.items[i0 + i];
            qmax = std::max(qmax, (int)S.items[i0 + i].n);
        }
        c.qmax = qmax;
        c.rec_off = (int32_t)roff;
        if (fp32) {
            // transposed block: point q of item t at rec_off + 64 q + t
            S.trec32.resize((size_t)(roff + (int64_t)qmax * kItemsPerWg), PtRec{0, 0.f});
            for (int i = 0; i < c.nitem; ++i) {
                const Item &it = S.items[i0 + i];
                for (int q = 0; q < it.n; ++q)
                    S.trec32[(size_t)(roff + (int64_t)q * kItemsPerWg + i)] = S.rec32[(size_t)(it.p0 + q)];
            }
            roff += (int64_t)qmax * kItemsPerWg;
        }
        S.launch[g] = c;
    }
    if (roff >= ((int64_t)1 << 31)) {
        err = "too many padded records";
        return false;
    }
    return true;
}

// FFT factorization chosen at plan time (copied into FftArgs)
struct FftPlan {
    int32_t N2 = 0, n1 = 0, n2 = 0, npassA = 0, npassB = 0;
    int radA[kMaxPasses] = {}, radB[kMaxPasses] = {};
    int32_t batchA = 0, batchB = 0, threadsA = 0, threadsB = 0, S = 0;
};

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

// ---------------------------------------------------------------------------
struct nnfft_plan_s {
    nnfft_info_t info{};
    PlanDev desc{};
    PlanDev *ddesc = nullptr;          // device copy of desc (batched launches)
    std::vector<void *> allocs;
    int64_t bytes = 0;
    std::vector<hipEvent_t> prof_ev;   // 4 events per profiled exec
    int prof_max = 0, prof_used = 0;

    void drop_events()
    {
        for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
        prof_ev.clear();
        prof_max = prof_used = 0;
    }
    ~nnfft_plan_s()
    {
        drop_events();
        for (void *p : allocs) (void)hipFree(p);
    }
    template <typename T>
    T *upload(const std::vector<T> &v, hipStream_t s)
    {
        const size_t n = std::max<size_t>(1, v.size());
        void *p = nullptr;
        hip_check(hipMalloc(&p, n * sizeof(T)), "hipMalloc");
        allocs.push_back(p);
        bytes += (int64_t)(n * sizeof(T));
        if (!v.empty()) hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s),
                                  "hipMemcpyAsync");
        return static_cast<T *>(p);
    }
    void *scratch(size_t nbytes)
    {
        void *p = nullptr;
        hip_check(hipMalloc(&p, std::max<size_t>(nbytes, 16)), "hipMalloc");
        allocs.push_back(p);
        bytes += (int64_t)nbytes;
        return p;
    }
};

struct sinc_plan_s {
    nnfft_plan_t p1 = nullptr, p2 = nullptr;
    double *w = nullptr;      // [n_nodes] quadrature weights (FP64, device)
    void *g = nullptr;        // [n_nodes] complex intermediate
    int64_t n_nodes = 0;
    int32_t prec = 0;
    ~sinc_plan_s()
    {
        if (p1) nnfft_destroy(p1);
        if (p2) nnfft_destroy(p2);
        if (w) (void)hipFree(w);
        if (g) (void)hipFree(g);
    }
};

namespace nnfft {
// sinc weight multiply (kernels_sinc.hip)
hipError_t launch_scale_by_weights(int prec, const double *w, const void *src, void *dst, int64_t n,
                                   hipStream_t s);
}

// ---------------------------------------------------------------------------
extern "C" {

const char *nnfft_last_error(void) { return g_last_error.c_str(); }

const char *nnfft_version(void) { return "nnfft-mi355x 0.1 (gfx950)"; }

nnfft_status nnfft_derive_params(int64_t N, double sigma1, double sigma2, int m1, int m2,
                                 nnfft_info_t *out)
{
    if (!out) return fail(NNFFT_ERR_ARG, "null output");
    const nnfft_status st = derive_params(N, sigma1, sigma2, m1, m2, out);
    if (st != NNFFT_OK) return fail(st, "invalid NNFFT parameters (N >= 1, m >= 2, sigma > 1, "
                                        "2 m1 < N1 and 2 m2 <= (1 - 1/sigma1) N2 are required)");
    return NNFFT_OK;
}

static nnfft_status plan_impl(nnfft_plan_t *out, int64_t N, int64_t M1, int64_t M2, double sigma1,
                              double sigma2, int m1, int m2, nnfft_precision prec,
                              const std::vector<double> &v, const std::vector<double> &x,
                              hipStream_t s)
{
    nnfft_info_t P;
    nnfft_status st = derive_params(N, sigma1, sigma2, m1, m2, &P);
    if (st != NNFFT_OK) return fail(st, "invalid NNFFT parameters");
    if (m1 > kMaxM || m2 > kMaxM) return fail(NNFFT_ERR_UNSUPPORTED, "m > 16 is not implemented");
    const bool fp32 = (prec == NNFFT_FP32_COMP);
    if (fp32 && (m1 < 4 || m2 < 4))
        return fail(NNFFT_ERR_UNSUPPORTED, "the FP32 path needs m >= 4 (its window polynomials "
                                           "cannot reach FP32 accuracy for smaller m)");
    if (P.N2 > ((int64_t)1 << 24) || P.G1 > ((int64_t)1 << 24))
        return fail(NNFFT_ERR_UNSUPPORTED, "grid longer than 2^24");
    for (int64_t k = 0; k < M1; ++k)
        if (!(std::fabs(v[k]) <= 0.5)) return fail(NNFFT_ERR_DOMAIN, "frequency node outside [-1/2, 1/2]");
    for (int64_t j = 0; j < M2; ++j)
        if (!(std::fabs(x[j]) <= 0.5)) return fail(NNFFT_ERR_DOMAIN, "spatial node outside [-1/2, 1/2]");

    P.M1 = M1;
    P.M2 = M2;
    P.precision = prec;

    // tables in FP64 -----------------------------------------------------
    std::vector<double> C1d, C2d;
    double e1 = 0.0, e2 = 0.0;
    if (fp32) {
        C1d = fit_window_taps(m1, P.beta1, kDeg, &e1);
        C2d = fit_window_taps(m2, P.beta2, kDeg, &e2);
        P.window_degree = kDeg;
        P.window_fit_err = std::max(e1, e2);
        if (P.window_fit_err > 5e-8)
            return fail(NNFFT_ERR_UNSUPPORTED, "window polynomial misses FP32 accuracy for these sigma, m");
    }
    double corr_err = 0.0;
    std::vector<double> corr = fit_inverse_phi1(P, fp32 ? 1e-9 : 1e-14, fp32 ? kCorr32 : kMaxCorrDeg, &corr_err);
    P.corr_degree = (int32_t)corr.size() - 1;
    P.corr_fit_err = corr_err;
    if (corr_err > (fp32 ? 1e-8 : 1e-12))
        return fail(NNFFT_ERR_UNSUPPORTED, "1/phi_hat_1 series does not converge for this sigma1");
    if (fp32) corr.resize(kCorr32 + 1, 0.0);   // zero-padded to the unrolled length

    std::vector<double> deconv(P.G1);
    for (int64_t c = 0; c < P.G1; ++c) {
        const double l = (double)(c - P.G1 / 2);
        const double phi2 = (double)m2 / (double)P.N2 * window_sinh_hat(m2 * l / (double)P.N2, P.beta2);
        deconv[c] = 1.0 / ((double)P.N1 * (double)P.N2 * phi2);
    }
    const std::vector<double> tw = twiddles(P.N2);

    // node layouts ----------------------------------------------------------
    const Layout lay1 = choose_layout(M1, fp32), lay2 = choose_layout(M2, fp32);
    SideHost sp, ip;
    std::string err;
    // spreading: t_k = N1 v*_k = N1 N v_k / N*, bin = floor(t_k) + G1/2
    if (!build_side(v, (double)P.N1 * (double)N / (double)P.N_star, P.G1 / 2, P.G1, lay1, fp32, m1, sp, err))
        return fail(NNFFT_ERR_ARG, err);
    // interpolation: u_j = N2 N* x_j / N1, bin = floor(u_j) + N2/2
    if (!build_side(x, (double)P.N2 * (double)P.N_star / (double)P.N1, P.N2 / 2, P.N2 + 1, lay2, fp32, 0,
                    ip, err))
        return fail(NNFFT_ERR_ARG, err);
    if (sp.part_cells >= ((int64_t)1 << 31)) return fail(NNFFT_ERR_UNSUPPORTED, "too many partial cells");

    // merge lists: for each grid cell the partial cells of the chunks covering it
    std::vector<int32_t> moff(P.G1 + 1, 0), midx;
    for (const Chunk &c : sp.chunks) {
        const int W = c.nbin + 2 * m1 - 1;
        for (int w = 0; w < W; ++w) {
            const int64_t cell = (int64_t)c.bin_lo - m1 + 1 + w;
            if (cell < 0 || cell >= P.G1) return fail(NNFFT_ERR_ARG, "internal: window outside the grid");
            moff[cell + 1]++;
        }
    }
    for (int64_t c = 0; c < P.G1; ++c) moff[c + 1] += moff[c];
    midx.resize(moff[P.G1]);
    {
        std::vector<int32_t> cur(moff.begin(), moff.end() - 1);
        for (const Chunk &c : sp.chunks) {
            const int W = c.nbin + 2 * m1 - 1;
            for (int w = 0; w < W; ++w) {
                const int64_t cell = (int64_t)c.bin_lo - m1 + 1 + w;
                midx[cur[cell]++] = c.part_off + w;
            }
        }
    }

    // FFT factorization -----------------------------------------------------
    FftPlan fd{};
    fd.N2 = (int32_t)P.N2;
    // one workgroup for short transforms; longer ones as two launches of
    // many workgroups (one or two columns each) so that the partial merge in
    // the first stage's load runs with enough workgroups in flight
    const int64_t single_max = 1024;
    const int kvals = 4096;
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
        if (!fft_factor(P.N2, kvals, n1, n2)) return fail(NNFFT_ERR_UNSUPPORTED, "FFT length cannot be split");
        const std::vector<int> rA = radix_passes(n2), rB = radix_passes(n1);
        if (rA.empty() || rB.empty()) return fail(NNFFT_ERR_UNSUPPORTED, "FFT length not 2,3,5-smooth");
        fd.n1 = (int32_t)n1;
        fd.n2 = (int32_t)n2;
        fd.npassA = (int32_t)rA.size();
        fd.npassB = (int32_t)rB.size();
        std::copy(rA.begin(), rA.end(), fd.radA);
        std::copy(rB.begin(), rB.end(), fd.radB);
        fd.batchA = (int32_t)std::max<int64_t>(1, std::min<int64_t>(n1 / 128, kvals / n2));
        fd.batchB = (int32_t)std::max<int64_t>(1, std::min<int64_t>(n2 / 128, kvals / n1));
        fd.threadsA = threads_for((int64_t)fd.batchA * n2);
        fd.threadsB = threads_for((int64_t)fd.batchB * n1);
    }
    {
        const double U = (double)P.N2 * (double)P.N_star / (2.0 * (double)P.N1);
        int64_t S = (int64_t)std::ceil(U) + m2;
        fd.S = (int32_t)std::min<int64_t>(S, P.N2 / 2);
    }

    // device upload -----------------------------------------------------------
    nnfft_plan_s *pl = new nnfft_plan_s();
    try {
        PlanDev &D = pl->desc;
        D.prec = prec;
        if (const char *e = std::getenv("NNFFT_GRID_MAX")) D.sp_grid_max = D.ip_grid_max = atoi(e);
        SpreadArgs &SA = D.sp;
        InterpArgs &IA = D.ip;
        FftArgs &FA = D.fft;
        SA.items = pl->upload(sp.launch_items, s);
        SA.chunks = pl->upload(sp.launch, s);
        SA.ngrid = (int32_t)sp.launch.size();
        SA.m = m1;
        SA.beta = P.beta1;
        SA.inv_den = 1.0 / (1.0 - std::exp(-2.0 * P.beta1));
        IA.items = pl->upload(ip.launch_items, s);
        IA.chunks = pl->upload(ip.launch, s);
        IA.ngrid = (int32_t)ip.launch.size();
        IA.m = m2;
        IA.beta = P.beta2;
        IA.inv_den = 1.0 / (1.0 - std::exp(-2.0 * P.beta2));
        IA.N2 = (int32_t)P.N2;
        IA.ip_off = (int32_t)(P.N2 / 2);
        IA.u_to_x = (double)P.N1 / ((double)P.N2 * (double)P.N_star);
        IA.corr = pl->upload(corr, s);
        IA.corr_deg = P.corr_degree;
        if (fp32) {
            SA.rec32 = pl->upload(sp.trec32, s);
            IA.rec32 = pl->upload(ip.trec32, s);
            std::vector<float> c1(C1d.begin(), C1d.end()), c2(C2d.begin(), C2d.end());
            SA.C = pl->upload(c1, s);
            IA.C = pl->upload(c2, s);
        } else {
            SA.perm = pl->upload(sp.perm, s);
            SA.frac64 = pl->upload(sp.frac64, s);
            IA.perm = pl->upload(ip.perm, s);
            IA.frac64 = pl->upload(ip.frac64, s);
        }
        const size_t csz = fp32 ? 8 : 16;
        SA.partial = pl->scratch((size_t)sp.part_cells * 16);
        FA.partial = SA.partial;
        FA.merge_off = pl->upload(moff, s);
        FA.merge_idx = pl->upload(midx, s);
        FA.deconv = pl->upload(deconv, s);
        if (fp32) {
            std::vector<float> tw32(tw.begin(), tw.end());
            FA.tw = pl->upload(tw32, s);
        } else {
            FA.tw = pl->upload(tw, s);
        }
        FA.Y = pl->scratch((size_t)P.N2 * csz);
        FA.hlin = pl->scratch((size_t)(P.N2 + 1) * csz);
        IA.hlin = FA.hlin;
        FA.N2 = (int32_t)P.N2;
        FA.G1 = (int32_t)P.G1;
        FA.n1 = fd.n1;
        FA.n2 = fd.n2;
        FA.batchA = fd.batchA;
        FA.batchB = fd.batchB;
        FA.threadsA = fd.threadsA;
        FA.threadsB = fd.threadsB;
        FA.S = fd.S;
        FA.npassA = fd.npassA;
        FA.npassB = fd.npassB;
        for (int i = 0; i < kMaxPasses; ++i) {
            FA.radA[i] = (int8_t)fd.radA[i];
            FA.radB[i] = (int8_t)fd.radB[i];
        }
        pl->ddesc = static_cast<PlanDev *>(pl->scratch(sizeof(PlanDev)));
        hip_check(hipMemcpyAsync(pl->ddesc, &pl->desc, sizeof(PlanDev), hipMemcpyHostToDevice, s),
                  "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
        P.device_bytes = pl->bytes;
        P.block_points = lay1.block;
        P.items_points = lay1.Q;
        P.spread_workgroups = D.sp.ngrid;
        P.interp_workgroups = D.ip.ngrid;
        P.fft_n1 = fd.n1;
        P.fft_n2 = fd.n2;
        pl->info = P;
    } catch (const HipError &e) {
        delete pl;
        return fail(e.err == hipErrorOutOfMemory ? NNFFT_ERR_NOMEM : NNFFT_ERR_DEVICE,
                    std::string(e.what) + ": " + hipGetErrorString(e.err));
    }
    *out = pl;
    return NNFFT_OK;
}

static nnfft_status copy_nodes(const double *d, int64_t n, std::vector<double> &h, hipStream_t s)
{
    h.resize(n);
    if (n == 0) return NNFFT_OK;
    hipError_t e = hipMemcpyAsync(h.data(), d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("copying nodes: ") + hipGetErrorString(e));
    return NNFFT_OK;
}

nnfft_status nnfft_plan(nnfft_plan_t *out, int64_t N, int64_t M1, int64_t M2, double sigma1,
                        double sigma2, int m1, int m2, nnfft_precision prec, const double *v,
                        const double *x, void *stream)
{
    if (!out) return fail(NNFFT_ERR_ARG, "null plan pointer");
    *out = nullptr;
    if (M1 < 1 || M2 < 1 || M1 > ((int64_t)1 << 30) || M2 > ((int64_t)1 << 30))
        return fail(NNFFT_ERR_ARG, "node counts must be in [1, 2^30]");
    if (prec != NNFFT_FP64_PLAIN && prec != NNFFT_FP32_COMP) return fail(NNFFT_ERR_ARG, "unknown precision");
    if (!v || !x) return fail(NNFFT_ERR_ARG, "null node array");
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<double> hv, hx;
        nnfft_status st = copy_nodes(v, M1, hv, s);
        if (st != NNFFT_OK) return st;
        st = copy_nodes(x, M2, hx, s);
        if (st != NNFFT_OK) return st;
        return plan_impl(out, N, M1, M2, sigma1, sigma2, m1, m2, prec, hv, hx, s);
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status nnfft_exec(nnfft_plan_t p, const void *f, void *y, void *stream)
{
    if (!p || !f || !y) return fail(NNFFT_ERR_ARG, "null argument");
    hipEvent_t *ev = nullptr;
    if (p->prof_used < p->prof_max) ev = &p->prof_ev[4 * (size_t)p->prof_used++];
    const hipError_t e = launch_exec(p->desc, f, y, static_cast<hipStream_t>(stream), ev);
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
            if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, std::string("batched launch: ") + hipGetErrorString(e));
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
    p->prof_ev.resize(4 * (size_t)max_execs);
    for (auto &e : p->prof_ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            p->drop_events();
            return fail(NNFFT_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    p->prof_max = max_execs;
    p->prof_used = 0;
    return NNFFT_OK;
}

nnfft_status nnfft_profile_stop(nnfft_plan_t p, double *stage_ms, int *nexecs)
{
    if (!p || !stage_ms) return fail(NNFFT_ERR_ARG, "bad argument");
    const int n = p->prof_used;
    double acc[3] = {0.0, 0.0, 0.0};
    if (n > 0 && hipEventSynchronize(p->prof_ev[4 * (size_t)(n - 1) + 3]) != hipSuccess) {
        p->drop_events();
        return fail(NNFFT_ERR_DEVICE, "hipEventSynchronize failed");
    }
    for (int i = 0; i < n; ++i)
        for (int s = 0; s < 3; ++s) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p->prof_ev[4 * (size_t)i + s], p->prof_ev[4 * (size_t)i + s + 1]) !=
                hipSuccess) {
                p->drop_events();
                return fail(NNFFT_ERR_DEVICE, "hipEventElapsedTime failed");
            }
            acc[s] += ms;
        }
    for (int s = 0; s < 3; ++s) stage_ms[s] = n > 0 ? acc[s] / n : 0.0;
    if (nexecs) *nexecs = n;
    p->drop_events();
    return NNFFT_OK;
}

nnfft_status nnfft_destroy(nnfft_plan_t p)
{
    if (!p) return fail(NNFFT_ERR_ARG, "null plan");
    delete p;
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
        std::vector<double> z, w;
        if (quad == SINC_QUAD_GAUSS_LEGENDRE) gauss_legendre_rule(n_quad, z, w);
        else clenshaw_curtis_rule(n_quad, z, w);
        const int64_t nn = (int64_t)z.size();
        std::vector<double> xs(nn), vs(nn);
        for (int64_t j = 0; j < nn; ++j) {
            xs[j] = 0.5 * z[j];    // step 1: spatial nodes z_j / 2
            vs[j] = -0.5 * z[j];   // step 3: frequencies -z_j / 2
        }
        std::vector<double> ha, hb;
        nnfft_status st = copy_nodes(a, L1, ha, s);
        if (st != NNFFT_OK) return st;
        st = copy_nodes(b, L2, hb, s);
        if (st != NNFFT_OK) return st;
        sinc_plan_s *sp = new sinc_plan_s();
        sp->n_nodes = nn;
        sp->prec = prec;
        st = plan_impl(&sp->p1, N, L1, nn, sigma1, sigma2, m1, m2, prec, ha, xs, s);
        if (st == NNFFT_OK) st = plan_impl(&sp->p2, N, nn, L2, sigma1, sigma2, m1, m2, prec, vs, hb, s);
        if (st != NNFFT_OK) {
            delete sp;
            return st;
        }
        const size_t csz = (prec == NNFFT_FP32_COMP) ? 8 : 16;
        hipError_t e = hipMalloc(&sp->w, (size_t)nn * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&sp->g, (size_t)nn * csz);
        if (e == hipSuccess) e = hipMemcpyAsync(sp->w, w.data(), (size_t)nn * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            delete sp;
            return fail(e == hipErrorOutOfMemory ? NNFFT_ERR_NOMEM : NNFFT_ERR_DEVICE, hipGetErrorString(e));
        }
        *out = sp;
        return NNFFT_OK;
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}

nnfft_status sinc_exec(sinc_plan_t p, const void *c, void *h, void *stream)
{
    if (!p || !c || !h) return fail(NNFFT_ERR_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    nnfft_status st = nnfft_exec(p->p1, c, p->g, stream);          // step 1
    if (st != NNFFT_OK) return st;
    const hipError_t e = launch_scale_by_weights(p->prec, p->w, p->g, p->g, p->n_nodes, s);   // step 2
    if (e != hipSuccess) return fail(NNFFT_ERR_DEVICE, hipGetErrorString(e));
    return nnfft_exec(p->p2, p->g, h, stream);                     // step 3
}

nnfft_status nnfft_quadrature(sinc_quad quad, int64_t n_quad, double *z, double *w)
{
    if (n_quad < 1 || n_quad > ((int64_t)1 << 24) || !z || !w) return fail(NNFFT_ERR_ARG, "bad argument");
    if (quad != SINC_QUAD_GAUSS_LEGENDRE && quad != SINC_QUAD_CLENSHAW_CURTIS)
        return fail(NNFFT_ERR_ARG, "unknown quadrature rule");
    try {
        std::vector<double> zz, ww;
        if (quad == SINC_QUAD_GAUSS_LEGENDRE) gauss_legendre_rule(n_quad, zz, ww);
        else clenshaw_curtis_rule(n_quad, zz, ww);
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

nnfft_status sinc_destroy(sinc_plan_t p)
{
    if (!p) return fail(NNFFT_ERR_ARG, "null plan");
    delete p;
    return NNFFT_OK;
}

}  // extern "C"
