// Layout autotuner of include/nnfft.h: times candidate node layouts on the
// device and installs the fastest in the tuning table.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "../../include/nnfft.h"
#include "internal.h"
#include "plan.h"

using namespace nnfft;

namespace {

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the synthetic tuning nodes.
uint64_t splitmix64(uint64_t &s)
{
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform_half(uint64_t &s)
{
    return (double)(splitmix64(s) >> 11) * 0x1.0p-53 - 0.5;   // [-1/2, 1/2)
}

struct Bufs {
    void *f = nullptr, *y = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Bufs()
    {
        if (f) (void)hipFree(f);
        if (y) (void)hipFree(y);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace

extern "C" nnfft_status nnfft_autotune(int64_t N, int64_t M, int m, nnfft_precision prec, int reps,
                                       void *stream, nnfft_tuning_t *best)
{
    if (!best || M < 1 || M > ((int64_t)1 << 30) || reps < 1 ||
        (prec != NNFFT_FP64_PLAIN && prec != NNFFT_FP32_COMP))
        return fail(NNFFT_ERR_ARG, "bad autotune argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool fp32 = prec == NNFFT_FP32_COMP;
    try {
        std::vector<double> v(M), x(M);
        uint64_t seed = 0x2107026710000001ull;
        for (int64_t k = 0; k < M; ++k) {
            v[k] = uniform_half(seed);
            x[k] = uniform_half(seed);
        }
        const size_t csz = fp32 ? 8 : 16;
        Bufs B;
        if (hipMalloc(&B.f, (size_t)M * csz) != hipSuccess || hipMalloc(&B.y, (size_t)M * csz) != hipSuccess)
            return fail(NNFFT_ERR_NOMEM, "autotune buffers");
        if (hipMemsetAsync(B.f, 0, (size_t)M * csz, s) != hipSuccess || hipEventCreate(&B.e0) != hipSuccess ||
            hipEventCreate(&B.e1) != hipSuccess)
            return fail(NNFFT_ERR_DEVICE, "autotune setup");

        std::vector<Layout> cand;
        cand.push_back(rule_layout(M, fp32));
        const std::vector<int> Qs = fp32 ? std::vector<int>{4, 8, 16, 32} : std::vector<int>{2, 4, 8};
        const std::vector<int64_t> blocks = {(int64_t)1 << 13, (int64_t)1 << 14, (int64_t)1 << 15,
                                             (int64_t)1 << 16, (int64_t)1 << 17, (int64_t)1 << 18};
        for (int Q : Qs)
            for (int64_t b : blocks)
                {
                    Layout L;
                    L.Q = Q;
                    L.block = b;
                    L = sanitize_layout(L, M, fp32);
                    bool dup = false;
                    for (const Layout &c : cand) dup = dup || (c.Q == L.Q && c.block == L.block);
                    if (!dup) cand.push_back(L);
                }

        double best_ms = 1e300;
        Layout best_L = cand[0];
        int timed = 0;
        nnfft_status last = NNFFT_OK;
        for (const Layout &L : cand) {
            HostPlan H;
            nnfft_status st = plan_host(H, N, M, M, 2.0, 2.0, m, m, prec, v, x, &L, &L);
            if (st != NNFFT_OK) {
                if (st != NNFFT_ERR_ARG) return st;   // parameters themselves are unsupported
                last = st;
                continue;
            }
            nnfft_plan_t p = nullptr;
            st = plan_create(H, hip_mem(), s, &p);
            if (st != NNFFT_OK) return st;
            for (int i = 0; i < 2 && st == NNFFT_OK; ++i) st = nnfft_exec(p, B.f, B.y, stream);
            if (st == NNFFT_OK && hipEventRecord(B.e0, s) != hipSuccess) st = NNFFT_ERR_DEVICE;
            for (int i = 0; i < reps && st == NNFFT_OK; ++i) st = nnfft_exec(p, B.f, B.y, stream);
            float ms = 0.f;
            if (st == NNFFT_OK && (hipEventRecord(B.e1, s) != hipSuccess || hipEventSynchronize(B.e1) != hipSuccess ||
                                   hipEventElapsedTime(&ms, B.e0, B.e1) != hipSuccess))
                st = NNFFT_ERR_DEVICE;
            nnfft_destroy(p);
            if (st != NNFFT_OK) return fail(st, "autotune exec failed");
            ++timed;
            if (ms / reps < best_ms) {
                best_ms = ms / reps;
                best_L = L;
            }
        }
        if (timed == 0) return fail(last, "no candidate layout could be planned");
        set_tuned_layout(fp32, M, best_L);
        *best = nnfft_tuning_t{};
        best->items_points = best_L.Q;
        best->block_points = best_L.block;
        best->exec_ms = best_ms;
        best->candidates = timed;
        best->tuned = 1;
        return NNFFT_OK;
    } catch (const std::bad_alloc &) {
        return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    }
}
