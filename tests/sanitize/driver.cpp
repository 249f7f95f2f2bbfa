// Plans every window family and precision for a spread of bandwidths, kernel
// sizes and node sets (uniform, clustered, edge nodes, single nodes) on the
// host only, through the dry-run entry point and the NFFT planner (2^18-point
// sides too, whose node blocks are sorted on several threads).  Built
// with sanitizers, it checks the planner's memory accesses and, with planner
// threads of its own on top of the two-sided builds, its threading.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>
#include "../../include/nnfft.h"
#include "../../paper_2107_02671_amd/csrc/plan.h"

static int run(unsigned seed, bool small)
{
    std::mt19937_64 g(seed);
    std::uniform_real_distribution<double> U(-0.5, 0.5);
    std::normal_distribution<double> Nrm(0.0, 1e-3);
    int refused = 0;
    const std::vector<int64_t> Ms = small ? std::vector<int64_t>{1, 65, 1000, 40000}
                                          : std::vector<int64_t>{1, 2, 63, 64, 65, 1000, 40000};
    for (int64_t M : Ms)
        for (int prec : {0, 1})
            for (int win : {0, 1, 2, 3})
                for (int N : {2, 64, 333, 4096})
                    for (int m : {4, 6, 16})
                        for (int clustered : {0, 1}) {
                            if (M >= 40000 && m != 6) continue;
                            std::vector<double> v(M), x(M);
                            for (int64_t k = 0; k < M; ++k) {
                                if (clustered) {
                                    const double c = (double)(k % 7) * 0.1 - 0.3;
                                    v[k] = std::clamp(c + Nrm(g), -0.5, 0.5);
                                    x[k] = std::clamp(-c + Nrm(g), -0.5, 0.5);
                                } else {
                                    v[k] = U(g);
                                    x[k] = U(g);
                                }
                            }
                            if (M > 2) {
                                v[0] = -0.5;
                                v[1] = 0.5;
                                x[0] = 0.5;
                                x[1] = -0.5;
                            }
                            nnfft_info_t info;
                            if (nnfft_plan_window_dry_run(N, M, M, 2.0, 1.5, m, m, (nnfft_precision)prec,
                                                          (nnfft_window)win, v.data(), x.data(), &info) != NNFFT_OK)
                                ++refused;
                            nnfft::HostPlan H;
                            if (nnfft::nfft_plan_host(H, 2 * N, M, 2.0, m, (nnfft_precision)prec, x) != NNFFT_OK)
                                ++refused;
                        }
    // one side large enough for its node blocks to be sorted on several threads
    for (int prec : {0, 1}) {
        const int64_t M = (int64_t)1 << 18;
        std::vector<double> v(M), x(M);
        for (int64_t k = 0; k < M; ++k) {
            v[k] = U(g);
            x[k] = U(g);
        }
        nnfft_info_t info;
        if (nnfft_plan_window_dry_run(4096, M, M, 2.0, 2.0, 6, 6, (nnfft_precision)prec, NNFFT_WINDOW_SINH, v.data(),
                                      x.data(), &info) != NNFFT_OK)
            ++refused;
        // the layout image and its digest (tables cached by the first plan)
        uint64_t d1 = 0, d2 = 0;
        if (nnfft_plan_window_dry_run_digest(4096, M, M, 2.0, 2.0, 6, 6, (nnfft_precision)prec, NNFFT_WINDOW_SINH,
                                             v.data(), x.data(), &d1) != NNFFT_OK ||
            nnfft_plan_window_dry_run_digest(4096, M, M, 2.0, 2.0, 6, 6, (nnfft_precision)prec, NNFFT_WINDOW_SINH,
                                             v.data(), x.data(), &d2) != NNFFT_OK || d1 != d2)
            std::abort();
    }
    // fast sinc transform plans with the middle operator (both rules, both
    // precisions, Chebyshev-crowded nodes, small and large bands)
    for (int prec : {0, 1})
        for (int quad : {0, 1})
            for (int N : {64, 1024})
                for (int m : {4, 6}) {
                    const int64_t L = small ? 3000 : 20000;
                    std::vector<double> a(L), b(L);
                    for (int64_t k = 0; k < L; ++k) {
                        a[k] = 0.5 * std::cos(3.141592653589793 * (k + 0.5) / (double)L);
                        b[k] = U(g);
                    }
                    nnfft::SincHostPlan S;
                    if (nnfft::sinc_host(S, N, L, L, (sinc_quad)quad, 2 * N, 2.0, 2.0, m, m, (nnfft_precision)prec, a,
                                         b, true) != NNFFT_OK) {
                        ++refused;
                        continue;
                    }
                    if (!S.mid_ok || S.mid.Wb < 2 * m || S.mid.K.size() != (size_t)S.mid.Wb * S.mid.lo.size())
                        std::abort();
                }
    return refused;
}

int main(int argc, char **argv)
{
    // "threads": four planner threads at once (smaller node sets each)
    if (argc > 1 && std::strcmp(argv[1], "threads") == 0) {
        std::vector<std::thread> th;
        int refused[4] = {0, 0, 0, 0};
        for (int t = 0; t < 4; ++t) th.emplace_back([t, &refused] { refused[t] = run(100 + t, true); });
        for (auto &x : th) x.join();
        std::printf("refused %d\n", refused[0] + refused[1] + refused[2] + refused[3]);
        return 0;
    }
    std::printf("refused %d\n", run(11, false));
    return 0;
}
