// Request serving layer (include/nnfft_serve.h): device arena, planner
// threads, a continuous-batching executor and per-stream completion threads.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/nnfft.h"
#include "../../include/nnfft_serve.h"
#include "internal.h"
#include "plan.h"

using namespace nnfft;

namespace {

// First-fit arena over one device allocation; blocks are 256-byte aligned
// and coalesced when released.
class Arena {
public:
    char *base = nullptr;
    size_t size = 0;

    void *alloc(size_t n)
    {
        n = (std::max<size_t>(n, 1) + 255) & ~(size_t)255;
        std::lock_guard<std::mutex> g(mu_);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            used_[off] = n;
            in_use_ += n;
            peak_ = std::max(peak_, in_use_);
            return base + off;
        }
        return nullptr;
    }
    void release(void *p)
    {
        std::lock_guard<std::mutex> g(mu_);
        const size_t off = static_cast<char *>(p) - base;
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second, start = off;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    void reset(size_t n)
    {
        free_.clear();
        used_.clear();
        free_[0] = n;
        size = n;
    }
    size_t in_use()
    {
        std::lock_guard<std::mutex> g(mu_);
        return in_use_;
    }
    size_t peak()
    {
        std::lock_guard<std::mutex> g(mu_);
        return peak_;
    }

private:
    std::mutex mu_;
    std::map<size_t, size_t> free_;   // offset -> length
    std::map<size_t, size_t> used_;
    size_t in_use_ = 0, peak_ = 0;
};

void *arena_alloc(void *ctx, size_t n) { return static_cast<Arena *>(ctx)->alloc(n); }
void arena_release(void *ctx, void *p) { static_cast<Arena *>(ctx)->release(p); }

struct Resident;

struct Req {
    uint64_t ticket = 0;
    nnfft_request_t r{};
    nnfft_plan_t plan = nullptr;    // NNFFT request
    sinc_plan_t splan = nullptr;    // sinc request
    Resident *res = nullptr;        // keyed request: its resident plan
    nnfft_result_t out{};
    bool done = false;
};

struct Resident {
    uint64_t key = 0;
    nnfft_request_t shape{};
    nnfft_plan_t plan = nullptr;
    sinc_plan_t splan = nullptr;
    bool busy = false;          // a request that uses it is admitted or in flight
    bool building = true;       // its first request is still planning it
    bool evict_when_idle = false;
    std::deque<Req *> waiting;  // requests for this key behind the current one
    uint64_t last_use = 0;
    int64_t bytes = 0;
};

struct Group {
    std::vector<Req *> reqs;
    hipEvent_t ev = nullptr;
};

bool same_shape(const nnfft_request_t &a, const nnfft_request_t &b)
{
    return a.kind == b.kind && a.precision == b.precision && a.N == b.N && a.M1 == b.M1 && a.M2 == b.M2 &&
           a.sigma1 == b.sigma1 && a.sigma2 == b.sigma2 && a.m1 == b.m1 && a.m2 == b.m2 &&
           (a.kind != NNFFT_REQ_SINC || (a.quad == b.quad && a.n_quad == b.n_quad)) &&
           (a.kind == NNFFT_REQ_SINC || a.window == b.window);
}

}  // namespace

struct nnfft_server_s {
    nnfft_server_config_t cfg{};
    Arena arena;
    void *arena_mem = nullptr;
    DevMem mem{};
    std::vector<hipStream_t> streams;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_pending, cv_ready, cv_done, cv_space;
    std::deque<Req *> pending;   // submitted, not yet planned
    std::deque<Req *> ready;     // admitted, not yet launched
    std::vector<std::deque<Group *>> inflight;
    std::vector<std::unique_ptr<std::condition_variable>> cv_inflight;
    std::unordered_map<uint64_t, Req *> tickets;
    std::unordered_map<uint64_t, Resident *> residents;
    uint64_t next_ticket = 1, use_clock = 0;
    int64_t planning = 0;        // requests being planned
    int64_t active_bytes = 0;    // arena bytes reserved by live plans (admitted, in flight, resident)
    int64_t groups_inflight = 0; // launch groups issued and not yet completed
    bool stopping = false;
    bool exec_done = false;      // the executor has left its loop
    nnfft_server_stats_t st{};

    std::vector<std::thread> planners, completers;
    std::thread executor;

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }

    void finish(Req *q, nnfft_status status, const std::string &msg)   // mu held
    {
        q->out.status = status;
        if (status != NNFFT_OK) {
            std::snprintf(q->out.message, sizeof(q->out.message), "%s", msg.c_str());
            st.failed++;
        }
        q->out.done_ms = now_ms();
        q->done = true;
        st.completed++;
        cv_done.notify_all();
        if (stopping) cv_ready.notify_all();   // the executor leaves once all are done
    }

    void drop_resident(Resident *rs)   // mu held
    {
        residents.erase(rs->key);
        if (rs->plan) nnfft_destroy(rs->plan);
        if (rs->splan) sinc_destroy(rs->splan);
        active_bytes -= rs->bytes;
        delete rs;
        cv_space.notify_all();
    }

    void planner_loop();
    void executor_loop();
    void completion_loop(int si);
    bool admit(size_t bytes, std::unique_lock<std::mutex> &lk, std::string &err);
    void release_resident_if_evicted(Resident *rs);   // mu held
    // the least recently used resident plan that no request uses or waits for
    Resident *idle_resident()   // mu held
    {
        Resident *lru = nullptr;
        for (auto &kv : residents) {
            Resident *r = kv.second;
            if (!r->busy && !r->building && r->waiting.empty() && (!lru || r->last_use < lru->last_use)) lru = r;
        }
        return lru;
    }
};

// Reserves `bytes` of the arena for a plan about to be created, evicting
// idle resident plans (least recently used first) and otherwise waiting for
// finished requests to release theirs.  mu is held on entry and exit.
// Fails only when nothing else holds arena space, i.e. the plan can never fit.
bool nnfft_server_s::admit(size_t bytes, std::unique_lock<std::mutex> &lk, std::string &err)
{
    for (;;) {
        if (active_bytes + (int64_t)bytes <= (int64_t)arena.size) {
            active_bytes += (int64_t)bytes;
            return true;
        }
        Resident *lru = idle_resident();
        if (lru) {
            drop_resident(lru);
            st.evictions++;
            continue;
        }
        if (active_bytes == 0) {
            err = "the plan needs " + std::to_string(bytes) + " bytes of device memory, more than the arena (" +
                  std::to_string(arena.size) + " bytes)";
            return false;
        }
        st.admission_waits++;
        cv_space.wait(lk);
    }
}

void nnfft_server_s::planner_loop()
{
    hipStream_t s = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    NodePrepScratch prep;   // this planner's node-sort memory, reused request after request
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_pending.wait(lk, [&] { return stopping || !pending.empty(); });
        if (pending.empty()) {
            if (stopping) break;
            continue;
        }
        Req *q = pending.front();
        pending.pop_front();
        const nnfft_request_t r = q->r;
        q->out.plan_ms = now_ms();

        // keyed request whose plan is resident (or being built): reuse it
        if (r.plan_key != 0) {
            auto it = residents.find(r.plan_key);
            if (it != residents.end()) {
                Resident *rs = it->second;
                if (!same_shape(rs->shape, r)) {
                    finish(q, NNFFT_ERR_ARG, "plan_key names a resident plan of other parameters");
                    continue;
                }
                q->res = rs;
                q->out.plan_reused = 1;
                q->out.footprint_bytes = rs->bytes;
                if (rs->busy || rs->building) {
                    rs->waiting.push_back(q);
                } else {
                    rs->busy = true;
                    rs->last_use = ++use_clock;
                    q->plan = rs->plan;
                    q->splan = rs->splan;
                    q->out.admit_ms = now_ms();
                    ready.push_back(q);
                    cv_ready.notify_one();
                }
                continue;
            }
            Resident *rs = new Resident();
            rs->key = r.plan_key;
            rs->shape = r;
            rs->busy = true;
            residents[r.plan_key] = rs;
            q->res = rs;
        }
        ++planning;
        lk.unlock();

        // Algorithm 2.2 step 0: NNFFT requests order their nodes on the device
        // (planner stream) and schedule on the host; sinc requests (and keys
        // wider than 32 bits) plan on the host from node copies
        nnfft_status status = have_stream ? NNFFT_OK : NNFFT_ERR_DEVICE;
        std::string err = have_stream ? "" : "planner stream";
        HostPlan H;
        SincHostPlan S;
        DevRecords R;
        bool dev_nodes = false;
        size_t bytes = 0;
        if (status == NNFFT_OK) {
            try {
                bool host = true;
                if (r.kind != NNFFT_REQ_SINC) {
                    status = plan_device_nodes(H, R, prep, r.N, r.M1, r.M2, r.sigma1, r.sigma2, r.m1, r.m2,
                                               (nnfft_precision)r.precision, r.window, r.v, r.x, s, &host);
                    dev_nodes = !host;
                }
                if (status == NNFFT_OK && host) {
                    std::vector<double> hv, hx;
                    H = HostPlan{};
                    status = copy_nodes(r.v, r.M1, hv, s);
                    if (status == NNFFT_OK) status = copy_nodes(r.x, r.M2, hx, s);
                    if (status == NNFFT_OK) {
                        if (r.kind == NNFFT_REQ_SINC)
                            status = sinc_host(S, r.N, r.M1, r.M2, (sinc_quad)r.quad, r.n_quad, r.sigma1, r.sigma2,
                                               r.m1, r.m2, (nnfft_precision)r.precision, hv, hx);
                        else
                            status = plan_host(H, r.N, r.M1, r.M2, r.sigma1, r.sigma2, r.m1, r.m2,
                                               (nnfft_precision)r.precision, hv, hx, nullptr, nullptr, r.window);
                    }
                }
                if (status != NNFFT_OK) err = nnfft_last_error();
                // arena blocks are 256-byte granular: one per NNFFT plan, three per sinc plan
                auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
                bytes = r.kind == NNFFT_REQ_SINC ? r256(S.h1.total_bytes) + r256(S.h2.total_bytes) + r256(S.wg_bytes)
                                                 : r256(H.total_bytes);
            } catch (const HipError &e) {
                status = NNFFT_ERR_DEVICE;
                err = std::string(e.what) + ": " + hipGetErrorString(e.err);
            } catch (const std::bad_alloc &) {
                status = NNFFT_ERR_NOMEM;
                err = "host allocation failed";
            }
        }

        lk.lock();
        // admission: reserve, create in the arena; an allocation that fails
        // on fragmentation waits for the next release and tries again.  Plans
        // leave the arena only under mu, together with their reservation, so
        // active_bytes == 0 here means the arena emptied while this create
        // ran: retry at once, and give up only if that retry fails as well.
        bool retried_empty = false;
        while (status == NNFFT_OK) {
            if (!admit(bytes, lk, err)) {
                status = NNFFT_ERR_NOMEM;
                break;
            }
            lk.unlock();
            if (r.kind == NNFFT_REQ_SINC) status = sinc_create(S, mem, s, &q->splan);
            else status = plan_create(H, mem, s, &q->plan, dev_nodes ? &R : nullptr);
            if (status != NNFFT_OK) err = nnfft_last_error();
            lk.lock();
            if (status == NNFFT_OK) break;
            active_bytes -= (int64_t)bytes;
            cv_space.notify_all();
            if (status != NNFFT_ERR_NOMEM) break;
            if (Resident *lru = idle_resident()) {   // free space held by an idle resident plan
                drop_resident(lru);
                st.evictions++;
            } else if (active_bytes == 0) {
                if (retried_empty) break;
                retried_empty = true;
            } else {
                st.admission_waits++;
                cv_space.wait(lk);
            }
            status = NNFFT_OK;
        }
        --planning;
        q->out.footprint_bytes = (int64_t)bytes;
        Resident *rs = q->res;
        if (status != NNFFT_OK) {
            if (rs) {   // the key's plan could not be built: fail its queue too
                residents.erase(rs->key);
                for (Req *w : rs->waiting) finish(w, status, err);
                delete rs;
                q->res = nullptr;
            }
            finish(q, status, err);
            continue;
        }
        if (rs) {
            rs->plan = q->plan;
            rs->splan = q->splan;
            rs->bytes = (int64_t)bytes;
            rs->building = false;
            rs->last_use = ++use_clock;
        }
        q->out.admit_ms = now_ms();
        ready.push_back(q);
        cv_ready.notify_one();
    }
    lk.unlock();
    if (have_stream) (void)hipStreamDestroy(s);
}

void nnfft_server_s::executor_loop()
{
    int next_stream = 0;
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // continuous batching: launch at once while fewer than two groups per
        // stream are on the device; beyond that, let ready requests gather
        // into the next group until one completes
        const int64_t cap = 2 * (int64_t)streams.size();
        cv_ready.wait(lk, [&] {
            return (!ready.empty() && groups_inflight < cap) || (stopping && st.completed == st.submitted);
        });
        if (ready.empty()) break;
        Group *g = new Group();
        while (!ready.empty() && (int)g->reqs.size() < cfg.max_batch) {
            g->reqs.push_back(ready.front());
            ready.pop_front();
        }
        const int si = next_stream;
        next_stream = (next_stream + 1) % (int)streams.size();
        const double t_launch = now_ms();
        lk.unlock();

        hipStream_t s = streams[si];
        std::vector<nnfft_plan_t> p1, p3;
        std::vector<const void *> f1, f3;
        std::vector<void *> y1, y3;
        std::vector<Req *> direct;   // sinc requests with NFFT steps: not batched
        for (Req *q : g->reqs) {
            q->out.launch_ms = t_launch;
            q->out.group_size = (int32_t)g->reqs.size();
            if (q->splan && (q->splan->step1_nfft || q->splan->step3_nfft)) {
                direct.push_back(q);
            } else if (q->splan) {
                p1.push_back(q->splan->p1);
                f1.push_back(q->r.f);
                y1.push_back(q->splan->g);
                p3.push_back(q->splan->p2);
                f3.push_back(q->splan->g);
                y3.push_back(q->r.y);
            } else {
                p1.push_back(q->plan);
                f1.push_back(q->r.f);
                y1.push_back(q->r.y);
            }
        }
        nnfft_status status = nnfft_exec_batch((int)p1.size(), p1.data(), f1.data(), y1.data(), s);
        for (Req *q : direct)
            if (status == NNFFT_OK) status = sinc_exec(q->splan, q->r.f, q->r.y, s);
        for (Req *q : g->reqs) {
            if (status != NNFFT_OK || !q->splan || q->splan->step1_nfft || q->splan->step3_nfft) continue;
            const sinc_plan_t sp = q->splan;
            if (launch_scale_by_weights(sp->prec, sp->w, sp->g, sp->g, sp->n_nodes, s) != hipSuccess)
                status = NNFFT_ERR_DEVICE;
        }
        if (status == NNFFT_OK && !p3.empty())
            status = nnfft_exec_batch((int)p3.size(), p3.data(), f3.data(), y3.data(), s);
        std::string err = status == NNFFT_OK ? "" : nnfft_last_error();
        if (status == NNFFT_OK && (hipEventCreateWithFlags(&g->ev, hipEventDisableTiming) != hipSuccess ||
                                   hipEventRecord(g->ev, s) != hipSuccess)) {
            status = NNFFT_ERR_DEVICE;
            err = "event record failed";
        }
        lk.lock();
        st.groups++;
        groups_inflight++;
        if (status != NNFFT_OK) {
            for (Req *q : g->reqs) {
                q->out.status = status;
                std::snprintf(q->out.message, sizeof(q->out.message), "%s", err.c_str());
            }
            if (g->ev) (void)hipEventDestroy(g->ev);
            g->ev = nullptr;
        }
        inflight[si].push_back(g);
        cv_inflight[si]->notify_one();
    }
    exec_done = true;
    for (auto &c : cv_inflight) c->notify_all();
}

void nnfft_server_s::release_resident_if_evicted(Resident *rs)
{
    if (!rs->evict_when_idle || rs->busy || rs->building || !rs->waiting.empty()) return;
    drop_resident(rs);
}

void nnfft_server_s::completion_loop(int si)
{
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_inflight[si]->wait(lk, [&] { return !inflight[si].empty() || exec_done; });
        if (inflight[si].empty()) break;   // the executor has finished and this stream is drained
        Group *g = inflight[si].front();
        lk.unlock();
        hipError_t e = hipSuccess;
        if (g->ev) {
            e = hipEventSynchronize(g->ev);
            (void)hipEventDestroy(g->ev);
        }
        lk.lock();
        inflight[si].pop_front();
        groups_inflight--;
        cv_ready.notify_all();
        for (Req *q : g->reqs) {
            nnfft_status status = (nnfft_status)q->out.status;
            std::string err = q->out.message;
            if (status == NNFFT_OK && e != hipSuccess) {
                status = NNFFT_ERR_DEVICE;
                err = hipGetErrorString(e);
            }
            Resident *rs = q->res;
            if (rs) {
                rs->busy = false;
                rs->last_use = ++use_clock;
                if (!rs->waiting.empty()) {   // the next request of this key
                    Req *w = rs->waiting.front();
                    rs->waiting.pop_front();
                    rs->busy = true;
                    w->plan = rs->plan;
                    w->splan = rs->splan;
                    w->out.admit_ms = now_ms();
                    ready.push_back(w);
                    cv_ready.notify_one();
                }
            } else {
                active_bytes -= q->out.footprint_bytes;
                if (q->plan) nnfft_destroy(q->plan);
                if (q->splan) sinc_destroy(q->splan);
                q->plan = nullptr;
                q->splan = nullptr;
            }
            finish(q, status, err);
            if (rs) release_resident_if_evicted(rs);
        }
        delete g;
        cv_space.notify_all();
    }
}

extern "C" {

nnfft_status nnfft_server_create(nnfft_server_t *out, const nnfft_server_config_t *cfg)
{
    if (!out) return fail(NNFFT_ERR_ARG, "null server pointer");
    *out = nullptr;
    nnfft_server_config_t c{};
    if (cfg) c = *cfg;
    if (c.hbm_budget_bytes < 0 || c.planner_threads < 0 || c.streams < 0 || c.max_batch < 0 ||
        c.max_batch > kMaxBatch || c.planner_threads > 64 || c.streams > 16)
        return fail(NNFFT_ERR_ARG, "bad server configuration");
    if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = (int64_t)8 << 30;
    if (c.planner_threads == 0) c.planner_threads = 8;
    if (c.streams == 0) c.streams = 2;
    if (c.max_batch == 0) c.max_batch = kMaxBatch;
    nnfft_server_s *S = new (std::nothrow) nnfft_server_s();
    if (!S) return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    S->cfg = c;
    S->t0 = std::chrono::steady_clock::now();
    if (hipMalloc(&S->arena_mem, (size_t)c.hbm_budget_bytes) != hipSuccess) {
        delete S;
        return fail(NNFFT_ERR_NOMEM, "arena of " + std::to_string(c.hbm_budget_bytes) + " bytes");
    }
    S->arena.base = static_cast<char *>(S->arena_mem);
    S->arena.reset((size_t)c.hbm_budget_bytes);
    S->mem = DevMem{arena_alloc, arena_release, &S->arena};
    for (int i = 0; i < c.streams; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : S->streams) (void)hipStreamDestroy(t);
            (void)hipFree(S->arena_mem);
            delete S;
            return fail(NNFFT_ERR_DEVICE, "stream creation failed");
        }
        S->streams.push_back(s);
        S->inflight.emplace_back();
        S->cv_inflight.emplace_back(new std::condition_variable());
    }
    S->st.arena_bytes = c.hbm_budget_bytes;
    for (int i = 0; i < c.planner_threads; ++i) S->planners.emplace_back([S] { S->planner_loop(); });
    S->executor = std::thread([S] { S->executor_loop(); });
    for (int i = 0; i < c.streams; ++i) S->completers.emplace_back([S, i] { S->completion_loop(i); });
    *out = S;
    return NNFFT_OK;
}

nnfft_status nnfft_server_submit(nnfft_server_t s, const nnfft_request_t *req, uint64_t *ticket)
{
    if (!s || !req || !ticket) return fail(NNFFT_ERR_ARG, "null argument");
    if (req->kind != NNFFT_REQ_NNFFT && req->kind != NNFFT_REQ_SINC) return fail(NNFFT_ERR_ARG, "unknown request kind");
    if (!req->v || !req->x || !req->f || !req->y) return fail(NNFFT_ERR_ARG, "null device array in the request");
    Req *q = new (std::nothrow) Req();
    if (!q) return fail(NNFFT_ERR_NOMEM, "host allocation failed");
    q->r = *req;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stopping) {
        delete q;
        return fail(NNFFT_ERR_BUSY, "server is shutting down");
    }
    q->ticket = s->next_ticket++;
    q->out.submit_ms = s->now_ms();
    s->tickets[q->ticket] = q;
    s->pending.push_back(q);
    s->st.submitted++;
    s->cv_pending.notify_one();
    *ticket = q->ticket;
    return NNFFT_OK;
}

static nnfft_status take_result(nnfft_server_t s, uint64_t ticket, nnfft_result_t *res, bool block)
{
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(NNFFT_ERR_ARG, "unknown ticket");
    Req *q = it->second;
    if (!q->done) {
        if (!block) return NNFFT_ERR_BUSY;
        s->cv_done.wait(lk, [&] { return q->done; });
    }
    if (res) *res = q->out;
    s->tickets.erase(ticket);
    delete q;
    return NNFFT_OK;
}

nnfft_status nnfft_server_wait(nnfft_server_t s, uint64_t ticket, nnfft_result_t *res)
{
    if (!s) return fail(NNFFT_ERR_ARG, "null server");
    return take_result(s, ticket, res, true);
}

nnfft_status nnfft_server_poll(nnfft_server_t s, uint64_t ticket, nnfft_result_t *res)
{
    if (!s) return fail(NNFFT_ERR_ARG, "null server");
    return take_result(s, ticket, res, false);
}

nnfft_status nnfft_server_stats(nnfft_server_t s, nnfft_server_stats_t *out)
{
    if (!s || !out) return fail(NNFFT_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->st;
    out->arena_in_use = (int64_t)s->arena.in_use();
    out->arena_peak = (int64_t)s->arena.peak();
    out->resident_plans = (int64_t)s->residents.size();
    return NNFFT_OK;
}

nnfft_status nnfft_server_evict(nnfft_server_t s, uint64_t plan_key)
{
    if (!s) return fail(NNFFT_ERR_ARG, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->residents.find(plan_key);
    if (it == s->residents.end()) return fail(NNFFT_ERR_ARG, "no resident plan with this key");
    Resident *rs = it->second;
    rs->evict_when_idle = true;
    s->release_resident_if_evicted(rs);
    return NNFFT_OK;
}

nnfft_status nnfft_server_destroy(nnfft_server_t s)
{
    if (!s) return fail(NNFFT_ERR_ARG, "null server");
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stopping = true;
        s->cv_pending.notify_all();
        s->cv_ready.notify_all();
        s->cv_space.notify_all();
    }
    for (auto &t : s->planners) t.join();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->cv_ready.notify_all();
    }
    s->executor.join();
    for (auto &t : s->completers) t.join();
    {
        std::lock_guard<std::mutex> g(s->mu);
        while (!s->residents.empty()) s->drop_resident(s->residents.begin()->second);
    }
    for (auto &kv : s->tickets) delete kv.second;   // results never collected
    for (hipStream_t t : s->streams) (void)hipStreamDestroy(t);
    (void)hipFree(s->arena_mem);
    delete s;
    return NNFFT_OK;
}

}  // extern "C"
