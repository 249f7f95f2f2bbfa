/*
 * nnfft_serve.h - request serving layer of the MI355X NNFFT library.
 *
 * A server owns one device arena (its HBM budget) and runs NNFFT (Algorithm
 * 2.2) and fast sinc (Algorithm 6.1) requests with continuous batching:
 *   - planner threads copy each request's nodes to the host, build its plan
 *     (Algorithm 2.2 step 0) and admit it when its exact device footprint
 *     fits in the arena; a plan that does not fit waits until finished
 *     requests release space;
 *   - an executor thread takes every admitted request that is ready (up to
 *     max_batch) and issues them as one launch group, using the batched
 *     launches of nnfft_exec_batch (one launch per stage for all plans of a
 *     precision), on one of several streams, without waiting for earlier
 *     groups, so groups on different streams overlap on the device;
 *   - one completion thread per stream waits for its groups, stamps the
 *     results and returns the plans' memory to the arena (no hipFree while
 *     serving).
 * Plans with a nonzero plan_key stay resident after their request and serve
 * later requests with the same key (the caller promises the same nodes);
 * resident plans that are idle are evicted, least recently used first, when
 * a new plan needs their space.
 *
 * Results are those of nnfft_exec / sinc_exec on the same plan (sinc
 * requests: in the two-kernel form, sinc_middle(p, 0)): every request's
 * output is bitwise the same alone or in any mix.
 *
 * Conventions: as in nnfft.h.  The request's device arrays (v, x, f, y) are
 * the caller's; they must hold their data before nnfft_server_submit (the
 * server's streams are not ordered after the caller's) and stay valid until
 * the request's result has been returned by nnfft_server_wait or
 * nnfft_server_poll.  All functions are thread-safe.
 */
#ifndef NNFFT_SERVE_H
#define NNFFT_SERVE_H

#include <stdint.h>

#include "nnfft.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnfft_server_s *nnfft_server_t;

typedef enum {
    NNFFT_REQ_NNFFT = 0,   /* y[M2] = NNFFT of f[M1] (Algorithm 2.2)                    */
    NNFFT_REQ_SINC = 1     /* y[M2] = fast sinc transform of f[M1] (Algorithm 6.1)       */
} nnfft_request_kind;

typedef struct {
    int32_t kind;          /* nnfft_request_kind                                         */
    int32_t precision;     /* nnfft_precision                                            */
    int64_t N;             /* bandwidth                                                  */
    int64_t M1, M2;        /* node counts (sinc: L1, L2)                                 */
    double sigma1, sigma2;
    int32_t m1, m2;
    int32_t quad;          /* sinc: sinc_quad                                            */
    int32_t window;        /* NNFFT: nnfft_window (0: sinh); sinc requests use sinh      */
    int64_t n_quad;        /* sinc: quadrature size                                      */
    const double *v;       /* device FP64 [M1]: frequencies v_k (sinc: a_k)              */
    const double *x;       /* device FP64 [M2]: spatial nodes x_j (sinc: b_l)            */
    const void *f;         /* device [M1] c64 (FP32 plans) or c128 (FP64 plans)          */
    void *y;               /* device [M2], same type                                     */
    uint64_t plan_key;     /* 0: a plan for this request only; else kept under this key  */
} nnfft_request_t;

typedef struct {
    int32_t status;           /* nnfft_status of the request                             */
    int32_t group_size;       /* requests in the launch group that carried it            */
    int64_t footprint_bytes;  /* device bytes of its plan                                */
    int32_t plan_reused;      /* 1 if a resident plan served it                          */
    int32_t reserved;
    double submit_ms;         /* server clock (ms since creation): submitted             */
    double plan_ms;           /* a planner thread took it up                             */
    double admit_ms;          /* plan built and admitted into the arena                  */
    double launch_ms;         /* launch group issued                                     */
    double done_ms;           /* completion observed                                     */
    char message[160];        /* error description when status != NNFFT_OK               */
} nnfft_result_t;

typedef struct {
    int64_t hbm_budget_bytes; /* arena size (0: 8 GiB)                                   */
    int32_t planner_threads;  /* host threads building plans (0: 8)                      */
    int32_t streams;          /* execution streams (0: 2)                                */
    int32_t max_batch;        /* requests per launch group, 1..32 (0: 32)                */
    int32_t reserved;
} nnfft_server_config_t;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t groups;           /* launch groups issued                                    */
    int64_t admission_waits;  /* times a built plan waited for arena space               */
    int64_t evictions;        /* resident plans evicted for space                        */
    int64_t arena_bytes, arena_in_use, arena_peak;
    int64_t resident_plans;
} nnfft_server_stats_t;

/*
 * Creates a server: allocates the arena, the streams (default priority,
 * non-blocking) and the threads.  cfg may be NULL (defaults).
 * Errors: ARG (negative sizes, max_batch > 32), NOMEM (arena), DEVICE.
 */
nnfft_status nnfft_server_create(nnfft_server_t *out, const nnfft_server_config_t *cfg);

/*
 * Queues a request (copied) and returns its ticket.  Parameter errors of the
 * plan (as nnfft_plan / sinc_plan) and arena overflow (a plan larger than
 * the whole arena: NOMEM) are reported in the request's result.
 * Errors here: ARG (null arguments, unknown kind), BUSY (server shutting down).
 */
nnfft_status nnfft_server_submit(nnfft_server_t s, const nnfft_request_t *req, uint64_t *ticket);

/* Blocks until the request is finished and returns its result; the ticket is
 * then released.  Errors: ARG (unknown ticket). */
nnfft_status nnfft_server_wait(nnfft_server_t s, uint64_t ticket, nnfft_result_t *res);

/* Non-blocking: NNFFT_OK and the result (ticket released) if finished, else
 * NNFFT_ERR_BUSY.  Errors: ARG (unknown ticket). */
nnfft_status nnfft_server_poll(nnfft_server_t s, uint64_t ticket, nnfft_result_t *res);

nnfft_status nnfft_server_stats(nnfft_server_t s, nnfft_server_stats_t *out);

/* Drops the resident plan of plan_key once it is idle.  Errors: ARG (no such key). */
nnfft_status nnfft_server_evict(nnfft_server_t s, uint64_t plan_key);

/* Finishes every submitted request, then frees plans, arena, streams, threads. */
nnfft_status nnfft_server_destroy(nnfft_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* NNFFT_SERVE_H */
