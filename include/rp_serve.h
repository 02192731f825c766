/*
 * rp_serve.h -- request loop over one resident base graph (C-ABI).
 *
 * RP-Tuning (Section 3 of arXiv 2602.08097) makes a pruned graph at any alpha
 * (and degree bound R) from the resident base graph with one RobustPrune pass
 * per vertex (Algorithm 1), and GreedySearch (Algorithm 2) answers queries on
 * any graph.  A server keeps the base graph and the pruned graphs it made
 * resident in device memory and serves a stream of two request types:
 *
 *   PRUNE(alpha, R)                    make the pruned graph resident (and,
 *                                      if out_nbr/out_deg are given, copy it
 *                                      there, n x R and n int32);
 *   QUERY(graph, queries, nq, k, L)    GreedySearch of nq queries on the base
 *                                      graph (alpha = {0, 0}) or on the pruned
 *                                      graph (alpha, R), which is made
 *                                      resident first if it is not.
 *
 * Scheduling (one worker thread per server):
 * - Continuous batching: whenever a stream has room, every request that has
 *   arrived by then is eligible.  Prune requests with the same R are merged
 *   into one sweep launch of up to 8 alphas (one gather of each vertex's rows
 *   for all of them); queries with the same (graph, k, L) are merged into one
 *   search launch of up to max_query_batch queries, each query with its own
 *   row and outputs.
 * - Overlap: sweeps run on stream 0, query batches on streams 1..n_streams-1;
 *   one launch per stream is in flight at a time, so the next batch is formed
 *   from whatever arrived meanwhile.
 * - Memory: pruned graphs live in one arena of budget_bytes allocated at
 *   creation (each takes n (R + 1) 4 bytes, rounded up to 256).  A graph is
 *   admitted when it fits after evicting least-recently-used graphs that no
 *   launch uses; otherwise its requests wait.  The base graph is never evicted.
 * - FIFO modes, the baselines the batching is compared with: one request at a
 *   time in arrival order, no merging, no overlap; fifo = 1 prunes with the
 *   batched kernel (one alpha per launch), fifo = 2 with the plain
 *   one-workgroup-per-vertex kernel.
 *
 * Results do not depend on scheduling: a request's outputs are identical
 * whether it runs alone or in any mix (every kernel is deterministic and
 * computes each vertex and each query independently).
 *
 * All pointers in rp_request are DEVICE pointers owned by the caller and must
 * stay valid until the request completes.  The server's streams are not
 * ordered after the caller's: a request's input rows must be complete when it
 * is submitted (synchronise the stream that produced them first).  Calls are
 * thread-safe.
 */
#ifndef RP_SERVE_H
#define RP_SERVE_H

#include <stdint.h>

#include "rp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rp_server* rp_server_t; /* opaque, library-owned */

typedef enum { RP_REQ_PRUNE = 1, RP_REQ_QUERY = 2 } rp_request_type;

typedef struct {
  int32_t type;         /* rp_request_type */
  rp_alpha alpha;       /* PRUNE: alpha; QUERY: target graph, {0, 0} = the base graph */
  int32_t R;            /* degree bound of the pruned graph (1 <= R <= the base r_max) */
  const void* queries;  /* QUERY: nq x d rows, the points' dtype */
  int64_t nq;
  int32_t k, L;         /* QUERY: 1 <= k <= L <= 1024 */
  int32_t* out_ids;     /* QUERY: nq x k; PRUNE: n x R copy of the graph (nullable) */
  double* out_dist;     /* QUERY: nq x k FP64 (nullable) */
  int32_t* out_hops;    /* QUERY: nq (nullable); PRUNE: n out-degrees (nullable) */
  int64_t tag;          /* caller's id, returned in the completion */
} rp_request;

typedef struct {
  int64_t tag;
  int32_t status;       /* rp_status of the request */
  int32_t batch;        /* requests in the launch that served it (1 in FIFO mode) */
  double t_submit;      /* seconds on the host's monotonic clock */
  double t_start;       /* launch enqueued */
  double t_done;        /* completion observed */
} rp_completion;

typedef struct {
  int64_t sweeps;            /* prune launches */
  int64_t swept_alphas;      /* alphas over all sweeps */
  int64_t searches;          /* search launches */
  int64_t searched_queries;  /* queries over all search launches */
  int64_t evictions;
  int64_t resident_graphs;   /* pruned graphs resident now */
  int64_t resident_bytes;    /* arena bytes in use now */
} rp_server_stats;

/*
 * rp_server_create -- start a server over `base` (uint8 or float32 points).
 *   budget_bytes   : arena for pruned graphs (device memory, allocated here).
 *   n_streams      : 2..8 (one sweep stream, the rest for query batches).
 *   max_query_batch: queries per search launch, 1..65536.
 *   fifo           : 0 batching; 1 or 2 the one-request-at-a-time baselines.
 * The base handle must outlive the server.
 */
rp_status rp_server_create(rp_graph_t base, int64_t budget_bytes, int32_t n_streams,
                           int32_t max_query_batch, int32_t fifo, rp_server_t* out);

/* rp_server_submit -- enqueue one request (non-blocking).  Argument errors
 * are returned here and the request is not enqueued. */
rp_status rp_server_submit(rp_server_t s, const rp_request* req);

/* rp_server_poll -- move up to `max` completions to out (host array), waiting
 * up to wait_ms milliseconds for the first one.  Returns the number moved,
 * or -1 on a null argument. */
int32_t rp_server_poll(rp_server_t s, rp_completion* out, int32_t max, int32_t wait_ms);

/*
 * rp_server_replay -- submit reqs[i] at arrival_s[i] seconds after the call
 * (ascending times; host arrays) from the calling thread, wait for every
 * completion and store completion i in out[i] (host array).  Times are kept
 * by the library, so the caller's language adds no jitter.
 */
rp_status rp_server_replay(rp_server_t s, const rp_request* reqs, const double* arrival_s,
                           int32_t n, rp_completion* out);

rp_status rp_server_stats_get(rp_server_t s, rp_server_stats* out);

/* rp_server_destroy -- finish every submitted request, then free the arena
 * and the streams (NULL is ignored). */
void rp_server_destroy(rp_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* RP_SERVE_H */
