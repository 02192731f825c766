/*
 * rp.h -- C-ABI of the MI355X (gfx950) RP-Tuning library.
 *
 * Paper: "Prune, Don't Rebuild: Efficiently Tuning alpha-Reachable Graphs for
 * Nearest Neighbor Search" (arXiv 2602.08097).
 *
 * RP-Tuning (Section 3) re-runs RobustPrune (Algorithm 1) on the existing
 * out-list of every vertex of a base graph at a new alpha (and a degree bound
 * R), instead of rebuilding the index.  GreedySearch (Algorithm 2) scores the
 * pruned graphs.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller, unless the
 *   argument says "host".  The library never frees caller memory.
 * - Work is enqueued on the HIP stream passed as `stream` (a hipStream_t; NULL
 *   is the default stream) and is ordered with the caller's other work on that
 *   stream.  Calls return once the work is enqueued, except where noted.
 * - Argument errors are detected on the host and returned before any launch.
 *   A HIP launch failure returns RP_EDEVICE.  No exception or abort crosses
 *   the ABI.  rp_last_error() describes the last failure of the calling thread.
 * - Distances are squared Euclidean (every experiment of Section 4 uses
 *   Euclidean distance; both sides of every comparison are non-negative, so
 *   comparing squares is equivalent):
 *     uint8 points  : exact integers;
 *     float32 points: the canonical FP64 value
 *                       acc = 0; for k in 0..d-1:
 *                         t = (double)a[k] - (double)b[k]; acc = fma(t, t, acc)
 * - alpha = num/den, num >= den >= 1, both <= 65535.  The pruning condition of
 *   Algorithm 1, alpha * D(p*, p') <= D(p, p'), is evaluated as
 *     uint8  : num^2 * S(p*, p') <= den^2 * S(p, p')          (exact integers)
 *     float32: fl(num^2 * S(p*, p')) <= fl(den^2 * S(p, p'))  (FP64, one rounding
 *                                                              per product)
 * - Ties in every argmin, truncation and top-k are broken by (S, id), smallest
 *   first, so every result is unique and bit-reproducible.
 * - A graph's adjacency is a fixed-stride n x r_max int32 array: row p holds
 *   deg[p] ids (0 <= deg[p] <= r_max), the rest of the row is ignored.  A list
 *   may contain p itself and repeated ids; RobustPrune drops both
 *   (V <- (V u N_out(p)) \ {p} in Algorithm 1).
 */
#ifndef RP_H
#define RP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rp_graph* rp_graph_t; /* opaque, library-owned */

typedef enum { RP_U8 = 1, RP_F32 = 2 } rp_dtype;

typedef struct {
  int32_t num;
  int32_t den;
} rp_alpha; /* alpha = num / den */

typedef enum {
  RP_OK = 0,
  RP_EINVAL = 1,  /* invalid argument (null pointer, bad size, alpha < 1, k > L, ...) */
  RP_ERANGE = 2,  /* an id or degree in the adjacency is out of range */
  RP_ENOMEM = 3,  /* device allocation failed */
  RP_EDEVICE = 4, /* a HIP call or kernel launch failed */
  RP_ESTATE = 5   /* the graph handle is unusable (e.g. freed base) */
} rp_status;

/* Device-side counters of a graph handle (see rp_read_counters). */
typedef struct {
  int64_t nodes;      /* vertex-prunes enqueued (vertices x outputs)            */
  int64_t rechecks;   /* pairs re-evaluated in canonical FP64 (float32 data)    */
} rp_counters;

/*
 * rp_load_graph -- register a point set and its base graph (the input of
 * RP-Tuning, Section 3).
 *   points : n x d row-major, uint8 (dtype RP_U8) or float32 (RP_F32).
 *   n      : 1 <= n < 2^31.   d: 1 <= d <= 4096.
 *   nbr    : n x r_max int32 out-lists, deg: n int32 out-degrees.
 *   r_max  : 1 <= r_max <= 256.
 *   start  : start vertex s of GreedySearch (Algorithm 2), 0 <= start < n.
 * The library BORROWS points, nbr and deg until rp_free_graph: they must stay
 * valid and unmodified.  The adjacency is validated on the device; this call
 * is synchronous (it returns once everything it enqueued on `stream` is done,
 * so the handle may be used from any stream) and returns RP_ERANGE if any
 * degree is outside [0, r_max] or any listed id outside [0, n), RP_EINVAL if
 * a float32 point has a NaN or infinite coordinate.  On success *out receives a new
 * handle.  The handle owns one device array per point (|x|^2 for uint8 points,
 * max_k |x_k| for float32 ones) and, for float32 graphs that the batched
 * kernel serves (see rp_graph_derive), one byte per vertex: the scale exponent of the vertex's frame, computed from
 * its list here so that sweeps need not read it per candidate.
 */
rp_status rp_load_graph(const void* points, int32_t dtype, int64_t n, int32_t d,
                        const int32_t* nbr, const int32_t* deg, int32_t r_max,
                        int32_t start, void* stream, rp_graph_t* out);

/*
 * rp_graph_derive -- a handle on another graph over the same points (for
 * example a pruned graph, to search it).  Shares base's points and start
 * vertex; borrows nbr/deg like rp_load_graph and validates them the same way
 * (synchronous, as rp_load_graph), and computes its own per-vertex frame
 * exponents for float32 graphs that the batched kernel serves (r_max <= 128,
 * 97..128 only with d % 4 == 0 and 16-byte aligned points, and one vertex's
 * LDS within the device's LDS per workgroup: every d on gfx950; n bytes).  base must outlive the derived
 * handle.
 */
rp_status rp_graph_derive(rp_graph_t base, const int32_t* nbr, const int32_t* deg,
                          int32_t r_max, void* stream, rp_graph_t* out);

/*
 * rp_prune -- RP-Tuning of the whole graph at one (alpha, R): for every
 * vertex p, RobustPrune(p, N_out(p), alpha, R) (Algorithm 1; Section 3 with a
 * finite degree bound).  R >= 1; R >= deg means no bound in effect.
 *   out_nbr: n x R int32, row p receives the kept ids in the order Algorithm 1
 *            adds them (ascending (S(p, .), id)), padded with -1.
 *   out_deg: n int32, the kept counts.
 * Outputs must not alias the graph's arrays.  Uses the batched kernels.
 */
rp_status rp_prune(rp_graph_t g, rp_alpha alpha, int32_t R, int32_t* out_nbr,
                   int32_t* out_deg, void* stream);

/*
 * rp_prune_sweep -- RP-Tuning at several (alpha, R) from one pass over the
 * graph: n_a alphas x n_R degree bounds, output index o = ia * n_R + iR.
 *   alphas : host array of n_a (1 <= n_a <= 8).
 *   Rs     : host array of n_R (1 <= n_R <= 4), each >= 1.
 *   out_nbr: host array of n_a*n_R device pointers, output o is n x Rs[iR].
 *   out_deg: host array of n_a*n_R device pointers, each n int32.
 * Every output equals rp_prune at its own (alpha, R).
 */
rp_status rp_prune_sweep(rp_graph_t g, const rp_alpha* alphas, int32_t n_a,
                         const int32_t* Rs, int32_t n_R, int32_t* const* out_nbr,
                         int32_t* const* out_deg, void* stream);

/*
 * rp_prune_sweep_unsorted -- RP-Tuning with UnsortedRobustPrune (Section 3,
 * defined after RP-Tuning; the setting of Theorem 3.1): Algorithm 1 with p*
 * taken as an arbitrary remaining out-neighbour of p instead of the argmin
 * of D(p, .).  "Arbitrary" is read as the first remaining candidate in the
 * order the list stores them (a repeated id counts at its first occurrence;
 * p itself is dropped).  Arguments, output layout and errors as
 * rp_prune_sweep; each output row holds the kept ids in that list order.
 */
rp_status rp_prune_sweep_unsorted(rp_graph_t g, const rp_alpha* alphas, int32_t n_a,
                                  const int32_t* Rs, int32_t n_R, int32_t* const* out_nbr,
                                  int32_t* const* out_deg, void* stream);

/*
 * rp_prune_plain -- the same result as rp_prune from the plain baseline
 * kernel: one workgroup per vertex, direct-difference distances evaluated
 * lazily (FP32 with an FP64 recheck near the threshold for float32 data,
 * exact integers for uint8), no shared gather across alphas.  Kept as the
 * comparison point for the batched kernels.
 */
rp_status rp_prune_plain(rp_graph_t g, rp_alpha alpha, int32_t R, int32_t* out_nbr,
                         int32_t* out_deg, void* stream);

/*
 * rp_search -- GreedySearch(s, q, k, L) (Algorithm 2) from the graph's start
 * vertex for nq queries.
 *   queries : nq x d, same dtype as the points.   1 <= k <= L <= 1024.
 *   out_ids : nq x k int32, the k closest ids of the final list by (S, id),
 *             padded with -1 when the list holds fewer than k.
 *   out_dist: nq x k FP64 squared distances (nullable; -1 where padded).
 *   out_hops: nq int32, |V| = the number of expanded vertices (nullable).
 */
rp_status rp_search(rp_graph_t g, const void* queries, int64_t nq, int32_t k, int32_t L,
                    int32_t* out_ids, double* out_dist, int32_t* out_hops, void* stream);

/*
 * rp_knn_u8 -- exact K nearest neighbours of uint8 points: the input lists of
 * the base graphs.  The experiments of Section 4 start from a Vamana index
 * built by RobustPrune (Algorithm 1) over candidate lists; here the candidate
 * list of a point is its K nearest points, and the base graph is RobustPrune
 * of that list (rp_load_graph on the lists, then rp_prune).
 *   points   : n x d uint8, row-major, 16-byte aligned; d a multiple of 16 in
 *              [16, 256]; 1 <= n < 2^31.
 *   query_ids: nq point ids whose lists are computed (nullable: points
 *              0 .. nq - 1).
 *   cand_ids : nc distinct point ids the lists are drawn from (nullable:
 *              points 0 .. nc - 1).
 *   K        : 1 <= K <= 128.
 *   out_ids  : nq x K int32; row i lists the K candidates nearest to
 *              query_ids[i] in ascending (S, id) order, S the exact squared
 *              distance, the query itself excluded; -1 pads a row when fewer
 *              candidates exist.
 * A query or candidate id outside [0, n) is ignored (the query's row is all
 * -1; the candidate is never listed).  All arrays are device arrays.  When
 * the candidates are split across workgroups (few queries), the partial
 * lists take a workspace of slices x nq x 1 KiB, allocated and freed in
 * stream order on `stream` (RP_ENOMEM if that fails).
 */
rp_status rp_knn_u8(const uint8_t* points, int64_t n, int32_t d, const int32_t* query_ids,
                    int64_t nq, const int32_t* cand_ids, int64_t nc, int32_t K,
                    int32_t* out_ids, void* stream);

/*
 * rp_knn_u8_noalloc -- rp_knn_u8 for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, hosts that
 * forbid allocation.  It calls no allocator.  When the candidates are split
 * into slices, the partial lists go to a fixed workspace of the library:
 * 64 MiB of device memory per GPU, held until the process ends.
 *   slices: 1..64 candidate slices (1 needs no workspace; more give few
 *           queries more parallelism), or 0 for the library's choice reduced
 *           to fit the workspace.  A call whose slices x nq x 1 KiB exceeds
 *           64 MiB returns RP_EINVAL before any launch.
 * Other arguments, outputs and errors as rp_knn_u8; the outputs equal
 * rp_knn_u8's for every slice count.  Every call on a GPU shares that GPU's
 * workspace, so calls that overlap in time on one GPU (different streams or
 * threads without ordering) race; calls ordered on one stream do not.  The
 * kernels write every partial list before reading it, so nothing left by an
 * earlier call is read.
 */
rp_status rp_knn_u8_noalloc(const uint8_t* points, int64_t n, int32_t d,
                            const int32_t* query_ids, int64_t nq, const int32_t* cand_ids,
                            int64_t nc, int32_t K, int32_t slices, int32_t* out_ids,
                            void* stream);

/*
 * rp_read_counters -- copy the graph's device counters to *out (host) and,
 * if reset != 0, zero them.  Synchronises `stream`.
 */
rp_status rp_read_counters(rp_graph_t g, rp_counters* out, int32_t reset, void* stream);

/*
 * Captured sweeps.  rp_plan_sweep records the launches that rp_prune_sweep
 * would enqueue for these arguments into a HIP graph (stream capture on
 * `stream`, nothing runs) and instantiates it; rp_plan_launch replays it on
 * any stream, with no host-side work beyond one graph launch.  The graph
 * handle and every output array must outlive the plan.  The outputs of a
 * replay are identical to those of the call it captured.
 */
typedef struct rp_plan* rp_plan_t; /* opaque, library-owned */

rp_status rp_plan_sweep(rp_graph_t g, const rp_alpha* alphas, int32_t n_a, const int32_t* Rs,
                        int32_t n_R, int32_t* const* out_nbr, int32_t* const* out_deg,
                        void* stream, rp_plan_t* out);
rp_status rp_plan_launch(rp_plan_t p, void* stream);
void rp_plan_free(rp_plan_t p); /* NULL is ignored */

/*
 * Launch tuning.  The batched kernels run one vertex per wavefront and pack
 * `waves` vertices into each workgroup (1, 2, 4 or 8, within the device's
 * LDS per workgroup, 160 KiB on gfx950).  rp_autotune_sweep times the sweep of these arguments for
 * every candidate (one warm-up and three timed launches each, HIP events on
 * `stream`), keeps the fastest for this graph shape (dtype, d, r_max) and
 * sweep shape (n_a, n_R) for the rest of the process, and returns it in
 * *waves (host); ms (host, 4 entries, nullable) receives each candidate's
 * median time, 0 for a candidate that does not fit.  The outputs hold the
 * sweep's result afterwards.  Synchronises `stream`.  Graphs that take the
 * plain kernel have nothing to tune (*waves = 1).
 * rp_tune_set records a choice (for instance from a cache of earlier
 * tunings); waves = 0 forgets it.  rp_tune_get returns the current choice
 * (0 = untuned, which launches 1).
 */
rp_status rp_autotune_sweep(rp_graph_t g, const rp_alpha* alphas, int32_t n_a, const int32_t* Rs,
                            int32_t n_R, int32_t* const* out_nbr, int32_t* const* out_deg,
                            void* stream, int32_t* waves, float* ms);
rp_status rp_tune_set(rp_graph_t g, int32_t n_a, int32_t n_R, int32_t waves);
rp_status rp_tune_get(rp_graph_t g, int32_t n_a, int32_t n_R, int32_t* waves);

/*
 * rp_gram_error -- measured error of the float32 batched kernel's approximate
 * candidate distances.  For each listed vertex p (nodes: device int32, each in
 * [0, n)), the kernel's own S~(i, j) for every pair of listed candidates is
 * compared with the canonical FP64 S(i, j):
 *   out[0] = max |S~ - S| / S,  out[1] = mean of the same,  out[2] = pairs,
 *   out[3] = max |S~ - S| / E_j, where E_j is the bound the kernel proves and
 *            uses to decide which pairs to recompute in FP64 (<= 1 means
 *            every approximate decision was safe).
 * out is a host array of 4 doubles.  Float32 graphs that the batched kernel
 * serves only (see rp_graph_derive; uint8 distances are exact integers).  Synchronises `stream`.
 */
rp_status rp_gram_error(rp_graph_t g, const int32_t* nodes, int64_t n_nodes, double* out,
                        void* stream);

/*
 * rp_build_slow -- the "slow preprocessing" construction (Section 2.1):
 * RobustPrune(p, P \ {p}, alpha, R) (Algorithm 1) for every point p of the
 * point set (n x d, dtype RP_U8 or RP_F32, finite coordinates).  With
 * R >= n - 1 the graph is alpha-reachable (Lemma 2.2); RP-Tuning (Section 3)
 * is measured against rebuilding it at the new alpha.  O(n^2) work per point.
 *   out_nbr: n x R int32, row p the kept ids in the order Algorithm 1 adds
 *            them (ascending (S(p, .), id)), -1 padded; out_deg: n int32.
 * Distances and the alpha test as everywhere in this header.  Coordinates
 * are not checked here: a NaN or infinity gives unspecified lists (the call
 * still ends).  A workspace of at most 1 GiB is allocated and freed in stream
 * order on `stream`; the call returns once the work is enqueued.
 */
rp_status rp_build_slow(const void* points, int32_t dtype, int64_t n, int32_t d, rp_alpha alpha,
                        int32_t R, int32_t* out_nbr, int32_t* out_deg, void* stream);

/*
 * rp_f32_band -- the rounding band of the float32 batched kernel for points of
 * dimension d (1 <= d <= 4096): out (host, 4 doubles) receives c1, c2, c3 of
 *   |S~(i, j) - S(i, j) 2^2e| <= c1 s + c2 sqrt(s) + c3,   s = S(p, j) 2^2e,
 * for every pair of candidates i before j of a vertex p, where S~ is the
 * kernel's split-FP16 matrix-unit value in the vertex's frame scaled by 2^e
 * and S the canonical FP64 value.  A pair is decided from S~ only when the
 * alpha test holds or fails by more than this band; otherwise S is recomputed.
 * out[3] is the number of dimensions the kernel sums in one accumulator
 * before adding it to the running total (d when it does not restart).
 * Host only (no device work).
 */
rp_status rp_f32_band(int32_t d, double* out);

/* rp_free_graph -- release a handle (NULL is ignored).  Synchronises the
 * device; the caller's arrays are not freed. */
void rp_free_graph(rp_graph_t g);

/* rp_last_error -- message of the calling thread's last failure ("" if none). */
const char* rp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RP_H */
