/*
 * rpo.h -- plain, single-threaded CPU oracle for RP-Tuning (RobustPrune over
 * existing out-lists) and GreedySearch.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this library; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no source, header or helper with the HIP
 * library and is built by plain gcc with -ffp-contract=off.
 *
 * Paper: "Prune, Don't Rebuild: Efficiently Tuning alpha-Reachable Graphs for
 * Nearest Neighbor Search" (arXiv 2602.08097).
 *   RobustPrune            -- Algorithm 1 (Section 2.1)
 *   RP-Tuning              -- Section 3, first paragraph
 *   GreedySearch           -- Algorithm 2 (Section 2.1)
 *   alpha-reachability     -- Definition 2.1
 *
 * Distances.  The paper works with a metric D; every experiment uses
 * Euclidean distance (Section 4.1).  Both sides of every comparison are
 * non-negative, so the oracle compares squared distances S = D^2:
 *   alpha * D(a,b) <= D(c,e)   <=>   num^2 * S(a,b) <= den^2 * S(c,e)
 * with alpha = num/den given as a rational.
 *   uint8 data   : S is the exact integer sum of squared differences (int64).
 *   float32 data : S is the canonical FP64 value
 *                    acc = 0; for k = 0..d-1: t = (double)a_k - (double)b_k;
 *                                              acc = fma(t, t, acc)
 *                  and the alpha test is fl(num^2 * S1) <= fl(den^2 * S2),
 *                  each product rounded once.
 * Ties in every argmin / truncation / top-k are broken by (S, id), smallest
 * first.
 *
 * Return codes: >= 0 success (a count), RPO_EINVAL (-1) bad argument,
 * RPO_ERANGE (-2) an id outside [0, n).
 */
#ifndef RPO_H
#define RPO_H
#include <stdint.h>

#define RPO_U8 1
#define RPO_F32 2
#define RPO_EINVAL (-1)
#define RPO_ERANGE (-2)

#ifdef __cplusplus
extern "C" {
#endif

/* Squared distances: exact int64 for uint8 rows, canonical FP64 for float32. */
int64_t rpo_sqdist_u8(const uint8_t* a, const uint8_t* b, int32_t d);
double rpo_sqdist_f32(const float* a, const float* b, int32_t d);

/*
 * RobustPrune(p, V, alpha = num/den, R) on a point set X (n x d, row-major,
 * dtype RPO_U8 or RPO_F32), Algorithm 1.  V = cand[0..m).  Writes the kept ids,
 * in the order Algorithm 1 adds them, to out[0..R) (out must hold
 * min(R, m) ids) and returns how many were kept.  R <= 0 means no bound.
 * *pairs (nullable) is increased by the number of candidate-candidate
 * distances evaluated.
 */
int32_t rpo_robust_prune(const void* X, int32_t dt, int64_t n, int32_t d,
                         int32_t p, const int32_t* cand, int32_t m,
                         int32_t num, int32_t den, int32_t R,
                         int32_t* out, int64_t* pairs);

/*
 * Same algorithm on an explicit matrix of squared distances
 * Smat[a*n + b] (FP64, symmetric, zero diagonal): used for the worked
 * instances in the paper's proofs, which are stated as distance matrices.
 */
int32_t rpo_robust_prune_smat(const double* Smat, int32_t n, int32_t p,
                              const int32_t* cand, int32_t m,
                              int32_t num, int32_t den, int32_t R, int32_t* out);

/*
 * UnsortedRobustPrune (Section 3, defined right after RP-Tuning): Algorithm 1
 * with p* taken as an arbitrary remaining out-neighbour of p instead of the
 * argmin.  Read here as the first id of V still present, in the order the
 * list stores them (V keeps the first occurrence of a repeated id).  Same
 * arguments and outputs as rpo_robust_prune / rpo_robust_prune_smat.
 */
int32_t rpo_robust_prune_unsorted(const void* X, int32_t dt, int64_t n, int32_t d,
                                  int32_t p, const int32_t* cand, int32_t m,
                                  int32_t num, int32_t den, int32_t R,
                                  int32_t* out, int64_t* pairs);
int32_t rpo_robust_prune_unsorted_smat(const double* Smat, int32_t n, int32_t p,
                                       const int32_t* cand, int32_t m,
                                       int32_t num, int32_t den, int32_t R, int32_t* out);

/*
 * RP-Tuning (Section 3): RobustPrune(p, N_out(p), alpha, R) for every node p
 * listed in nodes[0..n_nodes) (nodes == NULL means all n nodes in order).
 * Adjacency: nbr is n x stride int32 (row p holds deg[p] ids, rest ignored).
 * Output row t (for nodes[t]) goes to out_nbr[t*R .. t*R+R) padded with -1,
 * its count to out_deg[t].  R must be >= 1 here.  Returns 0 or an error.
 */
int32_t rpo_prune_graph(const void* X, int32_t dt, int64_t n, int32_t d,
                        const int32_t* nbr, const int32_t* deg, int32_t stride,
                        const int32_t* nodes, int64_t n_nodes,
                        int32_t num, int32_t den, int32_t R,
                        int32_t* out_nbr, int32_t* out_deg, int64_t* pairs);

/* RP-Tuning with UnsortedRobustPrune in place of RobustPrune (Theorem 3.1's
 * setting); same arguments as rpo_prune_graph. */
int32_t rpo_prune_graph_unsorted(const void* X, int32_t dt, int64_t n, int32_t d,
                                 const int32_t* nbr, const int32_t* deg, int32_t stride,
                                 const int32_t* nodes, int64_t n_nodes,
                                 int32_t num, int32_t den, int32_t R,
                                 int32_t* out_nbr, int32_t* out_deg, int64_t* pairs);

/*
 * GreedySearch(s, q, k, L), Algorithm 2, for nq queries (nq x d, same dtype
 * as X).  out_ids: nq x k (-1 padded), out_dist: nq x k squared distances
 * as FP64 (nullable), out_hops: nq counts of visited vertices (nullable).
 */
int32_t rpo_search(const void* X, int32_t dt, int64_t n, int32_t d,
                   const int32_t* nbr, const int32_t* deg, int32_t stride,
                   int32_t start, const void* Q, int64_t nq, int32_t k, int32_t L,
                   int32_t* out_ids, double* out_dist, int32_t* out_hops);

/* Exact k nearest points of each query by (S, id), by brute force. */
int32_t rpo_groundtruth(const void* X, int32_t dt, int64_t n, int32_t d,
                        const void* Q, int64_t nq, int32_t k, int32_t* out_ids);

#ifdef __cplusplus
}
#endif
#endif
