/*
 * rpo.c -- plain, single-threaded CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Follows the paper's Algorithm 1 (RobustPrune), the RP-Tuning paragraph of
 * Section 3 and Algorithm 2 (GreedySearch) step by step, in their order and
 * notation, with no blocking, fusion or reordering.  See rpo.h for the
 * distance conventions (squared Euclidean, exact int for uint8, canonical
 * FP64 for float32, rational alpha, ties broken by (S, id)).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no -ffast-math:
 * the FP64 evaluation order is part of the definition).
 */
#include "rpo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Distances                                                                 */
/* ------------------------------------------------------------------------ */

int64_t rpo_sqdist_u8(const uint8_t* a, const uint8_t* b, int32_t d) {
  int64_t acc = 0;
  for (int32_t k = 0; k < d; ++k) {
    int64_t t = (int64_t)a[k] - (int64_t)b[k];
    acc += t * t;
  }
  return acc;
}

double rpo_sqdist_f32(const float* a, const float* b, int32_t d) {
  double acc = 0.0;
  for (int32_t k = 0; k < d; ++k) {
    double t = (double)a[k] - (double)b[k];
    acc = fma(t, t, acc);
  }
  return acc;
}

/* A "metric" is either a point set (uint8 / float32 rows) or an explicit
 * matrix of squared distances.  Every squared distance is carried as a
 * double: uint8 sums are integers below 2^53, so the conversion is exact and
 * order preserving, and the alpha test converts them back to integers. */
typedef struct {
  int32_t kind; /* RPO_U8, RPO_F32, or 3 = matrix */
  const void* X;
  int64_t n;
  int32_t d;
  const double* smat;
} metric_t;

#define KIND_SMAT 3

static double sq(const metric_t* M, int64_t a, int64_t b) {
  if (M->kind == RPO_U8) {
    const uint8_t* X = (const uint8_t*)M->X;
    return (double)rpo_sqdist_u8(X + a * M->d, X + b * M->d, M->d);
  }
  if (M->kind == RPO_F32) {
    const float* X = (const float*)M->X;
    return rpo_sqdist_f32(X + a * M->d, X + b * M->d, M->d);
  }
  return M->smat[a * M->n + b];
}

/* (S, id) lexicographic order: is (sa, ia) strictly before (sb, ib)? */
static int before(double sa, int32_t ia, double sb, int32_t ib) {
  if (sa < sb) return 1;
  if (sa > sb) return 0;
  return ia < ib;
}

/* The pruning condition of Algorithm 1, alpha * D(p*, p') <= D(p, p'),
 * on squared distances with alpha = num/den:
 *   num^2 * S(p*, p') <= den^2 * S(p, p').                                  */
static int alpha_test(const metric_t* M, int32_t num, int32_t den, double s_star,
                      double s_p) {
  if (M->kind == RPO_U8) {
    __int128 lhs = (__int128)num * num * (__int128)(int64_t)s_star;
    __int128 rhs = (__int128)den * den * (__int128)(int64_t)s_p;
    return lhs <= rhs;
  }
  {
    double a2 = (double)num * (double)num;
    double b2 = (double)den * (double)den;
    double lhs = a2 * s_star;
    double rhs = b2 * s_p;
    return lhs <= rhs;
  }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: RobustPrune(p, V, alpha, R)                                  */
/* ------------------------------------------------------------------------ */

/* sorted != 0: RobustPrune, Algorithm 1.  sorted == 0: UnsortedRobustPrune
 * (Section 3, the paragraph after the RP-Tuning definition): the same
 * procedure with p* taken as an arbitrary out-neighbour of p instead of the
 * argmin; "arbitrary" is read as the first candidate still in V in the order
 * the list stores them. */
static int32_t robust_prune(const metric_t* M, int32_t p, const int32_t* cand,
                            int32_t m, int32_t num, int32_t den, int32_t R,
                            int32_t* out, int64_t* pairs, int sorted) {
  if (m < 0 || num < 1 || den < 1 || num < den) return RPO_EINVAL;
  if (m == 0) return 0;
  int32_t* V = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
  double* Sp = (double*)malloc(sizeof(double) * (size_t)m); /* S(p, V[t]) */
  char* inV = (char*)malloc((size_t)m);
  if (!V || !Sp || !inV) {
    free(V); free(Sp); free(inV);
    return RPO_EINVAL;
  }

  /* V <- (V u N_out(p)) \ {p}.  In RP-Tuning V is N_out(p) itself, so V is
   * the set of distinct listed ids other than p. */
  int32_t nv = 0;
  for (int32_t t = 0; t < m; ++t) {
    int32_t c = cand[t];
    if (c < 0 || (int64_t)c >= M->n) {
      free(V); free(Sp); free(inV);
      return RPO_ERANGE;
    }
    if (c == p) continue;
    int dup = 0;
    for (int32_t u = 0; u < nv; ++u)
      if (V[u] == c) { dup = 1; break; }
    if (dup) continue;
    V[nv] = c;
    Sp[nv] = sq(M, p, c);
    inV[nv] = 1;
    ++nv;
  }

  /* N_out(p) <- empty */
  int32_t kept = 0;
  int32_t remaining = nv;
  while (remaining > 0) {
    /* p* <- argmin_{p' in V} D(p, p')  (unsorted: the first p' still in V) */
    int32_t best = -1;
    for (int32_t t = 0; t < nv; ++t) {
      if (!inV[t]) continue;
      if (!sorted) { best = t; break; }
      if (best < 0 || before(Sp[t], V[t], Sp[best], V[best])) best = t;
    }
    /* N_out(p) <- N_out(p) u {p*} */
    out[kept++] = V[best];
    /* if |N_out(p)| = R: break */
    if (R > 0 && kept == R) break;
    /* for p' in V: if alpha * D(p*, p') <= D(p, p'): remove p' from V.
     * p* itself satisfies the test in exact arithmetic (D(p*, p*) = 0);
     * it is removed explicitly so that no rounding can keep it. */
    inV[best] = 0;
    --remaining;
    for (int32_t t = 0; t < nv; ++t) {
      if (!inV[t]) continue;
      double s_star = sq(M, V[best], V[t]);
      if (pairs) ++*pairs;
      if (alpha_test(M, num, den, s_star, Sp[t])) {
        inV[t] = 0;
        --remaining;
      }
    }
  }
  free(V);
  free(Sp);
  free(inV);
  return kept;
}

int32_t rpo_robust_prune(const void* X, int32_t dt, int64_t n, int32_t d,
                         int32_t p, const int32_t* cand, int32_t m,
                         int32_t num, int32_t den, int32_t R,
                         int32_t* out, int64_t* pairs) {
  if (!X || (dt != RPO_U8 && dt != RPO_F32) || n < 1 || d < 1) return RPO_EINVAL;
  if (p < 0 || (int64_t)p >= n) return RPO_ERANGE;
  metric_t M = {dt, X, n, d, NULL};
  return robust_prune(&M, p, cand, m, num, den, R, out, pairs, 1);
}

int32_t rpo_robust_prune_unsorted(const void* X, int32_t dt, int64_t n, int32_t d,
                                  int32_t p, const int32_t* cand, int32_t m,
                                  int32_t num, int32_t den, int32_t R,
                                  int32_t* out, int64_t* pairs) {
  if (!X || (dt != RPO_U8 && dt != RPO_F32) || n < 1 || d < 1) return RPO_EINVAL;
  if (p < 0 || (int64_t)p >= n) return RPO_ERANGE;
  metric_t M = {dt, X, n, d, NULL};
  return robust_prune(&M, p, cand, m, num, den, R, out, pairs, 0);
}

int32_t rpo_robust_prune_smat(const double* Smat, int32_t n, int32_t p,
                              const int32_t* cand, int32_t m,
                              int32_t num, int32_t den, int32_t R, int32_t* out) {
  if (!Smat || n < 1) return RPO_EINVAL;
  if (p < 0 || p >= n) return RPO_ERANGE;
  metric_t M = {KIND_SMAT, NULL, n, 0, Smat};
  return robust_prune(&M, p, cand, m, num, den, R, out, NULL, 1);
}

int32_t rpo_robust_prune_unsorted_smat(const double* Smat, int32_t n, int32_t p,
                                       const int32_t* cand, int32_t m,
                                       int32_t num, int32_t den, int32_t R, int32_t* out) {
  if (!Smat || n < 1) return RPO_EINVAL;
  if (p < 0 || p >= n) return RPO_ERANGE;
  metric_t M = {KIND_SMAT, NULL, n, 0, Smat};
  return robust_prune(&M, p, cand, m, num, den, R, out, NULL, 0);
}

/* ------------------------------------------------------------------------ */
/* RP-Tuning: RobustPrune(p, N_out(p), alpha, R) for every p                 */
/* ------------------------------------------------------------------------ */

static int32_t prune_graph(const void* X, int32_t dt, int64_t n, int32_t d,
                           const int32_t* nbr, const int32_t* deg, int32_t stride,
                           const int32_t* nodes, int64_t n_nodes,
                           int32_t num, int32_t den, int32_t R,
                           int32_t* out_nbr, int32_t* out_deg, int64_t* pairs, int sorted) {
  if (!X || !nbr || !deg || !out_nbr || !out_deg) return RPO_EINVAL;
  if ((dt != RPO_U8 && dt != RPO_F32) || n < 1 || d < 1 || stride < 1 || R < 1)
    return RPO_EINVAL;
  metric_t M = {dt, X, n, d, NULL};
  int64_t count = nodes ? n_nodes : n;
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)stride);
  if (!tmp) return RPO_EINVAL;
  for (int64_t t = 0; t < count; ++t) {
    int64_t p = nodes ? nodes[t] : t;
    if (p < 0 || p >= n) { free(tmp); return RPO_ERANGE; }
    int32_t m = deg[p];
    if (m < 0 || m > stride) { free(tmp); return RPO_EINVAL; }
    int32_t k = robust_prune(&M, (int32_t)p, nbr + p * stride, m, num, den, R, tmp, pairs,
                             sorted);
    if (k < 0) { free(tmp); return k; }
    for (int32_t u = 0; u < R; ++u) out_nbr[t * R + u] = u < k ? tmp[u] : -1;
    out_deg[t] = k;
  }
  free(tmp);
  return 0;
}

int32_t rpo_prune_graph(const void* X, int32_t dt, int64_t n, int32_t d,
                        const int32_t* nbr, const int32_t* deg, int32_t stride,
                        const int32_t* nodes, int64_t n_nodes,
                        int32_t num, int32_t den, int32_t R,
                        int32_t* out_nbr, int32_t* out_deg, int64_t* pairs) {
  return prune_graph(X, dt, n, d, nbr, deg, stride, nodes, n_nodes, num, den, R, out_nbr,
                     out_deg, pairs, 1);
}

int32_t rpo_prune_graph_unsorted(const void* X, int32_t dt, int64_t n, int32_t d,
                                 const int32_t* nbr, const int32_t* deg, int32_t stride,
                                 const int32_t* nodes, int64_t n_nodes,
                                 int32_t num, int32_t den, int32_t R,
                                 int32_t* out_nbr, int32_t* out_deg, int64_t* pairs) {
  return prune_graph(X, dt, n, d, nbr, deg, stride, nodes, n_nodes, num, den, R, out_nbr,
                     out_deg, pairs, 0);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: GreedySearch(s, q, k, L)                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  double s;
  int32_t id;
} entry_t;

static int entry_cmp(const void* a, const void* b) {
  const entry_t* x = (const entry_t*)a;
  const entry_t* y = (const entry_t*)b;
  if (before(x->s, x->id, y->s, y->id)) return -1;
  if (before(y->s, y->id, x->s, x->id)) return 1;
  return 0;
}

static double sq_query(int32_t dt, const void* X, int32_t d, int64_t j, const void* q) {
  if (dt == RPO_U8)
    return (double)rpo_sqdist_u8((const uint8_t*)q, (const uint8_t*)X + j * d, d);
  return rpo_sqdist_f32((const float*)q, (const float*)X + j * d, d);
}

int32_t rpo_search(const void* X, int32_t dt, int64_t n, int32_t d,
                   const int32_t* nbr, const int32_t* deg, int32_t stride,
                   int32_t start, const void* Q, int64_t nq, int32_t k, int32_t L,
                   int32_t* out_ids, double* out_dist, int32_t* out_hops) {
  if (!X || !nbr || !deg || !Q || !out_ids) return RPO_EINVAL;
  if ((dt != RPO_U8 && dt != RPO_F32) || n < 1 || d < 1 || stride < 1) return RPO_EINVAL;
  if (k < 1 || L < k) return RPO_EINVAL;
  if (start < 0 || (int64_t)start >= n) return RPO_ERANGE;
  size_t esz = dt == RPO_U8 ? 1 : 4;
  entry_t* Lset = (entry_t*)malloc(sizeof(entry_t) * (size_t)(L + stride + 1));
  char* visited = (char*)malloc((size_t)n);
  if (!Lset || !visited) { free(Lset); free(visited); return RPO_EINVAL; }

  for (int64_t qi = 0; qi < nq; ++qi) {
    const void* q = (const char*)Q + (size_t)qi * (size_t)d * esz;
    memset(visited, 0, (size_t)n);
    int32_t hops = 0;
    /* L <- {s}, V <- empty */
    int32_t cnt = 1;
    Lset[0].id = start;
    Lset[0].s = sq_query(dt, X, d, start, q);
    for (;;) {
      /* p* <- argmin_{p in L \ V} D(p, q) */
      int32_t best = -1;
      for (int32_t t = 0; t < cnt; ++t) {
        if (visited[Lset[t].id]) continue;
        if (best < 0 || before(Lset[t].s, Lset[t].id, Lset[best].s, Lset[best].id)) best = t;
      }
      if (best < 0) break; /* L \ V is empty */
      int32_t pstar = Lset[best].id;
      /* L <- L u N_out(p*) */
      int32_t m = deg[pstar];
      if (m < 0 || m > stride) { free(Lset); free(visited); return RPO_EINVAL; }
      for (int32_t u = 0; u < m; ++u) {
        int32_t j = nbr[(int64_t)pstar * stride + u];
        if (j < 0 || (int64_t)j >= n) { free(Lset); free(visited); return RPO_ERANGE; }
        int in = 0;
        for (int32_t t = 0; t < cnt; ++t)
          if (Lset[t].id == j) { in = 1; break; }
        if (in) continue;
        Lset[cnt].id = j;
        Lset[cnt].s = sq_query(dt, X, d, j, q);
        ++cnt;
      }
      /* V <- V u {p*} */
      visited[pstar] = 1;
      ++hops;
      /* if |L| > L: retain the closest L points to q */
      if (cnt > L) {
        qsort(Lset, (size_t)cnt, sizeof(entry_t), entry_cmp);
        cnt = L;
      }
    }
    /* return the closest k points of L */
    qsort(Lset, (size_t)cnt, sizeof(entry_t), entry_cmp);
    for (int32_t t = 0; t < k; ++t) {
      out_ids[qi * k + t] = t < cnt ? Lset[t].id : -1;
      if (out_dist) out_dist[qi * k + t] = t < cnt ? Lset[t].s : -1.0;
    }
    if (out_hops) out_hops[qi] = hops;
  }
  free(Lset);
  free(visited);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact ground truth by brute force                                         */
/* ------------------------------------------------------------------------ */

int32_t rpo_groundtruth(const void* X, int32_t dt, int64_t n, int32_t d,
                        const void* Q, int64_t nq, int32_t k, int32_t* out_ids) {
  if (!X || !Q || !out_ids || (dt != RPO_U8 && dt != RPO_F32) || n < 1 || d < 1 || k < 1)
    return RPO_EINVAL;
  size_t esz = dt == RPO_U8 ? 1 : 4;
  entry_t* top = (entry_t*)malloc(sizeof(entry_t) * (size_t)k);
  if (!top) return RPO_EINVAL;
  for (int64_t qi = 0; qi < nq; ++qi) {
    const void* q = (const char*)Q + (size_t)qi * (size_t)d * esz;
    int32_t cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
      double s = sq_query(dt, X, d, j, q);
      if (cnt == k && !before(s, (int32_t)j, top[k - 1].s, top[k - 1].id)) continue;
      int32_t pos = cnt < k ? cnt++ : k - 1;
      while (pos > 0 && before(s, (int32_t)j, top[pos - 1].s, top[pos - 1].id)) {
        top[pos] = top[pos - 1];
        --pos;
      }
      top[pos].s = s;
      top[pos].id = (int32_t)j;
    }
    for (int32_t t = 0; t < k; ++t) out_ids[qi * k + t] = t < cnt ? top[t].id : -1;
  }
  free(top);
  return 0;
}
