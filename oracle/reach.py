"""alpha-reachability meter and Table 1 closed forms (TEST INFRASTRUCTURE ONLY).

* Definition 2.1: q is alpha-reachable from p if (p, q) is an edge, or some
  out-neighbour p' of p has alpha * D(p', q) <= D(p, q).  The reachability
  alpha* of a graph is the largest alpha for which every ordered pair is
  alpha-reachable, i.e.

      alpha* = min over p != q with (p, q) not an edge of
               max over p' in N_out(p) of D(p, q) / D(p', q)

  (a witness with D(p', q) = 0 reaches q for every alpha; a p with no
  out-neighbour and a missing edge gives alpha* = 0).
* Table 1 / Theorems 3.1 and 3.2: worst-case reachability after RP-Tuning of
  an alpha_1-reachable graph at alpha_2.
* Appendix A: beta(a1, a2) = 2 sin(theta_1 + theta_2) with
  theta_i = asin(1 / (2 a_i)).

Everything is plain numpy / math in FP64.
"""
from __future__ import annotations

import math

import numpy as np


def distance_matrix(X: np.ndarray) -> np.ndarray:
    """Euclidean distance matrix in FP64 (plain pairwise differences)."""
    X = np.asarray(X, dtype=np.float64)
    diff = X[:, None, :] - X[None, :, :]
    return np.sqrt((diff * diff).sum(axis=2))


def reachability(D: np.ndarray, adj) -> float:
    """alpha* of the graph ``adj`` (list of out-lists) under distances D."""
    n = D.shape[0]
    best = math.inf
    for p in range(n):
        out = set(int(v) for v in adj[p] if v >= 0 and v != p)
        for q in range(n):
            if q == p or q in out:
                continue
            r = 0.0
            for w in out:
                if D[w, q] == 0.0:
                    r = math.inf
                    break
                r = max(r, D[p, q] / D[w, q])
            best = min(best, r)
    return best


def pair_reach(D: np.ndarray, adj, p: int, q: int) -> float:
    """Largest alpha for which q is alpha-reachable from p."""
    out = set(int(v) for v in adj[p] if v >= 0 and v != p)
    if q in out:
        return math.inf
    r = 0.0
    for w in out:
        if D[w, q] == 0.0:
            return math.inf
        r = max(r, D[p, q] / D[w, q])
    return r


def unsorted_bound(a1: float, a2: float) -> float:
    """Unsorted worst case (Theorem 3.1): a1 a2 / (a1 + a2 + 1).

    This is the value the proof of Theorem 3.1 derives and that the collinear
    instance of Lemma 3.5 attains, 1 / (1/a1 + 1/a2 + 1/(a1 a2)).  Table 1 and
    the theorem statement print the last term of the denominator as 1; the
    proof's value is taken here."""
    return a1 * a2 / (a1 + a2 + 1.0)


def sorted_general_bound(a1: float, a2: float) -> float:
    """Table 1, sorted row, general metric (Theorem 3.2): 1 / (1/a1 + 1/a2)."""
    return 1.0 / (1.0 / a1 + 1.0 / a2)


def beta(a1: float, a2: float) -> float:
    """Optimum of the Euclidean problem of Lemma 3.8 (Appendix A)."""
    return (1.0 / a1) * math.sqrt(1.0 - 1.0 / (4.0 * a2 * a2)) + \
           (1.0 / a2) * math.sqrt(1.0 - 1.0 / (4.0 * a1 * a1))


def sorted_euclid_bound(a1: float, a2: float) -> float:
    """Table 1, sorted row, Euclidean (Theorem 3.2): 1 / beta(a1, a2)."""
    return 1.0 / beta(a1, a2)


def appendix_points(a1: float, a2: float):
    """The planar construction of Appendix A attaining beta: p at the origin,
    z = (1, 0), y at angle 2 theta_1, x at angle 2 (theta_1 + theta_2)."""
    t1 = math.asin(1.0 / (2.0 * a1))
    t2 = math.asin(1.0 / (2.0 * a2))
    p = np.array([0.0, 0.0])
    z = np.array([1.0, 0.0])
    y = np.array([math.cos(2 * t1), math.sin(2 * t1)])
    x = np.array([math.cos(2 * (t1 + t2)), math.sin(2 * (t1 + t2))])
    return p, x, y, z
