"""Exact pins of the graph-level reachability meter (Definition 2.1), of the
oracle's pair counter and of UnsortedRobustPrune (Section 3), on instances
small enough to trace by hand.

Every expected value below is worked out in the comments from the distances
alone; none is computed by the function under test.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import reach


def _complete_except(n, lists):
    """Out-lists: the given ones, every other vertex linked to all others."""
    return [lists[v] if v in lists else [u for u in range(n) if u != v] for v in range(n)]


def _permute(D, adj, perm):
    """The same graph with vertex v renamed perm[v]."""
    n = len(adj)
    Dp = np.empty_like(D)
    for a in range(n):
        for b in range(n):
            Dp[perm[a], perm[b]] = D[a, b]
    ap = [None] * n
    for v in range(n):
        ap[perm[v]] = [perm[u] for u in adj[v]]
    return Dp, ap


# Lemma 3.7 instance (alpha_1 = 3, alpha_2 = 2, distances x 6): p x y z with
# D(p, .) = 6, D(x, y) = 3, D(y, z) = 2, D(x, z) = 5.  After RP-Tuning p keeps
# {x}; x, y, z keep everything.  The pairs without an edge are (p, y) and
# (p, z), each with the single witness x:
#   (p, y): D(p, y) / D(x, y) = 6 / 3 = 2
#   (p, z): D(p, z) / D(x, z) = 6 / 5
# so alpha* = min(2, 6/5) = 6/5 = alpha_1 alpha_2 / (alpha_1 + alpha_2).
LEMMA37_D = np.array([[0, 6, 6, 6], [6, 0, 3, 5], [6, 3, 0, 2], [6, 5, 2, 0]], np.float64)


@pytest.mark.parametrize("perm", [(0, 1, 2, 3), (3, 0, 1, 2), (2, 3, 0, 1), (1, 2, 3, 0)])
def test_reachability_lemma37_full_graph(perm):
    adj = _complete_except(4, {0: [1]})
    D, A = _permute(LEMMA37_D, adj, perm)
    # the binding pair sits at every id order, so a meter that skips pairs
    # (only q > p, only q < p) misses it under one of the renamings
    assert reach.reachability(D, A) == 6.0 / 5.0
    assert reach.pair_reach(D, A, perm[0], perm[2]) == 2.0


def test_reachability_takes_the_best_witness_and_the_worst_pair():
    """Points on a line at 0, 1, 3, 4 (ids a b c e); D is |u - v|.
    Graph 1: a -> {b}; everyone else complete.  Pairs without an edge:
      (a, c): witness b, 3 / 2;   (a, e): witness b, 4 / 3   -> alpha* = 4/3.
    Graph 2: a -> {b, c}.  Only (a, e) lacks an edge; witnesses b (4 / 3) and
      c (4 / 1): the best witness counts, so alpha* = 4.
    A meter that took the worst witness would give 4/3 on graph 2; one that
    took the largest pair would give 3/2 on graph 1."""
    x = np.array([0.0, 1.0, 3.0, 4.0])
    D = np.abs(x[:, None] - x[None, :])
    g1 = _complete_except(4, {0: [1]})
    g2 = _complete_except(4, {0: [1, 2]})
    assert reach.reachability(D, g1) == 4.0 / 3.0
    assert reach.reachability(D, g2) == 4.0
    assert reach.pair_reach(D, g1, 0, 2) == 3.0 / 2.0


def test_reachability_degenerate_graphs():
    x = np.array([0.0, 1.0, 3.0])
    D = np.abs(x[:, None] - x[None, :])
    # complete graph: no pair lacks an edge
    assert reach.reachability(D, _complete_except(3, {})) == math.inf
    # a vertex with no out-neighbour cannot reach anyone: alpha* = 0
    assert reach.reachability(D, _complete_except(3, {1: []})) == 0.0
    # a witness at distance 0 from the target reaches it at every alpha
    x2 = np.array([0.0, 2.0, 2.0])
    D2 = np.abs(x2[:, None] - x2[None, :])
    assert reach.reachability(D2, _complete_except(3, {0: [1]})) == math.inf
    # self ids and -1 padding in a list are ignored
    assert reach.reachability(D, [[0, 1, -1], [0, 2], [0, 1]]) == 3.0 / 2.0


@pytest.mark.parametrize("a1,a2", [(3.0, 2.0), (1.2, 1.1), (2.0, 1.5)])
def test_reachability_appendix_construction(a1, a2):
    """Appendix A's planar points with p -> {x} and the rest complete:
    (p, y) has witness x at |p - y| / |x - y| = 1 / (2 sin theta_2) = alpha_2,
    (p, z) has witness x at 1 / |x - z| = 1 / beta, and 1 / beta < alpha_2
    here, so alpha* = 1 / beta (Table 1, sorted Euclidean entry)."""
    P = np.stack(reach.appendix_points(a1, a2))
    D = reach.distance_matrix(P)
    got = reach.reachability(D, _complete_except(4, {0: [1]}))
    t1, t2 = math.asin(1 / (2 * a1)), math.asin(1 / (2 * a2))
    assert got == pytest.approx(1.0 / (2.0 * math.sin(t1 + t2)), rel=1e-12)
    assert got < a2


# --------------------------------------------------------------------------
# The oracle's pair counter, traced by hand
# --------------------------------------------------------------------------

# uint8, d = 1: p = 10, candidates 11, 12, 5, 4 (ids 1..4); S(p, .) = 1, 4, 25, 36.
LINE_X = np.array([[10], [11], [12], [5], [4]], np.uint8)


def test_pair_counter_alpha_one():
    """alpha = 1: keep 11; test 12 (S = 1 <= 4: gone), 5 (36 > 25: stays),
    4 (49 > 36: stays) -> 3 pairs; keep 5; test 4 (1 <= 36: gone) -> 1 pair.
    Kept [11, 5] after 4 pair evaluations."""
    assert oracle.robust_prune(LINE_X, 0, [1, 2, 3, 4], 1, 1, 0, count_pairs=True) == ([1, 3], 4)


def test_pair_counter_degree_bound_stops_before_testing():
    """R = 1: the first keep reaches the bound and the loop breaks before any
    pair is evaluated."""
    assert oracle.robust_prune(LINE_X, 0, [4, 3, 2, 1], 1, 1, 1, count_pairs=True) == ([1], 0)


def test_pair_counter_nothing_pruned():
    """alpha = 100 prunes nothing here, so every pair after a keep is tested
    once: 3 + 2 + 1 = 6, and all four are kept by distance."""
    got = oracle.robust_prune(LINE_X, 0, [3, 1, 4, 2], 100, 1, 0, count_pairs=True)
    assert got == ([1, 2, 3, 4], 6)


def test_pair_counter_of_prune_graph_is_the_sum():
    nbr = np.array([[1, 2, 3, 4], [0, 2, -1, -1], [0, 1, 3, -1], [0, 4, -1, -1],
                    [0, 3, -1, -1]], np.int32)
    deg = np.array([4, 2, 3, 2, 2], np.int32)
    _, _, pairs = oracle.prune_graph(LINE_X, nbr, deg, 1, 1, 4)
    per = sum(oracle.robust_prune(LINE_X, p, nbr[p, :deg[p]], 1, 1, 4, count_pairs=True)[1]
              for p in range(5))
    assert pairs == per
    # vertex 0 as traced above contributes 4
    _, _, p0 = oracle.prune_graph(LINE_X, nbr, deg, 1, 1, 4, nodes=[0])
    assert p0 == 4


# --------------------------------------------------------------------------
# UnsortedRobustPrune (Section 3): p* is the first remaining listed candidate
# --------------------------------------------------------------------------

def test_unsorted_follows_list_order():
    """alpha = 1 on the line list [4, 3, 2, 1] (coordinates 4, 5, 12, 11):
    keep 4 (first listed); 5 is pruned (S(4, 5) = 1 <= 25), 12 and 11 stay;
    keep 12; 11 is pruned (S(12, 11) = 1 <= S(10, 11) = 1, equality).
    Sorted RobustPrune on the same list keeps [11, 5] instead."""
    got = oracle.robust_prune(LINE_X, 0, [4, 3, 2, 1], 1, 1, 0, count_pairs=True, unsorted=True)
    assert got == ([4, 2], 4)
    assert oracle.robust_prune(LINE_X, 0, [4, 3, 2, 1], 1, 1, 0) == [1, 3]


def test_unsorted_drops_self_and_repeats_keeping_first_occurrence():
    # list [2, 0, 4, 2, 1]: p = 0 and the second 2 are dropped; order 2, 4, 1
    got = oracle.robust_prune(LINE_X, 0, [2, 0, 4, 2, 1], 100, 1, 0, unsorted=True)
    assert got == [2, 4, 1]
    assert oracle.robust_prune(LINE_X, 0, [2, 0, 4, 2, 1], 100, 1, 2, unsorted=True) == [2, 4]
    assert oracle.robust_prune(LINE_X, 0, [], 1, 1, 0, unsorted=True) == []


def test_unsorted_equals_sorted_on_lists_in_distance_order():
    rng = np.random.default_rng(5)
    X = rng.integers(0, 40, (60, 3)).astype(np.uint8)
    for t in range(40):
        p = int(rng.integers(0, 60))
        cand = [int(c) for c in rng.choice(60, 25, replace=False) if c != p]
        key = sorted(cand, key=lambda c: (oracle.sqdist(X[p], X[c]), c))
        for a in ((1, 1), (6, 5), (3, 2)):
            assert oracle.robust_prune(X, p, key, *a, 0, unsorted=True) == \
                oracle.robust_prune(X, p, key, *a, 0)


def test_unsorted_lemma35_collinear_instance():
    """Lemma 3.5's collinear points (alpha_1 = 3, alpha_2 = 2, distances x 3):
    p = 0, z = 3, y = 4, x = 6 on a line, so D(p, z) = 3, D(z, y) = 1 = D(p, z)
    / alpha_1 and D(y, x) = 2 = D(p, y) / alpha_2.  The base list of p is
    [x, y]: y witnesses (p, z) at 3 = alpha_1.
      UnsortedRobustPrune(p, [x, y], 2): keeps x first; 2 D(x, y) = 4 <= D(p, y)
      = 4 prunes y.  Then (p, z) has only the witness x: D(p, z) / D(x, z) =
      3 / 3 = 1 = alpha_1 alpha_2 / (alpha_1 + alpha_2 + 1), the proof's value
      (the printed 1 / (1/alpha_1 + 1/alpha_2 + 1) would be 6/11).
      Sorted RobustPrune keeps y (nearer) and prunes x (4 <= 6): (p, z) keeps
      witness y at 3."""
    X = np.array([[0], [6], [4], [3]], np.uint8)  # ids p x y z
    assert oracle.robust_prune(X, 0, [1, 2], 2, 1, 0, unsorted=True) == [1]
    assert oracle.robust_prune(X, 0, [1, 2], 2, 1, 0) == [2]
    D = reach.distance_matrix(X.astype(np.float64))
    base = _complete_except(4, {0: [1, 2]})
    assert reach.pair_reach(D, base, 0, 3) == 3.0
    unsorted_g = _complete_except(4, {0: [1]})
    sorted_g = _complete_except(4, {0: [2]})
    assert reach.reachability(D, unsorted_g) == 1.0
    assert reach.unsorted_bound(3.0, 2.0) == 1.0
    # sorted: (p, x) through y at 6/2 = 3, (p, z) through y at 3
    assert reach.reachability(D, sorted_g) == 3.0


def test_unsorted_smat_matches_points():
    rng = np.random.default_rng(12)
    X = rng.integers(0, 30, (25, 4)).astype(np.uint8)
    S = np.array([[oracle.sqdist(X[i], X[j]) for j in range(25)] for i in range(25)],
                 dtype=np.float64)
    for p in range(25):
        cand = rng.integers(0, 25, 20).tolist()
        assert oracle.robust_prune_smat(S, p, cand, 6, 5, 0, unsorted=True) == \
            oracle.robust_prune(X, p, cand, 6, 5, 0, unsorted=True)


def test_unsorted_prune_graph_and_threads_match_per_node():
    rng = np.random.default_rng(13)
    X = rng.standard_normal((50, 6)).astype(np.float32)
    nbr = rng.integers(0, 50, (50, 14)).astype(np.int32)
    deg = rng.integers(0, 15, 50).astype(np.int32)
    for unsorted in (False, True):
        out, od, pairs = oracle.prune_graph(X, nbr, deg, 11, 10, 6, unsorted=unsorted)
        out4, od4, pairs4 = oracle.prune_graph(X, nbr, deg, 11, 10, 6, unsorted=unsorted,
                                               threads=4)
        assert (out == out4).all() and (od == od4).all() and pairs == pairs4
        for p in range(50):
            want = oracle.robust_prune(X, p, nbr[p, :deg[p]], 11, 10, 6, unsorted=unsorted)
            assert out[p, :od[p]].tolist() == want


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_theorem31_unsorted_bound_on_shuffled_lists(seed):
    """Theorem 3.1: UnsortedRobustPrune at alpha_2 of an alpha_1-reachable graph
    keeps reachability >= alpha_1 alpha_2 / (alpha_1 + alpha_2 + 1), whatever
    the list order (lists shuffled here)."""
    rng = np.random.default_rng(400 + seed)
    X = rng.standard_normal((26, 2)).astype(np.float32)
    n = X.shape[0]
    base = [oracle.robust_prune(X, p, [q for q in range(n) if q != p], 3, 1, 0) for p in range(n)]
    for lst in base:
        rng.shuffle(lst)
    pruned = [oracle.robust_prune(X, p, base[p], 2, 1, 0, unsorted=True) for p in range(n)]
    D = reach.distance_matrix(X)
    assert reach.reachability(D, base) >= 3.0 * (1 - 1e-9)
    assert reach.reachability(D, pruned) >= reach.unsorted_bound(3.0, 2.0) * (1 - 1e-9)
