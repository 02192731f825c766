"""Pins of the oracle's GreedySearch (Algorithm 2), ground truth and recall."""
from collections import deque

import numpy as np
import pytest

import oracle
from exact import Exact


def _pad(lists, width):
    nbr = np.full((len(lists), max(width, 1)), -1, np.int32)
    deg = np.zeros(len(lists), np.int32)
    for i, l in enumerate(lists):
        nbr[i, :len(l)] = l
        deg[i] = len(l)
    return nbr, deg


def _topk_exact(X, q, k, allowed=None):
    E = Exact(np.vstack([X, q[None, :]]))
    qi = X.shape[0]
    ids = range(X.shape[0]) if allowed is None else allowed
    return sorted(ids, key=lambda j: (E.S(qi, j), j))[:k]


def test_groundtruth_is_exact_topk():
    rng = np.random.default_rng(0)
    X = rng.integers(0, 5, (200, 3)).astype(np.uint8)  # many exact ties
    Q = rng.integers(0, 5, (10, 3)).astype(np.uint8)
    gt = oracle.groundtruth(X, Q, 15)
    for i in range(10):
        assert gt[i].tolist() == _topk_exact(X, Q[i], 15)
    Xf = rng.standard_normal((150, 4)).astype(np.float32)
    Qf = rng.standard_normal((5, 4)).astype(np.float32)
    gtf = oracle.groundtruth(Xf, Qf, 7)
    for i in range(5):
        assert gtf[i].tolist() == _topk_exact(Xf, Qf[i], 7)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_search_complete_graph_is_exact(dtype):
    """On the complete graph the first expansion inserts every point, so
    GreedySearch returns the exact top-k."""
    rng = np.random.default_rng(1)
    n = 60
    if dtype == "u8":
        X = rng.integers(0, 6, (n, 3)).astype(np.uint8)
        Q = rng.integers(0, 6, (12, 3)).astype(np.uint8)
    else:
        X = rng.standard_normal((n, 5)).astype(np.float32)
        Q = rng.standard_normal((12, 5)).astype(np.float32)
    nbr, deg = _pad([[j for j in range(n) if j != i] for i in range(n)], n - 1)
    for L in (10, 25, 60):
        ids, dist, hops = oracle.search(X, nbr, deg, 7, Q, 10, L)
        gt = oracle.groundtruth(X, Q, 10)
        assert (ids == gt).all()
        assert (hops >= 1).all()


def _reachable(lists, s):
    seen = {s}
    dq = deque([s])
    while dq:
        u = dq.popleft()
        for v in lists[u]:
            if v not in seen:
                seen.add(v)
                dq.append(v)
    return seen


def test_search_unbounded_beam_is_exact_on_reachable_set():
    """With L >= n nothing is ever truncated: every vertex reachable from s is
    inserted and expanded, so the result is the exact top-k of that set and the
    visited count is its size."""
    rng = np.random.default_rng(2)
    n = 80
    X = rng.integers(0, 50, (n, 4)).astype(np.uint8)
    lists = [sorted(set(rng.integers(0, n, rng.integers(0, 4)).tolist()) - {i}) for i in range(n)]
    nbr, deg = _pad(lists, 4)
    Q = rng.integers(0, 50, (8, 4)).astype(np.uint8)
    for s in (0, 5, 33):
        R = _reachable(lists, s)
        ids, dist, hops = oracle.search(X, nbr, deg, s, Q, 5, n)
        for i in range(8):
            want = _topk_exact(X, Q[i], 5, sorted(R))
            got = [v for v in ids[i].tolist() if v >= 0]
            assert got == want
            assert hops[i] == len(R)
            if len(R) < 5:
                assert (ids[i, len(R):] == -1).all()


def test_search_line_worked_example():
    """Points 0..9 on a line, each linked to its right neighbour only, start 0,
    query at 9: the walk visits every point; with L = 2 the beam holds the last
    two points at the end."""
    X = np.arange(10, dtype=np.uint8)[:, None]
    lists = [[i + 1] if i < 9 else [] for i in range(10)]
    nbr, deg = _pad(lists, 1)
    ids, dist, hops = oracle.search(X, nbr, deg, 0, np.array([[9]], np.uint8), 2, 2)
    assert ids[0].tolist() == [9, 8]
    assert dist[0].tolist() == [0.0, 1.0]
    assert hops[0] == 10
    # query at 0: the start is the answer; the beam keeps {0, 1}, then 1 is
    # expanded (adds 2, truncated away), and the search stops
    ids, dist, hops = oracle.search(X, nbr, deg, 0, np.array([[0]], np.uint8), 2, 2)
    assert ids[0].tolist() == [0, 1]
    assert hops[0] == 2


def test_search_evicted_visited_vertex_is_not_expanded_again():
    """Algorithm 2's beam keeps the L closest; a visited vertex evicted by the
    truncation is re-inserted by later expansions (it is no longer in the beam)
    and truncated again, and is never expanded twice."""
    X = np.array([[5], [4], [3], [60]], np.uint8)
    lists = [[1, 2], [0, 3], [0], []]
    nbr, deg = _pad(lists, 2)
    ids, dist, hops = oracle.search(X, nbr, deg, 0, np.array([[0]], np.uint8), 2, 2)
    # {0} -> expand 0 -> {0,1,2} -> keep {2,1}; expand 2 -> +0 -> keep {2,1};
    # expand 1 -> +0,+3 -> keep {2,1}; nothing unvisited -> stop
    assert ids[0].tolist() == [2, 1]
    assert dist[0].tolist() == [9.0, 16.0]
    assert hops[0] == 3


def test_search_argument_errors():
    X = np.zeros((3, 2), np.uint8)
    nbr, deg = _pad([[1], [2], [0]], 1)
    Q = np.zeros((1, 2), np.uint8)
    with pytest.raises(ValueError):
        oracle.search(X, nbr, deg, 0, Q, 3, 2)  # L < k
    with pytest.raises(IndexError):
        oracle.search(X, nbr, deg, 5, Q, 1, 2)  # bad start
    bad, bdeg = _pad([[1], [7], [0]], 1)
    with pytest.raises(IndexError):
        oracle.search(X, bad, bdeg, 0, Q, 1, 4)


def test_recall_definition():
    gt = np.array([[1, 2, 3, 4], [5, 6, 7, 8]])
    assert oracle.recall_at_k(gt, gt, 4) == 1.0
    got = np.array([[1, 2, 9, -1], [8, 7, 6, 0]])
    assert oracle.recall_at_k(got, gt, 4) == pytest.approx((2 + 3) / 8)
