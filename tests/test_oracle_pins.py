"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test would fail under a plausible slip in the oracle: a reversed or
strict comparison, alpha applied to squared distances, a wrong sort key or
tie-break, a missing degree cap, dropped self/duplicate handling, or a
contracted FP64 evaluation.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import reach
from exact import Exact, ExactMatrix, brute_force_prune, canon_sq, characterises, int_sq

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_fixture(name):
    rows = {}
    D = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            if key == "D":
                D.append([int(v) for v in vals])
            else:
                rows[key] = vals
    return rows, D


# --------------------------------------------------------------------------
# Distances: exact integers and the canonical FP64 definition
# --------------------------------------------------------------------------

def test_sqdist_u8_exact():
    rng = np.random.default_rng(1)
    for d in (1, 3, 32, 128, 960):
        a = rng.integers(0, 256, d).astype(np.uint8)
        b = rng.integers(0, 256, d).astype(np.uint8)
        assert oracle.sqdist(a, b) == int_sq(a, b)
    a = np.zeros(128, np.uint8)
    b = np.full(128, 255, np.uint8)
    assert oracle.sqdist(a, b) == 128 * 255 * 255


def test_sqdist_f32_canonical_fp64():
    rng = np.random.default_rng(2)
    for d in (1, 2, 7, 32, 96):
        for scale in (1e-3, 1.0, 1e3):
            a = (rng.standard_normal(d) * scale).astype(np.float32)
            b = (rng.standard_normal(d) * scale).astype(np.float32)
            assert oracle.sqdist(a, b) == canon_sq(a, b)
    # operands whose exact difference needs more than 53 bits: the definition
    # rounds t_k first, then fuses
    a = np.array([2.0 ** 40, 1.0 + 2.0 ** -20, 3.0], np.float32)
    b = np.array([2.0 ** -30, -(2.0 ** 30), 1e-7], np.float32)
    assert oracle.sqdist(a, b) == canon_sq(a, b)


def test_sqdist_f32_uses_fma_not_separate_rounding():
    # find a vector where fma and mul-then-add disagree: proves the fused form is used
    rng = np.random.default_rng(3)
    for _ in range(2000):
        a = rng.standard_normal(8).astype(np.float32)
        b = rng.standard_normal(8).astype(np.float32)
        acc_sep = 0.0
        for x, y in zip(a.tolist(), b.tolist()):
            t = float(x) - float(y)
            acc_sep = acc_sep + t * t
        if acc_sep != canon_sq(a, b):
            assert oracle.sqdist(a, b) == canon_sq(a, b)
            assert oracle.sqdist(a, b) != acc_sep
            return
    pytest.skip("no separating example found")


# --------------------------------------------------------------------------
# Algorithm 1 against a brute-force search over all candidate subsequences
# --------------------------------------------------------------------------

ALPHAS = [(1, 1), (11, 10), (6, 5), (3, 2), (2, 1)]


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_prune_matches_brute_force(dtype):
    rng = np.random.default_rng(10 if dtype == "u8" else 11)
    trials = 0
    for _ in range(120):
        n = int(rng.integers(3, 11))
        dim = int(rng.integers(1, 4))
        if dtype == "u8":
            X = rng.integers(0, 7, (n, dim)).astype(np.uint8)  # heavy ties
        else:
            X = rng.integers(-3, 4, (n, dim)).astype(np.float32) * np.float32(0.5)
        E = Exact(X)
        p = int(rng.integers(0, n))
        m = int(rng.integers(0, n + 3))
        cand = rng.integers(0, n, m).tolist()  # may hold p and duplicates
        num, den = ALPHAS[int(rng.integers(0, len(ALPHAS)))]
        R = [0, 1, 2, 3][int(rng.integers(0, 4))]
        got = oracle.robust_prune(X, p, cand, num, den, R)
        sols = brute_force_prune(E, p, cand, num, den, R)
        assert len(sols) == 1, (X, p, cand, num, den, R, sols)
        assert got == sols[0], (X, p, cand, num, den, R, got, sols)
        trials += 1
    assert trials == 120


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_prune_characterisation_random(dtype):
    """The declarative characterisation on larger random candidate lists."""
    rng = np.random.default_rng(20 if dtype == "u8" else 21)
    n, dim = 60, 8
    if dtype == "u8":
        X = rng.integers(0, 40, (n, dim)).astype(np.uint8)
    else:
        X = rng.standard_normal((n, dim)).astype(np.float32)
    E = Exact(X)
    for t in range(40):
        p = int(rng.integers(0, n))
        cand = rng.integers(0, n, int(rng.integers(5, 70))).tolist()
        num, den = ALPHAS[t % len(ALPHAS)]
        R = [0, 4, 64][t % 3]
        got = oracle.robust_prune(X, p, cand, num, den, R)
        assert characterises(E, p, cand, num, den, R, got)


def test_prune_nonstrict_comparison_matters():
    """Algorithm 1 prunes on alpha * D(p*, p') <= D(p, p') (non-strict): on a
    line, p = 0, p* = 1, p' = 2, alpha = 2 gives 2 * 1 <= 2 -> pruned."""
    X = np.array([[0], [1], [2]], np.uint8)
    assert oracle.robust_prune(X, 0, [1, 2], 2, 1, 0) == [1]
    # a hair above the boundary keeps it
    assert oracle.robust_prune(X, 0, [1, 2], 201, 100, 0) == [1, 2]


def test_prune_alpha_scales_distance_not_square():
    """alpha multiplies D, not D^2: p = 0, p* = 2, p' = 3 (D = 1 vs 3) is pruned
    for alpha = 3 and kept for alpha = 3.01; with alpha on squares it would be
    pruned up to alpha = 9."""
    X = np.array([[0], [2], [3]], np.uint8)
    assert oracle.robust_prune(X, 0, [1, 2], 3, 1, 0) == [1]
    assert oracle.robust_prune(X, 0, [1, 2], 301, 100, 0) == [1, 2]


def test_prune_sorted_ties_by_id_and_order():
    # four candidates at equal distance, pairwise far apart: all kept, in id order
    X = np.array([[10, 10], [10, 20], [20, 10], [10, 0], [0, 10]], np.uint8)
    assert oracle.robust_prune(X, 0, [4, 3, 2, 1], 1, 1, 0) == [1, 2, 3, 4]
    # degree bound stops right after the R-th keep
    assert oracle.robust_prune(X, 0, [4, 3, 2, 1], 1, 1, 2) == [1, 2]


def test_prune_self_duplicates_and_empty():
    X = np.array([[0, 0], [3, 0], [0, 4], [5, 5]], np.uint8)
    assert oracle.robust_prune(X, 0, [], 6, 5, 0) == []
    assert oracle.robust_prune(X, 0, [0, 0], 6, 5, 0) == []
    a = oracle.robust_prune(X, 0, [3, 1, 1, 2, 0, 3], 1, 1, 0)
    b = oracle.robust_prune(X, 0, [1, 2, 3], 1, 1, 0)
    assert a == b
    with pytest.raises(IndexError):
        oracle.robust_prune(X, 0, [1, 4], 1, 1, 0)
    with pytest.raises(ValueError):
        oracle.robust_prune(X, 0, [1], 1, 2, 0)  # alpha < 1


def test_prune_duplicate_of_p_at_alpha_one():
    """A candidate with the coordinates of p, kept first (S = 0), removes every
    other candidate at alpha = 1: 1 * D(p*, p') = D(p, p')."""
    X = np.array([[5, 5], [5, 5], [1, 9], [9, 1], [7, 7]], np.uint8)
    assert oracle.robust_prune(X, 0, [1, 2, 3, 4], 1, 1, 0) == [1]
    assert oracle.robust_prune(X, 0, [1, 2, 3, 4], 11, 10, 0)[0] == 1


def test_prune_huge_alpha_keeps_all_distinct_points_sorted():
    rng = np.random.default_rng(5)
    X = rng.integers(0, 256, (50, 16)).astype(np.uint8)
    X = np.unique(X, axis=0)
    cand = list(range(1, X.shape[0]))
    E = Exact(X)
    got = oracle.robust_prune(X, 0, cand, 10 ** 4, 1, 0)
    assert got == sorted(cand, key=lambda j: (E.S(0, j), j))


def test_prune_collinear_alpha_one_keeps_one_per_side():
    X = np.array([[50], [51], [53], [56], [48], [45], [40]], np.uint8)
    got = oracle.robust_prune(X, 0, list(range(1, 7)), 1, 1, 0)
    assert got == [1, 4]  # nearest on each side


def test_prune_degree_cap_is_prefix_and_idempotent():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((80, 6)).astype(np.float32)
    for t in range(30):
        p = int(rng.integers(0, 80))
        cand = rng.choice(80, 60, replace=False).tolist()
        num, den = ALPHAS[t % len(ALPHAS)]
        full = oracle.robust_prune(X, p, cand, num, den, 0)
        for R in (1, 3, 8):
            assert oracle.robust_prune(X, p, cand, num, den, R) == full[:R]
        # re-pruning an output at the same (alpha, R) returns it unchanged
        assert oracle.robust_prune(X, p, full, num, den, 0) == full
        capped = oracle.robust_prune(X, p, cand, num, den, 5)
        assert oracle.robust_prune(X, p, capped, num, den, 5) == capped


def test_prune_graph_matches_per_node():
    rng = np.random.default_rng(8)
    X = rng.integers(0, 256, (40, 8)).astype(np.uint8)
    nbr = rng.integers(0, 40, (40, 12)).astype(np.int32)
    deg = rng.integers(0, 13, 40).astype(np.int32)
    out, od, pairs = oracle.prune_graph(X, nbr, deg, 11, 10, 5)
    assert pairs > 0
    for p in range(40):
        want = oracle.robust_prune(X, p, nbr[p, :deg[p]], 11, 10, 5)
        assert od[p] == len(want)
        assert out[p, :od[p]].tolist() == want
        assert (out[p, od[p]:] == -1).all()
    nodes = [3, 17, 39]
    out2, od2, _ = oracle.prune_graph(X, nbr, deg, 11, 10, 5, nodes=nodes)
    assert (out2 == out[nodes]).all() and (od2 == od[nodes]).all()


# --------------------------------------------------------------------------
# Worked instances and closed forms from the proofs
# --------------------------------------------------------------------------

def test_lemma37_instance():
    rows, D = _read_fixture("lemma37_instance.txt")
    D = np.array(D, dtype=np.float64)
    Smat = D * D
    a1n, a1d = (int(v) for v in rows["alpha1"])
    a2n, a2d = (int(v) for v in rows["alpha2"])
    base_p = [int(v) for v in rows["base_p"]]
    p, z = 0, 3
    # constraints of Lemma 3.6 (sorted, general metric), scaled by D(p,z) = 6
    x, y = 1, 2
    assert D[y, z] * a1n <= D[p, z] * a1d
    assert D[x, y] * a2n <= D[p, y] * a2d
    assert D[x, y] <= D[p, y] <= D[p, z]
    # triangle inequalities: a metric
    for i in range(4):
        for j in range(4):
            for k in range(4):
                assert D[i, j] <= D[i, k] + D[k, j]
    # the base list is alpha_1-reachable for (p, z)
    assert reach.pair_reach(D, [base_p, [], [], []], p, z) >= a1n / a1d
    got = oracle.robust_prune_smat(Smat, p, base_p, a2n, a2d, 0)
    assert got == [int(v) for v in rows["expect_p"]]
    num, den = (int(v) for v in rows["expect_reach_pz"])
    r = reach.pair_reach(D, [got, [], [], []], p, z)
    assert r == pytest.approx(num / den, rel=1e-15)
    a1, a2 = a1n / a1d, a2n / a2d
    assert r == pytest.approx(reach.sorted_general_bound(a1, a2), rel=1e-15)
    # the printed (uncorrected) assignment violates the lemma's constraint
    assert not (Fraction_le(1, a2n, 1, a1n))  # 1/alpha_2 <= 1/alpha_1 is false


def Fraction_le(an, ad, bn, bd):
    return an * bd <= bn * ad


def test_table1_example_values():
    rows, _ = _read_fixture("table1_example.txt")
    a1 = float(rows["alpha1"][0])
    a2 = float(rows["alpha2"][0])
    approx, tol = float(rows["sorted_euclid_approx"][0]), float(rows["sorted_euclid_approx"][1])
    assert abs(reach.sorted_euclid_bound(a1, a2) - approx) <= tol
    assert reach.sorted_general_bound(a1, a2) == pytest.approx(float(rows["sorted_general"][0]))
    # the Euclidean bound exceeds the general one, which exceeds the unsorted one
    assert reach.sorted_euclid_bound(a1, a2) > reach.sorted_general_bound(a1, a2) > \
        reach.unsorted_bound(a1, a2)


@pytest.mark.parametrize("a1,a2", [(3.0, 2.0), (1.2, 1.1), (2.0, 2.0), (1.5, 1.01)])
def test_appendix_construction(a1, a2):
    p, x, y, z = reach.appendix_points(a1, a2)
    nrm = np.linalg.norm
    assert nrm(y - z) == pytest.approx(1 / a1, rel=1e-12)
    assert nrm(x - y) == pytest.approx(1 / a2, rel=1e-12)
    assert nrm(x - z) == pytest.approx(reach.beta(a1, a2), rel=1e-12)
    t1, t2 = math.asin(1 / (2 * a1)), math.asin(1 / (2 * a2))
    assert reach.beta(a1, a2) == pytest.approx(2 * math.sin(t1 + t2), rel=1e-12)
    # pruned list {x} at p: reachability of (p, z) is exactly 1/beta
    P = np.stack([p, x, y, z])
    D = reach.distance_matrix(P)
    assert reach.pair_reach(D, [[1], [], [], []], 0, 3) == pytest.approx(1 / reach.beta(a1, a2))


def test_unsorted_collinear_example():
    """Lemma 3.5's collinear setting gives D(x,z) = (a1 + a2 + 1)/(a1 a2)."""
    a1, a2 = 3.0, 2.0
    p, z = 0.0, 1.0
    y = z + 1 / a1
    x = y + (abs(y - p)) / a2
    assert abs(x - z) == pytest.approx((a1 + a2 + 1) / (a1 * a2))
    assert 1 / abs(x - z) == pytest.approx(reach.unsorted_bound(a1, a2))


# --------------------------------------------------------------------------
# Graph-level theorems on small random point sets
# --------------------------------------------------------------------------

def _slow_preprocessing(X, num, den):
    """RobustPrune(p, P \\ {p}, alpha, inf) for every p (Lemma 2.2)."""
    n = X.shape[0]
    return [oracle.robust_prune(X, p, [q for q in range(n) if q != p], num, den, 0)
            for p in range(n)]


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("alpha", [(6, 5), (3, 2), (2, 1)])
def test_lemma22_slow_preprocessing_is_alpha_reachable(seed, alpha):
    rng = np.random.default_rng(100 + seed)
    X = rng.standard_normal((30, 3)).astype(np.float32)
    adj = _slow_preprocessing(X, *alpha)
    D = reach.distance_matrix(X)
    a = alpha[0] / alpha[1]
    assert reach.reachability(D, adj) >= a * (1 - 1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("a1,a2", [((3, 1), (2, 1)), ((3, 2), (6, 5)), ((2, 1), (11, 10))])
def test_theorem32_euclidean_bound(seed, a1, a2):
    rng = np.random.default_rng(200 + seed)
    X = rng.standard_normal((28, 2)).astype(np.float32)
    base = _slow_preprocessing(X, *a1)
    pruned = [oracle.robust_prune(X, p, base[p], a2[0], a2[1], 0) for p in range(len(base))]
    D = reach.distance_matrix(X)
    A1, A2 = a1[0] / a1[1], a2[0] / a2[1]
    bound = min(A2, reach.sorted_euclid_bound(A1, A2))
    assert reach.reachability(D, pruned) >= bound * (1 - 1e-9)
    # every pruned list is a subsequence of the base list
    for p in range(len(base)):
        assert set(pruned[p]) <= set(base[p])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_theorem32_general_metric_bound(seed):
    """L1 distances form a (non-Euclidean) metric; sorted RP-Tuning keeps
    reachability >= a1 a2 / (a1 + a2)."""
    rng = np.random.default_rng(300 + seed)
    P = rng.integers(0, 20, (26, 3)).astype(np.float64)
    D = np.abs(P[:, None, :] - P[None, :, :]).sum(axis=2)
    S = D * D
    n = P.shape[0]
    a1, a2 = (3, 1), (2, 1)
    base = [oracle.robust_prune_smat(S, p, [q for q in range(n) if q != p], *a1, 0)
            for p in range(n)]
    pruned = [oracle.robust_prune_smat(S, p, base[p], *a2, 0) for p in range(n)]
    assert reach.reachability(D, base) >= 3.0 * (1 - 1e-12)
    A1, A2 = a1[0] / a1[1], a2[0] / a2[1]
    assert reach.reachability(D, pruned) >= reach.sorted_general_bound(A1, A2) * (1 - 1e-12)


def test_smat_and_points_agree():
    rng = np.random.default_rng(9)
    X = rng.integers(0, 30, (25, 4)).astype(np.uint8)
    E = Exact(X)
    S = np.array([[E.S(i, j) for j in range(25)] for i in range(25)], dtype=np.float64)
    for p in range(25):
        cand = rng.integers(0, 25, 20).tolist()
        assert oracle.robust_prune_smat(S, p, cand, 6, 5, 0) == \
            oracle.robust_prune(X, p, cand, 6, 5, 0)
    assert characterises(ExactMatrix(S), 0, [1, 2, 3], 1, 1, 0,
                         oracle.robust_prune_smat(S, 0, [1, 2, 3], 1, 1, 0))


def test_uint8_decisions_on_the_alpha_boundary():
    """Algorithm 1 prunes p' when alpha D(p*, p') <= D(p, p'), i.e. on squared
    integer distances num^2 S(p*, p') <= den^2 S(p, p'): at equality and at
    S(p*, p') = T = floor(den^2 S(p, p') / num^2) p' is pruned, one unit above
    it is kept.  Pairs built on exactly those relations, for six alphas, with
    lists in and out of rank order; a strict comparison, a rounded threshold or
    alpha applied to squared distances each flips some of them."""
    from boundary_cases import boundary_clusters, cluster_graph

    alphas = [(1, 1), (21, 20), (11, 10), (6, 5), (3, 2), (2, 1)]
    found = boundary_clusters(alphas)
    assert all(len(c) == 4 for (a, kind), c in found.items() if a != (1, 1) or kind != "floor")
    X, nbr, deg, kinds = cluster_graph(found)
    for a in alphas:
        e_nbr, e_deg, _ = oracle.prune_graph(X, nbr, deg, *a, 2)
        for base, ca, kind in kinds:
            if ca != a:
                continue
            want = [base + 1, base + 2] if kind == "above" else [base + 1, -1]
            assert list(e_nbr[base]) == want, (a, kind)
            assert e_deg[base] == (2 if kind == "above" else 1), (a, kind)
