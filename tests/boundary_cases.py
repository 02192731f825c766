"""Exact-boundary uint8 inputs for the integer pruning test of Algorithm 1.

``boundary_clusters`` finds small integer offsets (v to p*, w to p') with
S(p, p*) < S(p, p') that put num^2 S(p*, p') <= den^2 S(p, p') at equality
("eq"), at S(p*, p') = T below the exact ratio ("floor"; none exists for
alpha 1) and at S(p*, p') = T + 1 ("above"), where
T = floor(den^2 S(p, p') / num^2).  ``cluster_graph`` turns them into
three-point clusters (p, p*, p') around the byte value 128 in which only p has
a list, [p*, p'] or, for every other cluster, [p', p*].  The search holds no
pruning arithmetic; the decisions themselves are left to the code under test.
"""
import numpy as np


def boundary_clusters(alphas, per_kind=4, seed=11):
    rng = np.random.default_rng(seed)
    found = {}
    for _ in range(20):
        v = rng.integers(-40, 41, (200_000, 4))
        w = rng.integers(-40, 41, (200_000, 4))
        sv, sw = (v * v).sum(1), (w * w).sum(1)
        s = ((w - v) ** 2).sum(1)
        ok = (sv > 0) & (sv < sw)
        for (num, den) in alphas:
            lhs, rhs = num * num * s, den * den * sw
            t = rhs // (num * num)
            for kind, sel in (("eq", lhs == rhs), ("floor", (lhs != rhs) & (s == t)),
                              ("above", s == t + 1)):
                have = found.setdefault(((num, den), kind), [])
                for i in np.nonzero(ok & sel)[0][: per_kind - len(have)]:
                    have.append((v[i], w[i]))
    # equality is rare at random for den^2 / num^2 near 1: take w = (num, 0, 0, 0),
    # so S(p, p') = num^2, and v on the circle S(p*, p') = den^2 in two dimensions
    for (num, den) in alphas:
        have = found[((num, den), "eq")]
        x, y = np.meshgrid(np.arange(-40, 41), np.arange(-40, 41))
        on = ((x - num) ** 2 + y ** 2 == den * den) & (x * x + y * y > 0) & (x * x + y * y < num * num)
        for xi, yi in zip(x[on], y[on]):
            if len(have) < per_kind:
                have.append((np.array([xi, yi, 0, 0]), np.array([num, 0, 0, 0])))
    return found


def cluster_graph(found, d=16):
    """(X uint8, nbr, deg, kinds): kinds lists (index of p, alpha, kind)."""
    pts, nbr, deg, kinds = [], [], [], []
    for (a, kind), cases in found.items():
        for v, w in cases:
            base = len(pts)
            p = np.full(d, 128, np.int64)
            for off in (np.zeros(4, np.int64), v, w):
                x = p.copy()
                x[:4] += off
                pts.append(x)
            first = [base + 1, base + 2] if (base // 3) % 2 == 0 else [base + 2, base + 1]
            nbr += [first, [-1, -1], [-1, -1]]
            deg += [2, 0, 0]
            kinds.append((base, a, kind))
    return (np.asarray(pts, np.uint8), np.asarray(nbr, np.int32), np.asarray(deg, np.int32),
            kinds)
