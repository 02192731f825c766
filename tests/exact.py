"""Exact-arithmetic helpers for pinning the oracle (no code shared with it).

* ``canon_sq`` evaluates the canonical FP64 squared distance of two float32
  rows from its definition -- t_k = fl(a_k - b_k), acc = fma(t_k, t_k, acc) in
  ascending k -- with the fused multiply-add done exactly in rationals and
  rounded once (CPython's int / int division is correctly rounded).
* ``characterises`` is a declarative description of RobustPrune's output
  (Algorithm 1): given the order of the candidates by (S(p, .), id), a list K
  is the output iff (i) K is a duplicate-free subsequence of that order,
  (ii) no j in K has an earlier kept i with the pruning condition true,
  (iii) every other candidate has such an earlier kept witness, except the
  ones after the R-th keep, which Algorithm 1 drops at its ``break``, and
  (iv) |K| <= R.  These conditions fix K uniquely (induction along the order).
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from typing import List, Sequence

import numpy as np


def fma_exact(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def canon_sq(a: np.ndarray, b: np.ndarray) -> float:
    acc = 0.0
    for x, y in zip(a.tolist(), b.tolist()):
        t = float(x) - float(y)
        acc = fma_exact(t, t, acc)
    return acc


def int_sq(a: np.ndarray, b: np.ndarray) -> int:
    return sum((int(x) - int(y)) ** 2 for x, y in zip(a.tolist(), b.tolist()))


class Exact:
    """Squared distances and the pruning condition for one point set."""

    def __init__(self, X: np.ndarray):
        self.X = X
        self.is_int = X.dtype == np.uint8
        self._cache = {}

    def S(self, a: int, b: int):
        key = (a, b) if a <= b else (b, a)
        if key not in self._cache:
            f = int_sq if self.is_int else canon_sq
            self._cache[key] = f(self.X[key[0]], self.X[key[1]])
        return self._cache[key]

    def test(self, num: int, den: int, i: int, j: int, p: int) -> bool:
        """alpha * D(i, j) <= D(p, j) with alpha = num/den, on squares."""
        if self.is_int:
            return num * num * self.S(i, j) <= den * den * self.S(p, j)
        return float(num * num) * self.S(i, j) <= float(den * den) * self.S(p, j)


class ExactMatrix(Exact):
    def __init__(self, Smat):
        self.Smat = Smat
        self.is_int = False

    def S(self, a: int, b: int):
        return float(self.Smat[a][b])


def candidate_order(E: Exact, p: int, cand: Sequence[int]) -> List[int]:
    V = sorted(set(int(c) for c in cand) - {p})
    return sorted(V, key=lambda j: (E.S(p, j), j))


def characterises(E: Exact, p: int, cand: Sequence[int], num: int, den: int, R: int,
                  K: Sequence[int]) -> bool:
    order = candidate_order(E, p, cand)
    pos = {j: t for t, j in enumerate(order)}
    K = [int(v) for v in K]
    if len(set(K)) != len(K) or any(v not in pos for v in K):
        return False
    if any(pos[K[t]] >= pos[K[t + 1]] for t in range(len(K) - 1)):
        return False
    if R > 0 and len(K) > R:
        return False
    capped = R > 0 and len(K) == R
    last = pos[K[-1]] if K else -1
    kept = set(K)
    for j in order:
        earlier = [i for i in K if pos[i] < pos[j]]
        hit = any(E.test(num, den, i, j, p) for i in earlier)
        if j in kept:
            if hit:
                return False
        else:
            if capped and pos[j] > last:
                continue
            if not hit:
                return False
    return True


def brute_force_prune(E: Exact, p: int, cand: Sequence[int], num: int, den: int, R: int):
    """Every subsequence of the candidate order that the characterisation
    accepts (there must be exactly one)."""
    order = candidate_order(E, p, cand)
    found = []
    for r in range(len(order) + 1):
        for sub in itertools.combinations(order, r):
            if characterises(E, p, cand, num, den, R, sub):
                found.append(list(sub))
    return found
