"""ctypes binding of the C oracle (TEST INFRASTRUCTURE ONLY).

Argument marshalling only: every step of RobustPrune, RP-Tuning and
GreedySearch runs in ``rpo.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

U8 = 1
F32 = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rpo.c")
_LIB = os.path.join(_HERE, "librpo.so")
_lib = None

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)


def lib_path() -> str:
    return _LIB


def build() -> str:
    """Compile the oracle with gcc.  -ffp-contract=off keeps the canonical FP64
    evaluation order (no fused multiply-add except the explicit fma calls)."""
    cmd = [
        "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
        "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp", "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    lib.rpo_sqdist_u8.restype = C.c_int64
    lib.rpo_sqdist_u8.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
    lib.rpo_sqdist_f32.restype = C.c_double
    lib.rpo_sqdist_f32.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
    lib.rpo_robust_prune.restype = C.c_int32
    lib.rpo_robust_prune.argtypes = [
        C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_int32, _i32p, C.c_int32,
        C.c_int32, C.c_int32, C.c_int32, _i32p, _i64p]
    lib.rpo_robust_prune_unsorted.restype = C.c_int32
    lib.rpo_robust_prune_unsorted.argtypes = lib.rpo_robust_prune.argtypes
    lib.rpo_robust_prune_smat.restype = C.c_int32
    lib.rpo_robust_prune_smat.argtypes = [
        _f64p, C.c_int32, C.c_int32, _i32p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _i32p]
    lib.rpo_robust_prune_unsorted_smat.restype = C.c_int32
    lib.rpo_robust_prune_unsorted_smat.argtypes = lib.rpo_robust_prune_smat.argtypes
    lib.rpo_prune_graph.restype = C.c_int32
    lib.rpo_prune_graph.argtypes = [
        C.c_void_p, C.c_int32, C.c_int64, C.c_int32, _i32p, _i32p, C.c_int32,
        _i32p, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _i32p, _i32p, _i64p]
    lib.rpo_prune_graph_unsorted.restype = C.c_int32
    lib.rpo_prune_graph_unsorted.argtypes = lib.rpo_prune_graph.argtypes
    lib.rpo_search.restype = C.c_int32
    lib.rpo_search.argtypes = [
        C.c_void_p, C.c_int32, C.c_int64, C.c_int32, _i32p, _i32p, C.c_int32,
        C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, _i32p, _f64p, _i32p]
    lib.rpo_groundtruth.restype = C.c_int32
    lib.rpo_groundtruth.argtypes = [
        C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_int64, C.c_int32, _i32p]
    _lib = lib
    return lib


def _dtype_code(X: np.ndarray) -> int:
    if X.dtype == np.uint8:
        return U8
    if X.dtype == np.float32:
        return F32
    raise TypeError(f"unsupported point dtype {X.dtype}")


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _check(rc: int, what: str) -> int:
    if rc == -1:
        raise ValueError(f"{what}: invalid argument")
    if rc == -2:
        raise IndexError(f"{what}: id out of range")
    return rc


def sqdist(a: np.ndarray, b: np.ndarray):
    """Squared distance: exact int for uint8, canonical FP64 for float32."""
    lib = _load()
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    assert a.shape == b.shape and a.ndim == 1 and a.dtype == b.dtype
    if a.dtype == np.uint8:
        return int(lib.rpo_sqdist_u8(a.ctypes.data, b.ctypes.data, a.shape[0]))
    return float(lib.rpo_sqdist_f32(a.ctypes.data, b.ctypes.data, a.shape[0]))


def robust_prune(X: np.ndarray, p: int, cand, num: int, den: int, R: int = 0,
                 count_pairs: bool = False, unsorted: bool = False):
    """RobustPrune(p, cand, alpha=num/den, R) (Algorithm 1).  R <= 0: no bound.
    unsorted: UnsortedRobustPrune (Section 3), p* = the first remaining
    candidate in list order."""
    lib = _load()
    fn = lib.rpo_robust_prune_unsorted if unsorted else lib.rpo_robust_prune
    X = np.ascontiguousarray(X)
    cand = np.ascontiguousarray(np.asarray(cand, dtype=np.int32))
    m = cand.shape[0]
    out = np.full(max(m, 1), -1, dtype=np.int32)
    pairs = np.zeros(1, dtype=np.int64)
    rc = fn(X.ctypes.data, _dtype_code(X), X.shape[0], X.shape[1], int(p),
            _ptr(cand, _i32p), m, int(num), int(den), int(R),
            _ptr(out, _i32p), _ptr(pairs, _i64p))
    k = _check(rc, "robust_prune")
    res = [int(v) for v in out[:k]]
    return (res, int(pairs[0])) if count_pairs else res


def robust_prune_smat(Smat: np.ndarray, p: int, cand, num: int, den: int, R: int = 0,
                      unsorted: bool = False):
    """RobustPrune (or UnsortedRobustPrune) on an explicit matrix of squared
    distances."""
    lib = _load()
    fn = lib.rpo_robust_prune_unsorted_smat if unsorted else lib.rpo_robust_prune_smat
    Smat = np.ascontiguousarray(Smat, dtype=np.float64)
    cand = np.ascontiguousarray(np.asarray(cand, dtype=np.int32))
    m = cand.shape[0]
    out = np.full(max(m, 1), -1, dtype=np.int32)
    rc = fn(_ptr(Smat, _f64p), Smat.shape[0], int(p), _ptr(cand, _i32p),
            m, int(num), int(den), int(R), _ptr(out, _i32p))
    k = _check(rc, "robust_prune_smat")
    return [int(v) for v in out[:k]]


def prune_graph(X: np.ndarray, nbr: np.ndarray, deg: np.ndarray, num: int, den: int, R: int,
                nodes=None, unsorted: bool = False, threads: int = 1):
    """RP-Tuning at alpha=num/den with degree bound R over all nodes, or over
    ``nodes`` only.  Returns (out_nbr [len x R, -1 padded], out_deg, pairs).
    unsorted: UnsortedRobustPrune in place of RobustPrune.  threads > 1 runs
    the single-threaded oracle on that many disjoint node shards at once (the
    vertices are independent); the result does not depend on it."""
    if threads > 1:
        return _prune_graph_sharded(X, nbr, deg, num, den, R, nodes, unsorted, threads)
    lib = _load()
    fn = lib.rpo_prune_graph_unsorted if unsorted else lib.rpo_prune_graph
    X = np.ascontiguousarray(X)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    deg = np.ascontiguousarray(deg, dtype=np.int32)
    if nodes is None:
        cnt = X.shape[0]
        nodes_p = None
    else:
        nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.int32))
        cnt = nodes.shape[0]
        nodes_p = _ptr(nodes, _i32p)
    out_nbr = np.empty((cnt, R), dtype=np.int32)
    out_deg = np.empty(cnt, dtype=np.int32)
    pairs = np.zeros(1, dtype=np.int64)
    rc = fn(X.ctypes.data, _dtype_code(X), X.shape[0], X.shape[1],
            _ptr(nbr, _i32p), _ptr(deg, _i32p), nbr.shape[1],
            nodes_p, cnt, int(num), int(den), int(R),
            _ptr(out_nbr, _i32p), _ptr(out_deg, _i32p), _ptr(pairs, _i64p))
    _check(rc, "prune_graph")
    return out_nbr, out_deg, int(pairs[0])


def _prune_graph_sharded(X, nbr, deg, num, den, R, nodes, unsorted, threads):
    """prune_graph over contiguous shards of the node list, one thread each
    (ctypes releases the interpreter lock during the call)."""
    from concurrent.futures import ThreadPoolExecutor

    X = np.ascontiguousarray(X)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    deg = np.ascontiguousarray(deg, dtype=np.int32)
    nodes = np.arange(X.shape[0], dtype=np.int32) if nodes is None else \
        np.ascontiguousarray(np.asarray(nodes, dtype=np.int32))
    parts = [p for p in np.array_split(nodes, threads) if p.size]
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        res = list(ex.map(lambda part: prune_graph(X, nbr, deg, num, den, R, nodes=part,
                                                   unsorted=unsorted), parts))
    if not res:
        return np.empty((0, R), np.int32), np.empty(0, np.int32), 0
    return (np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res]),
            sum(r[2] for r in res))


def search(X: np.ndarray, nbr: np.ndarray, deg: np.ndarray, start: int, Q: np.ndarray,
           k: int, L: int):
    """GreedySearch (Algorithm 2) for every query row.
    Returns (ids [nq x k, -1 padded], squared distances [nq x k], hops [nq])."""
    lib = _load()
    X = np.ascontiguousarray(X)
    Q = np.ascontiguousarray(Q, dtype=X.dtype)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    deg = np.ascontiguousarray(deg, dtype=np.int32)
    nq = Q.shape[0]
    ids = np.empty((nq, k), dtype=np.int32)
    dist = np.empty((nq, k), dtype=np.float64)
    hops = np.empty(nq, dtype=np.int32)
    rc = lib.rpo_search(X.ctypes.data, _dtype_code(X), X.shape[0], X.shape[1],
                        _ptr(nbr, _i32p), _ptr(deg, _i32p), nbr.shape[1], int(start),
                        Q.ctypes.data, nq, int(k), int(L), _ptr(ids, _i32p), _ptr(dist, _f64p),
                        _ptr(hops, _i32p))
    _check(rc, "search")
    return ids, dist, hops


def groundtruth(X: np.ndarray, Q: np.ndarray, k: int, threads: int = 1):
    """Exact k nearest points of each query by (S, id), brute force.
    threads > 1 runs the single-threaded routine on disjoint query shards."""
    if threads > 1 and Q.shape[0] > 1:
        from concurrent.futures import ThreadPoolExecutor

        parts = [p for p in np.array_split(np.arange(Q.shape[0]), threads) if p.size]
        with ThreadPoolExecutor(max_workers=len(parts)) as ex:
            res = list(ex.map(lambda idx: groundtruth(X, Q[idx], k), parts))
        return np.concatenate(res)
    lib = _load()
    X = np.ascontiguousarray(X)
    Q = np.ascontiguousarray(Q, dtype=X.dtype)
    ids = np.empty((Q.shape[0], k), dtype=np.int32)
    rc = lib.rpo_groundtruth(X.ctypes.data, _dtype_code(X), X.shape[0], X.shape[1],
                             Q.ctypes.data, Q.shape[0], int(k), _ptr(ids, _i32p))
    _check(rc, "groundtruth")
    return ids


def recall_at_k(ids: np.ndarray, gt: np.ndarray, k: int) -> float:
    """k-recall@k (Section 4): the share of the true k nearest neighbours found
    among the k returned ids, averaged over queries."""
    ids = np.asarray(ids)[:, :k]
    gt = np.asarray(gt)[:, :k]
    hit = 0
    for a, b in zip(ids, gt):
        hit += len(set(int(v) for v in a if v >= 0) & set(int(v) for v in b))
    return hit / (k * ids.shape[0]) if ids.shape[0] else 0.0
