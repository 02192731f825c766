"""Thin Python binding of the C-ABI in include/rp.h (ctypes; argument
marshalling only -- every step of pruning and search runs in the HIP kernels).

Tensors must be CUDA (HIP) tensors on the current device; the calls enqueue on
torch's current stream unless a stream is given.  The binding raises if the
HIP library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "librp.so")

RP_U8 = 1
RP_F32 = 2
_STATUS = {0: "RP_OK", 1: "RP_EINVAL", 2: "RP_ERANGE", 3: "RP_ENOMEM", 4: "RP_EDEVICE",
           5: "RP_ESTATE"}


class RPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Alpha(C.Structure):
    _fields_ = [("num", C.c_int32), ("den", C.c_int32)]


class Counters(C.Structure):
    _fields_ = [("nodes", C.c_int64), ("rechecks", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("type", C.c_int32), ("alpha", Alpha), ("R", C.c_int32),
                ("queries", C.c_void_p), ("nq", C.c_int64), ("k", C.c_int32), ("L", C.c_int32),
                ("out_ids", C.c_void_p), ("out_dist", C.c_void_p), ("out_hops", C.c_void_p),
                ("tag", C.c_int64)]


class Completion(C.Structure):
    _fields_ = [("tag", C.c_int64), ("status", C.c_int32), ("batch", C.c_int32),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("sweeps", C.c_int64), ("swept_alphas", C.c_int64), ("searches", C.c_int64),
                ("searched_queries", C.c_int64), ("evictions", C.c_int64),
                ("resident_graphs", C.c_int64), ("resident_bytes", C.c_int64)]


REQ_PRUNE = 1
REQ_QUERY = 2

EXPORTS = ["rp_load_graph", "rp_graph_derive", "rp_prune", "rp_prune_sweep", "rp_prune_plain",
           "rp_prune_sweep_unsorted", "rp_knn_u8", "rp_knn_u8_noalloc", "rp_f32_band", "rp_build_slow",
           "rp_search", "rp_read_counters", "rp_free_graph", "rp_last_error",
           "rp_plan_sweep", "rp_plan_launch", "rp_plan_free",
           "rp_autotune_sweep", "rp_tune_set", "rp_tune_get", "rp_gram_error",
           "rp_server_create", "rp_server_submit", "rp_server_poll", "rp_server_replay",
           "rp_server_stats_get", "rp_server_destroy"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load librp.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.rp_load_graph.restype = i32
    lib.rp_load_graph.argtypes = [vp, i32, i64, i32, vp, vp, i32, i32, vp, C.POINTER(vp)]
    lib.rp_graph_derive.restype = i32
    lib.rp_graph_derive.argtypes = [vp, vp, vp, i32, vp, C.POINTER(vp)]
    lib.rp_prune.restype = i32
    lib.rp_prune.argtypes = [vp, Alpha, i32, vp, vp, vp]
    lib.rp_prune_plain.restype = i32
    lib.rp_prune_plain.argtypes = [vp, Alpha, i32, vp, vp, vp]
    lib.rp_prune_sweep.restype = i32
    lib.rp_prune_sweep.argtypes = [vp, C.POINTER(Alpha), i32, C.POINTER(i32), i32,
                                   C.POINTER(vp), C.POINTER(vp), vp]
    lib.rp_prune_sweep_unsorted.restype = i32
    lib.rp_prune_sweep_unsorted.argtypes = lib.rp_prune_sweep.argtypes
    lib.rp_knn_u8.restype = i32
    lib.rp_knn_u8.argtypes = [vp, i64, i32, vp, i64, vp, i64, i32, vp, vp]
    lib.rp_knn_u8_noalloc.restype = i32
    lib.rp_knn_u8_noalloc.argtypes = [vp, i64, i32, vp, i64, vp, i64, i32, i32, vp, vp]
    lib.rp_build_slow.restype = i32
    lib.rp_build_slow.argtypes = [vp, i32, i64, i32, Alpha, i32, vp, vp, vp]
    lib.rp_f32_band.restype = i32
    lib.rp_f32_band.argtypes = [i32, C.POINTER(C.c_double)]
    lib.rp_search.restype = i32
    lib.rp_search.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp, vp]
    lib.rp_read_counters.restype = i32
    lib.rp_read_counters.argtypes = [vp, C.POINTER(Counters), i32, vp]
    lib.rp_free_graph.restype = None
    lib.rp_free_graph.argtypes = [vp]
    lib.rp_last_error.restype = C.c_char_p
    lib.rp_last_error.argtypes = []
    lib.rp_plan_sweep.restype = i32
    lib.rp_plan_sweep.argtypes = [vp, C.POINTER(Alpha), i32, C.POINTER(i32), i32,
                                  C.POINTER(vp), C.POINTER(vp), vp, C.POINTER(vp)]
    lib.rp_plan_launch.restype = i32
    lib.rp_plan_launch.argtypes = [vp, vp]
    lib.rp_plan_free.restype = None
    lib.rp_plan_free.argtypes = [vp]
    lib.rp_autotune_sweep.restype = i32
    lib.rp_autotune_sweep.argtypes = [vp, C.POINTER(Alpha), i32, C.POINTER(i32), i32,
                                      C.POINTER(vp), C.POINTER(vp), vp, C.POINTER(i32),
                                      C.POINTER(C.c_float)]
    lib.rp_gram_error.restype = i32
    lib.rp_gram_error.argtypes = [vp, vp, i64, C.POINTER(C.c_double), vp]
    lib.rp_tune_set.restype = i32
    lib.rp_tune_set.argtypes = [vp, i32, i32, i32]
    lib.rp_tune_get.restype = i32
    lib.rp_tune_get.argtypes = [vp, i32, i32, C.POINTER(i32)]
    lib.rp_server_create.restype = i32
    lib.rp_server_create.argtypes = [vp, i64, i32, i32, i32, C.POINTER(vp)]
    lib.rp_server_submit.restype = i32
    lib.rp_server_submit.argtypes = [vp, C.POINTER(Request)]
    lib.rp_server_poll.restype = i32
    lib.rp_server_poll.argtypes = [vp, C.POINTER(Completion), i32, i32]
    lib.rp_server_replay.restype = i32
    lib.rp_server_replay.argtypes = [vp, C.POINTER(Request), C.POINTER(C.c_double), i32,
                                     C.POINTER(Completion)]
    lib.rp_server_stats_get.restype = i32
    lib.rp_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
    lib.rp_server_destroy.restype = None
    lib.rp_server_destroy.argtypes = [vp]
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise RPError(rc, _lib.rp_last_error().decode())


def _stream_ptr(stream) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.uint8:
        return RP_U8
    if t.dtype == torch.float32:
        return RP_F32
    raise TypeError(f"points must be uint8 or float32, got {t.dtype}")


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("arguments must be contiguous device tensors")


def as_alpha(a) -> Tuple[int, int]:
    """(num, den) from a tuple or a fractions.Fraction."""
    if isinstance(a, tuple):
        return int(a[0]), int(a[1])
    return int(a.numerator), int(a.denominator)


def knn_u8(points: torch.Tensor, K: int, query_ids: Optional[torch.Tensor] = None,
           cand_ids: Optional[torch.Tensor] = None, nq: Optional[int] = None,
           nc: Optional[int] = None, out: Optional[torch.Tensor] = None, stream=None):
    """Exact K nearest neighbours (rp_knn_u8): an (nq, K) int32 tensor of
    candidate ids in ascending (S, id) order, the query itself excluded, -1
    padded.  query_ids / cand_ids: int32 device tensors of point ids (None:
    the first nq / nc points, by default all of them)."""
    lib = load_library()
    _need_cuda(points, query_ids, cand_ids)
    if points.dtype != torch.uint8 or points.dim() != 2:
        raise TypeError("points must be a 2-D uint8 tensor")
    for t in (query_ids, cand_ids):
        if t is not None and t.dtype != torch.int32:
            raise TypeError("ids must be int32")
    n, d = points.shape
    nq = int(query_ids.numel()) if query_ids is not None else int(n if nq is None else nq)
    nc = int(cand_ids.numel()) if cand_ids is not None else int(n if nc is None else nc)
    if out is None:
        out = torch.empty((nq, int(K)), dtype=torch.int32, device=points.device)
    _need_cuda(out)
    if tuple(out.shape) != (nq, int(K)) or out.dtype != torch.int32:
        raise ValueError(f"out must be int32 ({nq}, {K})")
    _check(lib.rp_knn_u8(points.data_ptr(), n, d, _ptr(query_ids), nq, _ptr(cand_ids), nc,
                         int(K), out.data_ptr(), _stream_ptr(stream)))
    return out


def knn_u8_sets(points: torch.Tensor, K: int, sets, stream=None) -> torch.Tensor:
    """Restricted exact K-NN lists with rp_knn_u8: `sets` holds (query ids,
    candidate ids) pairs (int32 arrays or device tensors); each query's list
    is its K nearest candidates by (S, id), itself excluded.  Returns an
    (n, K) int32 tensor, -1 padded and -1 for points in no set."""
    n = points.shape[0]
    out = torch.full((n, int(K)), -1, dtype=torch.int32, device=points.device)
    for q, c in sets:
        q = torch.as_tensor(q, dtype=torch.int32).to(points.device)
        c = torch.as_tensor(c, dtype=torch.int32).to(points.device)
        if q.numel() == 0:
            continue
        out[q.long()] = knn_u8(points, K, query_ids=q, cand_ids=c, stream=stream)
    return out


def build_slow(points: torch.Tensor, alpha, R: int, stream=None):
    """The slow-preprocessing graph (rp_build_slow): RobustPrune(p, P \\ {p},
    alpha, R) for every point; returns (nbr [n, R] int32, deg [n] int32)."""
    lib = load_library()
    _need_cuda(points)
    num, den = as_alpha(alpha)
    n, d = points.shape
    nb = torch.empty((n, int(R)), dtype=torch.int32, device=points.device)
    dg = torch.empty(n, dtype=torch.int32, device=points.device)
    _check(lib.rp_build_slow(points.data_ptr(), _dtype_code(points), n, d, Alpha(num, den),
                             int(R), nb.data_ptr(), dg.data_ptr(), _stream_ptr(stream)))
    return nb, dg


def f32_band(d: int) -> Tuple[float, float, float, int]:
    """(c1, c2, c3, chunk) of the float32 kernel's rounding band at dimension
    d and its accumulator chunk length (rp_f32_band; host only)."""
    lib = load_library()
    out = (C.c_double * 4)()
    _check(lib.rp_f32_band(int(d), out))
    return out[0], out[1], out[2], int(out[3])


def knn_u8_noalloc(points: torch.Tensor, K: int, out: torch.Tensor,
                   query_ids: Optional[torch.Tensor] = None,
                   cand_ids: Optional[torch.Tensor] = None, nq: Optional[int] = None,
                   nc: Optional[int] = None, slices: int = 0, stream=None) -> torch.Tensor:
    """rp_knn_u8_noalloc: knn_u8 into the caller's `out` with the library's
    fixed workspace (no device allocation); `slices` as in include/rp.h."""
    lib = load_library()
    _need_cuda(points, query_ids, cand_ids, out)
    if points.dtype != torch.uint8 or points.dim() != 2:
        raise TypeError("points must be a 2-D uint8 tensor")
    n, d = points.shape
    nq = int(query_ids.numel()) if query_ids is not None else int(n if nq is None else nq)
    nc = int(cand_ids.numel()) if cand_ids is not None else int(n if nc is None else nc)
    if tuple(out.shape) != (nq, int(K)) or out.dtype != torch.int32:
        raise ValueError(f"out must be int32 ({nq}, {K})")
    _check(lib.rp_knn_u8_noalloc(points.data_ptr(), n, d, _ptr(query_ids), nq, _ptr(cand_ids),
                                 nc, int(K), int(slices), out.data_ptr(), _stream_ptr(stream)))
    return out


class Graph:
    """A borrowed point set + adjacency registered with the library.

    The tensors passed in are kept referenced by this object so that they
    outlive the handle."""

    def __init__(self, points: torch.Tensor, nbr: torch.Tensor, deg: torch.Tensor, start: int,
                 stream=None, _base: "Graph" = None):
        lib = load_library()
        _need_cuda(points, nbr, deg)
        if nbr.dtype != torch.int32 or deg.dtype != torch.int32:
            raise TypeError("nbr and deg must be int32")
        self.points, self.nbr, self.deg = points, nbr, deg
        self.n, self.d = points.shape
        self.r_max = nbr.shape[1]
        self.start = int(start)
        self._base = _base
        h = C.c_void_p()
        if _base is None:
            rc = lib.rp_load_graph(points.data_ptr(), _dtype_code(points), self.n, self.d,
                                   nbr.data_ptr(), deg.data_ptr(), self.r_max, self.start,
                                   _stream_ptr(stream), C.byref(h))
        else:
            rc = lib.rp_graph_derive(_base.handle, nbr.data_ptr(), deg.data_ptr(), self.r_max,
                                     _stream_ptr(stream), C.byref(h))
        _check(rc)
        self.handle = h

    def derive(self, nbr: torch.Tensor, deg: torch.Tensor, stream=None) -> "Graph":
        return Graph(self.points, nbr, deg, self.start, stream, _base=self)

    def _check_out(self, nb: torch.Tensor, dg: torch.Tensor, R: int):
        _need_cuda(nb, dg)
        if nb.dtype != torch.int32 or dg.dtype != torch.int32:
            raise TypeError("outputs must be int32")
        if tuple(nb.shape) != (self.n, R) or tuple(dg.shape) != (self.n,):
            raise ValueError(f"outputs must be ({self.n}, {R}) and ({self.n},)")

    def _outs(self, R: int):
        dev = self.points.device
        return (torch.empty((self.n, R), dtype=torch.int32, device=dev),
                torch.empty(self.n, dtype=torch.int32, device=dev))

    def prune(self, alpha, R: int, out=None, stream=None):
        num, den = as_alpha(alpha)
        nb, dg = out if out is not None else self._outs(R)
        self._check_out(nb, dg, R)
        _check(_lib.rp_prune(self.handle, Alpha(num, den), int(R), nb.data_ptr(), dg.data_ptr(),
                             _stream_ptr(stream)))
        return nb, dg

    def prune_plain(self, alpha, R: int, out=None, stream=None):
        num, den = as_alpha(alpha)
        nb, dg = out if out is not None else self._outs(R)
        self._check_out(nb, dg, R)
        _check(_lib.rp_prune_plain(self.handle, Alpha(num, den), int(R), nb.data_ptr(),
                                   dg.data_ptr(), _stream_ptr(stream)))
        return nb, dg

    def prune_sweep(self, alphas: Sequence, Rs: Sequence[int], outs=None, stream=None,
                    unsorted: bool = False):
        """Returns a list of (nbr, deg) in order o = ia * len(Rs) + iR.
        unsorted: UnsortedRobustPrune (rp_prune_sweep_unsorted)."""
        al = [as_alpha(a) for a in alphas]
        na, nr = len(al), len(Rs)
        if outs is None:
            outs = [self._outs(Rs[o % nr]) for o in range(na * nr)]
        for o, (nb, dg) in enumerate(outs):
            self._check_out(nb, dg, int(Rs[o % nr]))
        A = (Alpha * na)(*[Alpha(a, b) for a, b in al])
        RR = (C.c_int32 * nr)(*[int(r) for r in Rs])
        NB = (C.c_void_p * (na * nr))(*[o[0].data_ptr() for o in outs])
        DG = (C.c_void_p * (na * nr))(*[o[1].data_ptr() for o in outs])
        fn = _lib.rp_prune_sweep_unsorted if unsorted else _lib.rp_prune_sweep
        _check(fn(self.handle, A, na, RR, nr, NB, DG, _stream_ptr(stream)))
        return outs

    def plan_sweep(self, alphas: Sequence, Rs: Sequence[int], outs=None, stream=None) -> "Plan":
        """Capture prune_sweep(alphas, Rs, outs) into a HIP graph (nothing runs);
        Plan.launch() replays it.  `stream` must not be the default stream."""
        al = [as_alpha(a) for a in alphas]
        na, nr = len(al), len(Rs)
        if outs is None:
            outs = [self._outs(Rs[o % nr]) for o in range(na * nr)]
        for o, (nb, dg) in enumerate(outs):
            self._check_out(nb, dg, int(Rs[o % nr]))
        A = (Alpha * na)(*[Alpha(a, b) for a, b in al])
        RR = (C.c_int32 * nr)(*[int(r) for r in Rs])
        NB = (C.c_void_p * (na * nr))(*[o[0].data_ptr() for o in outs])
        DG = (C.c_void_p * (na * nr))(*[o[1].data_ptr() for o in outs])
        h = C.c_void_p()
        _check(_lib.rp_plan_sweep(self.handle, A, na, RR, nr, NB, DG, _stream_ptr(stream),
                                  C.byref(h)))
        return Plan(h, self, outs)

    def _tune_key(self, na: int, nr: int) -> str:
        return f"{'u8' if self.points.dtype == torch.uint8 else 'f32'}:d{self.d}:r{self.r_max}:a{na}:R{nr}"

    def autotune_sweep(self, alphas: Sequence, Rs: Sequence[int], outs=None, cache: str = None,
                       stream=None) -> dict:
        """Choose the vertices per workgroup of the batched kernel for this
        graph shape and sweep shape (timed on this graph, or read from the
        JSON file `cache`, which then records the choice).  Returns
        {"waves": w, "ms": [per candidate 1, 2, 4, 8] or None, "cached": bool}."""
        import json

        al = [as_alpha(a) for a in alphas]
        na, nr = len(al), len(Rs)
        key = self._tune_key(na, nr)
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            _check(_lib.rp_tune_set(self.handle, na, nr, int(table[key]["waves"])))
            return {"waves": int(table[key]["waves"]), "ms": table[key].get("ms"), "cached": True}
        if outs is None:
            outs = [self._outs(Rs[o % nr]) for o in range(na * nr)]
        for o, (nb, dg) in enumerate(outs):
            self._check_out(nb, dg, int(Rs[o % nr]))
        A = (Alpha * na)(*[Alpha(a, b) for a, b in al])
        RR = (C.c_int32 * nr)(*[int(r) for r in Rs])
        NB = (C.c_void_p * (na * nr))(*[o[0].data_ptr() for o in outs])
        DG = (C.c_void_p * (na * nr))(*[o[1].data_ptr() for o in outs])
        w = C.c_int32()
        ms = (C.c_float * 4)()
        _check(_lib.rp_autotune_sweep(self.handle, A, na, RR, nr, NB, DG, _stream_ptr(stream),
                                      C.byref(w), ms))
        res = {"waves": int(w.value), "ms": [float(x) for x in ms], "cached": False}
        if cache:
            table[key] = {"waves": res["waves"], "ms": res["ms"]}
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return res

    def gram_error(self, nodes: torch.Tensor, stream=None) -> dict:
        """Measured error of the float32 kernel's approximate candidate
        distances on the listed vertices (see rp_gram_error)."""
        _need_cuda(nodes)
        if nodes.dtype != torch.int32:
            raise TypeError("nodes must be int32")
        out = (C.c_double * 4)()
        _check(_lib.rp_gram_error(self.handle, nodes.data_ptr(), nodes.numel(), out,
                                  _stream_ptr(stream)))
        return {"max_rel": out[0], "mean_rel": out[1], "pairs": int(out[2]),
                "max_err_over_bound": out[3]}

    def search(self, Q: torch.Tensor, k: int, L: int, want_dist: bool = True, stream=None):
        _need_cuda(Q)
        if Q.dtype != self.points.dtype or Q.shape[1] != self.d:
            raise ValueError("queries must match the points' dtype and dimension")
        nq = Q.shape[0]
        dev = self.points.device
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        dist = torch.empty((nq, k), dtype=torch.float64, device=dev) if want_dist else None
        hops = torch.empty(nq, dtype=torch.int32, device=dev)
        _check(_lib.rp_search(self.handle, Q.data_ptr(), nq, int(k), int(L), ids.data_ptr(),
                              dist.data_ptr() if dist is not None else None, hops.data_ptr(),
                              _stream_ptr(stream)))
        return ids, dist, hops

    def counters(self, reset: bool = False, stream=None) -> dict:
        c = Counters()
        _check(_lib.rp_read_counters(self.handle, C.byref(c), 1 if reset else 0,
                                     _stream_ptr(stream)))
        return {"nodes": c.nodes, "rechecks": c.rechecks}

    def free(self):
        if getattr(self, "handle", None) is not None and self.handle.value is not None:
            _lib.rp_free_graph(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Plan:
    """A captured sweep (keeps its graph and outputs alive)."""

    def __init__(self, handle, graph: Graph, outs):
        self.handle, self.graph, self.outs = handle, graph, outs

    def launch(self, stream=None):
        _check(_lib.rp_plan_launch(self.handle, _stream_ptr(stream)))
        return self.outs

    def free(self):
        if getattr(self, "handle", None) is not None and self.handle.value is not None:
            _lib.rp_plan_free(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _ptr(t: Optional[torch.Tensor]):
    return t.data_ptr() if t is not None else None


class Server:
    """Request loop over a resident base graph (include/rp_serve.h).

    fifo: 0 continuous batching; 1 one request at a time (batched kernel, one
    alpha per launch); 2 one request at a time with the plain prune kernel.

    Requests are built with prune_request()/query_request(); the tensors they
    reference are kept alive by this object until the request completes
    (completions are matched by tag)."""

    def __init__(self, base: Graph, budget_bytes: int, n_streams: int = 4,
                 max_query_batch: int = 4096, fifo: int = 0):
        lib = load_library()
        if base._base is not None:
            raise ValueError("the server needs a base graph, not a derived one")
        self.base = base
        h = C.c_void_p()
        _check(lib.rp_server_create(base.handle, int(budget_bytes), int(n_streams),
                                    int(max_query_batch), int(fifo), C.byref(h)))
        self.handle = h
        self._keep = {}

    def prune_request(self, alpha, R: int, out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
                      tag: int = 0) -> Request:
        num, den = as_alpha(alpha)
        nb, dg = out if out is not None else (None, None)
        if out is not None:
            self.base._check_out(nb, dg, R)
        r = Request(REQ_PRUNE, Alpha(num, den), int(R), None, 0, 0, 0, _ptr(nb), None, _ptr(dg),
                    int(tag))
        self._keep[int(tag)] = (nb, dg)
        return r

    def query_request(self, alpha, R: int, Q: torch.Tensor, k: int, L: int,
                      out_ids: torch.Tensor, out_dist: Optional[torch.Tensor] = None,
                      out_hops: Optional[torch.Tensor] = None, tag: int = 0) -> Request:
        """alpha None queries the base graph."""
        _need_cuda(Q, out_ids, out_dist, out_hops)
        if Q.dtype != self.base.points.dtype or Q.shape[1] != self.base.d:
            raise ValueError("queries must match the points' dtype and dimension")
        nq = Q.shape[0]
        if tuple(out_ids.shape) != (nq, k) or out_ids.dtype != torch.int32:
            raise ValueError("out_ids must be int32 (nq, k)")
        num, den = (0, 0) if alpha is None else as_alpha(alpha)
        r = Request(REQ_QUERY, Alpha(num, den), int(R), Q.data_ptr(), nq, int(k), int(L),
                    out_ids.data_ptr(), _ptr(out_dist), _ptr(out_hops), int(tag))
        self._keep[int(tag)] = (Q, out_ids, out_dist, out_hops)
        return r

    def submit(self, req: Request):
        _check(_lib.rp_server_submit(self.handle, C.byref(req)))

    def poll(self, max_n: int = 256, wait_ms: int = 0) -> List[Completion]:
        buf = (Completion * max_n)()
        n = _lib.rp_server_poll(self.handle, buf, max_n, int(wait_ms))
        out = [buf[i] for i in range(max(n, 0))]
        for c in out:
            self._keep.pop(int(c.tag), None)
        return out

    def replay(self, reqs: Sequence[Request], arrival_s: Sequence[float]) -> List[Completion]:
        n = len(reqs)
        R = (Request * n)(*reqs)
        T = (C.c_double * n)(*[float(t) for t in arrival_s])
        out = (Completion * n)()
        _check(_lib.rp_server_replay(self.handle, R, T, n, out))
        for c in out:
            self._keep.pop(int(c.tag), None)
        return [out[i] for i in range(n)]

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.rp_server_stats_get(self.handle, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value is not None:
            _lib.rp_server_destroy(self.handle)
            self.handle = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
