"""Seeded synthetic workloads (points, queries, exact k-NN lists, medoid).

Shapes mirror the paper's datasets (Section 4.1): SIFT-1M (1M x 128) ->
``sift_u8``; Deep-1M (1M x 96) -> ``deep_f32``; GIST-1M (1M x 960) ->
``gist_f32``.  The data itself is drawn from Gaussian mixtures; nothing is
copied from any benchmark suite.

RNG: numpy PCG64 streams from SeedSequence(seed).spawn(5), one per purpose,
in this order: points, labels, queries, degree targets, node sample.
Component weights are uniform.  uint8 data is rounded half-to-even and
clipped to [0, 255]; float32 data is cast from FP64.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

Alpha = Tuple[int, int]  # alpha = num / den


@dataclasses.dataclass(frozen=True)
class Spec:
    name: str
    n: int
    d: int
    dtype: str              # "u8" or "f32"
    comps: int
    centre_mean: float
    centre_sd: float
    sigma: Optional[float]  # None: per component, per dimension U[0.5, 2]
    unit_norm: bool
    knn_k: int              # K of the exact K-NN lists fed to the base prune
    base_alpha: Alpha
    base_R: int
    sweep: Tuple[Alpha, ...]
    Rs: Tuple[int, ...]
    nq: int
    k: int
    Ls: Tuple[int, ...]
    uneven_degrees: bool    # truncate base lists to t_p ~ U{16..64}
    sample: int             # nodes the oracle checks at full size
    knn_near: int = 0       # > 0: K-NN restricted to the point's component and this many
                            # components with the nearest centres (labelled, not exact)


CONFIGS = {
    # 10,000 x 32 float32, 16 components, centres ~ N(0, 4I), sigma 1.
    "tiny": Spec("tiny", 10_000, 32, "f32", 16, 0.0, 2.0, 1.0, False, 64, (3, 2), 64,
                 ((7, 5), (13, 10), (6, 5), (11, 10), (1, 1)), (64,), 1_000, 10, (64,),
                 False, 10_000),
    # 1M x 128 uint8, 64 components, centres ~ N(128, 10^2) per dim, sigma 20.
    "sift_u8": Spec("sift_u8", 1_000_000, 128, "u8", 64, 128.0, 10.0, 20.0, False, 128,
                    (6, 5), 64, ((23, 20), (11, 10), (21, 20), (1, 1)), (64,), 10_000, 100,
                    (100, 150, 200, 300, 400), False, 20_000),
    # 1M x 96 float32, 128 components, centres ~ N(0, 0.5^2 I), sigma 1, unit-normalised
    # (with centres ~ N(0, I) the components separate after normalisation and the
    # K-NN graph falls apart into one piece per component).
    "deep_f32": Spec("deep_f32", 1_000_000, 96, "f32", 128, 0.0, 0.5, 1.0, True, 128,
                     (13, 10), 64,
                     ((1, 1), (26, 25), (109, 100), (113, 100), (117, 100), (121, 100),
                      (63, 50), (13, 10)), (64,), 10_000, 100, (100, 150, 200, 300, 400),
                     True, 20_000),
    # 1M x 960 float32, 64 components, centres ~ N(0, 0.5^2 I), sigma ~ U[0.5, 2].
    "gist_f32": Spec("gist_f32", 1_000_000, 960, "f32", 64, 0.0, 0.5, None, False, 192,
                     (6, 5), 96, ((11, 10), (1, 1)), (96, 64, 32), 1_000, 100,
                     (100, 150, 200, 300, 400), False, 20_000),
    # Serving: 10M x 128 uint8 as sift_u8; base lists from the 128-NN within each
    # point's component and the 3 components with the nearest centres.
    "serve_u8": Spec("serve_u8", 10_000_000, 128, "u8", 64, 128.0, 10.0, 20.0, False, 128,
                     (6, 5), 64, (), (32, 48, 64), 20_000, 100, (100, 200, 400), False, 20_000,
                     knn_near=3),
}


@dataclasses.dataclass
class Workload:
    spec: Spec
    X: np.ndarray                 # n x d points (uint8 or float32)
    Q: np.ndarray                 # nq x d queries (same dtype)
    knn: Optional[np.ndarray]     # n x K int32 exact K-NN lists (self excluded)
    knn_deg: Optional[np.ndarray]  # n int32 (= K)
    start: int                    # medoid
    targets: Optional[np.ndarray]  # n int32 degree targets (uneven configs)
    sample: np.ndarray            # sorted node sample (int32)
    # component-restricted lists (knn_near > 0): per component, its members and
    # the candidate ids of their lists (both sorted int32)
    components: Optional[List[Tuple[np.ndarray, np.ndarray]]] = None


def _streams(seed: int):
    ss = np.random.SeedSequence(seed).spawn(5)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]


def _finish(Y: np.ndarray, spec: Spec) -> np.ndarray:
    if spec.dtype == "u8":
        return np.clip(np.rint(Y), 0, 255).astype(np.uint8)
    if spec.unit_norm:
        Y = Y / np.sqrt((Y * Y).sum(axis=1, keepdims=True))
    return Y.astype(np.float32)


def _mixture(rng_pts, labels, centres, sig, spec: Spec, chunk: int = 65_536) -> np.ndarray:
    n = labels.shape[0]
    out = np.empty((n, spec.d), dtype=np.uint8 if spec.dtype == "u8" else np.float32)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        lab = labels[a:b]
        noise = rng_pts.standard_normal((b - a, spec.d))
        Y = centres[lab] + sig[lab] * noise
        out[a:b] = _finish(Y, spec)
    return out


def _mixture_params(rng, spec: Spec):
    centres = spec.centre_mean + spec.centre_sd * rng.standard_normal((spec.comps, spec.d))
    if spec.sigma is None:
        sig = rng.uniform(0.5, 2.0, (spec.comps, spec.d))
    else:
        sig = np.full((spec.comps, spec.d), spec.sigma)
    return centres, sig


def make_points_labelled(spec: Spec, n: Optional[int] = None, seed: int = 0):
    """Points, their component labels and the component centres."""
    n = spec.n if n is None else n
    rng_pts, rng_lab, _, _, _ = _streams(seed)
    centres, sig = _mixture_params(rng_pts, spec)
    labels = rng_lab.integers(0, spec.comps, n)
    return _mixture(rng_pts, labels, centres, sig, spec), labels, centres


def make_points(spec: Spec, n: Optional[int] = None, seed: int = 0) -> np.ndarray:
    return make_points_labelled(spec, n, seed)[0]


def make_queries(spec: Spec, nq: Optional[int] = None, seed: int = 0) -> np.ndarray:
    nq = spec.nq if nq is None else nq
    rng_pts, _, rng_q, _, _ = _streams(seed)
    centres, sig = _mixture_params(rng_pts, spec)  # same mixture as the points
    labels = rng_q.integers(0, spec.comps, nq)
    return _mixture(rng_q, labels, centres, sig, spec)


def degree_targets(n: int, seed: int = 0) -> np.ndarray:
    """t_p ~ U{16..64} per node (uneven out-degrees)."""
    rng = _streams(seed)[3]
    return rng.integers(16, 65, n).astype(np.int32)


def node_sample(n: int, size: int, seed: int = 0) -> np.ndarray:
    rng = _streams(seed)[4]
    size = min(size, n)
    return np.sort(rng.choice(n, size=size, replace=False)).astype(np.int32)


def medoid(X: np.ndarray, chunk: int = 262_144) -> int:
    """Start vertex: the point nearest to the FP64 centroid (lowest id on ties)."""
    c = X.astype(np.float64).mean(axis=0) if X.shape[0] <= chunk else _centroid(X, chunk)
    best, best_id = np.inf, -1
    for a in range(0, X.shape[0], chunk):
        Y = X[a:a + chunk].astype(np.float64) - c
        d2 = (Y * Y).sum(axis=1)
        i = int(np.argmin(d2))
        if d2[i] < best:
            best, best_id = float(d2[i]), a + i
    return best_id


def _centroid(X: np.ndarray, chunk: int) -> np.ndarray:
    acc = np.zeros(X.shape[1], dtype=np.float64)
    for a in range(0, X.shape[0], chunk):
        acc += X[a:a + chunk].astype(np.float64).sum(axis=0)
    return acc / X.shape[0]


# --------------------------------------------------------------------------
# Exact K-NN lists by brute force (self excluded), ties by (S, id)
# --------------------------------------------------------------------------

def knn_lists(X: np.ndarray, K: int, device=None, batch: Optional[int] = None) -> np.ndarray:
    """n x K int32 nearest-neighbour lists, ascending by (S, id).

    uint8 data: exact (integer keys S * 2^b + id).  float32 data: FP64 on the
    CPU, FP32 GEMM on a GPU (the lists are input data; near-ties may resolve
    either way, which no later comparison depends on)."""
    n = X.shape[0]
    K = min(K, n - 1)
    if device is not None and str(device).startswith("cuda"):
        return _knn_torch(X, K, device, batch)
    return _knn_numpy(X, K, batch)


def _knn_numpy(X: np.ndarray, K: int, batch: Optional[int]) -> np.ndarray:
    n = X.shape[0]
    batch = batch or max(1, min(n, (1 << 26) // max(n, 1)))
    Xd = X.astype(np.float64)
    nrm = (Xd * Xd).sum(axis=1)
    out = np.empty((n, K), dtype=np.int32)
    ids = np.arange(n, dtype=np.int64)
    idbits = max(1, int(n - 1).bit_length())
    for a in range(0, n, batch):
        b = min(n, a + batch)
        S = nrm[a:b, None] + nrm[None, :] - 2.0 * (Xd[a:b] @ Xd.T)
        if X.dtype == np.uint8:
            key = (np.rint(S).astype(np.int64) << idbits) | ids[None, :]
            key[np.arange(b - a), np.arange(a, b)] = np.iinfo(np.int64).max
            part = np.argpartition(key, K - 1, axis=1)[:, :K]
            kk = np.take_along_axis(key, part, axis=1)
            order = np.argsort(kk, axis=1, kind="stable")
            out[a:b] = np.take_along_axis(part, order, axis=1)
        else:
            S[np.arange(b - a), np.arange(a, b)] = np.inf
            part = np.argpartition(S, K - 1, axis=1)[:, :K]
            ss = np.take_along_axis(S, part, axis=1)
            order = np.lexsort((part, ss), axis=1)
            out[a:b] = np.take_along_axis(part, order, axis=1)
    return out


def _knn_torch(X: np.ndarray, K: int, device, batch: Optional[int]) -> np.ndarray:
    import torch

    n, d = X.shape
    Xt = torch.from_numpy(X).to(device)
    out = torch.empty((n, K), dtype=torch.int32, device=device)
    rows = torch.arange(n, device=device, dtype=torch.int64)
    batch = batch or max(256, min(4096, (1 << 31) // max(n, 1)))
    if X.dtype == np.uint8:
        exact32 = d * 255 * 255 < (1 << 24)  # every FP32 partial sum is an exact integer
        Xf = Xt.to(torch.float32 if exact32 else torch.float64)
        nrm = (Xt.to(torch.int64) ** 2).sum(dim=1)
        idbits = max(1, int(n - 1).bit_length())
        mask = (1 << idbits) - 1
        big = torch.iinfo(torch.int64).max
        for a in range(0, n, batch):
            b = min(n, a + batch)
            ip = (Xf[a:b] @ Xf.T).to(torch.int64)
            key = nrm[None, :] - 2 * ip + nrm[a:b, None]          # exact S
            key = (key << idbits) | rows[None, :]
            key[torch.arange(b - a, device=device), rows[a:b]] = big
            vals, _ = torch.topk(key, K, dim=1, largest=False, sorted=True)
            out[a:b] = (vals & mask).to(torch.int32)
            del ip, key, vals
    else:
        Xf = Xt.to(torch.float32)
        nrm = (Xf * Xf).sum(dim=1)
        for a in range(0, n, batch):
            b = min(n, a + batch)
            S = nrm[None, :] - 2.0 * (Xf[a:b] @ Xf.T)
            S[torch.arange(b - a, device=device), rows[a:b]] = float("inf")
            _, idx = torch.topk(S, K, dim=1, largest=False, sorted=True)
            out[a:b] = idx.to(torch.int32)
            del S
    torch.cuda.synchronize(device)
    return out.cpu().numpy()


def component_sets(labels: np.ndarray, centres: np.ndarray, near: int
                   ) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Per component: its members and the candidates of their lists (the
    members of the component and of the `near` components with the nearest
    centres), both sorted int32."""
    comps = centres.shape[0]
    cd = ((centres[:, None, :] - centres[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(cd, np.inf)
    nearest = np.argsort(cd, axis=1, kind="stable")[:, :near]
    order = np.argsort(labels, kind="stable")
    bounds = np.concatenate([[0], np.cumsum(np.bincount(labels, minlength=comps))])
    members = [np.sort(order[bounds[c]:bounds[c + 1]]).astype(np.int32) for c in range(comps)]
    return [(members[c],
             np.sort(np.concatenate([members[c]] + [members[o] for o in nearest[c]]))
             .astype(np.int32)) for c in range(comps)]


def knn_by_component(X: np.ndarray, labels: np.ndarray, centres: np.ndarray, K: int, near: int,
                     device, batch: int = 2048) -> np.ndarray:
    """n x K int32 lists: for each uint8 point, its K nearest among the points
    of its own component and of the `near` components with the nearest centres
    (self excluded), ascending by the key (S, id), so the lists are exact and
    unique.  A labelled stand-in for exact K-NN at a size where the brute
    force over all points is too costly; the lists are input data."""
    return knn_on_sets(X, component_sets(labels, centres, near), K, device, batch=batch)


def knn_on_sets(X: np.ndarray, sets, K: int, device, rows: Optional[np.ndarray] = None,
                batch: int = 2048) -> np.ndarray:
    """n x K int32 lists over (members, candidates) sets as knn_by_component
    builds them; with `rows`, only those points' lists are computed (the rest
    stay -1)."""
    import torch

    assert X.dtype == np.uint8 and X.shape[1] * 255 * 255 * 2 < (1 << 24)
    n, d = X.shape
    if rows is not None:
        sets = [(np.intersect1d(mem, rows).astype(np.int32), cand) for mem, cand in sets]
    Xt = torch.from_numpy(X).to(device)
    Xf = Xt.to(torch.float32)                      # every partial sum is an exact integer
    nrm = (Xt.to(torch.int64) ** 2).sum(dim=1).to(torch.float32)
    out = torch.full((n, K), -1, dtype=torch.int32, device=device)
    for mem, cand in sets:
        if mem.size == 0:
            continue
        ct = torch.from_numpy(cand).to(device)
        Xc, nc = Xf[ct], nrm[ct]
        kk = min(K, cand.size - 1)
        for a in range(0, mem.size, batch):
            q = torch.from_numpy(mem[a:a + batch]).to(device)
            S = nrm[q][:, None] + nc[None, :] - 2.0 * (Xf[q] @ Xc.T)   # exact integers
            S[torch.arange(q.numel(), device=device), torch.searchsorted(ct, q)] = float("inf")
            vals, idx = torch.topk(S, kk, dim=1, largest=False, sorted=True)
            key = (vals.to(torch.int64) << 32) | ct[idx].to(torch.int64)
            # rows with more candidates at the K-th distance than places left:
            # take the smallest ids among the tied ones
            sk = vals[:, kk - 1:kk]
            for r in torch.nonzero((S <= sk).sum(dim=1) > kk).flatten().tolist():
                cols = torch.nonzero(S[r] <= sk[r]).flatten()
                kr = (S[r, cols].to(torch.int64) << 32) | ct[cols].to(torch.int64)
                key[r] = torch.sort(kr).values[:kk]
            key, _ = torch.sort(key, dim=1)
            out[q, :kk] = (key & 0xFFFFFFFF).to(torch.int32)
            del S, vals, idx, key
    if out.is_cuda:
        torch.cuda.synchronize(device)
    return out.cpu().numpy()


def build(name: str, n: Optional[int] = None, nq: Optional[int] = None, seed: int = 0,
          device=None, with_knn: bool = True, knn_k: Optional[int] = None,
          sample: Optional[int] = None) -> Workload:
    """Generate one configuration (optionally scaled down to n points)."""
    spec = CONFIGS[name]
    X, labels, centres = make_points_labelled(spec, n, seed)
    Q = make_queries(spec, nq, seed)
    K = knn_k or spec.knn_k
    comp = component_sets(labels, centres, spec.knn_near) if spec.knn_near > 0 else None
    if with_knn and spec.knn_near > 0 and device is not None:
        knn = knn_by_component(X, labels, centres, min(K, X.shape[0] - 1), spec.knn_near, device)
    else:
        knn = knn_lists(X, K, device) if with_knn else None
    knn_deg = None if knn is None else (knn >= 0).sum(axis=1).astype(np.int32)
    targets = degree_targets(X.shape[0], seed) if spec.uneven_degrees else None
    smp = node_sample(X.shape[0], sample or spec.sample, seed)
    return Workload(spec, X, Q, knn, knn_deg, medoid(X), targets, smp, comp)


def rational_str(a: Alpha) -> str:
    return f"{a[0]}/{a[1]}"


def alphas_as_float(al: Sequence[Alpha]) -> List[float]:
    return [a[0] / a[1] for a in al]
