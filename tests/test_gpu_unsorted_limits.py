"""GPU parity through the C-ABI for UnsortedRobustPrune (Section 3) and for
the limits of the batched kernels: ids above 2^21 (the uint8 sort key packs
more id bits there), float32 coordinates near 1e35 (frame exponents far below
zero), 96 candidates at d = 4000 (beyond the batched kernel's LDS: the plain
kernel serves it) and point sets with NaN or infinite coordinates (rejected).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _graph(X, nbr, deg, start=0):
    from paper_2602_08097_amd import Graph

    dev = _dev()
    return Graph(torch.from_numpy(np.ascontiguousarray(X)).to(dev),
                 torch.from_numpy(np.ascontiguousarray(nbr, dtype=np.int32)).to(dev),
                 torch.from_numpy(np.ascontiguousarray(deg, dtype=np.int32)).to(dev), start)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[limits] {msg}", file=sys.stderr, flush=True)


def _check(X, nbr, deg, outs, alphas, Rs, unsorted, nodes=None, threads=8):
    for o, (nb, dg) in enumerate(outs):
        a, R = alphas[o // len(Rs)], Rs[o % len(Rs)]
        e_nbr, e_deg, _ = oracle.prune_graph(X, nbr, deg, *a, R, nodes=nodes, unsorted=unsorted,
                                             threads=threads)
        got, gdg = _np(nb), _np(dg)
        if nodes is not None:
            got, gdg = got[nodes], gdg[nodes]
        bad = np.nonzero((got != e_nbr).any(axis=1) | (gdg != e_deg))[0]
        assert bad.size == 0, (a, R, unsorted, bad[:5], got[bad[:1]], e_nbr[bad[:1]])


def _random_lists(rng, n, r_max, self_and_repeats=True):
    nbr = rng.integers(0, n, (n, r_max)).astype(np.int32)
    if self_and_repeats and r_max > 3:
        nbr[:, 1] = np.arange(n)          # p itself
        nbr[:, 3] = nbr[:, 2]             # a repeated id
    deg = rng.integers(0, r_max + 1, n).astype(np.int32)
    deg[:2] = 0
    deg[2:6] = r_max
    return nbr, deg


# --------------------------------------------------------------------------
# UnsortedRobustPrune
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,d,r_max", [("u8", 32, 64), ("u8", 128, 17), ("f32", 24, 64),
                                           ("f32", 200, 96), ("u8", 16, 130), ("f32", 7, 130)])
def test_unsorted_matches_oracle(dtype, d, r_max):
    """Lists in random order with self ids, repeated ids, empty and full rows;
    the int8 and split-FP16 batched kernels (r_max <= 64 / 96) and the plain
    kernel (r_max 130) against the oracle's UnsortedRobustPrune, and the same
    graph's sorted sweep against RobustPrune."""
    rng = np.random.default_rng(d * 7 + r_max)
    n = 600
    if dtype == "u8":
        X = rng.integers(0, 6, (n, d)).astype(np.uint8)       # many exact ties
    else:
        X = (rng.integers(-3, 4, (n, d)) * 0.25).astype(np.float32)
    nbr, deg = _random_lists(rng, n, r_max)
    g = _graph(X, nbr, deg)
    alphas = [(1, 1), (21, 20), (6, 5), (2, 1)]
    Rs = [r_max, 5]
    for unsorted in (True, False):
        outs = g.prune_sweep(alphas, Rs, unsorted=unsorted)
        _check(X, nbr, deg, outs, alphas, Rs, unsorted)
    g.free()


def test_unsorted_tiny_workload_all_vertices():
    """The 10,000 x 32 float32 workload: base graph from the K-NN lists, every
    list then shuffled; UnsortedRobustPrune at the five alphas on every
    vertex equals the oracle, and differs from RobustPrune somewhere."""
    dev = _dev()
    w = workloads.build("tiny")
    spec = w.spec
    g0 = _graph(w.X, w.knn, w.knn_deg, w.start)
    nb, dg = g0.prune(spec.base_alpha, spec.base_R)
    nbr, deg = _np(nb), _np(dg)
    rng = np.random.default_rng(3)
    for p in range(nbr.shape[0]):
        rng.shuffle(nbr[p, :deg[p]])
    g = g0.derive(torch.from_numpy(nbr).to(dev), torch.from_numpy(deg).to(dev))
    outs = g.prune_sweep(spec.sweep, spec.Rs, unsorted=True)
    _check(w.X, nbr, deg, outs, list(spec.sweep), list(spec.Rs), True)
    s_outs = g.prune_sweep(spec.sweep, spec.Rs)
    assert any(not torch.equal(a[0], b[0]) for a, b in zip(outs, s_outs))
    g.free()
    g0.free()


# --------------------------------------------------------------------------
# Limits
# --------------------------------------------------------------------------

def test_u8_ids_above_2_21_sampled():
    """n = 2^21 + 4099 uint8 points (d = 16): the batched kernel's sort key
    carries 22 id bits.  Random lists of 64 ids, many near n; 3,000 sampled
    vertices and the last 64 vertices equal the oracle at four alphas, sorted
    and unsorted."""
    n = (1 << 21) + 4099
    rng = np.random.default_rng(21)
    X = rng.integers(0, 256, (n, 16)).astype(np.uint8)
    nbr = rng.integers(0, n, (n, 64)).astype(np.int32)
    nbr[:, :8] = n - 1 - rng.integers(0, 1 << 12, (n, 8))   # ids just below n
    deg = np.full(n, 64, np.int32)
    deg[::7] = rng.integers(0, 65, deg[::7].shape[0])
    g = _graph(X, nbr, deg)
    nodes = np.unique(np.concatenate([np.sort(rng.choice(n, 3000, replace=False)),
                                      np.arange(n - 64, n)])).astype(np.int32)
    alphas = [(1, 1), (21, 20), (11, 10), (6, 5)]
    for unsorted in (False, True):
        outs = g.prune_sweep(alphas, [64], unsorted=unsorted)
        _check(X, nbr, deg, outs, alphas, [64], unsorted, nodes=nodes)
        _say(f"n = {n}, unsorted={unsorted}: {nodes.size} sampled vertices identical")
    g.free()


def test_f32_coordinates_near_1e35():
    """Coordinates of magnitude up to ~1e35 (and a few near 1e-30): frame
    exponents down to about -104; the batched float32 kernel equals the
    oracle (canonical FP64 squares reach 1e72)."""
    rng = np.random.default_rng(35)
    n, d = 500, 40
    X = (rng.standard_normal((n, d)) * 1e35).astype(np.float32)
    X[100:120] = (rng.standard_normal((20, d)) * 1e-30).astype(np.float32)
    X[120:130] = X[0]
    nbr, deg = _random_lists(rng, n, 64)
    g = _graph(X, nbr, deg)
    alphas = [(1, 1), (11, 10), (3, 2)]
    outs = g.prune_sweep(alphas, [64, 9])
    _check(X, nbr, deg, outs, alphas, [64, 9], False)
    err = g.gram_error(torch.arange(0, n, dtype=torch.int32, device=_dev()))
    assert err["max_err_over_bound"] <= 1.0
    g.free()


@pytest.mark.parametrize("r_max,d", [(96, 4000), (128, 3000)])
def test_f32_long_rows_beyond_64_kib_of_lds(r_max, d):
    """One vertex of 96 candidates at d = 4000 (72 KiB) or of 128 at d = 3000
    (76 KiB) needs more than 64 KiB of LDS: on gfx950 (160 KiB per workgroup)
    the batched kernel takes it, elsewhere the plain kernel; either way the
    sweep equals the oracle, and the measured error stays in the band."""
    rng = np.random.default_rng(d + r_max)
    n = 140
    X = rng.standard_normal((n, d)).astype(np.float32)
    nbr, deg = _random_lists(rng, n, r_max)
    g = _graph(X, nbr, deg)
    alphas = [(1, 1), (6, 5)]
    outs = g.prune_sweep(alphas, [r_max, 20])
    _check(X, nbr, deg, outs, alphas, [r_max, 20], False)
    props = torch.cuda.get_device_properties(0)
    if getattr(props, "shared_memory_per_block", 0) >= 160 * 1024:
        err = g.gram_error(torch.arange(0, n, dtype=torch.int32, device=_dev()))
        assert err["pairs"] > 0 and err["max_err_over_bound"] <= 1.0
    g.free()


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_nonfinite_points_are_rejected(bad):
    from paper_2602_08097_amd.rp import RPError

    rng = np.random.default_rng(1)
    X = rng.standard_normal((50, 8)).astype(np.float32)
    X[17, 3] = bad
    nbr, deg = _random_lists(rng, 50, 8)
    with pytest.raises(RPError, match="RP_EINVAL"):
        _graph(X, nbr, deg)
