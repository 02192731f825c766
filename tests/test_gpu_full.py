"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times: 1,000,000 points, the whole graph pruned in one sweep launch,
the oracle recomputing a 20,000-vertex sample one vertex at a time (the rows
of a vertex depend only on its own list and the points), plus properties
that hold for every vertex at any size.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

THREADS = 8  # the oracle runs single-threaded on this many disjoint vertex shards at once


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _say(msg):
    print(f"[full] {msg}", file=sys.stderr, flush=True)


class Full:
    """A full-size workload with its GPU base graph and the oracle's base rows
    for the sampled vertices."""

    def __init__(self, name, sample):
        from paper_2602_08097_amd import Graph

        dev = _dev()
        _say(f"building {name}")
        w = workloads.build(name, device=dev)
        self.w, self.spec = w, w.spec
        self.X = torch.from_numpy(w.X).to(dev)
        g0 = Graph(self.X, torch.from_numpy(w.knn).to(dev), torch.from_numpy(w.knn_deg).to(dev),
                   w.start)
        nb, dg = g0.prune(self.spec.base_alpha, self.spec.base_R)
        self.nodes = w.sample[:sample]
        # the oracle's base rows for the sample, from the same K-NN lists
        _say(f"oracle base rows for {self.nodes.size} vertices")
        o_nbr, o_deg, _ = oracle.prune_graph(w.X, w.knn, w.knn_deg, *self.spec.base_alpha,
                                             self.spec.base_R, nodes=self.nodes, threads=THREADS)
        g_nbr, g_deg = _np(nb)[self.nodes], _np(dg)[self.nodes]
        assert np.array_equal(g_deg, o_deg), "base degrees differ on the sample"
        assert np.array_equal(g_nbr, o_nbr), "base rows differ on the sample"
        if w.targets is not None:
            dg = torch.minimum(dg, torch.from_numpy(w.targets).to(dev))
        self.base_nbr, self.base_deg = nb, dg
        self.g = g0.derive(nb, dg)
        self.g0 = g0
        n = w.X.shape[0]
        # oracle-side base graph restricted to the sample (other rows empty)
        self.o_nbr = np.zeros((n, self.spec.base_R), np.int32)
        self.o_deg = np.zeros(n, np.int32)
        self.o_nbr[self.nodes] = o_nbr
        self.o_deg[self.nodes] = o_deg if w.targets is None else np.minimum(
            o_deg, w.targets[self.nodes])


@pytest.fixture(scope="module")
def sift_full():
    return Full("sift_u8", 20_000)


def _check_sampled(f, outs):
    nr = len(f.spec.Rs)
    for o, (nb, dg) in enumerate(outs):
        a, R = f.spec.sweep[o // nr], f.spec.Rs[o % nr]
        e_nbr, e_deg, _ = oracle.prune_graph(f.w.X, f.o_nbr, f.o_deg, *a, R, nodes=f.nodes,
                                             threads=THREADS)
        got_nbr, got_deg = _np(nb)[f.nodes], _np(dg)[f.nodes]
        bad = np.nonzero((got_nbr != e_nbr).any(axis=1) | (got_deg != e_deg))[0]
        assert bad.size == 0, (f"alpha={a} R={R}: {bad.size} of {f.nodes.size} sampled rows "
                               f"differ, first vertices {f.nodes[bad[:5]]}")
        _say(f"alpha={a[0]}/{a[1]} R={R}: {f.nodes.size} sampled rows identical")


def test_sift_full_knn_lists(sift_full):
    """The 128-NN lists of all 1M points from rp_knn_u8 (int8 MFMA, exact
    (S, id) order): 300 sampled rows equal the oracle's brute force; every row
    equals the workload's integer-keyed lists."""
    import time

    from paper_2602_08097_amd import knn_u8

    f = sift_full
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = knn_u8(f.X, 128)
    torch.cuda.synchronize()
    _say(f"rp_knn_u8 1M x 128, K = 128: {time.perf_counter() - t0:.2f} s")
    got = _np(got)
    smp = f.nodes[:300]
    gt = oracle.groundtruth(f.w.X, f.w.X[smp], 129, threads=THREADS)
    for r, q in enumerate(smp):
        want = [int(i) for i in gt[r] if int(i) != int(q)][:128]
        assert got[q].tolist() == want, int(q)
    assert np.array_equal(got, f.w.knn)


def test_sift_full_sweep_sampled(sift_full):
    """1M x 128 uint8, the benchmark's sweep launch (4 alphas, R = 64): the
    20,000 sampled rows equal the oracle's, element by element."""
    f = sift_full
    outs = f.g.prune_sweep(f.spec.sweep, f.spec.Rs)
    _check_sampled(f, outs)


def test_sift_full_idempotent_all_vertices(sift_full):
    """Re-pruning a pruned graph at its own (alpha, R) returns it unchanged,
    for every one of the 1M vertices: the base graph at 6/5 and each sweep
    output at its alpha."""
    f = sift_full
    again = f.g.prune_sweep([f.spec.base_alpha], [f.spec.base_R])[0]
    assert torch.equal(again[1], f.base_deg)
    assert torch.equal(again[0], f.base_nbr)
    outs = f.g.prune_sweep(f.spec.sweep, f.spec.Rs)
    for a, (nb, dg) in zip(f.spec.sweep, outs):
        gp = f.g.derive(nb, dg)
        r_nb, r_dg = gp.prune_sweep([a], [f.spec.Rs[0]])[0]
        assert torch.equal(r_dg, dg) and torch.equal(r_nb, nb), f"alpha={a} not idempotent"
        gp.free()


def test_sift_full_plain_matches_batched(sift_full):
    """The plain one-workgroup-per-vertex kernel and the batched kernel give
    identical graphs on all 1M vertices (one alpha), and the plain rows equal
    the oracle's on the sample."""
    f = sift_full
    a, R = f.spec.sweep[-1], f.spec.Rs[0]
    p_nb, p_dg = f.g.prune_plain(a, R)
    b_nb, b_dg = f.g.prune_sweep([a], [R])[0]
    assert torch.equal(p_dg, b_dg) and torch.equal(p_nb, b_nb)
    e_nbr, e_deg, _ = oracle.prune_graph(f.w.X, f.o_nbr, f.o_deg, *a, R, nodes=f.nodes,
                                         threads=THREADS)
    assert np.array_equal(_np(p_nb)[f.nodes], e_nbr)
    assert np.array_equal(_np(p_dg)[f.nodes], e_deg)


def test_sift_full_search_sampled(sift_full):
    """GreedySearch on the 1M-vertex base graph and on the alpha = 1 graph:
    200 of the 10,000 queries at L = 100, k = 100 give the oracle's ids,
    distances and visited counts."""
    f = sift_full
    k, L = f.spec.k, 100
    qsel = np.arange(0, f.w.Q.shape[0], f.w.Q.shape[0] // 200)[:200]
    Q = f.w.Q[qsel]
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).to(f.X.device)
    a1 = f.g.prune_sweep([f.spec.sweep[-1]], [f.spec.Rs[0]])[0]
    for name, nb, dg in (("base", f.base_nbr, f.base_deg), ("alpha=1", a1[0], a1[1])):
        gg = f.g.derive(nb, dg)
        ids, dist, hops = gg.search(Qd, k, L)
        e_ids, e_dist, e_hops = oracle.search(f.w.X, _np(nb), _np(dg), f.w.start, Q, k, L)
        assert np.array_equal(_np(ids), e_ids), name
        assert np.array_equal(_np(dist), e_dist), name
        assert np.array_equal(_np(hops), e_hops), name
        _say(f"search {name}: 200 queries identical")
        gg.free()


@pytest.fixture(scope="module")
def deep_full():
    return Full("deep_f32", 20_000)


def test_deep_full_sweep_sampled(deep_full):
    """1M x 96 unit-normalised float32, out-degrees uneven in 16..64, eight
    alphas in one launch (FP16 Gram with FP64 recheck): the 20,000 sampled
    rows equal the oracle's."""
    f = deep_full
    f.g.counters(reset=True)
    outs = f.g.prune_sweep(f.spec.sweep, f.spec.Rs)
    c = f.g.counters()
    _say(f"rechecks per vertex-alpha: {c['rechecks'] / max(1, c['nodes']):.4f}")
    _check_sampled(f, outs)


@pytest.fixture(scope="module")
def gist_full():
    return Full("gist_f32", 2_000)


def test_gist_full_sweep_sampled(gist_full):
    """1M x 960 float32 (GIST shape), base lists of up to 96 from the 192-NN
    lists, the benchmark's sweep: alpha in {11/10, 1} x R in {96, 64, 32} (six
    outputs, one launch; split-FP16 Gram over 30 accumulator chunks, FP64
    recheck): 2,000 sampled rows of every output equal the oracle's."""
    f = gist_full
    f.g.counters(reset=True)
    outs = f.g.prune_sweep(f.spec.sweep, f.spec.Rs)
    c = f.g.counters()
    _say(f"rechecks per vertex-output: {c['rechecks'] / max(1, c['nodes']):.4f}")
    _check_sampled(f, outs)
