"""The serving workload at full size: 10,000,000 uint8 points (d = 128), the
resident base graph (RobustPrune at 6/5, R = 64 of each point's 128 nearest
among its own and the three nearest mixture components), one prune request
and one query batch through the request loop.  The batched uint8 kernel packs
24 id bits into its sort keys at this n.  2,000 sampled vertices of the base
graph and of the pruned graph, and 50 queries on each graph, equal the
oracle's.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

THREADS = 8


def _say(msg):
    print(f"[serve10M] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def serve10m():
    from paper_2602_08097_amd import Graph, knn_u8_sets

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    _say("generating serve_u8 (10M x 128)")
    w = workloads.build("serve_u8", nq=2_000, device=dev, with_knn=False)
    spec = w.spec
    K = spec.knn_k
    nodes = w.sample[:2000]
    # the generator's lists (input data) on the sampled rows only: the oracle's
    # base rows need no others
    _say("generator lists of the sampled rows")
    ref = workloads.synth.knn_on_sets(w.X, w.components, K, dev, rows=nodes)
    ref_deg = (ref >= 0).sum(axis=1).astype(np.int32)
    X = torch.from_numpy(w.X).to(dev)
    # the base lists on the GPU: exact (S, id) K-NN restricted to each point's
    # component sets (rp_knn_u8), equal to the generator's on the sample
    _say("rp_knn_u8 over the component sets")
    knn = knn_u8_sets(X, K, w.components)
    kdeg = (knn >= 0).sum(dim=1, dtype=torch.int32)
    assert np.array_equal(knn.cpu().numpy()[nodes], ref[nodes])
    g0 = Graph(X, knn, kdeg, w.start)
    nb, dg = g0.prune(spec.base_alpha, spec.base_R)
    torch.cuda.synchronize()
    g0.free()
    del knn, kdeg
    base = Graph(X, nb, dg, w.start)
    _say("oracle base rows on the sample")
    o_nbr, o_deg, _ = oracle.prune_graph(w.X, ref, ref_deg, *spec.base_alpha, spec.base_R,
                                         nodes=nodes, threads=THREADS)
    del ref
    return w, base, nodes, o_nbr, o_deg


def test_serve_10m_base_graph_sampled(serve10m):
    w, base, nodes, o_nbr, o_deg = serve10m
    assert np.array_equal(base.deg.cpu().numpy()[nodes], o_deg)
    assert np.array_equal(base.nbr.cpu().numpy()[nodes], o_nbr)


def test_serve_10m_prune_request_and_queries(serve10m):
    from paper_2602_08097_amd import Server

    w, base, nodes, o_nbr, o_deg = serve10m
    dev = base.points.device
    n = w.X.shape[0]
    a, R, k, L = (109, 100), 48, 10, 100
    server = Server(base, 2 * n * (R + 1) * 4 + (1 << 20), n_streams=2, max_query_batch=256)
    Q = torch.from_numpy(np.ascontiguousarray(w.Q[:50])).to(dev)
    out = (torch.empty((n, R), dtype=torch.int32, device=dev),
           torch.empty(n, dtype=torch.int32, device=dev))
    ids = torch.empty((50, k), dtype=torch.int32, device=dev)
    dist = torch.empty((50, k), dtype=torch.float64, device=dev)
    hops = torch.empty(50, dtype=torch.int32, device=dev)
    b_ids = torch.empty((50, k), dtype=torch.int32, device=dev)
    b_dist = torch.empty((50, k), dtype=torch.float64, device=dev)
    b_hops = torch.empty(50, dtype=torch.int32, device=dev)
    reqs = [server.prune_request(a, R, out=out, tag=0),
            server.query_request(a, R, Q, k, L, ids, dist, hops, tag=1),
            server.query_request(None, 0, Q, k, L, b_ids, b_dist, b_hops, tag=2)]
    comps = server.replay(reqs, [0.0, 0.001, 0.002])
    server.close()
    torch.cuda.synchronize()
    assert all(c.status == 0 for c in comps), [c.status for c in comps]
    _say(f"prune request {1e3 * (comps[0].t_done - comps[0].t_start):.1f} ms")
    # the pruned rows on the sample: RobustPrune of the oracle's own base rows
    full_nbr = np.zeros((n, 64), np.int32)
    full_deg = np.zeros(n, np.int32)
    full_nbr[nodes], full_deg[nodes] = o_nbr, o_deg
    e_nbr, e_deg, _ = oracle.prune_graph(w.X, full_nbr, full_deg, *a, R, nodes=nodes,
                                         threads=THREADS)
    del full_nbr, full_deg
    got_nbr = out[0].cpu().numpy()
    got_deg = out[1].cpu().numpy()
    assert np.array_equal(got_deg[nodes], e_deg)
    assert np.array_equal(got_nbr[nodes], e_nbr)
    _say("2,000 sampled pruned rows identical")
    # 50 queries on each graph (the oracle walks the graph the request searched)
    for name, gn, gd, (i_, d_, h_) in (("pruned", got_nbr, got_deg, (ids, dist, hops)),
                                       ("base", base.nbr.cpu().numpy(), base.deg.cpu().numpy(),
                                        (b_ids, b_dist, b_hops))):
        e_ids, e_dist, e_hops = oracle.search(w.X, gn, gd, w.start, w.Q[:50], k, L)
        assert np.array_equal(i_.cpu().numpy(), e_ids), name
        assert np.array_equal(d_.cpu().numpy(), e_dist), name
        assert np.array_equal(h_.cpu().numpy(), e_hops), name
        _say(f"50 queries on the {name} graph identical")
