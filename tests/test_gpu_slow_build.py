"""GPU parity for the slow-preprocessing construction (rp_build_slow:
RobustPrune(p, P \\ {p}, alpha, R) for every p, Section 2.1) and for RP-Tuning
of its graph (Section 3), against the oracle; graph-level checks of Lemma 2.2
(the graph is alpha-reachable) and Theorem 3.2 (after RP-Tuning the
reachability is at least min(alpha_2, 1 / beta)) with the reachability meter;
and the 10,000-point prune-versus-rebuild setting on sampled vertices."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import reach

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _oracle_slow(X, a, R, nodes):
    n = X.shape[0]
    out = {}
    for p in nodes:
        out[int(p)] = oracle.robust_prune(X, int(p), [q for q in range(n) if q != p], *a, R)
    return out


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_slow_build_all_vertices(dtype):
    from paper_2602_08097_amd import build_slow

    rng = np.random.default_rng(11)
    n = 400
    if dtype == "u8":
        X = rng.integers(0, 5, (n, 6)).astype(np.uint8)  # many exact ties
    else:
        X = (rng.integers(-3, 4, (n, 6)) * 0.5).astype(np.float32)
    X[50:55] = X[3]  # duplicate points
    Xd = torch.from_numpy(X).to(_dev())
    for a, R in (((6, 5), n - 1), ((1, 1), n - 1), ((3, 2), 7)):
        nb, dg = build_slow(Xd, a, R)
        nb, dg = _np(nb), _np(dg)
        want = _oracle_slow(X, a, R if R < n - 1 else 0, range(n))
        for p in range(n):
            assert dg[p] == len(want[p]), (a, R, p)
            assert nb[p, :dg[p]].tolist() == want[p], (a, R, p)
            assert (nb[p, dg[p]:] == -1).all()


@pytest.mark.parametrize("a1,a2", [((3, 1), (2, 1)), ((3, 2), (6, 5))])
def test_slow_graph_reachability_and_rp_tuning(a1, a2):
    """Lemma 2.2 on the GPU's slow-preprocessing graph, Theorem 3.2 on its
    RP-Tuning at alpha_2 (batched kernel), and both graphs equal the oracle's."""
    from paper_2602_08097_amd import Graph, build_slow

    dev = _dev()
    rng = np.random.default_rng(sum(a1) + sum(a2))
    n = 160
    X = rng.standard_normal((n, 2)).astype(np.float32)
    Xd = torch.from_numpy(X).to(dev)
    nb, dg = build_slow(Xd, a1, n - 1)
    nbn, dgn = _np(nb), _np(dg)
    D = reach.distance_matrix(X)
    adj = [list(nbn[p, :dgn[p]]) for p in range(n)]
    A1, A2 = a1[0] / a1[1], a2[0] / a2[1]
    assert reach.reachability(D, adj) >= A1 * (1 - 1e-9)
    r_max = int(dgn.max())
    g = Graph(Xd, nb[:, :r_max].contiguous(), dg, 0)
    pnb, pdg = g.prune(a2, r_max)
    e_nbr, e_deg, _ = oracle.prune_graph(X, nbn[:, :r_max], dgn, *a2, r_max)
    assert np.array_equal(_np(pnb), e_nbr) and np.array_equal(_np(pdg), e_deg)
    adj2 = [list(e_nbr[p, :e_deg[p]]) for p in range(n)]
    assert reach.reachability(D, adj2) >= min(A2, reach.sorted_euclid_bound(A1, A2)) * (1 - 1e-9)
    g.free()


def test_prune_versus_rebuild_10k_sampled():
    """The 10,000 x 32 float32 workload: the slow-preprocessing graph at
    alpha_1 = 3/2 (R = 256), the rebuild at alpha_2 = 11/10 and RP-Tuning of the
    alpha_1 graph at 11/10, each sampled on 40 vertices against the oracle."""
    from paper_2602_08097_amd import Graph, build_slow

    dev = _dev()
    w = workloads.build("tiny", with_knn=False)
    X = w.X
    Xd = torch.from_numpy(X).to(dev)
    R = 256
    nodes = w.sample[::250][:40]
    b_nb, b_dg = build_slow(Xd, (3, 2), R)
    r_nb, r_dg = build_slow(Xd, (11, 10), R)
    want_b = _oracle_slow(X, (3, 2), R, nodes)
    want_r = _oracle_slow(X, (11, 10), R, nodes)
    bn, bd, rn, rd = _np(b_nb), _np(b_dg), _np(r_nb), _np(r_dg)
    for p in nodes:
        assert bn[p, :bd[p]].tolist() == want_b[int(p)]
        assert rn[p, :rd[p]].tolist() == want_r[int(p)]
    r_max = int(bd.max())
    g = Graph(Xd, b_nb[:, :r_max].contiguous(), b_dg, w.start)
    t_nb, t_dg = g.prune((11, 10), R if r_max > R else r_max)
    o_nbr = np.zeros((X.shape[0], r_max), np.int32)
    o_deg = np.zeros(X.shape[0], np.int32)
    for p in nodes:
        o_nbr[p, :len(want_b[int(p)])] = want_b[int(p)]
        o_deg[p] = len(want_b[int(p)])
    e_nbr, e_deg, _ = oracle.prune_graph(X, o_nbr, o_deg, 11, 10, r_max, nodes=nodes)
    assert np.array_equal(_np(t_nb)[nodes], e_nbr) and np.array_equal(_np(t_dg)[nodes], e_deg)
    g.free()
