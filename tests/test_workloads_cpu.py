"""The synthetic input generator's component-restricted K-NN lists (the base
lists of the 10M serving workload) are exact: each point's K nearest
candidates by the key (S, id), ties at the K-th distance going to the
smaller ids, checked by brute force on a small, heavily tied instance."""
import numpy as np
import torch

from workloads import synth


def test_component_lists_are_exact_under_ties():
    rng = np.random.default_rng(3)
    n, d, K = 600, 16, 20
    X = rng.integers(0, 3, (n, d)).astype(np.uint8)  # coordinates in {0, 1, 2}: many ties
    labels = rng.integers(0, 4, n)
    centres = rng.standard_normal((4, d))
    out = synth.knn_by_component(X, labels, centres, K, 1, torch.device("cpu"), batch=64)
    Xi = X.astype(np.int64)
    sets = synth.component_sets(labels, centres, 1)
    assert sum(m.size for m, _ in sets) == n
    for mem, cand in sets:
        assert np.all(np.isin(mem, cand))
        for p in mem:
            S = ((Xi[cand] - Xi[p]) ** 2).sum(axis=1)
            keys = sorted((int(s), int(c)) for s, c in zip(S, cand) if c != p)[:K]
            assert out[p].tolist() == [c for _, c in keys], p
