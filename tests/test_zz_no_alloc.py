"""rp_knn_u8_noalloc (the entry point that allocates nothing) against
rp_knn_u8 through the C-ABI: identical lists on two calls in a row, the second
smaller, with the candidate set split into slices so the fixed workspace is
used; a call that needs more workspace than it holds is rejected."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_noalloc_equals_allocating_entry_point():
    from paper_2602_08097_amd.rp import RPError, knn_u8, knn_u8_noalloc

    dev = _dev()
    rng = np.random.default_rng(77)
    n, d = 60_000, 64
    X = torch.from_numpy(rng.integers(0, 256, (n, d)).astype(np.uint8)).to(dev)
    X[500:520] = X[3]  # duplicates: exact ties by id
    for nq, K, slices in ((300, 128, 0), (70, 33, 9)):
        q = torch.from_numpy(np.sort(rng.choice(n, nq, replace=False)).astype(np.int32)).to(dev)
        want = knn_u8(X, K, query_ids=q)
        out = torch.full((nq, K), -7, dtype=torch.int32, device=dev)
        got = knn_u8_noalloc(X, K, out, query_ids=q, slices=slices)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (nq, K, slices)
        # the same call again on the used workspace
        out.fill_(-7)
        knn_u8_noalloc(X, K, out, query_ids=q, slices=slices)
        torch.cuda.synchronize()
        assert torch.equal(out, want), (nq, K, slices, "repeat")
    # 64 slices of 2,000 queries need 125 MiB: more than the 64 MiB workspace
    q = torch.arange(2000, dtype=torch.int32, device=dev)
    out = torch.empty((2000, 16), dtype=torch.int32, device=dev)
    with pytest.raises(RPError, match="RP_EINVAL"):
        knn_u8_noalloc(X, 16, out, query_ids=q, slices=64)
