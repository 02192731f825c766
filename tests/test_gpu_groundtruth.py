"""The benchmark's float32 recall ground truth (exact_gt_f32: FP64 screening,
then re-ranking by FP64 distances and ids on the GPU) equals the oracle's
canonical (S, id) top-k (R9) on query samples of two float32 workloads, and
the uint8 one (integer keys) equals it as well."""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n,nq", [("tiny", 10_000, 200), ("deep_f32", 30_000, 100),
                                       ("sift_u8", 30_000, 100)])
def test_recall_ground_truth_equals_the_oracle(name, n, nq):
    import bench

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    w = workloads.build(name, n=n, nq=nq, device=dev, with_knn=False)
    k = 100
    X = torch.from_numpy(w.X).to(dev)
    Q = torch.from_numpy(w.Q).to(dev)
    gt = bench.exact_gt_u8(X, Q, k) if w.X.dtype == np.uint8 else bench.exact_gt_f32(X, Q, k)
    want = oracle.groundtruth(w.X, w.Q, k, threads=8)
    assert np.array_equal(gt.cpu().numpy(), want)
