"""GPU clustering scores (silhouette, cost, nearest-centroid assignment) from a
condensed distance matrix, through the C ABI, against the FP64 oracle run on the
same FP32 matrix values."""
import numpy as np
import pytest

from oracle import cluster
from paper_2307_04904_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu():
    from paper_2307_04904_amd import binding
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return binding


def _random_matrix(seed, N):
    rng = np.random.default_rng(seed)
    return (rng.random(N * (N - 1) // 2) * 100.0).astype(np.float32)


def _labels(seed, N, K, empty=()):
    rng = np.random.default_rng(seed)
    allowed = np.array([k for k in range(K) if k not in empty])
    lab = rng.choice(allowed, size=N).astype(np.int32)
    lab[:2] = allowed[:2]  # at least two non-empty clusters
    return lab


# N across the 512-row and 512-column super-tiles of the single-read kernel (K <= 16)
# and K past it (17, 64: the two-read kernel)
@pytest.mark.parametrize("N,K", [(2, 2), (3, 2), (65, 3), (130, 7), (255, 16), (257, 5), (513, 16), (1025, 12),
                                 (2100, 9), (300, 17), (300, 64), (1000, 10)])
def test_silhouette_random_matrices(N, K):
    B = _gpu()
    D = _random_matrix(N, N)
    lab = _labels(N + K, N, K, empty=(K - 1,) if K > 2 and N > 3 else ())
    if N >= 10:
        lab[5] = K - 1 if K > 2 else lab[5]  # a one-member cluster
    s_ref, mean_ref = cluster.silhouette(D.astype(np.float64), N, lab, K)
    d = torch.from_numpy(D).cuda()
    s = torch.full((N,), float("nan"), device="cuda")
    mean = B.silhouette(d, N, torch.from_numpy(lab).cuda(), K, s_out=s)
    torch.cuda.synchronize()
    assert np.allclose(s.cpu().numpy(), s_ref, rtol=0, atol=1e-6)
    assert abs(mean - mean_ref) <= 1e-12 * max(1.0, abs(mean_ref))
    # same result on a second run (fixed-order sums)
    assert B.silhouette(d, N, torch.from_numpy(lab).cuda(), K) == mean


def test_scores_on_a_dtw_matrix():
    # the matrix the library computes, then the scores of a k-medoids step on it
    B = _gpu()
    ds = synth.small_random(seed=90, N=257, len_lo=40, len_hi=300, window=20)
    D = B.pairwise(ds)
    torch.cuda.synchronize()
    Dh = D.cpu().numpy().astype(np.float64)
    cents = np.array([3, 40, 77, 200, 256], dtype=np.int32)
    lab_out = torch.full((ds.N,), -1, dtype=torch.int32, device="cuda")
    total, per = B.assign(D, ds.N, torch.from_numpy(cents).cuda(), lab_out)
    lab_ref, total_ref = cluster.assign(Dh, ds.N, cents)
    lab = lab_out.cpu().numpy()
    assert np.array_equal(lab, lab_ref)
    assert abs(total - total_ref) <= 1e-12 * total_ref
    ctot, cper = B.cluster_cost(D, ds.N, lab_out, torch.from_numpy(cents).cuda())
    rtot, rper = cluster.cluster_cost(Dh, ds.N, lab_ref, cents)
    assert abs(ctot - rtot) <= 1e-12 * rtot and np.allclose(cper, rper, rtol=1e-12, atol=0)
    assert np.allclose(per, rper, rtol=1e-12, atol=0)
    mean = B.silhouette(D, ds.N, lab_out, len(cents))
    _, mean_ref = cluster.silhouette(Dh, ds.N, lab_ref, len(cents))
    assert abs(mean - mean_ref) <= 1e-12


def test_assignment_ties_go_to_the_lowest_cluster():
    B = _gpu()
    # points 0, 5, 10 on a line: series 1 is at distance 5 from both centroids
    D = torch.tensor([5.0, 10.0, 5.0], device="cuda")
    lab = torch.full((3,), -1, dtype=torch.int32, device="cuda")
    total, per = B.assign(D, 3, torch.tensor([0, 2], dtype=torch.int32, device="cuda"), lab)
    assert lab.cpu().tolist() == [0, 0, 1] and total == 5.0 and per == [5.0, 0.0]


def test_out_of_range_labels_rejected():
    B = _gpu()
    D = torch.zeros(3, device="cuda")
    with pytest.raises(B.DtwError):
        B.silhouette(D, 3, torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda"), 2)
    with pytest.raises(B.DtwError):
        B.cluster_cost(D, 3, torch.tensor([0, 0, 1], dtype=torch.int32, device="cuda"),
                       torch.tensor([0, 3], dtype=torch.int32, device="cuda"))
