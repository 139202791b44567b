"""Pins of the clustering-score oracle (CPU): hand-worked examples, an
independent library implementation of the silhouette, brute force and
invariants."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import cluster

HERE = os.path.dirname(os.path.abspath(__file__))


def _examples():
    rows = []
    for line in open(os.path.join(HERE, "golden", "cluster_examples.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        f = [x.strip() for x in line.split(";")]
        N = int(f[0])
        cond = [float(v) for v in f[1].split()]
        labels = [int(v) for v in f[2].split()]
        cents = [int(v) for v in f[3].split()]
        cost = float(f[4])
        sil = [float(Fraction(v)) for v in f[5].split()]
        alab = [int(v) for v in f[6].split()]
        atot = float(f[7])
        rows.append((N, cond, labels, cents, cost, sil, alab, atot))
    return rows


@pytest.mark.parametrize("ex", _examples())
def test_hand_examples(ex):
    N, cond, labels, cents, cost, sil, alab, atot = ex
    total, per = cluster.cluster_cost(cond, N, labels, cents)
    assert total == cost and per.sum() == cost
    s, mean = cluster.silhouette(cond, N, labels, len(cents))
    assert np.allclose(s, sil, rtol=0, atol=1e-15) and abs(mean - np.mean(sil)) < 1e-15
    lab, tot = cluster.assign(cond, N, cents)
    assert list(lab) == alab and tot == atot


def _random_case(seed, N, K):
    rng = np.random.default_rng(seed)
    pts = rng.normal(size=(N, 3)) + rng.integers(0, K, size=N)[:, None] * 3.0
    D = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)) ** 2
    cond = D[np.triu_indices(N, 1)]
    labels = rng.integers(0, K, size=N)
    labels[:K] = np.arange(K)  # every cluster non-empty
    return cond, labels


@pytest.mark.parametrize("seed,N,K", [(0, 30, 2), (1, 60, 5), (2, 41, 7), (3, 12, 11)])
def test_silhouette_matches_scikit_learn(seed, N, K):
    from sklearn.metrics import silhouette_samples
    cond, labels = _random_case(seed, N, K)
    s, mean = cluster.silhouette(cond, N, labels, K)
    ref = silhouette_samples(cluster.square(cond, N), labels, metric="precomputed")
    assert np.allclose(s, ref, rtol=0, atol=1e-12)
    assert abs(mean - ref.mean()) < 1e-12


def test_silhouette_bounds_and_separated_clusters():
    cond, labels = _random_case(4, 50, 4)
    s, _ = cluster.silhouette(cond, 50, labels, 4)
    assert np.all(s >= -1) and np.all(s <= 1)
    # two tight, far-apart groups: silhouettes close to 1
    pts = np.concatenate([np.zeros(10), np.full(10, 100.0)]) + np.linspace(0, 1, 20)
    D = np.abs(pts[:, None] - pts[None, :])
    s, mean = cluster.silhouette(D[np.triu_indices(20, 1)], 20, np.repeat([0, 1], 10), 2)
    assert mean > 0.98


def test_assignment_is_the_best_labelling_for_its_centroids():
    cond, _ = _random_case(5, 9, 3)
    cents = [0, 4, 7]
    lab, tot = cluster.assign(cond, 9, cents)
    D = cluster.square(cond, 9)
    # brute force over all 3^9 labellings with these centroids
    best = np.inf
    for code in range(3 ** 9):
        l = [(code // 3 ** i) % 3 for i in range(9)]
        best = min(best, sum(D[i, cents[l[i]]] for i in range(9)))
    assert abs(tot - best) < 1e-12
    total, _ = cluster.cluster_cost(cond, 9, lab, cents)
    assert abs(total - tot) < 1e-12


def test_cost_zero_when_every_series_is_its_own_centroid():
    cond, _ = _random_case(6, 8, 2)
    total, per = cluster.cluster_cost(cond, 8, np.arange(8), np.arange(8))
    assert total == 0.0 and np.all(per == 0.0)
