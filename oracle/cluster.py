"""FP64 CPU oracle for the clustering scores computed from the DTW distance matrix.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  It shares no code with the GPU
library and never imports it.

The paper's method, after the distance matrix D, splits the series into k
clusters with a representative centroid series each, outputs the clustering
cost -- the sum of the distances between every series of a cluster and that
cluster's centroid -- and a silhouette score to help choose k (Introduction,
list of the method's steps).  The paper does not spell the silhouette out;
this module uses Rousseeuw's definition:

  for series i in cluster A,
    a(i) = mean of D(i, j) over the other members j of A,
    b(i) = smallest, over the other non-empty clusters B, of the mean of D(i, j) over j in B,
    s(i) = (b(i) - a(i)) / max(a(i), b(i)), taken as 0 when both are 0,
    s(i) = 0 when A has one member;
  the score is the mean of s(i).

A k-medoids assignment step puts each series in the cluster of its nearest
centroid; ties go to the lowest cluster index.

D is given as the condensed upper triangle of the symmetric matrix (zero
diagonal), entry k(i, j) = i*N - i*(i+1)/2 + (j-i-1) for i < j.
"""
from __future__ import annotations

import numpy as np


def square(condensed, N: int) -> np.ndarray:
    """The full symmetric N x N matrix (FP64) of a condensed upper triangle."""
    c = np.asarray(condensed, dtype=np.float64)
    if c.size != N * (N - 1) // 2:
        raise ValueError("condensed size %d does not match N=%d" % (c.size, N))
    D = np.zeros((N, N), dtype=np.float64)
    iu = np.triu_indices(N, 1)
    D[iu] = c
    D[(iu[1], iu[0])] = c
    return D


def cluster_cost(condensed, N: int, labels, centroids):
    """(total, per_cluster): sum over series i of D(i, centroids[labels[i]])."""
    D = square(condensed, N)
    labels = np.asarray(labels, dtype=np.int64)
    centroids = np.asarray(centroids, dtype=np.int64)
    K = len(centroids)
    per = np.zeros(K, dtype=np.float64)
    for i in range(N):
        per[labels[i]] += D[i, centroids[labels[i]]]
    return float(per.sum()), per


def assign(condensed, N: int, centroids):
    """(labels, total): each series joins its nearest centroid (lowest index on ties)."""
    D = square(condensed, N)
    centroids = np.asarray(centroids, dtype=np.int64)
    labels = np.empty(N, dtype=np.int32)
    total = 0.0
    for i in range(N):
        best, lab = np.inf, -1
        for c, m in enumerate(centroids):
            if D[i, m] < best:
                best, lab = D[i, m], c
        labels[i] = lab
        total += best
    return labels, total


def silhouette(condensed, N: int, labels, K: int):
    """(s, mean): per-series silhouette values and their mean."""
    D = square(condensed, N)
    labels = np.asarray(labels, dtype=np.int64)
    sizes = np.bincount(labels, minlength=K)
    s = np.zeros(N, dtype=np.float64)
    for i in range(N):
        A = labels[i]
        if sizes[A] <= 1:
            continue
        sums = np.bincount(labels, weights=D[i], minlength=K)  # D[i, i] = 0 adds nothing
        a = sums[A] / (sizes[A] - 1)
        b = min(sums[B] / sizes[B] for B in range(K) if B != A and sizes[B] > 0)
        m = max(a, b)
        s[i] = 0.0 if m == 0.0 else (b - a) / m
    return s, float(s.mean())
