"""Clustering and adjacency for the oracle (test infrastructure only).

Paper anchors: §2.1 (graph G=(V,E) of A, block partition and block graph G_b), §3
(2N = 2^L red nodes from recursive bisection, pairwise merge I^s_i = I^r_{2i-1} u I^r_{2i}),
§3.1 (adjacency is that of the original graph and never changes; well separated = not
a neighbour).

Readings taken here (the paper leaves them open):

* Depth: L is the integer nearest to log2(n/leaf) (halves round up), at least 0 and at
  most floor(log2 n) so that no leaf is empty. Decided with integers only:
  L is the smallest L >= 0 with n^2 < leaf^2 * 2^(2L+1).
* Bisection: split a cluster along the axis of largest coordinate extent (ties: lowest
  axis) at the median after sorting by (coordinate, original index); the first
  ceil(size/2) entries go to the left child 2c, the rest to the right child 2c+1.
  Without coordinates the coordinate is the original index (1-D).
* Inside a leaf, unknowns are kept in ascending original index.
* Adjacency at depth d: clusters i != j are neighbours iff some nonzero a_uv has u in i
  and v in j. A cluster at depth d is the union of its descendant leaves.
"""
from __future__ import annotations

import numpy as np


def tree_depth(n: int, leaf: int) -> int:
    if n <= 1:
        return 0
    if leaf < 1:
        raise ValueError("leaf size must be >= 1")
    L = 0
    while not (n * n < leaf * leaf * (1 << (2 * L + 1))):
        L += 1
    cap = n.bit_length() - 1          # floor(log2 n)
    return min(L, cap)


def cluster_leaves(coords: np.ndarray | None, n: int, L: int) -> list[np.ndarray]:
    """Return the 2^L leaf clusters (arrays of original indices, ascending)."""
    if coords is None:
        coords = np.arange(n, dtype=np.float64)[:, None]
    coords = np.asarray(coords, dtype=np.float64).reshape(n, -1)
    clusters = [np.arange(n, dtype=np.int64)]
    for _ in range(L):
        nxt = []
        for c in clusters:
            x = coords[c]
            ext = x.max(axis=0) - x.min(axis=0)
            axis = int(np.argmax(ext))                 # first maximum = lowest axis
            order = np.lexsort((c, x[:, axis]))        # by coordinate, then index
            srt = c[order]
            half = (len(c) + 1) // 2
            nxt.append(np.sort(srt[:half]))
            nxt.append(np.sort(srt[half:]))
        clusters = nxt
    return clusters


def leaf_index(clusters: list[np.ndarray], n: int) -> np.ndarray:
    leaf_of = np.empty(n, dtype=np.int64)
    for i, c in enumerate(clusters):
        leaf_of[c] = i
    return leaf_of


def footprint_adjacency(row_ptr, col_idx, leaf_of: np.ndarray, L: int, d: int) -> set:
    """Set of ordered pairs (i, j), i != j, of depth-d clusters joined by a nonzero of A."""
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    cols = np.asarray(col_idx, dtype=np.int64)
    ci = leaf_of[rows] >> (L - d)
    cj = leaf_of[cols] >> (L - d)
    off = ci != cj
    code = np.unique(ci[off] * (1 << 32) + cj[off])
    return set(zip((code >> 32).tolist(), (code & 0xFFFFFFFF).tolist()))


class GeometricNeighbours:
    """Neighbour test of §7's experiments: two clusters are well separated when their distance
    is larger than the size of the clusters (reading R6g). Every unknown is a unit cell at its
    coordinates (the unknown's index as a 1-D coordinate when there are none); a cluster is the
    bounding box of its cells, [min, max + 1) per axis; its size is the largest side; the
    distance of two clusters is the Euclidean gap between their boxes. Clusters i != j at
    depth d are neighbours iff gap <= max(size_i, size_j). ``(i, j) in obj`` answers for
    depth-d cluster indices."""

    def __init__(self, coords, leaves: list, L: int, d: int):
        n = sum(len(c) for c in leaves)
        if coords is None:
            coords = np.arange(n, dtype=np.float64)[:, None]
        coords = np.asarray(coords, dtype=np.float64).reshape(n, -1)
        k = 1 << (L - d)
        groups = [np.concatenate(leaves[i * k:(i + 1) * k]) for i in range(1 << d)]
        self.lo = np.array([coords[g].min(axis=0) if len(g) else np.full(coords.shape[1], np.inf)
                            for g in groups])
        self.hi = np.array([coords[g].max(axis=0) + 1.0 if len(g) else np.full(coords.shape[1], -np.inf)
                            for g in groups])
        self.size = np.max(self.hi - self.lo, axis=1)

    def __contains__(self, pair) -> bool:
        i, j = pair
        if i == j:
            return False
        gap = np.maximum(0.0, np.maximum(self.lo[j] - self.hi[i], self.lo[i] - self.hi[j]))
        return bool(np.sqrt(np.sum(gap * gap)) <= max(self.size[i], self.size[j]))
