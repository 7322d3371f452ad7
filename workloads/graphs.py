"""Seeded graph generators shaped like the paper's workloads (Section 5, Table 1).

The paper measures on public graphs (US airlines, migration, yeast, the
University of Florida matrices net50/100/150 and pattern1, a KDEEB-style
random graph). None of them is available here, so every workload below is a
synthetic stand-in drawn with numpy's PCG64 from a stated seed:

* ``tiny``            uniform random graph, 2 000 edges, one group, 256x256 grid;
* ``mid``             200 000 edges between 32 Gaussian node clusters, one group, 512x512;
* ``stack3d``         1 000 000 edges with Zipf(1.1) cluster popularity, 8 k-means
                      groups, 1024x1024x8 grid (the 3D density stack of Section 3.2);
* ``differentiation`` a sparse-matrix-pattern graph (rows on one axis, columns on the
                      other) with 5 000 000 edges, 8 groups, 2048x2048x8 grid;
* ``batched``         64 independent uniform graphs of uneven size, group count and grid.

Groups are drawn by k-means on the edge end points (Section 5 clusters edges by
origin and destination with k-means). Groups are data to the bundling method, so
the exact k-means details do not matter for parity: both the GPU path and the
oracle receive the same group array.

Node coordinates are float32 in [0, 1]^2 and the bounding box is the unit square,
so with power-of-two grid sides the map from node coordinates to pixel units is
exact in single precision.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    """One synthetic bundling problem: graph, groups, grid and schedule parameters."""

    name: str
    node_xy: np.ndarray          # float32 [n_nodes, 2], coordinates in the bounding box
    src: np.ndarray              # int32 [E]
    dst: np.ndarray              # int32 [E]
    group: np.ndarray            # int32 [E] in [0, B)
    M: np.ndarray                # float32 [B, B], M[l, b] = weight of bin b on layer l
    grid_w: int
    grid_h: int
    radii: List[int]             # box radius per iteration (last value repeats)
    n_iters: int
    delta: float = 1.0           # sampling step in pixels
    passes: int = 3              # box passes per map
    lam: float = 0.9             # bandwidth decay per iteration
    weight: Optional[np.ndarray] = None   # int32 [E] or None for unit weights
    bbox: tuple = (0.0, 0.0, 1.0, 1.0)
    seed: int = 0

    @property
    def n_edges(self) -> int:
        return int(self.src.shape[0])

    @property
    def n_groups(self) -> int:
        return int(self.M.shape[0])

    def describe(self) -> dict:
        return {
            "workload": self.name,
            "edges": self.n_edges,
            "nodes": int(self.node_xy.shape[0]),
            "groups": self.n_groups,
            "grid": [self.grid_w, self.grid_h],
            "delta_px": self.delta,
            "box_passes": self.passes,
            "iterations": self.n_iters,
            "radius_first_last": [self.radii[0], self.radii[-1]],
        }


# ---------------------------------------------------------------- building blocks

def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _pairs_without_loops(rng, draw, n_edges):
    """Draw (src, dst) with ``draw(rng, k) -> (s, t)`` and redraw self-loops."""
    s, t = draw(rng, n_edges)
    bad = np.nonzero(s == t)[0]
    while bad.size:
        s2, t2 = draw(rng, bad.size)
        s[bad], t[bad] = s2, t2
        bad = bad[s[bad] == t[bad]]
    return s.astype(np.int32), t.astype(np.int32)


def uniform_graph(n_nodes: int, n_edges: int, seed: int):
    """Nodes uniform in the unit square; edges between uniform node pairs."""
    rng = _rng(seed)
    xy = rng.random((n_nodes, 2)).astype(np.float32)

    def draw(r, k):
        return r.integers(0, n_nodes, k), r.integers(0, n_nodes, k)

    s, t = _pairs_without_loops(rng, draw, n_edges)
    return xy, s, t


def clustered_graph(n_clusters: int, per_cluster: int, n_edges: int, seed: int,
                    sigma: float = 0.02, intra: float = 0.7):
    """Isotropic Gaussian node clusters; a fraction ``intra`` of edges stays in one cluster."""
    rng = _rng(seed)
    centres = 0.1 + 0.8 * rng.random((n_clusters, 2))
    pts = centres[:, None, :] + sigma * rng.standard_normal((n_clusters, per_cluster, 2))
    xy = np.clip(pts.reshape(-1, 2), 0.0, 1.0).astype(np.float32)

    def draw(r, k):
        ca = r.integers(0, n_clusters, k)
        cb = r.integers(0, n_clusters - 1, k)
        cb = cb + (cb >= ca)                     # a distinct cluster
        same = r.random(k) < intra
        cb = np.where(same, ca, cb)
        s = ca * per_cluster + r.integers(0, per_cluster, k)
        t = cb * per_cluster + r.integers(0, per_cluster, k)
        return s, t

    s, t = _pairs_without_loops(rng, draw, n_edges)
    return xy, s, t


def zipf_cluster_graph(n_clusters: int, per_cluster: int, n_background: int,
                       n_edges: int, seed: int, zipf_a: float = 1.1,
                       p_background: float = 0.2, sigma: float = 0.02):
    """Gaussian clusters with Zipf(a) popularity plus a uniform background.

    Each end point is a uniform background node with probability
    ``p_background``; otherwise a cluster is drawn by Zipf rank (truncated to
    ``n_clusters``, rank mapped to a cluster by a seeded permutation) and the end
    point is a uniform node of that cluster.
    """
    rng = _rng(seed)
    centres = 0.1 + 0.8 * rng.random((n_clusters, 2))
    pts = centres[:, None, :] + sigma * rng.standard_normal((n_clusters, per_cluster, 2))
    cl_xy = np.clip(pts.reshape(-1, 2), 0.0, 1.0)
    bg_xy = rng.random((n_background, 2))
    xy = np.concatenate([cl_xy, bg_xy]).astype(np.float32)
    ranks = np.arange(1, n_clusters + 1, dtype=np.float64)
    pz = ranks ** (-zipf_a)
    pz /= pz.sum()
    perm = rng.permutation(n_clusters)
    n_cl = n_clusters * per_cluster

    def end(r, k):
        bg = r.random(k) < p_background
        cl = perm[r.choice(n_clusters, size=k, p=pz)]
        node_cl = cl * per_cluster + r.integers(0, per_cluster, k)
        node_bg = n_cl + r.integers(0, n_background, k)
        return np.where(bg, node_bg, node_cl)

    def draw(r, k):
        return end(r, k), end(r, k)

    s, t = _pairs_without_loops(rng, draw, n_edges)
    return xy, s, t


def matrix_pattern_graph(n: int, n_edges: int, seed: int, band: int = 100,
                         n_blocks: int = 64, block: int = 150, fill: float = 0.001):
    """Sparse-matrix pattern drawn as a graph: row i links to column j for nonzero (i, j).

    Row nodes sit on a vertical axis and column nodes on a horizontal axis of a
    square matrix plot. The pattern is a band |i-j| <= ``band``, ``n_blocks``
    dense ``block`` x ``block`` blocks at random places and a uniform fill,
    deduplicated and subsampled to exactly ``n_edges`` nonzeros.
    """
    rng = _rng(seed)
    parts = []
    # band
    for d in range(-band, band + 1):
        i = np.arange(max(0, -d), min(n, n - d), dtype=np.int64)
        parts.append(i * n + (i + d))
    # dense blocks
    for _ in range(n_blocks):
        r0 = int(rng.integers(0, n - block + 1))
        c0 = int(rng.integers(0, n - block + 1))
        ii, jj = np.meshgrid(np.arange(r0, r0 + block), np.arange(c0, c0 + block), indexing="ij")
        parts.append((ii * n + jj).ravel().astype(np.int64))
    # uniform fill
    k = int(round(fill * n * n))
    parts.append(rng.integers(0, n * n, k, dtype=np.int64))
    nz = np.unique(np.concatenate(parts))
    if nz.size > n_edges:
        nz = np.sort(rng.choice(nz, size=n_edges, replace=False))
    i = nz // n
    j = nz % n
    pos = (np.arange(n, dtype=np.float64) + 0.5) / n
    rows = np.stack([np.full(n, 0.02), 0.98 - 0.96 * pos], axis=1)
    cols = np.stack([0.02 + 0.96 * pos, np.full(n, 0.98)], axis=1)
    xy = np.concatenate([rows, cols]).astype(np.float32)
    return xy, i.astype(np.int32), (n + j).astype(np.int32)


def kmeans_groups(features: np.ndarray, k: int, seed: int, max_iter: int = 100) -> np.ndarray:
    """k-means++ initialisation and Lloyd iterations until the assignment is stable."""
    if k <= 1:
        return np.zeros(features.shape[0], dtype=np.int32)
    rng = _rng(seed)
    X = np.ascontiguousarray(features, dtype=np.float64)
    n = X.shape[0]
    sample = X if n <= 200_000 else X[rng.choice(n, 200_000, replace=False)]
    centres = [sample[rng.integers(0, sample.shape[0])]]
    d2 = ((sample - centres[0]) ** 2).sum(1)
    for _ in range(1, k):
        p = d2 / d2.sum() if d2.sum() > 0 else None
        c = sample[rng.choice(sample.shape[0], p=p)]
        centres.append(c)
        d2 = np.minimum(d2, ((sample - c) ** 2).sum(1))
    C = np.array(centres)
    labels = None
    xx = (X ** 2).sum(1)
    for _ in range(max_iter):
        dist = xx[:, None] - 2.0 * X @ C.T + (C ** 2).sum(1)[None, :]
        new = np.argmin(dist, axis=1)
        if labels is not None and np.array_equal(new, labels):
            break
        labels = new
        for c in range(k):
            m = labels == c
            if m.any():
                C[c] = X[m].mean(0)
    return labels.astype(np.int32)


def interaction_eq4(B: int, alpha: float = 0.25) -> np.ndarray:
    """Section 3.2, Eq. 4: one on the diagonal, -alpha/(B-1) elsewhere."""
    if B == 1:
        return np.ones((1, 1), dtype=np.float32)
    M = np.full((B, B), -alpha / (B - 1), dtype=np.float64)
    np.fill_diagonal(M, 1.0)
    return M.astype(np.float32)


def interaction_constant(B: int, diag: float = 1.0, off: float = 0.2) -> np.ndarray:
    M = np.full((B, B), off, dtype=np.float64)
    np.fill_diagonal(M, diag)
    return M.astype(np.float32)


def radius_schedule(r0: float, r_last: float, T: int) -> List[int]:
    """Geometric radius list from r0 to r_last over T iterations, rounded to integers."""
    if T == 1:
        return [int(math.floor(r0 + 0.5))]
    q = r_last / r0
    return [int(math.floor(r0 * q ** (i / (T - 1)) + 0.5)) for i in range(T)]


def _od_features(xy, s, t):
    return np.concatenate([xy[s], xy[t]], axis=1)


# ---------------------------------------------------------------- the five workloads

def tiny(seed: int = 0) -> Workload:
    """500 uniform nodes, 2 000 uniform edges, one group, 256x256, radius 8, 10 iterations."""
    xy, s, t = uniform_graph(500, 2000, seed)
    return Workload("tiny-2k-256x1", xy, s, t, np.zeros(2000, np.int32),
                    np.ones((1, 1), np.float32), 256, 256, [8] * 10, 10, seed=seed)


def mid(seed: int = 0) -> Workload:
    """32 Gaussian clusters of 625 nodes, 200 000 edges (70 % intra-cluster), 512x512, 20 iterations."""
    xy, s, t = clustered_graph(32, 625, 200_000, seed)
    return Workload("mid-200k-512x1", xy, s, t, np.zeros(200_000, np.int32),
                    np.ones((1, 1), np.float32), 512, 512,
                    radius_schedule(16, 4, 20), 20, seed=seed)


def stack3d(seed: int = 0, n_edges: int = 1_000_000, grid: int = 1024, groups: int = 8,
            n_iters: int = 30, name: Optional[str] = None) -> Workload:
    """64 Zipf-popular clusters + 20 % background, 8 k-means groups, 1024x1024x8, 30 iterations."""
    xy, s, t = zipf_cluster_graph(64, 1250, 20_000, n_edges, seed)
    g = kmeans_groups(_od_features(xy, s, t), groups, seed=1)
    r0 = grid / 32.0
    return Workload(name or f"stack3d-{n_edges // 1000}k-{grid}x{groups}", xy, s, t, g,
                    interaction_constant(groups, 1.0, 0.2), grid, grid,
                    radius_schedule(r0, r0 / 4.0, n_iters), n_iters, seed=seed)


def differentiation(seed: int = 2, n: int = 20_000, n_edges: int = 5_000_000,
                    grid: int = 2048, groups: int = 8, delta: float = 4.0,
                    n_iters: int = 5, band: int = 100, n_blocks: int = 64, block: int = 150,
                    fill: float = 0.001) -> Workload:
    """Matrix-pattern graph, 8 k-means groups, 2048x2048x8, sampling step 4 px, 5 iterations
    (the pattern's band, blocks and fill can be scaled down with the matrix)."""
    xy, s, t = matrix_pattern_graph(n, n_edges, seed, band, n_blocks, block, fill)
    g = kmeans_groups(_od_features(xy, s, t), groups, seed=1)
    r0 = grid / 32.0
    return Workload(f"differentiation-{n_edges // 1000}k-{grid}x{groups}", xy, s, t, g,
                    interaction_eq4(groups, 0.25), grid, grid,
                    radius_schedule(r0, r0 / 4.0, n_iters), n_iters, delta=delta, seed=seed)


def batched(n_graphs: int = 64, first_seed: int = 100, e_min: int = 1000,
            e_max: int = 500_000, n_iters: int = 20, sides=(256, 512, 1024),
            max_groups: int = 16) -> List[Workload]:
    """Independent uniform graphs of log-uniform size, 1..16 k-means groups, grids 256/512/1024."""
    out = []
    for gi in range(n_graphs):
        seed = first_seed + gi
        rng = _rng(seed)
        E = int(round(math.exp(rng.uniform(math.log(e_min), math.log(e_max)))))
        B = int(rng.integers(1, max_groups + 1))
        side = int(sides[int(rng.integers(0, len(sides)))])
        n_nodes = max(500, E // 4)
        xy, s, t = uniform_graph(n_nodes, E, seed)
        g = kmeans_groups(_od_features(xy, s, t), B, seed=seed)
        out.append(Workload(f"batch{gi:02d}-{E}-{side}x{B}", xy, s, t, g,
                            interaction_eq4(B, 0.25), side, side,
                            radius_schedule(side / 32.0, side / 128.0, n_iters), n_iters,
                            seed=seed))
    return out


def scaled(kind: str, n_edges: int, grid: int, groups: int = 1, n_iters: int = 3,
           seed: int = 7, delta: float = 1.0) -> Workload:
    """Small versions of the workload shapes for parity tests."""
    if kind == "uniform":
        xy, s, t = uniform_graph(max(50, n_edges // 4), n_edges, seed)
    elif kind == "clustered":
        xy, s, t = clustered_graph(16, max(8, n_edges // 64), n_edges, seed)
    elif kind == "zipf":
        xy, s, t = zipf_cluster_graph(16, max(8, n_edges // 40), max(8, n_edges // 10),
                                      n_edges, seed)
    else:
        raise ValueError(kind)
    g = kmeans_groups(_od_features(xy, s, t), groups, seed=1)
    M = interaction_eq4(groups, 0.25) if groups > 1 else np.ones((1, 1), np.float32)
    r0 = max(1.0, grid / 32.0)
    return Workload(f"{kind}-{n_edges}-{grid}x{groups}", xy, s, t, g, M, grid, grid,
                    radius_schedule(r0, max(1.0, r0 / 4.0), n_iters), n_iters,
                    delta=delta, seed=seed)


WORKLOADS = {
    "tiny": tiny,
    "mid": mid,
    "stack3d": stack3d,
    "differentiation": differentiation,
}
