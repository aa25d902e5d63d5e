"""Synthetic attributed-graph pairs standing in for the paper's datasets.

The paper evaluates on VGG affine image graphs (fully connected, distance
weights), CMU House and the SNAP Facebook ego network (Sec. 7, Table of
datasets).  None of those are available, so pairs are drawn here with the
same structure: a nonnegative symmetric edge matrix A with zero diagonal
(Sec. 3, "Graph"), and a second graph that is a relabelled, noisy copy of
it, so the hidden correspondence is known.

Conventions (fixed here, shared by every consumer):

* ``perm[k]`` is the node of the second graph that node ``k`` of the first
  graph maps to, i.e. ``B[perm[k], perm[l]] = A[k, l]`` before noise.
  The matching matrix of Sec. 3 is then ``M[k, perm[k]] = 1``.
* Noise is Gaussian, symmetric and only on existing edges; the result is
  clipped at zero so B stays nonnegative (Sec. 3 requires it); edges that
  reach zero count as deleted.
* Deletions zero an edge in both directions.
* Outlier nodes of B get fresh Erdos-Renyi rows/columns; the hidden
  correspondence is only meaningful on the remaining (inlier) nodes.

Seeds: pair ``i`` of workload ``c`` uses ``numpy.random.default_rng(1000*c + i)``.

Attributed pairs (node term of eq. 1) add nonnegative node features: F is
n x d with U(0,1) entries and unit-norm rows (descriptor-like histograms), the
second graph's features are the relabelled copy plus clipped Gaussian noise,
and K = F F~^T is their similarity matrix (K[k, perm[k]] is largest when the
noise is small).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class GraphPair:
    A: np.ndarray          # (n, n) float64, symmetric, >= 0, zero diagonal
    B: np.ndarray          # (n, n) float64, symmetric, >= 0, zero diagonal
    perm: np.ndarray       # (n,) int64 hidden correspondence, A node k -> B node perm[k]
    inlier: np.ndarray     # (n,) bool, A nodes whose image in B is not an outlier
    seed: int

    @property
    def n(self) -> int:
        return self.A.shape[0]


def er_adjacency(rng: np.random.Generator, n: int, p: float,
                 weights: str = "open") -> np.ndarray:
    """Symmetric Erdos-Renyi weighted adjacency with zero diagonal.

    ``weights="open"`` draws U(0,1) (numpy's [0,1) interval); ``"half_open_top"``
    draws U(0,1] as ``1 - rng.random()`` so that no present edge has weight 0.
    """
    present = rng.random((n, n)) < p
    w = rng.random((n, n))
    if weights == "half_open_top":
        w = 1.0 - w
    A = np.triu(np.where(present, w, 0.0), 1)
    return A + A.T


def _sym_upper(M: np.ndarray) -> np.ndarray:
    U = np.triu(M, 1)
    return U + U.T


def permuted_noisy_copy(rng: np.random.Generator, A: np.ndarray, sigma: float,
                        delete_frac: float = 0.0, outlier_frac: float = 0.0,
                        outlier_p: float = 0.0):
    """Relabel A by a random permutation and perturb it (see module conventions)."""
    n = A.shape[0]
    perm = rng.permutation(n)
    B = np.empty_like(A)
    B[np.ix_(perm, perm)] = A
    if sigma > 0:
        noise = _sym_upper(rng.normal(0.0, sigma, (n, n)))
        B = np.where(B > 0, np.maximum(B + noise, 0.0), 0.0)
    if delete_frac > 0:
        iu, ju = np.nonzero(np.triu(B, 1) > 0)
        k = int(round(delete_frac * iu.size))
        if k:
            pick = rng.choice(iu.size, size=k, replace=False)
            B[iu[pick], ju[pick]] = 0.0
            B[ju[pick], iu[pick]] = 0.0
    outlier_nodes = np.zeros(n, dtype=bool)
    if outlier_frac > 0:
        m = int(round(outlier_frac * n))
        out = rng.choice(n, size=m, replace=False)
        outlier_nodes[out] = True
        fresh = er_adjacency(rng, n, outlier_p)
        mask = outlier_nodes[:, None] | outlier_nodes[None, :]
        B = np.where(mask, fresh, B)
    np.fill_diagonal(B, 0.0)
    inlier = ~outlier_nodes[perm]
    return B, perm.astype(np.int64), inlier


# Workload table: the five synthetic workloads (sizes, densities, noise).
CONFIGS = {
    0: dict(n=50, p=0.2, weights="half_open_top", sigma=0.02, delete=0.0, outlier=0.0,
            theta=2.0, iters=100, tol=0.0, pairs=100),
    1: dict(n=1000, p=0.5, weights="open", sigma=0.05, delete=0.05, outlier=0.0,
            theta=2.0, iters=100, tol=0.0, pairs=10),
    2: dict(n=4000, p=0.3, weights="open", sigma=0.05, delete=0.0, outlier=0.10,
            theta=2.0, iters=100, tol=0.0, pairs=5),
}


def make_pair(n: int, p: float, sigma: float, seed: int, weights: str = "open",
              delete_frac: float = 0.0, outlier_frac: float = 0.0) -> GraphPair:
    rng = np.random.default_rng(seed)
    A = er_adjacency(rng, n, p, weights)
    B, perm, inlier = permuted_noisy_copy(rng, A, sigma, delete_frac, outlier_frac, p)
    return GraphPair(A=A, B=B, perm=perm, inlier=inlier, seed=seed)


@dataclasses.dataclass
class AttributedPair(GraphPair):
    K: np.ndarray | None = None   # (n, n) float64 node similarities F F~^T, >= 0


def make_attributed_pair(n: int, p: float, sigma: float, seed: int, d: int = 16,
                         feat_sigma: float = 0.05, weights: str = "open") -> AttributedPair:
    """A noisy relabelled pair (as make_pair, no deletions or outliers) with
    node features; see the module notes for K."""
    base = make_pair(n, p, sigma, seed, weights)
    rng = np.random.default_rng(seed + 7_000_000)
    F = rng.random((n, d))
    F /= np.linalg.norm(F, axis=1, keepdims=True)
    Ft = np.empty_like(F)
    Ft[base.perm] = F
    if feat_sigma > 0:
        Ft = np.maximum(Ft + rng.normal(0.0, feat_sigma, Ft.shape), 0.0)
    return AttributedPair(A=base.A, B=base.B, perm=base.perm, inlier=base.inlier,
                          seed=seed, K=F @ Ft.T)


def config_sizes(config: int) -> dict:
    return dict(CONFIGS[config])


def config_pairs(config: int, indices=None, n_override: int | None = None):
    """Yield the seeded pairs of workload 0, 1 or 2 (seed = 1000*config + index)."""
    cfg = CONFIGS[config]
    if indices is None:
        indices = range(cfg["pairs"])
    for i in indices:
        yield make_pair(n_override or cfg["n"], cfg["p"], cfg["sigma"], 1000 * config + i,
                        cfg["weights"], cfg["delete"], cfg["outlier"])


def batched_pairs(count: int = 512, n_lo: int = 20, n_hi: int = 300, seed: int = 3000):
    """Many independent pairs of uneven size: n ~ U{n_lo..n_hi}, p ~ U(0.1, 0.5),
    sigma = 0.03.  One master stream picks the sizes, pair i uses seed*1000+i."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ps = rng.uniform(0.1, 0.5, size=count)
    return [make_pair(int(ns[i]), float(ps[i]), 0.03, seed * 1000 + i) for i in range(count)]


def serve_requests(rate: float = 200.0, duration_s: float = 30.0, warmup_s: float = 5.0,
                   n_lo: int = 30, n_hi: int = 2000, seed: int = 4000):
    """Poisson arrival times and log-uniform sizes for the served workload.

    Returns a list of (arrival_time_s, n, pair_seed).  Graphs are drawn lazily
    with ``make_pair(n, 0.3, 0.05, pair_seed)`` so the list itself is cheap.
    """
    rng = np.random.default_rng(seed)
    total = warmup_s + duration_s
    t, out, i = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= total:
            break
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append((t, n, seed * 1000 + i))
        i += 1
    return out
