"""Seeded synthetic inputs for the APPD path (no method arithmetic lives here).

Both the GPU path and the CPU oracle consume what these functions return; this
module computes no minimax distance, spanning tree or selection.  The paper's
benchmark datasets (seven real datasets turned into complete graphs, Section 4,
Table 2) are not available, so these seeded recipes stand in for them:

  single_points_2d   n points uniform in [0,1]^2; Euclidean weights computed in
                     float64 and rounded once to float32 (n = 256 by default).
  gaussian_mixture   n points in R^16 from 10 equal-weight Gaussian components,
                     centres uniform in [0,1]^16, sigma 0.05 (n = 8192).
  uniform_symmetric  symmetric weights whose upper-triangle entries are i.i.d.
                     float32 uniform [0,1), zero diagonal (n = 32768).
  ragged_points      a batch of independent point-set graphs, n log-uniform in
                     [16, 1024], d drawn from {2, 8}, points uniform in [0,1]^d.
  diff_batch         a batch for the differentiable path: n uniform in
                     {64..2048}, X ~ N(0, I_8) float32, upstream gradient
                     G ~ N(0,1) float32 (full n x n, not symmetric).
  integer_weights    tie-heavy symmetric weights drawn from {0, 1, ..., L-1}.

Euclidean weights from points: W_ij = float32(sqrt(sum_t (x_it - x_jt)^2)) with
the differences, squares and the sum over t (in increasing t) in float64, so W
is exactly symmetric with a zero diagonal.
"""
from __future__ import annotations

import math

import numpy as np

SEEDS = {"single": 1, "mixture": 2, "uniform": 3, "ragged": 4, "diff": 5}


def euclid_w(X: np.ndarray, chunk: int = 64) -> np.ndarray:
    """float64 direct-difference Euclidean distances, rounded once to float32."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, d = X.shape
    W = np.empty((n, n), np.float32)
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        acc = np.zeros((i1 - i0, n), np.float64)
        for t in range(d):
            diff = X[i0:i1, t][:, None] - X[None, :, t]
            acc += diff * diff
        W[i0:i1] = np.sqrt(acc).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    return W


def single_points_2d(n: int = 256, seed: int = SEEDS["single"]) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, 2))


def gaussian_mixture_points(n: int = 8192, d: int = 16, k: int = 10, sigma: float = 0.05,
                            seed: int = SEEDS["mixture"]) -> np.ndarray:
    rng = np.random.default_rng(seed)
    centres = rng.random((k, d))
    label = rng.integers(0, k, n)
    return centres[label] + sigma * rng.standard_normal((n, d))


def uniform_symmetric(n: int = 32768, seed: int = SEEDS["uniform"], out: np.ndarray = None):
    """Symmetric float32 W, upper triangle i.i.d. uniform [0,1), zero diagonal.

    Row blocks are drawn in order and mirrored in place, so memory stays at one
    n x n float32 array."""
    rng = np.random.default_rng(seed)
    W = out if out is not None else np.empty((n, n), np.float32)
    blk = 1024
    for r0 in range(0, n, blk):
        r1 = min(n, r0 + blk)
        W[r0:r1] = rng.random((r1 - r0, n), dtype=np.float32)
    # keep the upper triangle, mirror it into the lower one
    for r0 in range(0, n, blk):
        r1 = min(n, r0 + blk)
        W[r0:r1, :r0] = W[:r0, r0:r1].T
        sub = W[r0:r1, r0:r1]
        iu = np.triu_indices(r1 - r0, 1)
        sub.T[iu] = sub[iu]
    np.fill_diagonal(W, 0.0)
    return W


def integer_weights(n: int, levels: int = 3, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    A = rng.integers(0, levels, (n, n)).astype(np.float32)
    W = np.triu(A, 1)
    W = W + W.T
    np.fill_diagonal(W, 0.0)
    return W


def random_symmetric(n: int, seed: int = 0) -> np.ndarray:
    """Small continuous symmetric test matrix (float32 uniform, zero diagonal)."""
    return uniform_symmetric(n, seed=seed)


def ragged_sizes(num_graphs: int = 4096, nmin: int = 16, nmax: int = 1024,
                 seed: int = SEEDS["ragged"]) -> np.ndarray:
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(nmin), math.log(nmax + 1), num_graphs)
    return np.minimum(np.floor(np.exp(u)).astype(np.int64), nmax)


def ragged_points(num_graphs: int = 4096, nmin: int = 16, nmax: int = 1024,
                  seed: int = SEEDS["ragged"]):
    """List of point sets (float64) for the batched workload."""
    ns = ragged_sizes(num_graphs, nmin, nmax, seed)
    rng = np.random.default_rng(seed + 1000)
    pts = []
    for n in ns:
        d = int(rng.choice([2, 8]))
        pts.append(rng.random((int(n), d)))
    return pts


def pack(Ws):
    """Pack square matrices back to back: (flat float32, int64 offsets, int32 ns)."""
    ns = np.array([w.shape[0] for w in Ws], np.int32)
    sz = ns.astype(np.int64) ** 2
    offsets = np.zeros(len(Ws), np.int64)
    if len(Ws) > 1:
        offsets[1:] = np.cumsum(sz)[:-1]
    flat = np.empty(int(sz.sum()), np.float32)
    for w, o, s in zip(Ws, offsets, sz):
        flat[o:o + s] = np.ascontiguousarray(w, dtype=np.float32).ravel()
    return flat, offsets, ns


def ragged_batch(num_graphs: int = 4096, nmin: int = 16, nmax: int = 1024,
                 seed: int = SEEDS["ragged"]):
    """Packed Euclidean weights of the ragged batch -> (flat, offsets, ns)."""
    return pack([euclid_w(x) for x in ragged_points(num_graphs, nmin, nmax, seed)])


def diff_batch(num_graphs: int = 256, nmin: int = 64, nmax: int = 2048, d: int = 8,
               seed: int = SEEDS["diff"]):
    """List of (X float32 n x d, G float32 n x n) for the differentiable path."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, num_graphs)
    out = []
    for n in ns:
        X = rng.standard_normal((int(n), d)).astype(np.float32)
        G = rng.standard_normal((int(n), int(n))).astype(np.float32)
        out.append((X, G))
    return out


def config_small():
    """256 points uniform in [0,1]^2 (the small single-graph case)."""
    return euclid_w(single_points_2d())


def config_mixture(n: int = 8192):
    return euclid_w(gaussian_mixture_points(n))


def config_uniform(n: int = 32768, out: np.ndarray = None):
    return uniform_symmetric(n, out=out)
