"""GPU results against closed forms at n = 8192, on every spanning-tree path.

The expected values here come from the mathematics, not from the oracle's
procedure:
  - a path-shaped graph (small weights on the edges of a Hamiltonian path, large
    ones elsewhere): the tree is the path, so M(i,j) is the largest path weight
    between the two vertices' positions and idx names that edge (a range max;
    Eq. 1-2 with the only useful path).  Increasing weights along the path make
    every vertex's parent edge the largest so far; decreasing weights make the
    nearest larger ancestor of each vertex its parent, a chain as deep as the
    graph, which is the deepest case of the order rebuilt from the tree;
  - an ultrametric W (W(i,k) <= max(W(i,j), W(j,k))): every direct edge is
    already a minimax path, so M = W (Section 5's argument with a one-edge path).
    Its idx, which depends on the tie rule, is compared with the oracle.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2407_07058_amd as appd
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N = 8192


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def path_graph(n, kind, seed):
    """W with path edges (perm[k], perm[k+1]) of weight vals[rank[k]] in [0, 1),
    every other edge 2 + U(0,1); returns W and the position-space expectation
    (M and idx as functions of path positions, then permuted)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n) if kind != "increasing_identity" else np.arange(n)
    m = n - 1
    if kind.startswith("increasing"):
        rank = np.arange(m)
    elif kind == "decreasing":
        rank = np.arange(m)[::-1].copy()
    else:
        rank = rng.permutation(m)
    vals = (np.arange(m, dtype=np.float64) + 1.0) / (m + 1)  # distinct, exact in float32
    w = vals[rank].astype(np.float32)
    W = workloads.random_symmetric(n, seed=seed + 1) + np.float32(2.0)
    u, v = perm[:-1], perm[1:]
    W[u, v] = w
    W[v, u] = w
    np.fill_diagonal(W, 0.0)
    flat = (np.minimum(u, v) * n + np.maximum(u, v)).astype(np.int64)
    # position space: for a < b the bottleneck is the path edge of largest rank in [a, b)
    Mp = np.zeros((n, n), np.float32)
    Ip = np.full((n, n), -1, np.int32)
    inv_rank = np.argsort(rank)  # inv_rank[r] = the path edge of rank r
    for a in range(n - 1):
        run = np.maximum.accumulate(rank[a:])  # rank of the max edge over [a, b), b = a+1..n-1
        k = inv_rank[run]
        Mp[a, a + 1:] = w[k]
        Ip[a, a + 1:] = flat[k]
    iu = np.triu_indices(n, 1)
    Mp.T[iu] = Mp[iu]
    Ip.T[iu] = Ip[iu]
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    return W, Mp[np.ix_(pos, pos)], Ip[np.ix_(pos, pos)]


def forward(W, tree, mode=appd.MINIMAX):
    Wd = torch.from_numpy(np.ascontiguousarray(W)).to(DEV)
    ws = torch.empty(appd.workspace_bytes(W.shape[0]), dtype=torch.uint8, device=DEV)
    M, idx = appd.forward(Wd, mode=mode, tree=tree, workspace=ws)
    torch.cuda.synchronize()
    st = appd.tree_stats(W.shape[0], ws, mode=mode, tree=tree)
    return M.cpu().numpy(), idx.cpu().numpy(), st


def same_bits(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint32),
                          np.ascontiguousarray(b).view(np.uint32))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("kind", ["increasing_identity", "increasing", "decreasing", "random"])
def test_path_range_max(kind):
    say("case path graph n=%d kind=%s: build" % (N, kind))
    W, Me, Ie = path_graph(N, kind, seed=len(kind))
    for tree in ("auto", "boruvka", "prim"):
        say("case path graph kind=%s tree=%s" % (kind, tree))
        M, idx, st = forward(W, tree)
        assert st["boruvka"] == (tree != "prim"), st
        assert not st["fallback"], st
        assert same_bits(M, Me), "M differs from the range max (tree=%s)" % tree
        assert np.array_equal(idx, Ie), "idx differs from the range argmax (tree=%s)" % tree
    # widest mode on the negated matrix: M_widest(-W) = -M(W), same edges
    say("case path graph kind=%s widest of -W" % kind)
    M, idx, _ = forward(-W, "boruvka", appd.WIDEST)
    Mneg = -Me
    Mneg[np.arange(N), np.arange(N)] = 0.0
    assert same_bits(M, Mneg) and np.array_equal(idx, Ie)


def ultrametric_levels(n, seed):
    """Tie-heavy ultrametric: W(i,j) = 0.25 * (2 + highest differing bit of two
    random 10-bit labels), 0.25 for equal labels.  The highest set bit of a ^ c
    is at most the larger of those of a ^ b and b ^ c, hence ultrametric."""
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, 1024, n)
    x = lab[:, None] ^ lab[None, :]
    hb = np.where(x > 0, np.floor(np.log2(np.maximum(x, 1))).astype(np.int64), -1)
    W = (0.25 * (hb + 2)).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    return W


def ultrametric_cophenetic(n, seed):
    """Continuous ultrametric: the single-linkage cophenetic distances of random
    points (scipy), rounded to float32 (rounding is monotone, so it stays
    ultrametric)."""
    from scipy.cluster.hierarchy import cophenet, linkage
    from scipy.spatial.distance import pdist, squareform
    rng = np.random.default_rng(seed)
    X = rng.random((n, 3))
    C = cophenet(linkage(pdist(X), "single"))
    W = squareform(C.astype(np.float32))
    np.fill_diagonal(W, 0.0)
    return np.ascontiguousarray(W)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("kind", ["levels", "cophenetic"])
def test_ultrametric_is_fixed_point(kind):
    say("case ultrametric n=%d kind=%s: build" % (N, kind))
    W = ultrametric_levels(N, 3) if kind == "levels" else ultrametric_cophenetic(N, 4)
    rng = np.random.default_rng(0)
    a, b, c = rng.integers(0, N, (3, 200000))
    assert (W[a, c] <= np.maximum(W[a, b], W[b, c])).all()  # the input really is ultrametric
    say("case ultrametric kind=%s: oracle" % kind)
    _, io = oracle.appd(W)
    for tree in ("auto", "boruvka", "prim"):
        say("case ultrametric kind=%s tree=%s" % (kind, tree))
        M, idx, st = forward(W, tree)
        assert same_bits(M, W + np.float32(0.0)), "M != W (tree=%s)" % tree
        assert np.array_equal(idx, io), "idx differs from the oracle (tree=%s)" % tree
