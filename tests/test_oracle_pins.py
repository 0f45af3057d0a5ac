"""Pins for the CPU oracle: it is checked against things other than itself.

Every reference here is computed independently of ``oracle/appd_oracle.c``:
brute-force path enumeration (Eq. 1-2), a numpy minimax Floyd-Warshall over
packed 64-bit keys, Kruskal with ascending edges (Section 3, the ascending
formulation), scipy's single-linkage cophenetic distances (Section 7: APPD read
off a single-linkage dendrogram), closed forms, and invariants from the
correctness argument of Section 5.
"""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.cluster.hierarchy import cophenet, linkage
from scipy.spatial.distance import squareform

import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- references
def ord32(w: np.ndarray) -> np.ndarray:
    """Order-preserving float32 -> uint32 map, -0.0 taken as +0.0."""
    w = np.asarray(w, np.float32) + np.float32(0.0)  # -0.0 + 0.0 = +0.0
    b = w.view(np.uint32).astype(np.uint64)
    neg = (b >> np.uint64(31)) == 1
    return np.where(neg, (~b) & np.uint64(0xFFFFFFFF), b | np.uint64(0x80000000))


def key_matrix(W: np.ndarray, widest: bool = False) -> np.ndarray:
    """64-bit edge keys (ord32(w) << 32 | flat); the diagonal is 0."""
    n = W.shape[0]
    Wk = -W if widest else W
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    flat = (np.minimum(i, j) * n + np.maximum(i, j)).astype(np.uint64)
    K = (ord32(Wk) << np.uint64(32)) | flat
    K[np.arange(n), np.arange(n)] = 0
    return K


def decode(K: np.ndarray, W: np.ndarray):
    n = W.shape[0]
    idx = (K & np.uint64(0xFFFFFFFF)).astype(np.int64)
    M = W.ravel()[idx] + np.float32(0.0)
    M[np.arange(n), np.arange(n)] = 0.0
    idx[np.arange(n), np.arange(n)] = -1
    return M.astype(np.float32), idx.astype(np.int32)


def fw_keys(W: np.ndarray, widest: bool = False):
    """Minimax Floyd-Warshall on packed keys (numpy, vectorised over pairs)."""
    K = key_matrix(W, widest)
    n = W.shape[0]
    for k in range(n):
        K = np.minimum(K, np.maximum(K[:, k:k + 1], K[k:k + 1, :]))
    return decode(K, W)


def brute_force(W: np.ndarray, widest: bool = False):
    """Eq. 1-2 literally: enumerate every simple path, min over paths of max key."""
    n = W.shape[0]
    K = key_matrix(W, widest)
    best = np.zeros((n, n), np.uint64)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            others = [v for v in range(n) if v not in (i, j)]
            b = None
            for r in range(len(others) + 1):
                for mid in itertools.permutations(others, r):
                    path = (i,) + mid + (j,)
                    mx = max(int(K[path[t], path[t + 1]]) for t in range(len(path) - 1))
                    b = mx if b is None else min(b, mx)
            best[i, j] = b
    return decode(best, W)


def kruskal_ascending(W: np.ndarray):
    """Section 3, ascending formulation: add edges from small to large to an
    empty forest; the edge that first joins two components is the minimax
    edge of every pair across them."""
    n = W.shape[0]
    K = key_matrix(W)
    iu, ju = np.triu_indices(n, 1)
    keys = K[iu, ju]
    order = np.argsort(keys, kind="stable")
    comp = list(range(n))
    members = {v: [v] for v in range(n)}
    M = np.zeros((n, n), np.float32)
    idx = np.full((n, n), -1, np.int32)
    joined = 0
    for e in order:
        a, b = int(iu[e]), int(ju[e])
        ca, cb = comp[a], comp[b]
        if ca == cb:
            continue
        A, B = members[ca], members[cb]
        w = W[a, b] + np.float32(0.0)
        ix = np.ix_(A, B)
        M[ix] = w
        M[np.ix_(B, A)] = w
        idx[ix] = a * n + b
        idx[np.ix_(B, A)] = a * n + b
        if len(A) < len(B):
            ca, cb, A, B = cb, ca, B, A
        for v in B:
            comp[v] = ca
        A.extend(B)
        del members[cb]
        joined += 1
        if joined == n - 1:
            break
    return M, idx


def cophenetic(W: np.ndarray) -> np.ndarray:
    n = W.shape[0]
    Z = linkage(squareform(W.astype(np.float64), checks=False), "single")
    C = squareform(cophenet(Z))
    return C.reshape(n, n)


def check_invariants(W, M, idx, samples=20000, seed=0):
    n = W.shape[0]
    d = np.arange(n)
    assert (M == M.T).all() and (idx == idx.T).all()
    assert (M[d, d] == 0).all() and (idx[d, d] == -1).all()
    off = ~np.eye(n, dtype=bool)
    assert (M[off] <= W[off]).all()
    # selection: M is the weight of the edge idx names
    sel = W.ravel()[np.where(off, idx, 0)]
    assert np.array_equal((sel + np.float32(0.0))[off], M[off])
    u, v = idx[off] // n, idx[off] % n
    assert (u < v).all()
    # idx names exactly n-1 distinct edges (the tree), every one minimax for its own pair
    edges = np.unique(idx[off])
    assert len(edges) == n - 1 if n > 1 else True
    eu, ev = edges // n, edges % n
    assert (idx[eu, ev] == edges).all()
    assert (M[eu, ev] == W[eu, ev] + np.float32(0.0)).all()
    # Kruskal counts: edge e is named by |A_e| * |B_e| unordered pairs
    _, counts = np.unique(idx[np.triu_indices(n, 1)], return_counts=True)
    assert counts.sum() == n * (n - 1) // 2
    # distinct off-diagonal values <= n - 1
    assert len(np.unique(M[off])) <= max(n - 1, 0)
    # ultrametric inequality on sampled triples
    rng = np.random.default_rng(seed)
    a, b, c = rng.integers(0, n, (3, samples))
    keep = a != c  # the zero diagonal is not below negative weights
    a, b, c = a[keep], b[keep], c[keep]
    assert (M[a, c] <= np.maximum(M[a, b], M[b, c])).all()


# ---------------------------------------------------------------- tests
def test_golden_hand_example(orc):
    g = json.load(open(os.path.join(GOLD, "hand_5vertex.json")))
    W = np.array(g["W"], np.float32)
    M, idx = orc.appd(W)
    assert np.array_equal(M, np.array(g["M"], np.float32))
    assert np.array_equal(idx, np.array(g["idx"], np.int32))
    Mw, iw = orc.appd_widest(W)
    assert np.array_equal(Mw, np.array(g["M_widest"], np.float32))
    assert np.array_equal(iw, np.array(g["idx_widest"], np.int32))


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_tiny(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    W = workloads.integer_weights(n, 3, seed) if seed % 2 else workloads.random_symmetric(n, seed)
    M, idx = orc.appd(W)
    Mb, ib = brute_force(W)
    assert np.array_equal(M, Mb) and np.array_equal(idx, ib)
    Mw, iw = orc.appd_widest(W)
    Mbw, ibw = brute_force(W, widest=True)
    assert np.array_equal(iw, ibw)
    assert np.array_equal(Mw, Mbw)


@pytest.mark.parametrize("seed", range(30))
def test_floyd_warshall(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 65))
    kind = seed % 3
    if kind == 0:
        W = workloads.random_symmetric(n, seed)
    elif kind == 1:
        W = workloads.integer_weights(n, 3, seed)
    else:
        W = workloads.integer_weights(n, 2, seed) - 0.5  # negative weights and ties
        np.fill_diagonal(W, 0)
    M, idx = orc.appd(W)
    Mf, i_f = fw_keys(W)
    assert np.array_equal(M, Mf) and np.array_equal(idx, i_f)
    # the C Floyd-Warshall (definition, separate routine) agrees as well
    Mc, ic = orc.appd_fw(W)
    assert np.array_equal(Mc, Mf) and np.array_equal(ic, i_f)
    check_invariants(W, M, idx)


@pytest.mark.parametrize("n,kind", [(200, "mix"), (513, "uni"), (700, "tie"), (1500, "pts")])
def test_kruskal_ascending(orc, n, kind):
    if kind == "mix":
        W = workloads.euclid_w(workloads.gaussian_mixture_points(n, seed=7))
    elif kind == "uni":
        W = workloads.uniform_symmetric(n, seed=8)
    elif kind == "tie":
        W = workloads.integer_weights(n, 4, seed=9)
    else:
        W = workloads.euclid_w(workloads.single_points_2d(n, seed=10))
    M, idx = orc.appd(W)
    Mk, ik = kruskal_ascending(W)
    assert np.array_equal(M, Mk) and np.array_equal(idx, ik)
    check_invariants(W, M, idx)


@pytest.mark.parametrize("n,kind", [(256, "small"), (1024, "mix"), (2048, "uni")])
def test_single_linkage_cophenetic(orc, n, kind):
    if kind == "small":
        W = workloads.config_small()
    elif kind == "mix":
        W = workloads.euclid_w(workloads.gaussian_mixture_points(n, seed=11))
    else:
        W = workloads.uniform_symmetric(n, seed=12)
    M, idx = orc.appd(W)
    C = cophenetic(W)
    assert np.array_equal(M.astype(np.float64), C)
    check_invariants(W, M, idx)


def test_closed_form_all_equal(orc):
    # the tree is the star at vertex 0 and idx(i, j) = max(i, j): pins the tie rule
    for n in (1, 2, 3, 17, 64):
        W = np.full((n, n), 2.5, np.float32)
        np.fill_diagonal(W, 0)
        M, idx = orc.appd(W)
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        off = i != j
        assert (M[off] == 2.5).all()
        assert (idx[off] == np.maximum(i, j)[off]).all()


def test_closed_form_path(orc):
    # cheap edges (i, i+1), huge elsewhere: M(i, j) = max of the path edges between
    rng = np.random.default_rng(3)
    n = 40
    w = rng.random(n - 1).astype(np.float32)
    W = np.full((n, n), 100.0, np.float32)
    for k in range(n - 1):
        W[k, k + 1] = W[k + 1, k] = w[k]
    np.fill_diagonal(W, 0)
    M, idx = orc.appd(W)
    for i in range(n):
        for j in range(i + 1, n):
            k = i + int(np.argmax(w[i:j]))
            assert M[i, j] == w[k] and idx[i, j] == k * n + k + 1


def test_closed_form_ultrametric(orc):
    # an ultrametric is its own minimax distance
    rng = np.random.default_rng(4)
    pts = rng.random((60, 3))
    U = cophenetic(workloads.euclid_w(pts)).astype(np.float32)
    M, _ = orc.appd(U)
    assert np.array_equal(M, U)


def test_n1_n2(orc):
    M, idx = orc.appd(np.zeros((1, 1), np.float32))
    assert M.tolist() == [[0.0]] and idx.tolist() == [[-1]]
    W = np.array([[0, 3.5], [3.5, 0]], np.float32)
    M, idx = orc.appd(W)
    assert M.tolist() == [[0, 3.5], [3.5, 0]] and idx.tolist() == [[-1, 1], [1, -1]]


def test_signed_zero_and_inf(orc):
    W = np.array([[0, -0.0, np.inf], [-0.0, 0, 1], [np.inf, 1, 0]], np.float32)
    M, idx = orc.appd(W)
    assert np.signbit(M).sum() == 0  # -0.0 reported as +0.0
    assert M[0, 2] == 1 and idx[0, 2] == 1 * 3 + 2
    W2 = np.full((4, 4), np.inf, np.float32)
    np.fill_diagonal(W2, 0)
    M2, idx2 = orc.appd(W2)
    off = ~np.eye(4, dtype=bool)
    assert np.isinf(M2[off]).all()


def test_widest_is_minimax_of_negation(orc):
    for seed in range(6):
        n = 50 + 37 * seed
        W = workloads.integer_weights(n, 5, seed) if seed % 2 else workloads.random_symmetric(n, seed)
        Mw, iw = orc.appd_widest(W)
        Mn, inn = orc.appd(-W)
        assert np.array_equal(iw, inn)
        assert np.array_equal(Mw, (-Mn) + np.float32(0.0))
        if n <= 64:
            Mf, i_f = orc.appd_fw(W, widest=True)
            assert np.array_equal(Mw, Mf) and np.array_equal(iw, i_f)


def test_rows_variant(orc):
    W = workloads.euclid_w(workloads.gaussian_mixture_points(600, seed=5))
    M, idx = orc.appd(W)
    rows = np.array([599, 0, 17, 300, 42])
    Mr, ir = orc.appd_rows(W, rows)
    assert np.array_equal(Mr, M[rows]) and np.array_equal(ir, idx[rows])
    Mw, iw = orc.appd_widest(W)
    Mr, ir = orc.appd_rows(W, rows, widest=True)
    assert np.array_equal(Mr, Mw[rows]) and np.array_equal(ir, iw[rows])


def test_f64_matches_f32_on_float_values(orc):
    W = workloads.euclid_w(workloads.single_points_2d(300, seed=6))
    M, idx = orc.appd(W)
    M64, idx64 = orc.appd_f64(W.astype(np.float64))
    assert np.array_equal(idx, idx64) and np.array_equal(M.astype(np.float64), M64)


def test_mst_prim_total_weight(orc):
    from scipy.sparse.csgraph import minimum_spanning_tree
    W = workloads.euclid_w(workloads.single_points_2d(400, seed=7)).astype(np.float64)
    order, parent, aw, af = orc.mst_prim(W.astype(np.float32))
    assert sorted(order.tolist()) == list(range(400))
    total = sum(float(W[v, parent[v]]) for v in range(1, 400))
    ref = minimum_spanning_tree(W).sum()  # no zero off-diagonal weights here
    assert abs(total - ref) <= 1e-9 * ref
    assert (aw[1:] == W.astype(np.float32)[order[1:], parent[order[1:]]]).all()


def test_pairwise_euclidean(orc):
    X = np.array([[0, 0], [3, 4], [6, 8], [0, 0]], np.float32)
    W = orc.pairwise_euclidean_f32(X)
    assert W[0, 1] == 5 and W[0, 2] == 10 and W[1, 2] == 5 and W[0, 3] == 0
    rng = np.random.default_rng(1)
    X = rng.standard_normal((300, 8)).astype(np.float32)
    W = orc.pairwise_euclidean_f32(X)
    assert np.array_equal(W, W.T) and (np.diag(W) == 0).all()
    W64 = orc.pairwise_euclidean_f64(X.astype(np.float64))
    assert np.allclose(W, W64, rtol=4e-7, atol=0)


def _euclid_f32_numpy(X):
    """The float32 distance evaluated by numpy, one IEEE float32 rounding per
    operation: subtract, square, add in increasing coordinate order, then the
    correctly rounded square root.  numpy never contracts a*b+c into a fused
    multiply-add, so this is exactly the operation sequence the oracle states."""
    X = np.asarray(X, np.float32)
    n, d = X.shape
    acc = np.zeros((n, n), np.float32)
    for t in range(d):
        diff = X[:, None, t] - X[None, :, t]
        sq = diff * diff
        acc = acc + sq
    W = np.sqrt(acc)
    W[np.arange(n), np.arange(n)] = 0.0
    return W


@pytest.mark.parametrize("d,scale,seed", [(1, 1.0, 2), (2, 1.0, 3), (8, 1.0, 4), (16, 3.0, 5),
                                          (5, 1e-19, 6), (7, 1e17, 7)])
def test_pairwise_euclidean_f32_bit_exact(orc, d, scale, seed):
    """Bit-for-bit against numpy's float32 evaluation in the same order.  A fused
    multiply-add, a different summation order, a float64 accumulator or a
    non-correctly-rounded square root each change some of these bits."""
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((257, d)) * scale).astype(np.float32)
    W = orc.pairwise_euclidean_f32(X)
    assert np.array_equal(W.view(np.uint32), _euclid_f32_numpy(X).view(np.uint32))


def test_pairwise_euclidean_f32_detects_reordering():
    """The reference above is sensitive to what the bit-exact pin claims: on this
    input, summing in decreasing coordinate order, accumulating in float64 or
    fusing the multiply-add each changes at least one distance."""
    rng = np.random.default_rng(8)
    X = rng.standard_normal((257, 8)).astype(np.float32)
    ref = _euclid_f32_numpy(X)
    rev = _euclid_f32_numpy(X[:, ::-1])
    assert not np.array_equal(ref, rev)
    acc64 = np.zeros((257, 257))
    for t in range(8):
        df = (X[:, None, t] - X[None, :, t]).astype(np.float64)
        acc64 += df * df
    w64 = np.sqrt(acc64).astype(np.float32)
    np.fill_diagonal(w64, 0)
    assert not np.array_equal(ref, w64)
    # a fused multiply-add rounds diff*diff + acc once: emulate it exactly in float64
    # (products of floats are exact in double, and one rounding to float32 follows)
    accf = np.zeros((257, 257), np.float32)
    for t in range(8):
        df = (X[:, None, t] - X[None, :, t]).astype(np.float64)
        accf = (df * df + accf.astype(np.float64)).astype(np.float32)
    wf = np.sqrt(accf)
    np.fill_diagonal(wf, 0)
    assert not np.array_equal(ref, wf)


def test_pairwise_euclidean_f32_one_dimension(orc):
    """d = 1: the distance is |x_i - x_j| rounded once, because the correctly
    rounded square root of a correctly rounded square gives the number back
    (round to nearest, no overflow or underflow)."""
    rng = np.random.default_rng(9)
    x = rng.standard_normal((300, 1)).astype(np.float32)
    W = orc.pairwise_euclidean_f32(x)
    ref = np.abs(x[:, None, 0] - x[None, :, 0])
    assert np.array_equal(W.view(np.uint32), ref.view(np.uint32))


def _fd_generic(orc, X, G, h=1e-6, ndir=4, seed=0):
    """Directional central differences of the float64 loss, kept only where the
    float64 bottleneck structure does not change within +-h."""
    rng = np.random.default_rng(seed)
    W = orc.pairwise_euclidean_f64(X)
    M, idx = orc.appd_f64(W)
    g = orc.grad_points(X, G, idx)
    kept = 0
    for _ in range(ndir):
        e = rng.standard_normal(X.shape)
        e /= np.linalg.norm(e)
        Mp, ip = orc.appd_f64(orc.pairwise_euclidean_f64(X + h * e))
        Mm, im = orc.appd_f64(orc.pairwise_euclidean_f64(X - h * e))
        if not (np.array_equal(ip, idx) and np.array_equal(im, idx)):
            continue
        fd = (orc.loss_f64(G, Mp) - orc.loss_f64(G, Mm)) / (2 * h)
        an = float((g * e).sum())
        assert abs(fd - an) <= 1e-4 * max(abs(an), 1e-3 * np.abs(g).sum()), (fd, an)
        kept += 1
    return kept


def test_gradient_finite_differences(orc):
    rng = np.random.default_rng(5)
    kept = 0
    for n in (8, 40, 120):
        X = rng.standard_normal((n, 8))
        G = rng.standard_normal((n, n))
        kept += _fd_generic(orc, X, G, seed=n)
    assert kept >= 8


def test_gradient_per_coordinate(orc):
    rng = np.random.default_rng(6)
    n, d, h = 12, 3, 1e-6
    X = rng.standard_normal((n, d))
    G = rng.standard_normal((n, n))
    M, idx = orc.appd_f64(orc.pairwise_euclidean_f64(X))
    g = orc.grad_points(X, G, idx)
    for i in range(n):
        for t in range(d):
            Xp = X.copy(); Xp[i, t] += h
            Xm = X.copy(); Xm[i, t] -= h
            Mp, ip = orc.appd_f64(orc.pairwise_euclidean_f64(Xp))
            Mm, im = orc.appd_f64(orc.pairwise_euclidean_f64(Xm))
            assert np.array_equal(ip, idx) and np.array_equal(im, idx)
            fd = (orc.loss_f64(G, Mp) - orc.loss_f64(G, Mm)) / (2 * h)
            assert abs(fd - g[i, t]) <= 1e-4 * max(1.0, abs(g[i, t]))


def test_gradient_two_points_closed_form(orc):
    # n = 2: L = (G01 + G10) * |x0 - x1|, so dL/dx0 = (G01 + G10) (x0 - x1) / |x0 - x1|
    X = np.array([[0.0, 0.0], [3.0, 4.0]])
    G = np.array([[0.0, 2.0], [0.5, 0.0]])
    _, idx = orc.appd_f64(orc.pairwise_euclidean_f64(X))
    g = orc.grad_points(X, G, idx)
    assert np.allclose(g[0], 2.5 * np.array([-3, -4]) / 5) and np.allclose(g[1], -g[0])


# ---------------------------------------------------------------- dendrogram
@pytest.mark.parametrize("n,kind", [(2, "uni"), (3, "uni"), (50, "uni"), (500, "uni"), (300, "pts")])
def test_linkage_matches_scipy(orc, n, kind):
    """Tie-free weights: the oracle's merge table equals scipy's single linkage
    (ids, weights and sizes), the library routine behind reading distances off
    the dendrogram."""
    from scipy.cluster.hierarchy import linkage
    from scipy.spatial.distance import squareform
    if kind == "uni":
        W = workloads.random_symmetric(n, seed=20 + n)
    else:
        W = workloads.euclid_w(workloads.single_points_2d(n, seed=21))
    Z = orc.linkage(W)
    Zs = linkage(squareform(W.astype(np.float64), checks=False), method="single")
    assert np.array_equal(Z, Zs)


@pytest.mark.parametrize("levels", [2, 3, 5])
def test_linkage_cophenetic_is_appd_with_ties(orc, levels):
    """With heavy ties the merge order is a convention, but the dendrogram's
    cophenetic distances must be the APPD matrix (Eq. 1-2) whatever it is."""
    from scipy.cluster.hierarchy import cophenet
    from scipy.spatial.distance import squareform
    W = workloads.integer_weights(257, levels, seed=levels)
    Z = orc.linkage(W)
    M, _ = orc.appd(W)
    assert np.array_equal(squareform(cophenet(Z)), M.astype(np.float64))
    assert Z[-1, 3] == 257 and (np.diff(Z[:, 2]) >= 0).all()


def test_linkage_closed_form_all_equal(orc):
    """All weights equal: the tree is the star at 0 and edges are taken by flat
    index, so merge i joins vertex i+1 to the cluster built so far."""
    for n in (2, 3, 9):
        W = np.full((n, n), 1.5, np.float32)
        np.fill_diagonal(W, 0)
        Z = orc.linkage(W)
        exp = [[0, 1, 1.5, 2]] + [[i + 1, n + i - 1, 1.5, i + 2] for i in range(1, n - 1)]
        assert np.array_equal(Z, np.array(exp, np.float64))


def test_linkage_widest_is_minimax_of_negation(orc):
    W = workloads.random_symmetric(120, seed=5)
    Zw = orc.linkage(W, widest=True)
    Zn = orc.linkage(-W)
    assert np.array_equal(Zw[:, [0, 1, 3]], Zn[:, [0, 1, 3]])
    assert np.array_equal(Zw[:, 2], -Zn[:, 2])
