"""GPU parity of the parallel spanning-tree path (Boruvka rounds + Prim order
rebuilt from the tree) against the CPU oracle, and against the sequential Prim
kernel: M, idx, the attachment order and the parents must all be identical."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2407_07058_amd as appd
import workloads
from gpu_helpers import assert_matches_digest, uniform32768_reference

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(W, tree, mode=appd.MINIMAX):
    Wd = torch.from_numpy(np.ascontiguousarray(W, np.float32)).to(DEV)
    out = appd.forward(Wd, mode=mode, return_tree=True, tree=tree)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def check(W, mode=appd.MINIMAX):
    M, idx, order, parent = run(W, "boruvka", mode)
    Mo, io = oracle.appd_widest(W) if mode == appd.WIDEST else oracle.appd(W)
    o, p, _, _ = oracle.mst_prim(W, widest=(mode == appd.WIDEST))
    assert np.array_equal(order, o), "attachment order differs"
    assert np.array_equal(parent, p), "parents differ"
    assert np.array_equal(M.view(np.uint32), Mo.view(np.uint32)) and np.array_equal(idx, io)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 17, 64, 100, 257, 1000, 1025, 3000, 4097, 6001])
def test_boruvka_random(n):
    say("case boruvka random n=%d" % n)
    check(workloads.random_symmetric(n, seed=n + 1))


@pytest.mark.parametrize("n", [2, 9, 300, 2048])
def test_boruvka_ties(n):
    say("case boruvka ties n=%d" % n)
    check(workloads.integer_weights(n, 3, seed=n))
    check(workloads.integer_weights(n, 2, seed=n + 7) - 1.0)


@pytest.mark.parametrize("n", [500, 3000])
def test_boruvka_points_and_mixture(n):
    say("case boruvka points/mixture n=%d" % n)
    check(workloads.euclid_w(workloads.single_points_2d(n, seed=n)))
    check(workloads.euclid_w(workloads.gaussian_mixture_points(n, seed=n)))


def test_boruvka_all_equal():
    say("case boruvka all-equal")
    n = 1500
    W = np.full((n, n), 0.5, np.float32)
    np.fill_diagonal(W, 0)
    check(W)


@pytest.mark.parametrize("n", [7, 600, 2500])
def test_boruvka_widest(n):
    say("case boruvka widest n=%d" % n)
    check(workloads.random_symmetric(n, seed=3 * n), appd.WIDEST)
    check(workloads.integer_weights(n, 4, seed=n), appd.WIDEST)


def test_boruvka_separated_clusters():
    """Far-apart tight clusters: every candidate list stays inside its cluster,
    so the refresh passes (and possibly the sequential fallback) are exercised."""
    say("case boruvka separated clusters")
    rng = np.random.default_rng(5)
    centres = rng.random((40, 3)) * 1000
    X = centres[rng.integers(0, 40, 2000)] + rng.standard_normal((2000, 3))
    check(workloads.euclid_w(X))
    # clusters within clusters within clusters
    X = np.concatenate([c + s * rng.standard_normal((50, 2))
                        for c in rng.random((8, 2)) * 1e6 for s in (1.0, 10.0, 100.0)])
    check(workloads.euclid_w(X))


def test_boruvka_equals_prim_mixture_full():
    say("case boruvka vs prim, mixture n=8192")
    W = workloads.config_mixture(8192)
    a = run(W, "boruvka")
    b = run(W, "prim")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    Mo, io = oracle.appd(W)
    assert np.array_equal(a[0].view(np.uint32), Mo.view(np.uint32)) and np.array_equal(a[1], io)


@pytest.mark.timeout(600)
def test_uniform_full_boruvka_and_prim():
    """n = 32768 uniform weights, forced Borůvka tree and forced Prim tree: the
    attachment order and parents equal the oracle's Prim, and every row slab of
    M and idx has the SHA-256 of the oracle's full output."""
    say("case uniform n=32768: generate")
    W, ref = uniform32768_reference()
    Wd = torch.from_numpy(W).to(DEV)
    o, p, _, _ = oracle.mst_prim(W)
    for tree in ("boruvka", "prim"):
        say("case uniform n=32768: forward tree=%s" % tree)
        Ma, Ia, oa, pa = appd.forward(Wd, return_tree=True, tree=tree)
        torch.cuda.synchronize()
        assert np.array_equal(oa.cpu().numpy(), o) and np.array_equal(pa.cpu().numpy(), p)
        say("case uniform n=32768: slab digests tree=%s" % tree)
        assert_matches_digest(Ma, Ia, ref, tree)
        del Ma, Ia
        torch.cuda.empty_cache()


@pytest.mark.parametrize("k,mode", [(3, appd.MINIMAX), (12, appd.MINIMAX), (12, appd.WIDEST)])
def test_boruvka_component_table(k, mode):
    """A few far-apart clusters: the candidate lists stay inside the clusters, so
    after the first rounds at most 16 components remain and the refresh pass
    builds the table of smallest inter-component edges, from which the tree is
    finished exactly.  Bit-exact against the oracle; no fallback to Prim."""
    say("case boruvka component table k=%d mode=%d" % (k, mode))
    rng = np.random.default_rng(40 + k)
    centres = rng.random((k, 4)) * 100
    X = centres[rng.integers(0, k, 2400)] + 0.3 * rng.standard_normal((2400, 4))
    W = workloads.euclid_w(X)
    Wd = torch.from_numpy(W).to(DEV)
    ws = torch.empty(appd.workspace_bytes(2400), dtype=torch.uint8, device=DEV)
    M, idx = appd.forward(Wd, mode=mode, tree="boruvka", workspace=ws)
    torch.cuda.synchronize()
    st = appd.tree_stats(2400, ws, mode=mode, tree="boruvka")
    ref = oracle.appd_widest if mode == appd.WIDEST else oracle.appd
    Mo, io = ref(W)
    assert np.array_equal(M.cpu().numpy().view(np.uint32), Mo.view(np.uint32))
    assert np.array_equal(idx.cpu().numpy(), io)
    assert st["boruvka"] and not st["fallback"] and st["tables"] >= 1, st


@pytest.mark.parametrize("mode", [appd.MINIMAX, appd.WIDEST])
def test_boruvka_prim_fallback(mode):
    """Clustered points need a component-table pass; limited to one pass over W,
    the rounds cannot finish and the sequential Prim fallback runs instead.
    Bit-exact against the oracle either way.  (In widest mode the weights are
    reflected, c - W, so that the maximum spanning tree has the clusters.)"""
    say("case prim fallback mode=%d" % mode)
    rng = np.random.default_rng(77)
    centres = rng.random((6, 3)) * 100
    X = centres[rng.integers(0, 6, 1500)] + 0.2 * rng.standard_normal((1500, 3))
    W = workloads.euclid_w(X)
    if mode == appd.WIDEST:  # the maximum spanning tree of c - W is the clustered one
        W = np.float32(W.max() + 1.0) - W
        np.fill_diagonal(W, 0.0)
    Wd = torch.from_numpy(W).to(DEV)
    ws = torch.empty(appd.workspace_bytes(1500), dtype=torch.uint8, device=DEV)
    M, idx, order, parent = appd.forward(Wd, mode=mode, tree="boruvka_one_pass", workspace=ws,
                                         return_tree=True)
    torch.cuda.synchronize()
    st = appd.tree_stats(1500, ws, mode=mode, tree="boruvka_one_pass")
    assert st["boruvka"] and st["fallback"] and st["passes"] == 1, st
    ref = oracle.appd_widest if mode == appd.WIDEST else oracle.appd
    Mo, io = ref(W)
    assert np.array_equal(M.cpu().numpy().view(np.uint32), Mo.view(np.uint32))
    assert np.array_equal(idx.cpu().numpy(), io)
    oo, po, _, _ = oracle.mst_prim(W, widest=mode == appd.WIDEST)
    assert np.array_equal(order.cpu().numpy(), oo)
    assert np.array_equal(parent.cpu().numpy(), po)


@pytest.mark.parametrize("n,mode", [(2401, appd.MINIMAX), (1999, appd.WIDEST)])
def test_boruvka_component_table_odd_n(n, mode):
    """The component-table pass on a size that is not a multiple of 4 (scalar
    loads) and odd (the middle row has no partner row): bit-exact against the
    oracle, and the table pass ran.  In widest mode the weights are reflected,
    c - W, so that the maximum spanning tree has the clusters."""
    say("case boruvka component table n=%d mode=%d" % (n, mode))
    rng = np.random.default_rng(n)
    centres = rng.random((5, 4)) * 100
    X = centres[rng.integers(0, 5, n)] + 0.3 * rng.standard_normal((n, 4))
    W = workloads.euclid_w(X)
    if mode == appd.WIDEST:
        W = np.float32(W.max() + 1.0) - W
        np.fill_diagonal(W, 0.0)
    Wd = torch.from_numpy(W).to(DEV)
    ws = torch.empty(appd.workspace_bytes(n), dtype=torch.uint8, device=DEV)
    M, idx = appd.forward(Wd, mode=mode, tree="boruvka", workspace=ws)
    torch.cuda.synchronize()
    st = appd.tree_stats(n, ws, mode=mode, tree="boruvka")
    ref = oracle.appd_widest if mode == appd.WIDEST else oracle.appd
    Mo, io = ref(W)
    assert np.array_equal(M.cpu().numpy().view(np.uint32), Mo.view(np.uint32))
    assert np.array_equal(idx.cpu().numpy(), io)
    assert st["boruvka"] and not st["fallback"] and st["tables"] >= 1, st
