"""GPU single-linkage dendrogram (appd_linkage) against the oracle's merge table.

The GPU reads the dendrogram off Prim's attachment order (a Cartesian tree of
the attachment keys); the oracle adds the tree edges best first with a
union-find.  Ids, weights and sizes are exact, so the comparison is bit for bit."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2407_07058_amd as appd
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(W, mode=appd.MINIMAX, tree="auto"):
    Z = appd.linkage(torch.from_numpy(W).to(DEV), mode=mode, tree=tree)
    torch.cuda.synchronize()
    Zo = oracle.linkage(W, widest=(mode == appd.WIDEST))
    assert np.array_equal(Z.cpu().numpy(), Zo)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 100, 511, 512, 513, 2000])
@pytest.mark.parametrize("tree", ["prim", "boruvka"])
def test_linkage_random(n, tree):
    say("case linkage random n=%d tree=%s" % (n, tree))
    check(workloads.random_symmetric(n, seed=n + 3), tree=tree)


@pytest.mark.parametrize("n", [64, 700])
def test_linkage_ties_and_widest(n):
    say("case linkage ties/widest n=%d" % n)
    W = workloads.integer_weights(n, 3, seed=n)
    check(W)
    check(W, mode=appd.WIDEST)
    check(W, tree="boruvka")


def test_linkage_all_equal():
    say("case linkage all-equal")
    W = np.full((40, 40), 2.0, np.float32)
    np.fill_diagonal(W, 0)
    check(W)
    check(W, tree="boruvka")


def test_linkage_mixture_full_size():
    say("case linkage n=8192 mixture")
    check(workloads.config_mixture(8192))
