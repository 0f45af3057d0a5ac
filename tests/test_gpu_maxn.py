"""GPU parity at the largest supported size, n = 46340 (the largest n whose flat
edge indices fit in int32).

Above n = 32768 the component and parent arrays of the Boruvka rounds no
longer fit in LDS (the rounds run on global arrays) and Prim's algorithm keeps
46 vertices per thread.  Three trees are exercised on this size: the automatic
choice (Boruvka), Prim's algorithm forced, and the Boruvka tree limited to one
pass over W on clustered points, which must fall back to Prim.  Sampled rows are
compared with the oracle's Algorithm 4 restricted to those rows, the tree with
the oracle's Prim, and the properties of the whole output are checked on the
GPU.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2407_07058_amd as appd
import workloads
from gpu_helpers import whole_matrix_properties

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N = 46340


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sample_rows(n):
    return np.unique(np.concatenate([np.arange(0, n, 1451), [1, n // 2, n - 2, n - 1]]))


def forward(Wd, tree):
    n = Wd.shape[0]
    ws = torch.empty(appd.workspace_bytes(n), dtype=torch.uint8, device=DEV)
    M, idx, order, parent = appd.forward(Wd, tree=tree, workspace=ws, return_tree=True)
    torch.cuda.synchronize()
    return M, idx, order, parent, appd.tree_stats(n, ws, tree=tree)


def check_rows_and_tree(W, M, idx, order, parent, rows, tree_ref):
    Mo, io = oracle.appd_rows(W, rows)
    assert np.array_equal(M[rows].cpu().numpy().view(np.uint32), Mo.view(np.uint32))
    assert np.array_equal(idx[rows].cpu().numpy(), io)
    o, p = tree_ref
    assert np.array_equal(order.cpu().numpy(), o) and np.array_equal(parent.cpu().numpy(), p)


@pytest.mark.timeout(900)
def test_uniform_max_n_boruvka_and_prim():
    say("case n=%d uniform: generate" % N)
    W = workloads.uniform_symmetric(N, seed=N)
    Wd = torch.from_numpy(W).to(DEV)
    say("case n=%d uniform: oracle Prim tree" % N)
    o, p, _, _ = oracle.mst_prim(W)
    rows = sample_rows(N)
    say("case n=%d uniform: forward tree=auto" % N)
    M, idx, order, parent, st = forward(Wd, "auto")
    assert st["boruvka"] and not st["fallback"], st
    say("case n=%d uniform: %d oracle rows" % (N, len(rows)))
    check_rows_and_tree(W, M, idx, order, parent, rows, (o, p))
    say("case n=%d uniform: whole-matrix properties" % N)
    whole_matrix_properties(Wd, M, idx, parent)
    say("case n=%d uniform: forward tree=prim" % N)
    M2, idx2, order2, parent2, st2 = forward(Wd, "prim")
    assert not st2["boruvka"], st2
    assert torch.equal(M2, M) and torch.equal(idx2, idx)
    assert torch.equal(order2, order) and torch.equal(parent2, parent)


@pytest.mark.timeout(900)
def test_clustered_max_n_prim_fallback():
    """Far-apart clusters keep every candidate list inside its cluster, so one
    pass cannot finish the tree and the sequential Prim fallback runs; the
    unrestricted Boruvka tree finishes it with the component table.  Both equal
    the oracle on sampled rows and its Prim tree."""
    say("case n=%d clustered: generate" % N)
    rng = np.random.default_rng(N + 1)
    centres = rng.random((7, 3)) * 100
    X = centres[rng.integers(0, 7, N)] + 0.3 * rng.standard_normal((N, 3))
    W = workloads.euclid_w(X, chunk=256)
    Wd = torch.from_numpy(W).to(DEV)
    say("case n=%d clustered: oracle Prim tree" % N)
    o, p, _, _ = oracle.mst_prim(W)
    rows = sample_rows(N)
    say("case n=%d clustered: forward tree=boruvka_one_pass" % N)
    M, idx, order, parent, st = forward(Wd, "boruvka_one_pass")
    assert st["boruvka"] and st["fallback"] and st["passes"] == 1, st
    say("case n=%d clustered: %d oracle rows" % (N, len(rows)))
    check_rows_and_tree(W, M, idx, order, parent, rows, (o, p))
    say("case n=%d clustered: forward tree=boruvka" % N)
    M2, idx2, order2, parent2, st2 = forward(Wd, "boruvka")
    say("case n=%d clustered: boruvka stats %s" % (N, st2))
    assert st2["boruvka"], st2
    assert torch.equal(M2, M) and torch.equal(idx2, idx)
    assert torch.equal(order2, order) and torch.equal(parent2, parent)
    say("case n=%d clustered: whole-matrix properties" % N)
    whole_matrix_properties(Wd, M2, idx2, parent2)
