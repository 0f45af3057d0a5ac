"""GPU parity of the single-graph forward against the CPU oracle (bit-exact).

M and idx are exact selections of input weights, so the HIP path must equal the
oracle element by element on the same seeded inputs."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2407_07058_amd as appd
import workloads
from gpu_helpers import assert_matches_digest, uniform32768_reference, whole_matrix_properties

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_forward(W, mode=appd.MINIMAX, tree=False):
    Wd = torch.from_numpy(np.ascontiguousarray(W, np.float32)).to(DEV)
    out = appd.forward(Wd, mode=mode, return_tree=tree)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def assert_same(W, mode=appd.MINIMAX):
    M, idx = gpu_forward(W, mode)
    Mo, io = oracle.appd_widest(W) if mode == appd.WIDEST else oracle.appd(W)
    bad = np.argwhere((M.view(np.uint32) != Mo.view(np.uint32)) | (idx != io))
    assert len(bad) == 0, "first mismatches %s gpu %s/%s oracle %s/%s" % (
        bad[:3].tolist(), M[tuple(bad[0])], idx[tuple(bad[0])], Mo[tuple(bad[0])],
        io[tuple(bad[0])])


SIZES = [1, 2, 3, 5, 63, 64, 65, 127, 256, 257, 1000, 1023, 1024, 1025, 1500, 2049, 3001]


@pytest.mark.parametrize("n", SIZES)
def test_random_continuous(n):
    say("case random_continuous n=%d" % n)
    assert_same(workloads.random_symmetric(n, seed=n))


@pytest.mark.parametrize("n", [2, 7, 64, 300, 1024, 1100, 2500])
def test_tie_heavy(n):
    say("case tie_heavy n=%d" % n)
    assert_same(workloads.integer_weights(n, 3, seed=n))
    assert_same(workloads.integer_weights(n, 2, seed=n + 1) - 1.0)  # negatives, -0/+0 mixes


def test_small_points_config():
    say("case points n=256 (2-D uniform)")
    assert_same(workloads.config_small())


@pytest.mark.parametrize("n", [5, 200, 1025, 2100])
def test_widest(n):
    say("case widest n=%d" % n)
    assert_same(workloads.random_symmetric(n, seed=7 * n), appd.WIDEST)
    assert_same(workloads.integer_weights(n, 4, seed=n), appd.WIDEST)


def test_all_equal_closed_form():
    say("case all-equal n=777")
    n = 777
    W = np.full((n, n), 1.25, np.float32)
    np.fill_diagonal(W, 0)
    M, idx = gpu_forward(W)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    off = i != j
    assert (M[off] == 1.25).all() and (idx[off] == np.maximum(i, j)[off]).all()
    assert (idx[~off] == -1).all() and (M[~off] == 0).all()


def test_infinite_and_signed_zero():
    say("case inf / signed zero n=300")
    W = workloads.integer_weights(300, 3, seed=3)
    W[W == 2] = np.inf
    W[W == 0] = -0.0
    np.fill_diagonal(W, 0)
    assert_same(W)
    assert_same(W, appd.WIDEST)


def test_tree_outputs_match_prim():
    say("case tree outputs n=1500")
    W = workloads.euclid_w(workloads.single_points_2d(1500, seed=4))
    M, idx, order, parent = gpu_forward(W, tree=True)
    o, par, _, _ = oracle.mst_prim(W)
    assert np.array_equal(order, o) and np.array_equal(parent, par)


def test_mixture_full_size():
    say("case gaussian mixture n=8192 (full)")
    assert_same(workloads.config_mixture(8192))


def test_repeat_is_deterministic():
    say("case determinism n=4000")
    W = workloads.integer_weights(4000, 3, seed=11)
    a = gpu_forward(W)
    b = gpu_forward(W)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.timeout(600)
def test_uniform_full_size():
    """n = 32768, symmetric i.i.d. uniform weights: every row slab of M and idx
    has the SHA-256 of the oracle's full output, and the properties of the whole
    output hold on the GPU."""
    say("case uniform n=32768: generate")
    W, ref = uniform32768_reference()
    n = W.shape[0]
    Wd = torch.from_numpy(W).to(DEV)
    say("case uniform n=32768: forward")
    M, idx, order, parent = appd.forward(Wd, return_tree=True)
    torch.cuda.synchronize()
    say("case uniform n=32768: slab digests against the oracle's")
    assert_matches_digest(M, idx, ref, "auto tree")
    say("case uniform n=32768: whole-matrix properties")
    whole_matrix_properties(Wd, M, idx, parent)
    del M, idx, Wd
    torch.cuda.empty_cache()
