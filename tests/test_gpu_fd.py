"""Float64 central finite differences on the differentiable batch (256 graphs,
n uniform in {64..2048}, X ~ N(0, I_8), L = sum_{i != j} G_ij M_ij).

The gradient is not in the paper: it is the gradient of the selection the
forward makes (each pair's G goes to its bottleneck edge, then through the
Euclidean edge length to the two endpoints).  It is defined where that
selection is locally constant, so each sample is taken in float64 throughout
(X -> W -> Algorithm 4 -> L with compensated summation) and kept only when

  - the float64 bottleneck indices at X equal the float32 ones the GPU used
    (otherwise the whole graph is excluded: float32 rounding of W changed the
    tree), and
  - the float64 indices at X + h e and X - h e equal those at X.

Exclusions are counted and printed.  The kept samples must satisfy
|FD - g.e| <= 1e-4 * max(|g.e|, floor * |g|_2) for the float64 analytic
gradient g and for the GPU's float32 gradient (h = 1e-6; the floor keeps a
direction nearly orthogonal to g from asking for more than relative accuracy
of the whole gradient).  Four random unit directions per graph on all 256
graphs, and every coordinate of three graphs with n <= 128.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import paper_2407_07058_amd as appd
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
H = 1e-6
RTOL = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def loss_at(X64, G64, idx_ref):
    M, idx = oracle.appd_f64(oracle.pairwise_euclidean_f64(X64))
    return oracle.loss_f64(G64, M), np.array_equal(idx, idx_ref)


def fd_samples(X32, G32, idx_gpu, dX_gpu, dirs):
    """Returns (graph kept, [(fd, g.e, gpu.e, |g|) or None per direction])."""
    X64 = X32.astype(np.float64)
    G64 = G32.astype(np.float64)
    _, idx64 = oracle.appd_f64(oracle.pairwise_euclidean_f64(X64))
    if not np.array_equal(idx64, idx_gpu):
        return False, []
    g = oracle.grad_points(X64, G64, idx64)
    gn = float(np.linalg.norm(g))
    out = []
    for e in dirs:
        lp, okp = loss_at(X64 + H * e, G64, idx64)
        lm, okm = loss_at(X64 - H * e, G64, idx64)
        if not (okp and okm):
            out.append(None)
            continue
        out.append(((lp - lm) / (2 * H), float((g * e).sum()), float((dX_gpu * e).sum()), gn))
    return True, out


def worst_ratio(samples, which, floor):
    w = 0.0
    for s in samples:
        fd, an, gp, gn = s
        ref = an if which == "f64" else gp
        w = max(w, abs(fd - ref) / (RTOL * max(abs(an), floor * gn)))
    return w


@pytest.fixture(scope="module")
def batch_gradients():
    say("case FD: differentiable batch 256 graphs, generate")
    items = workloads.diff_batch()
    ns = [x.shape[0] for x, _ in items]
    b = appd.Batch(ns, DEV)
    X = torch.from_numpy(np.concatenate([x for x, _ in items])).to(DEV).requires_grad_(True)
    G = torch.from_numpy(np.concatenate([g.ravel() for _, g in items])).to(DEV)
    say("case FD: GPU forward + backward")
    M, idx = appd.appd_points_batched(X, b, 8)
    (M * G).sum().backward()
    torch.cuda.synchronize()
    idx_h = idx.cpu().numpy()
    dX = X.grad.cpu().numpy().astype(np.float64)
    per = []
    for g, (x, _) in enumerate(items):
        n = x.shape[0]
        o, no = int(b.offsets[g]), int(b.noff[g])
        per.append((idx_h[o:o + n * n].reshape(n, n), dX[no:no + n]))
    return items, per


@pytest.mark.timeout(900)
def test_fd_directional_all_graphs(batch_gradients):
    items, per = batch_gradients
    say("case FD: 4 directions x %d graphs (float64 oracle)" % len(items))

    def one(g):
        x, G = items[g]
        rng = np.random.default_rng(10_000 + g)
        dirs = []
        for _ in range(4):
            e = rng.standard_normal(x.shape)
            dirs.append(e / np.linalg.norm(e))
        return fd_samples(x, G, per[g][0], per[g][1], dirs)

    with ThreadPoolExecutor(8) as ex:
        res = list(ex.map(one, range(len(items))))
    graphs_out = sum(not kept for kept, _ in res)
    samples = [s for kept, ss in res if kept for s in ss]
    dirs_out = sum(s is None for s in samples)
    kept = [s for s in samples if s is not None]
    w64 = worst_ratio(kept, "f64", 1e-3)
    wgpu = worst_ratio(kept, "gpu", 1e-2)
    say("FD directional: %d of %d graphs excluded (float64 tree differs from the float32 one), "
        "%d of %d directions excluded (tree changes within +-h), %d samples kept; "
        "worst |FD - g.e| / tol: float64 gradient %.3g, GPU gradient %.3g"
        % (graphs_out, len(items), dirs_out, len(samples), len(kept), w64, wgpu))
    assert len(kept) >= 0.8 * 4 * len(items)
    assert w64 <= 1.0 and wgpu <= 1.0


@pytest.mark.timeout(600)
def test_fd_per_coordinate_small_graphs(batch_gradients):
    items, per = batch_gradients
    small = [g for g, (x, _) in enumerate(items) if x.shape[0] <= 128][:3]
    assert len(small) == 3
    say("case FD: every coordinate of graphs %s (n = %s)"
        % (small, [items[g][0].shape[0] for g in small]))

    def one(g):
        x, G = items[g]
        n, d = x.shape
        dirs = []
        for i in range(n):
            for t in range(d):
                e = np.zeros((n, d))
                e[i, t] = 1.0
                dirs.append(e)
        return fd_samples(x, G, per[g][0], per[g][1], dirs)

    with ThreadPoolExecutor(3) as ex:
        res = list(ex.map(one, small))
    kept_graphs = [ss for k, ss in res if k]
    samples = [s for ss in kept_graphs for s in ss]
    kept = [s for s in samples if s is not None]
    w64 = worst_ratio(kept, "f64", 1e-3)
    wgpu = worst_ratio(kept, "gpu", 1e-2)
    say("FD per coordinate: %d of 3 graphs kept, %d of %d coordinates kept; worst ratio "
        "float64 %.3g, GPU %.3g" % (len(kept_graphs), len(kept), len(samples), w64, wgpu))
    assert kept_graphs and len(kept) >= 0.9 * len(samples)
    assert w64 <= 1.0 and wgpu <= 1.0
