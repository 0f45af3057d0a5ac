"""Helpers shared by the GPU parity tests at large n: per-slab SHA-256 digests of
a device matrix, the n = 32768 uniform workload with the oracle's stored
digests of its full output, and properties of the whole output that hold at any
size (checked on the GPU, slab by slab)."""
import hashlib
import json
import os

import numpy as np
import torch

import workloads

DEV = "cuda:0"


def slab_digests(A, slab):
    """SHA-256 of the raw bytes of each row slab of a device matrix."""
    out = []
    for r0 in range(0, A.shape[0], slab):
        h = A[r0:r0 + slab].cpu().numpy()
        out.append(hashlib.sha256(memoryview(np.ascontiguousarray(h)).cast("B")).hexdigest())
    return out


def uniform32768_reference():
    """The n = 32768 uniform workload and the oracle's per-slab digests of its
    full output (tests/golden/make_uniform32768_digest.py writes them by calling
    only the oracle)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "uniform32768_digest.json")) as f:
        ref = json.load(f)
    W = workloads.config_uniform(ref["n"])
    w_digest = hashlib.sha256(memoryview(W).cast("B")).hexdigest()
    assert w_digest == ref["W_sha256"], "the seeded generator no longer gives the stored W"
    return W, ref


def assert_matches_digest(M, idx, ref, what):
    dm = slab_digests(M, ref["slab_rows"])
    di = slab_digests(idx, ref["slab_rows"])
    badm = [s for s, (a, b) in enumerate(zip(dm, ref["M_sha256"])) if a != b]
    badi = [s for s, (a, b) in enumerate(zip(di, ref["idx_sha256"])) if a != b]
    assert not badm and not badi, "%s: row slabs of %d differing from the oracle: M %s, idx %s" % (
        what, ref["slab_rows"], badm, badi)


def whole_matrix_properties(Wd, M, idx, parent, slab=4096):
    """Properties of the whole output that hold at any size: symmetry, the
    diagonal, M is the weight idx names, M <= W, M = W on tree edges, each tree
    edge named by exactly |A||B| pairs (the sizes of the two sides it joins in
    the ascending construction), and the ultrametric inequality on samples."""
    n = M.shape[0]
    for r0 in range(0, n, slab):
        r1 = min(n, r0 + slab)
        Mb, Ib = M[r0:r1], idx[r0:r1]
        assert torch.equal(Mb, M[:, r0:r1].t()) and torch.equal(Ib, idx[:, r0:r1].t())
        dg = torch.arange(r0, r1, device=DEV)
        assert (Ib[dg - r0, dg] == -1).all() and (Mb[dg - r0, dg] == 0).all()
        sel = Wd.view(-1)[Ib.clamp(min=0).long()] + 0.0
        sel[dg - r0, dg] = 0
        assert torch.equal(sel, Mb)
        assert (Mb <= Wd[r0:r1]).all()
        del sel
    p = parent.long()
    v = torch.arange(1, n, device=DEV)
    assert torch.equal(M[v, p[1:]], Wd[v, p[1:]] + 0.0)
    # Kruskal counts: ascending union of the tree edges gives |A||B| per edge
    pc = parent.cpu().numpy().astype(np.int64)
    vv = np.arange(1, n)
    a, b = np.minimum(vv, pc[1:]), np.maximum(vv, pc[1:])
    flat = a * n + b
    Wh = Wd[v, p[1:]].cpu().numpy()
    order = np.lexsort((flat, Wh))  # ascending weight, then flat index
    up = np.arange(n)
    size = np.ones(n, np.int64)

    def find(x):
        while up[x] != x:
            up[x] = up[up[x]]
            x = up[x]
        return x
    expect = np.empty(n - 1, np.int64)
    for e in order:
        ra, rb = find(a[e]), find(b[e])
        expect[e] = size[ra] * size[rb]
        if size[ra] < size[rb]:
            ra, rb = rb, ra
        up[rb] = ra
        size[ra] += size[rb]
    fs = torch.from_numpy(np.sort(flat)).to(DEV)
    counts = torch.zeros(n - 1, dtype=torch.int64, device=DEV)
    for r0 in range(0, n, slab):
        Ib = torch.triu(idx[r0:min(n, r0 + slab)].long() + 1, diagonal=r0 + 1) - 1
        Ib = Ib[Ib >= 0]
        e = torch.searchsorted(fs, Ib)
        assert torch.equal(fs[e.clamp(max=n - 2)], Ib), "idx names an edge outside the tree"
        counts += torch.bincount(e, minlength=n - 1)
    exp_sorted = expect[np.argsort(flat)]
    assert np.array_equal(counts.cpu().numpy(), exp_sorted)
    # ultrametric inequality on sampled triples
    g = torch.Generator(device=DEV)
    g.manual_seed(0)
    t = torch.randint(0, n, (3, 1 << 20), device=DEV, generator=g)
    t = t[:, t[0] != t[2]]
    assert (M[t[0], t[2]] <= torch.maximum(M[t[0], t[1]], M[t[1], t[2]])).all()
