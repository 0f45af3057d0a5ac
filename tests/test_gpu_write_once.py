"""Write-once property of the fill (Algorithm 4, Section 3: calculation and
copy assigns every entry of M once): with the library's store counting on,
every entry of M and of idx is stored exactly once, by the single-graph fill
(full and short column blocks, rows aligned and misaligned) and by every
batched fill (the Prim classes' fills, the position-space fill of the Boruvka
classes, the persistent launch).  The outputs of the counted forward equal the
oracle's bit for bit."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2407_07058_amd as appd
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ONCE = 0x00010001


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def graph(n, seed):
    if seed % 2:
        return workloads.random_symmetric(n, seed=seed)
    return workloads.integer_weights(n, 3, seed=seed)


# 1027: rows misaligned, short last block; 2052 and 4100: 16-byte rows with a
# short last block; 8192: full blocks only; 300 and 511: Prim's tree
@pytest.mark.parametrize("n,tree", [(1, "auto"), (2, "auto"), (5, "auto"), (64, "auto"),
                                    (300, "prim"), (511, "auto"), (1027, "auto"),
                                    (2052, "boruvka"), (2052, "prim"), (4100, "auto"),
                                    (8192, "auto")])
def test_single_fill_writes_each_entry_once(n, tree):
    say("case write-once single n=%d tree=%s" % (n, tree))
    W = graph(n, n)
    M, idx, counts = appd.write_counts(torch.from_numpy(W).to(DEV), tree=tree)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    bad = np.argwhere(c != ONCE)
    assert bad.size == 0, "entries not stored once: %s counts %s" % (
        bad[:4].tolist(), [hex(int(c[tuple(b)])) for b in bad[:4]])
    Mo, io = oracle.appd(W)
    assert np.array_equal(M.cpu().numpy().view(np.uint32), Mo.view(np.uint32))
    assert np.array_equal(idx.cpu().numpy(), io)


def test_single_fill_widest_writes_each_entry_once():
    n = 2052
    say("case write-once single widest n=%d" % n)
    W = graph(n, 3)
    M, idx, counts = appd.write_counts(torch.from_numpy(W).to(DEV), mode=appd.WIDEST)
    torch.cuda.synchronize()
    assert (counts.cpu().numpy() == ONCE).all()
    Mo, io = oracle.appd_widest(W)
    assert np.array_equal(M.cpu().numpy().view(np.uint32), Mo.view(np.uint32))
    assert np.array_equal(idx.cpu().numpy(), io)


SIZES = [1, 2, 3, 16, 63, 64, 65, 200, 256, 257, 500, 513, 1024, 1025, 1500, 2047, 2048]


def batch(sizes, seed):
    Ws = [graph(n, seed + k) for k, n in enumerate(sizes)]
    flat, offsets, ns = workloads.pack(Ws)
    return Ws, flat, offsets, ns


def check_batch_counts(b, Ws, flat, offsets, ns, what):
    M, idx, counts = b.write_counts(torch.from_numpy(flat).to(DEV))
    appd.sync(DEV)
    c = counts.cpu().numpy()
    bad = np.flatnonzero(c != ONCE)
    assert bad.size == 0, "%s: %d entries not stored once, first at %s" % (
        what, bad.size, bad[:4].tolist())
    Mh, Ih = M.cpu().numpy(), idx.cpu().numpy()
    for g, W in enumerate(Ws):
        o, n = int(offsets[g]), int(ns[g])
        Mo, io = oracle.appd(W)
        assert np.array_equal(Mh[o:o + n * n].view(np.uint32), Mo.ravel().view(np.uint32)), (what, g)
        assert np.array_equal(Ih[o:o + n * n], io.ravel()), (what, g)


@pytest.mark.parametrize("trees", ["boruvka", "prim"])
def test_batched_fills_write_each_entry_once(trees):
    """Every class's fill, with Borůvka trees (position-space fill) or Prim
    workgroups (the 64-bit fill up to n = 256, the coded fill above)."""
    say("case write-once batched trees=%s" % trees)
    Ws, flat, offsets, ns = batch(SIZES, 40)
    b = appd.Batch(ns, DEV)
    b.set_schedule(trees=[trees] * appd.BATCH_CLASSES, rows=7, streams=3, split_count=0)
    check_batch_counts(b, Ws, flat, offsets, ns, trees)


def test_persistent_fill_writes_each_entry_once():
    say("case write-once batched persistent")
    Ws, flat, offsets, ns = batch([n for n in SIZES if n <= 1024], 70)
    b = appd.Batch(ns, DEV)
    b.set_schedule(rows=5, persistent=True)
    check_batch_counts(b, Ws, flat, offsets, ns, "persistent")


def test_forward_after_counting_is_uncounted():
    """The counting switch is off again after the call: a plain forward that
    follows runs as usual (and equals the counted one)."""
    say("case write-once switch off")
    W = graph(700, 5)
    Wd = torch.from_numpy(W).to(DEV)
    M1, I1, _ = appd.write_counts(Wd)
    M2, I2 = appd.forward(Wd)
    torch.cuda.synchronize()
    assert torch.equal(M1, M2) and torch.equal(I1, I2)
