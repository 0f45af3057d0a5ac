"""GPU parity of the batched forward, the point-to-graph kernel and the backward.

Forward outputs are exact selections, so they are compared bit for bit with the
CPU oracle.  The point-to-graph kernel follows the same operation order as the
oracle's float32 routine, so W is compared bit for bit too.  Gradients use float
atomics on the GPU, so they are compared with a tolerance against the oracle's
float64 reference gradient taken through the same bottleneck edges."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pool():
    return ThreadPoolExecutor(8)


def unpack(flat, ns, offsets):
    return [flat[o:o + n * n].reshape(n, n) for n, o in zip(ns, offsets)]


def check_batch(Ws, mode=appd.MINIMAX):
    flat, offsets, ns = workloads.pack(Ws)
    b = appd.Batch(ns, DEV)
    assert (b.offsets == offsets).all()
    M, idx, parent = b.forward(torch.from_numpy(flat).to(DEV), mode=mode, return_parent=True)
    torch.cuda.synchronize()
    Ms = unpack(M.cpu().numpy(), ns, offsets)
    Is = unpack(idx.cpu().numpy(), ns, offsets)
    ref = oracle.appd_widest if mode == appd.WIDEST else oracle.appd

    def one(g):
        Mo, io = ref(Ws[g])
        return np.array_equal(Ms[g].view(np.uint32), Mo.view(np.uint32)) and np.array_equal(Is[g], io)

    with pool() as ex:
        okays = list(ex.map(one, range(len(Ws))))
    bad = [g for g, o in enumerate(okays) if not o]
    assert not bad, "graphs differing from the oracle: %s (n=%s)" % (bad[:5], [int(ns[g]) for g in bad[:5]])
    return b, M, idx, parent


SIZES = [1, 2, 3, 16, 63, 64, 65, 200, 256, 257, 500, 1024, 1025, 1500, 2047, 2048]


def mixed_graphs(seed):
    rng = np.random.default_rng(seed)
    Ws = []
    for k, n in enumerate(SIZES * 2):
        if k % 3 == 0:
            Ws.append(workloads.integer_weights(n, 3, seed=seed + k))
        elif k % 3 == 1:
            Ws.append(workloads.random_symmetric(n, seed=seed + k))
        else:
            Ws.append(workloads.euclid_w(rng.random((n, int(rng.choice([2, 8]))))))
    order = rng.permutation(len(Ws))
    return [Ws[i] for i in order]


def test_batched_mixed_sizes():
    say("case batched mixed sizes (32 graphs, n 1..2048)")
    check_batch(mixed_graphs(1))


def test_batched_widest():
    say("case batched widest")
    check_batch(mixed_graphs(2)[:20], appd.WIDEST)


def special_values_graphs(seed):
    """Graphs whose rows stress the candidate selection of the batched tree
    pass: signed zeros, negative weights, +inf and -inf entries (symmetric, a
    diagonal of NaN, which the method never reads), long runs of one value,
    and sizes on both sides of the 17-lane threshold rule."""
    rng = np.random.default_rng(seed)
    Ws = []
    for k, n in enumerate([2, 5, 16, 17, 18, 40, 65, 130, 300, 700, 1024]):
        W = rng.uniform(-1.0, 1.0, (n, n)).astype(np.float32)
        r = rng.random((n, n))
        W[r < 0.10] = np.inf
        W[(r >= 0.10) & (r < 0.15)] = -np.inf
        W[(r >= 0.15) & (r < 0.25)] = 0.0
        W[(r >= 0.25) & (r < 0.35)] = -0.0
        W[(r >= 0.35) & (r < 0.45)] = 0.5
        W = np.triu(W, 1)
        W = W + W.T
        np.fill_diagonal(W, np.nan)
        Ws.append(W)
    return Ws


def test_batched_special_values():
    say("case batched special values (signed zeros, infinities, runs of ties)")
    check_batch(special_values_graphs(11))
    check_batch(special_values_graphs(12), appd.WIDEST)


def test_batched_parent_matches_single():
    say("case batched parent vs single-graph tree")
    Ws = mixed_graphs(3)[:12]
    b, M, idx, parent = check_batch(Ws)
    par = parent.cpu().numpy()
    for g, W in enumerate(Ws):
        n = W.shape[0]
        _, p, _, _ = oracle.mst_prim(W)
        assert np.array_equal(par[b.noff[g]:b.noff[g] + n], p)


@pytest.mark.timeout(600)
def test_batched_ragged_full_config():
    """4096 graphs, n log-uniform in [16, 1024], d in {2, 8}: every graph bit-exact."""
    say("case ragged batch 4096 graphs: generate")
    pts = workloads.ragged_points()
    with pool() as ex:
        Ws = list(ex.map(workloads.euclid_w, pts))
    say("case ragged batch 4096 graphs: forward + oracle")
    check_batch(Ws)


def test_batched_graph_capture_replays():
    """The prepared batched forward launches kernels only, so it can be captured
    in a HIP graph; every replay must equal the eager result."""
    say("case batched HIP graph capture")
    Ws = mixed_graphs(4)
    flat, offsets, ns = workloads.pack(Ws)
    b = appd.Batch(ns, DEV)
    Wd = torch.from_numpy(flat).to(DEV)
    M0, I0 = b.forward(Wd)
    torch.cuda.synchronize()
    M = torch.empty_like(M0)
    I = torch.empty_like(I0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.forward(Wd, out=(M, I))  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.forward(Wd, out=(M, I))
    for rep in range(4):
        M.fill_(-7.0)
        I.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(M, M0) and torch.equal(I, I0), "replay %d differs" % rep
        _ = (M0 * 2).sum().item()  # eager work between replays


def test_batched_schedules_identical():
    """Every Prim workgroup size, rows per fill item and class concurrency gives
    the same bits as the default schedule.  (Rows per item change the fill work
    tables, which the schedule call rebuilds.)"""
    say("case batched schedules")
    Ws = mixed_graphs(6)
    flat, offsets, ns = workloads.pack(Ws)
    Wd = torch.from_numpy(flat).to(DEV)
    b0 = appd.Batch(ns, DEV)
    M0, I0 = b0.forward(Wd)
    torch.cuda.synchronize()
    _, io = oracle.appd(Ws[0])
    assert np.array_equal(unpack(I0.cpu().numpy(), ns, offsets)[0], io)
    narrow = [64, 64, 64, 256, 256, 256]
    wide = [64, 128, 256, 512, 512, 1024]
    mid = [64, 128, 128, 128, 512, 512]
    b = appd.Batch(ns, DEV)
    for threads, rows, streams, stagger in [(narrow, 16, 1, 0), (wide, 32, 3, 0), (mid, 7, 6, 0),
                                            (wide, 64, 2, 0), (narrow, 16, 4, 1), (mid, 7, 3, 1)]:
        b.set_schedule(threads=threads, rows=rows, streams=streams, split_count=0, stagger=stagger)
        M, I = b.forward(Wd)
        torch.cuda.synchronize()
        assert torch.equal(M, M0) and torch.equal(I, I0), (threads, rows, streams, stagger)
    # staggered with the largest class on Prim workgroups: the classes start at once
    b.set_schedule(threads=narrow, rows=16, streams=3, stagger=1, trees="prim")
    M, I = b.forward(Wd)
    torch.cuda.synchronize()
    assert torch.equal(M, M0) and torch.equal(I, I0)
    b.set_schedule(trees="boruvka", stagger=0)
    # a field edited behind the work tables' back is rejected before any launch
    b.plan.class_rows[0] += 1
    with pytest.raises(appd.APPDError):
        b.forward(Wd)


def test_batched_split_largest_class():
    """The largest class cut in two launch pairs on two streams (its biggest
    graphs, then the rest from a chunk offset) gives the same bits as the
    default schedule, at several cuts and stream counts; an out-of-range cut is
    rejected before any launch."""
    say("case batched split of the largest class")
    Ws = mixed_graphs(8)
    flat, offsets, ns = workloads.pack(Ws)
    Wd = torch.from_numpy(flat).to(DEV)
    M0, I0 = appd.Batch(ns, DEV).forward(Wd)
    torch.cuda.synchronize()
    ns = np.asarray(ns)
    cls = np.array([next(c for c in range(appd.BATCH_CLASSES) if n <= 64 << c) for n in ns])
    top = int(cls.max())
    members = np.sort(ns[cls == top])[::-1]  # the class in launch order (n descending)
    assert len(members) >= 2, members
    for h, streams in [(1, 2), (len(members) // 2, 3), (len(members) - 1, 5)]:
        b = appd.Batch(ns, DEV)
        b.set_schedule(streams=streams, split_count=int(h))
        rows = b.plan.class_rows[top]
        assert b.plan.split_count == h
        assert b.plan.split_chunks == sum((int(n) + rows - 1) // rows for n in members[:h])
        M, I = b.forward(Wd)
        torch.cuda.synchronize()
        assert torch.equal(M, M0) and torch.equal(I, I0), (h, streams)
        # a cut edited by hand no longer matches the work tables: rejected
        b.plan.split_chunks += 1
        with pytest.raises(appd.APPDError):
            b.forward(Wd)
    b = appd.Batch(ns, DEV)
    with pytest.raises(appd.APPDError):
        b.set_schedule(streams=3, split_count=len(members))


def test_batched_autotune_bit_exact():
    """The autotuner picks a schedule by timing; whatever it picks, every graph
    still equals the oracle."""
    say("case batched autotune")
    Ws = mixed_graphs(7)
    flat, offsets, ns = workloads.pack(Ws)
    b = appd.Batch(ns, DEV)
    Wd = torch.from_numpy(flat).to(DEV)
    ms = b.autotune(Wd)
    assert ms > 0
    sched = b.schedule()
    say("  chose", sched, "%.3f ms" % ms)
    M, idx = b.forward(Wd)
    torch.cuda.synchronize()
    Ms = unpack(M.cpu().numpy(), ns, offsets)
    Is = unpack(idx.cpu().numpy(), ns, offsets)
    for g, W in enumerate(Ws):
        Mo, io = oracle.appd(W)
        assert np.array_equal(Ms[g].view(np.uint32), Mo.view(np.uint32)) and np.array_equal(Is[g], io), g


def small_mixed_graphs(seed):
    """mixed_graphs without the sizes above 1024 (the persistent form's limit)."""
    return [W for W in mixed_graphs(seed) if W.shape[0] <= 1024]


def test_batched_persistent_form():
    """The whole forward as one persistent launch over the work queue (pass,
    tree and fill items with in-queue dependencies): every graph equals the
    oracle, at several rows per fill item, in both modes; a batch with a graph
    above 1024 vertices cannot take this form."""
    say("case batched persistent form")
    Ws = small_mixed_graphs(9)
    flat, offsets, ns = workloads.pack(Ws)
    Wd = torch.from_numpy(flat).to(DEV)
    for rows in (16, 5, 64):
        b = appd.Batch(ns, DEV)
        b.set_schedule(rows=rows, persistent=True)
        assert b.schedule()["persistent"] == 1 and b.plan.persist_items > 0
        for mode, ref in ((appd.MINIMAX, oracle.appd), (appd.WIDEST, oracle.appd_widest)):
            M, idx = b.forward(Wd, mode=mode)
            appd.sync(DEV)  # also reports a wait of the launch that gave up
            Ms = unpack(M.cpu().numpy(), ns, offsets)
            Is = unpack(idx.cpu().numpy(), ns, offsets)
            for g, W in enumerate(Ws):
                Mo, io = ref(W)
                assert np.array_equal(Ms[g].view(np.uint32), Mo.view(np.uint32)), (rows, mode, g)
                assert np.array_equal(Is[g], io), (rows, mode, g)
    big = mixed_graphs(9)
    _, _, ns_big = workloads.pack(big)
    b = appd.Batch(ns_big, DEV)
    with pytest.raises(appd.APPDError):
        b.set_schedule(persistent=True)


def test_batched_persistent_ragged_and_capture():
    """The persistent form on the ragged 4096-graph batch equals the launch
    sequence bit for bit, and inside a HIP graph every replay equals it too
    (the queue counters are cleared by a kernel, not a memset)."""
    say("case persistent ragged batch + capture")
    with pool() as ex:
        Ws = list(ex.map(workloads.euclid_w, workloads.ragged_points()))
    flat, offsets, ns = workloads.pack(Ws)
    del Ws
    Wd = torch.from_numpy(flat).to(DEV)
    M0, I0 = appd.Batch(ns, DEV).forward(Wd)
    b = appd.Batch(ns, DEV)
    b.set_schedule(persistent=True)
    M, I = b.forward(Wd)
    appd.sync(DEV)
    assert torch.equal(M, M0) and torch.equal(I, I0)
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.forward(Wd, out=(M, I))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        b.forward(Wd, out=(M, I))
    for rep in range(3):
        M.fill_(-7.0)
        I.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        appd.sync(DEV)
        assert torch.equal(M, M0) and torch.equal(I, I0), "replay %d differs" % rep


def test_batched_autotune_plan_cache(tmp_path, monkeypatch):
    """APPD_TUNE_CACHE: the first autotune times the candidates and stores the
    winner under this GPU and class histogram; the file is one JSON object; a
    second Batch of the same histogram takes the stored schedule without
    timing (same milliseconds back, same schedule) and still matches the
    oracle."""
    import json
    say("case autotune plan cache")
    path = tmp_path / "tune.json"
    monkeypatch.setenv("APPD_TUNE_CACHE", str(path))
    Ws = small_mixed_graphs(10)
    flat, offsets, ns = workloads.pack(Ws)
    Wd = torch.from_numpy(flat).to(DEV)
    b1 = appd.Batch(ns, DEV)
    ms1 = b1.autotune(Wd)
    data = json.loads(path.read_text())
    assert len(data) == 1
    (key, entry), = data.items()
    assert "classes" in key and abs(entry["ms"] - ms1) < 1e-3
    assert entry["streams"] == b1.plan.streams and entry["persistent"] == b1.plan.persistent
    assert entry["stagger"] == b1.plan.stagger
    b2 = appd.Batch(ns, DEV)
    ms2 = b2.autotune(Wd)
    assert abs(ms2 - entry["ms"]) < 1e-3
    s1, s2 = b1.schedule(), b2.schedule()
    for k in ("class_rows", "class_tree", "streams", "persistent", "stagger"):
        assert s1[k] == s2[k], k
    M, idx = b2.forward(Wd)
    torch.cuda.synchronize()
    Ms = unpack(M.cpu().numpy(), ns, offsets)
    Is = unpack(idx.cpu().numpy(), ns, offsets)
    for g, W in enumerate(Ws):
        Mo, io = oracle.appd(W)
        assert np.array_equal(Ms[g].view(np.uint32), Mo.view(np.uint32)) and np.array_equal(Is[g], io), g


@pytest.mark.parametrize("stagger", [0, 1])
def test_batched_streams_graph_capture_replays(stagger):
    """Classes on concurrent library streams (fork/join events; staggered: the
    fork after the largest class's pass) inside a HIP graph: every replay
    equals the eager result."""
    say("case batched streams + HIP graph capture stagger=%d" % stagger)
    Ws = mixed_graphs(8)
    flat, offsets, ns = workloads.pack(Ws)
    b = appd.Batch(ns, DEV)
    b.set_schedule(threads=[64, 128, 256, 512, 512, 1024], rows=16, streams=4, stagger=stagger)
    Wd = torch.from_numpy(flat).to(DEV)
    M0, I0 = b.forward(Wd)
    torch.cuda.synchronize()
    M = torch.empty_like(M0)
    I = torch.empty_like(I0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.forward(Wd, out=(M, I))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.forward(Wd, out=(M, I))
    for rep in range(4):
        M.fill_(-7.0)
        I.fill_(-7)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(M, M0) and torch.equal(I, I0), "replay %d differs" % rep
        _ = (M0 * 2).sum().item()


@pytest.mark.parametrize("n,d", [(1, 3), (7, 2), (100, 8), (257, 16), (1000, 8), (2100, 5)])
def test_pairwise_single(n, d):
    say("case pairwise n=%d d=%d" % (n, d))
    rng = np.random.default_rng(n + d)
    X = rng.standard_normal((n, d)).astype(np.float32)
    W = appd.pairwise_euclidean(torch.from_numpy(X).to(DEV))
    torch.cuda.synchronize()
    Wo = oracle.pairwise_euclidean_f32(X)
    assert np.array_equal(W.cpu().numpy().view(np.uint32), Wo.view(np.uint32))


@pytest.mark.parametrize("scale", [1e-21, 1e-3, 1e18])
def test_pairwise_extreme_scales(scale):
    """Tiny coordinates push the sums into the subnormal range, huge ones near
    the top of float32: the square root must still be correctly rounded."""
    say("case pairwise scale=%g" % scale)
    rng = np.random.default_rng(11)
    X = (rng.standard_normal((300, 3)) * scale).astype(np.float32)
    W = appd.pairwise_euclidean(torch.from_numpy(X).to(DEV))
    torch.cuda.synchronize()
    Wo = oracle.pairwise_euclidean_f32(X)
    assert np.array_equal(W.cpu().numpy().view(np.uint32), Wo.view(np.uint32))


def test_pairwise_batched():
    say("case pairwise batched")
    rng = np.random.default_rng(5)
    ns = [1, 5, 64, 65, 300, 1024, 2048, 17]
    d = 8
    Xs = [rng.standard_normal((n, d)).astype(np.float32) for n in ns]
    b = appd.Batch(ns, DEV)
    W = b.pairwise(torch.from_numpy(np.concatenate(Xs)).to(DEV).contiguous(), d)
    torch.cuda.synchronize()
    Ws = unpack(W.cpu().numpy(), ns, b.offsets)
    for X, Wg in zip(Xs, Ws):
        assert np.array_equal(Wg.view(np.uint32), oracle.pairwise_euclidean_f32(X).view(np.uint32))


def grad_close(got, ref):
    tol = 1e-4 * np.abs(ref).max() + 1e-4 * np.abs(ref)
    err = np.abs(got - ref)
    assert (err <= tol).all(), "max err %g (ref max %g)" % (err.max(), np.abs(ref).max())


def ref_grad(X, G):
    """Oracle float64 gradient through the oracle's own float32 forward."""
    W32 = oracle.pairwise_euclidean_f32(X)
    _, idx = oracle.appd(W32)
    return oracle.grad_points(X.astype(np.float64), G.astype(np.float64), idx), W32, idx


# 9001: parents read from global memory (above the LDS-staged limit), odd rows
@pytest.mark.parametrize("n", [2, 3, 50, 513, 2048, 9001])
def test_backward_points_single(n):
    say("case backward points n=%d" % n)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 8)).astype(np.float32)
    G = rng.standard_normal((n, n)).astype(np.float32)
    Xd = torch.from_numpy(X).to(DEV).requires_grad_(True)
    M, idx = appd.appd_points(Xd)
    (M * torch.from_numpy(G).to(DEV)).sum().backward()
    torch.cuda.synchronize()
    ref, W32, io = ref_grad(X, G)
    assert np.array_equal(idx.cpu().numpy(), io)
    grad_close(Xd.grad.cpu().numpy().astype(np.float64), ref)


def test_backward_w_single():
    say("case backward W n=700")
    n = 700
    W = workloads.integer_weights(n, 5, seed=2) + workloads.random_symmetric(n, seed=3)
    np.fill_diagonal(W, 0)
    G = np.random.default_rng(4).standard_normal((n, n)).astype(np.float32)
    Wd = torch.from_numpy(W).to(DEV).requires_grad_(True)
    M, idx = appd.APPDWeights.apply(Wd)
    (M * torch.from_numpy(G).to(DEV)).sum().backward()
    torch.cuda.synchronize()
    _, io = oracle.appd(W)
    ref = np.zeros(n * n)
    off = io >= 0
    np.add.at(ref, io[off], G.astype(np.float64)[off])
    grad_close(Wd.grad.cpu().numpy().ravel().astype(np.float64), ref)


def test_backward_w_batched():
    """Packed dL/dW of a batch of weight matrices: per graph, G_ij onto the
    upper-triangle entry of each pair's bottleneck edge (the oracle's idx)."""
    say("case backward W batched")
    Ws = mixed_graphs(9)[:16]
    flat, offsets, ns = workloads.pack(Ws)
    b = appd.Batch(ns, DEV)
    M, idx, parent = b.forward(torch.from_numpy(flat).to(DEV), return_parent=True)
    rng = np.random.default_rng(10)
    G = rng.standard_normal(flat.size).astype(np.float32)
    dW = b.backward_w(torch.from_numpy(G).to(DEV), idx, parent)
    torch.cuda.synchronize()
    dWh = dW.cpu().numpy()
    for g, W in enumerate(Ws):
        n = W.shape[0]
        o = int(offsets[g])
        _, io = oracle.appd(W)
        ref = np.zeros(n * n)
        off = io >= 0
        np.add.at(ref, io[off], G[o:o + n * n].reshape(n, n).astype(np.float64)[off])
        grad_close(dWh[o:o + n * n].astype(np.float64), ref)


@pytest.mark.timeout(600)
def test_differentiable_batch_full_config():
    """256 graphs, n uniform in {64..2048}, X ~ N(0, I_8): W bit-exact, M and idx
    bit-exact, dX against the float64 reference gradient of every graph."""
    say("case differentiable batch 256 graphs: generate")
    items = workloads.diff_batch()
    ns = [x.shape[0] for x, _ in items]
    d = 8
    b = appd.Batch(ns, DEV)
    X = torch.from_numpy(np.concatenate([x for x, _ in items])).to(DEV).requires_grad_(True)
    Gflat = torch.from_numpy(np.concatenate([g.ravel() for _, g in items])).to(DEV)
    say("case differentiable batch: forward + backward")
    M, idx = appd.appd_points_batched(X, b, d)
    (M * Gflat).sum().backward()
    torch.cuda.synchronize()
    Ms = unpack(M.detach().cpu().numpy(), ns, b.offsets)
    Is = unpack(idx.cpu().numpy(), ns, b.offsets)
    dX = X.grad.cpu().numpy().astype(np.float64)
    say("case differentiable batch: oracle")

    def one(g):
        x, G = items[g]
        ref, W32, io = ref_grad(x, G)
        Mo, _ = oracle.appd(W32)
        o = int(b.noff[g])
        okf = np.array_equal(Ms[g].view(np.uint32), Mo.view(np.uint32)) and np.array_equal(Is[g], io)
        got = dX[o:o + x.shape[0]]
        tol = 1e-4 * np.abs(ref).max() + 1e-4 * np.abs(ref)
        return okf, bool((np.abs(got - ref) <= tol).all()), float(np.abs(got - ref).max())

    with pool() as ex:
        res = list(ex.map(one, range(len(items))))
    assert all(r[0] for r in res), "forward mismatch in graphs %s" % [g for g, r in enumerate(res) if not r[0]][:5]
    bad = [(g, r[2]) for g, r in enumerate(res) if not r[1]]
    assert not bad, "gradient outside tolerance: %s" % bad[:5]


def clustered_graph(k, per, seed, dim=3):
    """k far-apart clusters of `per` points: every vertex's 16 nearest
    neighbours lie in its own cluster once per > 16."""
    rng = np.random.default_rng(seed)
    centres = rng.random((k, dim)) * 1000.0
    X = np.repeat(centres, per, axis=0) + 0.5 * rng.standard_normal((k * per, dim))
    X = X[rng.permutation(len(X))]
    return workloads.euclid_w(X)


@pytest.mark.parametrize("mode", [appd.MINIMAX, appd.WIDEST])
def test_batched_boruvka_refresh_and_fallback(mode):
    """Graphs of many far-apart clusters: their candidate lists stay inside the
    clusters, so the per-graph Boruvka workgroup must refresh the lists of a
    stuck component's used-up vertices (rank top-K with the component masked,
    or the insertion list in 1024-thread workgroups), and with more stuck
    components than refreshes allowed it finishes with Prim's algorithm.
    Every graph equals the oracle; the stats show both paths taken."""
    say("case batched refresh and fallback mode=%d" % mode)
    Ws = [clustered_graph(3, 40, 1), clustered_graph(5, 60, 2), clustered_graph(20, 20, 3),
          clustered_graph(12, 70, 4), clustered_graph(30, 30, 5), clustered_graph(4, 300, 6),
          clustered_graph(30, 50, 7), workloads.random_symmetric(700, seed=8)]
    if mode == appd.WIDEST:  # the maximum spanning tree of c - W keeps the clusters
        Ws = [np.float32(W.max() + 1.0) - W for W in Ws]
        for W in Ws:
            np.fill_diagonal(W, 0.0)
    flat, offsets, ns = workloads.pack(Ws)
    b = appd.Batch(ns, DEV)
    b.set_schedule(trees="boruvka", streams=1)
    M, idx = b.forward(torch.from_numpy(flat).to(DEV), mode=mode)
    torch.cuda.synchronize()
    st = b.tree_stats()
    Ms = unpack(M.cpu().numpy(), ns, offsets)
    Is = unpack(idx.cpu().numpy(), ns, offsets)
    ref = oracle.appd_widest if mode == appd.WIDEST else oracle.appd
    for g, W in enumerate(Ws):
        Mo, io = ref(W)
        assert np.array_equal(Ms[g].view(np.uint32), Mo.view(np.uint32)), (g, int(ns[g]))
        assert np.array_equal(Is[g], io), (g, int(ns[g]))
    assert st["multi_pass"] >= 2 and st["fallback"] >= 1, st
