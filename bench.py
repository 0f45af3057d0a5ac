#!/usr/bin/env python3
"""APPD benchmark on one MI355X.

Headline workload: one complete graph of n = 8192 points in R^16 drawn from a
10-component Gaussian mixture (centres uniform in [0,1]^16, sigma 0.05, seed 2);
float32 Euclidean weights (computed in float64, rounded once), so W is 256 MiB.
A step is one whole forward -- spanning tree, attachment order and the
calculation-and-copy fill -- through appd_forward_ex, writing the float32 M and
int32 idx matrices, with W already resident in HBM.  `value` is n^2 entries per
second over the timed steps.

Beside it, on the same GPU:
  large    -- one dense graph of n = 32768, upper triangle iid uniform(0,1)
              fp32, mirrored, zero diagonal (drawn on the GPU with torch's
              generator: the recipe of the n = 32768 test workload, another
              random stream), 4 GiB each of W, M and idx;
  batched  -- 4096 graphs, n log-uniform in [16, 1024], points uniform in
              [0,1]^d, d in {2, 8}: the batched forward replayed from a HIP graph
              against a loop of single-graph forward calls;
  fwd_bwd  -- 256 graphs, n uniform in {64..2048}, X ~ N(0, I_8), upstream
              gradient G ~ N(0, 1): point-to-graph weights, forward and backward
              to the points, batched against a per-graph loop;
  reference -- what a plain streaming copy and store reach on this GPU, the
              latency of a chain of dependent loads (HBM and L2), and the
              sequential Prim step for comparison with it.
The roofline entry describes the kernel that takes the most time per headline
step; its launches are bracketed by HIP events on the library's launch stream
(appd_timer_*) inside the timed region.  The CPU oracle (plain Algorithm 4, one
thread) is timed on the host as a reference point.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
K_LIST = 16             # candidate-list length of the parallel tree (appd_tree.hip)

CSRC = "paper_2407_07058_amd/csrc/"
KERNEL_SOURCES = {
    "fill_kernel": [CSRC + "appd_fill.h", CSRC + "appd_device.h", CSRC + "appd_single.hip"],
    "tree_pass_kernel": [CSRC + "appd_tree.hip", CSRC + "appd_device.h"],
    "tree_refresh_kernel": [CSRC + "appd_tree.hip", CSRC + "appd_device.h"],
    "tree_rounds_kernel": [CSRC + "appd_tree.hip", CSRC + "appd_device.h"],
    "prim_single_kernel": [CSRC + "appd_prim.h", CSRC + "appd_device.h",
                           CSRC + "appd_single.hip"],
}


# Single-graph kernels whose time is set by HBM traffic (the roofline
# candidates); the rest of the tree kernels are bound by latency.
HBM_BOUND_KERNELS = ("fill_kernel", "prim_single_kernel", "tree_pass_kernel",
                     "tree_refresh_kernel", "fill_prep_kernel")


def alg_bytes_per_launch(kernel, n, launches=1.0, stats=None):
    """Algorithmic HBM bytes one launch of `kernel` moves on average for one
    n-vertex graph.  The tree kernels are launched a fixed number of times per
    forward and return at once when the tree is already complete, so their
    per-launch figure is the work of the launches that ran (stats: the tree's
    own count of passes over W) spread over all launches."""
    stats = stats or {}
    per = {
        "fill_kernel": 8.0 * n * n,          # M (fp32) + idx (int32) written once
        "prim_single_kernel": 4.0 * n * n,   # W read once (one row per Prim step)
    }
    if kernel in per:
        return per[kernel]
    if kernel == "tree_pass_kernel":         # the first pass: W read once, always runs
        return 4.0 * n * n
    if kernel == "tree_refresh_kernel":      # later passes that ran: a list pass reads W,
        tables = stats.get("tables", 0)      # a component-table pass its upper triangle
        lists = max(stats.get("passes", 1) - 1 - tables, 0)
        return (4.0 * n * n * lists + 2.0 * n * (n - 1) * tables) / launches
    if kernel == "tree_rounds_kernel":       # candidate lists (2-byte id + 4-byte weight
        return (6.0 * K_LIST + 12.0) * n * stats.get("passes", launches) / launches  # each) + labels
    return None


def source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's
    readings) from the committed rocprofv3 counter summary, or None when missing
    or taken on a different version of the kernel's sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    rec = json.load(open(path)).get("%s@%s" % (kernel, workload))
    if not rec:
        return None
    if rec.get("source_sha") != source_sha(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(W, n, runs=5):
    """The oracle (plain Algorithm 4, one thread; it is sequential) on the
    headline graph, built for this host with -O3 -march=native."""
    import numpy as np

    import oracle
    lib = oracle.native_build()
    M = np.empty((n, n), np.float32)
    idx = np.empty((n, n), np.int32)
    ts = []
    for _ in range(runs):
        t = time.perf_counter()
        oracle.appd(W, lib=lib, out=(M, idx))
        ts.append(time.perf_counter() - t)
    t = float(np.median(ts))
    return {"value": n * n / t, "unit": "entries/s", "cores": 1, "kind": "oracle",
            "sample": "the full n=%d graph, %d runs of the single-threaded C oracle (plain "
                      "Algorithm 4, gcc -O3 -march=native), median %.2f s; M and idx written"
                      % (n, runs, t)}


def cpu_batch_oracle(jobs, entries_of, threads):
    """Wall time of the oracle over independent graphs on `threads` host
    threads, largest first (LPT); ctypes releases the GIL during each call."""
    from concurrent.futures import ThreadPoolExecutor
    order = sorted(range(len(jobs)), key=lambda i: -entries_of(i))
    t = time.perf_counter()
    if threads == 1:
        for i in order:
            jobs[i]()
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda i: jobs[i](), order))
    return time.perf_counter() - t


def elapsed(a, b):
    return a.elapsed_time(b)


def bench_single(appd, torch, Wd, n, steps, warmup, graph_replay=True):
    dev = Wd.device
    M = torch.empty((n, n), dtype=torch.float32, device=dev)
    I = torch.empty((n, n), dtype=torch.int32, device=dev)
    ws = torch.empty(appd.workspace_bytes(n), dtype=torch.uint8, device=dev)

    def step():
        appd.forward(Wd, out=(M, I), workspace=ws)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # kernel census (untimed): every launch bracketed, two steps
    census = {}
    with appd.LaunchTimer("*") as tm:
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        for name in tm.names():
            cnt, tot, _ = tm.read(name)
            census[name] = {"launches_per_step": cnt / 2.0, "ms_per_step": tot / 2.0,
                            "avg_launch_ms": tot / max(cnt, 1)}
    # the roofline kernel: the longest of the kernels bound by HBM traffic (the
    # Boruvka rounds run in one workgroup, bound by latency; the census shows
    # them, and the line reports the longest kernel of all beside)
    hbm_bound = [k for k in census if k in HBM_BOUND_KERNELS] or list(census)
    dominant = max(hbm_bound, key=lambda k: census[k]["ms_per_step"])

    # timed region: only the dominant kernel's launches are bracketed
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    with appd.LaunchTimer(dominant) as tm:
        torch.cuda.synchronize()
        t0.record()
        for _ in range(steps):
            step()
        t1.record()
        torch.cuda.synchronize()
        launches, kern_ms, overflow = tm.read()
    ms = elapsed(t0, t1) / steps
    assert not overflow and launches > 0
    avg_launch_ms = kern_ms / launches

    stats = appd.tree_stats(n, ws)
    if not graph_replay:
        return ms, census, dominant, launches / steps, avg_launch_ms, None, stats
    # the same forward captured once in a HIP graph and replayed (the call only
    # launches kernels when given a workspace)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        graph.replay()
    t1.record()
    torch.cuda.synchronize()
    graph_ms = elapsed(t0, t1) / steps
    return ms, census, dominant, launches / steps, avg_launch_ms, graph_ms, stats


def roofline_of(dom, n, dom_launches, dom_ms, stats, wl_key):
    alg = alg_bytes_per_launch(dom, n, dom_launches, stats)
    r = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": HBM_PEAK_GBPS,
         "unit": "GB/s", "frac": None, "traffic": measured_traffic(dom, wl_key),
         "alg_bytes_per_launch": alg, "launches_per_step": dom_launches,
         "avg_launch_ms": dom_ms}
    if alg is not None:
        r["achieved"] = alg / dom_ms / 1e6
        r["frac"] = r["achieved"] / HBM_PEAK_GBPS
    return r


def uniform_on_gpu(torch, n, seed):
    """Symmetric fp32 W, upper triangle iid uniform [0,1), zero diagonal,
    drawn on the GPU in row blocks (4 GiB at n = 32768)."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    W = torch.empty((n, n), dtype=torch.float32, device=dev)
    blk = 4096
    for r0 in range(0, n, blk):
        W[r0:r0 + blk] = torch.rand((min(blk, n - r0), n), generator=g, device=dev)
    for r0 in range(0, n, blk):  # mirror the upper triangle, block row by block row
        r1 = min(n, r0 + blk)
        W[r0:r1, :r0] = W[:r0, r0:r1].t()
        sub = W[r0:r1, r0:r1]
        sub.copy_(torch.triu(sub, 1) + torch.triu(sub, 1).t())
    return W


def bench_large(appd, torch, n=32768, steps=5, warmup=1):
    """The largest single-GPU configuration: one n = 32768 dense graph."""
    Wd = uniform_on_gpu(torch, n, seed=3)
    torch.cuda.synchronize()
    ms, census, dom, dom_launches, dom_ms, _, stats = bench_single(
        appd, torch, Wd, n, steps, warmup, graph_replay=False)
    del Wd
    torch.cuda.empty_cache()
    entries = float(n) * n
    return {"workload": "single dense graph, n=%d, upper triangle iid uniform(0,1) fp32 "
                        "drawn on the GPU (torch generator, seed 3), mirrored, zero diagonal; "
                        "W resident in HBM; outputs fp32 M + int32 idx" % n,
            "n": n, "steps": steps, "warmup": warmup, "ms_per_step": ms,
            "entries_per_s": entries / (ms / 1e3),
            "alg_hbm_gbps": 12.0 * entries / (ms / 1e3) / 1e9,
            "alg_hbm_frac": 12.0 * entries / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS,
            "kernels": census, "tree": stats,
            "longest_kernel": max(census, key=lambda k: census[k]["ms_per_step"]),
            "roofline": roofline_of(dom, n, dom_launches, dom_ms, stats, "single-%d" % n)}


def bench_reference(appd, torch, prim_n=8192):
    """Reference points on this GPU: streaming copy and store of 1 GiB, the
    latency of dependent loads (a random cycle over 1 GiB, four times the
    last-level cache, and over 1 MiB, inside one L2), and the sequential Prim
    step (the spanning tree by Prim's algorithm, per step)."""
    import numpy as np
    dev = torch.device("cuda:0")
    L = appd.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    P = ctypes.c_void_p
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    out = {}
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0.record()
        for _ in range(reps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        return elapsed(t0, t1) / reps

    ms = timed(lambda: L.appd_membench_copy(P(src.data_ptr()), P(dst.data_ptr()), nbytes, stream), 10)
    out["copy_gbps"] = 2.0 * nbytes / ms / 1e6
    ms = timed(lambda: L.appd_membench_write(P(dst.data_ptr()), nbytes, 7, stream), 10)
    out["write_gbps"] = nbytes / ms / 1e6
    del src, dst
    rng = np.random.default_rng(0)
    for name, entries in (("chase_hbm_ns", 1 << 28), ("chase_l2_ns", 1 << 18)):
        perm = rng.permutation(entries).astype(np.uint32)
        nxt = np.empty(entries, np.uint32)
        nxt[perm] = np.roll(perm, -1)  # one cycle through every entry
        del perm
        nd = torch.from_numpy(nxt.view(np.int32)).to(dev)
        res = torch.empty(1, dtype=torch.int32, device=dev)
        steps = 20000
        ms = timed(lambda: L.appd_membench_chase(P(nd.data_ptr()), entries, 0, steps,
                                                 P(res.data_ptr()), stream), 3)
        out[name] = ms * 1e6 / steps
        del nd
    W = workloads_mixture(prim_n)
    Wd = torch.from_numpy(W).to(dev)
    ws = torch.empty(appd.workspace_bytes(prim_n), dtype=torch.uint8, device=dev)
    ms = timed(lambda: appd.tree(Wd, ws, tree="prim"), 3)
    out["prim_tree_ms_n%d" % prim_n] = ms
    out["prim_ns_per_step"] = ms * 1e6 / (prim_n - 1)
    out["note"] = ("copy: 1 GiB read + 1 GiB written per launch; write: 1 GiB stored; chase: "
                   "one lane, each load's address from the previous load; prim: the spanning "
                   "tree of the n=%d mixture by Prim's algorithm in one workgroup "
                   "(n-1 dependent steps)" % prim_n)
    return out


def workloads_mixture(n):
    import workloads
    return workloads.config_mixture(n)


def bench_batched(appd, torch, steps, lean=False):
    """4096 ragged graphs: batched forward (HIP graph replay) vs per-graph loop."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import workloads
    with ThreadPoolExecutor(8) as ex:
        Ws = list(ex.map(workloads.euclid_w, workloads.ragged_points()))
    flat, offsets, ns = workloads.pack(Ws)
    dev = torch.device("cuda:0")
    b = appd.Batch(ns, dev)
    Wd = torch.from_numpy(flat).to(dev)
    del flat
    M = torch.empty_like(Wd)
    I = torch.empty(Wd.numel(), dtype=torch.int32, device=dev)
    entries = float(b.total_nn)

    tw = time.perf_counter()
    tune_ms = None if lean else b.autotune(Wd, out=(M, I))
    tune_wall = time.perf_counter() - tw
    sched = b.schedule()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.forward(Wd, out=(M, I))
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.forward(Wd, out=(M, I))
    graph.replay()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        graph.replay()
    t1.record()
    torch.cuda.synchronize()
    ms_b = elapsed(t0, t1) / steps
    tstats = b.tree_stats()
    if lean:  # profiling: the replays alone
        return {"batched_ms": ms_b, "entries": entries, "schedule": sched, "lean": True,
                "tree_stats": tstats}
    Mb = M.clone()
    Ib = I.clone()

    # per-graph loop: one appd_forward_ws call per graph, same stream, same buffers
    L = appd.lib()
    wsz = max(appd.workspace_bytes(int(n)) for n in ns)
    ws = torch.empty(wsz, dtype=torch.uint8, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    wp, mp, ip, sp = Wd.data_ptr(), M.data_ptr(), I.data_ptr(), ws.data_ptr()
    calls = [(ctypes.c_void_p(wp + 4 * int(o)), int(n), ctypes.c_void_p(mp + 4 * int(o)),
              ctypes.c_void_p(ip + 4 * int(o))) for o, n in zip(offsets, ns)]
    fwd = L.appd_forward_ws

    def loop():
        for w, n, m, i in calls:
            rc = fwd(w, n, m, i, ctypes.c_void_p(sp), wsz, stream)
            if rc:
                raise RuntimeError("appd_forward_ws failed (%d)" % rc)

    loop()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        loop()
    t1.record()
    torch.cuda.synchronize()
    ms_l = elapsed(t0, t1) / steps
    same = bool(torch.equal(M, Mb) and torch.equal(I, Ib))
    cpu = cpu_batch_leg(Ws, ns, lambda W: (lambda: oracle_appd_native(W)))
    del Ws
    return {"workload": "4096 graphs, n log-uniform in [16,1024] (sum n^2 = %d), points "
                        "uniform in [0,1]^d, d in {2,8}, seed 4; fp32 Euclidean W packed "
                        "in HBM" % b.total_nn,
            "entries": entries,
            "batched_ms": ms_b, "batched_entries_per_s": entries / ms_b * 1e3,
            "batched_alg_gbps": 12.0 * entries / ms_b / 1e6,
            "loop_ms": ms_l, "loop_entries_per_s": entries / ms_l * 1e3,
            "speedup_vs_loop": ms_l / ms_b,
            "batched": "one prepared plan, schedule chosen by the autotuner, replayed from a "
                       "HIP graph",
            "schedule": sched, "autotune_best_ms_per_forward": tune_ms,
            "autotune_wall_s": tune_wall,
            "loop": "%d appd_forward_ws calls on one stream" % len(ns),
            "outputs_identical": same, "tree_stats": tstats, "cpu_oracle": cpu}


def oracle_appd_native(W):
    import oracle
    return oracle.appd(W, lib=oracle.native_build())


def cpu_batch_leg(items, ns, job_of):
    """The oracle over a sample of the batch's graphs on 1 and on 8 host threads
    (every 8th graph for one thread, every 2nd for eight), as entries per
    second; the graphs are independent, so the batch splits over threads."""
    import numpy as np
    out = {}
    for threads, every in ((1, 8), (8, 2)):
        sel = list(range(0, len(items), every))
        jobs = [job_of(items[i]) for i in sel]
        ent = [float(ns[i]) ** 2 for i in sel]
        t = cpu_batch_oracle(jobs, lambda k: ent[k], threads)
        out["threads_%d" % threads] = {"entries_per_s": sum(ent) / t, "seconds": t,
                                       "sample": "every %d-th graph (%d graphs, sum n^2 = %d)"
                                                 % (every, len(sel), int(sum(ent)))}
    out["kind"] = "oracle (gcc -O3 -march=native), LPT order over the sampled graphs"
    return out


def bench_fwd_bwd(appd, torch, steps, lean=False):
    """256 graphs: W from X + forward + backward to X, batched vs per-graph loop."""
    import numpy as np

    import workloads
    items = workloads.diff_batch()
    ns = np.array([x.shape[0] for x, _ in items], np.int32)
    d = 8
    dev = torch.device("cuda:0")
    b = appd.Batch(ns, dev)
    X = torch.from_numpy(np.concatenate([x for x, _ in items])).to(dev).contiguous()
    G = torch.from_numpy(np.concatenate([g.ravel() for _, g in items])).to(dev)
    W = torch.empty(b.total_nn, dtype=torch.float32, device=dev)
    M = torch.empty_like(W)
    I = torch.empty(b.total_nn, dtype=torch.int32, device=dev)
    entries = float(b.total_nn)

    b.pairwise(X, d, out=W)
    if not lean:
        b.autotune(W, out=(M, I))

    def batched():
        b.pairwise(X, d, out=W)
        _, _, parent = b.forward(W, out=(M, I), return_parent=True)
        return b.backward_points(X, d, W, G, I, parent)

    dXb = batched()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        batched()
    t1.record()
    torch.cuda.synchronize()
    ms_b = elapsed(t0, t1) / steps
    tstats = b.tree_stats()
    if lean:  # profiling: the batched steps alone
        return {"batched_ms": ms_b, "entries": entries, "schedule": b.schedule(), "lean": True,
                "tree_stats": tstats}

    L = appd.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    fsz = max(appd.workspace_bytes(int(n)) for n in ns)
    gsz = max(int(L.appd_grad_workspace_bytes(int(n))) for n in ns)
    fws = torch.empty(fsz, dtype=torch.uint8, device=dev)
    gws = torch.empty(gsz, dtype=torch.uint8, device=dev)
    parent = torch.empty(b.total_n, dtype=torch.int32, device=dev)
    dX = torch.empty(b.total_n * d, dtype=torch.float32, device=dev)
    P = ctypes.c_void_p
    xp, wp, mp, ip, gp = X.data_ptr(), W.data_ptr(), M.data_ptr(), I.data_ptr(), G.data_ptr()
    pp, dp = parent.data_ptr(), dX.data_ptr()
    calls = []
    for g, n in enumerate(ns):
        o, no = int(b.offsets[g]), int(b.noff[g])
        calls.append((int(n), P(xp + 4 * d * no), P(wp + 4 * o), P(mp + 4 * o), P(ip + 4 * o),
                      P(gp + 4 * o), P(pp + 4 * no), P(dp + 4 * d * no)))

    def loop():
        for n, x, w, m, i, gg, par, dx in calls:
            rc = L.appd_pairwise_euclidean(x, n, d, w, P(gws.data_ptr()), gsz, stream)
            rc = rc or L.appd_forward_ex(w, n, 0, m, i, None, par, P(fws.data_ptr()), fsz, stream)
            rc = rc or L.appd_backward_points(x, n, d, w, gg, i, par, dx, P(gws.data_ptr()), gsz,
                                              stream)
            if rc:
                raise RuntimeError("per-graph call failed (%d)" % rc)

    loop()
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        loop()
    t1.record()
    torch.cuda.synchronize()
    ms_l = elapsed(t0, t1) / steps
    err = float((dX - dXb).abs().max() / dXb.abs().max().clamp_min(1e-30))

    def job_of(item):
        import oracle
        lib = oracle.native_build()

        def job():
            x, gg = item
            W32 = oracle.pairwise_euclidean_f32(x, lib=lib)
            _, idx = oracle.appd(W32, lib=lib)
            oracle.grad_points(x, gg, idx, lib=lib)
        return job
    cpu = cpu_batch_leg(items, ns, job_of)
    cpu["step"] = "W from X (float32), Algorithm 4, gradient to X (float64) per graph"
    del items
    return {"workload": "256 graphs, n uniform in {64..2048} (sum n^2 = %d), X ~ N(0, I_8) "
                        "fp32, G ~ N(0,1) fp32, seed 5" % b.total_nn,
            "entries": entries,
            "batched_ms": ms_b, "batched_entries_per_s": entries / ms_b * 1e3,
            "loop_ms": ms_l, "loop_entries_per_s": entries / ms_l * 1e3,
            "speedup_vs_loop": ms_l / ms_b,
            "alg_bytes": "W build 4n^2 + forward 12n^2 + backward 8n^2 per graph",
            "batched_alg_gbps": 24.0 * entries / ms_b / 1e6,
            "loop": "%d x (appd_pairwise_euclidean, appd_forward_ex, appd_backward_points)"
                    % len(ns),
            "schedule": b.schedule(),
            "dX_rel_diff_loop_vs_batched": err, "tree_stats": tstats, "cpu_oracle": cpu}


LEGS = ("single", "large", "batched", "fwd_bwd", "reference")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batches", action="store_true",
                    help="skip the batched and forward+backward comparisons")
    ap.add_argument("--only", choices=LEGS, default=None,
                    help="run one leg alone (for profiling); prints its JSON object")
    ap.add_argument("--lean", action="store_true",
                    help="with --only batched / fwd_bwd: default schedule, no per-graph loop, "
                         "no CPU timing (for profiler runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this APPD build runs on a single MI355X and "
              "has no multi-GPU path (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(max(args.steps, 1)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "launches": max(args.steps, 1)}))
        return

    import torch

    import paper_2407_07058_amd as appd
    import workloads

    if args.only in ("large", "batched", "fwd_bwd", "reference"):
        print("step %s" % args.only, file=sys.stderr, flush=True)
        fn = {"large": lambda: bench_large(appd, torch, steps=min(args.steps, 5)),
              "batched": lambda: bench_batched(appd, torch, 3, args.lean),
              "fwd_bwd": lambda: bench_fwd_bwd(appd, torch, 3, args.lean),
              "reference": lambda: bench_reference(appd, torch)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return

    n = args.n
    if n == 8192:
        W = workloads.config_mixture(n)
        wl = ("single complete graph, n=8192 points in R^16 from a 10-component Gaussian "
              "mixture (sigma 0.05, seed 2); fp32 Euclidean W resident in HBM; outputs fp32 M "
              "+ int32 idx")
    elif n == 32768:
        W = workloads.config_uniform(n)
        wl = ("single dense graph, n=32768, upper triangle iid uniform(0,1) fp32 (seed 3), "
              "mirrored, zero diagonal; outputs fp32 M + int32 idx")
    else:
        W = workloads.config_mixture(n)
        wl = "single complete graph, n=%d points from the 10-component mixture (seed 2)" % n
    wl_key = "single-%d" % n
    print("step single-graph forward n=%d" % n, file=sys.stderr, flush=True)
    Wd = torch.from_numpy(W).to("cuda:0")
    ms, census, dom, dom_launches, dom_ms, graph_ms, stats = bench_single(
        appd, torch, Wd, n, args.steps, args.warmup)
    del Wd
    torch.cuda.empty_cache()

    entries = float(n) * n
    out = {
        "metric": "APPD entries/sec (n^2/s)",
        "value": entries / (ms / 1e3),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl, "n": n, "mode": "minimax"},
        "alg_hbm_gbps": 12.0 * entries / (ms / 1e3) / 1e9,
        "alg_hbm_frac": 12.0 * entries / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS,
        "graph_replay_ms_per_step": graph_ms,
        "graph_replay_value": entries / (graph_ms / 1e3),
        "kernels": census,
        "tree": stats,
        "longest_kernel": max(census, key=lambda k: census[k]["ms_per_step"]),
        "roofline": roofline_of(dom, n, dom_launches, dom_ms, stats, wl_key),
    }
    if args.only is None and n != 32768:
        print("step large graph n=32768", file=sys.stderr, flush=True)
        out["large"] = bench_large(appd, torch)
    if args.only is None and not args.no_batches:
        print("step batched forward vs loop", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(appd, torch, 3)
        torch.cuda.empty_cache()
        print("step fwd+bwd vs loop", file=sys.stderr, flush=True)
        out["fwd_bwd"] = bench_fwd_bwd(appd, torch, 3)
        torch.cuda.empty_cache()
    if args.only is None:
        print("step reference points", file=sys.stderr, flush=True)
        out["reference"] = bench_reference(appd, torch)
    if not args.no_cpu_baseline:
        print("step cpu oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W, n, runs=5 if n <= 8192 else 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
