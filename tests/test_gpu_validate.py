"""GPU checks of appd_validate: the precondition flags of crafted matrices.

The method takes an undirected weighted graph (Section 1), so W must be
symmetric; the library also asks for a NaN-free W with a zero diagonal.  Each
case plants one violation (or none) at a known place, including the ragged last
tile and the diagonal tiles, and compares the flags with what was planted."""
import sys

import numpy as np
import pytest
import torch

import paper_2407_07058_amd as appd
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def flags_of(W):
    return appd.validate(torch.from_numpy(np.ascontiguousarray(W, np.float32)).to(DEV))


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 130, 1000, 4099])
def test_valid_matrices_pass(n):
    say("case validate clean n=%d" % n)
    assert flags_of(workloads.random_symmetric(n, seed=n)) == 0
    W = workloads.integer_weights(n, 3, seed=n) - 1.0  # negatives, ties
    W[W == 0] = -0.0  # -0.0 against +0.0 mirrors: equal weights
    np.fill_diagonal(W, 0.0)
    W[np.arange(n), np.arange(n)] = -0.0 if n > 1 else 0.0
    assert flags_of(W) == 0
    W = workloads.random_symmetric(n, seed=n + 1)
    if n > 1:
        W[0, n - 1] = W[n - 1, 0] = np.inf
    assert flags_of(W) == 0


@pytest.mark.parametrize("n", [2, 65, 1000, 4099])
def test_planted_violations(n):
    say("case validate planted n=%d" % n)
    rng = np.random.default_rng(n)
    base = workloads.random_symmetric(n, seed=n)
    for trial in range(6):
        i, j = (int(x) for x in rng.integers(0, n, 2))
        if i == j:
            j = (i + 1) % n
        W = base.copy()
        W[i, j] = np.nan
        assert flags_of(W) == appd.VALID_NAN, (i, j)
        W = base.copy()
        W[i, j] = W[i, j] + 1.0
        assert flags_of(W) == appd.VALID_ASYM, (i, j)
        W = base.copy()
        W[i, i] = 0.5
        assert flags_of(W) == appd.VALID_DIAG, i
        W = base.copy()
        W[i, i] = np.nan
        W[j, i] = -3.0
        assert flags_of(W) == appd.VALID_NAN | appd.VALID_ASYM | appd.VALID_DIAG, (i, j)
    # the last element of the ragged last tile
    W = base.copy()
    W[n - 1, n - 2] = 7.0
    assert flags_of(W) == appd.VALID_ASYM


def test_async_input_error_surfaces_at_sync():
    """With APPD_VALIDATE set, the single-graph forward enqueues the input
    check before its kernels and returns at once; the bad input (an asymmetric
    pair, planted by the host: all entries finite, nothing for a kernel to trip
    on) is reported by appd_sync, and through appd_get_last_error, on the next
    synchronisation, once.  A clean W afterwards reports nothing."""
    import os
    L = appd.lib()
    n = 300
    W = workloads.random_symmetric(n, seed=9)
    W[5, 17] = W[17, 5] + 0.25
    Wd = torch.from_numpy(W).to(DEV)
    Wc = torch.from_numpy(workloads.random_symmetric(n, seed=10)).to(DEV)
    stream = torch.cuda.current_stream(DEV).cuda_stream
    os.environ["APPD_VALIDATE"] = "1"
    try:
        say("case async input error: asymmetric W, validated forward")
        M, idx = appd.forward(Wd)
        assert L.appd_get_last_error() == appd.APPD_OK  # the call itself succeeded
        assert L.appd_sync(stream) == appd.APPD_EDATA
        assert L.appd_get_last_error() == appd.APPD_EDATA
        assert L.appd_sync(stream) == appd.APPD_OK  # reported once
        say("case async input error: clean W")
        appd.forward(Wc)
        appd.sync(DEV)
        assert L.appd_get_last_error() == appd.APPD_OK
        appd.forward(Wd)
        with pytest.raises(appd.APPDError) as ei:
            appd.sync(DEV)
        assert ei.value.code == appd.APPD_EDATA
    finally:
        del os.environ["APPD_VALIDATE"]
    say("case async input error: unvalidated forward reports nothing")
    appd.forward(Wd)
    assert L.appd_sync(stream) == appd.APPD_OK


def test_launch_log():
    """APPD_LOG=1: every kernel launch of a forward is written to stderr."""
    import subprocess
    say("case launch log")
    code = ("import torch, workloads, paper_2407_07058_amd as appd\n"
            "W = torch.from_numpy(workloads.random_symmetric(200, seed=1)).to('cuda:0')\n"
            "appd.forward(W); torch.cuda.synchronize()\n")
    import os
    env = dict(os.environ, APPD_LOG="1")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stderr.splitlines() if l.startswith("appd: launch ")]
    assert len(lines) >= 3, r.stderr[-2000:]
    assert any("fill" in l for l in lines)
