"""appd_forward_noalloc (the forward whose workspace is a library-owned device
array, for callers that cannot allocate) against appd_forward_ws, called
through the C ABI: bit-identical M and idx on two calls in a row, the second
on a smaller graph, so the second runs on the array the first left behind."""
import ctypes
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


def stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream(torch.device(DEV)).cuda_stream)


def via_ws(Wd):
    n = Wd.shape[0]
    M = torch.empty((n, n), dtype=torch.float32, device=DEV)
    I = torch.empty((n, n), dtype=torch.int32, device=DEV)
    nb = appd.lib().appd_forward_workspace_bytes(n)
    ws = torch.empty(nb, dtype=torch.uint8, device=DEV)
    rc = appd.lib().appd_forward_ws(ctypes.c_void_p(Wd.data_ptr()), n, ctypes.c_void_p(M.data_ptr()),
                                    ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nb,
                                    stream_ptr())
    assert rc == appd.APPD_OK
    return M, I


def via_noalloc(Wd):
    n = Wd.shape[0]
    M = torch.full((n, n), -7.0, dtype=torch.float32, device=DEV)
    I = torch.full((n, n), -7, dtype=torch.int32, device=DEV)
    rc = appd.lib().appd_forward_noalloc(ctypes.c_void_p(Wd.data_ptr()), n,
                                         ctypes.c_void_p(M.data_ptr()), ctypes.c_void_p(I.data_ptr()),
                                         stream_ptr())
    assert rc == appd.APPD_OK, rc
    return M, I


@pytest.mark.parametrize("sizes", [(3001, 1000), (8192, 257), (2500, 2)])
def test_noalloc_matches_ws_twice(sizes):
    for k, n in enumerate(sizes):
        say("case noalloc n=%d (call %d of %d)" % (n, k + 1, len(sizes)))
        if n >= 2500 and k == 0 and sizes[0] == 2500:
            # clustered points: the Boruvka tree with its component-table pass
            rng = np.random.default_rng(n)
            centres = rng.random((5, 3)) * 100
            X = centres[rng.integers(0, 5, n)] + 0.3 * rng.standard_normal((n, 3))
            W = workloads.euclid_w(X)
        else:
            W = workloads.random_symmetric(n, seed=n)
        Wd = torch.from_numpy(W).to(DEV)
        M0, I0 = via_ws(Wd)
        M1, I1 = via_noalloc(Wd)
        torch.cuda.synchronize()
        assert torch.equal(M1.view(torch.int32), M0.view(torch.int32)), "M differs (n=%d)" % n
        assert torch.equal(I1, I0), "idx differs (n=%d)" % n


def test_noalloc_rejects_bad_sizes():
    L = appd.lib()
    p = ctypes.c_void_p(256)
    assert L.appd_forward_noalloc(p, 0, p, p, None) == appd.APPD_EINVAL
    assert L.appd_forward_noalloc(p, appd.MAX_N + 1, p, p, None) == appd.APPD_EINVAL
    assert L.appd_get_last_error() == appd.APPD_EINVAL
    assert L.appd_forward_noalloc(None, 10, p, p, None) == appd.APPD_EINVAL
