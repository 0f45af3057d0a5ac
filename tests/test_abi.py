"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2407_07058_amd as appd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(appd_[a-z0-9_]+)\s*\(", txt))
    return names


def test_header_declares_the_core_calls():
    names = declared_symbols()
    for n in ("appd_forward", "appd_forward_ws", "appd_forward_ex",
              "appd_forward_workspace_bytes", "appd_error_string", "appd_get_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(appd.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    # and the Python binding knows every one of them
    assert declared_symbols() <= set(appd.SIGNATURES)


def test_error_strings():
    L = appd.lib()
    for c in (0, -1, -2, -3, -4):
        assert L.appd_error_string(c)
        assert b"unknown" not in L.appd_error_string(c)
    assert b"unknown" in L.appd_error_string(7)


def test_workspace_bytes():
    L = appd.lib()
    assert L.appd_forward_workspace_bytes(0) == 0
    assert L.appd_forward_workspace_bytes(46341) == 0
    small = L.appd_forward_workspace_bytes(1)
    big = L.appd_forward_workspace_bytes(46340)
    assert 0 < small < big
    assert big % 256 == 0
    # O(n): a few hundred bytes per vertex (candidate lists of the parallel tree)
    assert big < 512 * 46340


@pytest.mark.parametrize("n", [0, -5, 46341])
def test_forward_rejects_bad_n(n):
    L = appd.lib()
    p = ctypes.c_void_p(16)
    assert L.appd_forward(p, n, p, p, None) == appd.APPD_EINVAL
    assert L.appd_get_last_error() == appd.APPD_EINVAL


def test_forward_rejects_null_and_mode():
    L = appd.lib()
    p = ctypes.c_void_p(256)
    assert L.appd_forward(None, 4, p, p, None) == appd.APPD_EINVAL
    assert L.appd_forward(p, 4, None, p, None) == appd.APPD_EINVAL
    assert L.appd_forward(p, 4, p, None, None) == appd.APPD_EINVAL
    assert L.appd_forward_ex(p, 4, 2, p, p, None, None, p, 1 << 20, None) == appd.APPD_EINVAL
    assert L.appd_forward_ws(p, 4, p, p, None, 0, None) == appd.APPD_EINVAL


def test_forward_rejects_small_or_misaligned_workspace():
    L = appd.lib()
    p = ctypes.c_void_p(256)
    need = L.appd_forward_workspace_bytes(100)
    assert L.appd_forward_ws(p, 100, p, p, p, need - 1, None) == appd.APPD_EINVAL
    assert L.appd_forward_ws(p, 100, p, p, ctypes.c_void_p(260), need, None) == appd.APPD_EINVAL


def test_write_count_calls_reject_bad_arguments():
    """The write-once check rejects a missing counter array or workspace and
    bad sizes before anything reaches the GPU."""
    L = appd.lib()
    p = ctypes.c_void_p(256)
    need = L.appd_forward_workspace_bytes(100)
    assert L.appd_debug_write_counts(p, 100, 0, p, p, None, p, need, None) == appd.APPD_EINVAL
    assert L.appd_debug_write_counts(p, 100, 0, p, p, p, None, need, None) == appd.APPD_EINVAL
    assert L.appd_debug_write_counts(p, 0, 0, p, p, p, p, need, None) == appd.APPD_EINVAL
    assert L.appd_debug_write_counts(p, 46341, 0, p, p, p, p, need, None) == appd.APPD_EINVAL
    assert L.appd_debug_write_counts_batched(p, 0, p, p, None, None, p, None) == appd.APPD_EINVAL
    assert L.appd_debug_write_counts_batched(p, 0, p, p, p, None, p, None) == appd.APPD_EINVAL
    assert L.appd_get_last_error() == appd.APPD_EINVAL


def test_batch_plan_struct_layout_matches_header(tmp_path):
    """The ctypes mirror of appd_batch_plan has the C layout."""
    import subprocess
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "appd.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(appd_batch_plan),'
                   'offsetof(appd_batch_plan, class_first), offsetof(appd_batch_plan, class_threads),'
                   'offsetof(appd_batch_plan, streams), offsetof(appd_batch_plan, pair_tiles),'
                   'offsetof(appd_batch_plan, ws_bytes), offsetof(appd_batch_plan, tables_key),'
                   'offsetof(appd_batch_plan, split_vertices));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    P = appd.BatchPlan
    assert got == [ctypes.sizeof(P), P.class_first.offset, P.class_threads.offset,
                   P.streams.offset, P.pair_tiles.offset, P.ws_bytes.offset, P.tables_key.offset,
                   P.split_vertices.offset]


def test_batch_workspace_and_bad_sizes():
    import numpy as np
    L = appd.lib()
    ns = np.array([16, 1024, 3], np.int32)
    P = ctypes.c_void_p
    assert L.appd_batch_workspace_bytes(ns.ctypes.data_as(P), 3) > 0
    bad = np.array([16, 2049], np.int32)
    assert L.appd_batch_workspace_bytes(bad.ctypes.data_as(P), 2) == 0
    zero = np.array([0], np.int32)
    assert L.appd_batch_workspace_bytes(zero.ctypes.data_as(P), 1) == 0
    plan = appd.BatchPlan()
    assert L.appd_batch_prepare(bad.ctypes.data_as(P), 2, P(256), 1 << 30, ctypes.byref(plan),
                                None) == appd.APPD_EINVAL
    # a plan that was never prepared is rejected before any launch
    assert L.appd_forward_batched(P(256), 0, P(256), P(256), None, ctypes.byref(plan), P(256),
                                  None) == appd.APPD_EINVAL


def test_grad_calls_reject_bad_arguments():
    L = appd.lib()
    P = ctypes.c_void_p
    p = P(256)
    assert L.appd_grad_workspace_bytes(0) == 0
    assert L.appd_pairwise_euclidean(p, 10, 0, p, p, 1 << 20, None) == appd.APPD_EINVAL
    assert L.appd_pairwise_euclidean(p, 10, 65, p, p, 1 << 20, None) == appd.APPD_EINVAL
    assert L.appd_pairwise_euclidean(p, 10, 3, p, p, 1, None) == appd.APPD_EINVAL
    assert L.appd_backward_points(p, 32769, 3, p, p, p, p, p, p, 1 << 30, None) == appd.APPD_EINVAL
    assert L.appd_backward_w(p, p, None, 10, p, p, 1 << 20, None) == appd.APPD_EINVAL


def test_batched_plan_out_of_step_with_its_tables_is_rejected():
    """A plan whose rows per item or cut were edited after the device work
    tables were built (the stamp no longer matches) is rejected before any
    launch, like one that was never prepared."""
    L = appd.lib()
    P = ctypes.c_void_p
    plan = appd.BatchPlan()
    plan.num_graphs = 3
    plan.total_n = 48
    plan.total_nn = 768
    plan.ws_bytes = 1 << 20
    plan.streams = 2
    plan.class_count[0] = 3
    plan.class_rows[0] = 16
    plan.class_threads[0] = 64
    plan.class_chunks[0] = 3
    plan.split_count = 1
    plan.split_chunks = 2  # inconsistent with one 16-row item per graph
    plan.tables_key = 12345
    assert L.appd_forward_batched(P(256), 0, P(256), P(256), None, ctypes.byref(plan), P(256),
                                  None) == appd.APPD_EINVAL
    assert L.appd_get_last_error() == appd.APPD_EINVAL
    assert L.appd_batch_autotune(P(256), P(256), P(256), ctypes.byref(plan), P(256), None,
                                 None) == appd.APPD_EINVAL


def test_validate_rejects_bad_arguments():
    L = appd.lib()
    P = ctypes.c_void_p
    assert L.appd_validate(None, 4, P(256), None) == appd.APPD_EINVAL
    assert L.appd_validate(P(256), 4, None, None) == appd.APPD_EINVAL
    assert L.appd_validate(P(256), 0, P(256), None) == appd.APPD_EINVAL
    assert L.appd_validate(P(256), 46341, P(256), None) == appd.APPD_EINVAL


def test_backward_w_batched_rejects_bad_arguments():
    L = appd.lib()
    P = ctypes.c_void_p
    plan = appd.BatchPlan()
    assert L.appd_backward_w_batched(P(256), P(256), P(256), P(256), ctypes.byref(plan), P(256),
                                     None) == appd.APPD_EINVAL
    assert L.appd_backward_w_batched(None, P(256), P(256), P(256), ctypes.byref(plan), P(256),
                                     None) == appd.APPD_EINVAL


def test_batch_prepare_host_tables_without_a_device():
    """The host half of appd_batch_prepare (size classes, the n-descending
    order, work tables, the per-row graph table) runs to its first device copy,
    which fails when no GPU is present (APPD_EHIP).  Run under the sanitizer
    test, this checks the table construction's memory accesses."""
    import numpy as np
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present: the copy to a made-up workspace would reach it")
    L = appd.lib()
    P = ctypes.c_void_p
    rng = np.random.default_rng(5)
    ns = rng.integers(1, 2049, 300).astype(np.int32)
    need = L.appd_batch_workspace_bytes(ns.ctypes.data_as(P), len(ns))
    assert need > 0
    plan = appd.BatchPlan()
    rc = L.appd_batch_prepare(ns.ctypes.data_as(P), len(ns), P(1 << 20), need, ctypes.byref(plan),
                              None)
    assert rc == appd.APPD_EHIP
