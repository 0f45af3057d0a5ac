"""MI355X-native all-points minimax path distance (APPD).

Thin ctypes binding over ``libappd.so`` (HIP, gfx950); the C ABI is declared in
``include/appd.h``.  This module only checks arguments, allocates the output
tensors and workspaces through PyTorch's caching allocator, and passes device
pointers plus the current HIP stream; every step of the computation runs in the
library's kernels.  There is no CPU fallback: if the library is missing or no
GPU is present the calls raise.

Method: arXiv 2407.07058, Algorithm 4 (MMJ distance by Calculation and Copy).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# APPD_LIB names another build of the same library (the sanitizer test loads a
# host-instrumented one); by default the in-tree build.
LIB_PATH = os.environ.get("APPD_LIB") or os.path.join(_PKG, "libappd.so")

MINIMAX = 0
WIDEST = 1
MAX_N = 46340
TREE_FLAGS = {"auto": 0x00, "prim": 0x10, "boruvka": 0x20,
              # testing aid: one pass over W, then the Prim fallback if needed
              "boruvka_one_pass": 0x60}

APPD_OK = 0
APPD_EINVAL = -1
APPD_EHIP = -2
APPD_ENOMEM = -3
APPD_EDATA = -4

# every symbol include/appd.h declares, with its ctypes signature
_P = ctypes.c_void_p
_I = ctypes.c_int
_SZ = ctypes.c_size_t
SIGNATURES = {
    "appd_error_string": ([_I], ctypes.c_char_p),
    "appd_validate": ([_P, _I, _P, _P], _I),
    "appd_sync": ([_P], _I),
    "appd_get_last_error": ([], _I),
    "appd_forward_workspace_bytes": ([_I], _SZ),
    "appd_forward": ([_P, _I, _P, _P, _P], _I),
    "appd_forward_ws": ([_P, _I, _P, _P, _P, _SZ, _P], _I),
    "appd_forward_ex": ([_P, _I, _I, _P, _P, _P, _P, _P, _SZ, _P], _I),
    "appd_forward_noalloc": ([_P, _I, _P, _P, _P], _I),
    "appd_tree": ([_P, _I, _I, _P, _P, _P, _SZ, _P], _I),
    "appd_fill": ([_I, _I, _P, _SZ, _P, _P, _P], _I),
    "appd_linkage": ([_P, _I, _I, _P, _P, _SZ, _P], _I),
    "appd_tree_stats": ([_I, _I, _P, _SZ, _P, _P], _I),
    "appd_batch_workspace_bytes": ([_P, _I], _SZ),
    "appd_batch_prepare": ([_P, _I, _P, _SZ, _P, _P], _I),
    "appd_forward_batched": ([_P, _I, _P, _P, _P, _P, _P, _P], _I),
    "appd_batch_set_schedule": ([_P, _P, _P], _I),
    "appd_batch_tree_stats": ([_P, _P, _P, _P], _I),
    "appd_batch_autotune": ([_P, _P, _P, _P, _P, _P, _P], _I),
    "appd_pairwise_euclidean_batched": ([_P, _I, _P, _P, _P, _P], _I),
    "appd_backward_points_batched": ([_P, _I, _P, _P, _P, _P, _P, _P, _P, _P], _I),
    "appd_grad_workspace_bytes": ([_I], _SZ),
    "appd_pairwise_euclidean": ([_P, _I, _I, _P, _P, _SZ, _P], _I),
    "appd_backward_points": ([_P, _I, _I, _P, _P, _P, _P, _P, _P, _SZ, _P], _I),
    "appd_backward_w": ([_P, _P, _P, _I, _P, _P, _SZ, _P], _I),
    "appd_backward_w_batched": ([_P, _P, _P, _P, _P, _P, _P], _I),
    "appd_membench_copy": ([_P, _P, _SZ, _P], _I),
    "appd_membench_write": ([_P, _SZ, ctypes.c_uint32, _P], _I),
    "appd_membench_chase": ([_P, ctypes.c_uint32, ctypes.c_uint32, _I, _P, _P], _I),
    "appd_timer_start": ([ctypes.c_char_p, _I], _I),
    "appd_timer_read": ([ctypes.c_char_p, _P, _P, _P], _I),
    "appd_timer_names": ([_P, _I], _I),
    "appd_debug_write_counts": ([_P, _I, _I, _P, _P, _P, _P, _SZ, _P], _I),
    "appd_debug_write_counts_batched": ([_P, _I, _P, _P, _P, _P, _P, _P], _I),
}

VALID_NAN = 0x1
VALID_ASYM = 0x2
VALID_DIAG = 0x4

BATCH_MAX_N = 2048
BATCH_TREES = {"prim": 0, "boruvka": 1}
BATCH_CLASSES = 6
MAX_DIM = 64
GRAD_MAX_N = 32768


class BatchPlan(ctypes.Structure):
    """Mirror of appd_batch_plan (include/appd.h)."""
    _fields_ = [("num_graphs", ctypes.c_int), ("max_n", ctypes.c_int),
                ("total_n", ctypes.c_int64), ("total_nn", ctypes.c_int64),
                ("class_first", ctypes.c_int * BATCH_CLASSES),
                ("class_count", ctypes.c_int * BATCH_CLASSES),
                ("class_chunks", ctypes.c_int * BATCH_CLASSES),
                ("class_rows", ctypes.c_int * BATCH_CLASSES),
                ("class_threads", ctypes.c_int * BATCH_CLASSES),
                ("streams", ctypes.c_int), ("pair_tiles", ctypes.c_int),
                ("grad_chunks", ctypes.c_int), ("chain_blocks", ctypes.c_int),
                ("ws_bytes", ctypes.c_size_t), ("split_count", ctypes.c_int),
                ("split_chunks", ctypes.c_int), ("tables_key", ctypes.c_uint64),
                ("class_tree", ctypes.c_int * BATCH_CLASSES),
                ("class_vertices", ctypes.c_int * BATCH_CLASSES),
                ("split_vertices", ctypes.c_int),
                ("persistent", ctypes.c_int),
                ("persist_items", ctypes.c_int),
                ("stagger", ctypes.c_int)]

_lib = None


class APPDError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().appd_error_string(code).decode()
        super().__init__("%s: %s (code %d)" % (what, msg, code))
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libappd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libappd.so is not built (%s); run __graft_entry__.build()"
                               % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = res
        _lib = l
    return _lib


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _check(rc: int, what: str):
    if rc != APPD_OK:
        raise APPDError(rc, what)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_tensor(t, name: str, dtype, numel: int, device: torch.device):
    """Every tensor handed to the library: a contiguous tensor of the given dtype
    and element count on the given device (the library trusts these)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.numel() != numel:
        raise ValueError("%s must have %d elements, got %d" % (name, numel, t.numel()))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _check_out(out, n2: int, device: torch.device):
    if out is None:
        return (torch.empty(n2, dtype=torch.float32, device=device),
                torch.empty(n2, dtype=torch.int32, device=device))
    M, idx = out
    _check_tensor(M, "out M", torch.float32, n2, device)
    _check_tensor(idx, "out idx", torch.int32, n2, device)
    return M, idx


def _check_workspace(ws, need: int, device: torch.device):
    if not isinstance(ws, torch.Tensor) or not ws.is_cuda or ws.device != device:
        raise ValueError("workspace must be a CUDA tensor on %s" % device)
    if not ws.is_contiguous() or ws.numel() * ws.element_size() < need:
        raise ValueError("workspace must be contiguous and hold at least %d bytes" % need)
    return ws


def _check_square(W: torch.Tensor):
    if not isinstance(W, torch.Tensor) or not W.is_cuda:
        raise ValueError("W must be a CUDA (HIP) tensor")
    if W.dtype != torch.float32 or W.dim() != 2 or W.shape[0] != W.shape[1]:
        raise ValueError("W must be a square float32 matrix")
    if not W.is_contiguous():
        raise ValueError("W must be contiguous (row-major)")
    n = W.shape[0]
    if n < 1 or n > MAX_N:
        raise ValueError("n must be in [1, %d]" % MAX_N)
    return n


def workspace_bytes(n: int) -> int:
    return int(lib().appd_forward_workspace_bytes(int(n)))


def validate(W: torch.Tensor) -> int:
    """Precondition flags of W (0: symmetric, NaN-free, zero diagonal); an or of
    VALID_NAN, VALID_ASYM and VALID_DIAG.  Synchronises the current stream."""
    n = _check_square(W)
    flags = torch.empty(1, dtype=torch.int32, device=W.device)
    _check(lib().appd_validate(_ptr(W), n, _ptr(flags), _stream(W.device)), "appd_validate")
    return int(flags.item()) & 0xffffffff


def sync(device=None) -> None:
    """Wait for the device's current stream and raise APPDError for what went
    wrong on it asynchronously (appd_sync): a failed kernel, or a forward
    enqueued with APPD_VALIDATE set that read a W with a NaN or an asymmetric
    pair."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    _check(lib().appd_sync(_stream(dev)), "appd_sync")


def _mode(mode: int, tree: str) -> int:
    if tree not in TREE_FLAGS:
        raise ValueError("tree must be one of %s" % sorted(TREE_FLAGS))
    return int(mode) | TREE_FLAGS[tree]


def forward(W: torch.Tensor, mode: int = MINIMAX, return_tree: bool = False, out=None,
            workspace: torch.Tensor = None, tree: str = "auto"):
    """APPD of one graph: (M float32, idx int32[, order int32, parent int32]).

    W: n x n float32 on the GPU, symmetric, zero diagonal, no NaN.
    mode: MINIMAX (Eq. 1-2) or WIDEST (Section 4.2).
    out: optional (M, idx) tensors to write into.
    tree: "auto", "prim" or "boruvka" -- how the spanning tree is found (the
        results are identical).
    """
    n = _check_square(W)
    mode = _mode(mode, tree)
    dev = W.device
    M, idx = _check_out(out, n * n, dev)
    M, idx = M.view(n, n), idx.view(n, n)
    order = parent = None
    if return_tree:
        order = torch.empty(n, dtype=torch.int32, device=dev)
        parent = torch.empty(n, dtype=torch.int32, device=dev)
    nb = workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
    _check_workspace(workspace, nb, dev)
    rc = lib().appd_forward_ex(_ptr(W), n, int(mode), _ptr(M), _ptr(idx), _ptr(order),
                               _ptr(parent), _ptr(workspace), workspace.numel(), _stream(dev))
    _check(rc, "appd_forward_ex")
    if return_tree:
        return M, idx, order, parent
    return M, idx


def write_counts(W: torch.Tensor, mode: int = MINIMAX, tree: str = "auto"):
    """(M, idx, counts): the forward with every output store counted (a check
    that the fill writes each entry once).  counts is n x n int32 holding
    (stores of idx) << 16 | (stores of M); synchronises the device's stream,
    and nothing else may run on the GPU meanwhile."""
    n = _check_square(W)
    mode = _mode(mode, tree)
    dev = W.device
    M = torch.empty(n, n, dtype=torch.float32, device=dev)
    idx = torch.empty(n, n, dtype=torch.int32, device=dev)
    counts = torch.empty(n, n, dtype=torch.int32, device=dev)
    ws = torch.empty(workspace_bytes(n), dtype=torch.uint8, device=dev)
    _check(lib().appd_debug_write_counts(_ptr(W), n, int(mode), _ptr(M), _ptr(idx), _ptr(counts),
                                         _ptr(ws), ws.numel(), _stream(dev)),
           "appd_debug_write_counts")
    return M, idx, counts


def tree_stats(n: int, workspace: torch.Tensor, mode: int = MINIMAX, tree: str = "auto") -> dict:
    """What the last spanning-tree run in `workspace` did: Boruvka or Prim,
    passes over W (of which `tables` were component-table passes over its
    upper triangle), Boruvka rounds, fallback to Prim."""
    st = (ctypes.c_int32 * 5)()
    _check(lib().appd_tree_stats(int(n), _mode(mode, tree), _ptr(workspace), workspace.numel(),
                                 ctypes.cast(st, ctypes.c_void_p), _stream(workspace.device)),
           "appd_tree_stats")
    return {"boruvka": bool(st[0]), "passes": st[1], "rounds": st[2], "fallback": bool(st[3]),
            "tables": st[4]}


def linkage(W: torch.Tensor, mode: int = MINIMAX, tree: str = "auto",
            workspace: torch.Tensor = None) -> torch.Tensor:
    """Single-linkage dendrogram of one graph: (n-1) x 4 float64 rows
    (cluster a < b, weight, size); ids >= n are earlier merges."""
    n = _check_square(W)
    mode = _mode(mode, tree)
    Z = torch.empty((max(n - 1, 0), 4), dtype=torch.float64, device=W.device)
    if workspace is None:
        workspace = torch.empty(workspace_bytes(n), dtype=torch.uint8, device=W.device)
    _check_workspace(workspace, workspace_bytes(n), W.device)
    _check(lib().appd_linkage(_ptr(W), n, int(mode), _ptr(Z) if n > 1 else None,
                              _ptr(workspace), workspace.numel(), _stream(W.device)),
           "appd_linkage")
    return Z


def tree(W: torch.Tensor, workspace: torch.Tensor, mode: int = MINIMAX, tree: str = "auto"):
    """Phase 1 only: spanning tree and attachment order into `workspace`."""
    n = _check_square(W)
    _check_workspace(workspace, workspace_bytes(n), W.device)
    _check(lib().appd_tree(_ptr(W), n, _mode(mode, tree), None, None, _ptr(workspace),
                           workspace.numel(), _stream(W.device)), "appd_tree")


def fill(n: int, workspace: torch.Tensor, M: torch.Tensor, idx: torch.Tensor,
         mode: int = MINIMAX):
    """Phase 2 only: M and idx from the tree `tree()` left in `workspace`."""
    _check_workspace(workspace, workspace_bytes(n), workspace.device)
    _check_tensor(M, "M", torch.float32, n * n, workspace.device)
    _check_tensor(idx, "idx", torch.int32, n * n, workspace.device)
    _check(lib().appd_fill(int(n), int(mode), _ptr(workspace), workspace.numel(), _ptr(M),
                           _ptr(idx), _stream(M.device)), "appd_fill")


# ------------------------------------------------------------------ batches
class Batch:
    """A prepared batch of independent graphs with sizes `ns` (host ints).

    Packed layout (graph-id order): graph g's n_g x n_g matrices start at
    ``offsets[g] = sum_{h<g} n_h^2`` elements, its per-vertex arrays at
    ``noff[g] = sum_{h<g} n_h`` and its points (n_g x d) at ``d * noff[g]``.
    """

    def __init__(self, ns, device="cuda:0"):
        self.ns = np.ascontiguousarray(ns, dtype=np.int32)
        if self.ns.ndim != 1 or len(self.ns) < 1:
            raise ValueError("ns must be a non-empty 1-D sequence")
        if (self.ns < 1).any() or (self.ns > BATCH_MAX_N).any():
            raise ValueError("every n must be in [1, %d]" % BATCH_MAX_N)
        self.device = torch.device(device)
        self.G = len(self.ns)
        sq = self.ns.astype(np.int64) ** 2
        self.offsets = np.concatenate([[0], np.cumsum(sq)[:-1]]).astype(np.int64)
        self.noff = np.concatenate([[0], np.cumsum(self.ns.astype(np.int64))[:-1]]).astype(np.int64)
        self.total_nn = int(sq.sum())
        self.total_n = int(self.ns.astype(np.int64).sum())
        nbytes = int(lib().appd_batch_workspace_bytes(self.ns.ctypes.data_as(_P), self.G))
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.plan = BatchPlan()
        _check(lib().appd_batch_prepare(self.ns.ctypes.data_as(_P), self.G, _ptr(self.ws), nbytes,
                                        ctypes.byref(self.plan), _stream(self.device)),
               "appd_batch_prepare")

    def autotune(self, W: torch.Tensor, out=None) -> float:
        """Time the candidate schedules on this batch's W (median of 5 forwards
        each) and keep the fastest; returns its milliseconds per forward.  With
        APPD_TUNE_CACHE naming a JSON file, a schedule kept there for this GPU
        and class histogram is taken without timing, and a new one is stored.
        Synchronises; not capturable."""
        _check_tensor(W, "W", torch.float32, self.total_nn, self.device)
        M, idx = _check_out(out, self.total_nn, self.device)
        ms = ctypes.c_float()
        _check(lib().appd_batch_autotune(_ptr(W), _ptr(M), _ptr(idx), ctypes.byref(self.plan),
                                         _ptr(self.ws), _stream(self.device), ctypes.byref(ms)),
               "appd_batch_autotune")
        return ms.value

    def set_schedule(self, threads=None, rows=None, streams=None, split_count=None, trees=None,
                     persistent=None, stagger=None):
        """Set the schedule by hand (Prim workgroup size and fill rows per item of
        each class, streams, and how many of the largest class's biggest graphs
        run on their own, -1 for a cut into halves of equal work; persistent:
        the whole forward as one launch over a work queue; stagger: the other
        classes start after the largest class's candidate-list pass); rebuilds
        the device work tables.  Synchronises."""
        p = self.plan
        for c in range(BATCH_CLASSES):
            if threads is not None:
                p.class_threads[c] = int(threads[c] if hasattr(threads, "__len__") else threads)
            if rows is not None:
                p.class_rows[c] = int(rows[c] if hasattr(rows, "__len__") else rows)
            if trees is not None:  # "prim" / "boruvka" per class, or one for all
                tr = trees[c] if isinstance(trees, (list, tuple)) else trees
                p.class_tree[c] = BATCH_TREES[tr]
        if streams is not None:
            p.streams = int(streams)
        if split_count is not None:
            p.split_count = int(split_count)
        if persistent is not None:
            p.persistent = int(bool(persistent))
        if stagger is not None:
            p.stagger = int(bool(stagger))
        _check(lib().appd_batch_set_schedule(ctypes.byref(p), _ptr(self.ws), _stream(self.device)),
               "appd_batch_set_schedule")

    def tree_stats(self) -> dict:
        """How the last forward found each graph's tree: counts of graphs by
        Prim / Boruvka, the passes over W and rounds they took, fallbacks."""
        st = np.empty(self.G, np.int32)
        _check(lib().appd_batch_tree_stats(ctypes.byref(self.plan), _ptr(self.ws),
                                           st.ctypes.data_as(_P), _stream(self.device)),
               "appd_batch_tree_stats")
        b = st[st >= 0]
        return {"prim": int((st < 0).sum()), "boruvka": int(len(b)),
                "fallback": int(((b >> 16) & 1).sum()),
                "passes_max": int(((b >> 8) & 0xff).max()) if len(b) else 0,
                "multi_pass": int((((b >> 8) & 0xff) > 1).sum()),
                "rounds_max": int((b & 0xff).max()) if len(b) else 0,
                "rounds_mean": float((b & 0xff).mean()) if len(b) else 0.0}

    def schedule(self) -> dict:
        """The plan's per-class schedule (classes n <= 64 .. 2048); split_count:
        graphs of the largest class launched on their own (0: not cut)."""
        p = self.plan
        names = {v: k for k, v in BATCH_TREES.items()}
        return {"class_count": list(p.class_count), "class_threads": list(p.class_threads),
                "class_rows": list(p.class_rows), "streams": p.streams,
                "split_count": p.split_count,
                "class_tree": [names.get(x, x) for x in p.class_tree],
                "persistent": int(p.persistent), "stagger": int(p.stagger)}

    def forward(self, W: torch.Tensor, mode: int = MINIMAX, return_parent: bool = False,
                out=None):
        """Packed (M, idx[, parent]) of every graph of the batch."""
        _check_tensor(W, "W", torch.float32, self.total_nn, self.device)
        M, idx = _check_out(out, self.total_nn, self.device)
        parent = torch.empty(self.total_n, dtype=torch.int32, device=self.device) \
            if return_parent else None
        _check(lib().appd_forward_batched(_ptr(W), int(mode), _ptr(M), _ptr(idx), _ptr(parent),
                                          ctypes.byref(self.plan), _ptr(self.ws),
                                          _stream(self.device)), "appd_forward_batched")
        return (M, idx, parent) if return_parent else (M, idx)

    def write_counts(self, W: torch.Tensor, mode: int = MINIMAX):
        """Packed (M, idx, counts): the batched forward with every output store
        counted, as write_counts() for one graph."""
        _check_tensor(W, "W", torch.float32, self.total_nn, self.device)
        M = torch.empty(self.total_nn, dtype=torch.float32, device=self.device)
        idx = torch.empty(self.total_nn, dtype=torch.int32, device=self.device)
        counts = torch.empty(self.total_nn, dtype=torch.int32, device=self.device)
        _check(lib().appd_debug_write_counts_batched(_ptr(W), int(mode), _ptr(M), _ptr(idx),
                                                     _ptr(counts), ctypes.byref(self.plan),
                                                     _ptr(self.ws), _stream(self.device)),
               "appd_debug_write_counts_batched")
        return M, idx, counts

    def pairwise(self, X: torch.Tensor, d: int, out: torch.Tensor = None) -> torch.Tensor:
        """Packed Euclidean W of the batch's point sets (X: total_n x d float32)."""
        _check_tensor(X, "X", torch.float32, self.total_n * d, self.device)
        W = out if out is not None else torch.empty(self.total_nn, dtype=torch.float32,
                                                     device=self.device)
        _check_tensor(W, "out W", torch.float32, self.total_nn, self.device)
        _check(lib().appd_pairwise_euclidean_batched(_ptr(X), int(d), _ptr(W),
                                                     ctypes.byref(self.plan), _ptr(self.ws),
                                                     _stream(self.device)),
               "appd_pairwise_euclidean_batched")
        return W

    def _check_grad_args(self, G, idx, parent):
        _check_tensor(G, "G", torch.float32, self.total_nn, self.device)
        _check_tensor(idx, "idx", torch.int32, self.total_nn, self.device)
        _check_tensor(parent, "parent", torch.int32, self.total_n, self.device)

    def backward_points(self, X, d, W, G, idx, parent) -> torch.Tensor:
        _check_tensor(X, "X", torch.float32, self.total_n * d, self.device)
        _check_tensor(W, "W", torch.float32, self.total_nn, self.device)
        self._check_grad_args(G, idx, parent)
        dX = torch.empty(self.total_n * d, dtype=torch.float32, device=self.device)
        _check(lib().appd_backward_points_batched(_ptr(X), int(d), _ptr(W), _ptr(G), _ptr(idx),
                                                  _ptr(parent), _ptr(dX), ctypes.byref(self.plan),
                                                  _ptr(self.ws), _stream(self.device)),
               "appd_backward_points_batched")
        return dX

    def backward_w(self, G, idx, parent) -> torch.Tensor:
        """Packed dL/dW for L = sum G_ij M_ij: G_ij onto the upper-triangle entry
        of each pair's bottleneck edge, per graph."""
        self._check_grad_args(G, idx, parent)
        dW = torch.empty(self.total_nn, dtype=torch.float32, device=self.device)
        _check(lib().appd_backward_w_batched(_ptr(G), _ptr(idx), _ptr(parent), _ptr(dW),
                                             ctypes.byref(self.plan), _ptr(self.ws),
                                             _stream(self.device)), "appd_backward_w_batched")
        return dW


# ------------------------------------------------------------------ points, gradients
def _grad_ws(n, dev):
    return torch.empty(int(lib().appd_grad_workspace_bytes(int(n))), dtype=torch.uint8, device=dev)


def pairwise_euclidean(X: torch.Tensor) -> torch.Tensor:
    """W_ij = ||x_i - x_j||, float32, summed in increasing coordinate order."""
    if X.dtype != torch.float32 or X.dim() != 2 or not X.is_cuda or not X.is_contiguous():
        raise ValueError("X must be a contiguous float32 CUDA matrix")
    n, d = X.shape
    W = torch.empty((n, n), dtype=torch.float32, device=X.device)
    ws = _grad_ws(n, X.device)
    _check(lib().appd_pairwise_euclidean(_ptr(X), n, d, _ptr(W), _ptr(ws), ws.numel(),
                                         _stream(X.device)), "appd_pairwise_euclidean")
    return W


def _check_single_grad(G, idx, parent, n, dev):
    if n < 1 or n > GRAD_MAX_N:
        raise ValueError("n must be in [1, %d] for the backward" % GRAD_MAX_N)
    _check_tensor(G, "G", torch.float32, n * n, dev)
    _check_tensor(idx, "idx", torch.int32, n * n, dev)
    _check_tensor(parent, "parent", torch.int32, n, dev)


def backward_points(X, W, G, idx, parent) -> torch.Tensor:
    if X.dim() != 2:
        raise ValueError("X must be n x d")
    n, d = X.shape
    _check_tensor(X, "X", torch.float32, n * d, X.device)
    _check_tensor(W, "W", torch.float32, n * n, X.device)
    _check_single_grad(G, idx, parent, n, X.device)
    dX = torch.empty((n, d), dtype=torch.float32, device=X.device)
    ws = _grad_ws(n, X.device)
    _check(lib().appd_backward_points(_ptr(X), n, d, _ptr(W), _ptr(G), _ptr(idx), _ptr(parent),
                                      _ptr(dX), _ptr(ws), ws.numel(), _stream(X.device)),
           "appd_backward_points")
    return dX


def backward_w(G, idx, parent) -> torch.Tensor:
    n = G.shape[0]
    _check_single_grad(G, idx, parent, n, G.device)
    dW = torch.empty((n, n), dtype=torch.float32, device=G.device)
    ws = _grad_ws(n, G.device)
    _check(lib().appd_backward_w(_ptr(G), _ptr(idx), _ptr(parent), n, _ptr(dW), _ptr(ws),
                                 ws.numel(), _stream(G.device)), "appd_backward_w")
    return dW


class APPDPoints(torch.autograd.Function):
    """M = APPD(||x_i - x_j||) for one point set; idx is returned, not differentiated."""

    @staticmethod
    def forward(ctx, X):
        X = X.contiguous()
        W = pairwise_euclidean(X)
        M, idx, _, parent = forward(W, return_tree=True)
        ctx.save_for_backward(X, W, idx, parent)
        ctx.mark_non_differentiable(idx)
        return M, idx

    @staticmethod
    def backward(ctx, gM, gidx):
        X, W, idx, parent = ctx.saved_tensors
        return backward_points(X, W, gM.contiguous(), idx, parent)


class APPDWeights(torch.autograd.Function):
    """M = APPD(W) for a weight matrix; the gradient goes to the upper-triangle
    entry of each pair's bottleneck edge."""

    @staticmethod
    def forward(ctx, W):
        W = W.contiguous()
        M, idx, _, parent = forward(W, return_tree=True)
        ctx.save_for_backward(idx, parent)
        ctx.mark_non_differentiable(idx)
        return M, idx

    @staticmethod
    def backward(ctx, gM, gidx):
        idx, parent = ctx.saved_tensors
        return backward_w(gM.contiguous(), idx, parent)


class APPDPointsBatched(torch.autograd.Function):
    """Packed M of a batch of point sets (X: total_n x d float32, packed)."""

    @staticmethod
    def forward(ctx, X, batch, d):
        X = X.contiguous()
        W = batch.pairwise(X, d)
        M, idx, parent = batch.forward(W, return_parent=True)
        ctx.save_for_backward(X, W, idx, parent)
        ctx.batch = batch
        ctx.d = d
        ctx.mark_non_differentiable(idx)
        return M, idx

    @staticmethod
    def backward(ctx, gM, gidx):
        X, W, idx, parent = ctx.saved_tensors
        dX = ctx.batch.backward_points(X, ctx.d, W, gM.contiguous(), idx, parent)
        return dX.view_as(X), None, None


def appd_points(X: torch.Tensor):
    """Differentiable APPD of a point set: (M, idx)."""
    return APPDPoints.apply(X)


def appd_points_batched(X: torch.Tensor, batch: Batch, d: int):
    return APPDPointsBatched.apply(X, batch, d)


class LaunchTimer:
    """HIP events around every launch of one library kernel (appd_timer_*).

    `kernel` is the kernel's base name ("fill_kernel", "tree_rounds_kernel", ...)
    or "*" for all of them; the events are created here, so the region being
    timed only records them.  read() waits for them."""

    def __init__(self, kernel: str = "*", capacity: int = 4096):
        _check(lib().appd_timer_start(kernel.encode(), capacity), "appd_timer_start")
        self.kernel = kernel

    def read(self, kernel: str = None):
        """(launches, total milliseconds, overflowed) of `kernel` (default: the
        timed kernel)."""
        k = (kernel or self.kernel).encode()
        cnt, tot, ovf = ctypes.c_int(), ctypes.c_double(), ctypes.c_int()
        _check(lib().appd_timer_read(k, ctypes.byref(cnt), ctypes.byref(tot), ctypes.byref(ovf)),
               "appd_timer_read")
        return cnt.value, tot.value, bool(ovf.value)

    def names(self):
        n = lib().appd_timer_names(None, 0)
        arr = (ctypes.c_char_p * max(n, 1))()
        lib().appd_timer_names(ctypes.cast(arr, ctypes.c_void_p), n)
        return [arr[i].decode() for i in range(n)]

    def close(self):
        _check(lib().appd_timer_start(None, 0), "appd_timer_start")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

