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

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libappd.so")

MINIMAX = 0
WIDEST = 1
MAX_N = 46340

APPD_OK = 0
APPD_EINVAL = -1
APPD_EHIP = -2
APPD_ENOMEM = -3

# every symbol include/appd.h declares, with its ctypes signature
_P = ctypes.c_void_p
_I = ctypes.c_int
_SZ = ctypes.c_size_t
SIGNATURES = {
    "appd_error_string": ([_I], ctypes.c_char_p),
    "appd_get_last_error": ([], _I),
    "appd_forward_workspace_bytes": ([_I], _SZ),
    "appd_forward": ([_P, _I, _P, _P, _P], _I),
    "appd_forward_ws": ([_P, _I, _P, _P, _P, _SZ, _P], _I),
    "appd_forward_ex": ([_P, _I, _I, _P, _P, _P, _P, _P, _SZ, _P], _I),
}

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


def forward(W: torch.Tensor, mode: int = MINIMAX, return_tree: bool = False, out=None,
            workspace: torch.Tensor = None):
    """APPD of one graph: (M float32, idx int32[, order int32, parent int32]).

    W: n x n float32 on the GPU, symmetric, zero diagonal, no NaN.
    mode: MINIMAX (Eq. 1-2) or WIDEST (Section 4.2).
    out: optional (M, idx) tensors to write into.
    """
    n = _check_square(W)
    dev = W.device
    if out is None:
        M = torch.empty((n, n), dtype=torch.float32, device=dev)
        idx = torch.empty((n, n), dtype=torch.int32, device=dev)
    else:
        M, idx = out
    order = parent = None
    if return_tree:
        order = torch.empty(n, dtype=torch.int32, device=dev)
        parent = torch.empty(n, dtype=torch.int32, device=dev)
    nb = workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(nb, dtype=torch.uint8, device=dev)
    rc = lib().appd_forward_ex(_ptr(W), n, int(mode), _ptr(M), _ptr(idx), _ptr(order),
                               _ptr(parent), _ptr(workspace), workspace.numel(), _stream(dev))
    _check(rc, "appd_forward_ex")
    if return_tree:
        return M, idx, order, parent
    return M, idx
