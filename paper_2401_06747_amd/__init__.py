"""Python binding of libhdi (argument marshalling only).

Every step of the solve runs in the HIP kernels of libhdi.so; this module only
checks tensor shapes, allocates the workspace through torch, and passes device
pointers and the current HIP stream across the C ABI declared in include/hdi.h.
If libhdi.so is missing, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import HdiError, check

__all__ = ["inpaint_solve", "hdi_block_count", "SolveParams", "HdiError"]


@dataclass
class SolveParams:
    rel_tol: float = 0.0       # 0 -> 1e-6
    max_outer: int = 0         # 0 -> 40
    overlap: int = 0           # 0 -> 4
    local_iters: int = 0       # 0 -> 8
    coarse_iters: int = 0      # 0 -> 64
    flags: int = 0

    def c(self):
        return _lib.hdi_solve_params(self.rel_tol, self.max_outer, self.overlap, self.local_iters,
                                     self.coarse_iters, self.flags)


def _stream_ptr(dev) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _img(shape) -> _lib.hdi_image:
    C, H, W = shape
    return _lib.hdi_image(W, H, C)


def _check_inputs(f: torch.Tensor, mask: torch.Tensor):
    if f.dim() != 3 or mask.dim() != 2 or tuple(f.shape[1:]) != tuple(mask.shape):
        raise ValueError(f"need f (C,H,W) and mask (H,W); got {tuple(f.shape)} and {tuple(mask.shape)}")
    if not (f.is_cuda and mask.is_cuda) or f.device != mask.device:
        raise ValueError("f and mask must be on the same GPU")
    if f.dtype != torch.float32 or mask.dtype != torch.uint8:
        raise ValueError("f must be float32 and mask uint8")
    if not (f.is_contiguous() and mask.is_contiguous()):
        raise ValueError("f and mask must be contiguous")


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def inpaint_solve(f: torch.Tensor, mask: torch.Tensor, u0: torch.Tensor | None = None,
                  params: SolveParams | None = None, ws: torch.Tensor | None = None,
                  out: torch.Tensor | None = None):
    """u = A^{-1} C f per channel (eq. inp-discrete-lsi). Returns (u float64, report dict)."""
    _check_inputs(f, mask)
    L = _lib.lib()
    img = _img(f.shape)
    need = L.hdi_inpaint_workspace_bytes(img)
    if ws is None:
        ws = workspace(need, f.device)
    u = out if out is not None else torch.empty(f.shape, dtype=torch.float64, device=f.device)
    if u0 is not None and (u0.shape != f.shape or u0.dtype != torch.float64 or not u0.is_contiguous()):
        raise ValueError("u0 must be a contiguous float64 tensor shaped like f")
    rep = _lib.hdi_solve_report()
    p = (params or SolveParams()).c()
    st = L.inpaint_solve(img, _ptr(mask), _ptr(f), _ptr(u), _ptr(u0), _ptr(ws), ws.numel(),
                         ctypes.byref(p), ctypes.byref(rep), _stream_ptr(f.device))
    report = {"status": st, "rel_residual": list(rep.rel_residual)[:f.shape[0]],
              "outer_iters": rep.outer_iters, "vcycles": rep.vcycles, "ms": rep.ms}
    if st not in (_lib.HDI_OK, _lib.HDI_ERR_NO_CONVERGENCE):
        check(st)
    return u, report


def hdi_block_count(width: int, height: int, overlap: int) -> int:
    return int(_lib.lib().hdi_block_count(width, height, overlap))
