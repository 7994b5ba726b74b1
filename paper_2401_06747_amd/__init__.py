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

__all__ = ["inpaint_solve", "inpaint_solve_noalloc", "solve_batch", "tonal_optimize", "densify_step", "error_map", "initial_mask",
           "spatial_optimize", "Server", "DELAUNAY", "VORONOI",
           "INPAINT", "TONAL", "hdi_block_count", "SolveParams", "TonalParams", "HdiError", "PCG_RAS", "RAS", "CGNR",
           "FLAG_NO_FMG", "FLAG_CG", "voronoi_init", "VINIT_DIRECT", "VINIT_VORONOI", "VINIT_VORONOI_LOG",
           "voronoi_labels", "JFA"]

PCG_RAS, RAS, CGNR = _lib.HDI_TONAL_PCG_RAS, _lib.HDI_TONAL_RAS, _lib.HDI_TONAL_CGNR
# solve flags: cold start without the FMG initial guess; plain FP64 CG instead of multigrid (comparator)
FLAG_NO_FMG, FLAG_CG = _lib.HDI_FLAG_NO_FMG, _lib.HDI_FLAG_CG
DELAUNAY, VORONOI = _lib.HDI_PART_DELAUNAY, _lib.HDI_PART_VORONOI
JFA = _lib.HDI_PART_JFA   # or'ed into a partition: jump-flooding labels (Sec. 4.2)
VINIT_DIRECT, VINIT_VORONOI, VINIT_VORONOI_LOG = (_lib.HDI_VINIT_DIRECT, _lib.HDI_VINIT_VORONOI,
                                                  _lib.HDI_VINIT_VORONOI_LOG)


@dataclass
class SolveParams:
    rel_tol: float = 0.0       # 0 -> 1e-6
    max_outer: int = 0         # 0 -> 40
    overlap: int = 0           # 0 -> 6
    local_iters: int = 0       # 0 -> 12
    coarse_iters: int = 0      # 0 -> 64
    flags: int = 0
    small_from: int = 0        # first level with 16x16 blocks: 0 automatic, -1 none, k level k
    robin: float = 0.0         # Robin weight at inner block boundaries (0 -> 0.6, < 0: Dirichlet), up to 0.9
    local_stop: float = 0.0    # > 0: finest-level local CG stops at this fraction of the global squared residual
    mid_iters: int = 0         # local CG steps on the levels between finest and coarsest (0 -> 8)

    def c(self):
        return _lib.hdi_solve_params(self.rel_tol, self.max_outer, self.overlap, self.local_iters,
                                     self.coarse_iters, self.flags, self.small_from, self.robin, self.local_stop,
                                     self.mid_iters)


@dataclass
class TonalParams:
    rel_tol: float = 0.0       # 0 -> 1e-6
    max_outer: int = 0         # 0 -> 500
    mode: int = 0              # PCG_RAS, RAS or CGNR
    overlap: int = 0           # 0 -> 16 (64x64 blocks) or 14 (32x32)
    local_outer: int = 0       # 0 -> 5 (64x64 blocks) or 3 (32x32)
    local_inner: int = 0       # 0 -> 20 (64x64 blocks) or 24 (32x32)
    flags: int = 0
    inner: SolveParams | None = None
    mse_gain: float = 0.0      # > 0: also stop when an iteration lowers the MSE by less than this fraction
    block: int = 0             # RAS block edge: 0 -> 64, or 32

    def c(self):
        return _lib.hdi_tonal_params(self.rel_tol, self.max_outer, self.mode, self.overlap, self.local_outer,
                                     self.local_inner, self.flags, (self.inner or SolveParams()).c(), self.mse_gain,
                                     self.block)


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
    if st != _lib.HDI_OK:
        report["message"] = L.hdi_last_error().decode()
    if st not in (_lib.HDI_OK, _lib.HDI_ERR_NO_CONVERGENCE):
        check(st)
    return u, report


def inpaint_solve_noalloc(f: torch.Tensor, mask: torch.Tensor, u0: torch.Tensor | None = None,
                          params: SolveParams | None = None, out: torch.Tensor | None = None):
    """inpaint_solve on the library's own fixed scratch array (no workspace and
    no allocation inside the call; images up to hdi_noalloc_scratch_bytes of
    workspace). Returns (u float64, report dict)."""
    _check_inputs(f, mask)
    L = _lib.lib()
    img = _img(f.shape)
    u = out if out is not None else torch.empty(f.shape, dtype=torch.float64, device=f.device)
    if u.shape != f.shape or u.dtype != torch.float64 or not u.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor shaped like f")
    if u0 is not None and (u0.shape != f.shape or u0.dtype != torch.float64 or not u0.is_contiguous()):
        raise ValueError("u0 must be a contiguous float64 tensor shaped like f")
    rep = _lib.hdi_solve_report()
    p = (params or SolveParams()).c()
    st = L.inpaint_solve_noalloc(img, _ptr(mask), _ptr(f), _ptr(u), _ptr(u0), ctypes.byref(p), ctypes.byref(rep),
                                 _stream_ptr(f.device))
    report = {"status": st, "rel_residual": list(rep.rel_residual)[:f.shape[0]],
              "outer_iters": rep.outer_iters, "vcycles": rep.vcycles, "ms": rep.ms}
    if st != _lib.HDI_OK:
        report["message"] = L.hdi_last_error().decode()
    if st not in (_lib.HDI_OK, _lib.HDI_ERR_NO_CONVERGENCE):
        check(st)
    return u, report


def hdi_block_count(width: int, height: int, overlap: int) -> int:
    return int(_lib.lib().hdi_block_count(width, height, overlap))


def lds_calibrate(device="cuda:0", iters: int = 4096) -> float:
    """Measured LDS bandwidth of `device` in bytes/s (hdi_lds_calibrate)."""
    sink = torch.empty(1, dtype=torch.float32, device=device)
    out = ctypes.c_double()
    check(_lib.lib().hdi_lds_calibrate(iters, _ptr(sink), ctypes.byref(out), _stream_ptr(sink.device)))
    return out.value


def tonal_optimize(f: torch.Tensor, mask: torch.Tensor, g0: torch.Tensor | None = None,
                   params: TonalParams | None = None, ws: torch.Tensor | None = None,
                   want_u: bool = False, out: torch.Tensor | None = None):
    """Optimal values on the mask (eq. tonal-opt-minimisation). Starts from f on
    the mask unless g0 is given. Returns (g float64, report dict[, u = B g])."""
    _check_inputs(f, mask)
    L = _lib.lib()
    img = _img(f.shape)
    p = params or TonalParams()
    if g0 is None:
        p = TonalParams(**{**p.__dict__, "flags": p.flags | _lib.HDI_TONAL_INIT_FROM_F})
        g = out if out is not None else torch.empty(f.shape, dtype=torch.float64, device=f.device)
    else:
        if g0.shape != f.shape or g0.dtype != torch.float64:
            raise ValueError("g0 must be float64 shaped like f")
        g = g0.clone() if out is None else out.copy_(g0)
    if ws is None:
        ws = workspace(L.hdi_tonal_workspace_bytes(img), f.device)
    u = torch.empty(f.shape, dtype=torch.float64, device=f.device) if want_u else None
    rep = _lib.hdi_tonal_report()
    pc = p.c()
    st = L.tonal_optimize(img, _ptr(mask), _ptr(f), _ptr(g), _ptr(u), _ptr(ws), ws.numel(), ctypes.byref(pc),
                          ctypes.byref(rep), _stream_ptr(f.device))
    report = {"status": st, "mse_initial": rep.mse_initial, "mse_final": rep.mse_final,
              "rel_normal_residual": rep.rel_normal_residual, "outer_iters": rep.outer_iters,
              "inner_solves": rep.inner_solves, "inner_vcycles": rep.inner_vcycles, "ms": rep.ms}
    if st != _lib.HDI_OK:
        report["message"] = L.hdi_last_error().decode()
    if st not in (_lib.HDI_OK, _lib.HDI_ERR_NO_CONVERGENCE):
        check(st)
    return (g, report, u) if want_u else (g, report)


def voronoi_init(f: torch.Tensor, mask: torch.Tensor, weighting: int = VINIT_VORONOI_LOG, max_iters: int = 20,
                 tau: float = 1.0, stop: bool = True, g0: torch.Tensor | None = None,
                 solve: SolveParams | None = None, ws: torch.Tensor | None = None, want_u: bool = False):
    """Starting values for tonal optimisation (Sec. 5.3): Richardson steps on
    C W B g = C W f from g = f (or g0) on the mask, keeping the best iterate.
    Returns (g float64 with zeros off the mask, report dict[, u = B g])."""
    _check_inputs(f, mask)
    L = _lib.lib()
    img = _img(f.shape)
    flags = 0 if stop else _lib.HDI_VINIT_NO_STOP
    if g0 is None:
        flags |= _lib.HDI_VINIT_FROM_F
        g = torch.empty(f.shape, dtype=torch.float64, device=f.device)
    else:
        if g0.shape != f.shape or g0.dtype != torch.float64:
            raise ValueError("g0 must be float64 shaped like f")
        g = g0.clone()
    if ws is None:
        ws = workspace(L.hdi_vinit_workspace_bytes(img), f.device)
    u = torch.empty(f.shape, dtype=torch.float64, device=f.device) if want_u else None
    p = _lib.hdi_vinit_params(weighting, max_iters, tau, flags, (solve or SolveParams()).c())
    rep = _lib.hdi_vinit_report()
    check(L.voronoi_init(img, _ptr(mask), _ptr(f), _ptr(g), _ptr(u), _ptr(ws), ws.numel(), ctypes.byref(p),
                         ctypes.byref(rep), _stream_ptr(f.device)))
    report = {"steps": rep.steps, "best": rep.best, "solves": rep.solves,
              "mse": list(rep.mse)[:min(rep.steps, _lib.HDI_VINIT_TRACE - 1) + 1], "ms": rep.ms}
    return (g, report, u) if want_u else (g, report)


def error_map(u: torch.Tensor, f: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """err = fp32(sum_c (u - f)^2) per pixel (FP64 sum, one rounding)."""
    if u.shape != f.shape or u.dim() != 3 or u.dtype != torch.float64 or f.dtype != torch.float32:
        raise ValueError("need u (C,H,W) float64 and f (C,H,W) float32")
    if not (u.is_cuda and f.is_cuda and u.is_contiguous() and f.is_contiguous()):
        raise ValueError("u and f must be contiguous GPU tensors")
    err = out if out is not None else torch.empty(u.shape[1:], dtype=torch.float32, device=u.device)
    check(_lib.lib().hdi_error_map(_img(u.shape), _ptr(u), _ptr(f), _ptr(err), _stream_ptr(u.device)))
    return err


def initial_mask(f: torch.Tensor, rand: torch.Tensor, n0: int):
    """Laplacian-magnitude random dithering (Sec. 4.2) with the given uniforms
    (H, W) float64. Returns (mask uint8, count)."""
    if f.dim() != 3 or rand.shape != f.shape[1:] or rand.dtype != torch.float64 or f.dtype != torch.float32:
        raise ValueError("need f (C,H,W) float32 and rand (H,W) float64")
    if not (f.is_cuda and rand.is_cuda and f.is_contiguous() and rand.is_contiguous()):
        raise ValueError("f and rand must be contiguous GPU tensors")
    L = _lib.lib()
    img = _img(f.shape)
    mask = torch.empty(f.shape[1:], dtype=torch.uint8, device=f.device)
    ws = workspace(L.hdi_initial_mask_workspace_bytes(img), f.device)
    n = ctypes.c_int64(0)
    check(L.hdi_initial_mask(img, _ptr(f), _ptr(rand), int(n0), _ptr(mask), ctypes.byref(n), _ptr(ws), ws.numel(),
                             _stream_ptr(f.device)))
    return mask, n.value


def spatial_optimize(f: torch.Tensor, rand: torch.Tensor, density: float, n_steps: int = 20, t: float = 1.0,
                     n0: int = 0, partition: int = DELAUNAY, solve: SolveParams | None = None, hook=None,
                     ws: torch.Tensor | None = None):
    """Spatial optimisation (Sec. 4, Alg. 1): Laplacian-dithered initial mask,
    then n_steps of inpainting, error map and densification. hook(step,
    mask_before, err, added) receives numpy copies after each step. Returns
    (mask uint8, u float64, report dict)."""
    import numpy as np
    if f.dim() != 3 or rand.shape != f.shape[1:] or rand.dtype != torch.float64 or f.dtype != torch.float32:
        raise ValueError("need f (C,H,W) float32 and rand (H,W) float64")
    if not (f.is_cuda and rand.is_cuda and f.is_contiguous() and rand.is_contiguous()):
        raise ValueError("f and rand must be contiguous GPU tensors")
    L = _lib.lib()
    img = _img(f.shape)
    C, H, W = f.shape
    mask = torch.empty((H, W), dtype=torch.uint8, device=f.device)
    u = torch.empty(f.shape, dtype=torch.float64, device=f.device)
    if ws is None:
        ws = workspace(L.hdi_spatial_workspace_bytes(img), f.device)
    p = _lib.hdi_spatial_params(float(density), float(t), int(n0), int(n_steps), int(partition),
                                (solve or SolveParams()).c())
    rep = _lib.hdi_spatial_report()
    if hook is not None:
        def _cb(step, m_ptr, e_ptr, a_ptr, n_added, _user):
            m = np.ctypeslib.as_array(m_ptr, shape=(H * W,)).reshape(H, W).copy()
            e = np.ctypeslib.as_array(e_ptr, shape=(H * W,)).reshape(H, W).copy()
            a = np.ctypeslib.as_array(a_ptr, shape=(max(int(n_added), 1),))[:int(n_added)].copy()
            hook(int(step), m, e, a)
        cb = _lib.HDI_STEP_HOOK(_cb)
    else:
        cb = _lib.HDI_STEP_HOOK()
    st = L.spatial_optimize(img, _ptr(f), _ptr(rand), ctypes.byref(p), _ptr(mask), _ptr(u), _ptr(ws), ws.numel(),
                            ctypes.byref(rep), cb, None, _stream_ptr(f.device))
    check(st)
    report = {"initial_count": rep.initial_count, "final_count": rep.final_count, "solve_rounds": rep.solve_rounds,
              "rel_residual": list(rep.rel_residual)[:C], "ms": rep.ms}
    return mask, u, report


def densify_step(mask: torch.Tensor, err: torch.Tensor, n_add: int, partition: int = DELAUNAY,
                 ws: torch.Tensor | None = None):
    """One densification step (Alg. 1). Updates `mask` in place and returns the
    added linear indices (int32, ascending)."""
    if mask.dim() != 2 or err.shape != mask.shape or mask.dtype != torch.uint8 or err.dtype != torch.float32:
        raise ValueError("need mask (H,W) uint8 and err (H,W) float32")
    if not (mask.is_cuda and err.is_cuda and mask.is_contiguous() and err.is_contiguous()):
        raise ValueError("mask and err must be contiguous GPU tensors")
    L = _lib.lib()
    H, W = mask.shape
    if ws is None:
        ws = workspace(L.hdi_densify_workspace_bytes(W, H), mask.device)
    added = torch.empty(max(int(n_add), 1), dtype=torch.int32, device=mask.device)
    n = ctypes.c_int64(0)
    st = L.densify_step(W, H, _ptr(mask), _ptr(err), int(n_add), int(partition), _ptr(added), ctypes.byref(n),
                        _ptr(ws), ws.numel(), _stream_ptr(mask.device))
    check(st)
    return added[:n.value]


def voronoi_labels(mask: torch.Tensor, jfa_step: int = 0, ws: torch.Tensor | None = None):
    """Nearest-mask-pixel labels (int32 linear indices): exact for jfa_step 0,
    jump flooding from the default start for -1 or from a given power of two.
    Returns (labels, largest squared pixel-to-label distance)."""
    if mask.dim() != 2 or mask.dtype != torch.uint8 or not (mask.is_cuda and mask.is_contiguous()):
        raise ValueError("need a contiguous (H,W) uint8 GPU mask")
    L = _lib.lib()
    H, W = mask.shape
    if ws is None:
        ws = workspace(L.hdi_labels_workspace_bytes(W, H), mask.device)
    labels = torch.empty((H, W), dtype=torch.int32, device=mask.device)
    d2 = ctypes.c_uint64(0)
    check(L.hdi_voronoi_labels(W, H, _ptr(mask), _ptr(labels), int(jfa_step), ctypes.byref(d2), _ptr(ws), ws.numel(),
                               _stream_ptr(mask.device)))
    return labels, int(d2.value)


INPAINT, TONAL = _lib.HDI_REQ_INPAINT, _lib.HDI_REQ_TONAL


def solve_batch(fs, masks, params=None, ws: torch.Tensor | None = None, outs=None, kinds=None, tonal_params=None):
    """Inpainting and tonal jobs in shared launches (hdi_solve_batch). kinds:
    None (all INPAINT) or a list of INPAINT / TONAL; params: inpainting
    parameters (one or per job); tonal_params: TonalParams for the tonal jobs
    (one or per job). Returns (list of outputs float64: u or g, list of report
    dicts)."""
    n = len(fs)
    if n == 0 or len(masks) != n:
        raise ValueError("need equally many images and masks")
    for f, m in zip(fs, masks):
        _check_inputs(f, m)
    kinds = list(kinds) if kinds is not None else [INPAINT] * n
    if len(kinds) != n or any(k not in (INPAINT, TONAL) for k in kinds):
        raise ValueError("kinds must list INPAINT or TONAL for every job")
    L = _lib.lib()
    us = outs if outs is not None else [torch.empty(f.shape, dtype=torch.float64, device=f.device) for f in fs]
    tlist = tonal_params if isinstance(tonal_params, (list, tuple)) else [tonal_params] * n
    tps = [t.c() if (k == TONAL and t is not None) else None for k, t in zip(kinds, tlist)]
    treps = [_lib.hdi_tonal_report() if k == TONAL else None for k in kinds]
    jobs = (_lib.hdi_job * n)(*[
        _lib.hdi_job(k, _img(f.shape), m.data_ptr(), f.data_ptr(), u.data_ptr(),
                     ctypes.pointer(tp) if tp is not None else None,
                     ctypes.pointer(tr) if tr is not None else None)
        for k, f, m, u, tp, tr in zip(kinds, fs, masks, us, tps, treps)])
    need = L.hdi_batch_workspace_bytes(n, jobs)
    if ws is None or ws.numel() < need:
        ws = workspace(need, fs[0].device)
    if params is None:
        pc = None
    else:
        plist = params if isinstance(params, (list, tuple)) else [params] * n
        pc = (_lib.hdi_solve_params * n)(*[p.c() for p in plist])
    reps = (_lib.hdi_solve_report * n)()
    st = L.hdi_solve_batch(n, jobs, _ptr(ws), ws.numel(), pc, reps, _stream_ptr(fs[0].device))
    reports = []
    for r, f, k, tr in zip(reps, fs, kinds, treps):
        d = {"status": st, "kind": k, "rel_residual": list(r.rel_residual)[:f.shape[0]],
             "outer_iters": r.outer_iters, "vcycles": r.vcycles, "ms": r.ms}
        if tr is not None:
            d.update(mse_initial=tr.mse_initial, mse_final=tr.mse_final, rel_normal_residual=tr.rel_normal_residual,
                     inner_solves=tr.inner_solves, inner_vcycles=tr.inner_vcycles)
        reports.append(d)
    if st not in (_lib.HDI_OK, _lib.HDI_ERR_NO_CONVERGENCE):
        check(st)
    return us, reports


class Server:
    """Request loop over one GPU (hdi_server_*): continuous batching of
    inpainting requests, tonal requests on worker streams, admission by the
    bytes of a caller-owned arena. `tonal_shared=True` runs the tonal requests'
    inner solves in the engine's shared rounds; `plain=True` runs one request
    at a time through inpaint_solve / tonal_optimize (the control)."""

    def __init__(self, arena_bytes: int, max_slots: int = 64, tonal_workers: int = 3, plain: bool = False,
                 tonal_shared: bool = False, device="cuda:0"):
        L = _lib.lib()
        self.device = torch.device(device)
        self.arena = workspace(arena_bytes, self.device)
        torch.cuda.synchronize(self.device)
        flags = (_lib.HDI_SERVER_PLAIN if plain else 0) | (_lib.HDI_SERVER_TONAL_SHARED if tonal_shared else 0)
        with torch.cuda.device(self.device):
            h = L.hdi_server_create(_ptr(self.arena), self.arena.numel(), int(max_slots), int(tonal_workers), flags)
        if not h:
            raise HdiError(_lib.HDI_ERR_ARG, L.hdi_last_error().decode())
        self._h = ctypes.c_void_p(h)
        self._live = {}

    @staticmethod
    def request_bytes(kind: int, shape) -> int:
        req = _lib.hdi_request(kind, 0, _img(shape))
        return int(_lib.lib().hdi_request_bytes(ctypes.byref(req)))

    def submit(self, kind: int, f: torch.Tensor, mask: torch.Tensor, params=None,
               out: torch.Tensor | None = None) -> int:
        """Queue a request; returns its ticket. The inputs must not change until
        it is done; the output (u or g, float64) is returned by poll()."""
        host = not f.is_cuda
        if host:
            # pinned host tensors: the server copies them in and the result out
            if mask.is_cuda or not (f.is_pinned() and mask.is_pinned()):
                raise ValueError("host requests need pinned f and mask (tensor.pin_memory())")
            if f.dim() != 3 or tuple(f.shape[1:]) != tuple(mask.shape) or f.dtype != torch.float32 \
                    or mask.dtype != torch.uint8 or not (f.is_contiguous() and mask.is_contiguous()):
                raise ValueError("need contiguous f (C,H,W) float32 and mask (H,W) uint8")
            out = out if out is not None else torch.empty(f.shape, dtype=torch.float64, pin_memory=True)
        else:
            _check_inputs(f, mask)
            out = out if out is not None else torch.empty(f.shape, dtype=torch.float64, device=f.device)
        L = _lib.lib()
        solve = (params if isinstance(params, SolveParams) else SolveParams()).c()
        tp = params.c() if isinstance(params, TonalParams) else None
        req = _lib.hdi_request(kind, _lib.HDI_REQ_HOST_IO if host else 0, _img(f.shape), mask.data_ptr(),
                               f.data_ptr(), out.data_ptr(), solve, ctypes.pointer(tp) if tp is not None else None)
        # the inputs were written on torch's stream; the server's streams do not wait for it
        if not host:
            torch.cuda.current_stream(f.device).synchronize()
        ticket = ctypes.c_uint64(0)
        check(L.hdi_server_submit(self._h, ctypes.byref(req), ctypes.byref(ticket)))
        self._live[ticket.value] = (f, mask, out)
        return ticket.value

    def poll(self, ticket: int):
        """None while the request runs; then (output, report dict)."""
        L = _lib.lib()
        done = ctypes.c_int32(0)
        rep = _lib.hdi_request_report()
        check(L.hdi_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(done), ctypes.byref(rep)))
        if not done.value:
            return None
        out = self._live.pop(ticket)[2]
        report = {"status": rep.status, "kind": rep.kind, "outer_iters": rep.outer_iters,
                  "inner_solves": rep.inner_solves, "max_running": rep.max_running,
                  "rel_residual": list(rep.rel_residual), "mse_initial": rep.mse_initial,
                  "mse_final": rep.mse_final, "t_submit_ms": rep.t_submit_ms, "t_start_ms": rep.t_start_ms,
                  "t_done_ms": rep.t_done_ms}
        if rep.status != _lib.HDI_OK:
            report["message"] = L.hdi_last_error().decode()
        return out, report

    def drain(self):
        check(_lib.lib().hdi_server_drain(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().hdi_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()
