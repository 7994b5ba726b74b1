"""Per-image parameter choice for the inpainting solver, with a JSON cache.

The measurement itself runs in the library (hdi_autotune: one inpainting solve
per candidate, timed with HIP events on the device). This module only builds
the candidate grid, keys the cache by (width bucket, height bucket, channels,
density bucket) and reads/writes the JSON file. Parameters are chosen per image,
so a batch of uneven images carries one parameter set per image.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import torch

from . import _lib
from . import SolveParams, _check_inputs, _img, _ptr, _stream_ptr, workspace
from ._lib import check

OVERLAPS = (4, 6)
LOCAL_ITERS = (8, 10, 12, 14)
COARSE_ITERS = (32, 64)
SMALL_FROM = (0, -1)          # 16x16 blocks on the coarse levels: automatic rule, or none
ROBIN = (-1.0, 0.6)           # Dirichlet block boundaries, or the Robin condition with weight 0.6
LOCAL_STOP = (0.0, 1e-7)      # fixed local CG steps, or the global-relative stop


def candidates():
    return [SolveParams(overlap=o, local_iters=k, coarse_iters=c, small_from=t, robin=w, local_stop=q)
            for o in OVERLAPS for k in LOCAL_ITERS for c in COARSE_ITERS for t in SMALL_FROM for w in ROBIN
            for q in LOCAL_STOP]


def bucket(shape, density: float) -> str:
    C, H, W = shape
    wb = 2 ** round(math.log2(max(W, 1)))
    hb = 2 ** round(math.log2(max(H, 1)))
    db = round(math.log2(max(density, 1e-4)) * 2) / 2
    return f"{wb}x{hb}x{C}@{db:+.1f}"


class Autotuner:
    def __init__(self, path: str | None = None, reps: int = 2):
        self.path = path
        self.reps = reps
        self.cache = {}
        if path and os.path.exists(path):
            with open(path) as fh:
                self.cache = json.load(fh)

    def params_for(self, f: torch.Tensor, mask: torch.Tensor) -> SolveParams:
        """Cached parameters for this image's bucket, tuned on this image if absent."""
        _check_inputs(f, mask)
        key = bucket(tuple(f.shape), float(mask.float().mean()))
        if key not in self.cache:
            self.cache[key] = self.tune(f, mask)
            if self.path:
                with open(self.path, "w") as fh:
                    json.dump(self.cache, fh, indent=1, sort_keys=True)
        return SolveParams(**self.cache[key]["params"])

    def tune(self, f: torch.Tensor, mask: torch.Tensor) -> dict:
        L = _lib.lib()
        img = _img(f.shape)
        cands = candidates()
        arr = (_lib.hdi_solve_params * len(cands))(*[c.c() for c in cands])
        need = L.hdi_inpaint_workspace_bytes(img) + f.numel() * 8 + 512
        ws = workspace(need, f.device)
        best, ms = ctypes.c_int32(-1), ctypes.c_float(0.0)
        st = L.hdi_autotune(img, _ptr(mask), _ptr(f), _ptr(ws), ws.numel(), arr, len(cands), self.reps,
                            ctypes.byref(best), ctypes.byref(ms), _stream_ptr(f.device))
        check(st)
        p = cands[best.value]
        return {"params": {"overlap": p.overlap, "local_iters": p.local_iters, "coarse_iters": p.coarse_iters,
                           "small_from": p.small_from, "robin": p.robin, "local_stop": p.local_stop},
                "ms": float(ms.value)}
