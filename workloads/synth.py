"""Seeded synthetic images and masks shared by the oracle tests, the GPU tests and
the benchmark.

This module holds none of the solver's arithmetic: it only draws inputs. The
paper evaluates on twelve 4K nature photographs (Sec. 6.1) that are not
available here; these families stand in for them with the paper's shapes,
densities and structure (smooth regions, sharp edges, fine noise).

Every random draw comes from ``numpy.random.Generator(PCG64(SeedSequence(key)))``
with ``key = [2401, 6747, config, item, stream]``: ``stream`` is the channel
index for image data and ``MASK_STREAM`` for the mask, so that a given
(config, item) reproduces the same bytes everywhere.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

MASK_STREAM = 1000
_HERE = os.path.dirname(os.path.abspath(__file__))
_FS_LIB = os.path.join(_HERE, "_fs_dither.so")


def rng_for(config: int, item: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([2401, 6747, config, item, stream])))


# ---------------------------------------------------------------- images

def _gauss_add(f: np.ndarray, a: float, mx: float, my: float, s: float) -> None:
    """Add a*exp(-|p-mu|^2/(2 s^2)) at pixel centres, inside a +-6 s window."""
    H, W = f.shape
    x0, x1 = max(0, int(mx - 6 * s)), min(W, int(mx + 6 * s) + 1)
    y0, y1 = max(0, int(my - 6 * s)), min(H, int(my + 6 * s) + 1)
    if x0 >= x1 or y0 >= y1:
        return
    gx = np.exp(-((np.arange(x0, x1) + 0.5 - mx) ** 2) / (2 * s * s))
    gy = np.exp(-((np.arange(y0, y1) + 0.5 - my) ** 2) / (2 * s * s))
    f[y0:y1, x0:x1] += a * gy[:, None] * gx[None, :]


def _polygon_add(f: np.ndarray, px: np.ndarray, py: np.ndarray, h: float) -> None:
    """Add h inside a polygon (even-odd rule at pixel centres)."""
    H, W = f.shape
    x0, x1 = max(0, int(np.floor(px.min()))), min(W, int(np.ceil(px.max())) + 1)
    y0, y1 = max(0, int(np.floor(py.min()))), min(H, int(np.ceil(py.max())) + 1)
    if x0 >= x1 or y0 >= y1:
        return
    yy = (np.arange(y0, y1) + 0.5)[:, None]
    xx = (np.arange(x0, x1) + 0.5)[None, :]
    inside = np.zeros((y1 - y0, x1 - x0), dtype=bool)
    n = len(px)
    j = n - 1
    for i in range(n):
        if py[i] != py[j]:
            crosses = (py[i] > yy) != (py[j] > yy)
            xint = (px[j] - px[i]) * (yy - py[i]) / (py[j] - py[i]) + px[i]
            inside ^= crosses & (xx < xint)
        j = i
    f[y0:y1, x0:x1] += h * inside


def bumps_and_rects(H: int, W: int, config: int = 1, item: int = 0) -> np.ndarray:
    """128 + 12 Gaussian bumps + 4 constant rectangles, clipped to [0, 255]
    (the CPU-sized grayscale family). Returned as float32 values held in float64."""
    rng = rng_for(config, item, 0)
    S = min(H, W)
    f = np.full((H, W), 128.0)
    for _ in range(12):
        mx, my = rng.uniform(0, W), rng.uniform(0, H)
        s = rng.uniform(0.04, 0.25) * S
        a = rng.uniform(-90, 90)
        _gauss_add(f, a, mx, my, s)
    for _ in range(4):
        sw, sh = rng.uniform(0.1, 0.4) * W, rng.uniform(0.1, 0.4) * H
        cx, cy = rng.uniform(0, W - sw), rng.uniform(0, H - sh)
        hgt = rng.uniform(-70, 70)
        xs, ys = int(round(cx)), int(round(cy))
        f[ys:int(round(cy + sh)), xs:int(round(cx + sw))] += hgt
    return np.clip(f, 0, 255).astype(np.float32).astype(np.float64)


def textured_channel(H: int, W: int, config: int, item: int, channel: int) -> np.ndarray:
    """One channel of the 4K-style family: 128 + 200 Gaussians + 30 star-shaped
    polygons + uniform noise of standard deviation 2, clipped to [0, 255]."""
    rng = rng_for(config, item, channel)
    S = min(H, W)
    f = np.full((H, W), 128.0)
    for _ in range(200):
        mx, my = rng.uniform(0, W), rng.uniform(0, H)
        s = rng.uniform(0.004, 0.08) * S
        a = rng.uniform(-50, 50)
        _gauss_add(f, a, mx, my, s)
    for _ in range(30):
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        R = rng.uniform(0.01, 0.15) * S
        nv = int(rng.integers(3, 10))
        ang = np.sort(rng.uniform(0, 2 * np.pi, nv))
        rad = R * rng.uniform(0.3, 1.0, nv)
        h = rng.uniform(-60, 60)
        _polygon_add(f, cx + rad * np.cos(ang), cy + rad * np.sin(ang), h)
    f += rng.uniform(-2 * np.sqrt(3), 2 * np.sqrt(3), size=(H, W))
    return np.clip(f, 0, 255)


def textured_image(H: int, W: int, C: int, config: int = 2, item: int = 0) -> np.ndarray:
    """C x H x W planar image, float32 values held in float64."""
    return np.stack([textured_channel(H, W, config, item, c) for c in range(C)]).astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------- masks

def uniform_mask(H: int, W: int, count: int, config: int, item: int = 0) -> np.ndarray:
    """Exactly `count` known pixels, uniform without replacement."""
    rng = rng_for(config, item, MASK_STREAM)
    m = np.zeros(H * W, np.uint8)
    m[rng.choice(H * W, size=count, replace=False)] = 1
    return m.reshape(H, W)


def _fs_python(p: np.ndarray) -> np.ndarray:
    H, W = p.shape
    q = p.copy()
    out = np.zeros((H, W), np.uint8)
    for y in range(H):
        row = q[y]
        for x in range(W):
            old = row[x]
            new = 1.0 if old >= 0.5 else 0.0
            out[y, x] = int(new)
            e = old - new
            if x + 1 < W:
                row[x + 1] += e * 7 / 16
            if y + 1 < H:
                if x > 0:
                    q[y + 1, x - 1] += e * 3 / 16
                q[y + 1, x] += e * 5 / 16
                if x + 1 < W:
                    q[y + 1, x + 1] += e * 1 / 16
    return out


def fs_dither(p: np.ndarray) -> np.ndarray:
    """Floyd-Steinberg dithering (raster order, threshold 0.5)."""
    p = np.ascontiguousarray(p, dtype=np.float64).copy()
    H, W = p.shape
    if os.path.exists(_FS_LIB):
        lib = ctypes.CDLL(_FS_LIB)
        out = np.zeros((H, W), np.uint8)
        lib.fs_dither(p.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(H), ctypes.c_int64(W),
                      out.ctypes.data_as(ctypes.c_void_p))
        return out
    if H * W > 600_000:
        raise RuntimeError("workloads/_fs_dither.so is not built; run __graft_entry__.build()")
    return _fs_python(p)


def gradient_mask(f: np.ndarray, density: float) -> np.ndarray:
    """FS dithering of p = min(1, alpha*|grad mean_c f|) with alpha bisected so
    that sum(p) = density*N. Central differences, mirrored border."""
    g = f.mean(axis=0) if f.ndim == 3 else f
    gp = np.pad(g, 1, mode="edge")
    gx = (gp[1:-1, 2:] - gp[1:-1, :-2]) * 0.5
    gy = (gp[2:, 1:-1] - gp[:-2, 1:-1]) * 0.5
    mag = np.hypot(gx, gy)
    target = density * g.size
    lo, hi = 0.0, 1.0
    while np.minimum(1.0, hi * mag).sum() < target:
        hi *= 2.0
    for _ in range(50):
        a = 0.5 * (lo + hi)
        if np.minimum(1.0, a * mag).sum() < target:
            lo = a
        else:
            hi = a
    m = fs_dither(np.minimum(1.0, hi * mag))
    if m.sum() == 0:
        m.flat[int(np.argmax(mag))] = 1
    return m


# ---------------------------------------------------------------- configurations

@dataclass
class Instance:
    f: np.ndarray      # C x H x W float64 (values exactly representable in float32)
    mask: np.ndarray   # H x W uint8
    name: str


def config1() -> Instance:
    """256x256 grayscale bumps+rectangles, exactly floor(0.05*N) = 3276 uniform mask pixels."""
    H = W = 256
    f = bumps_and_rects(H, W, 1, 0)[None]
    return Instance(f, uniform_mask(H, W, int(0.05 * H * W), 1, 0), "gray 256x256, 5% uniform mask")


def config2(H: int = 2160, W: int = 3840, C: int = 3, density: float = 0.03, item: int = 0) -> Instance:
    """Textured RGB image with a 3% FS-dithered gradient-magnitude mask."""
    f = textured_image(H, W, C, 2, item)
    return Instance(f, gradient_mask(f, density), f"{'RGB' if C == 3 else 'gray'} {W}x{H}, {density:.0%} FS-gradient mask")


def config3(H: int = 1080, W: int = 1920) -> Instance:
    """Grayscale textured image with a 0.5% uniform random starting mask."""
    f = textured_image(H, W, 1, 3, 0)
    n0 = int(0.005 * H * W)
    return Instance(f, uniform_mask(H, W, n0, 3, 0), f"gray {W}x{H}, 0.5% uniform start mask")


def config4_specs(n: int = 64):
    """(H, W, C, density) of the uneven batch: W~U{512..2048}, H~U{512..1152},
    half gray and half RGB (shuffled), density~U(0.01, 0.10)."""
    rng = rng_for(4, 0, 2000)
    Cs = np.array([1] * (n // 2) + [3] * (n - n // 2))
    rng.shuffle(Cs)
    out = []
    for i in range(n):
        W = int(rng.integers(512, 2049))
        H = int(rng.integers(512, 1153))
        d = float(rng.uniform(0.01, 0.10))
        out.append((H, W, int(Cs[i]), d))
    return out


def config4_item(i: int, spec) -> Instance:
    H, W, C, d = spec
    f = textured_image(H, W, C, 4, i)
    return Instance(f, gradient_mask(f, d), f"batch item {i}: {C}x{H}x{W} d={d:.3f}")
