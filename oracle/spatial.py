"""Oracle: image-adaptive initial mask and the densification loop (test infrastructure only).

Paper Sec. 4.2 (implementation details of the spatial optimisation): the
initial mask comes from a random dithering of the Laplacian magnitude, one
biased coin flip per pixel with a probability proportional to that magnitude;
Alg. 1 then grows the mask over n steps, each one an inpainting, an error map
and one densification step, with the number of added pixels scaled by a factor
t from step to step.

The paper leaves the discrete details open. This module follows one reading,
step by step, so that a GPU implementation can be compared bit for bit:

  L1 magnitude   l_p = sum over channels of |(Delta f_c)_p|, with the 5-point
                 Laplacian under the reflecting boundary (a neighbour outside
                 the image is the pixel itself), in float64, added up, down,
                 left, right, minus four times the centre, channels in order
                 (exact for image data, whose values span few binades).
  L2 scale       the coin of pixel p lands with probability alpha * l_p, where
                 alpha = n0 / (S 2^-16) and S = sum_p round(l_p 2^16) as an
                 integer (exact and order independent), so the expected mask
                 size is n0 where no probability exceeds 1. An image with
                 S = 0 (constant) falls back to the uniform probability n0 / N.
  L3 coins       pixel p joins the mask iff r_p < alpha * l_p (float64), for
                 the given uniform numbers r in [0, 1).
  L4 loop        targets M_1..M_n from the schedule of the densification
                 oracle (from the realised initial size to floor(d N), the
                 density convention of the paper); step k solves the inpainting,
                 forms e = fp32(sum_c (u_c - f_c)^2) and adds M_k - |c| pixels
                 with densify_step; a last solve gives the reconstruction.
  L5 start size  n0 = round(floor(d N) / (n + 1)) unless given: the initial mask
                 then holds about as many pixels as one step adds.
"""
from __future__ import annotations

import numpy as np

from . import densify as od
from . import inpaint as oi

FIXED_SHIFT = 16


def laplacian_magnitude(f: np.ndarray) -> np.ndarray:
    """L1: sum over channels of |Delta f_c| (reflecting boundary), float64."""
    f = np.asarray(f, np.float64)
    if f.ndim == 2:
        f = f[None]
    out = np.zeros(f.shape[1:])
    for c in range(f.shape[0]):
        g = np.pad(f[c], 1, mode="edge")   # mirror: the outside neighbour equals the pixel
        lap = g[:-2, 1:-1] + g[2:, 1:-1] + g[1:-1, :-2] + g[1:-1, 2:] - 4.0 * f[c]
        out += np.abs(lap)
    return out


def initial_mask(f: np.ndarray, n0: int, r: np.ndarray) -> np.ndarray:
    """L2-L3: random dithering of the Laplacian magnitude with given uniforms r."""
    lap = laplacian_magnitude(f)
    N = lap.size
    S = int(np.rint(np.ldexp(lap, FIXED_SHIFT)).astype(np.int64).sum())
    if S > 0:
        alpha = float(n0) / (S * 2.0 ** -FIXED_SHIFT)
        p = alpha * lap
    else:
        p = np.full(lap.shape, float(n0) / N)
    return (np.asarray(r, np.float64).reshape(lap.shape) < p).astype(np.uint8)


def start_size(n_target: int, n_steps: int) -> int:
    """L5: about one step's worth of pixels."""
    return int(round(n_target / (n_steps + 1)))


def error_map(u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """e = fp32(sum_c (u_c - f_c)^2), summed in float64 in channel order."""
    u = np.asarray(u, np.float64)
    f = np.asarray(f, np.float64)
    if f.ndim == 2:
        f = f[None]
        u = u.reshape(f.shape)
    acc = np.zeros(f.shape[1:])
    for c in range(f.shape[0]):
        d = u[c] - f[c]
        acc = acc + d * d
    return acc.astype(np.float32)


def spatial_optimize(f: np.ndarray, density: float, n_steps: int, r: np.ndarray, t: float = 1.0,
                     n0: int | None = None, partition: str = "delaunay", jfa: bool = False):
    """L4: the whole loop with exact (direct) inpaintings. Returns (mask, u,
    list of per-step added pixel arrays). jfa: the partition's labels come from
    jump flooding with the shrinking start step of the densification oracle (J3)."""
    f = np.asarray(f, np.float64)
    if f.ndim == 2:
        f = f[None]
    N = f.shape[1] * f.shape[2]
    n_target = int(np.floor(density * N))
    mask = initial_mask(f, start_size(n_target, n_steps) if n0 is None else n0, r)
    targets = od.schedule(int(mask.sum()), n_target, n_steps, t)
    steps = []
    k0 = None
    for M in targets:
        u = oi.inpaint(f, mask)
        e = error_map(u, f)
        labels = None
        if jfa:
            labels = od.jfa_labels(mask, k0)
            k0 = od.jfa_next_step(od.label_max_d2(labels))
        mask, added, _ = od.densify_step(mask, e, max(M - int(mask.sum()), 0), partition, labels)
        steps.append(added)
    return mask, oi.inpaint(f, mask), steps
