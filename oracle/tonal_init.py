"""Oracle: Voronoi initialisation of tonal optimisation (test infrastructure only).

Paper Sec. 5.3: instead of making the inpainting reproduce f at the mask
pixels, make it reproduce local averages of f around them, C W B g = C W f for
a row-normalised weight matrix W, and solve that surrogate with a Richardson
iteration started at g = f on the mask. One step with tau = 1 and W the 3x3
neighbourhood mean is the error balancing of Galic et al.; the paper's choice
averages over each mask pixel's Voronoi cell, weighted down with the distance
to the mask pixel, and stops once the MSE rises (Sec. 6.3: keep the best
iteration).

The paper leaves the details open. This module follows one reading:

  V1 direct      W_ij = 1 / |N(i)| for the pixels j of the 3x3 window around
                 mask pixel i clipped to the image (i itself included).
  V2 cells       cell(i) = pixels whose nearest mask pixel is i, with the exact
                 labels of the densification oracle (ties to the smaller index).
  V3 weights     w(d) = 1 (constant) or w(d) = 1 / (1 + ln(1 + d)) (inverse
                 logarithmic distance), d the Euclidean distance from j to i,
                 normalised over the cell: W_ij = w(d_ij) / sum_cell w.
  V4 step        g_K <- g_K + tau (W f - W B g)_K, tau = 1 unless given: the
                 Richardson step for C W B C g = C W f (the printed step has
                 C f where the constraint has C W f; with C W f the first step
                 at tau = 1 is exactly Galic's error balancing).
  V5 stop        MSE(g) = ||f - B g||^2 / (C N); after each step, if the MSE
                 rose strictly above the previous iterate's, stop and return
                 the previous iterate; otherwise stop after max_iters steps.
  V6 start       g^0 = f on the mask (or a given g0).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .densify import voronoi_labels
from .inpaint import _as_chw
from .tonal import TonalOperator

DIRECT, VORONOI, VORONOI_LOG = "direct", "voronoi", "voronoi_log"


def weight_matrix(mask: np.ndarray, weighting: str = VORONOI_LOG) -> sp.csr_matrix:
    """W restricted to the mask rows: m x N, rows in ascending mask-pixel order."""
    H, W = mask.shape
    seeds = np.flatnonzero(mask.ravel())
    m = seeds.size
    if m == 0:
        raise ValueError("empty mask")
    rank = np.full(H * W, -1, np.int64)
    rank[seeds] = np.arange(m)
    if weighting == DIRECT:
        rows, cols = [], []
        sy, sx = np.divmod(seeds, W)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                y, x = sy + dy, sx + dx
                ok = (y >= 0) & (y < H) & (x >= 0) & (x < W)
                rows.append(np.arange(m)[ok])
                cols.append((y * W + x)[ok])
        rows, cols = np.concatenate(rows), np.concatenate(cols)
        M = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(m, H * W))
    elif weighting in (VORONOI, VORONOI_LOG):
        lab = voronoi_labels(mask).ravel()
        yy, xx = np.divmod(np.arange(H * W), W)
        ly, lx = np.divmod(lab, W)
        d = np.sqrt((yy - ly) ** 2.0 + (xx - lx) ** 2.0)
        w = np.ones(H * W) if weighting == VORONOI else 1.0 / (1.0 + np.log1p(d))
        M = sp.csr_matrix((w, (rank[lab], np.arange(H * W))), shape=(m, H * W))
    else:
        raise ValueError(f"unknown weighting {weighting!r}")
    rs = np.asarray(M.sum(axis=1)).ravel()
    return sp.diags(1.0 / rs) @ M


def voronoi_init(f: np.ndarray, mask: np.ndarray, weighting: str = VORONOI_LOG, tau: float = 1.0,
                 max_iters: int = 20, stop_on_increase: bool = True, g0: np.ndarray | None = None):
    """V4-V6. Returns (g, u = B g, list of MSEs of g^0, g^1, ..., index of g).
    g is C x H x W with zeros off the mask."""
    f = _as_chw(np.asarray(f, np.float64))
    C = f.shape[0]
    K = mask.ravel() != 0
    Wm = weight_matrix(mask, weighting)
    op = TonalOperator(mask)
    g = np.zeros((C, K.size))
    g[:, K] = (f if g0 is None else _as_chw(np.asarray(g0, np.float64))).reshape(C, -1)[:, K]
    fl = f.reshape(C, -1)
    Wf = np.stack([Wm @ fl[c] for c in range(C)])

    def recon(gk):
        return np.stack([op.B(gk[c]) for c in range(C)])

    u = recon(g)
    trace = [float(((fl - u) ** 2).sum() / fl.size)]
    best = (g, u, 0)
    for k in range(1, max_iters + 1):
        g_new = g.copy()
        for c in range(C):
            g_new[c, K] = g[c, K] + tau * (Wf[c] - Wm @ u[c])
        u_new = recon(g_new)
        trace.append(float(((fl - u_new) ** 2).sum() / fl.size))
        if stop_on_increase and trace[-1] > trace[-2]:
            break
        g, u = g_new, u_new
        best = (g, u, k)
    g, u, kb = best
    shape = f.shape
    return g.reshape(shape), u.reshape(shape), trace, kb
