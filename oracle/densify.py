"""Oracle: one Delaunay (or Voronoi) densification step (test infrastructure only).

Paper Sec. 4.1, Alg. 1: partition the image with the Delaunay triangulation of
the current mask pixels (obtained from their Voronoi diagram, Sec. 4.2),
accumulate the error map over each triangle (the triangle-error equation of
Sec. 4.1), take the triangles with the largest errors, and add in each of them
the pixel of largest pointwise error, at most one per triangle.

The paper does not fix the discrete details. This module follows one exact
reading, step by step, so that a GPU implementation can be compared bit for bit:

  S1 labels      V(p) = argmin over mask pixels s of (|p - s|^2, index(s)):
                 exact nearest mask pixel, ties to the smaller linear index.
  S2 triangles   for every 2x2 quad with corners q0=(x,y), q1=(x+1,y),
                 q2=(x+1,y+1), q3=(x,y+1) and labels l0..l3: three distinct
                 labels give one triangle, four give {l0,l1,l2} and {l0,l2,l3}.
                 A triangle is its sorted index triple; duplicates are merged
                 and collinear triples dropped.
  S3 coverage    a pixel centre lies in a triangle if it is inside or on the
                 boundary of the closed triangle (integer edge functions).
  S4 ownership   a pixel belongs to the covering triangle with the smallest
                 key; uncovered pixels belong to the Voronoi cell of V(p).
                 Cells are ordered: triangles by key, then Voronoi cells by
                 mask-pixel index.
  S5 cell error  E = sum over the cell of q(e_p), q(e) = round(e * 2^20) as an
                 unsigned integer (exact and order independent).
  S6 ranking     cells by (E descending, cell order ascending).
  S7 selection   walking the ranking, each cell with a non-mask pixel adds its
                 pixel of largest e (float32 comparison; ties to the smaller
                 index), until n_add pixels are added.
  S8 Voronoi     the partition="voronoi" variant (the paper's ablation, Sec. 6.2)
                 skips S2-S4: every pixel belongs to the Voronoi cell of V(p).

The paper builds its Voronoi diagram with the jump flooding algorithm of Rong
and Tan (Sec. 4.2), which is approximate. jfa_labels follows one reading of it,
integer-exact so that it too can be compared bit for bit:

  J1 passes      labels start as the pixel's own index on mask pixels and none
                 elsewhere; a pass with step k gives every pixel the best label
                 among those held before the pass at the nine pixels p + k (i, j),
                 i, j in {-1, 0, 1}, inside the image, by (|p - s|^2, index(s));
                 the steps are k0, k0/2, ..., 1.
  J2 start       k0 = the largest power of two below max(W, H) unless given.
  J3 loop        in the densification loop the next step's k0 is the smallest
                 power of two at least the largest pixel-to-label distance of the
                 current labels (the mask only grows, so that distance bounds the
                 next one); the first step uses J2.
A step with JFA labels runs S2-S8 on them unchanged (every mask pixel keeps its
own label, so the Voronoi cells are still one per mask pixel).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

FIXED_SHIFT = 20


def voronoi_labels(mask: np.ndarray, method: str = "auto") -> np.ndarray:
    """S1. int64 H x W array of the nearest mask pixel's linear index. Brute
    force for small grids, a k-d tree with exact tie expansion otherwise."""
    H, W = mask.shape
    seeds = np.flatnonzero(mask.ravel())
    if seeds.size == 0:
        raise ValueError("empty mask")
    sy, sx = np.divmod(seeds, W)
    yy, xx = np.divmod(np.arange(H * W), W)
    if method == "brute" or (method == "auto" and seeds.size * H * W <= 4_000_000):
        d2 = (yy[:, None] - sy[None, :]) ** 2 + (xx[:, None] - sx[None, :]) ** 2
        return seeds[np.argmin(d2, axis=1)].reshape(H, W)   # first minimum = smallest index
    tree = cKDTree(np.stack([sx, sy], axis=1))
    out = np.empty(H * W, np.int64)
    todo = np.arange(H * W)
    k = min(8, seeds.size)
    while todo.size:
        _, nb = tree.query(np.stack([xx[todo], yy[todo]], axis=1), k=k)
        nb = nb.reshape(todo.size, -1)
        d2 = (xx[todo, None] - sx[nb]) ** 2 + (yy[todo, None] - sy[nb]) ** 2
        best = d2.min(axis=1)
        cand = np.where(d2 == best[:, None], seeds[nb], np.iinfo(np.int64).max)
        # all nearest seeds found when the k-th neighbour is strictly farther
        done = (d2[:, -1] > best) | (k >= seeds.size)
        out[todo[done]] = cand[done].min(axis=1)
        todo = todo[~done]
        k = min(2 * k, seeds.size)
    return out.reshape(H, W)


def jfa_default_step(H: int, W: int) -> int:
    """J2: the largest power of two below max(W, H) (0: no passes)."""
    n = max(H, W)
    k = 1
    while 2 * k < n:
        k *= 2
    return k if n > 1 else 0


def jfa_labels(mask: np.ndarray, k0: int | None = None) -> np.ndarray:
    """J1. int64 H x W labels after jump-flooding passes k0, k0/2, ..., 1."""
    H, W = mask.shape
    if not np.any(mask):
        raise ValueError("empty mask")
    lab = np.where(np.asarray(mask).ravel() != 0, np.arange(H * W), -1).reshape(H, W)
    yy, xx = np.mgrid[0:H, 0:W]
    k = jfa_default_step(H, W) if k0 is None else int(k0)
    while k >= 1:
        best_d = np.full((H, W), np.iinfo(np.int64).max, np.int64)
        best_l = np.full((H, W), -1, np.int64)
        for dy in (-k, 0, k):
            for dx in (-k, 0, k):
                ny, nx = yy + dy, xx + dx
                ok = (ny >= 0) & (ny < H) & (nx >= 0) & (nx < W)
                cand = np.where(ok, lab[np.clip(ny, 0, H - 1), np.clip(nx, 0, W - 1)], -1)
                cy, cx = np.divmod(np.maximum(cand, 0), W)
                d = (cy - yy) ** 2 + (cx - xx) ** 2
                better = (cand >= 0) & ((d < best_d) | ((d == best_d) & (cand < best_l)))
                best_d = np.where(better, d, best_d)
                best_l = np.where(better, cand, best_l)
        lab = best_l
        k //= 2
    return lab


def label_max_d2(labels: np.ndarray) -> int:
    """Largest squared distance from a pixel to its label (unlabelled pixels,
    -1, are skipped)."""
    H, W = labels.shape
    yy, xx = np.mgrid[0:H, 0:W]
    ok = labels >= 0
    ly, lx = np.divmod(np.where(ok, labels, 0), W)
    return int(np.where(ok, (ly - yy) ** 2 + (lx - xx) ** 2, 0).max())


def jfa_next_step(max_d2: int) -> int:
    """J3: the smallest power of two at least sqrt(max_d2) (at least 1)."""
    k = 1
    while k * k < max_d2:
        k *= 2
    return k


def _orient(ax, ay, bx, by, cx, cy):
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)


def triangles(labels: np.ndarray) -> np.ndarray:
    """S2. Sorted, unique, non-collinear index triples (n x 3, int64), in key order."""
    H, W = labels.shape
    if H < 2 or W < 2:
        return np.zeros((0, 3), np.int64)
    l0, l1 = labels[:-1, :-1].ravel(), labels[:-1, 1:].ravel()
    l2, l3 = labels[1:, 1:].ravel(), labels[1:, :-1].ravel()
    q = np.stack([l0, l1, l2, l3], axis=1)
    nd = np.array([len(set(r)) for r in q]) if q.shape[0] < 50 else \
        (np.sort(q, axis=1)[:, 1:] != np.sort(q, axis=1)[:, :-1]).sum(axis=1) + 1
    out = []
    three = q[nd == 3]
    if three.size:
        s = np.sort(three, axis=1)
        # the three distinct values of a sorted row with one duplicate
        uniq = np.where((s[:, 0] == s[:, 1])[:, None], s[:, [0, 2, 3]],
                        np.where((s[:, 1] == s[:, 2])[:, None], s[:, [0, 1, 3]], s[:, [0, 1, 2]]))
        out.append(uniq)
    four = q[nd == 4]
    if four.size:
        out.append(np.sort(four[:, [0, 1, 2]], axis=1))
        out.append(np.sort(four[:, [0, 2, 3]], axis=1))
    if not out:
        return np.zeros((0, 3), np.int64)
    t = np.unique(np.concatenate(out), axis=0)   # lexicographic order = key order
    ay, ax = np.divmod(t[:, 0], W)
    by, bx = np.divmod(t[:, 1], W)
    cy, cx = np.divmod(t[:, 2], W)
    return t[_orient(ax, ay, bx, by, cx, cy) != 0]


def ownership(labels: np.ndarray, tris: np.ndarray, partition: str = "delaunay"):
    """S3/S4. Cell id per pixel: triangle rank (0..T-1) or T + rank of the
    Voronoi seed among the mask pixels (ascending)."""
    H, W = labels.shape
    seeds = np.unique(labels)
    seed_rank = np.full(H * W, -1, np.int64)
    all_seeds = np.sort(seeds)
    T = 0 if partition == "voronoi" else len(tris)
    owner = np.full((H, W), np.iinfo(np.int64).max, np.int64)
    if partition != "voronoi":
        for r, (a, b, c) in enumerate(tris):
            ay, ax = divmod(int(a), W)
            by, bx = divmod(int(b), W)
            cy, cx = divmod(int(c), W)
            if _orient(ax, ay, bx, by, cx, cy) < 0:
                bx, by, cx, cy = cx, cy, bx, by
            x0, x1 = min(ax, bx, cx), max(ax, bx, cx)
            y0, y1 = min(ay, by, cy), max(ay, by, cy)
            yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
            inside = ((_orient(ax, ay, bx, by, xx, yy) >= 0) & (_orient(bx, by, cx, cy, xx, yy) >= 0)
                      & (_orient(cx, cy, ax, ay, xx, yy) >= 0))
            sub = owner[y0:y1 + 1, x0:x1 + 1]
            sub[inside] = np.minimum(sub[inside], r)
    seed_rank[all_seeds] = np.arange(all_seeds.size)
    uncovered = owner == np.iinfo(np.int64).max
    owner[uncovered] = T + seed_rank[labels[uncovered]]
    return owner, T + all_seeds.size


def quantise(e: np.ndarray) -> np.ndarray:
    """S5. q(e) = rint(e * 2^20) as uint64 (e is float32, e >= 0)."""
    return np.rint(np.ldexp(np.asarray(e, np.float32).astype(np.float64), FIXED_SHIFT)).astype(np.uint64)


def densify_step(mask: np.ndarray, err: np.ndarray, n_add: int, partition: str = "delaunay",
                 labels: np.ndarray | None = None):
    """One densification step. Returns (new mask, added pixel indices ascending,
    and a dict of intermediate results for tests). labels: the partition's
    Voronoi labels if not the exact ones (S1), e.g. jfa_labels(mask)."""
    mask = np.asarray(mask).astype(np.uint8)
    err = np.asarray(err, np.float32)
    H, W = mask.shape
    labels = voronoi_labels(mask) if labels is None else np.asarray(labels, np.int64)
    tris = triangles(labels) if partition == "delaunay" else np.zeros((0, 3), np.int64)
    owner, ncells = ownership(labels, tris, partition)
    cells = owner.ravel()
    E = np.zeros(ncells, np.uint64)
    np.add.at(E, cells, quantise(err).ravel())
    # S6: E descending, then cell order ascending
    rank = np.lexsort((np.arange(ncells), -E.astype(np.float64))) if E.max() < 2 ** 52 else \
        sorted(range(ncells), key=lambda i: (-int(E[i]), i))
    rank = np.asarray(rank)
    # S7: per cell, the non-mask pixel of largest e (float32), ties to smaller index
    idx = np.arange(H * W)
    free = mask.ravel() == 0
    fc, fe, fi = cells[free], err.ravel()[free], idx[free]
    order = np.lexsort((fi, -fe.astype(np.float64), fc))   # by cell, e desc, index asc
    first = np.ones(order.size, bool)
    first[1:] = fc[order][1:] != fc[order][:-1]
    best = np.full(ncells, -1, np.int64)
    best[fc[order][first]] = fi[order][first]
    added = []
    for c in rank:
        if len(added) >= n_add:
            break
        if best[c] >= 0:
            added.append(best[c])
    added = np.sort(np.asarray(added, np.int64))
    out = mask.copy().ravel()
    out[added] = 1
    return out.reshape(H, W), added, {"labels": labels, "triangles": tris, "owner": owner, "E": E,
                                      "rank": rank, "best": best}


def schedule(n0: int, n_target: int, n_steps: int, t: float = 1.0) -> list:
    """Cumulative mask sizes M_k after step k = 1..n (Alg. 1 with m_i = t m_{i-1}):
    the added counts grow by the factor t and sum to n_target - n0; with t = 1
    (the paper's experiments) every step adds the same amount, rounded so that
    the totals are exact."""
    delta = n_target - n0
    if t == 1.0:
        return [n0 + int(round(delta * k / n_steps)) for k in range(1, n_steps + 1)]
    tk, tn = 1.0, t ** n_steps
    out = []
    for _ in range(n_steps):
        tk *= t
        out.append(n0 + int(np.floor(delta * (tk - 1) / (tn - 1) + 0.5)))
    return out
