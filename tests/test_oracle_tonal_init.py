"""Pins for the Voronoi-initialisation oracle (Sec. 5.3): the weight matrices
against brute-force constructions, closed forms for one mask pixel (where the
constant-weight cell average is the true tonal optimum), a hand-solved 1D fixed
point, and the best-iteration rule."""
import math

import numpy as np
import pytest

from oracle import tonal as ot
from oracle import tonal_init as oti


def test_direct_weights_are_clipped_3x3_means():
    H, W = 5, 6
    mask = np.zeros((H, W), np.uint8)
    pts = [(0, 0), (0, 3), (2, 2), (4, 5), (2, 5)]
    for y, x in pts:
        mask[y, x] = 1
    Wm = oti.weight_matrix(mask, oti.DIRECT).toarray()
    seeds = sorted(y * W + x for y, x in pts)
    for r, s in enumerate(seeds):
        sy, sx = divmod(s, W)
        expect = np.zeros(H * W)
        win = [(y, x) for y in range(sy - 1, sy + 2) for x in range(sx - 1, sx + 2) if 0 <= y < H and 0 <= x < W]
        for y, x in win:
            expect[y * W + x] = 1.0 / len(win)
        np.testing.assert_allclose(Wm[r], expect, rtol=0, atol=1e-15)
    # corner 4, edge 6, interior 9 pixels
    assert [np.count_nonzero(Wm[r]) for r in range(len(seeds))] == [4, 6, 9, 6, 4]


@pytest.mark.parametrize("weighting", [oti.VORONOI, oti.VORONOI_LOG])
def test_voronoi_weights_partition_the_image(weighting):
    rng = np.random.default_rng(5)
    H, W = 9, 13
    mask = (rng.random((H, W)) < 0.12).astype(np.uint8)
    mask[4, 6] = 1
    Wm = oti.weight_matrix(mask, weighting).toarray()
    seeds = np.flatnonzero(mask.ravel())
    np.testing.assert_allclose(Wm.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    assert np.all((Wm > 0).sum(axis=0) == 1)            # every pixel in exactly one cell
    for j in range(H * W):                               # ... the one of its nearest mask pixel
        y, x = divmod(j, W)
        d2 = [((y - s // W) ** 2 + (x - s % W) ** 2, s) for s in seeds]
        owner = min(d2)[1]
        r = int(np.flatnonzero(Wm[:, j])[0])
        assert seeds[r] == owner
    if weighting == oti.VORONOI_LOG:                     # weights fall with the distance inside a cell
        r = int(np.flatnonzero(seeds == 4 * W + 6)[0])
        row = Wm[r]
        assert row[4 * W + 6] == row.max()


@pytest.mark.parametrize("weighting", [oti.DIRECT, oti.VORONOI, oti.VORONOI_LOG])
def test_single_mask_pixel_closed_forms(weighting):
    """One mask pixel inpaints to a constant, so one step at tau = 1 lands on
    the weighted average of f over the support, which is a fixed point."""
    rng = np.random.default_rng(6)
    H, W, sy, sx = 7, 10, 2, 7
    f = rng.uniform(0, 255, (2, H, W))
    mask = np.zeros((H, W), np.uint8)
    mask[sy, sx] = 1
    num, den = np.zeros(2), 0.0
    for y in range(H):
        for x in range(W):
            if weighting == oti.DIRECT:
                w = 1.0 if abs(y - sy) <= 1 and abs(x - sx) <= 1 else 0.0
            elif weighting == oti.VORONOI:
                w = 1.0
            else:
                w = 1.0 / (1.0 + math.log(1.0 + math.hypot(y - sy, x - sx)))
            num += w * f[:, y, x]
            den += w
    g, u, trace, k = oti.voronoi_init(f, mask, weighting, max_iters=3, stop_on_increase=False)
    np.testing.assert_allclose(g[:, sy, sx], num / den, rtol=1e-13)
    np.testing.assert_allclose(u, np.broadcast_to((num / den)[:, None, None], u.shape), rtol=1e-12)
    assert abs(trace[1] - trace[2]) <= 1e-12 * trace[1] and k == 3
    if weighting == oti.VORONOI:
        # the cell is the whole image and the constant that minimises the MSE is the mean
        gopt = ot.tonal_optimize(f, mask)
        np.testing.assert_allclose(g[:, sy, sx], gopt[:, sy, sx], rtol=1e-10)


def test_two_seeds_in_1d_reach_the_hand_solved_fixed_point():
    """1D homogeneous diffusion interpolates linearly between two mask pixels
    and is flat outside, so each cell's average of u is linear in (g_a, g_b);
    the fixed point solves that 2 x 2 system."""
    rng = np.random.default_rng(7)
    n, a, b = 23, 4, 15
    f = rng.uniform(0, 255, (1, 1, n))
    mask = np.zeros((1, n), np.uint8)
    mask[0, a] = mask[0, b] = 1
    cells = ([j for j in range(n) if abs(j - a) <= abs(j - b)], [j for j in range(n) if abs(j - a) > abs(j - b)])

    def coef(j):   # u_j = ca g_a + cb g_b
        if j <= a:
            return 1.0, 0.0
        if j >= b:
            return 0.0, 1.0
        t = (j - a) / (b - a)
        return 1.0 - t, t

    M = np.array([[np.mean([coef(j)[0] for j in cell]), np.mean([coef(j)[1] for j in cell])] for cell in cells])
    rhs = np.array([np.mean(f[0, 0, cell]) for cell in cells])
    fix = np.linalg.solve(M, rhs)
    g, u, trace, k = oti.voronoi_init(f, mask, oti.VORONOI, max_iters=300, stop_on_increase=False)
    np.testing.assert_allclose([g[0, 0, a], g[0, 0, b]], fix, rtol=1e-10)


def test_constant_image_stays_put():
    f = np.full((3, 12, 9), 31.0)
    mask = np.zeros((12, 9), np.uint8)
    mask[::4, ::3] = 1
    g, u, trace, k = oti.voronoi_init(f, mask)
    assert trace[0] <= 1e-24          # the direct solve reproduces a constant up to rounding
    np.testing.assert_allclose(u, f, rtol=0, atol=1e-12)
    assert np.all(g[:, mask == 0] == 0) and np.allclose(g[:, mask != 0], 31.0)


@pytest.mark.parametrize("weighting", [oti.DIRECT, oti.VORONOI_LOG])
def test_best_iteration_rule_and_bounds(weighting):
    rng = np.random.default_rng(8)
    H, W = 24, 30
    yy, xx = np.mgrid[0:H, 0:W]
    f = (100 + 60 * np.sin(xx / 3.0) * np.cos(yy / 4.0) + rng.normal(0, 5, (H, W)))[None]
    mask = (rng.random((H, W)) < 0.08).astype(np.uint8)
    g, u, trace, k = oti.voronoi_init(f, mask, weighting, max_iters=40)
    # stopped at the first rise (or the cap), returned the iterate before it
    rises = [i for i in range(1, len(trace)) if trace[i] > trace[i - 1]]
    assert k == (rises[0] - 1 if rises else len(trace) - 1)
    assert all(trace[i] <= trace[i - 1] for i in range(1, k + 1))
    m = ot.mse(g, f, mask)
    assert abs(m - trace[k]) <= 1e-10 * m
    np.testing.assert_allclose(u, ot.reconstruct(g, mask), rtol=0, atol=1e-9)
    # the surrogate improves on f but cannot beat the true optimum
    m_opt = ot.mse(ot.tonal_optimize(f, mask), f, mask)
    assert m_opt <= m <= trace[0]
    assert m < trace[0]
