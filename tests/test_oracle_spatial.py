"""Pins for the spatial-optimisation oracle (Sec. 4.2 implementation details,
Alg. 1): closed forms of the Laplacian magnitude, the coin-flip rule on
hand-made inputs, its expected size, and the loop's bookkeeping."""
import numpy as np

from oracle import densify as od
from oracle import inpaint as oi
from oracle import spatial as osp


def test_laplacian_magnitude_closed_forms():
    # constant image: zero everywhere
    assert np.all(osp.laplacian_magnitude(np.full((2, 7, 9), 42.0)) == 0)
    # linear ramp in x: zero inside, the slope at the two mirrored border columns
    H, W, s = 6, 10, 3.5
    ramp = np.tile(s * np.arange(W, dtype=np.float64), (H, 1))
    lap = osp.laplacian_magnitude(ramp)
    assert np.all(lap[:, 1:-1] == 0)
    assert np.all(lap[:, 0] == s) and np.all(lap[:, -1] == s)
    # one bright pixel a: 4a on it, a on its four neighbours, channels add up
    a = 10.0
    img = np.zeros((3, 9, 9))
    img[:, 4, 4] = [a, 2 * a, 0.0]
    lap = osp.laplacian_magnitude(img)
    assert lap[4, 4] == 4 * 3 * a
    for y, x in [(3, 4), (5, 4), (4, 3), (4, 5)]:
        assert lap[y, x] == 3 * a
    assert lap.sum() == 4 * 3 * a + 4 * 3 * a


def test_laplacian_magnitude_is_the_grid_laplacian():
    """The mirrored 5-point stencil is the grid-graph Laplacian of the inpainting
    oracle with the opposite sign."""
    rng = np.random.default_rng(0)
    f = rng.uniform(0, 255, (1, 13, 17))
    L = oi.grid_laplacian(13, 17)
    np.testing.assert_allclose(osp.laplacian_magnitude(f).ravel(), np.abs(L @ f.ravel()), rtol=0, atol=1e-9)


def test_coin_rule_on_hand_made_input():
    # a 1 x 4 image with one bright pixel: |Lap| = [0, 1, 2, 1], alpha = n0 / sum(l)
    f = np.array([[[0.0, 0.0, 1.0, 0.0]]])
    lap = osp.laplacian_magnitude(f)
    assert list(lap.ravel()) == [0.0, 1.0, 2.0, 1.0]
    # n0 = 2: alpha = 2 / 4 = 0.5, probabilities [0, 0.5, 1, 0.5]
    r = np.array([0.0, 0.49, 0.99, 0.5])
    m = osp.initial_mask(f, 2, r)
    assert list(m.ravel()) == [0, 1, 1, 0]        # r < p strictly
    # constant image falls back to uniform n0 / N
    m = osp.initial_mask(np.zeros((1, 2, 2)), 2, np.array([0.1, 0.6, 0.49, 0.5]))
    assert list(m.ravel()) == [1, 0, 1, 0]


def test_expected_size_and_adaptivity():
    """Over many draws the mask size averages n0, and pixels land where the
    Laplacian is large."""
    rng = np.random.default_rng(1)
    yy, xx = np.mgrid[0:128, 0:128]
    f = 100.0 + 80.0 * ((xx > 64) ^ (yy > 40))          # edges only
    sizes = []
    hits = np.zeros((128, 128))
    for k in range(40):
        m = osp.initial_mask(f, 300, rng.random((128, 128)))
        sizes.append(int(m.sum()))
        hits += m
    assert abs(np.mean(sizes) - 300) < 3 * np.sqrt(300 / 40) + 1
    lap = osp.laplacian_magnitude(f)
    assert hits[lap == 0].sum() == 0                     # never in flat regions
    assert hits[lap > 0].sum() == sum(sizes)


def test_error_map_is_fp32_of_the_channel_sum():
    rng = np.random.default_rng(2)
    u = rng.normal(100, 30, (3, 5, 6))
    f = rng.uniform(0, 255, (3, 5, 6)).astype(np.float32).astype(np.float64)
    e = osp.error_map(u, f)
    d = u - f
    assert e.dtype == np.float32
    assert np.array_equal(e, ((d[0] ** 2 + d[1] ** 2) + d[2] ** 2).astype(np.float32))


def test_loop_bookkeeping():
    """Masks grow by exactly the schedule, each step's pixels are new and the
    final count is floor(d N)."""
    rng = np.random.default_rng(3)
    H, W = 40, 56
    f = rng.uniform(0, 255, (1, H, W))
    mask, u, steps = osp.spatial_optimize(f, 0.05, 4, rng.random((H, W)))
    n_target = int(np.floor(0.05 * H * W))
    assert int(mask.sum()) == n_target
    m0 = int(mask.sum()) - sum(len(s) for s in steps)
    sched = od.schedule(m0, n_target, 4)
    assert [m0 + sum(len(s) for s in steps[:k + 1]) for k in range(4)] == sched
    allp = np.concatenate(steps)
    assert np.unique(allp).size == allp.size
    np.testing.assert_allclose(u, oi.inpaint(f, mask))


def test_loop_with_jump_flooding_labels():
    """With J3's shrinking jump-flooding start the loop keeps its bookkeeping,
    and its steps are densification steps on the jump-flooding labels."""
    rng = np.random.default_rng(4)
    H, W = 36, 50
    f = rng.uniform(0, 255, (1, H, W))
    r = rng.random((H, W))
    mask, u, steps = osp.spatial_optimize(f, 0.06, 3, r, jfa=True)
    n_target = int(np.floor(0.06 * H * W))
    assert int(mask.sum()) == n_target
    m = osp.initial_mask(f, osp.start_size(n_target, 3), r)
    k0 = None
    for k, M in enumerate(od.schedule(int(m.sum()), n_target, 3)):
        lab = od.jfa_labels(m, k0)
        k0 = od.jfa_next_step(od.label_max_d2(lab))
        e = osp.error_map(oi.inpaint(f, m), f)
        m, added, _ = od.densify_step(m, e, M - int(m.sum()), "delaunay", lab)
        np.testing.assert_array_equal(added, steps[k])
    np.testing.assert_array_equal(m, mask)
