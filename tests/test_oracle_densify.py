"""Pins for the densification oracle (Sec. 4.1 Alg. 1, Sec. 4.2): brute force on
small grids, hand-checkable examples, and the invariants every step must keep."""
import numpy as np
import pytest
from scipy.spatial import Delaunay

from oracle import densify as od


def _rand_mask(rng, H, W, n):
    m = np.zeros(H * W, np.uint8)
    m[rng.choice(H * W, n, replace=False)] = 1
    return m.reshape(H, W)


def test_labels_tree_path_matches_brute_force():
    rng = np.random.default_rng(0)
    for H, W, n in [(40, 50, 30), (64, 64, 7), (33, 90, 200), (100, 80, 3), (60, 60, 3600 // 2)]:
        m = _rand_mask(rng, H, W, n)
        seeds = np.flatnonzero(m.ravel())
        yy, xx = np.divmod(np.arange(H * W), W)
        sy, sx = np.divmod(seeds, W)
        d2 = (yy[:, None] - sy[None, :]) ** 2 + (xx[:, None] - sx[None, :]) ** 2
        brute = seeds[np.argmin(d2, axis=1)].reshape(H, W)
        np.testing.assert_array_equal(od.voronoi_labels(m, "brute"), brute)
        np.testing.assert_array_equal(od.voronoi_labels(m, "tree"), brute)


def test_labels_tie_goes_to_smaller_index():
    """Two seeds 4 apart on a row: the middle pixel is equidistant and takes the
    seed with the smaller linear index; the split is the perpendicular bisector."""
    m = np.zeros((3, 9), np.uint8)
    m[1, 2] = m[1, 6] = 1
    lab = od.voronoi_labels(m)
    left, right = 1 * 9 + 2, 1 * 9 + 6
    assert np.all(lab[:, :4] == left) and np.all(lab[:, 5:] == right)
    assert np.all(lab[:, 4] == left)
    # vertical pair: the smaller index is the upper seed
    m = np.zeros((9, 3), np.uint8)
    m[2, 1] = m[6, 1] = 1
    lab = od.voronoi_labels(m)
    assert np.all(lab[4, :] == 2 * 3 + 1)


def test_three_seeds_give_one_triangle_and_fallback_cells():
    m = np.zeros((20, 20), np.uint8)
    pts = [(2, 3), (15, 4), (8, 16)]          # (x, y)
    for x, y in pts:
        m[y, x] = 1
    lab = od.voronoi_labels(m)
    tris = od.triangles(lab)
    assert tris.shape == (1, 3)
    assert sorted(tris[0]) == sorted(y * 20 + x for x, y in pts)
    owner, ncells = od.ownership(lab, tris)
    assert ncells == 4
    # a pixel inside the triangle belongs to it, the corners of the image do not
    assert owner[7, 8] == 0
    assert owner[0, 0] != 0 and owner[19, 19] != 0
    # the fallback cell of a corner is its Voronoi cell
    assert owner[0, 0] == 1 + list(np.sort(np.flatnonzero(m.ravel()))).index(lab[0, 0])


def test_collinear_seeds_give_no_triangle():
    m = np.zeros((10, 30), np.uint8)
    m[5, [3, 10, 20]] = 1
    tris = od.triangles(od.voronoi_labels(m))
    assert tris.shape[0] == 0


def test_triangles_mostly_agree_with_delaunay():
    """Sanity only (not parity): the quad rule on the exact discrete Voronoi
    recovers most triangles of scipy's Delaunay triangulation for random points."""
    rng = np.random.default_rng(1)
    m = _rand_mask(rng, 200, 200, 300)
    tris = od.triangles(od.voronoi_labels(m))
    seeds = np.flatnonzero(m.ravel())
    pts = np.stack([seeds % 200, seeds // 200], axis=1)
    dl = {tuple(sorted(seeds[s])) for s in Delaunay(pts).simplices}
    ours = {tuple(t) for t in tris}
    assert len(dl & ours) / len(dl) > 0.8


def test_quantisation_is_exact_and_order_free():
    e = np.array([0.0, 1.0, 2.5e-7, 195075.0, 0.1], np.float32)
    q = od.quantise(e)
    assert q[0] == 0 and q[1] == 2 ** 20 and q[3] == 195075 * 2 ** 20
    assert q[2] == 0 and q[4] == round(float(np.float32(0.1)) * 2 ** 20)


@pytest.mark.parametrize("partition", ["delaunay", "voronoi"])
def test_step_invariants(partition):
    rng = np.random.default_rng(2)
    H, W = 60, 80
    m = _rand_mask(rng, H, W, 40)
    err = (rng.random((H, W)) * 100).astype(np.float32)
    err[m != 0] = 0
    new, added, info = od.densify_step(m, err, 25, partition)
    owner, E, rank, best = info["owner"], info["E"], info["rank"], info["best"]
    assert added.size == 25 and np.unique(added).size == 25
    assert np.all(m.ravel()[added] == 0) and np.all(new.ravel()[added] == 1)
    assert int((new != m).sum()) == 25
    cells = owner.ravel()[added]
    assert np.unique(cells).size == added.size                     # at most one per cell
    # each added pixel is its cell's largest-error free pixel
    for p, c in zip(added, cells):
        free = np.flatnonzero((owner.ravel() == c) & (m.ravel() == 0))
        top = free[err.ravel()[free] == err.ravel()[free].max()].min()
        assert p == top
    # the chosen cells are the first non-empty cells of the ranking
    nonempty = [c for c in rank if best[c] >= 0]
    assert set(cells) == set(nonempty[:25])
    # ranking is by E descending, then cell order
    Er = E[rank].astype(np.float64)
    assert np.all(np.diff(Er) <= 0)
    # the cell sums conserve the quantised error
    assert int(E.sum()) == int(od.quantise(err).sum())


def test_step_adds_fewer_when_cells_run_out():
    m = np.zeros((8, 8), np.uint8)
    m[1, 1] = m[6, 6] = 1
    err = np.ones((8, 8), np.float32)
    new, added, info = od.densify_step(m, err, 100, "voronoi")
    assert added.size == 2                                           # two Voronoi cells


def test_schedule():
    s = od.schedule(10368, 82944, 8)
    assert s[-1] == 82944 and len(s) == 8
    steps = np.diff([10368] + s)
    assert np.all(steps == 9072)
    g = od.schedule(100, 1000, 5, 1.08)
    assert g[-1] == 1000 and np.all(np.diff([100] + g) > 0)
    d = np.diff([100] + g)
    assert np.all(d[1:] >= d[:-1])


def test_four_label_quad_splits_along_the_l0_l2_diagonal():
    """S2: a quad q0=(x,y), q1=(x+1,y), q2=(x+1,y+1), q3=(x,y+1) with four distinct
    labels gives the triangles {l0,l1,l2} and {l0,l2,l3}, never the other diagonal
    ({l0,l1,l3}, {l1,l2,l3}). Labels are hand-placed, with seeds far from the quad."""
    W, H = 12, 10
    a, b, c, d = 1 * W + 1, 1 * W + 10, 8 * W + 9, 9 * W + 2      # four non-collinear seeds
    for l0, l1, l2, l3 in [(a, b, c, d), (b, c, d, a), (d, a, b, c)]:
        lab = np.full((H, W), a, np.int64)
        lab[:, 6:] = b
        lab[5:, 6:] = c
        lab[5:, :6] = d
        # the only quad with four labels is the one at (x, y) = (5, 4); put the
        # requested labels on its corners
        lab[4, 5], lab[4, 6], lab[5, 6], lab[5, 5] = l0, l1, l2, l3
        tris = {tuple(t) for t in od.triangles(lab)}
        four = {tuple(sorted((l0, l1, l2))), tuple(sorted((l0, l2, l3)))}
        assert four <= tris
        other = {tuple(sorted((l0, l1, l3))), tuple(sorted((l1, l2, l3)))}
        # a triangle of the other diagonal may only appear if a 3-label quad made it
        q = np.stack([lab[:-1, :-1].ravel(), lab[:-1, 1:].ravel(), lab[1:, 1:].ravel(), lab[1:, :-1].ravel()], 1)
        from_three = {tuple(sorted(set(r))) for r in q if len(set(r)) == 3}
        assert not ((other & tris) - from_three)


def test_pixel_on_a_shared_edge_belongs_to_the_smaller_key():
    """S3/S4: triangles are closed, so a pixel centre on the edge two triangles
    share is covered by both, and the triangle with the smaller key owns it.
    Seeds at the corners of a 5x5 image; the triangles (0, 4, 24) and (0, 20, 24)
    share the diagonal from (0,0) to (4,4)."""
    W = H = 5
    a, b, c, d = 0, 4, 24, 20                 # (0,0), (4,0), (4,4), (0,4)
    tris = np.array([[a, b, c], [a, d, c]], np.int64)
    tris = np.sort(tris, axis=1)
    assert tuple(tris[0]) < tuple(tris[1])
    lab = np.full((H, W), a, np.int64)        # labels only matter for uncovered pixels
    owner, ncells = od.ownership(lab, tris)
    assert ncells == 2 + 1
    for k in range(5):
        assert owner[k, k] == 0               # on the shared diagonal: smaller key
    assert owner[1, 3] == 0 and owner[3, 1] == 1      # strictly inside each triangle
    assert owner[4, 0] == 1 and owner[0, 4] == 0      # corners d and b
    # mirrored (x -> 4 - x): the triangles (0, 4, 20) and (4, 20, 24) share the
    # anti-diagonal, which goes to the smaller key (0, 4, 20), the upper-left one
    tris2 = np.array([[0, 4, 20], [4, 20, 24]], np.int64)
    owner2, _ = od.ownership(np.zeros((H, W), np.int64), tris2)
    for k in range(5):
        assert owner2[k, 4 - k] == 0
    assert owner2[1, 1] == 0 and owner2[3, 3] == 1


def test_negative_zero_error_ties_with_zero():
    """An error of -0.0 is a valid e >= 0 and equals 0: in a cell whose free
    pixels all have zero error, the smallest index wins, whatever the sign bit."""
    m = np.zeros((6, 6), np.uint8)
    m[0, 0] = 1
    err = np.zeros((6, 6), np.float32)
    err[3, 3] = np.float32(-0.0)
    err[5, 5] = np.float32(-0.0)
    _, added, _ = od.densify_step(m, err, 1, "voronoi")
    assert list(added) == [1]
