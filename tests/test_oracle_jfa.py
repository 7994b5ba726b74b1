"""Pins for the jump-flooding labels of the densification oracle (Sec. 4.2,
readings J1-J3): exactness where jump flooding is provably exact, tie order and
the nine offsets on a lattice where one unit pass decides everything, the
bound against the exact labels, a small disagreement rate on random masks, and
the start-step rules."""
import numpy as np
import pytest

from oracle import densify as od


@pytest.mark.parametrize("shape,seed", [((37, 53), (5, 40)), ((64, 64), (0, 0)), ((1, 77), (0, 76)), ((90, 1), (45, 0)),
                                        ((129, 65), (128, 64))])
def test_one_seed_reaches_every_pixel(shape, seed):
    H, W = shape
    m = np.zeros(shape, np.uint8)
    m[seed] = 1
    lab = od.jfa_labels(m)
    assert np.all(lab == seed[0] * W + seed[1])


def test_one_unit_pass_on_a_spacing_two_lattice_is_exact():
    """Every pixel has a mask pixel among its 3x3 neighbours, so a single pass
    with step 1 must find the exact label, ties included (the diagonal
    neighbours decide the odd-odd pixels, four-way ties go to the smallest
    index)."""
    H, W = 11, 14
    m = np.zeros((H, W), np.uint8)
    m[::2, ::2] = 1
    lab = od.jfa_labels(m, k0=1)
    np.testing.assert_array_equal(lab, od.voronoi_labels(m, "brute"))
    # the pixel (1, 1) is equidistant from four lattice points; the smallest index wins
    assert lab[1, 1] == 0


@pytest.mark.parametrize("density", [0.005, 0.02, 0.08, 0.3])
def test_bounded_disagreement_with_exact_labels(density):
    rng = np.random.default_rng(int(density * 1000))
    H, W = 97, 131
    m = (rng.random((H, W)) < density).astype(np.uint8)
    m[rng.integers(H), rng.integers(W)] = 1
    lab = od.jfa_labels(m)
    ex = od.voronoi_labels(m)
    yy, xx = np.mgrid[0:H, 0:W]
    d = lambda L: np.sqrt((L // W - yy) ** 2.0 + (L % W - xx) ** 2.0)
    assert np.all(m.ravel()[lab.ravel()] == 1)                        # labels are mask pixels
    seeds = np.flatnonzero(m.ravel())
    assert np.all(lab.ravel()[seeds] == seeds)                        # seeds keep their own label
    dj, de = d(lab), d(ex)
    assert np.all(dj >= de - 1e-12)                                  # never closer than the nearest
    tie = np.isclose(dj, de)
    assert np.all(lab[tie & (lab != ex)] > ex[tie & (lab != ex)])     # equal distance: exact has the smaller index
    wrong = lab != ex
    assert wrong.mean() < 0.01, wrong.mean()
    assert np.all(dj - de <= 2.0)


def test_start_step_rules():
    assert [od.jfa_default_step(1, n) for n in (1, 2, 3, 4, 5, 3840)] == [0, 1, 2, 2, 4, 2048]
    assert [od.jfa_next_step(d2) for d2 in (0, 1, 2, 4, 5, 16, 17)] == [1, 1, 2, 2, 4, 4, 8]
    # the shrinking start finds the same labels once the mask has grown
    rng = np.random.default_rng(9)
    m = (rng.random((60, 80)) < 0.02).astype(np.uint8)
    m[0, 0] = 1
    k = od.jfa_next_step(od.label_max_d2(od.jfa_labels(m)))
    m2 = m | (rng.random(m.shape) < 0.02).astype(np.uint8)
    a, b = od.jfa_labels(m2), od.jfa_labels(m2, k)
    assert (a != b).mean() < 0.01


def test_densify_with_labels_that_equal_the_exact_ones():
    rng = np.random.default_rng(10)
    H, W = 11, 14
    m = np.zeros((H, W), np.uint8)
    m[::2, ::2] = 1
    err = rng.random((H, W)).astype(np.float32)
    a = od.densify_step(m, err, 9)
    b = od.densify_step(m, err, 9, labels=od.jfa_labels(m, k0=1))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
