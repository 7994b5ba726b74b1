"""Pins for the inpainting oracle: facts fixed by the paper and by the mathematics,
independent of the oracle's own code path (Sec. 2.1, eq. inp-discrete-lsi)."""
import json
import os

import numpy as np
import pytest

from oracle import inpaint as oi
from workloads import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_mask(rng, H, W, p):
    m = (rng.random((H, W)) < p).astype(np.uint8)
    if m.sum() == 0:
        m[rng.integers(H), rng.integers(W)] = 1
    return m


def test_laplacian_dct2_eigenpairs():
    """Sec. 2.1: the eigenvectors of L are the DCT-II basis images. That pins the
    reflecting boundary as the half-sample mirror (grid-graph Laplacian): a
    Dirichlet or whole-sample-mirror border fails this."""
    H, W = 7, 9
    L = oi.grid_laplacian(H, W)
    y, x = np.mgrid[0:H, 0:W]
    for k, l in [(0, 0), (1, 0), (0, 1), (3, 2), (W - 1, H - 1), (4, 6)]:
        v = (np.cos(np.pi * k * (x + 0.5) / W) * np.cos(np.pi * l * (y + 0.5) / H)).ravel()
        lam = 4 - 2 * np.cos(np.pi * k / W) - 2 * np.cos(np.pi * l / H)
        np.testing.assert_allclose(L @ v, lam * v, atol=1e-12)


def test_laplacian_structure():
    L = oi.grid_laplacian(5, 6).toarray()
    np.testing.assert_allclose(L, L.T)
    np.testing.assert_allclose(L.sum(axis=1), 0, atol=1e-14)
    # corner pixel has 2 neighbours, edge 3, interior 4
    assert L[0, 0] == 2 and L[1, 1] == 3 and L[7, 7] == 4


def test_full_mask_returns_f():
    rng = np.random.default_rng(0)
    f = rng.uniform(0, 255, (2, 6, 5))
    u = oi.inpaint(f, np.ones((6, 5), np.uint8))
    np.testing.assert_array_equal(u, f)


def test_constant_image_reproduced():
    rng = np.random.default_rng(1)
    m = _rand_mask(rng, 17, 23, 0.05)
    u = oi.inpaint(np.full((17, 23), 87.25), m)
    np.testing.assert_allclose(u, 87.25, rtol=0, atol=1e-10)


def test_single_pixel_gives_flat_image():
    """One known pixel: the solution is flat with that pixel's value (Sec. 2.1)."""
    f = np.random.default_rng(2).uniform(0, 255, (11, 13))
    m = np.zeros((11, 13), np.uint8)
    m[3, 8] = 1
    u = oi.inpaint(f, m)
    np.testing.assert_allclose(u[0], f[3, 8], atol=1e-10)


def test_1d_is_piecewise_linear_with_flat_ends():
    """H = 1: discrete Laplace between known samples is linear interpolation, and
    the reflecting boundary makes it constant beyond the first/last sample."""
    rng = np.random.default_rng(3)
    W = 61
    f = rng.uniform(0, 255, (1, W))
    m = np.zeros((1, W), np.uint8)
    pos = np.sort(rng.choice(np.arange(3, W - 3), 7, replace=False))
    m[0, pos] = 1
    u = oi.inpaint(f, m)[0, 0]
    ref = np.interp(np.arange(W), pos, f[0, pos])   # np.interp holds the end values
    np.testing.assert_allclose(u, ref, atol=1e-10)


def test_column_mask_reduces_to_1d():
    """Full known columns with column-constant data: every row is the 1D case."""
    rng = np.random.default_rng(4)
    H, W = 9, 40
    cols = np.array([5, 17, 18, 33])
    vals = rng.uniform(0, 255, W)
    f = np.tile(vals, (H, 1))
    m = np.zeros((H, W), np.uint8)
    m[:, cols] = 1
    u = oi.inpaint(f, m)[0]
    ref = np.interp(np.arange(W), cols, vals[cols])
    np.testing.assert_allclose(u, np.tile(ref, (H, 1)), atol=1e-10)


def test_dense_brute_force_agrees():
    """Reduced sparse solve vs dense solve of the full system A u = C f."""
    rng = np.random.default_rng(5)
    for H, W, p in [(8, 8, 0.1), (13, 29, 0.05), (1, 50, 0.1), (40, 1, 0.1), (2, 2, 0.3), (31, 33, 0.02)]:
        m = _rand_mask(rng, H, W, p)
        f = rng.uniform(0, 255, (2, H, W))
        np.testing.assert_allclose(oi.inpaint(f, m), oi.inpaint_dense(f, m), rtol=1e-10, atol=1e-9)


def test_min_max_principle_and_exact_mask_values():
    rng = np.random.default_rng(6)
    m = _rand_mask(rng, 40, 50, 0.03)
    f = rng.uniform(0, 255, (40, 50))
    u = oi.inpaint(f, m)[0]
    K = m != 0
    assert u.min() >= f[K].min() - 1e-9 and u.max() <= f[K].max() + 1e-9
    np.testing.assert_array_equal(u[K], f[K])


def test_linearity_and_channel_independence():
    rng = np.random.default_rng(7)
    m = _rand_mask(rng, 20, 24, 0.05)
    f1, f2 = rng.uniform(0, 255, (2, 20, 24))
    u = oi.inpaint(np.stack([f1, f2, 2.0 * f1 - 0.5 * f2]), m)
    np.testing.assert_allclose(u[2], 2.0 * u[0] - 0.5 * u[1], atol=1e-9)
    np.testing.assert_allclose(u[0], oi.inpaint(f1, m)[0], atol=1e-12)


def test_flip_and_transpose_equivariance():
    """Flipping or transposing image and mask together does the same to u; an
    index that mixes x and y, or an off-by-one border, breaks this."""
    rng = np.random.default_rng(8)
    m = _rand_mask(rng, 15, 22, 0.06)
    f = rng.uniform(0, 255, (15, 22))
    u = oi.inpaint(f, m)[0]
    np.testing.assert_allclose(oi.inpaint(f[:, ::-1], m[:, ::-1])[0], u[:, ::-1], atol=1e-9)
    np.testing.assert_allclose(oi.inpaint(f[::-1], m[::-1])[0], u[::-1], atol=1e-9)
    np.testing.assert_allclose(oi.inpaint(f.T.copy(), m.T.copy())[0], u.T, atol=1e-9)


def test_cg_fallback_matches_direct():
    rng = np.random.default_rng(9)
    m = _rand_mask(rng, 60, 70, 0.03)
    f = rng.uniform(0, 255, (60, 70))
    a = oi.inpaint(f, m, method="direct")
    b = oi.inpaint(f, m, method="cg")
    assert oi.rel_l2(b, a)[0] < 1e-10


def test_empty_mask_rejected():
    with pytest.raises(ValueError):
        oi.inpaint(np.zeros((4, 4)), np.zeros((4, 4), np.uint8))


def test_relres_zero_at_solution_and_positive_off_it():
    rng = np.random.default_rng(10)
    m = _rand_mask(rng, 30, 30, 0.05)
    f = rng.uniform(0, 255, (30, 30))
    u = oi.inpaint(f, m)
    assert oi.relres(u, f, m)[0] < 1e-12
    assert oi.relres(u + 1e-3 * rng.standard_normal(u.shape), f, m)[0] > 1e-8


def test_paper_density_convention():
    """Sec. 1.2 prints m ~ 400000 and ~640 GB for a 5% 4K mask; floor(d*N) with
    4-byte entries reproduces both."""
    g = json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))
    N = 3840 * 2160
    m = int(0.05 * N)
    assert m == 414720
    assert abs(m - g["mask_pixels_5pct_4k"]["approx_value"]) / 4e5 < 0.05
    assert abs(m * m * 4 / 2 ** 30 - g["dense_normal_matrix_gb_5pct_4k"]["approx_value_gb"]) < 5


def test_workload_generators_are_seeded_and_shaped():
    a, b = synth.config1(), synth.config1()
    np.testing.assert_array_equal(a.f, b.f)
    np.testing.assert_array_equal(a.mask, b.mask)
    assert a.f.shape == (1, 256, 256) and int(a.mask.sum()) == 3276
    assert a.f.min() >= 0 and a.f.max() <= 255
    inst = synth.config2(96, 160, 3, 0.03)
    assert inst.f.shape == (3, 96, 160)
    assert abs(inst.mask.mean() - 0.03) < 0.01
    np.testing.assert_array_equal(inst.f.astype(np.float32).astype(np.float64), inst.f)


def test_fs_dither_c_matches_python():
    rng = np.random.default_rng(11)
    p = rng.random((37, 53)) * 0.2
    np.testing.assert_array_equal(synth.fs_dither(p), synth._fs_python(p))


def test_relres_of_zero_is_one_per_channel():
    """The stopping measure is ||C f - A u|| / ||C f|| per channel (the relative
    residual of eq. inp-discrete-lsi): at u = 0 the residual is C f itself, so
    every channel gives exactly 1, whatever its scale."""
    rng = np.random.default_rng(12)
    m = _rand_mask(rng, 17, 23, 0.08)
    f = np.stack([rng.uniform(0, 255, (17, 23)), 1e-3 * rng.uniform(0, 1, (17, 23)), rng.uniform(50, 60, (17, 23))])
    assert np.array_equal(oi.relres(np.zeros_like(f), f, m), np.ones(3))


def test_relres_of_one_pixel_perturbation_by_hand():
    """u* + delta e_p at an unknown pixel p: A e_p has deg(p) in row p, -1 in the
    rows of p's unknown 4-neighbours and nothing on the mask rows (they are
    identity rows). So the residual norm is delta sqrt(deg(p)^2 + #unknown
    neighbours), divided by ||C f|| of that channel only; the other channels
    keep their (rounding-level) residual. A denominator of ||f||, or norms taken
    over all channels together, fail this."""
    H, W = 9, 11
    m = np.zeros((H, W), np.uint8)
    m[0, 0] = m[4, 8] = m[7, 2] = m[5, 5] = 1
    rng = np.random.default_rng(13)
    f = np.stack([rng.uniform(0, 255, (H, W)), rng.uniform(0, 255, (H, W))])
    u = oi.inpaint(f, m)
    delta = 0.5
    cases = [((5, 4), 4, 3),    # interior, right neighbour (5,5) known
             ((0, 1), 3, 2),    # top border, left neighbour (0,0) known
             ((8, 10), 2, 2)]   # corner
    for (y, x), deg, n_unknown in cases:
        assert m[y, x] == 0
        v = u.copy()
        v[1, y, x] += delta
        rr = oi.relres(v, f, m)
        cf = np.linalg.norm(f[1][m != 0])
        expect = delta * np.sqrt(deg * deg + n_unknown) / cf
        assert abs(rr[1] - expect) <= 1e-9 * expect
        assert rr[0] < 1e-12


def test_nested_dissection_is_a_permutation_and_solves_match():
    """The direct solver's fill-reducing order is a permutation of the pixels, and
    the solution does not depend on it (compared with SuperLU's own column order)."""
    import scipy.sparse.linalg as spla
    for H, W in [(1, 1), (1, 37), (29, 1), (17, 23), (64, 65)]:
        p = oi.nested_dissection(H, W)
        assert np.array_equal(np.sort(p), np.arange(H * W))
    rng = np.random.default_rng(14)
    m = _rand_mask(rng, 41, 53, 0.04)
    f = rng.uniform(0, 255, (41, 53))
    rs = oi.ReducedSystem(m)
    b = -(rs.LUK @ f.ravel()[rs.K])
    ref = spla.splu(rs.LUU.tocsc()).solve(b)
    np.testing.assert_allclose(rs.solve_UU(b), ref, rtol=0, atol=1e-10 * np.abs(ref).max())
