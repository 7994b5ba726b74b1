"""Pins for the tonal-optimisation oracle (Sec. 5, eqs. tonal-opt-minimisation and
tonal-normal-equations): closed forms, brute force and the optimality certificate."""
import numpy as np

from oracle import inpaint as oi
from oracle import tonal as ot


def _rand_mask(rng, H, W, p):
    m = (rng.random((H, W)) < p).astype(np.uint8)
    if m.sum() == 0:
        m[rng.integers(H), rng.integers(W)] = 1
    return m


def test_full_mask_returns_f_with_zero_error():
    rng = np.random.default_rng(0)
    f = rng.uniform(0, 255, (7, 9))
    m = np.ones((7, 9), np.uint8)
    g = ot.tonal_optimize(f, m)
    np.testing.assert_allclose(g[0], f, atol=1e-9)
    assert ot.mse(g, f, m) < 1e-18


def test_constant_image():
    rng = np.random.default_rng(1)
    m = _rand_mask(rng, 20, 25, 0.05)
    f = np.full((20, 25), 42.0)
    g = ot.tonal_optimize(f, m)
    np.testing.assert_allclose(g[0][m != 0], 42.0, atol=1e-9)
    assert np.all(g[0][m == 0] == 0)
    assert ot.mse(g, f, m) < 1e-18


def test_single_pixel_gives_mean_and_variance():
    """One known pixel reconstructs a flat image, so the best value is the mean
    of f and the error is its population variance."""
    f = np.random.default_rng(2).uniform(0, 255, (12, 10))
    m = np.zeros((12, 10), np.uint8)
    m[5, 2] = 1
    g = ot.tonal_optimize(f, m)
    assert abs(g[0, 5, 2] - f.mean()) < 1e-9
    assert abs(ot.mse(g, f, m) - f.var()) < 1e-8


def test_1d_is_least_squares_linear_spline_fit():
    """H = 1: B's columns are hat functions over the mask positions with flat
    ends (piecewise-linear interpolation), so g* is the least-squares fit of f in
    that spline space. The basis is built with np.interp, not with the oracle."""
    rng = np.random.default_rng(3)
    W = 80
    f = rng.uniform(0, 255, W)
    pos = np.sort(rng.choice(W, 9, replace=False))
    m = np.zeros((1, W), np.uint8)
    m[0, pos] = 1
    basis = np.stack([np.interp(np.arange(W), pos, np.eye(len(pos))[j]) for j in range(len(pos))], axis=1)
    ref = np.linalg.lstsq(basis, f, rcond=None)[0]
    g = ot.tonal_optimize(f[None], m)[0, 0]
    np.testing.assert_allclose(g[pos], ref, atol=1e-8)
    # the normal matrix of hat functions is tridiagonal
    BtB = basis.T @ basis
    assert np.all(np.abs(np.triu(BtB, 2)) < 1e-12)


def test_dense_lstsq_agrees():
    rng = np.random.default_rng(4)
    for H, W, p in [(8, 9, 0.15), (16, 16, 0.05), (30, 31, 0.04), (1, 40, 0.2), (3, 3, 0.4)]:
        m = _rand_mask(rng, H, W, p)
        f = rng.uniform(0, 255, (2, H, W))
        g = ot.tonal_optimize(f, m)
        gd = ot.tonal_dense(f, m)
        np.testing.assert_allclose(g, gd, rtol=1e-8, atol=1e-7)


def test_normal_matrix_lambda_min_at_least_one():
    """On the mask entries B^T B = I + H^T H, so its smallest eigenvalue is >= 1;
    this is what makes the certificate ||g - g*|| <= ||B^T(f - B g)|| valid."""
    rng = np.random.default_rng(5)
    m = _rand_mask(rng, 14, 15, 0.08)
    K = m.ravel() != 0
    A = oi.system_matrix(m).toarray()
    Bd = np.linalg.solve(A, np.eye(m.size)[:, K])
    lam = np.linalg.eigvalsh(Bd.T @ Bd)
    assert lam.min() >= 1 - 1e-12
    f = rng.uniform(0, 255, (14, 15))
    gs = ot.tonal_optimize(f, m)
    g = gs.copy()
    g[0][m != 0] += rng.standard_normal(int(K.sum()))
    assert np.linalg.norm(g - gs) <= ot.error_bound(g, f, m)[0] + 1e-9


def test_bt_definition_matches_reduced_gather():
    """B^T y = C A^{-T} y equals y_K + sum over unknown 4-neighbours j of z_j,
    with L_UU z_U = y_U (the symmetrised form of Sec. 5.1)."""
    rng = np.random.default_rng(6)
    m = _rand_mask(rng, 11, 13, 0.1)
    y = rng.standard_normal(m.size)
    direct = ot.TonalOperator(m, "direct").Bt(y)
    reduced = ot.TonalOperator(m, "cg").Bt(y)
    np.testing.assert_allclose(direct, reduced, atol=1e-9)
    np.testing.assert_allclose(direct, ot.TonalOperator(m, "reduced").Bt(y), atol=1e-11)
    g = rng.standard_normal(m.size) * (m.ravel() != 0)
    np.testing.assert_allclose(ot.TonalOperator(m, "direct").B(g), ot.TonalOperator(m, "reduced").B(g), atol=1e-11)
    # several channels as columns give the same as one at a time
    Y = rng.standard_normal((m.size, 3))
    op = ot.TonalOperator(m, "reduced")
    np.testing.assert_allclose(op.Bt(Y), np.stack([op.Bt(Y[:, j]) for j in range(3)], 1), atol=1e-12)
    # gather written out by neighbours
    rs = oi.ReducedSystem(m)
    z = np.zeros(m.size)
    z[rs.U] = rs.solve_UU(y[rs.U])
    H, W = m.shape
    g = np.zeros(m.size)
    for i in np.flatnonzero(rs.K):
        yy, xx = divmod(i, W)
        s = y[i]
        for dy, dx in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            qy, qx = yy + dy, xx + dx
            if 0 <= qy < H and 0 <= qx < W and not rs.K[qy * W + qx]:
                s += z[qy * W + qx]
        g[i] = s
    np.testing.assert_allclose(direct, g, atol=1e-9)


def test_optimum_beats_perturbations_and_plain_values():
    rng = np.random.default_rng(7)
    m = _rand_mask(rng, 24, 24, 0.05)
    f = rng.uniform(0, 255, (24, 24))
    g = ot.tonal_optimize(f, m)
    best = ot.mse(g, f, m)
    assert best <= ot.mse(f * (m != 0), f, m) + 1e-12
    for _ in range(3):
        d = np.zeros_like(g)
        d[0][m != 0] = rng.standard_normal(int(m.sum()))
        assert best < ot.mse(g + 0.1 * d, f, m)
    assert ot.normal_residual(g, f, m)[0] < 1e-10


def test_cg_path_matches_direct_path():
    rng = np.random.default_rng(8)
    m = _rand_mask(rng, 40, 33, 0.04)
    f = rng.uniform(0, 255, (40, 33))
    a = ot.tonal_optimize(f, m, method="direct")
    b = ot.tonal_optimize(f, m, method="cg")
    np.testing.assert_allclose(a, b, atol=1e-7)


def test_psnr_closed_form():
    """PSNR = 10 log10(255^2 / MSE) (the quality measure reported beside the MSE
    in Sec. 6.3): an MSE of 255^2 / 100 is 20 dB, each 10x smaller MSE adds 10 dB."""
    assert abs(ot.psnr(255.0 ** 2 / 100) - 20.0) < 1e-12
    assert abs(ot.psnr(255.0 ** 2 / 1000) - 30.0) < 1e-12


def test_normal_residual_of_zero_is_one():
    """At g = 0 the normal residual B^T (f - B g) is B^T f itself, so the relative
    measure is exactly 1 per channel."""
    rng = np.random.default_rng(20)
    m = _rand_mask(rng, 13, 17, 0.1)
    f = np.stack([rng.uniform(0, 255, (13, 17)), 1e-2 * rng.uniform(0, 1, (13, 17))])
    nr = ot.normal_residual(np.zeros_like(f), f, m)
    np.testing.assert_allclose(nr, 1.0, rtol=1e-14)


def test_normal_residual_closed_forms():
    """Two masks where B is known in closed form (Sec. 5):
    - full mask: B = I, so B^T (f - B g) = f - g and the measure is ||f - g|| / ||f||;
    - one mask pixel k: B g is the constant image g_k and B^T y is the sum of y
      placed at k, so the measure is |mean f - g_k| / |mean f|.
    A residual taken before applying B^T (||f - B g|| / ||f||) fails the second."""
    rng = np.random.default_rng(21)
    f = rng.uniform(0, 255, (6, 8))
    full = np.ones((6, 8), np.uint8)
    g = f + rng.standard_normal(f.shape)
    expect = np.linalg.norm(f - g) / np.linalg.norm(f)
    np.testing.assert_allclose(ot.normal_residual(g, f, full), [expect], rtol=1e-12)
    one = np.zeros((6, 8), np.uint8)
    one[2, 5] = 1
    g = np.zeros_like(f)
    g[2, 5] = 17.0
    expect = abs(f.mean() - 17.0) / abs(f.mean())
    np.testing.assert_allclose(ot.normal_residual(g, f, one), [expect], rtol=1e-10)
    # and the error bound there is N |mean f - g_k| (||B^T y|| = |sum y|)
    np.testing.assert_allclose(ot.error_bound(g, f, one), [f.size * abs(f.mean() - 17.0)], rtol=1e-10)


def test_certificate_bounds_the_true_error_of_perturbed_optima():
    """certificate(): against the brute-force optimum (dense lstsq) of a small
    RGB image, for g = g* + d with d on the mask:
    - steps = 0 gives ||r|| with r = B^T (f - B g), and it bounds ||d||;
    - more CG steps tighten the bound but never below ||d||;
    - with as many steps as mask pixels the bound is ||d|| itself;
    - the MSE excess d^T (B^T B) d / (C N) (computed densely) stays below its bound.
    A bound that dropped the residual term of the estimate, or used B instead of
    B^T B, falls below ||d|| for some of these perturbations."""
    rng = np.random.default_rng(31)
    H, W = 14, 17
    m = _rand_mask(rng, H, W, 0.08)
    f = rng.uniform(0, 255, (3, H, W))
    gs = ot.tonal_dense(f, m)
    K = m.ravel() != 0
    A = oi.system_matrix(m).toarray()
    Bd = np.linalg.solve(A, np.eye(m.size)[:, K])
    M = Bd.T @ Bd
    for scale, kind in [(1e-3, "smooth"), (1e-1, "rough")]:
        d = np.zeros_like(gs)
        for c in range(3):
            v = rng.standard_normal(int(K.sum()))
            if kind == "smooth":   # along the smallest eigenvectors of M (slow to resolve)
                w, V = np.linalg.eigh(M)
                v = V[:, :3] @ rng.standard_normal(3)
            d[c].ravel()[K] = scale * v
        g = gs + d
        dn = np.array([np.linalg.norm(d[c].ravel()[K]) for c in range(3)])
        c0 = ot.certificate(g, f, m)
        rK = np.stack([Bd.T @ (f[c].ravel() - Bd @ g[c].ravel()[K]) for c in range(3)], axis=1)
        np.testing.assert_allclose(c0["normal_residual"], np.linalg.norm(rK, axis=0), rtol=1e-8)
        np.testing.assert_allclose(c0["error_bound"], c0["normal_residual"], rtol=0)
        assert np.all(c0["error_bound"] >= dn * (1 - 1e-9))
        prev = c0["error_bound"]
        for steps in (1, 3, 8):
            ck = ot.certificate(g, f, m, steps=steps)
            assert np.all(ck["error_bound"] >= dn * (1 - 1e-9)), (steps, ck["error_bound"], dn)
            assert np.all(ck["error_bound"] <= prev * (1 + 1e-12))
        full = ot.certificate(g, f, m, steps=int(K.sum()) + 5)
        np.testing.assert_allclose(full["error_bound"], dn, rtol=1e-6)
        excess = sum(d[c].ravel()[K] @ M @ d[c].ravel()[K] for c in range(3)) / f.size
        assert excess <= full["mse_excess_bound"] * (1 + 1e-9)
        assert excess <= c0["mse_excess_bound"] * (1 + 1e-9)
        # (a difference of two MSEs near 1e3: absolute rounding about 1e-12)
        np.testing.assert_allclose(ot.mse(g, f, m) - ot.mse(gs, f, m), excess, rtol=1e-6, atol=1e-10)


def test_tonal_operator_reuses_a_factored_system():
    """A TonalOperator built on a given ReducedSystem applies the same B and B^T
    as one that factors its own; a system of another mask is refused."""
    rng = np.random.default_rng(32)
    m = _rand_mask(rng, 30, 41, 0.05)
    rs = oi.ReducedSystem(m)
    a = ot.TonalOperator(m, system=rs)
    b = ot.TonalOperator(m, method="direct")
    y = rng.standard_normal((m.size, 3))
    np.testing.assert_allclose(a.B(y), b.B(y), rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(a.Bt(y), b.Bt(y), rtol=1e-10, atol=1e-9)
    other = m.copy()
    other[0, 0] ^= 1
    try:
        ot.TonalOperator(other, system=rs)
    except ValueError:
        pass
    else:
        raise AssertionError("a system of another mask was accepted")
