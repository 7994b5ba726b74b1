"""Oracle: tonal optimisation (test infrastructure only).

Paper Sec. 5, eq. (tonal-opt-minimisation): for a fixed mask, the inpainting
operator B = A^{-1} C is linear in the stored values, and tonal optimisation
finds

    g* = argmin_g || f - B g ||_2^2,   g_i = 0 for i not in K,

whose minimiser satisfies the normal equations (eq. tonal-normal-equations)
B^T B g = B^T f. Restricted to the mask entries this matrix is the identity
plus a positive semi-definite term, so the minimiser is unique for a non-empty
mask (Sec. 1) and every method converges to the same values (Sec. 6.3).

B g and B^T y are applied by their definitions, B g = A^{-1}(C g) and
B^T y = C A^{-T} y, with one SuperLU factorisation of A reused for both.
For grids too large for that factorisation the symmetric reduced form is used
instead (Sec. 5.1, symmetrised system): B g equals g on K and solves
L_UU u_U = -L_UK g_K on U, and B^T y equals y_K - L_KU z_U on K with
L_UU z_U = y_U, solved with one factorisation of L_UU (or, on request, by
conjugate gradients to a tight tolerance).

The operators take one channel as a length-N vector or several channels as the
columns of an N x C array; the channels never mix.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .inpaint import DIRECT_LIMIT, ReducedSystem, _as_chw, _check_mask, system_matrix


class TonalOperator:
    """B and B^T for one mask, acting on flat length-N vectors or N x C arrays.
    method: "direct" (factor A itself), "reduced" (factor L_UU), "cg" (reduced
    form with conjugate gradients), "auto" (direct up to DIRECT_LIMIT pixels)."""

    def __init__(self, mask: np.ndarray, method: str = "auto", system: ReducedSystem | None = None):
        self.shape = mask.shape
        self.K = _check_mask(mask)
        self.c = self.K.astype(np.float64)
        N = mask.size
        if system is not None:
            # reuse a factorised reduced system of this same mask
            if system.H * system.W != N or not np.array_equal(system.K, self.K):
                raise ValueError("the given reduced system belongs to another mask")
            self.method = "cg" if system.lu is None else "reduced"
            self.rs = system
            return
        if method == "auto":
            method = "direct" if N <= DIRECT_LIMIT else "reduced"
        self.method = method
        if method == "direct":
            self.lu = spla.splu(system_matrix(mask).tocsc())
        else:
            self.rs = ReducedSystem(mask, "cg" if method == "cg" else "direct")

    def _cols(self, fn, x):
        # the CG fallback solves one right-hand side at a time
        if x.ndim == 1 or self.method != "cg":
            return fn(x)
        return np.stack([fn(x[:, j]) for j in range(x.shape[1])], axis=1)

    def B(self, g: np.ndarray) -> np.ndarray:
        """u = A^{-1} C g."""
        if self.method == "direct":
            cg = self.c * g if g.ndim == 1 else self.c[:, None] * g
            return self.lu.solve(np.ascontiguousarray(cg))
        rs = self.rs
        u = np.zeros_like(g, dtype=np.float64)
        u[rs.K] = g[rs.K]
        u[rs.U] = self._cols(rs.solve_UU, -(rs.LUK @ g[rs.K]))
        return u

    def Bt(self, y: np.ndarray) -> np.ndarray:
        """C A^{-T} y (zero off the mask)."""
        if self.method == "direct":
            z = self.lu.solve(np.ascontiguousarray(y, dtype=np.float64), trans="T")
            return self.c * z if z.ndim == 1 else self.c[:, None] * z
        rs = self.rs
        z = np.zeros_like(y, dtype=np.float64)
        zU = self._cols(rs.solve_UU, np.ascontiguousarray(y[rs.U], dtype=np.float64))
        z[rs.K] = y[rs.K] - rs.LKU @ zU
        return z

    def normal(self, gK: np.ndarray) -> np.ndarray:
        """(B^T B) restricted to the mask entries."""
        g = np.zeros((self.K.size,) + gK.shape[1:])
        g[self.K] = gK
        return self.Bt(self.B(g))[self.K]


def _cg(matvec, rhs, x0, rtol, maxiter):
    """Textbook conjugate gradients for a symmetric positive definite operator.
    rhs and x0 may hold several independent systems as columns: each column
    keeps its own step sizes and stops on its own residual."""
    x = x0.copy()
    r = rhs - matvec(x)
    p = r.copy()
    rr = (r * r).sum(axis=0)
    stop = (rtol * np.sqrt((rhs * rhs).sum(axis=0))) ** 2
    it = 0
    while np.any(rr > stop) and it < maxiter:
        act = rr > stop                       # columns still iterating
        q = matvec(p)
        a = np.where(act, rr / np.where(act, (p * q).sum(axis=0), 1.0), 0.0)
        x += a * p
        r -= a * q
        rr_new = (r * r).sum(axis=0)
        p = r + np.where(act, rr_new / np.where(act, rr, 1.0), 0.0) * p
        rr = np.where(act, rr_new, rr)
        it += 1
    return x, it


def tonal_optimize(f: np.ndarray, mask: np.ndarray, rtol: float = 1e-12, maxiter: int = 5000,
                   method: str = "auto") -> np.ndarray:
    """g* per channel by CG on the normal equations restricted to K, started at
    g = f on K (the usual start, Sec. 5.3). The channels are independent
    systems, iterated side by side. Returns (C,H,W) with zeros off K."""
    f = _as_chw(f)
    op = TonalOperator(mask, method)
    F = np.stack([fc.ravel() for fc in f], axis=1)          # N x C
    rhs = op.Bt(F)[op.K]
    gK, _ = _cg(op.normal, rhs, F[op.K].copy(), rtol, maxiter)
    g = np.zeros_like(F)
    g[op.K] = gK
    return np.stack([g[:, c].reshape(mask.shape) for c in range(f.shape[0])])


def tonal_dense(f: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Brute force for tiny images: B = A^{-1} C[:, K] as a dense matrix, then
    numpy.linalg.lstsq(B, f) per channel."""
    f = _as_chw(f)
    K = _check_mask(mask)
    if mask.size > 4096:
        raise ValueError("dense brute force is for N <= 4096")
    A = system_matrix(mask).toarray()
    Bd = np.linalg.solve(A, np.eye(mask.size)[:, K])
    out = []
    for fc in f:
        gK = np.linalg.lstsq(Bd, fc.ravel(), rcond=None)[0]
        g = np.zeros(mask.size)
        g[K] = gK
        out.append(g.reshape(mask.shape))
    return np.stack(out)


def reconstruct(g: np.ndarray, mask: np.ndarray, method: str = "auto") -> np.ndarray:
    """B g per channel, (C,H,W)."""
    g = _as_chw(g)
    op = TonalOperator(mask, method)
    u = op.B(np.stack([gc.ravel() for gc in g], axis=1))
    return np.stack([u[:, c].reshape(mask.shape) for c in range(g.shape[0])])


def mse(g: np.ndarray, f: np.ndarray, mask: np.ndarray, method: str = "auto") -> float:
    """||f - B g||^2 / (C N) over all channels (the paper's error measure)."""
    f = _as_chw(f)
    u = reconstruct(g, mask, method)
    return float(((f - u) ** 2).sum() / f.size)


def psnr(m: float) -> float:
    """10 log10(255^2 / MSE)."""
    return float(10.0 * np.log10(255.0 ** 2 / m))


def _normal_parts(g, f, mask, method):
    g, f = _as_chw(g), _as_chw(f)
    op = TonalOperator(mask, method)
    G = np.stack([gc.ravel() for gc in g], axis=1)
    F = np.stack([fc.ravel() for fc in f], axis=1)
    return op, G, F


def normal_residual(g: np.ndarray, f: np.ndarray, mask: np.ndarray, method: str = "auto") -> np.ndarray:
    """||B^T (f - B g)|| / ||B^T f|| per channel (relative normal-equation residual)."""
    op, G, F = _normal_parts(g, f, mask, method)
    r = np.linalg.norm(op.Bt(F - op.B(G)), axis=0)
    return r / np.maximum(np.linalg.norm(op.Bt(F), axis=0), 1e-300)


def error_bound(g: np.ndarray, f: np.ndarray, mask: np.ndarray, method: str = "auto") -> np.ndarray:
    """Certificate: on K, B^T B = I + (positive semi-definite), so its smallest
    eigenvalue is at least 1 and ||g - g*|| <= ||B^T (f - B g)|| per channel."""
    op, G, F = _normal_parts(g, f, mask, method)
    return np.linalg.norm(op.Bt(F - op.B(G)), axis=0)


def certificate(g: np.ndarray, f: np.ndarray, mask: np.ndarray, steps: int = 0,
                op: TonalOperator | None = None) -> dict:
    """Rigorous bounds on the distance of g from the optimum g*, per channel.

    With M = B^T B restricted to K (smallest eigenvalue at least 1) and the
    normal residual r = B^T (f - B g) on K, the error e = g - g* solves
    M e = -r. For any estimate e_h of e, ||e - e_h|| <= ||M (e - e_h)||
    = ||-r - M e_h||, hence ||e|| <= ||e_h|| + ||r + M e_h||. With steps = 0
    (e_h = 0) this is the plain bound ||e|| <= ||r||; steps > 0 takes e_h from
    that many conjugate-gradient steps on M e_h = -r started at zero, which
    tightens the bound when r is dominated by large eigenvalues of M.

    The MSE excess follows from e^T M e = r^T M^{-1} r <= ||r|| ||e||:
    MSE(g) - MSE(g*) <= sum_c ||r_c|| E_c / (C N), with E_c the error bound.

    Returns per-channel arrays 'normal_residual' (||r||), 'error_bound' (E),
    'g_norm' (||g_K||) and the scalar 'mse_excess_bound'."""
    f, g = _as_chw(f), _as_chw(g)
    if op is None:
        op = TonalOperator(mask)
    G = np.stack([gc.ravel() for gc in g], axis=1)
    F = np.stack([fc.ravel() for fc in f], axis=1)
    r = op.Bt(F - op.B(G))[op.K]
    rn = np.linalg.norm(r, axis=0)
    E = rn.copy()
    if steps > 0:
        eh, _ = _cg(op.normal, -r, np.zeros_like(r), 0.0, steps)
        E = np.minimum(E, np.linalg.norm(eh, axis=0) + np.linalg.norm(r + op.normal(eh), axis=0))
    return {"normal_residual": rn, "error_bound": E, "g_norm": np.linalg.norm(G[op.K], axis=0),
            "mse_excess_bound": float((rn * E).sum() / F.size)}
