"""Oracle: homogeneous diffusion inpainting (test infrastructure only).

Paper Sec. 2.1, eq. (inp-discrete-lsi): with mask c in {0,1}^N, C = diag(c)
and L the 5-point negated Laplacian with reflecting boundary conditions, the
reconstruction u solves

    A u = b,   A = C + (I - C) L,   b = C f.

Reading of "reflecting boundary conditions" (Sec. 2.1, the DCT-II remark):
L is the Laplacian of the 4-neighbour grid graph with unit grid spacing,
(L u)_p = sum_{q in N4(p)} (u_p - u_q) over in-image neighbours q. Its
eigenvectors are the separable DCT-II basis images, which is what the paper
states; the tests check that.

A is non-singular iff the mask is non-empty (Sec. 2.1). Colour images are
inpainted channel by channel with the same matrix (Sec. 2.1).

Functions here build the matrices from their definitions and solve them with
SciPy's sparse direct solver (SuperLU) or, on request, with plain conjugate
gradients on the symmetric reduced system to a tight tolerance. The direct
solver factors the reduced system with its unknowns numbered by nested
dissection of the pixel grid (a fill-reducing order: the solution is the same
for any numbering, up to rounding), which keeps 4K factorisations within
minutes and a few GB.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DIRECT_LIMIT = 600_000     # pixels above which the tonal operator uses the reduced system


def grid_laplacian(H: int, W: int) -> sp.csr_matrix:
    """L = D - Adj of the 4-neighbour grid graph of an H x W image (row-major,
    index i = y*W + x). Each edge {p, q} adds +1 to (p,p), (q,q) and -1 to (p,q), (q,p)."""
    idx = np.arange(H * W, dtype=np.int64).reshape(H, W)
    a = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    b = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    rows = np.concatenate([a, b, a, b])
    cols = np.concatenate([b, a, a, b])
    vals = np.concatenate([-np.ones(2 * len(a)), np.ones(2 * len(a))])
    return sp.csr_matrix((vals, (rows, cols)), shape=(H * W, H * W))


def system_matrix(mask: np.ndarray) -> sp.csr_matrix:
    """A = C + (I - C) L for a mask of shape (H, W)."""
    H, W = mask.shape
    c = (mask.ravel() != 0).astype(np.float64)
    L = grid_laplacian(H, W)
    return (sp.diags(c) + sp.diags(1.0 - c) @ L).tocsr()


def _as_chw(f: np.ndarray) -> np.ndarray:
    f = np.asarray(f, dtype=np.float64)
    return f[None] if f.ndim == 2 else f


def _check_mask(mask: np.ndarray) -> np.ndarray:
    K = np.asarray(mask).ravel() != 0
    if not K.any():
        raise ValueError("empty mask: A = L is singular (Sec. 2.1)")
    return K


def nested_dissection(H: int, W: int, leaf: int = 64) -> np.ndarray:
    """A permutation of the H*W pixel indices: split the rectangle across its
    longer side, number both halves recursively, then the separating grid line;
    rectangles of at most `leaf` pixels are numbered row by row."""
    out = []

    def rec(y0, y1, x0, x1):
        h, w = y1 - y0, x1 - x0
        if h <= 0 or w <= 0:
            return
        if h * w <= leaf:
            yy, xx = np.mgrid[y0:y1, x0:x1]
            out.append((yy * W + xx).ravel())
        elif w >= h:
            xm = (x0 + x1) // 2
            rec(y0, y1, x0, xm)
            rec(y0, y1, xm + 1, x1)
            out.append(np.arange(y0, y1) * W + xm)
        else:
            ym = (y0 + y1) // 2
            rec(y0, ym, x0, x1)
            rec(ym + 1, y1, x0, x1)
            out.append(ym * W + np.arange(x0, x1))

    rec(0, H, 0, W)
    return np.concatenate(out).astype(np.int64)


class _OrderedLU:
    """SuperLU factors of P^T M P for a symmetric positive definite M and the
    permutation P given as an index array; solve() returns M^{-1} b. Diagonal
    pivots (no row exchanges), since M is SPD."""

    def __init__(self, M: sp.spmatrix, perm: np.ndarray):
        self.perm = perm
        Mp = M.tocsr()[perm][:, perm].tocsc()
        self.lu = spla.splu(Mp, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))

    def solve(self, b: np.ndarray) -> np.ndarray:
        y = self.lu.solve(np.ascontiguousarray(b[self.perm], dtype=np.float64))
        x = np.empty_like(y)
        x[self.perm] = y
        return x


class ReducedSystem:
    """The unknowns of A x = b are the non-mask pixels U; rows on K pin x_K = b_K.
    Eliminating them gives L_UU x_U = b_U - L_UK x_K, symmetric positive definite
    for a non-empty mask. Factor once per mask, solve many right-hand sides."""

    def __init__(self, mask: np.ndarray, method: str = "auto"):
        self.H, self.W = mask.shape
        self.K = _check_mask(mask)
        self.U = ~self.K
        L = grid_laplacian(self.H, self.W)
        Lr = L[self.U]
        self.LUU = Lr[:, self.U].tocsc()
        self.LUK = Lr[:, self.K].tocsr()
        self.LKU = L[self.K][:, self.U].tocsr()
        nU = int(self.U.sum())
        if method == "auto":
            method = "direct"
        self.method = method
        self.lu = None
        if method == "direct" and nU > 0:
            # unknowns in nested-dissection order of the full grid
            pos = np.full(self.H * self.W, -1, np.int64)
            pos[np.flatnonzero(self.U)] = np.arange(nU)
            nd = nested_dissection(self.H, self.W)
            self.lu = _OrderedLU(self.LUU, pos[nd[self.U[nd]]])
        self.dinv = 1.0 / self.LUU.diagonal() if nU > 0 else None

    def solve_UU(self, rhs: np.ndarray, rtol: float = 1e-13) -> np.ndarray:
        """x_U with L_UU x_U = rhs; rhs may hold several right-hand sides as
        columns (direct method)."""
        if rhs.size == 0:
            return rhs.copy()
        if self.lu is not None:
            return self.lu.solve(rhs)
        M = spla.LinearOperator(self.LUU.shape, matvec=lambda v: self.dinv * v)
        x, info = spla.cg(self.LUU, rhs, rtol=rtol, atol=0.0, maxiter=200_000, M=M)
        if info != 0:
            raise RuntimeError(f"oracle CG did not converge (info={info})")
        return x

    def solve(self, data: np.ndarray, source: np.ndarray | None = None) -> np.ndarray:
        """Solve A x = C data + (I - C) source for one channel (flat arrays).
        source=None means zero (plain inpainting)."""
        x = np.zeros(self.H * self.W)
        x[self.K] = data[self.K]
        rhs = -(self.LUK @ data[self.K])
        if source is not None:
            rhs = rhs + source[self.U]
        x[self.U] = self.solve_UU(rhs)
        return x


def inpaint(f: np.ndarray, mask: np.ndarray, method: str = "auto") -> np.ndarray:
    """u = A^{-1} C f per channel (Sec. 2.1). f: (H,W) or (C,H,W); returns (C,H,W)."""
    f = _as_chw(f)
    rs = ReducedSystem(mask, method)
    return np.stack([rs.solve(fc.ravel()).reshape(mask.shape) for fc in f])


def inpaint_dense(f: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Brute force for tiny images: dense numpy.linalg.solve(A, C f)."""
    f = _as_chw(f)
    _check_mask(mask)
    H, W = mask.shape
    if H * W > 4096:
        raise ValueError("dense brute force is for N <= 4096")
    A = system_matrix(mask).toarray()
    c = (mask.ravel() != 0).astype(np.float64)
    return np.stack([np.linalg.solve(A, c * fc.ravel()).reshape(H, W) for fc in f])


def residual_norms(u: np.ndarray, f: np.ndarray, mask: np.ndarray):
    """Per channel (||C f - A u||_2, ||C f||_2) in float64, A applied exactly."""
    u, f = _as_chw(u), _as_chw(f)
    A = system_matrix(mask)
    c = (mask.ravel() != 0).astype(np.float64)
    out = []
    for uc, fc in zip(u, f):
        b = c * fc.ravel()
        out.append((float(np.linalg.norm(b - A @ uc.ravel())), float(np.linalg.norm(b))))
    return out


def relres(u: np.ndarray, f: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Relative residual ||C f - A u|| / ||C f|| per channel (the stopping measure)."""
    return np.array([r / b if b > 0 else r for r, b in residual_norms(u, f, mask)])


def rel_l2(x: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """||x - ref|| / ||ref|| per channel."""
    x, ref = _as_chw(x), _as_chw(ref)
    return np.array([np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300) for a, b in zip(x, ref)])
