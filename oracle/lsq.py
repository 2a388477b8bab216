"""Least-squares ghost stencils at control points (oracle).

Sec. 2.1: each control point x_c has a set X_c of interpolation points on its
side: the control point itself, plus the side's grid points inside a
half-ellipse (2D) / half-ellipsoid (3D) centred on x_c, minus the grid point
closest to x_c.  A polynomial p_c of order k (total degree <= k-1) fitted to the
values on X_c in the least-squares sense gives each ghost value as a stencil
    p_c(x_g) = s_c^g u(x_c) + sum_alpha s_alpha^g u(x_alpha),
obtained from one QR factorisation per control point followed by one triangular
solve and one matrix-vector product per stencil.  Neumann and interface
closures add one more stencil: the normal derivative of p_c at x_c.

Readings (the region sizes live in a companion paper that is not available):
  * half-ellipse semi-axes in units of h: a (tangential) and b (normal),
    a = k and b = k - 1/2 in 2D and 3D; a point y belongs if
    (y-x_c).nu >= -1e-12 h and T^2/a^2 + N^2/b^2 <= 1 + 1e-12, with N the normal
    and T the tangential distance (in units of h) and nu the unit normal
    pointing into the side;
  * "closest grid point": smallest Euclidean distance among the candidates,
    ties (within 1e-12 h^2) broken by the lowest flat index;
  * plain unweighted least squares; the control-point row is an ordinary row;
  * monomials in xi = (y - x_c)/(a h); rank test |R_ii| >= 1e-10 max |R_jj|,
    otherwise both semi-axes grow by 1/2 (at most 6 times).

Parity: pinned by polynomial reproduction -- every stencil reproduces every
monomial of degree <= k-1 to round-off (tests/test_oracle_lsq.py).
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np
import scipy.linalg

from . import INACTIVE, PLUS, MINUS, BOX

SET_TOL = 1e-12
RANK_TOL = 1e-10
MAX_GROW = 6


def default_axes(dim: int, order_k: int = 5) -> Tuple[float, float]:
    """Semi-axes (tangential a = k, normal b = k - 1/2) in units of h.  Smaller
    regions were tried in 3D; (k-1, k-1.5) already produces stencils whose
    weights sum in magnitude to ~2e4 at some control points of a 64^3 sphere,
    against <= 170 for this choice."""
    return float(order_k), order_k - 0.5


def monomial_exponents(dim: int, degree: int) -> List[Tuple[int, ...]]:
    """All exponents of total degree <= degree, by increasing total degree,
    x-power descending first (then y-power descending in 3D)."""
    out = []
    for t in range(degree + 1):
        if dim == 2:
            for i in range(t, -1, -1):
                out.append((i, t - i))
        else:
            for i in range(t, -1, -1):
                for j in range(t - i, -1, -1):
                    out.append((i, j, t - i - j))
    return out


def vandermonde(xi: np.ndarray, exps) -> np.ndarray:
    """A[r, c] = prod_d xi[r, d] ** exps[c][d]."""
    A = np.ones((xi.shape[0], len(exps)))
    for c, e in enumerate(exps):
        for d in range(xi.shape[1]):
            if e[d]:
                A[:, c] *= xi[:, d] ** e[d]
    return A


def candidate_set_periodic(grid, labels_flat: np.ndarray, xc: np.ndarray, nu: np.ndarray,
                           side: int, a: float, b: float):
    """The candidate set on a periodic grid: nodes are taken at their
    unwrapped positions around x_c (their labels and flat indices modulo n).
    Returns (flat indices, unwrapped coordinates), ordered by the unwrapped
    indices (z slowest), the closest point to x_c removed (ties: the first in
    that order)."""
    dim, h, n = grid.dim, grid.h, grid.n
    R = int(math.ceil(max(a, b))) + 1
    centre = [int(round((xc[d] - grid.lo) / h)) for d in range(dim)]
    axes_idx = [np.arange(centre[d] - R, centre[d] + R + 1) for d in range(dim)]
    mesh = np.meshgrid(*axes_idx, indexing="ij")
    idx = [m.ravel() for m in mesh]
    flat = np.zeros(idx[0].shape, dtype=np.int64)
    key = np.zeros(idx[0].shape, dtype=np.int64)
    span = 2 * R + 1
    for d in reversed(range(dim)):
        flat = flat * (n + 1) + np.mod(idx[d], n)
        key = key * span + (idx[d] - centre[d] + R)
    on_side = labels_flat[flat] == side
    flat, key = flat[on_side], key[on_side]
    idx = [v[on_side] for v in idx]
    pos = np.stack([grid.lo + idx[d] * h for d in range(dim)], axis=1)
    delta = (pos - xc[None, :]) / h
    nn = delta @ nu
    r2 = np.einsum("ij,ij->i", delta, delta)
    t2 = np.maximum(r2 - nn * nn, 0.0)
    keep = (nn >= -SET_TOL) & (t2 / (a * a) + nn * nn / (b * b) <= 1.0 + SET_TOL)
    flat, key, r2, pos = flat[keep], key[keep], r2[keep], pos[keep]
    if flat.size == 0:
        return [], np.zeros((0, dim))
    order = np.argsort(key)
    flat, key, r2, pos = flat[order], key[order], r2[order], pos[order]
    dmin = r2.min()
    closest = np.nonzero(r2 <= dmin + SET_TOL)[0].min()
    keep2 = np.arange(flat.size) != closest
    return [int(f) for f in flat[keep2]], pos[keep2]


def candidate_set(grid, labels_flat: np.ndarray, xc: np.ndarray, nu: np.ndarray,
                  side: int, a: float, b: float) -> List[int]:
    """Flat indices of the side's unknowns in the half-ellipse, in increasing
    flat order, with the closest one to x_c removed."""
    dim = grid.dim
    h = grid.h
    R = int(math.ceil(max(a, b))) + 1
    centre = [int(round((xc[d] - grid.lo) / h)) for d in range(dim)]
    axes_idx = [np.arange(max(0, centre[d] - R), min(grid.n, centre[d] + R) + 1) for d in range(dim)]
    mesh = np.meshgrid(*axes_idx, indexing="ij")
    idx = [m.ravel() for m in mesh]
    flat = np.zeros(idx[0].shape, dtype=np.int64)
    for d in reversed(range(dim)):
        flat = flat * (grid.n + 1) + idx[d]
    on_side = labels_flat[flat] == side
    flat = flat[on_side]
    idx = [v[on_side] for v in idx]
    delta = np.stack([(grid.lo + idx[d] * h - xc[d]) / h for d in range(dim)], axis=1)
    nn = delta @ nu
    r2 = np.einsum("ij,ij->i", delta, delta)
    t2 = np.maximum(r2 - nn * nn, 0.0)
    keep = (nn >= -SET_TOL) & (t2 / (a * a) + nn * nn / (b * b) <= 1.0 + SET_TOL)
    flat, r2 = flat[keep], r2[keep]
    if flat.size == 0:
        return []
    order = np.argsort(flat)
    flat, r2 = flat[order], r2[order]
    dmin = r2.min()
    closest = flat[r2 <= dmin + SET_TOL].min()
    return [int(f) for f in flat if f != closest]


def fit_weights(xc: np.ndarray, pts: np.ndarray, evals: np.ndarray, scale: float, exps):
    """Least-squares stencil weights.

    Rows of the LS matrix: x_c first, then the points `pts` (m, dim).
    `evals` (r, p): each row is an evaluation functional on the monomial
    coefficients.  With A = QR, the fitted coefficients are R^{-1} Q^T v, so
    the weights of functional e are s = Q R^{-T} e.  Returns S (m+1, r) and
    the R diagonal (for the rank test)."""
    xi = np.vstack([np.zeros((1, xc.size)), (pts - xc[None, :]) / scale])
    A = vandermonde(xi, exps)
    Q, R = np.linalg.qr(A, mode="reduced")
    Y = scipy.linalg.solve_triangular(R, evals.T, trans="T", lower=False)
    return Q @ Y, np.abs(np.diag(R))


def value_functional(xg: np.ndarray, xc: np.ndarray, scale: float, exps) -> np.ndarray:
    return vandermonde(((xg - xc) / scale)[None, :], exps)[0]


def normal_derivative_functional(n: np.ndarray, h_scale: float, exps) -> np.ndarray:
    """d/dn of the monomials at xi = 0: only the degree-1 monomials contribute,
    each with n_d / (a h)."""
    e = np.zeros(len(exps))
    for c, ex in enumerate(exps):
        if sum(ex) == 1:
            d = ex.index(1)
            e[c] = n[d] / h_scale
    return e


def cartesian_derivative_functional(d: int, dim: int, h_scale: float, exps) -> np.ndarray:
    """d/dx_d of the monomials at xi = 0 (the gradient of the fit at x_c,
    component d): the normal-derivative functional along the unit vector e_d."""
    e_d = np.zeros(dim)
    e_d[d] = 1.0
    return normal_derivative_functional(e_d, h_scale, exps)


class LSStencil:
    """Weights of one control point on one side.
    idx: flat indices of the m grid points; S: (m+1, r) weights whose row 0
    multiplies u(x_c); columns 0..w-1 are the ghosts j = 1..w, column w
    (when present) the normal derivative along n (without beta), and columns
    w+1..w+dim (when asked for) the Cartesian derivatives d/dx_d at x_c."""
    __slots__ = ("idx", "S", "a", "b", "rdiag")


def ls_stencil(grid, labels_flat, cp, side: int, order_k: int, w: int, with_deriv: bool,
               axes: Tuple[float, float], with_grad: bool = False) -> LSStencil:
    dim = grid.dim
    h = grid.h
    exps = monomial_exponents(dim, order_k - 1)
    nu = cp.n if side == PLUS else -cp.n
    a, b = axes
    a_node = cp.a[side]
    step = cp.dir[side]
    if getattr(grid, "periodic", False):
        xa = np.array(cp.xa[side])
    else:
        xa = np.array([grid.lo + i * h for i in grid.unflat(a_node)])
    for grow in range(MAX_GROW + 1):
        if getattr(grid, "periodic", False):
            idx, pts = candidate_set_periodic(grid, labels_flat, cp.x, nu, side, a, b)
        else:
            idx = candidate_set(grid, labels_flat, cp.x, nu, side, a, b)
            pts = np.array([[grid.lo + i * h for i in grid.unflat(f)] for f in idx])
        if len(idx) + 1 >= len(exps):
            scale = a * h
            rows = []
            for j in range(1, w + 1):
                xg = xa.copy()
                xg[cp.axis] = xa[cp.axis] + j * step * h
                rows.append(value_functional(xg, cp.x, scale, exps))
            if with_deriv or with_grad:
                rows.append(normal_derivative_functional(cp.n, scale, exps))
            if with_grad:
                for d in range(dim):
                    rows.append(cartesian_derivative_functional(d, dim, scale, exps))
            S, rdiag = fit_weights(cp.x, pts, np.array(rows), scale, exps)
            if rdiag.min() >= RANK_TOL * rdiag.max():
                st = LSStencil()
                st.idx, st.S, st.a, st.b, st.rdiag = idx, S, a, b, rdiag
                return st
        a += 0.5
        b += 0.5
    raise RuntimeError("least-squares set rank deficient after growth")
