"""Pin for the least-squares ghost stencils (Sec. 2.1-2.2): a least-squares fit
over polynomials of degree <= k-1 reproduces every such polynomial exactly, so
every stencil row applied to the samples of a monomial must return the
monomial's value at the ghost point (or its normal derivative at x_c)."""
import numpy as np
import pytest

import workloads as W
from oracle import PLUS, MINUS
from oracle.iim import IIMProblem
from oracle.lsq import monomial_exponents, default_axes

CASES = [
    ("circle-dirichlet", dict(dim=2, n=64, geom_kind=W.GEOM_SPHERE, geom_params=[0.013, -0.021, 0.55], side=0, bc=0)),
    ("circle-neumann-ext", dict(dim=2, n=64, geom_kind=W.GEOM_SPHERE_UNION,
                                geom_params=W.union_params(W.small_circles_union_2d()), side=1, bc=1)),
    ("star-interface", dict(dim=2, n=128, geom_kind=W.GEOM_STAR2D, geom_params=[0.0, 0.0, 0.5, 0.1, 5], side=2, bc=2)),
    ("sphere-dirichlet", dict(dim=3, n=24, geom_kind=W.GEOM_SPHERE, geom_params=[0.01, 0.02, -0.01, 0.6], side=0, bc=1)),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_polynomial_reproduction(name, kw):
    P = IIMProblem(**kw)
    g = P.grid
    exps = monomial_exponents(P.dim, P.order_k - 1)
    rng = np.random.default_rng(0)
    sel = rng.choice(P.ncp, size=min(25, P.ncp), replace=False)
    for c in sel:
        cp = P.cps[c]
        for side in P.sides:
            st = P.stencil(int(c), side)
            pts = np.array([[g.lo + i * g.h for i in g.unflat(f)] for f in st.idx])
            allpts = np.vstack([cp.x[None, :], pts])
            xa = np.array([g.lo + i * g.h for i in g.unflat(cp.a[side])])
            for e in exps:
                vals = np.prod([(allpts[:, d] - cp.x[d]) ** e[d] for d in range(P.dim)], axis=0)
                scale = np.abs(vals).max() + 1e-300
                for j in range(1, P.w + 1):
                    xg = xa.copy()
                    xg[cp.axis] += j * cp.dir[side] * g.h
                    want = np.prod([(xg[d] - cp.x[d]) ** e[d] for d in range(P.dim)])
                    got = st.S[:, j - 1] @ vals
                    assert abs(got - want) <= 1e-9 * max(scale, abs(want)), (name, c, side, e, j)
                if st.S.shape[1] > P.w:
                    want = cp.n[e.index(1)] if sum(e) == 1 else 0.0
                    got = st.S[:, P.w] @ vals
                    assert abs(got - want) <= 1e-9 * max(scale / g.h, 1.0), (name, c, side, e)


def test_ls_set_excludes_closest_and_respects_side():
    P = IIMProblem(**CASES[2][1])
    g = P.grid
    for c in range(0, P.ncp, 37):
        cp = P.cps[c]
        for side in P.sides:
            st = P.stencil(c, side)
            assert all(P.lab_flat[f] == side for f in st.idx)
            nu = cp.n if side == PLUS else -cp.n
            d = np.array([[(g.lo + i * g.h - cp.x[k]) / g.h for k, i in enumerate(g.unflat(f))] for f in st.idx])
            assert (d @ nu >= -1e-12).all()
            assert st.idx == sorted(st.idx)
            assert len(st.idx) + 1 >= len(monomial_exponents(2, 4))


def _min_norm_weights_extended(A, E):
    """The minimum-norm solution s = A (A^T A)^{-1} E^T of A^T s = E^T in
    x87 extended precision (64-bit significand): Cholesky of A^T A and two
    corrections with the residual E^T - A^T s, an independent route to the
    least-squares weights that the oracle takes by Householder QR in double."""
    Al = A.astype(np.longdouble)
    El = E.T.astype(np.longdouble)
    G = Al.T @ Al
    n = G.shape[0]
    L = np.zeros_like(G)
    for j in range(n):
        L[j, j] = np.sqrt(G[j, j] - L[j, :j] @ L[j, :j])
        for i in range(j + 1, n):
            L[i, j] = (G[i, j] - L[i, :j] @ L[j, :j]) / L[j, j]

    def solve(B):
        Y = np.zeros_like(B)
        for i in range(n):
            Y[i] = (B[i] - L[i, :i] @ Y[:i]) / L[i, i]
        Z = np.zeros_like(B)
        for i in reversed(range(n)):
            Z[i] = (Y[i] - L[i + 1:, i] @ Z[i + 1:]) / L[i, i]
        return Z

    z = solve(El)
    for _ in range(2):
        z = z + solve(El - Al.T @ (Al @ z))
    return Al @ z


def test_weights_are_the_minimum_norm_least_squares_solution():
    """The oracle's weights (value rows and the d/dn row of 3D Neumann fits,
    Sec. 2.2) equal the minimum-norm solution of A^T s = E^T computed in
    extended precision to within 1e-12 of the largest weight (measured: at
    most 4.7e-13 over every fit of the Neumann sphere at 24^3).  Polynomial
    reproduction alone does not fix the weights when the set has more points
    than monomials; a wrong row scaling or a weight vector outside the range
    of A passes it and fails this."""
    from oracle.lsq import vandermonde, value_functional, normal_derivative_functional
    P = IIMProblem(dim=3, n=24, geom_kind=W.GEOM_SPHERE, geom_params=[0.05, -0.1, 0.03, 0.6], side=1, bc=1)
    g = P.grid
    exps = monomial_exponents(3, P.order_k - 1)
    rng = np.random.default_rng(3)
    worst = 0.0
    for c in rng.choice(P.ncp, size=12, replace=False):
        cp = P.cps[int(c)]
        side = P.sides[0]
        st = P.stencil_d(int(c), side)
        pts = np.array([[g.lo + i * g.h for i in g.unflat(f)] for f in st.idx])
        scale = st.a * g.h
        A = vandermonde(np.vstack([np.zeros((1, 3)), (pts - cp.x[None, :]) / scale]), exps)
        xa = np.array([g.lo + i * g.h for i in g.unflat(cp.a[side])])
        rows = []
        for j in range(1, P.w + 1):
            xg = xa.copy()
            xg[cp.axis] += j * cp.dir[side] * g.h
            rows.append(value_functional(xg, cp.x, scale, exps))
        rows.append(normal_derivative_functional(cp.n, scale, exps))
        E = np.array(rows)
        assert st.S.shape == (A.shape[0], E.shape[0])
        sx = _min_norm_weights_extended(A, E)
        err = float(np.abs(st.S - sx).max() / np.abs(sx).max())
        worst = max(worst, err)
    assert worst <= 1e-12, worst
