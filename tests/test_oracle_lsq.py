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
