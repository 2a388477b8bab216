"""Pins for the Shortley-Weller rows (Sec. 3.1): every 1D row is exact on
{1, x, x^2} (this is what fixes the coefficients uniquely; it also exposes the
misprinted denominators of Neumann case (b)), the unshifted Dirichlet
discretisation converges at second order, and the shifted operator on every
multigrid level has an M-matrix sign pattern, row sums fixed by where its
walls sit, and a diagonal bounded by the shift."""
import numpy as np
import pytest

import workloads as W
from oracle.geometry import Grid, make_geometry
from oracle.sw import SWLevel, row_1d, neumann_wall_terms


@pytest.mark.parametrize("kinds", [("V", "V"), ("N", "V"), ("V", "N"), ("N", "N")])
def test_rows_exact_on_quadratics(kinds):
    rng = np.random.default_rng(7)
    for _ in range(50):
        pl, pr = rng.uniform(0.05, 1.0, size=2)
        left, right = (kinds[0], pl), (kinds[1], pr)
        cl, cc, cr = row_1d(left, right)
        gl, gr = neumann_wall_terms(left, right)
        for q in range(3):
            u = lambda x: x ** q
            du = lambda x: q * x ** (q - 1) if q else 0.0
            val = cc * u(0.0)
            val += cl * u(-pl) if kinds[0] == "V" else gl * du(-pl)
            val += cr * u(pr) if kinds[1] == "V" else gr * du(pr)
            want = 2.0 if q == 2 else 0.0
            if kinds == ("N", "N") and q == 2:
                want = 2.0   # (-u'(-pl) + u'(pr)) / (pl + pr) = 2 on x^2
            assert abs(val - want) < 1e-10 * (1 + abs(cc)), (kinds, q, pl, pr, val)


def test_printed_neumann_b_is_not_exact():
    """The row as printed (denominators psi^+(psi^- + 2 psi^+)) fails on u = x
    whenever psi^+ != 1, which is why the mirror of case (a) is used."""
    pl, pr = 1.0, 0.4
    c = 2.0 / (pr * (pl + 2 * pr))
    val = c * (-pl) - c * 0.0 + 2.0 / (pl + 2 * pr) * 1.0
    assert abs(val) > 1e-3


def test_unshifted_dirichlet_second_order():
    ms = W.ms_sin2pi_cos2pi()
    errs = []
    for n in (32, 64, 128, 256):
        g = Grid(2, n)
        geo = make_geometry(W.GEOM_SPHERE, [0.013, -0.021, 0.55], 2)
        lev = SWLevel(g, geo, W.SIDE_INTERIOR, W.BC_DIRICHLET, shift=False)
        X = g.node_coords()
        xf = [x.ravel(order="F")[lev.unknowns] for x in X]
        f = ms.lap_plus(*xf)
        rhs = f.copy()
        for r, c, xw in lev.wall_terms:
            rhs[r] -= c * ms.u_plus(*xw)
        import scipy.sparse.linalg as spla
        u = spla.spsolve(lev.A.tocsc(), rhs)
        errs.append(np.abs(u - ms.u_plus(*xf)).max())
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert min(orders[1:]) > 1.8, (orders, errs)


# -- the shifted operator on every level: sign structure and row sums ----------------

from oracle import PLUS, MINUS, BOX  # noqa: E402
from oracle.iim import IIMProblem  # noqa: E402
from oracle.mg import Hierarchy  # noqa: E402

SHIFTED = [
    ("dirichlet-interior-2d", 2, 64, W.GEOM_SPHERE, [0.013, -0.021, 0.55], 0, 0, 1.0, 1.0),
    ("dirichlet-exterior-2d", 2, 64, W.GEOM_SPHERE_UNION, W.union_params(W.small_circles_union_2d()), 1, 0, 1.0, 1.0),
    ("neumann-exterior-2d", 2, 64, W.GEOM_SPHERE_UNION, W.union_params(W.small_circles_union_2d()), 1, 1, 1.0, 1.0),
    ("interface-2d", 2, 128, W.GEOM_STAR2D, [0.0, 0.0, 0.5, 0.1, 5], 2, 2, 0.5, 1.0),
    ("dirichlet-interior-3d", 3, 24, W.GEOM_SPHERE, [0.01, 0.02, -0.01, 0.6], 0, 0, 1.0, 1.0),
    ("neumann-exterior-3d", 3, 24, W.GEOM_SPHERE, [0.02, -0.01, 0.03, 0.45], 1, 1, 1.0, 1.0),
]


@pytest.mark.parametrize("case", SHIFTED, ids=[c[0] for c in SHIFTED])
def test_shifted_operator_sign_structure_and_row_sums(case):
    """On every level of the hierarchy the shifted SW matrix has a non-positive
    diagonal and non-negative off-diagonal entries (an M-matrix pattern), and
    its row sums follow from where each row's neighbours sit: a Dirichlet wall
    or a box face moves its coefficient to the data side, so the row sum is
    strictly negative; a Neumann wall or an interface link (weights summing to
    one) keeps the row consistent on constants, so an interior row sums to 0."""
    name, dim, n, kind, params, side, bc, bp, bm = case
    P = IIMProblem(dim, n, kind, params, side, bc, bp, bm)
    H = Hierarchy(P)
    for l, lev in enumerate(H.levels):
        A = lev.A.tocsr()
        d = A.diagonal()
        off = A.copy()
        off.setdiag(0.0)
        off.eliminate_zeros()
        assert (d <= 0.0).all(), (name, l)
        assert (off.data >= 0.0).all(), (name, l)
        rs = A @ np.ones(A.shape[0])
        scale = np.abs(d).max()
        lab = lev.lab_flat
        nn = lev.grid.n + 1
        touch_dir = np.zeros(lev.unknowns.size, dtype=bool)  # a neighbour that takes data off the matrix
        for r, f in enumerate(lev.unknowns):
            idx = np.unravel_index(f, (nn,) * dim, order="F")
            for ax in range(dim):
                for s in (-1, 1):
                    j = list(idx)
                    j[ax] += s
                    q = np.ravel_multi_index(tuple(j), (nn,) * dim, order="F")
                    lq = lab[q]
                    if lq == BOX or (lq != lab[f] and bc == 0 and side != 2):
                        touch_dir[r] = True
        assert (rs[touch_dir] < -1e-12 * scale).all(), (name, l)
        assert np.abs(rs[~touch_dir]).max() <= 1e-12 * scale, (name, l, np.abs(rs[~touch_dir]).max() / scale)
        # the intersection shift (every wall at least h/2 away) bounds the
        # diagonal: a 1D row weighs 2 / (psi- psi+ h^2) <= 8 / h^2 per axis
        h2 = lev.grid.h ** 2
        assert np.abs(d).max() <= 8.0 * dim / h2 * (1 + 1e-12), (name, l)


def test_unshifted_operator_exceeds_the_shift_bound():
    """Without the shift, walls closer than h/2 make the diagonal exceed
    8 dim / h^2 on the same geometry: the bound above is the shift's doing."""
    P = IIMProblem(2, 64, W.GEOM_SPHERE, [0.013, -0.021, 0.55], 0, 0)
    lev = SWLevel(P.grid, P.geom, 0, 0, 1.0, 1.0, shift=False)
    assert np.abs(lev.A.diagonal()).max() > 8.0 * 2 / P.grid.h ** 2


def test_interface_wall_value_on_a_flat_interface(monkeypatch):
    """The interface rows' wall value (Sec. 3.1, with the interface shifted to
    the midpoint): on a flat interface x = x0 that already lies halfway between
    two grid columns the shift changes nothing, and for a piecewise-linear u
    with [u] = 0 and beta^+ du^+/dx = beta^- du^-/dx the flux-continuity wall
    value is exact, so every row of A u vanishes to round-off (A is the plain
    Laplacian of each side).  beta^-/beta^+ = 2 makes the slopes differ, so
    exchanging alpha^+ and alpha^- leaves an O(1/h) residual next to the
    interface.  The interface plane meets the box, which the library's labels
    reject; the test builds its own labels (x <= x0: Omega^-, box faces:
    known values)."""
    from oracle import PLUS, MINUS, BOX
    import oracle.sw as S

    n = 32
    h = 2.0 / n
    x0 = -1.0 + 13.5 * h

    def flat_labels(grid, geom, side):
        X = grid.node_coords()
        lab = np.where(X[0] <= x0, MINUS, PLUS).astype(np.uint8)
        for d in range(grid.dim):
            idx = [slice(None)] * grid.dim
            for end in (0, grid.n):
                idx[d] = end
                lab[tuple(idx)] = BOX
        return lab

    monkeypatch.setattr(S, "node_labels", flat_labels)
    for dim in (2, 3):
        grid = Grid(dim, n)
        lev = SWLevel(grid, None, 2, 2, beta_plus=1.0, beta_minus=2.0, shift=True)
        X = [c.ravel(order="F")[lev.unknowns] for c in grid.node_coords()]
        a_minus = 0.7
        a_plus = a_minus * 2.0 / 1.0     # beta^+ u'^+ = beta^- u'^-
        u = np.where(X[0] <= x0, a_minus * (X[0] - x0), a_plus * (X[0] - x0)) + 0.3 + 0.2 * X[1]
        r = lev.A @ u
        # rows whose stencil reaches a box face see the face value 0, not u
        ijk = np.array([grid.unflat(int(f)) for f in lev.unknowns])
        away = np.all((ijk >= 2) & (ijk <= n - 2), axis=1)
        scale = np.abs(lev.A).max() * np.abs(u).max()
        assert np.abs(r[away]).max() <= 1e-13 * scale, (dim, np.abs(r[away]).max() / scale)
        near = away & (np.abs(X[0] - x0) < h)
        assert near.sum() >= 2 * (n - 3) ** (dim - 1)
