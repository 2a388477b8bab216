"""Pins for the Shortley-Weller rows (Sec. 3.1): every 1D row is exact on
{1, x, x^2} (this is what fixes the coefficients uniquely; it also exposes the
misprinted denominators of Neumann case (b)), and the unshifted Dirichlet
discretisation converges at second order."""
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
