"""Pins for labels and control points (Sec. 2.1): exact lattice counts by
integer arithmetic, control points lying on Gamma between their two nodes, and
normals pointing into the solved region."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import PLUS, MINUS, BOX, INACTIVE
from oracle.geometry import Grid, make_geometry, node_labels, control_points


def test_circle_labels_match_integer_count():
    # r = 0.5, h = 1/32 -> r/h = 16: unknowns are lattice points with i^2 + j^2 < 256
    g = Grid(2, 64)
    geo = make_geometry(W.GEOM_SPHERE, [0.0, 0.0, 0.5], 2)
    lab = node_labels(g, geo, W.SIDE_INTERIOR)
    count = sum(1 for i in range(-32, 33) for j in range(-32, 33) if i * i + j * j < 256)
    assert int((lab == PLUS).sum()) == count
    # segments with one end strictly inside and the other not (integer test)
    inside = lambda i, j: i * i + j * j < 256
    ncross = sum(1 for i in range(-32, 32) for j in range(-32, 33) if inside(i, j) != inside(i + 1, j))
    ncross += sum(1 for i in range(-32, 33) for j in range(-32, 32) if inside(i, j) != inside(i, j + 1))
    cps = control_points(g, geo, W.SIDE_INTERIOR, lab)
    assert len(cps) == ncross


@pytest.mark.parametrize("kind,params,side,dim,n", [
    (W.GEOM_SPHERE, [0.013, -0.021, 0.55], W.SIDE_INTERIOR, 2, 48),
    (W.GEOM_STAR2D, [0.0, 0.0, 0.5, 0.1, 5], W.SIDE_INTERFACE, 2, 128),
    (W.GEOM_SPHERE_UNION, W.union_params(W.small_circles_union_2d()), W.SIDE_EXTERIOR, 2, 64),
    (W.GEOM_SPHERE, [0.01, 0.02, -0.01, 0.6], W.SIDE_INTERIOR, 3, 16),
])
def test_control_points_on_gamma(kind, params, side, dim, n):
    g = Grid(dim, n)
    geo = make_geometry(kind, params, dim)
    lab = node_labels(g, geo, side)
    cps = control_points(g, geo, side, lab)
    assert len(cps) > 0
    for cp in cps:
        xa = np.array([g.coord(i) for i in g.unflat(cp.p)])
        xb = np.array([g.coord(i) for i in g.unflat(cp.q)])
        # on the segment
        t = (cp.x[cp.axis] - xa[cp.axis]) / g.h
        assert -1e-14 <= t <= 1 + 1e-14
        assert np.allclose(np.delete(cp.x, cp.axis), np.delete(xa, cp.axis))
        # on Gamma: phi changes sign across x_c (tiny offsets along the axis)
        if kind == W.GEOM_STAR2D:
            phi = lambda x: geo.phi_scalar(*x)
        elif kind == W.GEOM_SPHERE:
            phi = lambda x: np.linalg.norm(x - np.array(params[:-1])) - params[-1]
        else:
            phi = lambda x: min(np.linalg.norm(x - np.array(c)) - r for c, r in W.small_circles_union_2d())
        assert abs(phi(cp.x)) < 1e-13
        # unit normal pointing from Omega^- into Omega^+ (into the solved region)
        assert abs(np.linalg.norm(cp.n) - 1) < 1e-13
        into_plus = phi(cp.x + 1e-6 * cp.n)
        if side == W.SIDE_INTERIOR:
            assert into_plus < 0
        else:
            assert into_plus > 0


def test_star_curvature_closed_form():
    """Curvature of r(theta) = r0 + eps cos(5 theta): at theta = 0 the polar
    formula gives (R^2 - R R'')/R^3 with R = r0 + eps, R'' = -25 eps."""
    geo = make_geometry(W.GEOM_STAR2D, [0.0, 0.0, 0.5, 0.1, 5], 2)
    R = 0.6
    want = (R * R - R * (-25 * 0.1)) / R ** 3
    assert abs(geo.curvature(np.array([R, 0.0])) - want) < 1e-12


def test_sphere_union_draw_has_gaps():
    sp = W.draw_sphere_union(16, 0)
    assert len(sp) == 16
    for i in range(16):
        for j in range(i):
            d = np.linalg.norm(np.array(sp[i][0]) - np.array(sp[j][0]))
            assert d - sp[i][1] - sp[j][1] >= 0.05
    assert all(0.08 <= r <= 0.2 and all(-0.7 <= c <= 0.7 for c in cen) for cen, r in sp)
