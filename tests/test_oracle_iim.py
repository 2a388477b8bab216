"""Pins for the assembled high-order system (Sec. 2.1-2.5):
  * patch test: with data from a polynomial of degree <= k-1 the discrete
    equations hold to round-off (truncation error O(h^(k-2)) vanishes);
  * solution convergence at order n = 4 for Dirichlet, Neumann and interface
    problems (Figs. of Sec. 2.4);
  * spectrum of L_Omega at N = 64: Re(h^2 lambda) in [-d sigma_max, 0];
  * interface closure reduces to the Neumann closure as beta^-/beta^+ -> 0;
  * dense solve equals the sparse solve on a tiny grid."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import PLUS, MINUS
from oracle.fd import sigma_max_exact
from oracle.iim import IIMProblem
from oracle.lsq import monomial_exponents


def _setup(wl, **kw):
    P = IIMProblem(wl.dim, wl.n, wl.geom_kind, wl.geom_params, wl.side, wl.bc,
                   wl.beta_plus, wl.beta_minus, **kw)
    L, LG = P.assemble()
    xyz, nrm = P.cp_arrays()
    ug = P.data_vector(wl.cp_data(xyz, nrm), wl.box_data())
    b = P.rhs(wl.rhs(P.labels), ug)
    return P, L, LG, ug, b


def _poly(dim, seed):
    rng = np.random.default_rng(seed)
    return W.ms_polynomial({e: rng.uniform(-1, 1) for e in monomial_exponents(dim, 4)}, dim)


PATCH = [
    ("dirichlet-2d", 2, 48, W.GEOM_SPHERE, [0.013, -0.021, 0.55], 0, 0, 1.0, 1.0),
    ("neumann-2d-exterior-box", 2, 64, W.GEOM_SPHERE_UNION, W.union_params(W.small_circles_union_2d()), 1, 1, 2.0, 1.0),
    ("interface-2d", 2, 128, W.GEOM_STAR2D, [0.0, 0.0, 0.5, 0.1, 5], 2, 2, 0.5, 1.0),
    ("dirichlet-3d", 3, 16, W.GEOM_SPHERE, [0.01, 0.02, -0.01, 0.6], 0, 0, 1.0, 1.0),
    ("neumann-3d-exterior-box", 3, 20, W.GEOM_SPHERE, [0.02, -0.01, 0.03, 0.45], 1, 1, 1.0, 1.0),
]


@pytest.mark.parametrize("case", PATCH, ids=[c[0] for c in PATCH])
def test_patch(case):
    name, dim, n, kind, params, side, bc, bp, bm = case
    ms = _poly(dim, 1)
    if side == W.SIDE_INTERFACE:
        m2 = _poly(dim, 2)
        ms = W.Manufactured(ms.u_plus, ms.grad_plus, ms.lap_plus, m2.u_plus, m2.grad_plus, m2.lap_plus)
    wl = W.Workload(name, dim, n, kind, params, side, bc, bp, bm, exact=ms)
    P, L, LG, ug, b = _setup(wl)
    uex = P.from_full(np.nan_to_num(wl.exact_solution(P.labels)))
    res = L @ uex - b
    scale = abs(L).max() * np.abs(uex).max()
    assert np.abs(res).max() <= 1e-11 * scale


def _err(wl):
    P, L, LG, ug, b = _setup(wl)
    x = P.direct_solve(b)
    return np.abs(x - P.from_full(wl.exact_solution(P.labels))).max()


def _order(make, ns):
    es = [_err(make(n)) for n in ns]
    return [np.log(es[i] / es[i + 1]) / np.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)], es


def _sol2d():
    m = W.ms_paper_interface()
    return W.Manufactured(m.u_minus, m.grad_minus, m.lap_minus)


def test_dirichlet_order4():
    orders, es = _order(lambda n: W.Workload("d", 2, n, W.GEOM_SPHERE, [0.013, -0.021, 0.55], 0, 0,
                                            exact=_sol2d()), [64, 128, 256])
    assert min(orders) > 3.7, (orders, es)


def test_neumann_order4():
    orders, es = _order(lambda n: W.Workload("n", 2, n, W.GEOM_SPHERE_UNION,
                                            W.union_params(W.small_circles_union_2d()), 1, 1,
                                            exact=_sol2d()), [64, 128, 256])
    assert orders[-1] > 3.7 and min(orders) > 3.0, (orders, es)


def test_interface_order4_paper_case():
    """The paper's material-interface case: beta^- = 1, beta^+ = 1/2."""
    orders, es = _order(lambda n: W.Workload("i", 2, n, W.GEOM_STAR2D, [0.0, 0.0, 0.5, 0.1, 5], 2, 2,
                                            0.5, 1.0, exact=W.ms_paper_interface()), [128, 256, 512])
    assert min(orders) > 3.6, (orders, es)


def test_config1_accuracy():
    wl = W.cfg1_circle(64)
    P, L, LG, ug, b = _setup(wl)
    assert P.unknowns.size == 793 and P.ncp == 124
    assert _err(wl) < 1e-3


@pytest.mark.parametrize("kind,params,side,bc,bp,bm", [
    (W.GEOM_SPHERE, [0.013, -0.021, 0.55], 0, 0, 1.0, 1.0),
    (W.GEOM_SPHERE_UNION, W.union_params(W.small_circles_union_2d()), 1, 1, 1.0, 1.0),
    (W.GEOM_SPHERE, [0.013, -0.021, 0.55], 2, 2, 1.0, 2.0),
], ids=["dirichlet", "neumann", "interface"])
def test_spectrum_bounds_n64(kind, params, side, bc, bp, bm):
    P = IIMProblem(2, 64, kind, params, side, bc, bp, bm)
    L, _ = P.assemble()
    A = L * (P.grid.h ** 2 / max(bp, bm))
    smax = float(sigma_max_exact(4))
    if A.shape[0] <= 600:
        lam = np.linalg.eigvals(A.toarray())
        hi, lo = lam.real.max(), lam.real.min()
    else:
        # extreme real parts only (Arnoldi); the dense solve is too slow here
        hi = spla.eigs(A, k=4, which="LR", return_eigenvectors=False, tol=1e-10, maxiter=20000).real.max()
        lo = spla.eigs(A, k=4, which="SR", return_eigenvectors=False, tol=1e-10, maxiter=20000).real.min()
    assert hi <= 1e-8
    assert lo >= -2 * smax * (1 + 1e-8)


def test_interface_tends_to_neumann():
    """As beta^-/beta^+ -> 0 the interface boundary value u^+(x_c) becomes the
    Neumann one with qbar = j1 (Sec. 2.2), so the Omega^+ ghost rows agree."""
    kw = dict(dim=2, n=64, geom_kind=W.GEOM_SPHERE, geom_params=[0.013, -0.021, 0.55], side=2, bc=2,
              beta_plus=1.0)
    Pi = IIMProblem(beta_minus=1e-13, **kw)
    Pn = IIMProblem(**dict(kw, side=1, bc=1, beta_minus=1.0))
    for c in range(0, Pi.ncp, 11):
        # the Omega^+ side is the exterior in both problems; match control points by position
        cn = [k for k, cp in enumerate(Pn.cps) if np.allclose(cp.x, Pi.cps[c].x)]
        assert len(cn) == 1
        for j in (1, 2):
            gi, di = Pi.ghost(c, PLUS, j)
            gn, dn = Pn.ghost(cn[0], PLUS, j)
            plus_nodes = [f for f in gi if Pi.lab_flat[f] == PLUS]
            for f in plus_nodes:
                assert abs(gi[f] - gn.get(f, 0.0)) < 1e-9
            assert abs(di[2 * c + 1] - dn[cn[0]]) < 1e-9


def test_dense_equals_sparse_tiny():
    wl = W.Workload("t", 2, 24, W.GEOM_SPHERE, [0.0, 0.0, 0.7], 0, 0, exact=W.ms_sin2pi_cos2pi())
    P, L, LG, ug, b = _setup(wl)
    xs = P.direct_solve(b)
    xd = np.linalg.solve(L.toarray(), b)
    assert np.abs(xs - xd).max() <= 1e-12 * np.abs(xd).max()


def test_dirichlet_3d_converges():
    orders, es = _order(lambda n: W.Workload("s", 3, n, W.GEOM_SPHERE, [0.01, 0.02, -0.01, 0.6], 0, 0,
                                            exact=W.ms_sin_pi_3d()), [24, 32])
    assert orders[0] > 2.5 and es[-1] < 2e-3, (orders, es)


# ---- sixth order, (n, k) = (6, 7): the next discretisation of the paper (2D) ----

@pytest.mark.parametrize("case", PATCH[:3], ids=[c[0] for c in PATCH[:3]])
def test_patch_order6(case):
    """With data from a polynomial of degree <= k - 1 = 6 the (6,7) equations hold
    to round-off: the order-6 central stencil, the degree-6 least-squares ghosts
    and the degree-6 box extrapolation are all exact on it."""
    name, dim, n, kind, params, side, bc, bp, bm = case
    rng = np.random.default_rng(7)
    poly = lambda: W.ms_polynomial({e: rng.uniform(-1, 1) for e in monomial_exponents(dim, 6)}, dim)
    ms = poly()
    if side == W.SIDE_INTERFACE:
        m2 = poly()
        ms = W.Manufactured(ms.u_plus, ms.grad_plus, ms.lap_plus, m2.u_plus, m2.grad_plus, m2.lap_plus)
    wl = W.Workload(name, dim, n, kind, params, side, bc, bp, bm, exact=ms)
    P, L, LG, ug, b = _setup(wl, order_n=6, order_k=7)
    uex = P.from_full(np.nan_to_num(wl.exact_solution(P.labels)))
    res = L @ uex - b
    scale = abs(L).max() * np.abs(uex).max()
    assert np.abs(res).max() <= 1e-11 * scale


def _err6(wl):
    P, L, LG, ug, b = _setup(wl, order_n=6, order_k=7)
    x = P.direct_solve(b)
    return np.abs(x - P.from_full(wl.exact_solution(P.labels))).max()


def test_dirichlet_order6():
    """Sixth-order convergence of the solution (the paper's (6,7) scheme)."""
    ns = [32, 64, 128]
    es = [_err6(W.Workload("d", 2, n, W.GEOM_SPHERE, [0.013, -0.021, 0.55], 0, 0, exact=_sol2d())) for n in ns]
    orders = [np.log(es[i] / es[i + 1]) / np.log(ns[i + 1] / ns[i]) for i in range(2)]
    assert orders[-1] > 5.7 and min(orders) > 5.0, (orders, es)


def test_neumann_order6():
    ns = [64, 128, 256]
    es = [_err6(W.Workload("n", 2, n, W.GEOM_SPHERE_UNION, W.union_params(W.small_circles_union_2d()), 1, 1,
                           exact=_sol2d())) for n in ns]
    orders = [np.log(es[i] / es[i + 1]) / np.log(ns[i + 1] / ns[i]) for i in range(2)]
    assert orders[-1] > 5.5 and min(orders) > 5.2, (orders, es)


# ---- sixth order in 3D: 84-column fits, half-width 3 -----------------------------------

PATCH_3D_O6 = [
    ("dirichlet-3d", 3, 16, W.GEOM_SPHERE, [0.01, 0.02, -0.01, 0.6], 0, 0, 1.0, 1.0),
    ("neumann-3d-exterior-box", 3, 24, W.GEOM_SPHERE, [0.02, -0.01, 0.03, 0.45], 1, 1, 1.0, 1.0),
]


@pytest.mark.parametrize("case", PATCH_3D_O6, ids=[c[0] for c in PATCH_3D_O6])
def test_patch_order6_3d(case):
    """3D (6,7): degree-6 data (84 monomials) satisfy the discrete equations to
    round-off, through the 84-column fits, the 19-point stencil and, outside
    the sphere, the degree-6 box extrapolation."""
    _patch6(case)


def _patch6(case):
    name, dim, n, kind, params, side, bc, bp, bm = case
    rng = np.random.default_rng(7)
    ms = W.ms_polynomial({e: rng.uniform(-1, 1) for e in monomial_exponents(dim, 6)}, dim)
    wl = W.Workload(name, dim, n, kind, params, side, bc, bp, bm, exact=ms)
    P, L, LG, ug, b = _setup(wl, order_n=6, order_k=7)
    uex = P.from_full(np.nan_to_num(wl.exact_solution(P.labels)))
    res = L @ uex - b
    scale = abs(L).max() * np.abs(uex).max()
    assert np.abs(res).max() <= 1e-10 * scale, np.abs(res).max() / scale

