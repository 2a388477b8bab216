"""Pins for periodic problems (Sec. 2.3 covers them through the augmented
system; Sec. 4.4.1 solves the gyroid heat problem in a periodic unit cube):
  * with no immersed boundary the periodic operator's spectrum is the closed
    form of Sec. 2.5 (every wave number of the grid) -- the wrap-around of the
    stencil;
  * L 1 = 0 for a periodic problem with a Neumann boundary;
  * order-4 convergence (mean-free for the singular case) on a body that
    crosses the periodic seam, so that stencils, control points and
    least-squares sets wrap around;
  * periodic coarsening: the multigrid cycle contracts and FGMRES with it
    reaches the bordered direct solve;
  * the gyroid level set: control points on Gamma, normals into phi > 0, the
    curvature formula against finite differences of the normal field."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fd
from oracle import singular as S
from oracle.iim import IIMProblem
from oracle.mg import Hierarchy
from oracle.krylov import fgmres


def _prob(wl, **kw):
    return IIMProblem(wl.dim, wl.n, wl.geom_kind, wl.geom_params, wl.side, wl.bc, wl.beta_plus, wl.beta_minus,
                      lo=wl.lo, hi=wl.hi, periodic=wl.periodic, **kw)


def _seam_circle(n, bc, side=W.SIDE_EXTERIOR):
    """Unit periodic square with a circle crossing the seam x = 1."""
    return W.Workload("seam", 2, n, W.GEOM_SPHERE, [0.87, 0.46, 0.23], side, bc, exact=W.ms_periodic(2),
                      lo=0.0, hi=1.0, periodic=True)


@pytest.mark.parametrize("order", [4, 6])
def test_periodic_box_spectrum_closed_form(order):
    """A periodic square with no unknown near the (vanishing) body: the
    eigenvalues are -(sigma(k_x h) + sigma(k_y h)) / h^2 over every grid wave
    number (Sec. 2.5)."""
    n = 16
    wl = W.Workload("box", 2, n, W.GEOM_SPHERE, [0.5 + 0.31 / n, 0.5 + 0.17 / n, 1e-6], W.SIDE_EXTERIOR,
                    W.BC_NEUMANN, exact=W.ms_periodic(2), lo=0.0, hi=1.0, periodic=True)
    P = _prob(wl, order_n=order, order_k=order + 1, check_kappa=False)
    assert P.ncp == 0 and P.unknowns.size == n * n
    L, _ = P.assemble()
    ev = np.sort(np.linalg.eigvals(L.toarray()).real)
    h = 1.0 / n
    k = 2 * math.pi * np.arange(n) / (n * h)
    sig = fd.sigma(k * h, order)
    closed = np.sort(-(sig[:, None] + sig[None, :]).ravel() / h ** 2)
    assert np.abs(ev - closed).max() <= 1e-9 * np.abs(closed).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_neumann_annihilates_constants(dim):
    if dim == 2:
        wl = _seam_circle(48, W.BC_NEUMANN)
    else:
        wl = W.Workload("g", 3, 28, W.GEOM_GYROID, W.gyroid_params(k=2 * math.pi), W.SIDE_EXTERIOR,
                        W.BC_NEUMANN, exact=W.ms_periodic(3), lo=0.0, hi=1.0, periodic=True)
    P = _prob(wl)
    assert S.is_singular(P)
    L, _ = P.assemble()
    assert np.abs(L @ np.ones(P.unknowns.size)).max() <= 1e-9 * abs(L).max()


def _mean_free_error(wl):
    P = _prob(wl)
    L, LG = P.assemble()
    xyz, nrm = P.cp_arrays()
    ug = P.data_vector(wl.cp_data(xyz, nrm), None)
    b = P.rhs(wl.rhs(P.labels), ug)
    ue = P.from_full(wl.exact_solution(P.labels))
    if S.is_singular(P):
        u, alpha = S.direct_solve(P, b)
        return np.abs(S.mean_free(u) - S.mean_free(ue)).max()
    return np.abs(P.direct_solve(b) - ue).max()


@pytest.mark.parametrize("bc", [W.BC_NEUMANN, W.BC_DIRICHLET], ids=["neumann", "dirichlet"])
def test_seam_crossing_body_converges_at_order4(bc):
    """A circle across the periodic seam: the solution (mean-free when
    singular) converges at fourth order."""
    ns = [32, 64, 128]
    e = [_mean_free_error(_seam_circle(n, bc)) for n in ns]
    rates = [math.log(e[i] / e[i + 1], 2) for i in range(2)]
    assert min(rates) > 3.5 and e[-1] < 1e-5, (e, rates)


def test_periodic_interface_converges_at_order4():
    """An interface across the seam, beta ratio 2, the manufactured u on both
    sides (zero jumps): singular, mean-free error of order 4."""
    ms = W.ms_periodic(2)
    ms2 = W.Manufactured(ms.u_plus, ms.grad_plus, ms.lap_plus, ms.u_plus, ms.grad_plus, ms.lap_plus)
    e = []
    for n in (32, 64, 128):
        wl = W.Workload("i", 2, n, W.GEOM_SPHERE, [0.87, 0.46, 0.23], W.SIDE_INTERFACE, W.BC_JUMP, 1.0, 2.0,
                        exact=ms2, lo=0.0, hi=1.0, periodic=True)
        e.append(_mean_free_error(wl))
    rates = [math.log(e[i] / e[i + 1], 2) for i in range(2)]
    assert min(rates) > 3.5, (e, rates)


def test_periodic_multigrid_and_fgmres():
    """Periodic coarsening: the V-cycle contracts on the periodic Neumann SW
    system, and bordered FGMRES(10) with it reaches the bordered direct solve."""
    wl = _seam_circle(64, W.BC_NEUMANN)
    P = _prob(wl)
    H = Hierarchy(P)
    assert H.bordered and H.sizes == [64, 32, 16, 8]
    L, LG = P.assemble()
    xyz, nrm = P.cp_arrays()
    b = P.rhs(wl.rhs(P.labels), P.data_vector(wl.cp_data(xyz, nrm), None))
    ud, ad = S.direct_solve(P, b)
    Lb = S.bordered_matrix(L)
    prec = lambda v: np.concatenate([H.precondition(v[:-1]), v[-1:]])
    x, hist, its, conv = fgmres(lambda v: Lb @ v, prec, np.concatenate([b, [0.0]]), rtol=1e-12)
    assert conv and its < 60, its
    assert np.abs(x[:-1] - ud).max() <= 1e-8 * np.abs(ud).max()


def test_gyroid_geometry():
    """Gyroid control points (coarse, k = 2 pi): phi(x_c) = 0 to round-off,
    normals unit and pointing into phi > 0, the largest principal curvature
    equal to the one from finite differences of the unit normal field."""
    from oracle.geometry import Gyroid
    G = Gyroid(*W.gyroid_params(k=2 * math.pi))
    wl = W.Workload("g", 3, 28, W.GEOM_GYROID, W.gyroid_params(k=2 * math.pi), W.SIDE_EXTERIOR,
                    W.BC_NEUMANN, exact=W.ms_periodic(3), lo=0.0, hi=1.0, periodic=True)
    P = _prob(wl)
    assert P.ncp > 100
    rng = np.random.default_rng(2)
    for c in rng.choice(P.ncp, 20, replace=False):
        cp = P.cps[int(c)]
        assert abs(G.phi(cp.x)) <= 1e-13
        assert abs(np.linalg.norm(cp.n) - 1.0) <= 1e-14
        assert G.phi(cp.x + 1e-6 * cp.n) > 0.0
        # shape operator from central differences of the unit normal
        e = 1e-5
        J = np.empty((3, 3))
        for d in range(3):
            dx = np.zeros(3)
            dx[d] = e
            J[:, d] = (G.grad_dir(cp.x + dx) - G.grad_dir(cp.x - dx)) / (2 * e)
        Pt = np.eye(3) - np.outer(cp.n, cp.n)
        ev = np.linalg.eigvalsh(0.5 * (Pt @ J @ Pt + (Pt @ J @ Pt).T))
        assert abs(np.abs(ev).max() - cp.kappa) <= 1e-5 * max(1.0, cp.kappa), (ev, cp.kappa)


def test_det_sincos_accuracy():
    """The IEEE-only sin/cos used for the gyroid (Cody-Waite reduction by pi/2
    in three parts, Taylor series on |r| <= pi/4) agrees with the platform's
    sin and cos to a few ulp over the arguments k x takes (|t| <= 8 pi), keeps
    sin^2 + cos^2 = 1, and is exact at the quadrant points where it must be."""
    from oracle.geometry import det_sincos
    t = np.concatenate([np.linspace(-8 * math.pi, 8 * math.pi, 200001),
                        np.random.default_rng(0).uniform(-30.0, 30.0, 100000)])
    s, c = det_sincos(t)
    assert np.abs(s - np.sin(t)).max() <= 4.5e-16
    assert np.abs(c - np.cos(t)).max() <= 4.5e-16
    assert np.abs(s * s + c * c - 1.0).max() <= 5e-16
    s0, c0 = det_sincos(np.array([0.0, math.pi / 2, -math.pi / 6]))
    assert s0[0] == 0.0 and c0[0] == 1.0 and s0[1] == 1.0
    assert abs(s0[2] + 0.5) <= 1.2e-16
