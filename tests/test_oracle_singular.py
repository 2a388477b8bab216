"""Pins of the oracle's singular pure-Neumann path: the bordered system of
Sec. 2.3 (L 1 = 0, alpha the compatibility shift, errors compared mean-free)."""
import numpy as np
import pytest

import workloads as W
from oracle.iim import IIMProblem
from oracle.mg import Hierarchy
from oracle import singular as S

CIRCLE = (W.GEOM_SPHERE, [0.0, 0.0, 0.5])


def _problem(n, dim=2, geom=CIRCLE):
    P = IIMProblem(dim, n, geom[0], geom[1], W.SIDE_INTERIOR, W.BC_NEUMANN)
    P.assemble()
    return P


def _manufactured(P, ex):
    wl = W.Workload("neu", P.dim, P.n, P.geom_kind, P.geom_params, W.SIDE_INTERIOR,
                    W.BC_NEUMANN, exact=ex)
    xyz, nrm = P.cp_arrays()
    ug = P.data_vector(wl.cp_data(xyz, nrm))
    return P.rhs(wl.rhs(P.labels), ug), P.from_full(wl.exact_solution(P.labels))


@pytest.mark.parametrize("dim,n,geom", [(2, 64, CIRCLE), (3, 16, (W.GEOM_SPHERE, [0.0, 0.0, 0.0, 0.6]))])
def test_operator_annihilates_constants(dim, n, geom):
    """Every row of the pure-Neumann operator sums to zero: the least-squares
    fits reproduce constants and the Neumann closure adds nothing for zero
    data.  A dropped or mis-signed closure term breaks this."""
    P = _problem(n, dim, geom)
    assert S.is_singular(P)
    scale = abs(P.L).max()
    assert abs(P.L @ np.ones(P.L.shape[0])).max() < 1e-12 * scale
    # and the row sums are not trivially zero: some rows touch the boundary data
    assert P.LG.nnz > 0


def test_planted_shift_is_recovered():
    """b = L v + c 1 is solved by u = v - mean(v) (gamma = 0) and alpha = c:
    1 is outside the column space of L, so the shift is unique."""
    P = _problem(64)
    rng = np.random.default_rng(11)
    v = rng.standard_normal(P.L.shape[0])
    for c in (0.37, -2.5):
        u, alpha = S.direct_solve(P, P.L @ v + c)
        assert abs(alpha - c) < 1e-10
        assert np.abs(u - S.mean_free(v)).max() < 1e-10
    # gamma moves the constant, nothing else
    u, alpha = S.direct_solve(P, P.L @ v, gamma=3.0 * v.size)
    assert abs(alpha) < 1e-10
    assert np.abs(u - (S.mean_free(v) + 3.0)).max() < 1e-10


def test_mean_free_error_and_shift_converge():
    """Order-4 convergence of the mean-free error (Sec. 2.3 compares singular
    solutions that way) and a compatibility shift that vanishes with h, on a
    solution with no symmetry about the circle's centre."""
    errs, alphas = [], []
    for n in (64, 128, 256):
        P = _problem(n)
        b, ue = _manufactured(P, W.ms_shifted_trig())
        u, alpha = S.direct_solve(P, b)
        assert abs(u.sum()) < 1e-9 * np.abs(u).max() * u.size
        errs.append(np.abs(S.mean_free(u) - S.mean_free(ue)).max())
        alphas.append(abs(alpha))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 3.5, (errs, rates)
    arates = np.log2(np.array(alphas[:-1]) / np.array(alphas[1:]))
    assert arates[-1] > 3.0 and alphas[0] > 1e-4, (alphas, arates)


def test_bordered_coarse_solve():
    """The singular coarsest SW matrix solved through its bordering: the
    result satisfies A z + a 1 = b on the solved rows and sums to zero."""
    P = _problem(64)
    H = Hierarchy(P)
    assert H.bordered
    lc = H.levels[-1]
    rng = np.random.default_rng(5)
    b = np.zeros(lc.unknowns.size)
    b[H.coarse_rows] = rng.standard_normal(H.coarse_rows.size)
    z = H.coarse_solve(b)
    rows = H.coarse_rows
    Ad = lc.A.toarray()[np.ix_(rows, rows)]
    assert abs(np.linalg.matrix_rank(Ad) - (rows.size - 1)) == 0
    r = b[rows] - Ad @ z[rows]
    assert np.ptp(r) < 1e-10 * np.abs(b).max()  # residual is the constant a
    assert abs(z[rows].sum()) < 1e-10 * np.abs(z).max() * rows.size


def test_fgmres_reaches_bordered_direct_solve():
    P = _problem(128)
    b, _ = _manufactured(P, W.ms_shifted_trig())
    u0, a0 = S.direct_solve(P, b)
    u, a, its, ok = S.fgmres_solve(P, Hierarchy(P), b, rtol=1e-10)
    assert ok and its < 60
    assert np.abs(u - u0).max() < 1e-8 * np.abs(u0).max()
    assert abs(a - a0) < 1e-8 * max(abs(a0), 1.0)
