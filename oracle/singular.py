"""Singular pure-Neumann problems through the augmented system (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 2.3 of the paper: with Neumann conditions on every boundary the system
matrix annihilates the constant vector, L_Omega 1 = 0, so the discrete solution
is fixed only up to a constant.  Following Trottenberg et al. (Sec. 5.6.4), the
system is bordered by one unknown alpha and one equation:
    [ L_Omega  1 ] [ u     ]   [ b     ]
    [ 1^T      0 ] [ alpha ] = [ gamma ],   b = f_Omega - L_Gamma u_Gamma.
1^T u = gamma fixes the constant; alpha is the shift that moves b into the
column space of L_Omega (the discrete form of the integrability condition).
Errors of singular problems are compared after removing the mean from both
the exact and the numerical solution.

Readings:
  * A problem is singular when its domain is the interior of the immersed body
    and the body carries a Neumann condition (interior domains never reach the
    box faces), or when the box is periodic and the immersed condition is a
    Neumann or jump condition: no Dirichlet value pins the constant.
  * gamma = 0: the unknowns sum to zero.
  * Preconditioner of the bordered system: one multigrid cycle on the first
    block, the identity on alpha; the cycle's coarsest SW matrix, singular in
    the same way, is solved through the same bordering (mg.Hierarchy).

Parity: pinned by L 1 = 0 on the assembled operator, by recovering a planted
shift (b = L v + c 1 returns alpha = c and u = v - mean(v)), by the mean-free
error converging at order n and alpha tending to zero with h, and by FGMRES on
the bordered system reaching the bordered direct solve
(tests/test_oracle_singular.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .geometry import SIDE_INTERIOR
from .iim import BC_NEUMANN, BC_DIRICHLET
from .krylov import fgmres


def is_singular(prob) -> bool:
    """Interior domain with a Neumann condition on its whole boundary, or a
    periodic domain whose immersed condition is not Dirichlet."""
    if getattr(prob, "periodic", False):
        return prob.bc != BC_DIRICHLET
    return prob.side == SIDE_INTERIOR and prob.bc == BC_NEUMANN


def bordered_matrix(L: sp.spmatrix) -> sp.csc_matrix:
    """[L 1; 1^T 0] as a sparse matrix."""
    one = np.ones((L.shape[0], 1))
    return sp.bmat([[L, one], [one.T, None]]).tocsc()


def direct_solve(prob, b: np.ndarray, gamma: float = 0.0):
    """Sparse direct solve of the bordered system; returns (u, alpha)."""
    if not hasattr(prob, "L"):
        prob.assemble()
    x = spla.spsolve(bordered_matrix(prob.L), np.concatenate([b, [gamma]]))
    return x[:-1], float(x[-1])


def bordered_apply(L, x: np.ndarray) -> np.ndarray:
    """[L u + alpha 1; 1^T u] for x = [u; alpha]."""
    u, alpha = x[:-1], x[-1]
    return np.concatenate([L @ u + alpha, [u.sum()]])


def fgmres_solve(prob, hier, b: np.ndarray, gamma: float = 0.0, rtol: float = 1e-10,
                 restart: int = 10, max_iters: int = 500):
    """Right-preconditioned FGMRES on the bordered system: the operator is
    bordered_apply, the preconditioner one multigrid cycle on the first block
    and the identity on alpha.  Returns (u, alpha, iterations, converged)."""
    if not hasattr(prob, "L"):
        prob.assemble()
    L = prob.L
    A = lambda x: bordered_apply(L, x)
    M = lambda v: np.concatenate([hier.precondition(v[:-1]), v[-1:]])
    x, _, its, ok = fgmres(A, M, np.concatenate([b, [gamma]]), rtol=rtol, restart=restart,
                           max_iters=max_iters)
    return x[:-1], float(x[-1]), its, ok


def mean_free(v: np.ndarray) -> np.ndarray:
    """v minus its average (how errors of singular problems are compared)."""
    return v - v.mean()
