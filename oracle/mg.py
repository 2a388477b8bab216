"""Geometric multigrid V-cycle on the Shortley-Weller operator (oracle).

Sec. 3.3 of the paper: factor-two coarsening, red-black Gauss-Seidel
smoothing, half-weighted restriction applied to the whole grid with zero values
outside the domain, and
  * Dirichlet boundaries: bilinear / trilinear interpolation with zero values
    outside the domain;
  * Neumann boundaries: the average of the neighbouring coarse values that lie
    in the domain (zero when there are none);
  * interfaces: standard interpolation, and the cycle solves Lap u = f / beta on
    each side.
The Shortley-Weller operator is rediscretised on every level from the level
set; a direct solve is used on the coarsest level (n <= 8).  One V-cycle with a
zero initial guess is the preconditioner.

Cycle option (Sec. 3.3 and the 2D multigrid results of Sec. 3): gamma = 2 gives
the W-cycle, which visits each coarser level twice per visit of the level above
(Trottenberg's cycle index gamma); the second visit starts from the iterate the
first one left.  gamma = 1 is the V-cycle.

Readings: vertex-centred coarsening (coarse node I = fine node 2I, ceil(n/2)
intervals; on a periodic grid n stays even down to the coarsest level and the
transfers take indices modulo n); half-weighting stencils 1/8 [0 1 0; 1 4 1; 0 1 0] in 2D and centre
1/2, faces 1/12 in 3D; red (even index sum) before black; V(2,2); box-face nodes
hold zero and count as in-domain for the averaging interpolation; the coarse
solve excludes rows with a zero diagonal (their value stays zero).  For a
singular problem (interior domain, Neumann boundary) the coarsest matrix
annihilates constants too; it is bordered like the fine system, [A 1; 1^T 0],
and the coarse solve returns the first block of the bordered solution with a
zero last entry on the right (the coarse values then sum to zero).

Parity: pinned by the Dirichlet V-cycle contraction on the standard (unshifted)
SW operator (rho < 0.09, independent of n, the rate the paper quotes), by the
shifted cycle staying fast and n-independent, by transfer operators reproducing
constants away from Gamma, by the averaging interpolation equalling the
multilinear one wherever every parent lies in the domain and reproducing
constants wherever one does, and by the FGMRES solution matching the direct
solve (tests/test_oracle_mg.py).  The
W-cycle is pinned by its identity with the V-cycle on two levels (the coarse
solve is exact, so the second visit changes nothing), by a contraction no
worse than the V-cycle's, by the cycle from a non-zero start equalling that
start plus the cycle of the residual, and by FGMRES reaching the direct solve.
"""
from __future__ import annotations

import itertools
import math
from typing import List

import numpy as np
import scipy.linalg

from . import INACTIVE, PLUS, MINUS, BOX
from .geometry import Grid, SIDE_INTERFACE, SIDE_INTERIOR
from .sw import SWLevel, BC_DIRICHLET, BC_NEUMANN, BC_JUMP


def is_singular_setup(prob) -> bool:
    """No Dirichlet value anywhere pins the constant: an interior domain with
    a Neumann boundary, or a periodic domain whose immersed condition is not
    Dirichlet (Neumann, or jumps)."""
    if getattr(prob.grid, "periodic", False):
        return prob.bc != BC_DIRICHLET
    return prob.side == SIDE_INTERIOR and prob.bc == BC_NEUMANN


def level_sizes(n: int, coarsest: int = 8) -> List[int]:
    out = [n]
    while out[-1] > coarsest:
        out.append((out[-1] + 1) // 2)
    return out


class Hierarchy:
    def __init__(self, prob, coarsest: int = 8, nu_pre: int = 2, nu_post: int = 2, gamma: int = 1,
                 shift: bool = True):
        """prob: an IIMProblem (provides grid, geometry, side, bc, beta);
        gamma: cycle index (1 = V-cycle, 2 = W-cycle); shift: the intersection
        shift of Sec. 3.2 on every level (the preconditioner's setting; False
        gives the standard Shortley-Weller operator whose cycle the paper
        quotes from Trottenberg et al.)."""
        self.prob = prob
        self.dim = prob.dim
        self.nu_pre, self.nu_post = nu_pre, nu_post
        self.gamma = gamma
        self.sizes = level_sizes(prob.n, coarsest)
        self.levels: List[SWLevel] = []
        for l, nl in enumerate(self.sizes):
            g = Grid(prob.dim, nl, prob.grid.h * 2 ** l, prob.grid.lo, prob.grid.periodic)
            self.levels.append(SWLevel(g, prob.geom, prob.side, prob.bc,
                                       prob.beta[PLUS], prob.beta[MINUS], shift=shift))
        if prob.side == SIDE_INTERFACE or prob.bc == BC_DIRICHLET:
            self.mode = "linear"
        else:
            self.mode = "average"
        # colour masks (red = even index sum) per level, over unknowns
        self.colour = []
        for lev in self.levels:
            idx = sum(self._multi_index(lev, lev.unknowns))
            self.colour.append(idx % 2)
        # coarsest: dense LU on rows with a non-zero diagonal
        lc = self.levels[-1]
        self.coarse_rows = np.nonzero(lc.diag != 0.0)[0]
        Ad = lc.A.toarray()[np.ix_(self.coarse_rows, self.coarse_rows)]
        self.bordered = is_singular_setup(prob)
        if self.bordered and Ad.size:
            nc = Ad.shape[0]
            Ab = np.zeros((nc + 1, nc + 1))
            Ab[:nc, :nc] = Ad
            Ab[:nc, nc] = 1.0
            Ab[nc, :nc] = 1.0
            Ad = Ab
        self.coarse_lu = scipy.linalg.lu_factor(Ad) if Ad.size else None

    # -- smoother ------------------------------------------------------------------
    def rbgs(self, l: int, z: np.ndarray, b: np.ndarray) -> None:
        """One red-black Gauss-Seidel sweep (red first), in place."""
        lev = self.levels[l]
        A, D = lev.A, lev.diag
        for c in (0, 1):
            rows = np.nonzero((self.colour[l] == c) & (D != 0.0))[0]
            Az = A[rows] @ z
            z[rows] = (b[rows] - Az + D[rows] * z[rows]) / D[rows]

    # -- transfers --------------------------------------------------------------------
    @staticmethod
    def _multi_index(lev, flat):
        n1 = lev.grid.n + 1
        return [(flat // n1 ** d) % n1 for d in range(lev.grid.dim)]

    def restrict(self, l: int, r: np.ndarray) -> np.ndarray:
        """Half-weighting of the fine residual (zero off the unknowns) onto
        the coarse unknowns:  r_c(I) = w0 r_f(2I) + w1 sum_d (r_f(2I+e_d) + r_f(2I-e_d))."""
        fine, coarse = self.levels[l], self.levels[l + 1]
        dim = self.dim
        rf = np.zeros(fine.lab_flat.size)
        rf[fine.unknowns] = r
        rf = rf.reshape(fine.grid.shape, order="F")
        w0, w1 = (0.5, 0.125) if dim == 2 else (0.5, 1.0 / 12.0)
        F = [2 * i for i in self._multi_index(coarse, coarse.unknowns)]
        out = w0 * rf[tuple(F)]
        for d in range(dim):
            for s in (-1, 1):
                G = list(F)
                G[d] = fine.grid.wrap(G[d] + s)   # modulo n on a periodic grid
                out = out + w1 * rf[tuple(G)]
        return out

    def prolong(self, l: int, zc: np.ndarray) -> np.ndarray:
        """Interpolation of the coarse correction onto the fine unknowns.  The
        parents of fine node F are the coarse nodes floor(F/2) and ceil(F/2)
        along each axis (one parent along axes where F is even)."""
        fine, coarse = self.levels[l - 1], self.levels[l]
        zfull = np.zeros(coarse.lab_flat.size)
        zfull[coarse.unknowns] = zc
        zfull = zfull.reshape(coarse.grid.shape, order="F")
        lab_c = coarse.labels
        F = self._multi_index(fine, fine.unknowns)
        lo = [Fd // 2 for Fd in F]
        odd = [(Fd % 2) == 1 for Fd in F]
        total = np.zeros(fine.unknowns.size)
        count = np.zeros(fine.unknowns.size)
        for bits in itertools.product((0, 1), repeat=self.dim):
            use = np.ones(fine.unknowns.size, dtype=bool)
            P = []
            for d in range(self.dim):
                if bits[d]:
                    use &= odd[d]
                P.append(lo[d] + bits[d])
            P = tuple(coarse.grid.wrap(np.where(use, P[d], lo[d])) for d in range(self.dim))
            if self.mode == "average":
                lab = lab_c[P]
                use &= (lab == PLUS) | (lab == MINUS) | (lab == BOX)
            total += np.where(use, zfull[P], 0.0)
            count += use
        if self.mode == "linear":
            return total / count
        return np.where(count > 0, total / np.maximum(count, 1), 0.0)

    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        z = np.zeros(b.size)
        if self.coarse_lu is not None:
            rhs = b[self.coarse_rows]
            if self.bordered:
                rhs = np.concatenate([rhs, [0.0]])
            sol = scipy.linalg.lu_solve(self.coarse_lu, rhs)
            z[self.coarse_rows] = sol[:self.coarse_rows.size]
        return z

    # -- cycle ---------------------------------------------------------------------------
    def cycle_level(self, l: int, b: np.ndarray, z0: np.ndarray = None) -> np.ndarray:
        """One multigrid cycle of index gamma on level l for A_l z = b, from z0
        (zero if None): pre-smoothing, restriction of the residual, gamma
        cycles on level l + 1 (the first from zero, each later one from the
        previous one's result), prolongation and correction, post-smoothing.
        The coarsest level is solved directly whatever the start."""
        if l == len(self.levels) - 1:
            return self.coarse_solve(b)
        lev = self.levels[l]
        z = np.zeros(b.size) if z0 is None else np.array(z0, dtype=np.float64)
        for _ in range(self.nu_pre):
            self.rbgs(l, z, b)
        r = b - lev.A @ z
        bc = self.restrict(l, r)
        zc = None
        for _ in range(self.gamma):
            zc = self.cycle_level(l + 1, bc, zc)
        z += self.prolong(l + 1, zc)
        for _ in range(self.nu_post):
            self.rbgs(l, z, b)
        return z

    def vcycle_level(self, l: int, b: np.ndarray) -> np.ndarray:
        """One cycle (of the hierarchy's index gamma) from a zero start."""
        return self.cycle_level(l, b)

    def precondition(self, v: np.ndarray) -> np.ndarray:
        """z = M^{-1} v: one cycle (V for gamma = 1, W for gamma = 2) on
        Lap z = v / beta (v on the level-0 unknowns, which coincide with the
        high-order unknowns)."""
        lev0 = self.levels[0]
        beta = np.where(lev0.lab_flat[lev0.unknowns] == MINUS,
                        self.prob.beta[MINUS], self.prob.beta[PLUS])
        return self.vcycle_level(0, v / beta)
