"""Shortley-Weller low-order discretisations (oracle).

Sec. 3.1 of the paper.  Along each axis, at an irregular node with a wall at
fractional distance psi^- (left) and/or psi^+ (right):
  Dirichlet (eq. for case (c); (a), (b) set the regular side to psi = 1):
     d2u ~ [2 u_w^-/(psi^-(psi^-+psi^+)) - 2 u_i/(psi^- psi^+) + 2 u_w^+/(psi^+(psi^-+psi^+))] / h^2
  Neumann wall on the left, value side on the right (case (a)):
     d2u ~ [-2 h dx u_w^-/(2psi^-+psi^+) - 2 u_i/(psi^+(2psi^-+psi^+)) + 2 u_{i+1}/(psi^+(2psi^-+psi^+))] / h^2
  Neumann wall on the right (case (b)), as the mirror image of (a):
     d2u ~ [2 u_{i-1}/(psi^-(psi^-+2psi^+)) - 2 u_i/(psi^-(psi^-+2psi^+)) + 2 h dx u_w^+/(psi^-+2psi^+)] / h^2
     (the printed denominators psi^+(psi^-+2psi^+) of the u_{i-1} and u_i terms
      are not exact on u = x unless psi^+ = 1; the mirror of (a) is exact on
      {1, x, x^2}, which a unit test pins.)
  Neumann walls on both sides (case (c)): no u_i term.
  Interface: wall value from the first-order jump conditions with
     alpha^pm = psi^pm / beta^pm,
     u_w = (alpha^+ u_(Omega^- node) + alpha^- u_(Omega^+ node)) / (alpha^+ + alpha^-)
     for homogeneous jumps ([u] = u^+ - u^-; the printed sign of [u] only matters
     for inhomogeneous jumps, which the preconditioner never sees).
Dimension splitting: rows are summed over the axes; Neumann data use
dn u ~ sign(n_i) d_i u (homogeneous inside the preconditioner).
Intersection shifting: boundary walls psi <- max(psi, 1/2); interfaces
psi^+ = psi^- = 1/2.  The operator here is the plain Laplacian: the
interface preconditioner solves Lap u = f / beta on each side (Sec. 3.3).
Box-face nodes are regular neighbours holding their (zero) value.  On a
periodic grid neighbours are taken modulo n.

Parity: the 1D rows are pinned by exactness on {1, x, x^2}; the unshifted
Dirichlet discretisation by its second-order convergence; the shifted operator
by invariants only (M-matrix signs, row sums fixed by its walls, a diagonal
bounded by the shift) and the multigrid convergence checks: its entries are
otherwise parity unpinned.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np
import scipy.sparse as sp

from . import INACTIVE, PLUS, MINUS, BOX
from .geometry import Grid, node_labels, SIDE_INTERFACE, SIDE_INTERIOR

BC_DIRICHLET, BC_NEUMANN, BC_JUMP = 0, 1, 2


def row_1d(left, right) -> Tuple[float, float, float]:
    """Coefficients (c_left, c_centre, c_right), in units of 1/h^2, of the 1D
    Shortley-Weller row.  Each side is ('V', psi) for a value (regular
    neighbour at psi = 1, Dirichlet or interface wall) or ('N', psi) for a
    Neumann wall; c_left / c_right multiply the value on that side."""
    (tl, pl), (tr, pr) = left, right
    if tl == "V" and tr == "V":
        return 2.0 / (pl * (pl + pr)), -2.0 / (pl * pr), 2.0 / (pr * (pl + pr))
    if tl == "N" and tr == "V":
        c = 2.0 / (pr * (2.0 * pl + pr))
        return 0.0, -c, c
    if tl == "V" and tr == "N":
        c = 2.0 / (pl * (pl + 2.0 * pr))
        return c, -c, 0.0
    return 0.0, 0.0, 0.0


def neumann_wall_terms(left, right) -> Tuple[float, float]:
    """Coefficients (in units of 1/h) of h*dx u at the walls for the rows with
    a Neumann wall (used only to check exactness of the 1D rows)."""
    (tl, pl), (tr, pr) = left, right
    if tl == "N" and tr == "V":
        return -2.0 / (2.0 * pl + pr), 0.0
    if tl == "V" and tr == "N":
        return 0.0, 2.0 / (pl + 2.0 * pr)
    if tl == "N" and tr == "N":
        return -1.0 / (pl + pr), 1.0 / (pl + pr)
    return 0.0, 0.0


class SWLevel:
    """The Shortley-Weller operator on one grid (full set of unknowns)."""

    def __init__(self, grid: Grid, geom, side: int, bc: int, beta_plus: float = 1.0,
                 beta_minus: float = 1.0, shift: bool = True):
        self.grid, self.geom, self.side, self.bc = grid, geom, side, bc
        self.beta = {PLUS: beta_plus, MINUS: beta_minus}
        self.labels = node_labels(grid, geom, side)
        self.lab_flat = self.labels.ravel(order="F")
        self.unknowns = np.nonzero((self.lab_flat == PLUS) | (self.lab_flat == MINUS))[0]
        self.uindex = np.full(self.lab_flat.size, -1, dtype=np.int64)
        self.uindex[self.unknowns] = np.arange(self.unknowns.size)
        self.strides = [(grid.n + 1) ** d for d in range(grid.dim)]
        self.shift = shift
        self.wall_terms: List[Tuple[int, float, np.ndarray]] = []   # (row, coef, wall point)
        self.box_terms: List[Tuple[int, float, int]] = []           # (row, coef, box node)
        self.A = self._assemble()
        self.diag = self.A.diagonal()

    def _neighbour(self, f: int, d: int, s: int):
        i = (f // self.strides[d]) % (self.grid.n + 1)
        if getattr(self.grid, "periodic", False):
            return f + (((i + s) % self.grid.n) - i) * self.strides[d]
        if not 0 <= i + s <= self.grid.n:
            return None
        return f + s * self.strides[d]

    def _wall(self, f: int, q: int, d: int, s: int):
        """Side description and value links for the neighbour q = f + s e_d."""
        lab_f, lab_q = self.lab_flat[f], self.lab_flat[q]
        g = self.grid
        if lab_q == lab_f:
            return ("V", 1.0), [(q, 1.0)], None
        if lab_q == BOX:
            return ("V", 1.0), [], ("box", q)
        xf = [g.lo + i * g.h for i in g.unflat(f)]
        if self.side == SIDE_INTERFACE:
            ap, am = 0.5 / self.beta[PLUS], 0.5 / self.beta[MINUS]
            minus_node, plus_node = (f, q) if lab_f == MINUS else (q, f)
            links = [(minus_node, ap / (ap + am)), (plus_node, am / (ap + am))]
            return ("V", 0.5), links, None
        inside = self.side == SIDE_INTERIOR
        root, _ = self.geom.crossing(xf, d, s, inside, g.h)
        lo_c, hi_c = min(xf[d], xf[d] + s * g.h), max(xf[d], xf[d] + s * g.h)
        root = min(max(root, lo_c), hi_c)
        psi = abs(root - xf[d]) / g.h
        if self.shift:
            psi = max(psi, 0.5)
        xw = np.array(xf)
        xw[d] = root
        kind = "N" if self.bc == BC_NEUMANN else "V"
        return (kind, psi), [], ("wall", xw)

    def _regular_mask(self) -> np.ndarray:
        """Unknowns whose 2d neighbours are all unknowns of the same side."""
        lab = self.labels
        if getattr(self.grid, "periodic", False):
            n, dim = self.grid.n, self.grid.dim
            core = lab[tuple(slice(0, n) for _ in range(dim))]
            ok = (core == PLUS) | (core == MINUS)
            for d in range(dim):
                for s in (-1, 1):
                    ok &= np.roll(core, -s, axis=d) == core
            full = np.zeros(lab.shape, dtype=bool)
            full[tuple(slice(0, n) for _ in range(dim))] = ok
            return full.ravel(order="F")
        pad = np.pad(lab, 1, constant_values=255)
        ok = (lab == PLUS) | (lab == MINUS)
        core = tuple(slice(1, 1 + s) for s in lab.shape)
        for d in range(self.grid.dim):
            for s in (-1, 1):
                sl = list(core)
                sl[d] = slice(1 + s, 1 + s + lab.shape[d])
                ok &= pad[tuple(sl)] == lab
        return ok.ravel(order="F")

    def _assemble(self):
        rows, cols, vals = [], [], []
        h2 = self.grid.h ** 2
        dim = self.grid.dim
        reg = self._regular_mask()
        rn = np.nonzero(reg)[0]
        ri = self.uindex[rn]
        rows.append(ri); cols.append(ri); vals.append(np.full(rn.size, -2.0 * dim / h2))
        for d in range(dim):
            for s in (-1, 1):
                if getattr(self.grid, "periodic", False):
                    i = (rn // self.strides[d]) % (self.grid.n + 1)
                    nb = rn + (np.mod(i + s, self.grid.n) - i) * self.strides[d]
                else:
                    nb = rn + s * self.strides[d]
                rows.append(ri); cols.append(self.uindex[nb])
                vals.append(np.full(rn.size, 1.0 / h2))
        r_l, c_l, v_l = [], [], []
        for f in np.nonzero(~reg & (self.uindex >= 0))[0]:
            f = int(f)
            r = self.uindex[f]
            for d in range(dim):
                ql = self._neighbour(f, d, -1)
                qr = self._neighbour(f, d, +1)
                left, llinks, ldata = self._wall(f, ql, d, -1)
                right, rlinks, rdata = self._wall(f, qr, d, +1)
                cl, cc, cr = row_1d(left, right)
                r_l.append(r); c_l.append(r); v_l.append(cc / h2)
                for links, cside, dat in ((llinks, cl, ldata), (rlinks, cr, rdata)):
                    for node, wgt in links:
                        r_l.append(r); c_l.append(self.uindex[node]); v_l.append(cside * wgt / h2)
                    if dat is not None and cside != 0.0:
                        if dat[0] == "wall":
                            self.wall_terms.append((r, cside / h2, dat[1]))
                        else:
                            self.box_terms.append((r, cside / h2, dat[1]))
        rows.append(np.array(r_l, dtype=np.int64)); cols.append(np.array(c_l, dtype=np.int64))
        vals.append(np.array(v_l, dtype=np.float64))
        nu = self.unknowns.size
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(nu, nu))
