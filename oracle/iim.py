"""The high-order immersed-interface discretisation, assembled (oracle).

Sec. 2.1-2.3 of the paper.  At an unknown node i of side sigma,
    (L u)_i = beta_sigma / h^2 * sum_d sum_{j=-w..w} a_|j| u~(i + j e_d),
where u~ is the *extended function* of the 1D stencil: the grid value at points
of side sigma, and, at points off side sigma, the least-squares polynomial p_c
of the first control point the stencil crosses in that direction (a stencil
that crosses a thin sliver of the other side and comes back uses grid values
again beyond it).  Collecting the coefficients of the
unknowns and of the boundary data gives the linear system
    L_Omega u_Omega + L_Gamma u_Gamma = f_Omega,
whose solution is what the iterative method reaches.

Closures (Sec. 2.1, 2.2):
  Dirichlet  u(x_c) = ubar;
  Neumann    u(x_c) = (qbar - beta sum_i s_i u_i) / (beta s_c), s = d/dn stencil;
  interface  D = beta+ s_c+ - beta- s_c-,
             ubar = -(beta+ sum s_i+ u_i+ - beta- sum s_i- u_i-) / D,
             u+(x_c) = ubar + (j1 - beta- s_c- j0) / D,
             u-(x_c) = ubar + (j1 - beta+ s_c+ j0) / D.
Box faces (a reading; the paper's box is periodic or absent): a face node holds
its known value; a stencil point beyond the face takes the degree-(k-1)
Lagrange extrapolation through the face value and the k-1 nearest nodes inside.

Data vector u_Gamma: per control point ubar or qbar (or j0, j1 interleaved),
followed by one value per grid node (flat, x fastest) of which only the box-face
entries are used.

Post-processing (Sec. 2.4): grad u at the unknowns by the order-n central
first derivative with the same extension (grad_row, gradient), the
boundary quantity left open by the condition at every control point
(boundary_quantity), and the gradient of the solved side's fit at every
control point (wall_gradient: the wall derivatives from which the potential-flow
application of Sec. 4.4.2 recovers the wall velocity and C_p).

Parity: pinned by the patch test (the operator is exact on polynomials of degree
<= k-1 with matching data), by the order-n convergence of the solution and by
the spectrum bounds of Sec. 2.5 (tests/test_oracle_iim.py).  The gradient and
the boundary quantity are pinned by patch tests (exact on polynomials of degree
<= n, resp. <= k-1, given exact nodal values) and by their order-n convergence
on solved problems; the wall gradient by a patch test (exact on degree k-1),
by its normal component equalling the Neumann datum for any nodal values, and
by the pressure coefficient of potential flow past a cylinder converging at
order 4 to its closed form (tests/test_oracle_post.py).
"""
from __future__ import annotations

import math
from collections import defaultdict
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

from . import INACTIVE, PLUS, MINUS, BOX
from .fd import stencil, first_stencil, half_width
from .geometry import (Grid, make_geometry, node_labels, control_points, check_curvature,
                       GeometryUnresolved, SIDE_INTERIOR, SIDE_EXTERIOR, SIDE_INTERFACE)
from .lsq import ls_stencil, default_axes

BC_DIRICHLET, BC_NEUMANN, BC_JUMP = 0, 1, 2


def lagrange_extrapolation(k: int, s: int) -> List[float]:
    """Weights l_t(-s), t = 0..k-1, of the Lagrange basis on the points 0..k-1
    (t = distance from the face, into the domain) evaluated s steps beyond it."""
    x = -float(s)
    out = []
    for t in range(k):
        v = 1.0
        for u in range(k):
            if u != t:
                v *= (x - u) / (t - u)
        out.append(v)
    return out


class IIMProblem:
    def __init__(self, dim: int, n: int, geom_kind: int, geom_params, side: int, bc: int,
                 beta_plus: float = 1.0, beta_minus: float = 1.0, order_n: int = 4,
                 order_k: int = 5, axes=None, check_kappa: bool = True, lo: float = -1.0, hi: float = 1.0,
                 periodic: bool = False):
        self.dim, self.n = dim, n
        self.periodic = periodic
        self.grid = Grid(dim, n, (hi - lo) / n, lo, periodic)
        self.geom = make_geometry(geom_kind, list(geom_params), dim)
        self.geom_kind, self.geom_params = geom_kind, list(geom_params)
        self.side, self.bc = side, bc
        self.beta = {PLUS: float(beta_plus), MINUS: float(beta_minus)}
        self.order_n, self.order_k = order_n, order_k
        self.w = half_width(order_n)
        self.a = stencil(order_n)
        self.g = first_stencil(order_n)
        self.axes = axes if axes is not None else default_axes(dim, order_k)
        self.labels = node_labels(self.grid, self.geom, side)
        self.lab_flat = self.labels.ravel(order="F")
        self.cps = control_points(self.grid, self.geom, side, self.labels)
        if check_kappa:
            check_curvature(self.cps, self.grid.h)
        self.seg = {}
        for c, cp in enumerate(self.cps):
            self.seg[(cp.axis, cp.p)] = c
        self.sides = [PLUS, MINUS] if side == SIDE_INTERFACE else [PLUS]
        self.unknowns = np.nonzero((self.lab_flat == PLUS) | (self.lab_flat == MINUS))[0]
        self.uindex = np.full(self.lab_flat.size, -1, dtype=np.int64)
        self.uindex[self.unknowns] = np.arange(self.unknowns.size)
        self.ncp = len(self.cps)
        self.ncp_data = self.ncp * (2 if bc == BC_JUMP else 1)
        self.ndata = self.ncp_data + self.lab_flat.size
        self.strides = [(n + 1) ** d for d in range(dim)]
        self._st = {}

    # -- least-squares stencils ------------------------------------------------
    def stencil(self, c: int, side: int):
        key = (c, side)
        if key not in self._st:
            need_d = self.bc in (BC_NEUMANN, BC_JUMP)
            self._st[key] = ls_stencil(self.grid, self.lab_flat, self.cps[c], side,
                                       self.order_k, self.w, need_d, self.axes)
        return self._st[key]

    def stencil_d(self, c: int, side: int):
        """The fit of control point c with the normal-derivative row (column
        w of S) also for Dirichlet problems, whose ghosts do not need it."""
        if self.bc in (BC_NEUMANN, BC_JUMP):
            return self.stencil(c, side)
        key = ("d", c, side)
        if key not in self._st:
            self._st[key] = ls_stencil(self.grid, self.lab_flat, self.cps[c], side,
                                       self.order_k, self.w, True, self.axes)
        return self._st[key]

    def stencil_g(self, c: int, side: int):
        """The fit of control point c with the normal-derivative row (column
        w) and the Cartesian derivative rows d/dx_d (columns w+1..w+dim)."""
        key = ("g", c, side)
        if key not in self._st:
            self._st[key] = ls_stencil(self.grid, self.lab_flat, self.cps[c], side,
                                       self.order_k, self.w, True, self.axes, with_grad=True)
        return self._st[key]

    def wall_gradient(self, u: np.ndarray, u_gamma: np.ndarray) -> np.ndarray:
        """Gradient of the solved side's fit at every control point, (ncp, dim)
        (the wall derivatives of Sec. 4.4.2): grad p_c(x_c) = s_c U_c + sum_i
        s_i u_i with the Cartesian derivative rows s of the fit and U_c the
        fit's value at x_c,
          Dirichlet  U_c = ubar;
          Neumann    U_c = (qbar - beta sum_i s^n_i u_i) / (beta s^n_c), the
                     closure of the normal row s^n;
          interface  U_c = u+(x_c) from the interface closure (the Omega^+ fit).
        """
        uf = np.zeros(self.lab_flat.size)
        uf[self.unknowns] = u
        w, dim = self.w, self.dim
        out = np.empty((self.ncp, dim))
        for c in range(self.ncp):
            st = self.stencil_g(c, PLUS)
            sn = st.S[:, w]
            su = lambda col: sum(st.S[1 + a, col] * uf[f] for a, f in enumerate(st.idx))
            if self.bc == BC_DIRICHLET:
                uc = u_gamma[c]
            elif self.bc == BC_NEUMANN:
                beta = self.beta[PLUS]
                uc = (u_gamma[c] - beta * su(w)) / (beta * sn[0])
            else:
                stm = self.stencil_g(c, MINUS)
                snm = stm.S[:, w]
                bp, bm = self.beta[PLUS], self.beta[MINUS]
                D = bp * sn[0] - bm * snm[0]
                sm_u = sum(snm[1 + a] * uf[f] for a, f in enumerate(stm.idx))
                ubar = -(bp * su(w) - bm * sm_u) / D
                j0, j1 = u_gamma[2 * c], u_gamma[2 * c + 1]
                uc = ubar + (j1 - bm * snm[0] * j0) / D
            for d in range(dim):
                out[c, d] = st.S[0, w + 1 + d] * uc + su(w + 1 + d)
        return out

    def boundary_quantity(self, u: np.ndarray, u_gamma: np.ndarray) -> np.ndarray:
        """The boundary quantity the condition leaves open, one value per
        control point (Sec. 2.4, boundary-quantity convergence):
          Dirichlet  du/dn(x_c) = s_c ubar + sum_i s_i u_i, s the normal-
                     derivative stencil of the fit;
          Neumann    u(x_c) = (qbar - beta sum_i s_i u_i) / (beta s_c);
          interface  du+/dn(x_c) = s+_c u+(x_c) + sum_i s+_i u+_i, with u+(x_c)
                     from the interface closure.
        n is the control point's normal (from Omega^- into Omega^+)."""
        uf = np.zeros(self.lab_flat.size)
        uf[self.unknowns] = u
        w = self.w
        out = np.empty(self.ncp)
        for c in range(self.ncp):
            if self.bc == BC_DIRICHLET:
                st = self.stencil_d(c, PLUS)
                sn = st.S[:, w]
                out[c] = sn[0] * u_gamma[c] + sum(sn[1 + a] * uf[f] for a, f in enumerate(st.idx))
            elif self.bc == BC_NEUMANN:
                st = self.stencil(c, PLUS)
                sn = st.S[:, w]
                beta = self.beta[PLUS]
                out[c] = (u_gamma[c] - beta * sum(sn[1 + a] * uf[f] for a, f in enumerate(st.idx))) / (beta * sn[0])
            else:
                stp, stm = self.stencil(c, PLUS), self.stencil(c, MINUS)
                snp, snm = stp.S[:, w], stm.S[:, w]
                bp, bm = self.beta[PLUS], self.beta[MINUS]
                D = bp * snp[0] - bm * snm[0]
                sp_u = sum(snp[1 + a] * uf[f] for a, f in enumerate(stp.idx))
                sm_u = sum(snm[1 + a] * uf[f] for a, f in enumerate(stm.idx))
                ubar = -(bp * sp_u - bm * sm_u) / D
                j0, j1 = u_gamma[2 * c], u_gamma[2 * c + 1]
                up = ubar + (j1 - bm * snm[0] * j0) / D
                out[c] = snp[0] * up + sp_u
        return out

    def ghost(self, c: int, side: int, j: int) -> Tuple[Dict[int, float], Dict[int, float]]:
        """Ghost value j (1..w) of control point c on `side` as a linear
        combination of grid values (flat index -> coefficient) and of data
        entries (data index -> coefficient)."""
        coef: Dict[int, float] = defaultdict(float)
        data: Dict[int, float] = defaultdict(float)
        w = self.w
        st = self.stencil(c, side)
        sg = st.S[:, j - 1]
        if self.bc == BC_DIRICHLET:
            for alpha, f in enumerate(st.idx):
                coef[f] += sg[1 + alpha]
            data[c] += sg[0]
        elif self.bc == BC_NEUMANN:
            beta = self.beta[PLUS]
            sn = st.S[:, w]
            # u(x_c) = (qbar - beta sum s_i u_i) / (beta s_c)
            for alpha, f in enumerate(st.idx):
                coef[f] += sg[1 + alpha] - sg[0] * sn[1 + alpha] / sn[0]
            data[c] += sg[0] / (beta * sn[0])
        else:
            stp, stm = self.stencil(c, PLUS), self.stencil(c, MINUS)
            snp, snm = stp.S[:, w], stm.S[:, w]
            bp, bm = self.beta[PLUS], self.beta[MINUS]
            D = bp * snp[0] - bm * snm[0]
            # ubar = -(beta+ sum s+ u+ - beta- sum s- u-) / D
            ubar: Dict[int, float] = defaultdict(float)
            for alpha, f in enumerate(stp.idx):
                ubar[f] += -bp * snp[1 + alpha] / D
            for alpha, f in enumerate(stm.idx):
                ubar[f] += bm * snm[1 + alpha] / D
            for f, v in ubar.items():
                coef[f] += sg[0] * v
            if side == PLUS:
                data[2 * c + 1] += sg[0] / D
                data[2 * c] += sg[0] * (-bm * snm[0] / D)
            else:
                data[2 * c + 1] += sg[0] / D
                data[2 * c] += sg[0] * (-bp * snp[0] / D)
            for alpha, f in enumerate(st.idx):
                coef[f] += sg[1 + alpha]
        return coef, data

    # -- operator rows ---------------------------------------------------------
    def _step(self, f: int, d: int, s: int):
        """Flat index of f + s e_d, or None outside the grid (taken modulo n
        on a periodic grid)."""
        i = (f // self.strides[d]) % (self.n + 1)
        if self.periodic:
            return f + (((i + s) % self.n) - i) * self.strides[d]
        if not 0 <= i + s <= self.n:
            return None
        return f + s * self.strides[d]

    def _half_line(self, f: int, side: int, d: int, dr: int, wts, coef, data) -> None:
        """Adds sum_{j=1..w} wts[j] u~(f + dr j e_d) to (coef, data): u~ is the
        extended function of the 1D stencil of node f on `side` (grid values on
        the side, the least-squares polynomial of the first crossing beyond it,
        box data and extrapolation past a box face)."""
        state, c, j0, face, jf = "u", None, None, None, None
        prev = f
        for j in range(1, self.w + 1):
            q = self._step(f, d, dr * j)
            wj = wts[j]
            if state == "u":
                if q is None:
                    raise GeometryUnresolved("stencil leaves the grid")
                lab = self.lab_flat[q]
                if lab == side:
                    coef[q] += wj
                elif lab == BOX:
                    state, face, jf = "box", q, j
                    data[self.ncp_data + q] += wj
                else:
                    # the segment's lower node: the one whose +e_d neighbour is the other
                    key = (d, prev if dr > 0 else q)
                    c = self.seg[key]
                    assert self.cps[c].a[side] == prev
                    state, j0 = "ghost", j
                    gc, gd = self.ghost(c, side, j - j0 + 1)
                    for k2, v in gc.items():
                        coef[k2] += wj * v
                    for k2, v in gd.items():
                        data[k2] += wj * v
            elif state == "ghost":
                # the extended function is u itself wherever the point is
                # back on the stencil's side (a thin sliver of the other
                # side); p_c of the first crossing elsewhere
                if q is not None and self.lab_flat[q] == side:
                    coef[q] += wj
                    prev = q
                    continue
                if q is not None and self.lab_flat[q] == BOX:
                    data[self.ncp_data + q] += wj
                    prev = q
                    continue
                gc, gd = self.ghost(c, side, j - j0 + 1)
                for k2, v in gc.items():
                    coef[k2] += wj * v
                for k2, v in gd.items():
                    data[k2] += wj * v
            else:  # beyond a box face: 1D extrapolation
                s = j - jf
                lw = lagrange_extrapolation(self.order_k, s)
                data[self.ncp_data + face] += wj * lw[0]
                for t in range(1, self.order_k):
                    node = self._step(face, d, -dr * t)
                    if node is None or self.lab_flat[node] != side:
                        raise GeometryUnresolved("box extrapolation line leaves the side")
                    coef[node] += wj * lw[t]
            prev = q

    def row(self, f: int) -> Tuple[Dict[int, float], Dict[int, float]]:
        """Row of unknown node f: (grid coefficients, data coefficients)."""
        side = int(self.lab_flat[f])
        assert side in (PLUS, MINUS)
        beta = self.beta[side]
        h2 = self.grid.h ** 2
        coef: Dict[int, float] = defaultdict(float)
        data: Dict[int, float] = defaultdict(float)
        coef[f] += beta * self.dim * self.a[0] / h2
        wts = [0.0] + [beta * self.a[j] / h2 for j in range(1, self.w + 1)]
        for d in range(self.dim):
            for dr in (1, -1):
                self._half_line(f, side, d, dr, wts, coef, data)
        return coef, data

    def grad_row(self, f: int, d: int) -> Tuple[Dict[int, float], Dict[int, float]]:
        """d/dx_d of u at unknown node f (the gradient post-processing of
        Sec. 2.3): the central first-derivative stencil of order n along axis
        d, with the same immersed-interface extension as the Laplacian, so the
        boundary conditions enter through the ghost values."""
        side = int(self.lab_flat[f])
        assert side in (PLUS, MINUS)
        h = self.grid.h
        coef: Dict[int, float] = defaultdict(float)
        data: Dict[int, float] = defaultdict(float)
        for dr in (1, -1):
            wts = [0.0] + [dr * self.g[j - 1] / h for j in range(1, self.w + 1)]
            self._half_line(f, side, d, dr, wts, coef, data)
        return coef, data

    def gradient(self, u: np.ndarray, u_gamma: np.ndarray) -> np.ndarray:
        """grad u at every unknown, shape (unknowns, dim), from the unknowns u
        and the data vector u_Gamma."""
        uf = np.zeros(self.lab_flat.size)
        uf[self.unknowns] = u
        out = np.empty((self.unknowns.size, self.dim))
        for r, f in enumerate(self.unknowns):
            for d in range(self.dim):
                coef, data = self.grad_row(int(f), d)
                out[r, d] = sum(c * uf[q] for q, c in coef.items()) + sum(c * u_gamma[q] for q, c in data.items())
        return out

    # -- assembly ----------------------------------------------------------------
    def regular_mask(self) -> np.ndarray:
        """Unknowns whose whole stencil stays on their own side (flat mask)."""
        w = self.w
        lab = self.labels
        if self.periodic:
            n = self.n
            core = lab[tuple(slice(0, n) for _ in range(self.dim))]
            ok = (core == PLUS) | (core == MINUS)
            for d in range(self.dim):
                for s in list(range(-w, 0)) + list(range(1, w + 1)):
                    ok &= np.roll(core, -s, axis=d) == core
            full = np.zeros(lab.shape, dtype=bool)
            full[tuple(slice(0, n) for _ in range(self.dim))] = ok
            return full.ravel(order="F")
        pad = np.pad(lab, w, constant_values=255)
        ok = (lab == PLUS) | (lab == MINUS)
        core = tuple(slice(w, w + s) for s in lab.shape)
        for d in range(self.dim):
            for s in list(range(-w, 0)) + list(range(1, w + 1)):
                sl = list(core)
                sl[d] = slice(w + s, w + s + lab.shape[d])
                ok &= pad[tuple(sl)] == lab
        return ok.ravel(order="F")

    def assemble(self):
        nu = self.unknowns.size
        reg = self.regular_mask()
        rows, cols, vals = [], [], []
        drows, dcols, dvals = [], [], []
        h2 = self.grid.h ** 2
        reg_nodes = np.nonzero(reg)[0]
        beta_node = np.where(self.lab_flat[reg_nodes] == PLUS, self.beta[PLUS], self.beta[MINUS])
        ri = self.uindex[reg_nodes]
        rows.append(ri); cols.append(ri); vals.append(beta_node * self.dim * self.a[0] / h2)
        for d in range(self.dim):
            for j in range(1, self.w + 1):
                for s in (j, -j):
                    if self.periodic:
                        i = (reg_nodes // self.strides[d]) % (self.n + 1)
                        nb = reg_nodes + (np.mod(i + s, self.n) - i) * self.strides[d]
                    else:
                        nb = reg_nodes + s * self.strides[d]
                    rows.append(ri); cols.append(self.uindex[nb]); vals.append(beta_node * self.a[j] / h2)
        for f in np.nonzero(~reg & (self.uindex >= 0))[0]:
            coef, data = self.row(int(f))
            r = self.uindex[f]
            for k2, v in coef.items():
                ui = self.uindex[k2]
                assert ui >= 0
                rows.append(np.array([r])); cols.append(np.array([ui])); vals.append(np.array([v]))
            for k2, v in data.items():
                drows.append(r); dcols.append(k2); dvals.append(v)
        L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nu, nu))
        LG = sp.csr_matrix((np.array(dvals, dtype=np.float64), (np.array(drows, dtype=np.int64),
                            np.array(dcols, dtype=np.int64))), shape=(nu, self.ndata))
        self.L, self.LG = L, LG
        return L, LG

    # -- data and right-hand side -------------------------------------------------
    def cp_arrays(self):
        xyz = np.array([cp.x for cp in self.cps]).reshape(-1, self.dim)
        nrm = np.array([cp.n for cp in self.cps]).reshape(-1, self.dim)
        return xyz, nrm

    def data_vector(self, cp_data: np.ndarray, box_full: np.ndarray = None) -> np.ndarray:
        box = np.zeros(self.lab_flat.size) if box_full is None else np.asarray(box_full).ravel(order="F")
        return np.concatenate([np.asarray(cp_data, dtype=np.float64).ravel(), box])

    def rhs(self, f_full: np.ndarray, u_gamma: np.ndarray) -> np.ndarray:
        """b = f_Omega - L_Gamma u_Gamma on the unknowns."""
        if not hasattr(self, "LG"):
            self.assemble()
        return np.asarray(f_full).ravel(order="F")[self.unknowns] - self.LG @ u_gamma

    def to_full(self, v: np.ndarray, fill=0.0) -> np.ndarray:
        out = np.full(self.lab_flat.size, fill, dtype=np.float64)
        out[self.unknowns] = v
        return out.reshape(self.grid.shape, order="F")

    def from_full(self, a: np.ndarray) -> np.ndarray:
        return np.asarray(a).ravel(order="F")[self.unknowns]

    def apply_rows(self, nodes, x_full: np.ndarray, with_data: bool = False,
                   u_gamma: np.ndarray = None) -> np.ndarray:
        """(L_Omega x)_i (+ (L_Gamma u_Gamma)_i) for the listed flat nodes, one row
        at a time (used for sampled checks on grids too large to assemble)."""
        xf = np.asarray(x_full).ravel(order="F")
        out = np.empty(len(nodes))
        for k, f in enumerate(nodes):
            coef, data = self.row(int(f))
            v = sum(c * xf[q] for q, c in coef.items())
            if with_data:
                v += sum(c * u_gamma[q] for q, c in data.items())
            out[k] = v
        return out

    def direct_solve(self, b: np.ndarray) -> np.ndarray:
        import scipy.sparse.linalg as spla
        if not hasattr(self, "L"):
            self.assemble()
        return spla.spsolve(self.L.tocsc(), b)
