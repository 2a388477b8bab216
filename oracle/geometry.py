"""Analytic level sets, node labels and control points (oracle).

Sec. 2.1 of the paper: a *control point* x_c is the intersection of a grid line
segment with the immersed surface Gamma; the grid point whose 1D stencil crosses
Gamma is *affected*.  The level set phi < 0 marks the inside of the body.

Readings used where the paper is silent (all shared with the GPU library):
  * vertex-centred grid, nodes x_i = -1 + i h, i = 0..n, h = 2/n;
  * a node with phi = 0 is not solved for in boundary problems; in interface
    problems phi <= 0 is Omega^-;
  * box-face nodes carry known Dirichlet values when the box bounds the domain;
  * n points from Omega^- into Omega^+ (into the solved region).

Parity: labels are pinned by exact counts on symmetric cases and by the
consistency of the crossings with them (tests/test_oracle_geometry.py).
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

from . import INACTIVE, PLUS, MINUS, BOX

SIDE_INTERIOR, SIDE_EXTERIOR, SIDE_INTERFACE = 0, 1, 2
GEOM_SPHERE, GEOM_STAR2D, GEOM_SPHERE_UNION, GEOM_GYROID = 0, 1, 2, 3


class Grid:
    """Uniform vertex-centred grid on [lo, lo + n h]^dim with n intervals per
    axis ([-1, 1] by default).  Coarse multigrid levels use the same origin
    and spacing h * 2^level.

    periodic: the domain is periodic in every direction (Sec. 2.3: the
    augmented system covers periodic problems); node n is then the image of
    node 0 along each axis, stored but never an unknown, and every neighbour
    index is taken modulo n (`wrap`)."""

    def __init__(self, dim: int, n: int, h: float = None, lo: float = -1.0, periodic: bool = False):
        self.dim = dim
        self.n = n
        self.h = (2.0 / n) if h is None else h
        self.lo = lo
        self.periodic = periodic
        self.shape = (n + 1,) * dim

    def wrap(self, i):
        """Index i taken into 0..n-1 (periodic grids); unchanged otherwise."""
        return np.mod(i, self.n) if self.periodic else i

    def coord(self, i):
        return self.lo + np.asarray(i) * self.h

    def node_coords(self) -> List[np.ndarray]:
        x1 = self.lo + np.arange(self.n + 1) * self.h
        return list(np.meshgrid(*([x1] * self.dim), indexing="ij"))

    def flat(self, idx) -> int:
        """Flat index with x fastest: ix + (n+1) iy + (n+1)^2 iz."""
        f = 0
        for d in reversed(range(self.dim)):
            f = f * (self.n + 1) + int(idx[d])
        return f

    def unflat(self, f: int) -> Tuple[int, ...]:
        out = []
        for d in range(self.dim):
            out.append(f % (self.n + 1))
            f //= (self.n + 1)
        return tuple(out)

    def inside(self, idx) -> bool:
        return all(0 <= int(i) <= self.n for i in idx)


# ---------------------------------------------------------------------------
# level sets
# ---------------------------------------------------------------------------
class Sphere:
    """phi = |x - c| - r (circle in 2D).  Classification compares the squared
    distance (summed over axes in x, y, z order) with r*r, so that it is exact
    for dyadic coordinates."""

    def __init__(self, center, r):
        self.c = [float(v) for v in center]
        self.r = float(r)

    def sign(self, X):
        d2 = 0.0
        for d in range(len(self.c)):
            t = X[d] - self.c[d]
            d2 = d2 + t * t
        return np.sign(d2 - self.r * self.r)

    def crossing(self, xa, axis, dir_, solved_inside: bool, h: float = None):
        """Root of phi on the segment from node xa (the solved-side node) to
        xa + dir_*h e_axis: walking from xa, the exit point of the sphere when
        xa is inside, the entry point otherwise.  Returns the coordinate along
        `axis` (not yet clamped) and the sphere index 0."""
        q = self.r * self.r
        for o in range(len(self.c)):
            if o != axis:
                t = xa[o] - self.c[o]
                q = q - t * t
        s = math.sqrt(max(q, 0.0))
        if solved_inside:
            return self.c[axis] + dir_ * s, 0
        return self.c[axis] - dir_ * s, 0

    def grad_dir(self, x, which=0):
        g = np.array([x[d] - self.c[d] for d in range(len(self.c))])
        return g / np.linalg.norm(g)

    def curvature(self, x, which=0):
        return 1.0 / self.r


def _cheb_t_u(L: int, c: float):
    """T_L(c) and U_{L-1}(c) by the three-term recurrences."""
    t0, t1 = 1.0, c
    u0, u1 = 1.0, 2.0 * c   # U_0, U_1
    if L == 0:
        return 1.0, 0.0
    for _ in range(L - 1):
        t0, t1 = t1, 2.0 * c * t1 - t0
    if L == 1:
        return c, 1.0
    for _ in range(L - 2):
        u0, u1 = u1, 2.0 * c * u1 - u0
    return t1, u1


class Star2D:
    """phi = rho - (r0 + eps cos(L theta)), theta measured about the centre.
    cos(L theta) = T_L(cos theta) (Chebyshev), so phi uses only +, *, / and sqrt."""

    def __init__(self, cx, cy, r0, eps, lobes):
        self.cx, self.cy, self.r0, self.eps, self.L = float(cx), float(cy), float(r0), float(eps), int(round(lobes))

    def phi_scalar(self, x, y):
        dx = x - self.cx
        dy = y - self.cy
        rho = math.sqrt(dx * dx + dy * dy)
        c = dx / rho if rho > 0.0 else 1.0
        t, _ = _cheb_t_u(self.L, c)
        return rho - (self.r0 + self.eps * t)

    def sign(self, X):
        """Vectorised form of phi_scalar (same operations, same order)."""
        x = np.asarray(X[0], dtype=np.float64)
        y = np.asarray(X[1], dtype=np.float64)
        dx = x - self.cx
        dy = y - self.cy
        rho = np.sqrt(dx * dx + dy * dy)
        with np.errstate(invalid="ignore", divide="ignore"):
            c = np.where(rho > 0.0, dx / np.where(rho > 0.0, rho, 1.0), 1.0)
        t0, t1 = np.ones_like(c), c
        for _ in range(self.L - 1):
            t0, t1 = t1, 2.0 * c * t1 - t0
        t = t1 if self.L >= 1 else np.ones_like(c)
        return np.sign(rho - (self.r0 + self.eps * t))

    def crossing(self, xa, axis, dir_, solved_inside=None, h: float = None):
        """Bisection (64 halvings) on the segment between the two nodes, using
        the sign of phi; a zero at an end point is the root."""
        lo_pt = list(xa)
        if dir_ < 0:
            lo_pt[axis] = xa[axis] - h
        hi_pt = list(lo_pt)
        hi_pt[axis] = lo_pt[axis] + h
        s_lo = np.sign(self.phi_scalar(*lo_pt))
        s_hi = np.sign(self.phi_scalar(*hi_pt))
        if s_lo == 0:
            return lo_pt[axis], 0
        if s_hi == 0:
            return hi_pt[axis], 0
        a, b = lo_pt[axis], hi_pt[axis]
        p = list(lo_pt)
        for _ in range(64):
            m = 0.5 * (a + b)
            p[axis] = m
            s = np.sign(self.phi_scalar(*p))
            if s == 0:
                return m, 0
            if s == s_lo:
                a = m
            else:
                b = m
        return 0.5 * (a + b), 0

    def grad_dir(self, x, which=0):
        dx = x[0] - self.cx
        dy = x[1] - self.cy
        rho = math.sqrt(dx * dx + dy * dy)
        c = dx / rho
        _, u = _cheb_t_u(self.L, c)
        dT = self.L * u                       # d T_L / dc
        r3 = rho * rho * rho
        gc = np.array([dy * dy / r3, -dx * dy / r3])   # grad of c = dx/rho
        g = np.array([dx / rho, dy / rho]) - self.eps * dT * gc
        return g / np.linalg.norm(g)

    def curvature(self, x, which=0):
        dx = x[0] - self.cx
        dy = x[1] - self.cy
        rho = math.sqrt(dx * dx + dy * dy)
        c, s = dx / rho, dy / rho
        t, u = _cheb_t_u(self.L, c)
        R = self.r0 + self.eps * t
        Rp = -self.eps * self.L * s * u           # R'(theta)
        Rpp = -self.eps * self.L * self.L * t     # R''(theta)
        return abs(R * R + 2 * Rp * Rp - R * Rpp) / (R * R + Rp * Rp) ** 1.5


class SphereUnion:
    """Union of spheres: a node is inside if inside any sphere, on Gamma if on
    some sphere and inside none, outside otherwise."""

    def __init__(self, spheres):
        self.spheres = [Sphere(c, r) for c, r in spheres]

    def sign(self, X):
        s = np.ones(np.shape(X[0]))
        on = np.zeros(np.shape(X[0]), dtype=bool)
        inside = np.zeros(np.shape(X[0]), dtype=bool)
        for sp in self.spheres:
            si = sp.sign(X)
            inside |= si < 0
            on |= si == 0
        s[on] = 0.0
        s[inside] = -1.0
        return s

    def crossing(self, xa, axis, dir_, solved_inside=False, h: float = None):
        """From the outside node xa towards its neighbour: the first entry
        point into any sphere whose chord overlaps the segment."""
        a0 = xa[axis]
        a1 = xa[axis] + dir_ * h
        lo, hi = min(a0, a1), max(a0, a1)
        best, best_i, best_x = None, -1, None
        for i, sp in enumerate(self.spheres):
            q = sp.r * sp.r
            for o in range(len(sp.c)):
                if o != axis:
                    t = xa[o] - sp.c[o]
                    q = q - t * t
            if q < 0.0:
                continue
            s = math.sqrt(q)
            c0, c1 = sp.c[axis] - s, sp.c[axis] + s
            if c1 < lo or c0 > hi:
                continue
            entry = c0 if dir_ > 0 else c1
            dist = (entry - a0) * dir_
            if best is None or dist < best:
                best, best_i, best_x = dist, i, entry
        return best_x, best_i

    def grad_dir(self, x, which=0):
        return self.spheres[which].grad_dir(x)

    def curvature(self, x, which=0):
        return 1.0 / self.spheres[which].r


# sin and cos for the gyroid from IEEE basic operations only (Cody-Waite
# reduction by pi/2 split into three parts, then the Taylor series of sin and
# cos on |r| <= pi/4 to degree 19 / 18, Horner form): the library evaluates
# the same steps, so both sides round every node's phi identically and their
# labels and bisection roots agree bit for bit (two libm implementations differ
# in the last bit, which decides the sign of phi at nodes within rounding of
# Gamma and grazing roots to about 1e-12).
_TWO_OVER_PI = 0.6366197723675814
_PIO2 = (1.570796325802803, 9.920935791635221e-10, 5.170182981794105e-19)
_SIN_C = (-0.16666666666666666, 0.008333333333333333, -0.0001984126984126984, 2.7557319223985893e-06,
          -2.505210838544172e-08, 1.6059043836821613e-10, -7.647163731819816e-13, 2.8114572543455206e-15,
          -8.22063524662433e-18)
_COS_C = (-0.5, 0.041666666666666664, -0.001388888888888889, 2.48015873015873e-05, -2.755731922398589e-07,
          2.08767569878681e-09, -1.1470745597729725e-11, 4.779477332387385e-14, -1.5619206968586225e-16)


def det_sincos(t):
    """(sin t, cos t) for float or float64 arrays, by the steps above."""
    t = np.asarray(t, dtype=np.float64)
    q = np.floor(t * _TWO_OVER_PI + 0.5)
    r = ((t - q * _PIO2[0]) - q * _PIO2[1]) - q * _PIO2[2]
    z = r * r
    ps = _SIN_C[-1]
    for c in reversed(_SIN_C[:-1]):
        ps = c + z * ps
    sn = r + r * (z * ps)
    pc = _COS_C[-1]
    for c in reversed(_COS_C[:-1]):
        pc = c + z * pc
    cs = 1.0 + z * pc
    m = np.mod(q, 4.0)
    sin_t = np.where(m == 0, sn, np.where(m == 1, cs, np.where(m == 2, -sn, -cs)))
    cos_t = np.where(m == 0, cs, np.where(m == 1, -sn, np.where(m == 2, -cs, sn)))
    return sin_t, cos_t


class Gyroid:
    """phi = cos(k1 x) sin(k2 y) + cos(k2 y) sin(k3 z) + cos(k3 z) sin(k1 x) - alpha
    (the paper's triply periodic heat-conduction domain, Sec. 4.4.1: the
    solved region is phi > 0), summed left to right, sin and cos by det_sincos."""

    def __init__(self, k1, k2, k3, alpha):
        self.k = (float(k1), float(k2), float(k3))
        self.alpha = float(alpha)

    def _trig(self, x):
        k1, k2, k3 = self.k
        sx, cx = det_sincos(k1 * np.asarray(x[0], dtype=np.float64))
        sy, cy = det_sincos(k2 * np.asarray(x[1], dtype=np.float64))
        sz, cz = det_sincos(k3 * np.asarray(x[2], dtype=np.float64))
        return sx, cx, sy, cy, sz, cz

    def phi(self, X):
        sx, cx, sy, cy, sz, cz = self._trig(X)
        return ((cx * sy + cy * sz) + cz * sx) - self.alpha

    def sign(self, X):
        return np.sign(self.phi(X))

    def crossing(self, xa, axis, dir_, solved_inside=None, h: float = None):
        """Bisection (64 halvings) on the segment between the two nodes, on the
        sign of phi; a zero at an end point is the root."""
        lo_pt = list(xa)
        if dir_ < 0:
            lo_pt[axis] = xa[axis] - h
        hi_pt = list(lo_pt)
        hi_pt[axis] = lo_pt[axis] + h
        s_lo = np.sign(self.phi(lo_pt))
        s_hi = np.sign(self.phi(hi_pt))
        if s_lo == 0:
            return lo_pt[axis], 0
        if s_hi == 0:
            return hi_pt[axis], 0
        a, b = lo_pt[axis], hi_pt[axis]
        p = list(lo_pt)
        for _ in range(64):
            m = 0.5 * (a + b)
            p[axis] = m
            sm = np.sign(self.phi(p))
            if sm == 0:
                return m, 0
            if sm == s_lo:
                a = m
            else:
                b = m
        return 0.5 * (a + b), 0

    def gradient(self, x):
        k1, k2, k3 = self.k
        sx, cx, sy, cy, sz, cz = (float(v) for v in self._trig(x))
        return np.array([-k1 * sx * sy + k1 * cz * cx,
                         k2 * cx * cy - k2 * sy * sz,
                         k3 * cy * cz - k3 * sz * sx])

    def hessian(self, x):
        k1, k2, k3 = self.k
        sx, cx, sy, cy, sz, cz = (float(v) for v in self._trig(x))
        H = np.empty((3, 3))
        H[0, 0] = -k1 * k1 * cx * sy - k1 * k1 * cz * sx
        H[1, 1] = -k2 * k2 * cx * sy - k2 * k2 * cy * sz
        H[2, 2] = -k3 * k3 * cy * sz - k3 * k3 * cz * sx
        H[0, 1] = H[1, 0] = -k1 * k2 * sx * cy
        H[1, 2] = H[2, 1] = -k2 * k3 * sy * cz
        H[0, 2] = H[2, 0] = -k1 * k3 * sz * cx
        return H

    def grad_dir(self, x, which=0):
        g = self.gradient(x)
        return g / np.linalg.norm(g)

    def curvature(self, x, which=0):
        """Largest absolute principal curvature of the level surface: the
        eigenvalues of the shape operator P H P / |grad phi| (P the tangent
        projector) other than the zero along the normal, from its trace and
        the sum of its principal 2x2 minors."""
        g = self.gradient(x)
        gn = np.linalg.norm(g)
        nrm = g / gn
        P = np.eye(3) - np.outer(nrm, nrm)
        Sh = P @ self.hessian(x) @ P / gn
        tr = np.trace(Sh)
        m2 = Sh[0, 0] * Sh[1, 1] - Sh[0, 1] * Sh[1, 0] + Sh[0, 0] * Sh[2, 2] - Sh[0, 2] * Sh[2, 0] \
            + Sh[1, 1] * Sh[2, 2] - Sh[1, 2] * Sh[2, 1]
        half = 0.5 * tr
        return abs(half) + math.sqrt(max(half * half - m2, 0.0))


def make_geometry(kind: int, params, dim: int):
    """Geometry from the parameter list of the C ABI: sphere [c..., r];
    star [cx, cy, r0, eps, lobes]; union [count, (c..., r) * count];
    gyroid [k1, k2, k3, alpha] (3D)."""
    if kind == GEOM_GYROID:
        return Gyroid(*params[:4])
    if kind == GEOM_SPHERE:
        g = Sphere(params[:-1], params[-1])
    elif kind == GEOM_STAR2D:
        g = Star2D(*params[:5])
    elif kind == GEOM_SPHERE_UNION:
        cnt = int(params[0])
        sp = []
        for i in range(cnt):
            base = 1 + (dim + 1) * i
            sp.append((params[base: base + dim], params[base + dim]))
        g = SphereUnion(sp)
    else:
        raise ValueError("unknown geometry kind")
    return g


# ---------------------------------------------------------------------------
# labels
# ---------------------------------------------------------------------------
class GeometryUnresolved(Exception):
    pass


def node_labels(grid: Grid, geom, side: int) -> np.ndarray:
    """Label per node (array indexed [ix, iy(, iz)]):
    PLUS = unknown in Omega^+, MINUS = unknown in Omega^- (interfaces only),
    BOX = box-face node with a known Dirichlet value, INACTIVE otherwise.
    Omega^+ is {phi < 0} for interior problems, {phi > 0} for exterior
    problems and interfaces; Omega^- = {phi <= 0} for interfaces."""
    X = grid.node_coords()
    s = geom.sign(X)
    if grid.periodic:
        # no box faces; nodes of the image planes (index n) are not unknowns
        image = np.zeros(grid.shape, dtype=bool)
        for d in range(grid.dim):
            idx = [slice(None)] * grid.dim
            idx[d] = grid.n
            image[tuple(idx)] = True
        lab = np.zeros(grid.shape, dtype=np.uint8)
        if side == SIDE_INTERIOR:
            lab[(s < 0) & ~image] = PLUS
        elif side == SIDE_EXTERIOR:
            lab[(s > 0) & ~image] = PLUS
        else:
            lab[(s <= 0) & ~image] = MINUS
            lab[(s > 0) & ~image] = PLUS
        return lab
    face = np.zeros(grid.shape, dtype=bool)
    for d in range(grid.dim):
        idx = [slice(None)] * grid.dim
        idx[d] = 0
        face[tuple(idx)] = True
        idx[d] = grid.n
        face[tuple(idx)] = True
    lab = np.zeros(grid.shape, dtype=np.uint8)
    if side == SIDE_INTERIOR:
        if np.any(face & (s <= 0)):
            raise GeometryUnresolved("body touches the box")
        lab[(s < 0) & ~face] = PLUS
    elif side == SIDE_EXTERIOR:
        if np.any(face & (s <= 0)):
            raise GeometryUnresolved("body touches the box")
        lab[(s > 0) & ~face] = PLUS
        lab[(s > 0) & face] = BOX
    else:
        if np.any(face & (s <= 0)):
            raise GeometryUnresolved("interface touches the box")
        lab[(s <= 0) & ~face] = MINUS
        lab[(s > 0) & ~face] = PLUS
        lab[(s > 0) & face] = BOX
    return lab


def is_crossing(la: int, lb: int, side: int) -> bool:
    """A control point lies on the segment between two nodes when one is an
    unknown and the other lies across Gamma (not a box-face node)."""
    if side == SIDE_INTERFACE:
        return {int(la), int(lb)} == {PLUS, MINUS}
    return {int(la), int(lb)} == {PLUS, INACTIVE}


class ControlPoint:
    __slots__ = ("axis", "p", "q", "x", "n", "kappa", "a", "dir", "which", "xa")

    def __repr__(self):
        return f"CP(axis={self.axis}, p={self.p}, x={self.x}, n={self.n})"


def control_points(grid: Grid, geom, side: int, labels: np.ndarray) -> List[ControlPoint]:
    """All control points, ordered by axis, then by the flat index of the
    lower node of the segment.  For each control point and each side sigma of
    the problem, a[sigma] is the adjacent unknown of that side and dir[sigma]
    the step (+1/-1 along the axis) from it towards Gamma."""
    if grid.periodic:
        return _control_points_periodic(grid, geom, side, labels)
    out: List[ControlPoint] = []
    lab_flat = labels.ravel(order="F")
    dim = grid.dim
    n1 = grid.n + 1
    strides = [n1 ** d for d in range(dim)]
    for axis in range(dim):
        # lower nodes p with p + e_axis inside the grid, in increasing flat order
        lower = [slice(None)] * dim
        upper = [slice(None)] * dim
        lower[axis] = slice(0, grid.n)
        upper[axis] = slice(1, grid.n + 1)
        la_arr = labels[tuple(lower)]
        lb_arr = labels[tuple(upper)]
        if side == SIDE_INTERFACE:
            mask = ((la_arr == PLUS) & (lb_arr == MINUS)) | ((la_arr == MINUS) & (lb_arr == PLUS))
        else:
            mask = ((la_arr == PLUS) & (lb_arr == INACTIVE)) | ((la_arr == INACTIVE) & (lb_arr == PLUS))
        idx = np.nonzero(mask)
        flat_p = np.zeros(idx[0].shape, dtype=np.int64)
        for d in reversed(range(dim)):
            flat_p = flat_p * n1 + idx[d]
        for p in np.sort(flat_p):
            p = int(p)
            q = p + strides[axis]
            la, lb = lab_flat[p], lab_flat[q]
            assert is_crossing(la, lb, side)
            cp = ControlPoint()
            cp.axis, cp.p, cp.q = axis, p, q
            # solved-side node used for the root search
            if side == SIDE_INTERFACE:
                a_node = p if la == MINUS else q          # walk from Omega^-
                inside = True
            else:
                a_node = p if la == PLUS else q
                inside = (side == SIDE_INTERIOR)
            dir_ = 1 if a_node == p else -1
            xa = [float(grid.coord(v)) for v in grid.unflat(a_node)]
            root, which = geom.crossing(xa, axis, dir_, inside, grid.h)
            lo_c = float(grid.coord(grid.unflat(p)[axis]))
            hi_c = float(grid.coord(grid.unflat(q)[axis]))
            root = min(max(root, lo_c), hi_c)
            x = list(xa)
            x[axis] = root
            cp.x = np.array(x)
            cp.which = which
            g = geom.grad_dir(cp.x, which)       # direction of grad phi (outward)
            cp.n = -g if side == SIDE_INTERIOR else g
            cp.kappa = geom.curvature(cp.x, which)
            cp.a, cp.dir = {}, {}
            if side == SIDE_INTERFACE:
                cp.a[PLUS] = p if la == PLUS else q
                cp.a[MINUS] = p if la == MINUS else q
            else:
                cp.a[PLUS] = p if la == PLUS else q
            for sg, node in cp.a.items():
                cp.dir[sg] = 1 if node == p else -1
            out.append(cp)
    return out


def _control_points_periodic(grid: Grid, geom, side: int, labels: np.ndarray) -> List[ControlPoint]:
    """Control points of a periodic grid: every segment from a node p with all
    indices in 0..n-1 to its neighbour p + e_axis, taken modulo n (the last
    segment of a line joins node n-1 to node 0 through the image node n).
    The segment's coordinates are unwrapped: x_c lies between x_p and
    x_p + h.  cp.xa[sigma] holds the unwrapped coordinates of the adjacent
    unknown of side sigma (node q is then at x_p + h e_axis)."""
    out: List[ControlPoint] = []
    dim, n = grid.dim, grid.n
    n1 = n + 1
    strides = [n1 ** d for d in range(dim)]
    core = labels[tuple(slice(0, n) for _ in range(dim))]
    for axis in range(dim):
        la_arr = core
        lb_arr = np.roll(core, -1, axis=axis)
        if side == SIDE_INTERFACE:
            mask = ((la_arr == PLUS) & (lb_arr == MINUS)) | ((la_arr == MINUS) & (lb_arr == PLUS))
        else:
            mask = ((la_arr == PLUS) & (lb_arr == INACTIVE)) | ((la_arr == INACTIVE) & (lb_arr == PLUS))
        idx = np.nonzero(mask)
        flat_p = np.zeros(idx[0].shape, dtype=np.int64)
        for d in reversed(range(dim)):
            flat_p = flat_p * n1 + idx[d]
        for p in np.sort(flat_p):
            p = int(p)
            ijk = list(grid.unflat(p))
            qk = list(ijk)
            qk[axis] = (qk[axis] + 1) % n
            q = grid.flat(qk)
            la, lb = labels[tuple(ijk)], labels[tuple(qk)]
            cp = ControlPoint()
            cp.axis, cp.p, cp.q = axis, p, q
            xp = [float(grid.coord(v)) for v in ijk]
            xq = list(xp)
            xq[axis] = xp[axis] + grid.h       # unwrapped
            if side == SIDE_INTERFACE:
                from_p = la == MINUS
                inside = True
            else:
                from_p = la == PLUS
                inside = (side == SIDE_INTERIOR)
            xa = xp if from_p else xq
            dir_ = 1 if from_p else -1
            root, which = geom.crossing(xa, axis, dir_, inside, grid.h)
            root = min(max(root, xp[axis]), xq[axis])
            x = list(xp)
            x[axis] = root
            cp.x = np.array(x)
            cp.which = which
            g = geom.grad_dir(cp.x, which)
            cp.n = -g if side == SIDE_INTERIOR else g
            cp.kappa = geom.curvature(cp.x, which)
            cp.a, cp.dir, cp.xa = {}, {}, {}
            sides = [PLUS, MINUS] if side == SIDE_INTERFACE else [PLUS]
            for sg in sides:
                at_p = la == sg
                cp.a[sg] = p if at_p else q
                cp.dir[sg] = 1 if at_p else -1
                cp.xa[sg] = np.array(xp if at_p else xq)
            out.append(cp)
    return out


def check_curvature(cps, h: float, limit: float = 0.25):
    """The curvature condition |kappa h| < 1/4 (Sec. 2.1)."""
    for cp in cps:
        if abs(cp.kappa * h) >= limit:
            raise GeometryUnresolved(f"|kappa h| = {abs(cp.kappa*h):.3f} >= 1/4 at {cp.x}")
