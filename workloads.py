"""Seeded synthetic workloads for the immersed-interface Poisson solver.

This module only *describes* problems: grid sizes, the analytic geometry
parameters, the manufactured solutions and the boundary/interface data they
induce, and the serving request stream.  It contains none of the method's
arithmetic (no level-set classification, no crossings, no stencils, no fits):
both the CPU oracle and the GPU library receive the geometry as parameters and
compute everything else themselves.  Data are sampled at the control points and
with the normals that the side under test reports.

Conventions (shared problem statement, Sec. 2.1-2.2 of the paper):
  * the PDE is  div(beta grad u) = f  (so f = beta * Laplacian(u));
  * n points from Omega^- into Omega^+ (into the solved region for boundary
    problems); Neumann data is  qbar = beta dn u;  interface data are
    j0 = u^+ - u^-  and  j1 = beta^+ dn u^+ - beta^- dn u^-.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

# geometry kinds, problem sides and boundary-condition kinds; the integer values
# are the ones the C ABI uses (include/iim.h)
GEOM_SPHERE, GEOM_STAR2D, GEOM_SPHERE_UNION, GEOM_GYROID = 0, 1, 2, 3
SIDE_INTERIOR, SIDE_EXTERIOR, SIDE_INTERFACE = 0, 1, 2
BC_DIRICHLET, BC_NEUMANN, BC_JUMP = 0, 1, 2


@dataclasses.dataclass
class Manufactured:
    """A manufactured solution on each side: u, grad u, Laplacian u."""
    u_plus: Callable
    grad_plus: Callable
    lap_plus: Callable
    u_minus: Optional[Callable] = None
    grad_minus: Optional[Callable] = None
    lap_minus: Optional[Callable] = None


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    n: int
    geom_kind: int
    geom_params: List[float]
    side: int
    bc: int
    beta_plus: float = 1.0
    beta_minus: float = 1.0
    exact: Optional[Manufactured] = None
    precision: str = "fp64"       # fp64 | mixed32 | mixed16
    note: str = ""
    order: Tuple[int, int] = (4, 5)  # (n, k): the (4,5) scheme, or (6,7) in 2D
    orthogonalisation: int = 1       # solver's Arnoldi step: 1 CGS + second pass where needed, 0 CGS2
    cycle: str = "V"                 # preconditioner's multigrid cycle: V or W
    lo: float = -1.0                 # domain [lo, hi]^dim
    hi: float = 1.0
    periodic: bool = False           # periodic in every direction (node n is node 0's image)
    source: Optional[Callable] = None  # f(x...) overriding beta Lap(u) (problems without a closed-form u)

    # -- data sampling (pure evaluation of the manufactured solution) ----------
    def cp_data(self, xyz: np.ndarray, normal: np.ndarray) -> np.ndarray:
        """Boundary/interface data at control points xyz (ncp, dim) with unit
        normals (ncp, dim).  Returns (ncp,) or (ncp, 2) for jumps (j0, j1)."""
        ex = self.exact
        X = [xyz[:, d] for d in range(self.dim)]
        if self.bc == BC_DIRICHLET:
            return np.asarray(ex.u_plus(*X), dtype=np.float64)
        if self.bc == BC_NEUMANN:
            g = ex.grad_plus(*X)
            dn = sum(g[d] * normal[:, d] for d in range(self.dim))
            return self.beta_plus * np.asarray(dn, dtype=np.float64)
        gp = ex.grad_plus(*X)
        gm = ex.grad_minus(*X)
        dnp = sum(gp[d] * normal[:, d] for d in range(self.dim))
        dnm = sum(gm[d] * normal[:, d] for d in range(self.dim))
        j0 = ex.u_plus(*X) - ex.u_minus(*X)
        j1 = self.beta_plus * dnp - self.beta_minus * dnm
        return np.stack([np.asarray(j0, np.float64), np.asarray(j1, np.float64)], axis=1)

    def node_coords(self) -> List[np.ndarray]:
        """Full-grid node coordinates, arrays of shape (n+1,)*dim indexed [ix,iy(,iz)]."""
        h = (self.hi - self.lo) / self.n
        x1 = self.lo + np.arange(self.n + 1) * h
        return list(np.meshgrid(*([x1] * self.dim), indexing="ij"))

    def box_data(self) -> np.ndarray:
        """u^+ sampled on every grid node (only box-face nodes are read)."""
        X = self.node_coords()
        return np.asarray(self.exact.u_plus(*X), dtype=np.float64) * np.ones_like(X[0])

    def rhs(self, labels: np.ndarray) -> np.ndarray:
        """f = beta * Lap(u) on every node, chosen per side from `labels`
        (1 = Omega^+, 2 = Omega^-), zero elsewhere."""
        X = self.node_coords()
        ex = self.exact
        f = np.zeros(labels.shape)
        if self.source is not None:
            fs = self.source(*X) * np.ones_like(X[0])
            f[(labels == 1) | (labels == 2)] = fs[(labels == 1) | (labels == 2)]
            return f
        fp = self.beta_plus * ex.lap_plus(*X) * np.ones_like(X[0])
        f[labels == 1] = fp[labels == 1]
        if ex.lap_minus is not None:
            fm = self.beta_minus * ex.lap_minus(*X) * np.ones_like(X[0])
            f[labels == 2] = fm[labels == 2]
        return f

    def exact_solution(self, labels: np.ndarray) -> np.ndarray:
        X = self.node_coords()
        ex = self.exact
        u = np.full(labels.shape, np.nan)
        up = ex.u_plus(*X) * np.ones_like(X[0])
        u[labels == 1] = up[labels == 1]
        if ex.u_minus is not None:
            um = ex.u_minus(*X) * np.ones_like(X[0])
            u[labels == 2] = um[labels == 2]
        return u


# ---------------------------------------------------------------------------
# manufactured solutions
# ---------------------------------------------------------------------------
TWO_PI = 2.0 * math.pi
PI = math.pi


def ms_sin2pi_cos2pi() -> Manufactured:
    """u = sin(2 pi x) cos(2 pi y)."""
    u = lambda x, y: np.sin(TWO_PI * x) * np.cos(TWO_PI * y)
    g = lambda x, y: (TWO_PI * np.cos(TWO_PI * x) * np.cos(TWO_PI * y),
                      -TWO_PI * np.sin(TWO_PI * x) * np.sin(TWO_PI * y))
    lap = lambda x, y: -2.0 * TWO_PI ** 2 * u(x, y)
    return Manufactured(u, g, lap)


def ms_sin_pi_3d() -> Manufactured:
    """u = sin(pi x) sin(pi y) sin(pi z)."""
    u = lambda x, y, z: np.sin(PI * x) * np.sin(PI * y) * np.sin(PI * z)
    g = lambda x, y, z: (PI * np.cos(PI * x) * np.sin(PI * y) * np.sin(PI * z),
                         PI * np.sin(PI * x) * np.cos(PI * y) * np.sin(PI * z),
                         PI * np.sin(PI * x) * np.sin(PI * y) * np.cos(PI * z))
    lap = lambda x, y, z: -3.0 * PI ** 2 * u(x, y, z)
    return Manufactured(u, g, lap)


def ms_star_interface() -> Manufactured:
    """Inside (Omega^-): u = e^x cos y; outside (Omega^+): u = x^2 - y^2.
    Both harmonic, so f = 0 on both sides."""
    up = lambda x, y: x * x - y * y
    gp = lambda x, y: (2.0 * x, -2.0 * y)
    lp = lambda x, y: 0.0 * x
    um = lambda x, y: np.exp(x) * np.cos(y)
    gm = lambda x, y: (np.exp(x) * np.cos(y), -np.exp(x) * np.sin(y))
    lm = lambda x, y: 0.0 * x
    return Manufactured(up, gp, lp, um, gm, lm)


def ms_shifted_trig() -> Manufactured:
    """u = sin(2 pi x + 0.7) cos(2 pi y - 0.4): no symmetry about the origin,
    so a pure-Neumann problem on a centred body has a non-trivial discrete
    compatibility shift."""
    a, c = 0.7, -0.4
    u = lambda x, y: np.sin(TWO_PI * x + a) * np.cos(TWO_PI * y + c)
    g = lambda x, y: (TWO_PI * np.cos(TWO_PI * x + a) * np.cos(TWO_PI * y + c),
                      -TWO_PI * np.sin(TWO_PI * x + a) * np.sin(TWO_PI * y + c))
    lap = lambda x, y: -2.0 * TWO_PI ** 2 * u(x, y)
    return Manufactured(u, g, lap)


def ms_cos_sinh() -> Manufactured:
    """u = cos(2x) sinh(y) + z^2."""
    u = lambda x, y, z: np.cos(2 * x) * np.sinh(y) + z * z
    g = lambda x, y, z: (-2 * np.sin(2 * x) * np.sinh(y), np.cos(2 * x) * np.cosh(y), 2 * z)
    lap = lambda x, y, z: -3.0 * np.cos(2 * x) * np.sinh(y) + 2.0
    return Manufactured(u, g, lap)


def ms_body_flow(dim: int = 3, center=(0.0, 0.0, 0.0), radius: float = 0.5, u_inf=(1.0, 0.0, 0.0)) -> Manufactured:
    """Disturbance potential of a uniform flow u_inf past a sphere (3D) or a
    circular cylinder (2D) of radius R (textbook potential flow):
    Phi = R^dim (u_inf . d) / ((dim - 1) |d|^dim), d = x - centre.  It is
    harmonic, and the total velocity grad Phi + u_inf is tangent to the body,
    so dPhi/dn = -u_inf . n there (n the outward normal)."""
    c = [float(v) for v in center][:dim]
    Rd = float(radius) ** dim
    U = [float(v) for v in u_inf][:dim]
    k = 1.0 / (dim - 1)

    def parts(X):
        d = [X[i] - c[i] for i in range(dim)]
        r2 = sum(di * di for di in d)
        ud = sum(U[i] * d[i] for i in range(dim))
        return d, r2, ud

    def u(*X):
        d, r2, ud = parts(X)
        return k * Rd * ud / r2 ** (0.5 * dim)

    def g(*X):
        d, r2, ud = parts(X)
        return tuple(k * Rd * (U[i] / r2 ** (0.5 * dim) - dim * ud * d[i] / r2 ** (0.5 * dim + 1.0))
                     for i in range(dim))

    return Manufactured(u, g, lambda *X: 0.0 * X[0])


def body_flow_cp(xyz, center=(0.0, 0.0, 0.0), u_inf=(1.0, 0.0, 0.0)) -> np.ndarray:
    """Surface pressure coefficient of that flow on the body:
    C_p = 1 - (dim / (dim - 1))^2 sin^2(theta), theta the angle between
    x - centre and u_inf (1 - 4 sin^2 on the cylinder, 1 - 9/4 sin^2 on the sphere)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    dim = xyz.shape[1]
    d = xyz - np.asarray(center, dtype=np.float64)[None, :dim]
    U = np.asarray(u_inf, dtype=np.float64)[:dim]
    cos_t = d @ U / (np.linalg.norm(d, axis=1) * np.linalg.norm(U))
    return 1.0 - (dim / (dim - 1.0)) ** 2 * (1.0 - cos_t ** 2)


def potential_body(dim: int, n: int, precision: str = "fp64", center=(0.02, -0.03, 0.01),
                   radius: float = 0.5) -> Workload:
    """Exterior potential flow past one circle (2D) or sphere (3D): Neumann data
    -u_inf . n on the body, the exact potential on the box faces, f = 0 (the
    wall-velocity and pressure-coefficient recovery of the paper's
    potential-flow application, on a body whose answer is known in closed form)."""
    return Workload("potential_body", dim, n, GEOM_SPHERE, list(center)[:dim] + [radius], SIDE_EXTERIOR,
                    BC_NEUMANN, exact=ms_body_flow(dim, center, radius), precision=precision)


def ms_periodic(dim: int, phase=(0.3, -0.7, 0.45)) -> Manufactured:
    """A periodic solution of the unit box: u = prod_d sin(2 pi x_d + phase_d)
    (its mean over a period is zero)."""
    ph = [float(v) for v in phase][:dim]

    def u(*X):
        out = 1.0
        for d in range(dim):
            out = out * np.sin(TWO_PI * X[d] + ph[d])
        return out

    def g(*X):
        comps = []
        for k in range(dim):
            t = TWO_PI * np.cos(TWO_PI * X[k] + ph[k])
            for d in range(dim):
                if d != k:
                    t = t * np.sin(TWO_PI * X[d] + ph[d])
            comps.append(t)
        return tuple(comps)

    return Manufactured(u, g, lambda *X: -dim * TWO_PI ** 2 * u(*X))


GYROID_K = 8.0 * math.pi
GYROID_ALPHA = -0.5 + 1e-9


def gyroid_params(k: float = GYROID_K, alpha: float = GYROID_ALPHA) -> List[float]:
    """phi = cos(k x) sin(k y) + cos(k y) sin(k z) + cos(k z) sin(k x) - alpha.
    The paper uses alpha = -0.5; at that value some 384^3 nodes lie on Gamma in
    exact arithmetic (x = z = 0, y = -1/48: sin(-pi/6) = -1/2), where the
    rounding of two independent sin/cos implementations would decide the
    label; alpha is moved by 1e-9 (Gamma moves by about 4e-11 h)."""
    return [k, k, k, alpha]


def compact_bump(center, gamma: float = 1.0 / 40.0, sigma: float = 1.0 / 80.0, amp: float = 1.0,
                 period: float = 1.0) -> Callable:
    """The paper's compact isotropic source profile (Sec. 4.4.1):
    f(r) = amp exp(-(r/sigma)^2 / (1 - (r/gamma)^2)) for r < gamma, 0 beyond;
    r measured to the nearest periodic image of the centre."""
    c = [float(v) for v in center]

    def f(*X):
        r2 = 0.0
        for d in range(len(c)):
            t = X[d] - c[d]
            t = t - period * np.round(t / period)
            r2 = r2 + t * t
        q = r2 / (gamma * gamma)
        with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
            val = amp * np.exp(-(r2 / (sigma * sigma)) / (1.0 - q))
        return np.where(q < 1.0, val, 0.0)

    return f


def gyroid_heat(n: int = 384, precision: str = "mixed32") -> Workload:
    """The paper's heat conduction in a triply periodic gyroid (Sec. 4.4.1):
    unit periodic cube, domain phi > 0, homogeneous Neumann (zero flux) on the
    gyroid, Lap u = -q with q two compact bumps of amplitude +-1e5 at
    x+ = (23, 19, 21)/32 and x- = (3, 7, 9)/32 (support 1/40, sigma 1/80).
    In the ABI's convention div(beta grad u) = f, so f = -q."""
    qp = compact_bump((23 / 32, 19 / 32, 21 / 32), amp=1e5)
    qm = compact_bump((3 / 32, 7 / 32, 9 / 32), amp=-1e5)
    zero = Manufactured(lambda *X: 0.0 * X[0], lambda *X: tuple(0.0 * X[0] for _ in range(3)),
                        lambda *X: 0.0 * X[0])
    return Workload("gyroid_heat", 3, n, GEOM_GYROID, gyroid_params(), SIDE_EXTERIOR, BC_NEUMANN,
                    exact=zero, precision=precision, lo=0.0, hi=1.0, periodic=True,
                    source=lambda *X: -(qp(*X) + qm(*X)))


def ms_paper_interface(dim: int = 2) -> Manufactured:
    """The paper's material-interface solution (Sec. 2.4):
    u^+ = 0.6 + 0.4 sin(4 pi x) sin(2 pi y),  u^- = sin(4 pi x) sin(2 pi y)."""
    s = lambda x, y: np.sin(2 * TWO_PI * x) * np.sin(TWO_PI * y)
    gs = lambda x, y: (2 * TWO_PI * np.cos(2 * TWO_PI * x) * np.sin(TWO_PI * y),
                       TWO_PI * np.sin(2 * TWO_PI * x) * np.cos(TWO_PI * y))
    ls = lambda x, y: -((2 * TWO_PI) ** 2 + TWO_PI ** 2) * s(x, y)
    up = lambda x, y: 0.6 + 0.4 * s(x, y)
    gp = lambda x, y: tuple(0.4 * c for c in gs(x, y))
    lp = lambda x, y: 0.4 * ls(x, y)
    return Manufactured(up, gp, lp, s, gs, ls)


def ms_polynomial(coefs: dict, dim: int) -> Manufactured:
    """u = sum_c coef * x^a y^b (z^c) — used by patch tests (exact for degree <= k-1)."""
    def u(*X):
        out = 0.0 * X[0]
        for e, c in coefs.items():
            t = c + 0.0 * X[0]
            for d in range(dim):
                t = t * X[d] ** e[d]
            out = out + t
        return out

    def g(*X):
        comps = []
        for dd in range(dim):
            out = 0.0 * X[0]
            for e, c in coefs.items():
                if e[dd] == 0:
                    continue
                t = c * e[dd] + 0.0 * X[0]
                for d in range(dim):
                    t = t * X[d] ** (e[d] - (1 if d == dd else 0))
                out = out + t
            comps.append(out)
        return tuple(comps)

    def lap(*X):
        out = 0.0 * X[0]
        for e, c in coefs.items():
            for dd in range(dim):
                if e[dd] < 2:
                    continue
                t = c * e[dd] * (e[dd] - 1) + 0.0 * X[0]
                for d in range(dim):
                    t = t * X[d] ** (e[d] - (2 if d == dd else 0))
                out = out + t
        return out

    return Manufactured(u, g, lap)


# ---------------------------------------------------------------------------
# geometry draws
# ---------------------------------------------------------------------------
def draw_sphere_union(count: int = 16, seed: int = 0, lo: float = -0.7, hi: float = 0.7,
                      rmin: float = 0.08, rmax: float = 0.2, min_gap: float = 0.05) -> List[Tuple]:
    """Spheres drawn in order from numpy default_rng(seed); sphere i is redrawn
    until its surface gap to every earlier sphere is at least min_gap."""
    rng = np.random.default_rng(seed)
    out: List[Tuple] = []
    while len(out) < count:
        c = rng.uniform(lo, hi, size=3)
        r = rng.uniform(rmin, rmax)
        ok = all(np.linalg.norm(c - np.array(c2)) - r - r2 >= min_gap for (c2, r2) in out)
        if ok:
            out.append((tuple(float(v) for v in c), float(r)))
    return out


def union_params(spheres: Sequence[Tuple]) -> List[float]:
    p: List[float] = [float(len(spheres))]
    for c, r in spheres:
        p += [float(v) for v in c] + [float(r)]
    return p


# ---------------------------------------------------------------------------
# the five workload configurations and small variants for parity tests
# ---------------------------------------------------------------------------
def cfg1_circle(n: int = 64) -> Workload:
    """2D Dirichlet, interior of the circle r=0.5 at the origin."""
    return Workload("cfg1_circle_dirichlet", 2, n, GEOM_SPHERE, [0.0, 0.0, 0.5],
                    SIDE_INTERIOR, BC_DIRICHLET, exact=ms_sin2pi_cos2pi(), precision="fp64")


def cfg2_star(n: int = 1024, beta_plus: float = 1.0, beta_minus: float = 1.0) -> Workload:
    """2D interface: star r(theta)=0.5+0.1cos(5 theta); Dirichlet box."""
    return Workload("cfg2_star_interface", 2, n, GEOM_STAR2D, [0.0, 0.0, 0.5, 0.1, 5.0],
                    SIDE_INTERFACE, BC_JUMP, beta_plus, beta_minus,
                    exact=ms_star_interface(), precision="fp64")


def cfg3_sphere(n: int = 256, precision: str = "mixed32") -> Workload:
    """3D Dirichlet, interior of the sphere r=0.6 at the origin."""
    return Workload("cfg3_sphere_dirichlet", 3, n, GEOM_SPHERE, [0.0, 0.0, 0.0, 0.6],
                    SIDE_INTERIOR, BC_DIRICHLET, exact=ms_sin_pi_3d(), precision=precision)


def cfg4_spheres(n: int = 384, count: int = 16, seed: int = 0, precision: str = "mixed16",
                 spheres: Optional[List[Tuple]] = None) -> Workload:
    """3D Neumann on a union of spheres, Dirichlet on the box, exterior domain."""
    sp = spheres if spheres is not None else draw_sphere_union(count, seed)
    return Workload("cfg4_spheres_neumann", 3, n, GEOM_SPHERE_UNION, union_params(sp),
                    SIDE_EXTERIOR, BC_NEUMANN, exact=ms_cos_sinh(), precision=precision,
                    note=f"{len(sp)} spheres, seed {seed}")


def singular_star(n: int = 1024, precision: str = "fp64") -> Workload:
    """2D pure-Neumann problem inside the star r = 0.5 + 0.1 cos 5t: singular,
    solved through the bordered system; u = sin(2 pi x + 0.7) cos(2 pi y - 0.4)."""
    return Workload("singular_star_neumann", 2, n, GEOM_STAR2D, [0.0, 0.0, 0.5, 0.1, 5.0],
                    SIDE_INTERIOR, BC_NEUMANN, exact=ms_shifted_trig(), precision=precision)


def singular_sphere(n: int = 256, precision: str = "mixed32") -> Workload:
    """3D pure-Neumann problem inside the sphere r = 0.6 centred at
    (0.05, -0.1, 0.03): singular; u = cos(2x) sinh(y) + z^2."""
    return Workload("singular_sphere_neumann", 3, n, GEOM_SPHERE, [0.05, -0.1, 0.03, 0.6],
                    SIDE_INTERIOR, BC_NEUMANN, exact=ms_cos_sinh(), precision=precision)


def small_spheres_union() -> List[Tuple]:
    """A resolvable-at-small-n stand-in for cfg 4 (3 spheres, radius >= 0.3)."""
    return [((-0.3, -0.3, 0.05), 0.3), ((0.35, 0.25, -0.2), 0.28), ((0.05, 0.38, 0.33), 0.27)]


def small_circles_union_2d() -> List[Tuple]:
    return [((-0.35, -0.3), 0.3), ((0.4, 0.3), 0.33)]


# ---------------------------------------------------------------------------
# serving stream (cfg 5)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    rid: int
    arrival: float
    workload: Workload


def serving_requests(count: int = 2000, rate: float = 10.0, seed: int = 1,
                     n2d: Tuple[int, int] = (128, 2048), n3d: Tuple[int, int] = (32, 192)) -> List[Request]:
    """Poisson arrivals at `rate` per second; each request is a 2D circle or 3D
    sphere interior Dirichlet problem with the cfg-1 / cfg-3 manufactured
    solutions, radius U[0.3,0.7], centre offset uniform in the ball of radius 0.2."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        dim = 2 if rng.uniform() < 0.5 else 3
        r = float(rng.uniform(0.3, 0.7))
        # uniform in the ball of radius 0.2 (rejection sampling)
        while True:
            off = rng.uniform(-0.2, 0.2, size=dim)
            if np.linalg.norm(off) <= 0.2:
                break
        if dim == 2:
            n = int(rng.integers(n2d[0], n2d[1] + 1))
            w = Workload(f"req{i}_circle", 2, n, GEOM_SPHERE, [float(off[0]), float(off[1]), r],
                         SIDE_INTERIOR, BC_DIRICHLET, exact=ms_sin2pi_cos2pi(), precision="mixed32")
        else:
            n = int(rng.integers(n3d[0], n3d[1] + 1))
            w = Workload(f"req{i}_sphere", 3, n, GEOM_SPHERE,
                         [float(off[0]), float(off[1]), float(off[2]), r],
                         SIDE_INTERIOR, BC_DIRICHLET, exact=ms_sin_pi_3d(), precision="mixed32")
        out.append(Request(i, t, w))
    return out
