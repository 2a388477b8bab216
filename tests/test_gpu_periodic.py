"""GPU parity of periodic problems (Sec. 2.3; the periodic gyroid of Sec.
4.4.1): the HIP path against the oracle on identical inputs through the C ABI
-- labels, control points and least-squares sets across the periodic seam,
the operator, every multigrid level operation, the cycle and the (bordered)
solve -- and, at 384^3, the gyroid heat problem checked by what holds at any
size."""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import singular as S
from oracle.mg import Hierarchy
from tests.gpu_helpers import oracle_for, gpu_for, oracle_data

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _seam(n, side, bc, bp=1.0, bm=1.0):
    ms = W.ms_periodic(2)
    if side == W.SIDE_INTERFACE:
        ms = W.Manufactured(ms.u_plus, ms.grad_plus, ms.lap_plus, ms.u_plus, ms.grad_plus, ms.lap_plus)
    return W.Workload("seam", 2, n, W.GEOM_SPHERE, [0.87, 0.46, 0.23], side, bc, bp, bm, exact=ms,
                      lo=0.0, hi=1.0, periodic=True, precision="fp64")


CASES = {
    "seam-neu64": lambda: _seam(64, W.SIDE_EXTERIOR, W.BC_NEUMANN, 1.5),
    "seam-dir64": lambda: _seam(64, W.SIDE_EXTERIOR, W.BC_DIRICHLET),
    "seam-jump64": lambda: _seam(64, W.SIDE_INTERFACE, W.BC_JUMP, 1.0, 2.0),
    "gyroid32": lambda: W.Workload("gyroid32", 3, 32, W.GEOM_GYROID, W.gyroid_params(k=2 * math.pi),
                                   W.SIDE_EXTERIOR, W.BC_NEUMANN, exact=W.ms_periodic(3), lo=0.0, hi=1.0,
                                   periodic=True, precision="fp64"),
}


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    print("case: periodic", request.param, file=sys.stderr, flush=True)
    wl = CASES[request.param]()
    O = oracle_for(wl)
    G = gpu_for(wl, precision="fp64", rtol=1e-13, max_iters=600)
    yield request.param, wl, O, G
    G.close()


def test_labels_points_stencils(pair):
    name, wl, O, G = pair
    assert (G.node_labels() == O.lab_flat).all()
    xyz, nrm = G.control_points()
    oxyz, onrm = O.cp_arrays()
    assert xyz.shape == oxyz.shape and len(xyz) > 0
    assert np.abs(xyz - oxyz).max() <= 1e-14
    assert np.abs(nrm - onrm).max() <= 1e-12
    # some control points sit on segments across the seam
    n, h = wl.n, 1.0 / wl.n
    assert np.any(xyz > (n - 1) * h)
    rng = np.random.default_rng(1)
    seam = np.nonzero(np.any(xyz > (n - 1) * h, axis=1))[0]
    pick = np.concatenate([rng.choice(seam, min(15, seam.size), replace=False),
                           rng.choice(O.ncp, min(25, O.ncp), replace=False)])
    for c in pick:
        for side in O.sides:
            idx, wts = G.ls_stencil(int(c), side)
            st = O.stencil(int(c), side)
            assert list(idx) == list(st.idx), (name, c, side)
            assert np.abs(wts - st.S).max() <= 1e-12 * np.abs(st.S).max(), (name, c)


def test_apply(pair):
    name, wl, O, G = pair
    L, LG = O.assemble()
    rng = np.random.default_rng(2)
    x = np.zeros(O.lab_flat.size)
    x[O.unknowns] = rng.standard_normal(O.unknowns.size)
    y = G.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    yo = np.zeros_like(x)
    yo[O.unknowns] = L @ x[O.unknowns]
    scale = abs(L).max() * np.abs(x).max()
    assert np.abs(y - yo).max() <= 1e-13 * scale
    cpd, box, f = oracle_data(O, wl)
    G.set_boundary_data(cpd, None)
    ug = O.data_vector(cpd, None)
    yd = G.apply(torch.tensor(x, device="cuda"), with_data=True).cpu().numpy()
    yod = np.zeros_like(x)
    yod[O.unknowns] = L @ x[O.unknowns] + LG @ ug
    assert np.abs(yd - yod).max() <= 1e-13 * max(scale, np.abs(LG @ ug).max())


def test_level_operators_and_cycle(pair):
    name, wl, O, G = pair
    H = Hierarchy(O)
    rng = np.random.default_rng(3)
    nl = len(H.levels)
    for l, lev in enumerate(H.levels):
        n, nu = G.level_info(l)
        assert n == lev.grid.n and nu == lev.unknowns.size
        assert (G.level_labels(l) == lev.lab_flat).all()
        v = np.zeros(lev.lab_flat.size)
        v[lev.unknowns] = rng.standard_normal(lev.unknowns.size)
        vt = torch.tensor(v, device="cuda")
        y = G.level_op(l, 0, vt, torch.zeros_like(vt)).cpu().numpy()[lev.unknowns]
        assert np.abs(y - lev.A @ v[lev.unknowns]).max() <= 1e-13 * abs(lev.A).max() * np.abs(v).max(), (l, "A")
        z0 = np.zeros_like(v)
        z0[lev.unknowns] = rng.standard_normal(lev.unknowns.size)
        zt = torch.tensor(z0, device="cuda")
        G.level_op(l, 1, vt, zt)
        zo = z0[lev.unknowns].copy()
        H.rbgs(l, zo, v[lev.unknowns])
        assert np.abs(zt.cpu().numpy()[lev.unknowns] - zo).max() <= 1e-12 * (np.abs(zo).max() + 1), (l, "rbgs")
        if l + 1 < nl:
            cl = H.levels[l + 1]
            rc = G.level_op(l, 2, vt, torch.zeros(cl.lab_flat.size, dtype=torch.float64, device="cuda"))
            rc = rc.cpu().numpy()[cl.unknowns]
            assert np.abs(rc - H.restrict(l, v[lev.unknowns])).max() <= 4e-14 * np.abs(v).max(), (l, "R")
        if l > 0:
            fl = H.levels[l - 1]
            pf = G.level_op(l, 3, vt, torch.zeros(fl.lab_flat.size, dtype=torch.float64, device="cuda"))
            pf = pf.cpu().numpy()[fl.unknowns]
            assert np.abs(pf - H.prolong(l, v[lev.unknowns])).max() <= 4e-14 * np.abs(v).max(), (l, "P")
    v = np.zeros(O.lab_flat.size)
    v[O.unknowns] = rng.standard_normal(O.unknowns.size)
    z = G.vcycle(torch.tensor(v, device="cuda")).cpu().numpy()[O.unknowns]
    zo = H.precondition(v[O.unknowns])
    assert np.abs(z - zo).max() <= 1e-11 * np.abs(zo).max(), np.abs(z - zo).max() / np.abs(zo).max()


def test_solve_matches_direct(pair):
    name, wl, O, G = pair
    L, LG = O.assemble()
    cpd, box, f = oracle_data(O, wl)
    G.set_boundary_data(cpd, None)
    G.set_rhs(f)
    u, _, st = G.solve()
    assert st["status"] == 0, st
    ug = O.data_vector(cpd, None)
    b = O.rhs(wl.rhs(O.labels), ug)
    uu = u.cpu().numpy()[O.unknowns]
    if S.is_singular(O):
        assert st["bordered"] == 1
        ud, ad = S.direct_solve(O, b)
        assert abs(st["shift_alpha"] - ad) <= 1e-10 * np.abs(b).max()
    else:
        assert st["bordered"] == 0
        ud = O.direct_solve(b)
    err = np.abs(uu - ud).max() / np.abs(ud).max()
    assert err <= 1e-10, err
    assert np.isnan(u.cpu().numpy()[O.lab_flat == 0]).all()


def _labels_and_geometry_checks(G, wl):
    """Labels repeat under the half-period shift s = (240, 144, 144) nodes
    (a translation of the gyroid by (5/8, 3/8, 3/8) leaves phi unchanged);
    sampled labels follow the sign of phi; sampled control points lie on Gamma
    with the unit normal of grad phi."""
    n = wl.n
    lab = G.node_labels().reshape((n + 1,) * 3, order="F")
    core = lab[:n, :n, :n]
    s = (240, 144, 144)
    assert np.array_equal(np.roll(core, (-s[0], -s[1], -s[2]), axis=(0, 1, 2)), core)
    from oracle.geometry import Gyroid
    Gy = Gyroid(*wl.geom_params)
    rng = np.random.default_rng(4)
    ijk = rng.integers(0, n, size=(20000, 3))
    ph = Gy.phi([ijk[:, d] / n for d in range(3)])
    assert np.array_equal(core[ijk[:, 0], ijk[:, 1], ijk[:, 2]], np.where(ph > 0, 1, 0))
    xyz, nrm = G.control_points()
    for c in rng.choice(len(xyz), 200, replace=False):
        x = xyz[c]
        assert abs(Gy.phi(x)) <= 1e-12
        gv = Gy.gradient(x)
        assert np.abs(nrm[c] - gv / np.linalg.norm(gv)).max() <= 1e-12
    return lab, xyz, nrm


def test_gyroid_384_manufactured():
    """The paper's gyroid (k = 8 pi) in the periodic unit cube at 384^3, with a
    periodic manufactured solution (Neumann data dn u on the gyroid, f = Lap u):
    the bordered mixed-precision solve converges, its unknowns sum to zero, and
    its mean-free error against the closed form is at the discretisation
    level -- a full-size check against a closed form (no oracle run at this size)."""
    print("case: gyroid manufactured 384^3", file=sys.stderr, flush=True)
    from paper_2503_22455_amd import iim
    base = W.gyroid_heat(384)
    wl = W.Workload("gyroid_ms", 3, 384, W.GEOM_GYROID, base.geom_params, W.SIDE_EXTERIOR, W.BC_NEUMANN,
                    exact=W.ms_periodic(3), lo=0.0, hi=1.0, periodic=True, precision="mixed32")
    G = gpu_for(wl, precision="mixed32", rtol=1e-10)
    lab, xyz, nrm = _labels_and_geometry_checks(G, wl)
    G.set_boundary_data(wl.cp_data(xyz, nrm), None)
    G.set_rhs(iim.grid_to_flat(wl.rhs(lab)))
    u, hist, st = G.solve()
    assert st["status"] == 0 and st["bordered"] == 1 and st["final_rel_residual"] <= 1e-10, st
    n = wl.n
    uc = u.cpu().numpy().reshape((n + 1,) * 3, order="F")
    act = lab == 1
    uu = uc[act]
    assert abs(uu.sum()) <= 1e-9 * np.abs(uu).sum()
    ue = np.asarray(wl.exact_solution(lab))[act]
    err = np.abs((uu - uu.mean()) - (ue - ue.mean())).max()
    print(f"gyroid 384^3: {G.info()['n_unknowns']} unknowns, {len(xyz)} control points, {st['iterations']} its, "
          f"mean-free max error {err:.2e}, alpha {st['shift_alpha']:.2e}", file=sys.stderr, flush=True)
    assert err <= 1e-5, err
    G.close()


def test_gyroid_heat_384():
    """The paper's heat problem itself (two compact sources of +-1e5, zero flux
    on the gyroid, 384^3): the bordered solve reaches 1e-10 and its unknowns sum
    to zero."""
    print("case: gyroid heat 384^3", file=sys.stderr, flush=True)
    from paper_2503_22455_amd import iim
    wl = W.gyroid_heat(384)
    G = gpu_for(wl, precision="mixed32", rtol=1e-10)
    n = wl.n
    lab = G.node_labels().reshape((n + 1,) * 3, order="F")
    ncp = G.info()["n_control_points"]
    G.set_boundary_data(np.zeros(ncp), None)
    G.set_rhs(iim.grid_to_flat(wl.rhs(lab)))
    u, hist, st = G.solve()
    print(f"gyroid heat 384^3: {st['iterations']} its, res {st['final_rel_residual']:.2e}, "
          f"alpha {st['shift_alpha']:.3e}", file=sys.stderr, flush=True)
    assert st["status"] == 0 and st["bordered"] == 1 and st["final_rel_residual"] <= 1e-10, st
    uu = u.cpu().numpy()[lab.ravel(order="F") == 1]
    assert abs(uu.sum()) <= 1e-9 * np.abs(uu).sum()
    G.close()


@pytest.mark.parametrize("n", [32, 128], ids=["gyroid32", "gyroid128"])
def test_periodic_colour_split_is_bitwise_identical(n):
    """On a periodic cell the colour-split level layout (its half-sweeps, fused
    last half-sweep, restriction and cell-wise prolongation wrapping across the
    seam) changes where values live, not the arithmetic: the V-cycle and the
    bordered solve equal those on the storage-box layout bit for bit.  At n = 128
    the level-0 half-sweeps take the four-entry kernel (rows of n / 2 entries),
    at n = 32 the one-entry kernel."""
    print(f"case: periodic colour split gyroid n = {n}", file=sys.stderr, flush=True)
    from paper_2503_22455_amd import iim
    wl = W.Workload("gyroid_ms", 3, n, W.GEOM_GYROID, W.gyroid_params(k=2 * math.pi), W.SIDE_EXTERIOR,
                    W.BC_NEUMANN, exact=W.ms_periodic(3), lo=0.0, hi=1.0, periodic=True, precision="mixed32")
    A = gpu_for(wl, precision="mixed32", rtol=1e-10, colour_split=False)
    B = gpu_for(wl, precision="mixed32", rtol=1e-10, colour_split=True)
    lab = A.node_labels()
    unk = lab == 1
    rng = np.random.default_rng(23)
    v = np.zeros(lab.size)
    v[unk] = rng.standard_normal(int(unk.sum()))
    vt = torch.tensor(v, device="cuda")
    assert np.array_equal(A.vcycle(vt).cpu().numpy(), B.vcycle(vt).cpu().numpy())
    xyz, nrm = A.control_points()
    outs = []
    for G in (A, B):
        G.set_boundary_data(wl.cp_data(xyz, nrm), None)
        G.set_rhs(iim.grid_to_flat(wl.rhs(iim.flat_to_grid(lab, 3, n))))
        u, hist, st = G.solve()
        assert st["status"] == 0 and st["bordered"] == 1, st
        outs.append((u.cpu().numpy(), hist, st["iterations"]))
    assert np.array_equal(outs[0][0], outs[1][0], equal_nan=True)
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]
    A.close()
    B.close()
