"""GPU parity of singular pure-Neumann problems (Sec. 2.3): an interior domain
with a Neumann boundary, solved through the bordered system
[L 1; 1^T 0] [u; alpha] = [b; 0].  The HIP path against the oracle's bordered
direct solve and bordered multigrid cycle, plus a planted shift that the device
must recover on its own."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.mg import Hierarchy
from oracle import singular as S
from tests.gpu_helpers import oracle_for, gpu_for, oracle_data

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wl(name, dim, n, geom, params, ex, order=(4, 5)):
    return W.Workload(name, dim, n, geom, params, W.SIDE_INTERIOR, W.BC_NEUMANN, exact=ex,
                      precision="fp64", order=order)


CASES = {
    "circle-neu64": lambda: _wl("circle-neu64", 2, 64, W.GEOM_SPHERE, [0.0, 0.0, 0.5], W.ms_shifted_trig()),
    "star-neu128": lambda: _wl("star-neu128", 2, 128, W.GEOM_STAR2D, [0.0, 0.0, 0.5, 0.1, 5.0],
                               W.ms_shifted_trig()),
    "circle-neu64-o6": lambda: _wl("circle-neu64-o6", 2, 64, W.GEOM_SPHERE, [0.0, 0.0, 0.5],
                                   W.ms_shifted_trig(), order=(6, 7)),
    "sphere-neu24": lambda: _wl("sphere-neu24", 3, 24, W.GEOM_SPHERE, [0.05, -0.1, 0.03, 0.6], W.ms_cos_sinh()),
}


def _announce(*what):
    print("case:", *what, file=sys.stderr, flush=True)


@pytest.mark.parametrize("name", list(CASES))
def test_bordered_solve_matches_oracle(name):
    """The bordered V-cycle against the oracle's (the coarsest SW matrix is
    singular and bordered on both sides), then the FP64 solve against the
    bordered direct solve: u, alpha, sum u = 0 and the bordered residual."""
    _announce("bordered solve", name)
    wl = CASES[name]()
    O = oracle_for(wl, order_n=wl.order[0], order_k=wl.order[1])
    assert S.is_singular(O)
    # the bordered FP64 residual floors at about 1.7e-14 (measured on the star)
    G = gpu_for(wl, precision="fp64", rtol=3e-14, max_iters=600)
    H = Hierarchy(O)
    rng = np.random.default_rng(8)
    v = np.zeros(O.lab_flat.size)
    v[O.unknowns] = rng.standard_normal(O.unknowns.size)
    z = G.vcycle(torch.tensor(v, device="cuda")).cpu().numpy()[O.unknowns]
    zo = H.precondition(v[O.unknowns])
    assert np.abs(z - zo).max() <= 1e-11 * np.abs(zo).max(), np.abs(z - zo).max() / np.abs(zo).max()
    L, LG = O.assemble()
    cpd, box, f = oracle_data(O, wl)
    G.set_boundary_data(cpd, None)
    G.set_rhs(f)
    u, hist, st = G.solve()
    assert st["status"] == 0 and st["bordered"] == 1, st
    ug = O.data_vector(cpd)
    b = O.rhs(wl.rhs(O.labels), ug)
    uu = u.cpu().numpy()[O.unknowns]
    alpha = st["shift_alpha"]
    r = np.concatenate([b - L @ uu - alpha, [-uu.sum()]])
    # the residual is taken with the oracle's operator: its Householder fits on
    # the Neumann sphere lie up to 4.7e-13 (of the largest weight) from the
    # least-squares weights computed in extended precision, the device's 3D fits
    # (Cholesky of A^T A plus one correction) within 6e-14; an operator built
    # from the latter leaves 1.1e-12 here while u agrees to 3e-13 (both measured
    # on the CPU), so the bound is 3e-12 and u keeps 1e-12 below
    assert np.linalg.norm(r) <= 3e-12 * np.linalg.norm(b), np.linalg.norm(r) / np.linalg.norm(b)
    ud, ad = S.direct_solve(O, b)
    # all-FP64, solved to its residual floor: u within 1e-12 of the bordered
    # direct solve, as for the non-singular cases
    eu = np.abs(uu - ud).max() / np.abs(ud).max()
    ea = abs(alpha - ad) / np.abs(b).max()
    _announce(f"{name}: {st['iterations']} its, u rel err {eu:.2e}, alpha err / max|b| {ea:.2e}")
    assert eu <= 1e-12, eu
    assert ea <= 1e-12, (alpha, ad)
    assert abs(ad) > 1e-6  # the shift is really exercised
    # the mean-free error is the oracle's
    ue = O.from_full(wl.exact_solution(O.labels))
    eg = np.abs(S.mean_free(uu) - S.mean_free(ue)).max()
    eo = np.abs(S.mean_free(ud) - S.mean_free(ue)).max()
    assert abs(eg - eo) <= 1e-6 * eo + 1e-12, (eg, eo)
    G.close()


@pytest.mark.parametrize("use_graph", [0, 1, 2])
def test_planted_shift(use_graph):
    """b = L v + c 1 with zero boundary data: the device must return
    u = v - mean(v) and alpha = c, whatever the launch mode."""
    _announce("planted shift", use_graph)
    wl = CASES["circle-neu64"]()
    O = oracle_for(wl)
    L, _ = O.assemble()
    G = gpu_for(wl, precision="fp64", rtol=1e-13, use_graph=use_graph)
    rng = np.random.default_rng(21)
    v = rng.standard_normal(O.unknowns.size)
    c = 0.37
    f = np.zeros(O.lab_flat.size)
    f[O.unknowns] = L @ v + c
    G.set_boundary_data(np.zeros(O.ncp), None)
    G.set_rhs(f)
    u, _, st = G.solve()
    assert st["status"] == 0 and st["bordered"] == 1, st
    uu = u.cpu().numpy()[O.unknowns]
    assert abs(st["shift_alpha"] - c) <= 1e-10, st["shift_alpha"]
    assert np.abs(uu - S.mean_free(v)).max() <= 1e-10 * np.abs(v).max()
    # a second solve from the first one's solution: alpha restarts at zero
    u2, _, st2 = G.solve(x0=u)
    assert st2["status"] == 0 and abs(st2["shift_alpha"] - c) <= 1e-10
    assert np.abs(u2.cpu().numpy()[O.unknowns] - uu).max() <= 1e-10 * np.abs(v).max()
    G.close()


@pytest.mark.parametrize("precision,name", [("mixed32", "star-neu128"), ("mixed16", "star-neu128"),
                                            ("mixed32", "sphere-neu24")])
def test_bordered_mixed_precision(precision, name):
    """Reduced-precision cycles precondition the FP64 bordered system: the
    solve still reaches 1e-10 and the oracle's bordered solution."""
    _announce("bordered mixed", precision, name)
    wl = CASES[name]()
    O = oracle_for(wl)
    O.assemble()
    G = gpu_for(wl, precision=precision, rtol=1e-10)
    cpd, box, f = oracle_data(O, wl)
    G.set_boundary_data(cpd, None)
    G.set_rhs(f)
    u, _, st = G.solve()
    assert st["status"] == 0 and st["bordered"] == 1 and st["final_rel_residual"] <= 1e-10, st
    b = O.rhs(wl.rhs(O.labels), O.data_vector(cpd))
    ud, ad = S.direct_solve(O, b)
    uu = u.cpu().numpy()[O.unknowns]
    assert np.abs(uu - ud).max() <= 1e-7 * np.abs(ud).max()
    assert abs(st["shift_alpha"] - ad) <= 1e-8 * np.abs(b).max()
    G.close()


def test_nonsingular_problems_are_not_bordered():
    _announce("not bordered")
    wl = W.cfg1_circle(64)
    O = oracle_for(wl)
    G = gpu_for(wl, precision="fp64")
    cpd, box, f = oracle_data(O, wl)
    G.set_boundary_data(cpd, box)
    G.set_rhs(f)
    _, _, st = G.solve()
    assert st["status"] == 0 and st["bordered"] == 0 and st["shift_alpha"] == 0.0, st
    G.close()


def test_fp16_storage_iterations_follow_emulation():
    """FP16 iterate storage costs the bordered solve iterations on the 2D
    singular star as the grid refines, as it does for non-singular problems:
    the oracle's cycle with its iterates rounded to half precision gives
    39 -> 39, 40 -> 48 and 41 -> 143 iterations at 256^2, 512^2 and 1024^2.
    At 512^2 the device (FP32 arithmetic, FP16 storage) stays near the
    emulation's count, and the FP64 counts agree."""
    from tests.test_gpu_mixed import _FP16Stored
    _announce("fp16 singular emulation")
    wl = W.singular_star(512)
    O = oracle_for(wl)
    L, _ = O.assemble()
    cpd, _, f = oracle_data(O, wl)
    b = O.rhs(wl.rhs(O.labels), O.data_vector(cpd))
    _, _, its64, ok64 = S.fgmres_solve(O, Hierarchy(O), b, rtol=1e-10, max_iters=400)
    _, _, its16, ok16 = S.fgmres_solve(O, _FP16Stored(O), b, rtol=1e-10, max_iters=400)
    assert ok64 and ok16 and its16 > its64
    counts = {}
    for prec in ("fp64", "mixed16"):
        G = gpu_for(wl, precision=prec, rtol=1e-10)
        G.set_boundary_data(cpd, None)
        G.set_rhs(f)
        _, _, st = G.solve()
        G.close()
        assert st["status"] == 0 and st["bordered"] == 1, st
        counts[prec] = st["iterations"]
    print("singular star 512^2 iterations: oracle", its64, its16, "device", counts, file=sys.stderr, flush=True)
    assert abs(counts["fp64"] - its64) <= 1, (counts, its64)
    assert abs(counts["mixed16"] - its16) <= max(4, its16 // 4), (counts, its16)


@pytest.mark.parametrize("name", ["circle-neu64", "sphere-neu24"])
def test_bordered_wcycle(name):
    """The W-cycle (cycle index 2) on a singular problem: every coarse visit
    ends in the bordered coarse solve.  Its cycle against the oracle's, and the
    bordered solve it preconditions against the bordered direct solve."""
    _announce("bordered W-cycle", name)
    wl = CASES[name]()
    O = oracle_for(wl)
    G = gpu_for(wl, precision="fp64", rtol=1e-12, cycle="W")
    H = Hierarchy(O, gamma=2)
    rng = np.random.default_rng(9)
    v = np.zeros(O.lab_flat.size)
    v[O.unknowns] = rng.standard_normal(O.unknowns.size)
    z = G.vcycle(torch.tensor(v, device="cuda")).cpu().numpy()[O.unknowns]
    zo = H.precondition(v[O.unknowns])
    assert np.abs(z - zo).max() <= 1e-11 * np.abs(zo).max(), np.abs(z - zo).max() / np.abs(zo).max()
    O.assemble()
    cpd, _, f = oracle_data(O, wl)
    G.set_boundary_data(cpd, None)
    G.set_rhs(f)
    u, _, st = G.solve()
    assert st["status"] == 0 and st["bordered"] == 1, st
    b = O.rhs(wl.rhs(O.labels), O.data_vector(cpd))
    ud, ad = S.direct_solve(O, b)
    uu = u.cpu().numpy()[O.unknowns]
    assert np.abs(uu - ud).max() <= 1e-10 * np.abs(ud).max()
    assert abs(st["shift_alpha"] - ad) <= 1e-10 * np.abs(b).max()
    G.close()


@pytest.mark.parametrize("name", ["circle-neu64", "sphere-neu24"])
def test_synthetic_error_is_mean_free(name):
    """Device-made manufactured data on a singular problem: the library's error
    is max |u - u_exact - mean(u - u_exact)| over the unknowns, the host's
    mean-free error of the same u, and small (the solution is accurate up to
    its constant)."""
    _announce("synthetic mean-free error", name)
    wl = CASES[name]()
    O = oracle_for(wl)
    G = gpu_for(wl, precision="fp64", rtol=1e-12)
    G.set_synthetic_data(1)
    u, _, st = G.solve()
    assert st["status"] == 0 and st["bordered"] == 1, st
    err = G.synthetic_error(u)
    ex = W.ms_sin2pi_cos2pi() if wl.dim == 2 else W.ms_sin_pi_3d()
    X = [c.ravel(order="F")[O.unknowns] for c in wl.node_coords()]
    d = u.cpu().numpy()[O.unknowns] - ex.u_plus(*X)
    host = np.abs(d - d.mean()).max()
    assert abs(err - host) <= 1e-12 * max(host, 1e-300) + 1e-15, (err, host)
    assert host < 2e-2 and np.abs(d).max() > 0.0
    G.close()
