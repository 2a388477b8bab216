"""Parity at the benchmark sizes, on outputs the oracle computes one row at a
time: the 1024^2 interface operator and the 256^3 sphere operator, with the
(4,5) and the (6,7) scheme, in the launch configuration the benchmark times."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import oracle_for, gpu_for, oracle_data

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _sampled_apply(wl, nsample, seed, order=(4, 5), tol=1e-13):
    O = oracle_for(wl, order_n=order[0], order_k=order[1])
    G = gpu_for(wl, precision="fp64", order=order)
    info = G.info()
    assert info["n_unknowns"] == O.unknowns.size
    assert (G.node_labels() == O.lab_flat).all()
    xyz, nrm = G.control_points()
    oxyz, onrm = O.cp_arrays()
    assert np.abs(xyz - oxyz).max() <= 1e-14
    rng = np.random.default_rng(seed)
    x = np.zeros(O.lab_flat.size)
    x[O.unknowns] = rng.standard_normal(O.unknowns.size)
    cpd, box, f = oracle_data(O, wl)
    G.set_boundary_data(cpd, box)
    ug = O.data_vector(cpd, wl.box_data())
    y = G.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    yd = G.apply(torch.tensor(x, device="cuda"), with_data=True).cpu().numpy()
    # sample: irregular nodes (next to Gamma or the box) and random interior nodes
    irr = np.nonzero(~O.regular_mask() & (O.uindex >= 0))[0]
    nodes = np.concatenate([rng.choice(irr, size=min(nsample, irr.size), replace=False),
                            rng.choice(O.unknowns, size=nsample, replace=False)])
    yo = O.apply_rows(nodes, x)
    yod = O.apply_rows(nodes, x, with_data=True, u_gamma=ug)
    scale = 25.0 / O.grid.h ** 2 * max(O.beta.values())
    assert np.abs(y[nodes] - yo).max() <= tol * scale
    assert np.abs(yd[nodes] - yod).max() <= tol * (scale + np.abs(yod).max())
    G.close()


def test_cfg2_star_1024_sampled():
    _sampled_apply(W.cfg2_star(1024), 300, 11)


def test_cfg3_sphere_256_sampled():
    _sampled_apply(W.cfg3_sphere(256, precision="fp64"), 200, 12)


# the (6,7) scheme at the same sizes: its degree-6 fits agree with the oracle's
# to about 5e-12 of their largest weight (the (4,5) ones to 7e-14), hence the
# looser bound
def test_cfg2_star_1024_order6_sampled():
    _sampled_apply(W.cfg2_star(1024), 300, 13, order=(6, 7), tol=1e-11)


def test_cfg3_sphere_256_order6_sampled():
    _sampled_apply(W.cfg3_sphere(256, precision="fp64"), 150, 14, order=(6, 7), tol=1e-11)


def test_singular_sphere_256_bordered_sampled():
    """The singular pure-Neumann sphere at 256^3, solved as benchmarked (FP32
    cycle, bordered FP64 system), checked by what holds at any size: the
    unknowns sum to zero, and the bordered residual rows f - L u - L_Gamma
    u_Gamma - alpha, with L's rows computed by the oracle one at a time, are
    within the solve's tolerance of ||b||."""
    import sys
    print("case: singular sphere 256^3 bordered", file=sys.stderr, flush=True)
    wl = W.singular_sphere(256)
    O = oracle_for(wl)
    G = gpu_for(wl, rtol=1e-10)
    assert (G.node_labels() == O.lab_flat).all()
    xyz, _ = G.control_points()
    assert np.abs(xyz - O.cp_arrays()[0]).max() <= 1e-14
    cpd, _, f = oracle_data(O, wl)
    G.set_boundary_data(cpd, None)
    G.set_rhs(f)
    u, _, st = G.solve()
    assert st["status"] == 0 and st["bordered"] == 1 and st["final_rel_residual"] <= 1e-10, st
    alpha = st["shift_alpha"]
    uf = np.nan_to_num(u.cpu().numpy())
    uu = uf[O.unknowns]
    assert abs(uu.sum()) <= 1e-9 * np.abs(uu).sum()
    # ||b|| with b = f - L_Gamma u_Gamma over the unknowns
    lg = G.apply(torch.zeros(O.lab_flat.size, dtype=torch.float64, device="cuda"), with_data=True).cpu().numpy()
    bnorm = np.linalg.norm((f - lg)[O.unknowns])
    ug = O.data_vector(cpd)
    rng = np.random.default_rng(15)
    irr = np.nonzero(~O.regular_mask() & (O.uindex >= 0))[0]
    nodes = np.concatenate([rng.choice(irr, size=150, replace=False), rng.choice(O.unknowns, size=150, replace=False)])
    r = f[nodes] - O.apply_rows(nodes, uf, with_data=True, u_gamma=ug) - alpha
    scale = 25.0 / O.grid.h ** 2
    assert np.abs(r).max() <= 1e-10 * bnorm + 1e-12 * scale * np.abs(uu).max(), (np.abs(r).max(), bnorm)
    G.close()
