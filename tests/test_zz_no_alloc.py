"""The entry point that allocates no device memory
(iim_set_boundary_data_noalloc) against the allocating one
(iim_set_boundary_data), through the C ABI: two calls in a row, the second on a
smaller problem, each checked bit for bit through the operator with data and
the right-hand side it builds."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import gpu_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _data(wl, P):
    from paper_2503_22455_amd import iim
    lab = P.node_labels()
    xyz, nrm = P.control_points()
    cpd = torch.tensor(np.ascontiguousarray(wl.cp_data(xyz, nrm), dtype=np.float64).ravel(), device="cuda")
    box = torch.tensor(iim.grid_to_flat(wl.box_data()), device="cuda")
    f = torch.tensor(iim.grid_to_flat(wl.rhs(iim.flat_to_grid(lab, wl.dim, wl.n))), device="cuda")
    return cpd, box, f


def _run(wl, noalloc):
    P = gpu_for(wl, precision="fp64", rtol=1e-12)
    cpd, box, f = _data(wl, P)
    before = P.info()["device_bytes"]
    if noalloc:
        P.set_boundary_data_noalloc(cpd, box)
        assert P.info()["device_bytes"] == before
    else:
        P.set_boundary_data(cpd, box)
    x = torch.tensor(np.random.default_rng(3).standard_normal(P.total), device="cuda")
    y = P.apply(x, with_data=True)
    P.set_rhs(f)
    u, _, st = P.solve()
    P.close()
    return y, u, st


@pytest.mark.parametrize("second", ["smaller-2d", "smaller-3d"])
def test_noalloc_equals_allocating_entry_point(second):
    """An exterior Neumann problem with box faces (box data are staged), then
    a smaller one: operator with data and solution bitwise those of the
    allocating entry point."""
    first = W.Workload("neu2", 2, 256, W.GEOM_SPHERE_UNION, W.union_params(W.small_circles_union_2d()),
                       W.SIDE_EXTERIOR, W.BC_NEUMANN, exact=W.ms_sin2pi_cos2pi())
    small = (dataclasses.replace(first, n=64) if second == "smaller-2d"
             else W.cfg4_spheres(32, spheres=W.small_spheres_union(), precision="fp64"))
    for wl in (first, small):
        ya, ua, sta = _run(wl, False)
        yb, ub, stb = _run(wl, True)
        assert torch.equal(ya, yb)
        assert sta["iterations"] == stb["iterations"]
        assert torch.equal(ua.nan_to_num(0.0), ub.nan_to_num(0.0))


def test_noalloc_rejects_box_data_beyond_its_array():
    """(n+1)^dim above IIM_NOALLOC_MAX_NODES fails with IIM_E_INVALID_ARG and
    leaves the handle usable."""
    from paper_2503_22455_amd import iim
    wl = dataclasses.replace(W.cfg1_circle(2048), precision="fp64")
    assert (wl.n + 1) ** 2 > 1 << 22
    P = gpu_for(wl, precision="fp64")
    cpd, box, f = _data(wl, P)
    with pytest.raises(iim.IIMError) as e:
        P.set_boundary_data_noalloc(cpd, box)
    assert e.value.code == -1
    P.set_boundary_data_noalloc(cpd, None)  # no box data: nothing to stage
    P.close()
