"""GPU checks of device-side manufactured data and of the solve server
(continuous batching), all through the C ABI."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import oracle_for, gpu_for, oracle_data, flat

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _same_both_sides(ms):
    return dataclasses.replace(ms, u_minus=ms.u_plus, grad_minus=ms.grad_plus, lap_minus=ms.lap_plus)


def _cases():
    return {
        "circle64-dir": W.cfg1_circle(64),
        "circle75-dir": W.cfg1_circle(75),
        "sphere24-dir": dataclasses.replace(W.cfg3_sphere(24), precision="fp64"),
        # smallest request of the serving mix: kappa h = 0.21, close to the 1/4 limit
        "sphere32-r03": W.Workload("sphere32_r03", 3, 32, W.GEOM_SPHERE, [0.05, -0.1, 0.08, 0.3], W.SIDE_INTERIOR,
                                   W.BC_DIRICHLET, exact=W.ms_sin_pi_3d(), precision="fp64"),
        "spheres32-neu": dataclasses.replace(W.cfg4_spheres(32, spheres=W.small_spheres_union()),
                                             exact=W.ms_sin_pi_3d(), precision="fp64"),
        "star128-jump": dataclasses.replace(W.cfg2_star(128, beta_plus=1.0, beta_minus=10.0),
                                            exact=_same_both_sides(W.ms_sin2pi_cos2pi())),
    }


@pytest.mark.parametrize("name", list(_cases()))
def test_synthetic_data_matches_oracle(name):
    """Data made on the device (kind 1) give the solution of the oracle's
    direct solve with the same manufactured u sampled on the host, and the
    reported max error equals the one measured from the returned u."""
    wl = _cases()[name]
    O = oracle_for(wl)
    cpd, box, f = oracle_data(O, wl)
    ug = O.data_vector(cpd, wl.box_data())
    ud = O.direct_solve(O.rhs(wl.rhs(O.labels), ug))
    G = gpu_for(wl, rtol=1e-13, max_iters=400)
    G.set_synthetic_data(1)
    u, _, st = G.solve()
    assert st["status"] == 0, st
    uu = u.cpu().numpy()[O.unknowns]
    assert np.abs(uu - ud).max() <= 1e-10 * np.abs(ud).max()
    exact = flat(wl.exact_solution(O.labels))[O.unknowns]
    err_host = np.abs(uu - exact).max()
    err_dev = G.synthetic_error(u, 1)
    assert abs(err_dev - err_host) <= 1e-8 * err_host + 1e-14
    G.close()


def _submit(srv, spec, u_out=None, **kw):
    dim, n, params = spec
    return srv.submit(dim, n, W.GEOM_SPHERE, params, W.SIDE_INTERIOR, W.BC_DIRICHLET, data_kind=1, u_out=u_out,
                      precision=kw.pop("precision", "mixed32"), rtol=1e-10, **kw)


MIX = [(2, 150, [0.1, -0.05, 0.5]), (3, 40, [0.05, 0.0, 0.1, 0.55]), (2, 333, [-0.12, 0.08, 0.62]),
       (3, 57, [0.0, -0.1, 0.05, 0.45]), (2, 128, [0.0, 0.0, 0.3]), (3, 33, [0.1, 0.1, -0.1, 0.6]),
       (2, 517, [0.15, 0.0, 0.41]), (3, 64, [-0.05, 0.02, 0.0, 0.66])]


def _numel(spec):
    return (spec[1] + 1) ** spec[0]


def test_server_result_same_alone_and_in_mix():
    """A request solved alone (one slot) and inside a mix of requests of other
    sizes and dimensions on four slots gives the bitwise-identical u, the same
    iteration count, and the same u as a plain handle; the mix overlaps."""
    from paper_2503_22455_amd import iim
    target = MIX[2]
    uA = torch.empty(_numel(target), dtype=torch.float64, device="cuda")
    s1 = iim.Server(64 << 30, 1)
    rA = s1.wait(_submit(s1, target, uA))
    s1.close()
    assert rA["status"] == 0 and rA["rel_residual"] <= 1e-10, rA

    uB = torch.empty_like(uA)
    s4 = iim.Server(64 << 30, 4)
    tickets = []
    for spec in MIX:
        tickets.append(_submit(s4, spec, uB if spec is target else None))
    res = [s4.wait(t) for t in tickets]
    st = s4.stats()
    s4.close()
    for (dim, n, _), r in zip(MIX, res):
        assert r["status"] == 0 and r["rel_residual"] <= 1e-10, r
        # fourth-order discretisation error: measured 48-80 h^4 (3D), 109-375 h^4 (2D)
        assert r["max_error"] <= 600.0 * (2.0 / n) ** 4, r
    rB = res[2]
    assert rB["iterations"] == rA["iterations"]
    assert torch.equal(torch.isnan(uA), torch.isnan(uB))
    assert torch.equal(uA.nan_to_num(0.0), uB.nan_to_num(0.0))
    assert st["completed"] == len(MIX) and st["failed"] == 0
    # some requests ran at the same time
    iv = sorted((r["t_start"], r["t_finish"]) for r in res)
    assert any(iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))

    # the same request through a plain handle
    dim, n, params = target
    P = iim.Problem(dim, n, W.GEOM_SPHERE, params, W.SIDE_INTERIOR, W.BC_DIRICHLET, precision="mixed32", rtol=1e-10)
    P.set_synthetic_data(1)
    uC, _, stc = P.solve()
    assert stc["iterations"] == rA["iterations"]
    assert torch.equal(uA.nan_to_num(0.0), uC.nan_to_num(0.0))
    assert abs(P.synthetic_error(uC, 1) - rA["max_error"]) == 0.0
    P.close()


def test_server_budget_admission():
    """Running requests never reserve more than the budget, each request's
    device bytes stay within its estimate, a request larger than the budget
    fails at once with IIM_E_BUDGET, and a failing request leaves the others
    unaffected."""
    from paper_2503_22455_amd import iim
    probe = iim.Server(64 << 30, 1)
    est = {}
    for spec in MIX:
        r = probe.wait(_submit(probe, spec))
        assert r["status"] == 0, r
        assert 0 < r["device_bytes"] <= r["estimated_bytes"], r
        est[id(spec)] = r["estimated_bytes"]
    probe.close()
    budget = int(1.3 * max(est.values()))
    srv = iim.Server(budget, 4)
    tickets = [_submit(srv, spec) for spec in MIX]
    bad = srv.submit(2, 64, W.GEOM_SPHERE, [0.0, 0.0, 1.2], W.SIDE_INTERIOR, W.BC_DIRICHLET, data_kind=1,
                     precision="mixed32")
    res = [srv.wait(t) for t in tickets]
    rbad = srv.wait(bad)
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in res), res
    assert rbad["status"] == -2, rbad
    assert st["peak_bytes_reserved"] <= budget
    assert st["completed"] == len(MIX) and st["failed"] == 1

    tiny = iim.Server(1 << 20, 2)
    t = _submit(tiny, MIX[0])
    r = tiny.poll(t)
    assert r["done"] == 1 and r["status"] == -3, r
    st = tiny.stats()
    tiny.close()
    assert st["failed"] == 1 and st["completed"] == 0


def test_server_rejects_bad_requests():
    from paper_2503_22455_amd import iim
    srv = iim.Server(1 << 30, 1)
    with pytest.raises(iim.IIMError) as e:
        srv.submit(4, 64, W.GEOM_SPHERE, [0.0, 0.0, 0.5], data_kind=1)
    assert e.value.code == -1
    with pytest.raises(iim.IIMError) as e:
        srv.submit(2, 64, W.GEOM_SPHERE, [0.0, 0.5], data_kind=1)
    assert e.value.code == -1
    with pytest.raises(iim.IIMError) as e:
        srv.submit(2, 64, W.GEOM_SPHERE, [0.0, 0.0, 0.5], data_kind=7)
    assert e.value.code == -1
    with pytest.raises(iim.IIMError):
        iim.Server(0, 1)
    with pytest.raises(iim.IIMError):
        iim.Server(1 << 30, 65)
    srv.close()


def test_server_singular_requests():
    """Singular pure-Neumann requests (interior domains with a Neumann
    boundary) served beside a Dirichlet one: each is solved through the
    bordered system, reports a mean-free error, and matches a plain handle's
    solve bit for bit."""
    from paper_2503_22455_amd import iim
    specs = [(2, 150, [0.1, -0.05, 0.5], W.BC_NEUMANN), (3, 40, [0.05, 0.0, 0.1, 0.55], W.BC_NEUMANN),
             (2, 128, [0.0, 0.0, 0.3], W.BC_DIRICHLET)]
    outs = [torch.empty((n + 1) ** dim, dtype=torch.float64, device="cuda") for dim, n, _, _ in specs]
    srv = iim.Server(64 << 30, 3)
    tickets = [srv.submit(dim, n, W.GEOM_SPHERE, params, W.SIDE_INTERIOR, bc, data_kind=1, u_out=u,
                          precision="mixed32", rtol=1e-10) for (dim, n, params, bc), u in zip(specs, outs)]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for (dim, n, params, bc), r, u in zip(specs, res, outs):
        assert r["status"] == 0 and r["rel_residual"] <= 1e-10, r
        assert r["max_error"] < 1e-2, r
        P = iim.Problem(dim, n, W.GEOM_SPHERE, params, W.SIDE_INTERIOR, bc, precision="mixed32", rtol=1e-10)
        P.set_synthetic_data(1)
        uP, _, st = P.solve()
        assert st["bordered"] == (1 if bc == W.BC_NEUMANN else 0)
        assert st["iterations"] == r["iterations"]
        assert torch.equal(u.nan_to_num(0.0), uP.nan_to_num(0.0))
        assert P.synthetic_error(uP, 1) == r["max_error"]
        if bc == W.BC_NEUMANN:
            uu = uP[~torch.isnan(uP)]
            assert abs(float(uu.sum())) <= 1e-9 * float(uu.abs().sum())
        P.close()


def _caller_specs():
    """Requests that carry the caller's problem (data_kind 0): an interface
    star with beta^-/beta^+ = 2 (two values per control point), and an exterior
    Neumann sphere union with box faces (box data)."""
    return [dataclasses.replace(W.cfg2_star(256, beta_plus=0.5, beta_minus=1.0), precision="mixed32"),
            dataclasses.replace(W.cfg4_spheres(32, spheres=W.small_spheres_union()), precision="mixed32")]


def _caller_data(wl, P):
    """f, cp_data, box_data sampled by the caller at the library's control
    points (device tensors)."""
    from paper_2503_22455_amd import iim
    lab = P.node_labels()
    xyz, nrm = P.control_points()
    cpd = torch.tensor(np.ascontiguousarray(wl.cp_data(xyz, nrm), dtype=np.float64).ravel(), device="cuda")
    box = torch.tensor(iim.grid_to_flat(wl.box_data()), device="cuda") if wl.side != W.SIDE_INTERIOR else None
    f = torch.tensor(iim.grid_to_flat(wl.rhs(iim.flat_to_grid(lab, wl.dim, wl.n))), device="cuda")
    return f, cpd, box


def _submit_wl(srv, wl, u_out, f, cpd, box, hist_cap=0, **kw):
    return srv.submit(wl.dim, wl.n, wl.geom_kind, wl.geom_params, wl.side, wl.bc, data_kind=0, u_out=u_out, f=f,
                      cp_data=cpd, box_data=box, hist_cap=hist_cap, beta_plus=wl.beta_plus,
                      beta_minus=wl.beta_minus, precision=wl.precision, rtol=1e-10, **kw)


@pytest.mark.parametrize("batch", [True, False], ids=["batched-tails", "own-tails"])
def test_server_caller_data_alone_and_in_mix(batch):
    """Requests carrying the caller's f, control-point data and box data
    (Sec. 2.1-2.3) give, alone on one slot and inside a mix of other requests on
    four slots, bit for bit the u and residual history of a plain handle given
    the same data."""
    from paper_2503_22455_amd import iim
    ref = []
    for wl in _caller_specs():
        P = gpu_for(wl, precision="mixed32", rtol=1e-10)
        f, cpd, box = _caller_data(wl, P)
        P.set_boundary_data(cpd, box)
        P.set_rhs(f)
        u, hist, st = P.solve()
        assert st["status"] == 0, st
        P.close()
        ref.append((wl, f, cpd, box, u, hist, st))
    # alone
    for wl, f, cpd, box, u, hist, st in ref:
        s1 = iim.Server(64 << 30, 1, batch_tails=batch, batch_window_us=200)
        uo = torch.empty_like(u)
        r = s1.wait(_submit_wl(s1, wl, uo, f, cpd, box, hist_cap=500))
        s1.close()
        assert r["status"] == 0 and r["iterations"] == st["iterations"], r
        assert torch.equal(uo.nan_to_num(0.0), u.nan_to_num(0.0))
        assert np.array_equal(r["hist"], hist)
    # in a mix
    s4 = iim.Server(64 << 30, 4, batch_tails=batch, batch_window_us=200)
    outs, tickets = [], []
    for i, spec in enumerate(MIX):
        tickets.append(_submit(s4, spec))
        if i < len(ref):
            wl, f, cpd, box, u, hist, st = ref[i]
            outs.append(torch.empty_like(u))
            tickets.append(_submit_wl(s4, wl, outs[-1], f, cpd, box, hist_cap=500))
    res = [s4.wait(t) for t in tickets]
    st4 = s4.stats()
    s4.close()
    assert all(r["status"] == 0 for r in res), res
    mine = [r for r in res if "hist" in r]
    for (wl, f, cpd, box, u, hist, st), r, uo in zip(ref, mine, outs):
        assert r["iterations"] == st["iterations"] and r["max_error"] == 0.0
        assert torch.equal(uo.nan_to_num(0.0), u.nan_to_num(0.0))
        assert np.array_equal(r["hist"], hist)
    if batch:
        assert st4["tail_batches"] > 0 and st4["tail_jobs"] > st4["tail_batches"], st4
    else:
        assert st4["tail_batches"] == 0


def test_server_batched_tails_bitwise_and_graphs():
    """The V-cycle tails of requests solving together run as batched launches
    (more tails than launches); every result equals the one with each request
    launching its own tails, bit for bit, also when the iterations are replayed
    as captured HIP graphs around the batched tails."""
    from paper_2503_22455_amd import iim
    outs = {}
    stats = {}
    for mode in ("own", "batched", "batched-graph"):
        srv = iim.Server(64 << 30, 4, batch_tails=mode != "own", batch_window_us=200)
        us = [torch.empty(_numel(spec), dtype=torch.float64, device="cuda") for spec in MIX]
        kw = dict(use_graph=1) if mode == "batched-graph" else {}
        tickets = [_submit(srv, spec, u, **kw) for spec, u in zip(MIX, us)]
        res = [srv.wait(t) for t in tickets]
        stats[mode] = srv.stats()
        srv.close()
        assert all(r["status"] == 0 and r["rel_residual"] <= 1e-10 for r in res), res
        outs[mode] = (us, [r["iterations"] for r in res])
    for mode in ("batched", "batched-graph"):
        assert outs[mode][1] == outs["own"][1]
        for a, b in zip(outs[mode][0], outs["own"][0]):
            assert torch.equal(a.nan_to_num(0.0), b.nan_to_num(0.0)), mode
        assert stats[mode]["tail_jobs"] > stats[mode]["tail_batches"] > 0, stats[mode]
    assert stats["own"]["tail_batches"] == 0


def test_server_rejects_mismatched_caller_data():
    """A caller-data request whose control-point data do not match the
    problem's control points fails with IIM_E_INVALID_ARG (and the server
    carries on)."""
    from paper_2503_22455_amd import iim
    wl = _caller_specs()[0]
    P = gpu_for(wl, precision="mixed32")
    f, cpd, box = _caller_data(wl, P)
    P.close()
    srv = iim.Server(64 << 30, 1)
    r = srv.wait(_submit_wl(srv, wl, None, f, cpd[:-2].contiguous(), box))
    ok = srv.wait(_submit(srv, MIX[0]))
    srv.close()
    assert r["status"] == -1, r
    assert ok["status"] == 0, ok
