"""Shared set-up for GPU parity tests: the same seeded workload given to the
HIP library and to the CPU oracle (which never sees library outputs)."""
import numpy as np

import workloads as W
from oracle.iim import IIMProblem


def oracle_for(wl, **kw):
    return IIMProblem(wl.dim, wl.n, wl.geom_kind, wl.geom_params, wl.side, wl.bc, wl.beta_plus, wl.beta_minus,
                      lo=wl.lo, hi=wl.hi, periodic=wl.periodic, **kw)


def gpu_for(wl, **kw):
    from paper_2503_22455_amd import iim
    return iim.from_workload(wl, **kw)


def flat(a):
    return np.ascontiguousarray(np.asarray(a).ravel(order="F"))


def oracle_data(O, wl):
    """cp data, box data (full grid, flat) and f (full grid, flat) from the oracle's own control points."""
    xyz, nrm = O.cp_arrays()
    cpd = wl.cp_data(xyz, nrm) if O.ncp else np.zeros(0)
    box = flat(wl.box_data())
    f = flat(wl.rhs(O.labels))
    return cpd, box, f
