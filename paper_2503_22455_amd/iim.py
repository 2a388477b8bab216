"""Python binding of the HIP immersed-interface Poisson library (libiim.so).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Device arrays are torch CUDA tensors (torch supplies device
memory and the stream); full-grid arrays are flat, contiguous, x fastest:
node (i, j, k) at i + (n+1) j + (n+1)^2 k.  The library must be built
(``python -m paper_2503_22455_amd.build``); importing this module without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiim.so")

GEOM_SPHERE, GEOM_STAR2D, GEOM_SPHERE_UNION, GEOM_GYROID = 0, 1, 2, 3
SIDE_INTERIOR, SIDE_EXTERIOR, SIDE_INTERFACE = 0, 1, 2
BC_DIRICHLET, BC_NEUMANN, BC_JUMP = 0, 1, 2
PREC = {"fp64": 0, "mixed32": 1, "mixed16": 2}
MEM_HOST, MEM_DEVICE = 0, 1
NOT_CONVERGED = 1


class IIMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("periodic", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("side", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("nparams", ctypes.c_int32), ("params", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("order_n", ctypes.c_int32), ("order_k", ctypes.c_int32), ("beta_plus", ctypes.c_double),
                ("beta_minus", ctypes.c_double), ("rtol", ctypes.c_double), ("max_iters", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
                ("coarsest_n", ctypes.c_int32), ("precision", ctypes.c_int32), ("ls_axis_t", ctypes.c_double),
                ("ls_axis_n", ctypes.c_double), ("use_graph", ctypes.c_int32), ("tail_nodes", ctypes.c_int32),
                ("fused_smoothing", ctypes.c_int32), ("colour_split", ctypes.c_int32),
                ("orthogonalisation", ctypes.c_int32), ("cycle_gamma", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("cycles", ctypes.c_int32),
                ("hist_len", ctypes.c_int32), ("final_rel_residual", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_apply_ms", ctypes.c_double),
                ("t_vcycle_ms", ctypes.c_double), ("t_krylov_ms", ctypes.c_double),
                ("second_passes", ctypes.c_int32), ("bordered", ctypes.c_int32),
                ("shift_alpha", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("levels", ctypes.c_int32), ("sides", ctypes.c_int32),
                ("n_unknowns", ctypes.c_int64), ("n_control_points", ctypes.c_int64),
                ("n_ls_entries", ctypes.c_int64), ("n_irregular", ctypes.c_int64),
                ("box_lo", ctypes.c_int64 * 3), ("box_dims", ctypes.c_int64 * 3),
                ("device_bytes", ctypes.c_int64), ("t_setup_ms", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("grid", Grid), ("geom", Geometry), ("opt", Options), ("data_kind", ctypes.c_int32),
                ("mem_kind", ctypes.c_int32), ("u_out", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("cp_data", ctypes.c_void_p), ("box_data", ctypes.c_void_p), ("n_cp_data", ctypes.c_int64),
                ("hist", ctypes.c_void_p), ("hist_cap", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("hist_len", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("max_error", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_finish", ctypes.c_double),
                ("n_unknowns", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("estimated_bytes", ctypes.c_int64), ("shift_alpha", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "running", "queued",
                                              "bytes_reserved", "bytes_budget", "peak_bytes_reserved",
                                              "tail_batches", "tail_jobs")]


class ServerOptions(ctypes.Structure):
    _fields_ = [("batch_tails", ctypes.c_int32), ("batch_window_us", ctypes.c_int32)]


_lib = None


def lib():
    """Load libiim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2503_22455_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        L.iim_last_error.restype = ctypes.c_char_p
        L.iim_default_options.argtypes = [ctypes.POINTER(Options)]
        L.iim_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Geometry), ctypes.POINTER(Options), vp,
                                 ctypes.POINTER(vp)]
        L.iim_destroy.argtypes = [vp]
        L.iim_destroy.restype = None
        L.iim_get_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.iim_control_points.argtypes = [vp, ctypes.POINTER(i64), vp, vp]
        L.iim_node_labels.argtypes = [vp, vp]
        L.iim_set_boundary_data.argtypes = [vp, vp, vp, i32]
        L.iim_set_rhs.argtypes = [vp, vp, i32]
        L.iim_set_boundary_data_noalloc.argtypes = [vp, vp, vp, i32]
        L.iim_solve.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(Stats)]
        L.iim_apply.argtypes = [vp, vp, vp, i32]
        L.iim_vcycle.argtypes = [vp, vp, vp]
        L.iim_gradient.argtypes = [vp, vp, vp]
        L.iim_boundary_quantity.argtypes = [vp, vp, vp]
        L.iim_wall_gradient.argtypes = [vp, vp, vp, vp, vp]
        L.iim_ls_stencil.argtypes = [vp, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, vp, i32]
        L.iim_level_info.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.iim_level_labels.argtypes = [vp, i32, vp]
        L.iim_level_op.argtypes = [vp, i32, i32, vp, vp]
        L.iim_time_kernel.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double)]
        L.iim_set_synthetic_data.argtypes = [vp, i32]
        L.iim_synthetic_error.argtypes = [vp, i32, vp, ctypes.POINTER(ctypes.c_double)]
        u64 = ctypes.c_uint64
        L.iim_server_create.argtypes = [i64, i32, ctypes.POINTER(vp)]
        L.iim_server_create_ex.argtypes = [i64, i32, ctypes.POINTER(ServerOptions), ctypes.POINTER(vp)]
        L.iim_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)]
        L.iim_server_poll.argtypes = [vp, u64, ctypes.POINTER(Result)]
        L.iim_server_wait.argtypes = [vp, u64, ctypes.POINTER(Result)]
        L.iim_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.iim_server_clock.argtypes = [vp]
        L.iim_server_clock.restype = ctypes.c_double
        L.iim_server_destroy.argtypes = [vp]
        L.iim_server_destroy.restype = None
        _lib = L
    return _lib


def _check(rc: int, allow_not_converged: bool = False) -> int:
    if rc == 0 or (allow_not_converged and rc == NOT_CONVERGED):
        return rc
    raise IIMError(rc, lib().iim_last_error().decode())


def _ptr(t) -> int:
    """Device pointer of a contiguous torch CUDA tensor."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def grid_to_flat(a: np.ndarray) -> np.ndarray:
    """Array indexed [ix, iy(, iz)] -> flat x-fastest vector."""
    return np.ascontiguousarray(np.asarray(a).ravel(order="F"))


def flat_to_grid(v: np.ndarray, dim: int, n: int) -> np.ndarray:
    return np.asarray(v).reshape((n + 1,) * dim, order="F")


def make_options(beta_plus: float = 1.0, beta_minus: float = 1.0, rtol: float = 1e-10, max_iters: int = 500,
                 restart: int = 10, nu_pre: int = 2, nu_post: int = 2, coarsest_n: int = 8,
                 precision: str = "fp64", ls_axes: Optional[Tuple[float, float]] = None, use_graph: int = 2,
                 tail_nodes: int = 0, fused_smoothing: bool = True, colour_split: bool = True,
                 order: Tuple[int, int] = (4, 5), orthogonalisation: int = 1, cycle: str = "V") -> Options:
    o = Options()
    lib().iim_default_options(ctypes.byref(o))
    o.order_n, o.order_k = int(order[0]), int(order[1])
    o.beta_plus, o.beta_minus, o.rtol, o.max_iters = beta_plus, beta_minus, rtol, max_iters
    o.restart, o.nu_pre, o.nu_post, o.coarsest_n = restart, nu_pre, nu_post, coarsest_n
    o.precision = PREC[precision]
    o.use_graph = int(use_graph)
    o.tail_nodes = int(tail_nodes)
    o.fused_smoothing = int(fused_smoothing)
    o.colour_split = int(colour_split)
    o.orthogonalisation = int(orthogonalisation)
    o.cycle_gamma = {"V": 1, "W": 2}[cycle.upper()]
    if ls_axes is not None:
        o.ls_axis_t, o.ls_axis_n = ls_axes
    return o


class Problem:
    """One immersed-interface Poisson problem resident on the current device."""

    def __init__(self, dim: int, n: int, geom_kind: int, geom_params, side: int, bc: int,
                 beta_plus: float = 1.0, beta_minus: float = 1.0, rtol: float = 1e-10, max_iters: int = 500,
                 restart: int = 10, nu_pre: int = 2, nu_post: int = 2, coarsest_n: int = 8,
                 precision: str = "fp64", ls_axes: Optional[Tuple[float, float]] = None,
                 lo: float = -1.0, hi: float = 1.0, use_graph: int = 2, tail_nodes: int = 0,
                 fused_smoothing: bool = True, colour_split: bool = True, order: Tuple[int, int] = (4, 5),
                 orthogonalisation: int = 1, cycle: str = "V", stream=None, periodic: bool = False):
        L = lib()
        self.dim, self.n = dim, n
        self.side, self.bc = side, bc
        self.total = (n + 1) ** dim
        g = Grid(dim, n, lo, hi, int(periodic), 0)
        pa = (ctypes.c_double * len(geom_params))(*[float(v) for v in geom_params])
        geo = Geometry(geom_kind, side, bc, len(geom_params), pa)
        o = make_options(beta_plus, beta_minus, rtol, max_iters, restart, nu_pre, nu_post, coarsest_n, precision,
                         ls_axes, use_graph, tail_nodes, fused_smoothing, colour_split, order,
                         orthogonalisation, cycle)
        self._h = ctypes.c_void_p()
        # default: the library orders its own stream after the legacy default stream
        s = 0 if stream is None else stream
        _check(L.iim_create(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(o), ctypes.c_void_p(s),
                            ctypes.byref(self._h)))

    # -- lifetime --------------------------------------------------------------
    def close(self):
        if self._h:
            lib().iim_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries ------------------------------------------------------------------
    def info(self) -> dict:
        inf = Info()
        _check(lib().iim_get_info(self._h, ctypes.byref(inf)))
        return {k: (list(getattr(inf, k)) if k in ("box_lo", "box_dims") else getattr(inf, k))
                for k, _ in Info._fields_}

    def control_points(self) -> Tuple[np.ndarray, np.ndarray]:
        cnt = ctypes.c_int64()
        _check(lib().iim_control_points(self._h, ctypes.byref(cnt), None, None))
        xyz = np.zeros((cnt.value, self.dim))
        nrm = np.zeros((cnt.value, self.dim))
        if cnt.value:
            _check(lib().iim_control_points(self._h, ctypes.byref(cnt), xyz.ctypes.data, nrm.ctypes.data))
        return xyz, nrm

    def node_labels(self) -> np.ndarray:
        out = np.zeros(self.total, dtype=np.uint8)
        _check(lib().iim_node_labels(self._h, out.ctypes.data))
        return out

    def ls_stencil(self, cp: int, side: int = 1) -> Tuple[np.ndarray, np.ndarray]:
        m, r = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().iim_ls_stencil(self._h, cp, side, ctypes.byref(m), ctypes.byref(r), None, None, 0))
        idx = np.zeros(m.value, dtype=np.int64)
        wts = np.zeros((m.value + 1, r.value))
        _check(lib().iim_ls_stencil(self._h, cp, side, ctypes.byref(m), ctypes.byref(r), idx.ctypes.data,
                                    wts.ctypes.data, m.value + 1))
        return idx, wts

    def level_info(self, level: int) -> Tuple[int, int]:
        n, nu = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().iim_level_info(self._h, level, ctypes.byref(n), ctypes.byref(nu)))
        return n.value, nu.value

    def level_labels(self, level: int) -> np.ndarray:
        n, _ = self.level_info(level)
        out = np.zeros((n + 1) ** self.dim, dtype=np.uint8)
        _check(lib().iim_level_labels(self._h, level, out.ctypes.data))
        return out

    # -- data ---------------------------------------------------------------------
    @staticmethod
    def _dev(a):
        import torch
        if hasattr(a, "is_cuda") and a.is_cuda:
            return a.contiguous()
        return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()

    def set_boundary_data(self, cp_data, box_data=None):
        """cp_data: one value per control point (two, j0 then j1, for jumps);
        box_data: full-grid array (only box faces are read) or None."""
        cpd = self._dev(cp_data)
        box = None if box_data is None else self._dev(box_data)
        _check(lib().iim_set_boundary_data(self._h, _ptr(cpd) if cpd.numel() else None,
                                           None if box is None else _ptr(box), MEM_DEVICE))

    def set_boundary_data_noalloc(self, cp_data, box_data=None):
        """As set_boundary_data, with no device allocation in the library
        (iim_set_boundary_data_noalloc: box data staged in its static array)."""
        cpd = self._dev(cp_data)
        box = None if box_data is None else self._dev(box_data)
        _check(lib().iim_set_boundary_data_noalloc(self._h, _ptr(cpd) if cpd.numel() else None,
                                                   None if box is None else _ptr(box), MEM_DEVICE))

    def set_rhs(self, f):
        ft = self._dev(f)
        _check(lib().iim_set_rhs(self._h, _ptr(ft), MEM_DEVICE))

    # -- operations on device tensors ---------------------------------------------------
    def apply(self, x, with_data: bool = False):
        import torch
        y = torch.empty_like(x)
        _check(lib().iim_apply(self._h, _ptr(x), _ptr(y), int(with_data)))
        return y

    def vcycle(self, v):
        import torch
        z = torch.empty_like(v)
        _check(lib().iim_vcycle(self._h, _ptr(v), _ptr(z)))
        return z

    def gradient(self, u):
        """grad u at the unknowns (order-n central first derivative over the
        extended function), shape (dim, (n+1)^dim) on the device, NaN
        elsewhere; u a full-grid device array (a solution of this problem)."""
        import torch
        g = torch.empty((self.dim, u.numel()), dtype=torch.float64, device=u.device)
        _check(lib().iim_gradient(self._h, _ptr(u), _ptr(g)))
        return g

    def boundary_quantity(self, u):
        """Per control point: du/dn (Dirichlet), u (Neumann) or du+/dn
        (interface) from the fits' normal-derivative rows."""
        import torch
        q = torch.empty(max(int(self.info()["n_control_points"]), 1), dtype=torch.float64, device=u.device)
        _check(lib().iim_boundary_quantity(self._h, _ptr(u), _ptr(q)))
        return q[: int(self.info()["n_control_points"])]

    def wall_gradient(self, u, u_inf=None):
        """Gradient of the solved side's fit at every control point, shape
        (n_control_points, dim) on the device; with a free stream u_inf (dim
        values) also the pressure coefficient 1 - |grad + u_inf|^2 / |u_inf|^2
        per control point (returned as a second tensor)."""
        import torch
        ncp = int(self.info()["n_control_points"])
        g = torch.empty((max(ncp, 1), self.dim), dtype=torch.float64, device=u.device)
        cp = None
        ui = None
        if u_inf is not None:
            cp = torch.empty(max(ncp, 1), dtype=torch.float64, device=u.device)
            ui = (ctypes.c_double * self.dim)(*[float(v) for v in u_inf])
        _check(lib().iim_wall_gradient(self._h, _ptr(u), _ptr(g), ui, None if cp is None else _ptr(cp)))
        return (g[:ncp], cp[:ncp]) if cp is not None else g[:ncp]

    def level_op(self, level: int, op: int, in1, out):
        _check(lib().iim_level_op(self._h, level, op, _ptr(in1), _ptr(out)))
        return out

    def time_kernel(self, kernel: int, reps: int = 20) -> float:
        """Average milliseconds per launch of one hot-path kernel (HIP events on
        the handle's stream); see iim_time_kernel for the ids."""
        ms = ctypes.c_double()
        _check(lib().iim_time_kernel(self._h, kernel, reps, ctypes.byref(ms)))
        return ms.value

    def solve(self, x0=None, hist_cap: int = 1000):
        import torch
        u = torch.empty(self.total, dtype=torch.float64, device="cuda")
        hist = np.zeros(hist_cap)
        st = Stats()
        rc = lib().iim_solve(self._h, _ptr(u), None if x0 is None else _ptr(x0), hist.ctypes.data, hist_cap,
                             ctypes.byref(st))
        _check(rc, allow_not_converged=True)
        stats = {k: getattr(st, k) for k, _ in Stats._fields_}
        return u, hist[: st.hist_len].copy(), stats


    def set_synthetic_data(self, kind: int = 1):
        """Device-side manufactured data (see iim_set_synthetic_data)."""
        _check(lib().iim_set_synthetic_data(self._h, kind))

    def synthetic_error(self, u, kind: int = 1) -> float:
        e = ctypes.c_double()
        _check(lib().iim_synthetic_error(self._h, kind, _ptr(u), ctypes.byref(e)))
        return e.value


class Server:
    """Continuous-batching solve server on the current device (iim_server_*)."""

    def __init__(self, budget_bytes: int, max_slots: int, batch_tails: bool = False, batch_window_us: int = 0):
        self._s = ctypes.c_void_p()
        self._keep = {}
        o = ServerOptions(int(batch_tails), int(batch_window_us))
        _check(lib().iim_server_create_ex(int(budget_bytes), int(max_slots), ctypes.byref(o), ctypes.byref(self._s)))

    def submit(self, dim: int, n: int, geom_kind: int, geom_params, side: int = SIDE_INTERIOR,
               bc: int = BC_DIRICHLET, data_kind: int = 1, u_out=None, lo: float = -1.0, hi: float = 1.0,
               f=None, cp_data=None, box_data=None, hist_cap: int = 0, periodic: bool = False, **opt) -> int:
        """data_kind 1: device-side manufactured data; data_kind 0: the caller's
        f (full grid), cp_data (per control point, in the library's order) and
        box_data (full grid or None), as contiguous CUDA tensors that stay
        alive (the server keeps references) until the result is collected;
        hist_cap > 0 collects the residual history (returned by wait/poll)."""
        pa = (ctypes.c_double * len(geom_params))(*[float(v) for v in geom_params])
        req = Request(Grid(dim, n, lo, hi, int(periodic), 0), Geometry(geom_kind, side, bc, len(geom_params), pa), make_options(**opt),
                      data_kind, MEM_DEVICE, None if u_out is None else _ptr(u_out))
        keep = [u_out]
        if data_kind == 0:
            req.f = _ptr(f)
            req.cp_data = _ptr(cp_data) if cp_data is not None and cp_data.numel() else None
            req.n_cp_data = 0 if cp_data is None else int(cp_data.numel())
            req.box_data = None if box_data is None else _ptr(box_data)
            keep += [f, cp_data, box_data]
        hist = None
        if hist_cap > 0:
            hist = np.zeros(int(hist_cap))
            req.hist, req.hist_cap = hist.ctypes.data, int(hist_cap)
        t = ctypes.c_uint64()
        _check(lib().iim_server_submit(self._s, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = (keep, hist)  # alive until the result is collected
        return t.value

    @staticmethod
    def _dict(r: Result) -> dict:
        return {k: getattr(r, k) for k, _ in Result._fields_}

    def _collect(self, ticket: int, r: Result) -> dict:
        d = self._dict(r)
        keep, hist = self._keep.pop(ticket, (None, None))
        if hist is not None:
            d["hist"] = hist[: r.hist_len].copy()
        return d

    def poll(self, ticket: int) -> dict:
        r = Result()
        _check(lib().iim_server_poll(self._s, ticket, ctypes.byref(r)))
        if r.done:
            return self._collect(ticket, r)
        return self._dict(r)

    def wait(self, ticket: int) -> dict:
        r = Result()
        _check(lib().iim_server_wait(self._s, ticket, ctypes.byref(r)))
        return self._collect(ticket, r)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().iim_server_stats_get(self._s, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def clock(self) -> float:
        return lib().iim_server_clock(self._s)

    def close(self):
        if self._s:
            lib().iim_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_workload(wl, precision: Optional[str] = None, **kw) -> Problem:
    """Problem for a workloads.Workload description."""
    kw.setdefault("order", tuple(getattr(wl, "order", (4, 5))))
    kw.setdefault("orthogonalisation", int(getattr(wl, "orthogonalisation", 1)))
    kw.setdefault("cycle", str(getattr(wl, "cycle", "V")))
    kw.setdefault("lo", getattr(wl, "lo", -1.0))
    kw.setdefault("hi", getattr(wl, "hi", 1.0))
    kw.setdefault("periodic", bool(getattr(wl, "periodic", False)))
    return Problem(wl.dim, wl.n, wl.geom_kind, wl.geom_params, wl.side, wl.bc, wl.beta_plus, wl.beta_minus,
                   precision=precision or wl.precision, **kw)
