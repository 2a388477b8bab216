"""The C ABI library loads and exports every function include/iim.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iim.h")
LIB = os.path.join(ROOT, "paper_2503_22455_amd", "libiim.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(iim_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_abi():
    names = declared_functions()
    for must in ("iim_create", "iim_destroy", "iim_solve", "iim_apply", "iim_vcycle", "iim_set_rhs",
                 "iim_set_boundary_data", "iim_control_points", "iim_last_error"):
        assert must in names


def test_library_exports_every_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libiim.so not built in this checkout")
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the Python binding mirrors has the header's size and field
    offsets (a C program built from include/iim.h with the host compiler prints
    them; nothing is loaded onto a GPU)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    from paper_2503_22455_amd import iim
    mirrors = {"iim_grid": iim.Grid, "iim_geometry": iim.Geometry, "iim_options": iim.Options,
               "iim_stats": iim.Stats, "iim_info": iim.Info, "iim_request": iim.Request,
               "iim_result": iim.Result, "iim_server_stats": iim.ServerStats,
               "iim_server_options": iim.ServerOptions}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "iim.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    import ctypes as C
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_default_options():
    """iim_default_options (a host-only call) fills the documented defaults."""
    if not os.path.exists(LIB):
        pytest.skip("libiim.so not built in this checkout")
    from paper_2503_22455_amd import iim
    o = iim.make_options()
    assert (o.order_n, o.order_k, o.restart, o.nu_pre, o.nu_post, o.coarsest_n) == (4, 5, 10, 2, 2, 8)
    assert o.rtol == 1e-10 and o.use_graph == 2 and o.colour_split == 1 and o.fused_smoothing == 1
    assert o.orthogonalisation == 1


def test_disconnected_interior_neumann_union_is_rejected():
    """A singular problem is bordered with one constant (Sec. 2.3), which pins
    the null space of a connected domain only: iim_create rejects the interior
    of two disjoint spheres with a Neumann condition before touching the
    device, and lets the interior of two overlapping ones through that check
    (a host-only path: no GPU is needed to see the rejection)."""
    if not os.path.exists(LIB):
        pytest.skip("libiim.so not built in this checkout")
    from paper_2503_22455_amd import iim
    L = iim.lib()

    def create(spheres):
        params = [float(len(spheres))]
        for c, r in spheres:
            params += list(c) + [r]
        pa = (ctypes.c_double * len(params))(*params)
        g = iim.Grid(3, 32, -1.0, 1.0)
        geo = iim.Geometry(iim.GEOM_SPHERE_UNION, iim.SIDE_INTERIOR, iim.BC_NEUMANN, len(params), pa)
        o = iim.make_options()
        h = ctypes.c_void_p()
        rc = L.iim_create(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(o), None, ctypes.byref(h))
        if rc == 0:
            L.iim_destroy(h)
        return rc, L.iim_last_error().decode()

    rc, msg = create([((-0.4, 0.0, 0.0), 0.3), ((0.4, 0.0, 0.0), 0.3)])
    assert rc == -1 and "not connected" in msg, (rc, msg)
    rc, msg = create([((-0.2, 0.0, 0.0), 0.3), ((0.2, 0.0, 0.0), 0.3)])
    assert "not connected" not in msg, (rc, msg)
