"""Host-side checks of libvsie.so: exported symbols and argument validation.

These run without a GPU: every case fails validation before the library
touches a device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def V():
    import paper_2607_06429_amd as V
    return V


def test_header_symbols_are_exported(V):
    hdr = open(os.path.join(ROOT, "include", "vsie.h")).read()
    declared = set(re.findall(r"^\s*(?:vsie_status|int64_t|void|const char \*)\s*\*?\s*(vsie_\w+)\s*\(", hdr, re.M))
    assert {"vsie_assemble", "vsie_matvec", "vsie_matvec_adjoint", "vsie_solve"} <= declared
    lib = ctypes.CDLL(V.library_path)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(V.EXPORTED) == declared


def _geom(V, mesh):
    return V.geometry_from_mesh(mesh, 1.0, 1.0)


def _assemble(V, g, rho, c, k=(2.0,)):
    return V.vsie_assemble(g, rho, c, list(k), stream=0)


@pytest.fixture(scope="module")
def small():
    mesh = W.nested_balls(6)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8)
    return mesh, mat


@pytest.mark.parametrize("mutate,msg", [
    (lambda g, r, c: g.__setitem__("snx", g["snx"] * 1.1), "unit length"),
    (lambda g, r, c: r.__setitem__(3, -1.0), "positive"),
    (lambda g, r, c: c.__setitem__(0, 0.0), "positive"),
    (lambda g, r, c: g.__setitem__("vdom", np.where(np.arange(len(g["vdom"])) == 2, 3, g["vdom"])), "subdomain"),
    (lambda g, r, c: g.__setitem__("scell_in", np.full(len(g["scell_in"]), 10 ** 6)), "inside cell"),
    (lambda g, r, c: g.__setitem__("vw", -np.asarray(g["vw"])), "volume"),
    (lambda g, r, c: g.__setitem__("vnb", np.full(len(g["vnb"]), 10 ** 7)), "neighbour"),
    (lambda g, r, c: g.__setitem__("rho0", 0.0), "rho0"),
    (lambda g, r, c: g.__setitem__("vx", np.full(len(g["vx"]), np.nan)), "centroid"),
])
def test_invalid_geometry_is_rejected(V, small, mutate, msg):
    mesh, mat = small
    g = _geom(V, mesh)
    g = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    rho, c = mat.vol_rho.copy(), mat.vol_c.copy()
    mutate(g, rho, c)
    with pytest.raises(V.VsieError) as e:
        _assemble(V, g, rho, c)
    assert e.value.status == V.VSIE_E_INVALID
    assert msg in str(e.value)


def test_invalid_wavenumber_is_rejected(V, small):
    mesh, mat = small
    for k in ([0.0], [-1.0], [np.inf]):
        with pytest.raises(V.VsieError) as e:
            _assemble(V, _geom(V, mesh), mat.vol_rho, mat.vol_c, k)
        assert e.value.status == V.VSIE_E_INVALID


def test_null_handles(V):
    lib = V.lib
    assert lib.vsie_size(None) == 0
    lib.vsie_destroy(None)
    st = lib.vsie_matvec(None, 0, 0, 1, None, 1, None, 1, None, 0, None)
    assert st == V.VSIE_E_INVALID and "NULL" in V.vsie_last_error()
    info = V.SolveInfo()
    st = lib.vsie_solve(None, 0, 0, 0, 1, None, 1, None, 1, None, ctypes.byref(info), None, 0, None)
    assert st == V.VSIE_E_INVALID and info.iterations == 0
    infos = (V.SolveInfo * 2)()
    infos[1].iterations = 5
    st = lib.vsie_solve_multi(None, 0, 2, 0, 1, None, 1, None, 1, None, infos, None, 0, None)
    assert st == V.VSIE_E_INVALID and infos[1].iterations == 0 and "NULL" in V.vsie_last_error()
    g = V.Geometry()
    h = ctypes.c_void_p(1234)
    st = lib.vsie_assemble(ctypes.byref(g), None, None, None, 0, None, ctypes.byref(h))
    assert st == V.VSIE_E_INVALID and h.value is None


def test_struct_layouts_match_header(V, tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's size
    and field offsets (a gcc program built from include/vsie.h prints them)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    structs = {"vsie_geometry": V.Geometry, "vsie_tuning": V.Tuning, "vsie_solve_opts": V.SolveOpts,
               "vsie_solve_info": V.SolveInfo, "vsie_kernel_stats": V.KernelStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "vsie.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(out["%s size" % cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out["%s.%s" % (cname, fname)]) == getattr(cls, fname).offset, (cname, fname)


def test_set_materials_lengths_checked_in_binding(V):
    """The C entry point reads n_vol doubles from each material pointer, so the
    binding rejects tensors of another length before calling it (NULL handle:
    n_vol = 0)."""
    import torch
    assert V.lib.vsie_num_cells(None) == 0
    short = torch.zeros(3, dtype=torch.float64)
    with pytest.raises(ValueError):
        V.vsie_set_materials(None, short, short)


def test_workspace_size_argument_checks(V):
    """vsie_workspace_size rejects a NULL handle and a NULL output before any
    device work (and zeroes the output)."""
    b = ctypes.c_size_t(77)
    st = V.lib.vsie_workspace_size(None, V.VSIE_OP_SOLVE, 0, 1, 0, 1, None, ctypes.byref(b))
    assert st == V.VSIE_E_INVALID and b.value == 0
    st = V.lib.vsie_workspace_size(None, V.VSIE_OP_MATVEC, 0, 1, 0, 1, None, None)
    assert st == V.VSIE_E_INVALID
    b.value = 5
    st = V.lib.vsie_workspace_size(None, V.VSIE_OP_SOLVE_MULTI, 0, 2, 1, 16, None, ctypes.byref(b))
    assert st == V.VSIE_E_INVALID and b.value == 0
    assert V.VSIE_OP_SOLVE_MULTI == 5
    # the solver options structure carries the Krylov budget after progress
    names = [f[0] for f in V.SolveOpts._fields_]
    assert names[-2:] == ["progress", "krylov_gib"]
    assert V._STATUS[V.VSIE_E_WORKSPACE] == "VSIE_E_WORKSPACE"
