"""Python binding of libvsie.so, the gfx950 implementation of the discretised
nested VSIE operator (see include/vsie.h for the full contract).

Argument marshalling only: every step of the operator, the solver and the
weights runs in the HIP library.  PyTorch supplies device memory and streams.
Import fails loudly when the library has not been built.

Vectors are torch complex128 CUDA tensors.  A block of R right-hand sides is a
contiguous tensor of shape (R, n) -- row r is column r of the column-major
n x R matrix the C ABI expects (leading dimension n); a single vector may be
shape (n,).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "VSIE_OK", "VSIE_FP64", "VSIE_FP32", "VsieError", "Problem", "lib", "library_path",
    "vsie_assemble", "vsie_set_materials", "vsie_matvec", "vsie_matvec_adjoint", "vsie_solve",
    "vsie_plane_wave", "vsie_field", "vsie_far_field", "vsie_source_sums", "vsie_plane_wave_at", "vsie_adjoint_rhs",
    "vsie_param_gradient", "vsie_assemble_dense", "vsie_release_dense", "vsie_profile",
    "vsie_profile_read", "vsie_destroy", "vsie_last_error",
    "vsie_size", "vsie_num_cells", "vsie_matvec_multi", "vsie_get_tuning", "vsie_set_tuning", "vsie_autotune",
    "vsie_workspace_size", "VSIE_OP_MATVEC", "VSIE_OP_MATVEC_ADJOINT", "VSIE_OP_MATVEC_MULTI", "VSIE_OP_SOLVE",
    "VSIE_OP_SOLVE_ADJOINT", "VSIE_OP_SOLVE_MULTI", "vsie_matvec_noalloc", "vsie_solve_multi",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libvsie.so")

VSIE_OK, VSIE_E_INVALID, VSIE_E_DEVICE, VSIE_E_NOMEM, VSIE_E_NOCONV, VSIE_E_NAN, VSIE_E_WORKSPACE = range(7)
VSIE_FP64, VSIE_FP32 = 0, 1
VSIE_OP_MATVEC, VSIE_OP_MATVEC_ADJOINT, VSIE_OP_MATVEC_MULTI, VSIE_OP_SOLVE, VSIE_OP_SOLVE_ADJOINT, \
    VSIE_OP_SOLVE_MULTI = range(6)
_STATUS = {0: "VSIE_OK", 1: "VSIE_E_INVALID", 2: "VSIE_E_DEVICE", 3: "VSIE_E_NOMEM",
           4: "VSIE_E_NOCONV", 5: "VSIE_E_NAN", 6: "VSIE_E_WORKSPACE"}
_SZ = ctypes.c_size_t

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double


class VsieError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [
        ("n_vol", _I64), ("vx", _P), ("vy", _P), ("vz", _P), ("vw", _P), ("vdom", _P),
        ("vnb", _P), ("vgrad_alpha", _P), ("vgrad_rho", _P),
        ("n_srf", _I64), ("sx", _P), ("sy", _P), ("sz", _P), ("snx", _P), ("sny", _P),
        ("snz", _P), ("sarea", _P), ("siface", _P), ("scell_in", _P), ("scell_out", _P),
        ("rho0", _D), ("c0", _D),
    ]


class KernelStats(ctypes.Structure):
    _fields_ = [("launches", _I64), ("ms", _D), ("pairs", _D), ("rhs_pairs", _D)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", _D), ("max_iter", _I32), ("restart", _I32), ("inner_tol", _D),
                ("max_outer", _I32), ("block", _I32), ("relax", _D), ("progress", _I32),
                ("krylov_gib", _I32)]


class Tuning(ctypes.Structure):
    _fields_ = [("mfma_min_rhs", _I32), ("mfma_tg", _I32), ("mfma_nb", _I32),
                ("items_per_wave", _I32), ("vec_target_waves", _I64), ("graph", _I32),
                ("sym_groups", _I32), ("cell_face", _I32), ("mfma_3m", _I32), ("mfma64_min_rhs", _I32),
                ("mfma_chunk_max", _I32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", _I32), ("outer_steps", _I32), ("matvecs_fp64", _I32),
                ("matvecs_fp32", _I32), ("rel_residual", _D)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(library_path):
        raise ImportError("libvsie.so is not built (run: python paper_2607_06429_amd/build.py)")
    L = ctypes.CDLL(library_path)
    L.vsie_assemble.argtypes = [ctypes.POINTER(Geometry), _P, _P, _P, _I32, _P, ctypes.POINTER(_P)]
    L.vsie_set_materials.argtypes = [_P, _P, _P, _P]
    L.vsie_size.argtypes = [_P]
    L.vsie_size.restype = _I64
    L.vsie_num_cells.argtypes = [_P]
    L.vsie_num_cells.restype = _I64
    L.vsie_matvec.argtypes = [_P, _I32, _I32, _I64, _P, _I64, _P, _I64, _P, _SZ, _P]
    L.vsie_matvec_adjoint.argtypes = [_P, _I32, _I32, _I64, _P, _I64, _P, _I64, _P, _SZ, _P]
    L.vsie_matvec_noalloc.argtypes = [_P, _I32, _I32, _I64, _P, _I64, _P, _I64, _P]
    L.vsie_solve.argtypes = [_P, _I32, _I32, _I32, _I64, _P, _I64, _P, _I64,
                             ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P, _SZ, _P]
    L.vsie_solve_multi.argtypes = [_P, _I32, _I32, _I32, _I64, _P, _I64, _P, _I64,
                                   ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P, _SZ, _P]
    L.vsie_workspace_size.argtypes = [_P, _I32, _I32, _I32, _I32, _I64, ctypes.POINTER(SolveOpts),
                                      ctypes.POINTER(_SZ)]
    L.vsie_plane_wave.argtypes = [_P, _I32, _I64, _P, _P, _I64, _P]
    L.vsie_field.argtypes = [_P, _I32, _I32, _I64, _P, _P, _P, _I64, _P, _I64, _P, _I64, _P]
    L.vsie_far_field.argtypes = [_P, _I32, _I32, _I64, _P, _P, _P, _I64, _P, _I64, _P, _I64, _P]
    L.vsie_source_sums.argtypes = [_P, _I32, _I64, _P, _P, _P, _I64, _P, _I64, _P, _I64, _P,
                                   _I64, _P]
    L.vsie_plane_wave_at.argtypes = [_P, _I32, _I64, _P, _I64, _P, _P, _P, _P, _I64, _P]
    L.vsie_adjoint_rhs.argtypes = [_P, _I32, _I64, _P, _I64, _P, _I64, _P, _I64, _P]
    L.vsie_param_gradient.argtypes = [_P, _I32, _I64] + [_P, _I64] * 6 + [_P, _P, _P]
    L.vsie_assemble_dense.argtypes = [_P, _I32, _P, _I64, _P]
    L.vsie_release_dense.argtypes = [_P, _I32]
    L.vsie_profile.argtypes = [_P, _I32]
    L.vsie_profile_read.argtypes = [_P, _I32, ctypes.POINTER(KernelStats)]
    L.vsie_matvec_multi.argtypes = [_P, _I32, _I32, _I32, _I64, _P, _I64, _P, _I64, _P, _SZ, _P]
    L.vsie_get_tuning.argtypes = [_P, ctypes.POINTER(Tuning)]
    L.vsie_set_tuning.argtypes = [_P, ctypes.POINTER(Tuning)]
    L.vsie_autotune.argtypes = [_P, _I32, _I64, ctypes.POINTER(Tuning), _P]
    L.vsie_destroy.argtypes = [_P]
    L.vsie_destroy.restype = None
    L.vsie_last_error.restype = ctypes.c_char_p
    for name in ("vsie_assemble", "vsie_set_materials", "vsie_matvec", "vsie_matvec_adjoint",
                 "vsie_solve", "vsie_plane_wave", "vsie_field", "vsie_far_field", "vsie_source_sums",
                 "vsie_profile", "vsie_profile_read", "vsie_plane_wave_at", "vsie_adjoint_rhs",
                 "vsie_param_gradient", "vsie_assemble_dense", "vsie_release_dense",
                 "vsie_matvec_multi", "vsie_get_tuning", "vsie_set_tuning", "vsie_autotune",
                 "vsie_workspace_size", "vsie_matvec_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()

EXPORTED = ("vsie_assemble", "vsie_set_materials", "vsie_size", "vsie_num_cells", "vsie_matvec",
            "vsie_matvec_adjoint", "vsie_solve", "vsie_plane_wave", "vsie_field", "vsie_far_field",
            "vsie_source_sums", "vsie_plane_wave_at", "vsie_adjoint_rhs", "vsie_param_gradient",
            "vsie_assemble_dense", "vsie_release_dense", "vsie_profile", "vsie_profile_read",
            "vsie_destroy", "vsie_last_error", "vsie_matvec_multi", "vsie_get_tuning",
            "vsie_set_tuning", "vsie_autotune", "vsie_workspace_size", "vsie_matvec_noalloc", "vsie_solve_multi")

# pair-kernel kinds reported by vsie_profile_read: 2 * mode + precision
KIND_NAMES = {0: "fwd_single_layer_fp64", 1: "fwd_single_layer_fp32", 2: "fwd_double_layers_fp64",
              3: "fwd_double_layers_fp32", 4: "adj_double_layers_fp64", 5: "adj_double_layers_fp32",
              6: "source_sums_fp64", 7: "source_sums_fp32",
              8: "mfma_fwd_single_layer_fp32", 9: "mfma_fwd_double_layers_fp32",
              10: "sym_single_layer_fp64", 11: "sym_single_layer_fp32",
              12: "cell_face_fp64", 13: "cell_face_fp32",
              14: "far_field_single_layer_fp64", 15: "far_field_single_layer_fp32",
              16: "far_field_double_layers_fp64", 17: "far_field_double_layers_fp32",
              18: "face_face_fp64", 19: "face_face_fp32", 20: "dense_product_fp32",
              21: "mfma_fwd_single_layer_fp64", 22: "mfma_fwd_double_layers_fp64"}


def vsie_last_error() -> str:
    return lib.vsie_last_error().decode()


def _check(st, allow=()):
    if st != VSIE_OK and st not in allow:
        raise VsieError(st, vsie_last_error())
    return st


def _stream(stream):
    if stream is None:
        import torch
        return _P(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _P(stream)
    return _P(stream.cuda_stream)


def _arr(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _cols(t, n):
    """(pointer, nrhs, ld) of a complex128 CUDA tensor of shape (n,) or (R, n)."""
    import torch
    if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous complex128 CUDA tensor")
    if t.dim() == 1:
        if t.shape[0] != n:
            raise ValueError("vector length %d != %d" % (t.shape[0], n))
        return _P(t.data_ptr()), 1, n
    if t.dim() != 2 or t.shape[1] != n:
        raise ValueError("expected shape (R, %d), got %s" % (n, tuple(t.shape)))
    return _P(t.data_ptr()), t.shape[0], n


def _ws(workspace):
    """(pointer, bytes) of an optional caller workspace: a contiguous CUDA
    tensor of any dtype (its storage is used as raw bytes), or None."""
    if workspace is None:
        return None, 0
    if not workspace.is_cuda or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous CUDA tensor")
    return _P(workspace.data_ptr()), workspace.numel() * workspace.element_size()


def _dptr(t):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return _P(t.data_ptr())


# ---------------------------------------------------------------------------
# C ABI, one function per entry point

def vsie_assemble(geom: dict, vrho, vc, k0, stream=None):
    """geom: dict of host arrays named like the fields of vsie_geometry
    (n_vol/n_srf are taken from the array lengths).  Returns (handle, keepalive)."""
    keep = {}

    def f64(name):
        keep[name] = _arr(geom.get(name), np.float64)
        return _ptr(keep[name])

    def i32(name):
        keep[name] = _arr(geom.get(name), np.int32)
        return _ptr(keep[name])

    g = Geometry()
    g.n_vol = 0 if geom.get("vw") is None else len(geom["vw"])
    g.n_srf = 0 if geom.get("sarea") is None else len(geom["sarea"])
    for nm in ("vx", "vy", "vz", "vw", "vgrad_alpha", "vgrad_rho", "sx", "sy", "sz", "snx", "sny", "snz", "sarea"):
        setattr(g, nm, f64(nm))
    for nm in ("vdom", "vnb", "siface", "scell_in", "scell_out"):
        setattr(g, nm, i32(nm))
    g.rho0 = float(geom["rho0"])
    g.c0 = float(geom["c0"])
    rho = _arr(vrho, np.float64)
    c = _arr(vc, np.float64)
    k = _arr(np.atleast_1d(k0), np.float64)
    h = _P()
    _check(lib.vsie_assemble(ctypes.byref(g), _ptr(rho), _ptr(c), _ptr(k), len(k), _stream(stream),
                             ctypes.byref(h)))
    return h


def vsie_set_materials(h, vrho_dev, vc_dev, stream=None):
    """vrho_dev, vc_dev: float64 CUDA tensors of n_vol entries each (the C entry
    point reads that many from each pointer, so the lengths are checked here)."""
    nv = vsie_num_cells(h)
    for name, t in (("rho", vrho_dev), ("c", vc_dev)):
        if t.numel() != nv:
            raise ValueError("%s holds %d values, the problem has %d cells" % (name, t.numel(), nv))
    _check(lib.vsie_set_materials(h, _dptr(vrho_dev), _dptr(vc_dev), _stream(stream)))


def vsie_size(h) -> int:
    return int(lib.vsie_size(h))


def vsie_num_cells(h) -> int:
    return int(lib.vsie_num_cells(h))


def vsie_matvec(h, f, prec, x, y, stream=None, workspace=None):
    n = vsie_size(h)
    px, R, ldx = _cols(x, n)
    py, Ry, ldy = _cols(y, n)
    if Ry != R:
        raise ValueError("x and y hold different numbers of columns")
    _check(lib.vsie_matvec(h, f, prec, R, px, ldx, py, ldy, *_ws(workspace), _stream(stream)))


def vsie_matvec_noalloc(h, f, prec, x, y, stream=None):
    """y = A_f x with the work buffers in the library's static device work
    area (no device allocation; see include/vsie.h)."""
    n = vsie_size(h)
    px, R, ldx = _cols(x, n)
    py, Ry, ldy = _cols(y, n)
    if Ry != R:
        raise ValueError("x and y hold different numbers of columns")
    _check(lib.vsie_matvec_noalloc(h, f, prec, R, px, ldx, py, ldy, _stream(stream)))


def vsie_matvec_adjoint(h, f, prec, x, y, stream=None, workspace=None):
    n = vsie_size(h)
    px, R, ldx = _cols(x, n)
    py, Ry, ldy = _cols(y, n)
    if Ry != R:
        raise ValueError("x and y hold different numbers of columns")
    _check(lib.vsie_matvec_adjoint(h, f, prec, R, px, ldx, py, ldy, *_ws(workspace), _stream(stream)))


def vsie_matvec_multi(h, f0, nf, prec, x, y, stream=None, workspace=None):
    """x, y: (nf * R, n) -- rows t R .. t R + R - 1 belong to frequency f0 + t."""
    n = vsie_size(h)
    px, C, ldx = _cols(x, n)
    py, Cy, ldy = _cols(y, n)
    if Cy != C or C % nf:
        raise ValueError("x and y must hold nf blocks of equally many columns")
    _check(lib.vsie_matvec_multi(h, f0, nf, prec, C // nf, px, ldx, py, ldy, *_ws(workspace), _stream(stream)))


def _opts(tol=1e-10, max_iter=3000, restart=500, inner_tol=1e-5, max_outer=20, block=False, relax=0.0,
          progress=False, krylov_gib=0):
    return SolveOpts(tol, max_iter, restart, inner_tol, max_outer, 1 if block else 0, relax, 1 if progress else 0,
                     krylov_gib)


def vsie_workspace_size(h, op, f, prec, nrhs, nf=1, **opts) -> int:
    """Bytes of caller workspace the call `op` (VSIE_OP_*) needs; opts are the
    solver options of vsie_solve (solves only)."""
    o = _opts(**opts)
    b = _SZ()
    _check(lib.vsie_workspace_size(h, op, f, nf, prec, nrhs, ctypes.byref(o), ctypes.byref(b)))
    return int(b.value)


def vsie_get_tuning(h) -> dict:
    t = Tuning()
    _check(lib.vsie_get_tuning(h, ctypes.byref(t)))
    return t.as_dict()


def vsie_set_tuning(h, **kw):
    t = Tuning()
    _check(lib.vsie_get_tuning(h, ctypes.byref(t)))
    for k, v in kw.items():
        if k not in dict(Tuning._fields_):
            raise KeyError(k)
        setattr(t, k, v)
    _check(lib.vsie_set_tuning(h, ctypes.byref(t)))


def vsie_autotune(h, f, nrhs, stream=None) -> dict:
    t = Tuning()
    _check(lib.vsie_autotune(h, f, nrhs, ctypes.byref(t), _stream(stream)))
    return t.as_dict()


def vsie_solve(h, f, prec, adjoint, b, x, tol=1e-10, max_iter=3000, restart=500, inner_tol=1e-5,
               max_outer=20, block=False, stream=None, allow_noconv=False, relax=0.0, progress=False,
               workspace=None, krylov_gib=0):
    """Solve in place into x (initial guess on entry).  Returns SolveInfo as a dict
    plus the status."""
    n = vsie_size(h)
    pb, R, ldb = _cols(b, n)
    px, Rx, ldx = _cols(x, n)
    if Rx != R:
        raise ValueError("b and x hold different numbers of columns")
    o = _opts(tol, max_iter, restart, inner_tol, max_outer, block, relax, progress, krylov_gib)
    info = SolveInfo()
    st = _check(lib.vsie_solve(h, f, prec, int(adjoint), R, pb, ldb, px, ldx, ctypes.byref(o),
                               ctypes.byref(info), *_ws(workspace), _stream(stream)),
                allow=(VSIE_E_NOCONV,) if allow_noconv else ())
    d = info.as_dict()
    d["status"] = st
    return d


def vsie_solve_multi(h, f0, nf, prec, b, x, tol=1e-10, max_iter=3000, restart=500, inner_tol=1e-5,
                     max_outer=20, stream=None, allow_noconv=False, progress=False, workspace=None,
                     krylov_gib=0):
    """Solve the nf frequencies f0 .. f0 + nf - 1 in lockstep, in place into x
    (initial guess on entry).  b, x: (nf * R, n) -- rows t R .. t R + R - 1
    belong to frequency f0 + t.  Returns one SolveInfo dict per frequency and
    the status."""
    n = vsie_size(h)
    pb, C, ldb = _cols(b, n)
    px, Cx, ldx = _cols(x, n)
    if Cx != C or C % nf:
        raise ValueError("b and x must hold nf blocks of equally many columns")
    o = _opts(tol, max_iter, restart, inner_tol, max_outer, True, 0.0, progress, krylov_gib)
    infos = (SolveInfo * nf)()
    st = _check(lib.vsie_solve_multi(h, f0, nf, prec, C // nf, pb, ldb, px, ldx, ctypes.byref(o), infos,
                                     *_ws(workspace), _stream(stream)),
                allow=(VSIE_E_NOCONV,) if allow_noconv else ())
    return [i.as_dict() for i in infos], st


def vsie_plane_wave(h, f, dirs, b, stream=None):
    n = vsie_size(h)
    pb, R, ldb = _cols(b, n)
    D = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
    if D.shape != (R, 3):
        raise ValueError("need one unit direction per column of b")
    _check(lib.vsie_plane_wave(h, f, R, _ptr(D), pb, ldb, _stream(stream)))


def vsie_field(h, f, prec, tx, ty, tz, x, out, stream=None):
    n = vsie_size(h)
    px, R, ldx = _cols(x, n)
    nt = tx.shape[0]
    po, Ro, ldo = _cols(out, nt)
    if Ro != R:
        raise ValueError("x and out hold different numbers of columns")
    _check(lib.vsie_field(h, f, prec, nt, _dptr(tx), _dptr(ty), _dptr(tz), R, px, ldx, po, ldo,
                          _stream(stream)))


def vsie_far_field(h, f, prec, dx, dy, dz, x, out, stream=None):
    n = vsie_size(h)
    px, R, ldx = _cols(x, n)
    nd = dx.shape[0]
    po, Ro, ldo = _cols(out, nd)
    if Ro != R:
        raise ValueError("x and out hold different numbers of columns")
    _check(lib.vsie_far_field(h, f, prec, nd, _dptr(dx), _dptr(dy), _dptr(dz), R, px, ldx, po, ldo,
                              _stream(stream)))


def vsie_source_sums(h, f, lam, z, Z, targets=None, stream=None):
    """z: (R, n) complex128; Z: (3R, n) complex128 (row 3 r + a)."""
    n = vsie_size(h)
    if targets is None:
        pl, R, ldl = _cols(lam, n)
        nt, tx, ty, tz = n, None, None, None
    else:
        tx, ty, tz = targets
        nt = tx.shape[0]
        pl, R, ldl = _cols(lam, nt)
        tx, ty, tz = _dptr(tx), _dptr(ty), _dptr(tz)
    pz, Rz, ldz = _cols(z, n)
    pZ, RZ, ldZ = _cols(Z, n)
    if Rz != R or RZ != 3 * R:
        raise ValueError("z must have R rows and Z 3R rows")
    _check(lib.vsie_source_sums(h, f, nt, tx, ty, tz, R, pl, ldl, pz, ldz, pZ, ldZ, _stream(stream)))


def vsie_plane_wave_at(h, f, dirs, tx, ty, tz, out, stream=None):
    nt = tx.shape[0]
    po, R, ldo = _cols(out, nt)
    D = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
    if D.shape != (R, 3):
        raise ValueError("need one unit direction per column of out")
    _check(lib.vsie_plane_wave_at(h, f, R, _ptr(D), nt, _dptr(tx), _dptr(ty), _dptr(tz), po, ldo,
                                  _stream(stream)))


def vsie_adjoint_rhs(h, f, zR, ZR, out, stream=None):
    """zR: (R, n), ZR: (3R, n), out: (R, n), complex128 CUDA tensors."""
    n = vsie_size(h)
    pz, R, ldz = _cols(zR, n)
    pZ, R3, ldZ = _cols(ZR, n)
    po, Ro, ldo = _cols(out, n)
    if R3 != 3 * R or Ro != R:
        raise ValueError("inconsistent right-hand-side counts")
    _check(lib.vsie_adjoint_rhs(h, f, R, pz, ldz, pZ, ldZ, po, ldo, _stream(stream)))


def vsie_param_gradient(h, f, P, lam, z, Z, zR, ZR, grad_c, grad_rho, stream=None):
    """P, lam, z, zR: (R, n); Z, ZR: (3R, n); grad_c, grad_rho: float64 (n_vol,)."""
    n = vsie_size(h)
    args = []
    R = None
    for t, mult in ((P, 1), (lam, 1), (z, 1), (Z, 3), (zR, 1), (ZR, 3)):
        pt, r, ld = _cols(t, n)
        if R is None:
            R = r
        if r != mult * R:
            raise ValueError("inconsistent right-hand-side counts")
        args += [pt, ld]
    _check(lib.vsie_param_gradient(h, f, R, *args, _dptr(grad_c), _dptr(grad_rho), _stream(stream)))


def vsie_assemble_dense(h, f, dense, ld, stream=None):
    """dense: CUDA tensor of at least 2 * ld * n float32 values (any shape): the
    real-part plane, then the imaginary-part plane, each column-major."""
    import torch
    if dense.dtype != torch.float32 or not dense.is_cuda or not dense.is_contiguous():
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if dense.numel() < 2 * ld * vsie_size(h):
        raise ValueError("dense buffer too small")
    _check(lib.vsie_assemble_dense(h, f, _P(dense.data_ptr()), ld, _stream(stream)))


def vsie_release_dense(h, f):
    _check(lib.vsie_release_dense(h, f))


def vsie_profile(h, enable):
    _check(lib.vsie_profile(h, 1 if enable else 0))


def vsie_profile_read(h, kind):
    st = KernelStats()
    _check(lib.vsie_profile_read(h, kind, ctypes.byref(st)))
    return {"launches": st.launches, "ms": st.ms, "pairs": st.pairs, "rhs_pairs": st.rhs_pairs}


def vsie_destroy(h):
    lib.vsie_destroy(h)


# ---------------------------------------------------------------------------
# convenience wrapper

def geometry_from_mesh(mesh, rho0, c0) -> dict:
    """Host arrays of vsie_geometry from a mesh object with the attributes of
    workloads.Mesh (vol_xyz, vol_w, vol_dom, vol_nb, srf_xyz, srf_n, srf_area,
    srf_iface, srf_cell_in, srf_cell_out)."""
    v, s, nrm = mesh.vol_xyz, mesh.srf_xyz, mesh.srf_n
    return dict(vx=v[:, 0], vy=v[:, 1], vz=v[:, 2], vw=mesh.vol_w, vdom=mesh.vol_dom,
                vnb=np.ascontiguousarray(mesh.vol_nb).ravel(),
                sx=s[:, 0], sy=s[:, 1], sz=s[:, 2], snx=nrm[:, 0], sny=nrm[:, 1], snz=nrm[:, 2],
                sarea=mesh.srf_area, siface=mesh.srf_iface, scell_in=mesh.srf_cell_in,
                scell_out=mesh.srf_cell_out, rho0=rho0, c0=c0)


class Problem:
    """Owns one vsie_problem handle."""

    def __init__(self, geom: dict, vrho, vc, k0, stream=None):
        self.k0 = list(np.atleast_1d(k0).astype(float))
        self.handle = vsie_assemble(geom, vrho, vc, self.k0, stream)
        self.n = vsie_size(self.handle)
        self.n_vol = vsie_num_cells(self.handle)
        self.material_version = 0   # bumped by every accepted set_materials

    @classmethod
    def from_mesh(cls, mesh, mat, k0, stream=None, grad_alpha=None, grad_rho=None):
        g = geometry_from_mesh(mesh, mat.rho0, mat.c0)
        if grad_alpha is not None:
            g["vgrad_alpha"] = np.ascontiguousarray(grad_alpha, dtype=np.float64).ravel()
        if grad_rho is not None:
            g["vgrad_rho"] = np.ascontiguousarray(grad_rho, dtype=np.float64).ravel()
        return cls(g, mat.vol_rho, mat.vol_c, k0, stream)

    def close(self):
        if self.handle:
            vsie_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out(self, x):
        import torch
        return torch.empty_like(x)

    def matvec(self, x, f=0, prec=VSIE_FP64, out=None, workspace=None):
        y = self._out(x) if out is None else out
        vsie_matvec(self.handle, f, prec, x, y, workspace=workspace)
        return y

    def matvec_adjoint(self, x, f=0, prec=VSIE_FP64, out=None, workspace=None):
        y = self._out(x) if out is None else out
        vsie_matvec_adjoint(self.handle, f, prec, x, y, workspace=workspace)
        return y

    def matvec_multi(self, x, f0=0, nf=1, prec=VSIE_FP32, out=None, workspace=None):
        y = self._out(x) if out is None else out
        vsie_matvec_multi(self.handle, f0, nf, prec, x, y, workspace=workspace)
        return y

    def workspace_size(self, op, nrhs=1, f=0, prec=VSIE_FP64, nf=1, **opts) -> int:
        return vsie_workspace_size(self.handle, op, f, prec, nrhs, nf=nf, **opts)

    def workspace(self, op, nrhs=1, f=0, prec=VSIE_FP64, nf=1, **opts):
        """A torch uint8 CUDA tensor of vsie_workspace_size bytes (the caching
        allocator's blocks are 512-byte aligned)."""
        import torch
        nb = self.workspace_size(op, nrhs, f, prec, nf, **opts)
        return torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")

    @property
    def tuning(self) -> dict:
        return vsie_get_tuning(self.handle)

    def set_tuning(self, **kw):
        vsie_set_tuning(self.handle, **kw)

    def autotune(self, nrhs, f=0) -> dict:
        return vsie_autotune(self.handle, f, nrhs)

    def solve(self, b, f=0, prec=VSIE_FP64, adjoint=False, x0=None, **kw):
        import torch
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        info = vsie_solve(self.handle, f, prec, adjoint, b, x, **kw)
        return x, info

    def solve_multi(self, b, f0=0, nf=None, prec=VSIE_FP32, x0=None, **kw):
        """Lockstep block GMRES over the frequencies f0 .. f0 + nf - 1 (all the
        problem's frequencies from f0 by default); b: (nf * R, n).  Returns x
        and a list of per-frequency info dicts (each with the overall status)."""
        import torch
        nf = len(self.k0) - f0 if nf is None else nf
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        infos, st = vsie_solve_multi(self.handle, f0, nf, prec, b, x, **kw)
        for d in infos:
            d["status"] = st
        return x, infos

    def plane_wave(self, dirs, f=0):
        import torch
        D = np.atleast_2d(dirs)
        b = torch.empty((D.shape[0], self.n), dtype=torch.complex128, device="cuda")
        vsie_plane_wave(self.handle, f, D, b)
        return b if np.ndim(dirs) == 2 else b[0]

    def field(self, targets, x, f=0, prec=VSIE_FP64):
        import torch
        T = torch.as_tensor(np.ascontiguousarray(targets, dtype=np.float64), device="cuda")
        tx, ty, tz = (T[:, a].contiguous() for a in range(3))
        shape = (T.shape[0],) if x.dim() == 1 else (x.shape[0], T.shape[0])
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        vsie_field(self.handle, f, prec, tx, ty, tz, x, out)
        return out

    def far_field(self, directions, x, f=0, prec=VSIE_FP64):
        """Far-field pattern pinf(d) of the scattered field of solution x at unit
        directions (m, 3): p - p_inc = exp(i k0 R)/R pinf(d) + O(R^-2)."""
        import torch
        D = np.ascontiguousarray(np.atleast_2d(directions), dtype=np.float64)
        if D.ndim != 2 or D.shape[1] != 3 or not np.allclose(np.linalg.norm(D, axis=1), 1.0, atol=1e-12):
            raise ValueError("directions must be unit vectors, shape (m, 3)")
        T = torch.as_tensor(D, device="cuda")
        dx, dy, dz = (T[:, a].contiguous() for a in range(3))
        shape = (D.shape[0],) if x.dim() == 1 else (x.shape[0], D.shape[0])
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        vsie_far_field(self.handle, f, prec, dx, dy, dz, x, out)
        return out

    def source_sums(self, lam, f=0, targets=None):
        import torch
        R = 1 if lam.dim() == 1 else lam.shape[0]
        lam2 = lam.reshape(R, -1).contiguous()
        z = torch.empty((R, self.n), dtype=torch.complex128, device="cuda")
        Z = torch.empty((3 * R, self.n), dtype=torch.complex128, device="cuda")
        tg = None
        if targets is not None:
            T = torch.as_tensor(np.ascontiguousarray(targets, dtype=np.float64), device="cuda")
            tg = tuple(T[:, a].contiguous() for a in range(3))
        vsie_source_sums(self.handle, f, lam2, z, Z, targets=tg)
        return z, Z.reshape(R, 3, self.n)

    def set_materials(self, rho_dev, c_dev):
        vsie_set_materials(self.handle, rho_dev, c_dev)
        self.material_version += 1

    def plane_wave_at(self, targets, dirs, f=0):
        import torch
        T = torch.as_tensor(np.ascontiguousarray(targets, dtype=np.float64), device="cuda")
        D = np.atleast_2d(dirs)
        out = torch.empty((D.shape[0], T.shape[0]), dtype=torch.complex128, device="cuda")
        vsie_plane_wave_at(self.handle, f, D, *(T[:, a].contiguous() for a in range(3)), out)
        return out

    def adjoint_rhs(self, zR, ZR, f=0):
        """zR: (R, n); ZR: (R, 3, n) or (3R, n)."""
        import torch
        R = zR.shape[0]
        out = torch.empty((R, self.n), dtype=torch.complex128, device="cuda")
        vsie_adjoint_rhs(self.handle, f, zR.contiguous(), ZR.reshape(3 * R, self.n).contiguous(), out)
        return out

    def param_gradient(self, P, lam, z, Z, zR, ZR, n_vol, f=0):
        import torch
        R = P.shape[0]
        gc = torch.empty(n_vol, dtype=torch.float64, device="cuda")
        gr = torch.empty(n_vol, dtype=torch.float64, device="cuda")
        vsie_param_gradient(self.handle, f, P.contiguous(), lam.contiguous(), z.contiguous(),
                            Z.reshape(3 * R, self.n).contiguous(), zR.contiguous(),
                            ZR.reshape(3 * R, self.n).contiguous(), gc, gr)
        return gc, gr

    def assemble_dense(self, f=0, ld=None):
        """Allocate and fill the FP32 operator of frequency f; returns the tensor
        (keep it alive while FP32 products should use it)."""
        import torch
        ld = self.n if ld is None else ld
        A = torch.empty((2, self.n, ld), dtype=torch.float32, device="cuda")  # real and imaginary planes
        vsie_assemble_dense(self.handle, f, A, ld)
        return A

    def release_dense(self, f=0):
        vsie_release_dense(self.handle, f)

    def profile(self, enable=True):
        vsie_profile(self.handle, enable)

    def kernel_stats(self):
        """{kind name: stats} of the pair launches recorded since profile(True)."""
        out = {}
        for k, nm in KIND_NAMES.items():
            st = vsie_profile_read(self.handle, k)
            if st["launches"]:
                out[nm] = st
        return out
