"""FP64 CPU oracle for the nested VSIE hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the GPU
library (``paper_2607_06429_amd``) and never imports it; the two meet only in
the seeded inputs of ``workloads``.

Everything here is plain FP64: numpy for O(n) work, the C file
``vsie_oracle.c`` (built with gcc) for the O(n^2) direct sums, scipy for the
dense LU and the special functions of the analytic references.

Sources followed (paper = "Nested Volume-Surface Integral Equations for
Acoustics"):

* material parameters alpha, beta ........ section 2.2.1, eqs. eq_alpha, eq_beta
* Green's function ......................... eq_greens_function
* the operator  m p - V p + T p + K p ...... Theorem 3, eq_vsie
* mass function m .......................... eq_mass_function
* P0 + centroid collocation + midpoint rule,
  equal-volume-sphere self-term ............ section 2.3.5 ("Discrete representation")
* plane wave ............................... eq_planewave
* relative error ........................... eq_error
* GMRES (no preconditioner) ................ section 3.1 ("Computational settings")
* exterior field by the representation formula (m = 1 in Omega_0) ... section 2.3.1
* its far-field pattern (leading terms of G and grad G as |x| -> inf) ... section 2.3.1

Readings where the paper is silent:

* the T and K self-terms are zero (a flat face has (y - x).n = 0; the gradient
  of a ball's potential vanishes at its centre);
* grad(alpha) from per-cell densities by central differences over face
  neighbours in the same subdomain, one-sided with one neighbour, zero with none;
* interface limit densities are those of the cells on either side of a face;
* the equal-volume-sphere self integral uses its power series for k a < 0.5
  (the closed form cancels catastrophically there).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vsie_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib_handle = None


def build(force: bool = True) -> str:
    """Compile vsie_oracle.c with gcc (-O2, OpenMP, IEEE arithmetic)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        I = ctypes.c_int
        L.vo_apply.argtypes = [I64, P, P, P, P, I64, I64, I64, P, P, P, P, P, P, P, P, P, P, P,
                               D, I, I64, P, P]
        L.vo_apply_adjoint.argtypes = [I64, P, P, P, I64, I64, P, P, P, P, P, P, P, P, P, P, P,
                                       D, I, I64, P, P]
        L.vo_source_sums.argtypes = [I64, P, P, P, I64, P, P, P, D, I, I64, P, P, P]
        L.vo_assemble.argtypes = [I64, I64, P, P, P, P, P, P, P, P, P, P, P, D, P]
        L.vo_num_threads.restype = ctypes.c_int
        _lib_handle = L
    return _lib_handle


def num_threads() -> int:
    return int(_lib().vo_num_threads())


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# material parameters (eq_alpha, eq_beta)

def alpha(rho, rho0):
    """alpha = rho0/rho - 1 (eq_alpha); zero in the exterior."""
    return rho0 / np.asarray(rho, dtype=np.float64) - 1.0


def beta(rho, c, rho0, c0, omega):
    """beta = (rho0/rho)(omega/c)^2 - (omega/c0)^2 (eq_beta)."""
    rho = np.asarray(rho, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    return (rho0 / rho) * (omega / c) ** 2 - (omega / c0) ** 2


def grad_alpha_stencil(mesh, a_cells):
    """grad(alpha) at cell centroids from per-cell alpha (reading of the paper's
    grad alpha for per-cell data): per axis, a central difference over the two
    face neighbours in the same subdomain, one-sided with one, zero with none."""
    x = mesh.vol_xyz
    dom = mesh.vol_dom
    g = np.zeros((mesh.n_vol, 3))
    for ax in range(3):
        lo = mesh.vol_nb[:, 2 * ax].astype(np.int64)
        hi = mesh.vol_nb[:, 2 * ax + 1].astype(np.int64)
        lo_ok = (lo >= 0) & (dom[np.maximum(lo, 0)] == dom)
        hi_ok = (hi >= 0) & (dom[np.maximum(hi, 0)] == dom)
        for i in range(mesh.n_vol):
            if lo_ok[i] and hi_ok[i]:
                g[i, ax] = (a_cells[hi[i]] - a_cells[lo[i]]) / (x[hi[i], ax] - x[lo[i], ax])
            elif hi_ok[i]:
                g[i, ax] = (a_cells[hi[i]] - a_cells[i]) / (x[hi[i], ax] - x[i, ax])
            elif lo_ok[i]:
                g[i, ax] = (a_cells[i] - a_cells[lo[i]]) / (x[i, ax] - x[lo[i], ax])
    return g


# ---------------------------------------------------------------------------
# self-interaction on the sphere of equal volume (section 2.3.5)

def ball_centre_integral(a, k):
    """S(a, k) = integral over the ball of radius a of G_k(0, y) dy
             = int_0^a r exp(i k r) dr = ((1 - i k a) exp(i k a) - 1) / k^2.

    For k a < 0.5 the power series sum_{n>=2} i^n k^(n-2) a^n (1 - n) / n!
    is used instead (the closed form loses digits to cancellation there)."""
    a = np.asarray(a, dtype=np.float64)
    ka = k * a
    out = np.empty(a.shape, dtype=np.complex128)
    big = ka >= 0.5
    if np.any(big):
        ab = a[big]
        out[big] = ((1.0 - 1j * k * ab) * np.exp(1j * k * ab) - 1.0) / k ** 2
    small = ~big
    if np.any(small):
        asml = a[small]
        acc = np.zeros(asml.shape, dtype=np.complex128)
        for n in range(2, 40):
            acc += (1j ** n) * k ** (n - 2) * asml ** n * (1 - n) / math.factorial(n)
        out[small] = acc
    return out


# ---------------------------------------------------------------------------
# the discretised operator

@dataclasses.dataclass
class Discretisation:
    k0: float
    n_vol: int
    n_srf: int
    pts: np.ndarray    # (n, 3) collocation points / source centroids
    sV: np.ndarray     # (n_vol,) |cell| (beta - k0^2 alpha)
    gT: np.ndarray     # (n_vol, 3) |cell| grad alpha
    nrm: np.ndarray    # (n_srf, 3) face normals
    dK: np.ndarray     # (n_srf,) |face| * alpha jump
    m: np.ndarray      # (n,) mass function
    D: np.ndarray      # (n,) self-term of -V (zero on surfaces)

    @property
    def n(self):
        return self.n_vol + self.n_srf

    @property
    def diag(self):
        return self.m - self.D


def grad_alpha_from_density_gradient(rho, grad_rho, rho0):
    """grad alpha of an analytic density: alpha = rho0/rho - 1 (eq_alpha), so
    grad alpha = -rho0 grad(rho) / rho^2 at each centroid."""
    rho = np.asarray(rho, dtype=np.float64)
    return -rho0 * np.asarray(grad_rho, dtype=np.float64) / (rho * rho)[:, None]


def discretise(mesh, mat, k0, grad_alpha=None, grad_rho=None) -> Discretisation:
    """Per-element data of the collocation system (Theorem 3 with P0 elements,
    centroid collocation and the midpoint rule).  grad alpha: given, else from
    an analytic density gradient grad_rho, else the neighbour stencil."""
    rho0, c0 = mat.rho0, mat.c0
    omega = k0 * c0
    rho = mat.vol_rho
    a_cells = alpha(rho, rho0)
    b_cells = beta(rho, mat.vol_c, rho0, c0, omega)
    w = mesh.vol_w
    sV = w * (b_cells - k0 ** 2 * a_cells)
    if grad_alpha is not None:
        ga = np.asarray(grad_alpha)
    elif grad_rho is not None:
        ga = grad_alpha_from_density_gradient(rho, grad_rho, rho0)
    else:
        ga = grad_alpha_stencil(mesh, a_cells)
    gT = w[:, None] * ga

    # surfaces: limit densities from the adjacent cells; exterior has rho0 (alpha = 0)
    rho_in = rho[mesh.srf_cell_in]
    rho_out = np.where(mesh.srf_cell_out >= 0, rho[np.maximum(mesh.srf_cell_out, 0)], rho0)
    a_in = alpha(rho_in, rho0)
    a_out = alpha(rho_out, rho0)
    # Gamma_1 carries alpha_1 (the exterior side has alpha = 0), Gamma_2 carries alpha_2 - alpha_1
    jump = np.where(mesh.srf_iface == 1, a_in, a_in - a_out)
    dK = mesh.srf_area * jump

    # mass function (eq_mass_function)
    m_vol = rho0 / rho
    m_srf = np.where(mesh.srf_iface == 1,
                     0.5 * (rho0 / rho_in + 1.0),
                     0.5 * (rho0 / rho_out + rho0 / rho_in))
    # self-term of the single layer on the equal-volume sphere
    a_eq = (3.0 * w / (4.0 * math.pi)) ** (1.0 / 3.0)
    D_vol = (b_cells - k0 ** 2 * a_cells) * ball_centre_integral(a_eq, k0)
    return Discretisation(
        k0=float(k0), n_vol=mesh.n_vol, n_srf=mesh.n_srf, pts=mesh.points(),
        sV=sV, gT=gT, nrm=np.asarray(mesh.srf_n, dtype=np.float64), dK=dK,
        m=np.concatenate([m_vol, m_srf]).astype(np.complex128),
        D=np.concatenate([D_vol, np.zeros(mesh.n_srf, np.complex128)]))


def _src_args(d: Discretisation):
    P = d.pts
    return dict(px=_c(P[:, 0]), py=_c(P[:, 1]), pz=_c(P[:, 2]), sV=_c(d.sV),
                gx=_c(d.gT[:, 0]), gy=_c(d.gT[:, 1]), gz=_c(d.gT[:, 2]),
                nx=_c(d.nrm[:, 0]), ny=_c(d.nrm[:, 1]), nz=_c(d.nrm[:, 2]), dK=_c(d.dK))


def _as_cols(x, n):
    x = np.asarray(x, dtype=np.complex128)
    one = x.ndim == 1
    x2 = x.reshape(n, -1, order="F") if not one else x.reshape(n, 1)
    return np.asfortranarray(x2), one


def offdiag_apply(d: Discretisation, x, rows=None, targets=None, exclude_self=True):
    """sum_j kappa(t_i, j) x_j over sources j (j != i for collocation targets)."""
    X, one = _as_cols(x, d.n)
    T = d.pts if targets is None else np.asarray(targets, dtype=np.float64)
    rr = None if rows is None else _c(rows, np.int64)
    nt = T.shape[0] if rr is None else rr.size
    out = np.zeros((nt, X.shape[1]), dtype=np.complex128, order="F")
    a = _src_args(d)
    tx, ty, tz = _c(T[:, 0]), _c(T[:, 1]), _c(T[:, 2])
    _lib().vo_apply(T.shape[0], _p(tx), _p(ty), _p(tz), _p(rr), 0 if rr is None else rr.size,
                    d.n_vol, d.n, _p(a["px"]), _p(a["py"]), _p(a["pz"]), _p(a["sV"]),
                    _p(a["gx"]), _p(a["gy"]), _p(a["gz"]), _p(a["nx"]), _p(a["ny"]),
                    _p(a["nz"]), _p(a["dK"]), d.k0, 1 if exclude_self else 0, X.shape[1],
                    _p(X), _p(out))
    return out[:, 0] if one else out


def matvec(d: Discretisation, x, rows=None):
    """(A x)_i = (m_i - D_i) x_i + sum_{j != i} kappa_ij x_j, optionally on selected rows."""
    X, one = _as_cols(x, d.n)
    off = offdiag_apply(d, X, rows=rows)
    if off.ndim == 1:
        off = off[:, None]
    idx = np.arange(d.n) if rows is None else np.asarray(rows, dtype=np.int64)
    y = d.diag[idx, None] * X[idx, :] + off
    return y[:, 0] if one else y


def adjoint_matvec(d: Discretisation, lam):
    """(A^H lam)_j = sum_i conj(A_ij) lam_i, from the definition."""
    L, one = _as_cols(lam, d.n)
    out = np.zeros((d.n, L.shape[1]), dtype=np.complex128, order="F")
    a = _src_args(d)
    _lib().vo_apply_adjoint(d.n, _p(a["px"]), _p(a["py"]), _p(a["pz"]), d.n_vol, d.n,
                            _p(a["px"]), _p(a["py"]), _p(a["pz"]), _p(a["sV"]), _p(a["gx"]),
                            _p(a["gy"]), _p(a["gz"]), _p(a["nx"]), _p(a["ny"]), _p(a["nz"]),
                            _p(a["dK"]), d.k0, 1, L.shape[1], _p(L), _p(out))
    y = np.conj(d.diag)[:, None] * L + out
    return y[:, 0] if one else y


def source_sums(d: Discretisation, lam, targets=None, exclude_self=True):
    """z_j = sum_i conj(G_ij) lam_i and Z_j = sum_i conj(F_ij)(t_i - y_j) lam_i.
    Returns z (n, R) and Z (n, 3, R)."""
    T = d.pts if targets is None else np.asarray(targets, dtype=np.float64)
    L, one = _as_cols(lam, T.shape[0])
    R = L.shape[1]
    z = np.zeros((d.n, R), dtype=np.complex128, order="F")
    Z = np.zeros((d.n, 3 * R), dtype=np.complex128, order="F")
    a = _src_args(d)
    tx, ty, tz = _c(T[:, 0]), _c(T[:, 1]), _c(T[:, 2])
    _lib().vo_source_sums(T.shape[0], _p(tx), _p(ty), _p(tz), d.n, _p(a["px"]), _p(a["py"]),
                          _p(a["pz"]), d.k0, 1 if exclude_self else 0, R, _p(L), _p(z), _p(Z))
    # columns are ordered (rhs c, axis a) -> 3 c + a
    Z = np.stack([Z[:, 3 * c:3 * c + 3] for c in range(R)], axis=2)
    return z, Z


def assemble(d: Discretisation):
    """Dense A (n x n complex128) with the diagonal m - D."""
    n = d.n
    A = np.zeros((n, n), dtype=np.complex128)
    a = _src_args(d)
    _lib().vo_assemble(d.n_vol, n, _p(a["px"]), _p(a["py"]), _p(a["pz"]), _p(a["sV"]),
                       _p(a["gx"]), _p(a["gy"]), _p(a["gz"]), _p(a["nx"]), _p(a["ny"]),
                       _p(a["nz"]), _p(a["dK"]), d.k0, _p(A))
    A[np.arange(n), np.arange(n)] = d.diag
    return A


# ---------------------------------------------------------------------------
# incident field, representation formula, errors

def plane_wave(points, k0, direction):
    """p_inc(x) = exp(i k0 x . d) (eq_planewave); (n,) or (n, R) for R directions."""
    P = np.asarray(points, dtype=np.float64)
    D = np.atleast_2d(np.asarray(direction, dtype=np.float64))
    out = np.exp(1j * k0 * (P @ D.T))
    return out[:, 0] if np.ndim(direction) == 1 else out


def exterior_field(d: Discretisation, targets, p, direction):
    """p(x) = p_inc(x) - sum_j kappa(x, j) p_j for x in Omega_0 (eq_vsie with m = 1)."""
    T = np.asarray(targets, dtype=np.float64)
    return plane_wave(T, d.k0, direction) - offdiag_apply(d, p, targets=T, exclude_self=False)


def far_field(d: Discretisation, directions, p):
    """Far-field pattern of the scattered field p_sc = p - p_inc in Omega_0:
    p_sc(R xhat) = exp(i k0 R)/R pinf(xhat) + O(R^-2) for unit directions xhat.

    The representation formula of section 2.3.1 (the exterior field above,
    -sum_j kappa(x, j) p_j) with the kernels replaced by their leading terms
    at |x| = R -> infinity:
        G(x, y)      ~ exp(i k0 R)/(4 pi R) exp(-i k0 xhat . y)
        grad_x G     ~  i k0 xhat G,     grad_y G ~ -i k0 xhat G.
    Cell j (kappa = -G sV + grad_x G . gT) and face j (kappa = dK grad_y G . n)
    then give
        pinf(xhat) = 1/(4 pi) sum_j exp(-i k0 xhat . y_j) a_j(xhat) p_j,
        a_j = sV_j - i k0 xhat . gT_j   (cells),   a_j = i k0 dK_j xhat . n_j   (faces).
    directions: (m, 3) unit vectors; p: (n,) or (n, R).  Returns (m,) or (m, R)."""
    X = np.atleast_2d(np.asarray(directions, dtype=np.float64))
    P, one = _as_cols(p, d.n)
    out = np.zeros((X.shape[0], P.shape[1]), dtype=np.complex128)
    nv = d.n_vol
    for a in range(0, X.shape[0], 256):
        Xb = X[a:a + 256]
        E = np.exp(-1j * d.k0 * (Xb @ d.pts.T))
        amp = np.empty(E.shape, dtype=np.complex128)
        amp[:, :nv] = d.sV[None, :] - 1j * d.k0 * (Xb @ d.gT.T)
        amp[:, nv:] = 1j * d.k0 * (Xb @ d.nrm.T) * d.dK[None, :]
        out[a:a + 256] = (E * amp) @ P / (4.0 * math.pi)
    return out[:, 0] if one else out


def rel_error(num, ref, ord=2):
    """E_rel = ||num - ref|| / ||ref|| (eq_error), 2-norm or max-norm over all entries."""
    num = np.ravel(num)
    ref = np.ravel(ref)
    if ord == np.inf:
        return float(np.max(np.abs(num - ref)) / np.max(np.abs(ref)))
    return float(np.linalg.norm(num - ref) / np.linalg.norm(ref))


# ---------------------------------------------------------------------------
# solvers

def solve_lu(d: Discretisation, b):
    import scipy.linalg as sla
    A = assemble(d)
    return sla.lu_solve(sla.lu_factor(A), b)


def gmres(apply, b, tol=1e-12, restart=200, maxiter=2000, x0=None, callback=None):
    """Restarted GMRES(m) with modified Gram-Schmidt Arnoldi and Givens rotations.
    Stops when ||b - A x|| <= tol ||b||.  Returns (x, iterations, rel. residual)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    x = np.zeros(n, np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    it = 0
    r = b - apply(x) if x0 is not None else b.copy()
    beta_ = np.linalg.norm(r)
    while it < maxiter and beta_ > tol * bnorm:
        m = min(restart, maxiter - it)
        V = np.zeros((n, m + 1), np.complex128)
        H = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m, np.complex128)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta_
        V[:, 0] = r / beta_
        k_done = 0
        for k in range(m):
            w = apply(V[:, k])
            for j in range(k + 1):
                H[j, k] = np.vdot(V[:, j], w)
                w = w - H[j, k] * V[:, j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0:
                V[:, k + 1] = w / H[k + 1, k]
            # unitary rotations [[conj(c), conj(s)], [-s, c]] with c = a/rho, s = b/rho
            # map (a, b) to (rho, 0); the same rotation acts on later columns and on g
            for j in range(k):
                t = np.conj(cs[j]) * H[j, k] + np.conj(sn[j]) * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            den = math.hypot(abs(H[k, k]), abs(H[k + 1, k]))
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0
            g[k + 1] = -sn[k] * g[k]
            g[k] = np.conj(cs[k]) * g[k]
            it += 1
            k_done = k + 1
            if callback:
                callback(it, abs(g[k + 1]) / bnorm)
            if abs(g[k + 1]) <= tol * bnorm:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + V[:, :k_done] @ y
        r = b - apply(x)
        beta_ = np.linalg.norm(r)
    return x, it, float(beta_ / bnorm)


def solve_gmres(d: Discretisation, b, tol=1e-12, restart=200, maxiter=3000, callback=None):
    return gmres(lambda v: matvec(d, v), b, tol=tol, restart=restart, maxiter=maxiter,
                 callback=callback)


# ---------------------------------------------------------------------------
# receiver misfit (for finite-difference checks of adjoint gradients)

def receiver_pressures(mesh, mat, k0, dirs, receivers, grad_rho=None):
    """p_rec (n_rec, Q) for the plane waves `dirs` (Q, 3): dense LU solve of the
    collocation system, then the representation formula at the receivers.
    grad_rho: analytic density gradient per cell (held fixed), or None."""
    d = discretise(mesh, mat, k0, grad_rho=grad_rho)
    D = np.atleast_2d(dirs)
    P = solve_lu(d, plane_wave(d.pts, k0, D))
    return exterior_field(d, receivers, P, D)


def receiver_misfit(mesh, mat, k0, dirs, receivers, data, grad_rho=None):
    """J = 1/2 sum |p_rec - data|^2 over receivers and incidences."""
    pr = receiver_pressures(mesh, mat, k0, dirs, receivers, grad_rho)
    return 0.5 * float(np.sum(np.abs(pr - data) ** 2))
