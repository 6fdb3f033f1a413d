"""Pins of the FP64 oracle against mathematics it does not share code with.

Each test fixes part of the oracle to something other than itself: high
precision evaluations (mpmath), numerical integration (scipy), closed forms
(ball potentials), the layered-sphere series solution, algebraic special cases
of the paper's VSIE (Theorem 3 and the remarks that follow it) and invariants.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

import oracle as O
import oracle.analytic as A
import workloads as W


# ---------------------------------------------------------------------------
# helpers

def _tiny_disc(k0, pts_vol, sV=None, gT=None, pts_srf=(), nrm=(), dK=()):
    pts_vol = np.asarray(pts_vol, dtype=np.float64).reshape(-1, 3)
    pts_srf = np.asarray(pts_srf, dtype=np.float64).reshape(-1, 3)
    nv, ns = pts_vol.shape[0], pts_srf.shape[0]
    return O.Discretisation(
        k0=k0, n_vol=nv, n_srf=ns, pts=np.concatenate([pts_vol, pts_srf]),
        sV=np.zeros(nv) if sV is None else np.asarray(sV, dtype=np.float64),
        gT=np.zeros((nv, 3)) if gT is None else np.asarray(gT, dtype=np.float64).reshape(nv, 3),
        nrm=np.asarray(nrm, dtype=np.float64).reshape(ns, 3),
        dK=np.asarray(dK, dtype=np.float64).reshape(ns),
        m=np.ones(nv + ns, np.complex128), D=np.zeros(nv + ns, np.complex128))


def _kappa(d, target):
    return O.offdiag_apply(d, np.ones(d.n), targets=np.asarray([target], float),
                           exclude_self=False)[0]


def _mp_G(k, x, y):
    r = mp.sqrt(sum((mp.mpf(a) - mp.mpf(b)) ** 2 for a, b in zip(x, y)))
    return mp.exp(1j * k * r) / (4 * mp.pi * r)


# ---------------------------------------------------------------------------
# kernel values against 30-digit arithmetic and numerical differentiation

@pytest.mark.parametrize("k0,x,y", [
    (2.0, (0.3, -0.2, 0.1), (0.0, 0.05, -0.4)),
    (10.0, (0.9, 0.1, -0.3), (-0.6, 0.2, 0.5)),
    (40.0, (0.01, 0.02, 0.03), (0.0, 0.0, 0.0)),
])
def test_green_and_gradients_vs_mpmath(k0, x, y):
    mp.mp.dps = 30
    # single layer: a volume source with sV = -1 gives G(x, y)
    d = _tiny_disc(k0, [y], sV=[-1.0])
    g_ref = complex(_mp_G(k0, x, y))
    assert abs(_kappa(d, x) - g_ref) <= 1e-14 * abs(g_ref)
    # adjoint double layer: grad_x G . e_a for a unit grad-alpha weight
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0
        d = _tiny_disc(k0, [y], sV=[0.0], gT=[e])

        def Gx(t, a=a):
            xx = list(x)
            xx[a] = mp.mpf(x[a]) + t
            return _mp_G(k0, xx, y)
        ref = complex(mp.diff(Gx, 0))
        assert abs(_kappa(d, x) - ref) <= 1e-12 * abs(ref) + 1e-300
    # double layer: dG/dn_y for a face through y with normal n and unit weight
    n = np.array([0.36, -0.48, 0.8])
    d = _tiny_disc(k0, np.zeros((0, 3)), pts_srf=[y], nrm=[n], dK=[1.0])

    def Gn(t):
        yy = [mp.mpf(y[i]) + t * mp.mpf(n[i]) for i in range(3)]
        return _mp_G(k0, x, yy)
    ref = complex(mp.diff(Gn, 0))
    assert abs(_kappa(d, x) - ref) <= 1e-12 * abs(ref)


# ---------------------------------------------------------------------------
# self-term on the equal-volume sphere

@pytest.mark.parametrize("a,k", [(3e-5, 1.0), (0.01, 2.0), (0.0258, 10.0), (0.04, 16.0),
                                 (0.2, 2.0), (0.45, 1.0), (0.6, 1.0), (0.3, 3.0), (1.0, 5.0)])
def test_self_term_vs_quadrature(a, k):
    # integral over the ball of G(0, y) in spherical coordinates, done numerically
    mp.mp.dps = 30
    ref = complex(mp.quad(lambda r: 4 * mp.pi * r ** 2 * mp.exp(1j * k * r) / (4 * mp.pi * r), [0, a]))
    got = O.ball_centre_integral(np.array([a]), k)[0]
    assert abs(got - ref) <= 1e-14 * abs(ref)


# ---------------------------------------------------------------------------
# worked per-element weights of the c0 medium, derived by hand from the paper's
# definitions: (rho0/rho)((omega/c)^2 - k0^2) and the mass function

def test_worked_weights_config0():
    mesh, mat, k0s, _, _ = W.config_problem("c0")
    d = O.discretise(mesh, mat, k0s[0])
    w = mesh.vol_w
    om1 = mesh.vol_dom == 1
    # omega = k0 c0 = 2: Omega_1 (rho 1.2, c 1.5), Omega_2 (rho 2, c 0.8)
    assert np.allclose(d.sV[om1] / w[om1], (1 / 1.2) * ((2 / 1.5) ** 2 - 4), rtol=1e-14)
    assert np.allclose(d.sV[~om1] / w[~om1], (1 / 2.0) * ((2 / 0.8) ** 2 - 4), rtol=1e-14)
    assert np.allclose(d.sV[om1] / w[om1], -1.8518518518518519, rtol=1e-14)
    assert np.allclose(d.sV[~om1] / w[~om1], 1.125, rtol=1e-14)
    mv = d.m[:mesh.n_vol].real
    ms = d.m[mesh.n_vol:].real
    assert np.allclose(mv[om1], 1 / 1.2) and np.allclose(mv[~om1], 0.5)
    g1 = mesh.srf_iface == 1
    assert np.allclose(ms[g1], 0.5 * (1 / 1.2 + 1)) and np.allclose(ms[~g1], 0.5 * (1 / 1.2 + 0.5))
    jump = d.dK / mesh.srf_area
    assert np.allclose(jump[g1], 1 / 1.2 - 1) and np.allclose(jump[~g1], (0.5 - 1) - (1 / 1.2 - 1))
    assert np.all(d.gT == 0.0)          # piecewise constant density: T vanishes


# ---------------------------------------------------------------------------
# special cases of the VSIE

def test_homogeneous_medium_gives_identity():
    mesh = W.nested_balls(8)
    mat = W.materials_piecewise(mesh, 1.3, 0.7, 1.3, 0.7, 1.3, 0.7)
    d = O.discretise(mesh, mat, 3.0)
    Amat = O.assemble(d)
    assert np.array_equal(Amat, np.eye(d.n, dtype=np.complex128))


def test_continuous_density_removes_surface_terms():
    mesh = W.nested_balls(8)
    d = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 1.0, 1.5, 1.0, 0.8), 2.0)
    assert np.all(d.dK == 0.0) and np.all(d.gT == 0.0)
    assert np.all(d.m == 1.0)
    # equal densities on both sides of Gamma_2 only: Gamma_2 weights vanish, Gamma_1 do not
    d = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 1.7, 1.5, 1.7, 0.8), 2.0)
    g2 = mesh.srf_iface == 2
    assert np.all(d.dK[g2] == 0.0) and np.all(d.dK[~g2] != 0.0)


def test_single_domain_reduction():
    """With the same material in Omega_2 as in Omega_1, the nested system must
    give the single-domain solution on the volume cells: the Gamma_2 unknowns
    decouple because their weight is alpha_2 - alpha_1 = 0."""
    mesh = W.nested_balls(8)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.4, 1.3, 1.4, 1.3)
    d = O.discretise(mesh, mat, 2.0)
    b = O.plane_wave(d.pts, 2.0, [0.0, 0.6, 0.8])
    p = O.solve_lu(d, b)
    g1 = np.concatenate([np.ones(mesh.n_vol, bool), mesh.srf_iface == 1])
    # single domain: drop the Gamma_2 elements altogether
    sub = O.Discretisation(k0=d.k0, n_vol=d.n_vol, n_srf=int(np.sum(mesh.srf_iface == 1)),
                           pts=d.pts[g1], sV=d.sV, gT=d.gT, nrm=d.nrm[mesh.srf_iface == 1],
                           dK=d.dK[mesh.srf_iface == 1], m=d.m[g1], D=d.D[g1])
    p1 = O.solve_lu(sub, b[g1])
    assert O.rel_error(p[g1], p1) < 1e-13


def test_lippmann_schwinger_symmetry():
    """Constant density (alpha = 0): off-diagonal A_ij = -G(r_ij) sV_j, so
    A_ij / sV_j is symmetric in (i, j)."""
    mesh = W.nested_balls(8)
    d = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 1.0, 1.5, 1.0, 0.8), 2.0)
    Amat = O.assemble(d)[:d.n_vol, :d.n_vol]
    np.fill_diagonal(Amat, 0)
    B = Amat / d.sV[None, :]
    assert np.max(np.abs(B - B.T)) <= 1e-14 * np.max(np.abs(B))
    # and the surface columns vanish
    assert np.all(O.assemble(d)[:, d.n_vol:] == np.eye(d.n)[:, d.n_vol:])


def _lognormal_small(N=8):
    mesh = W.nested_balls(N)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8)
    mat.vol_c = mat.vol_c * W.lognormal_voxel_field(mesh.vol_xyz, -1, 1, 32, 0.1, 0)
    mat.vol_rho = mat.vol_rho * W.lognormal_voxel_field(mesh.vol_xyz, -1, 1, 32, 0.1, 1)
    return mesh, mat


def test_adjoint_dot_product():
    mesh, mat = _lognormal_small()
    d = O.discretise(mesh, mat, 3.0)
    assert np.any(d.gT != 0)
    x = W.seeded_complex((d.n, 2), seed=1)
    y = W.seeded_complex((d.n, 2), seed=2)
    lhs = np.vdot(y, O.matvec(d, x))
    rhs = np.vdot(O.adjoint_matvec(d, y), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_source_sums_reproduce_adjoint():
    """(A^H lam)_j = conj(A_jj) lam_j - s_j z_j + v_j . Z_j with s_j = sV_j and
    v_j = gT_j on cells, s_j = 0 and v_j = -dK_j n_j on faces."""
    mesh, mat = _lognormal_small()
    d = O.discretise(mesh, mat, 3.0)
    lam = W.seeded_complex(d.n, seed=3)
    z, Z = O.source_sums(d, lam)
    z, Z = z[:, 0], Z[:, :, 0]
    s = np.concatenate([d.sV, np.zeros(d.n_srf)])
    v = np.concatenate([d.gT, -d.dK[:, None] * d.nrm])
    got = np.conj(d.diag) * lam - s * z + np.sum(v * Z, axis=1)
    assert O.rel_error(got, O.adjoint_matvec(d, lam)) < 1e-13


def test_translation_and_axis_permutation_invariance():
    mesh, mat = _lognormal_small()
    d = O.discretise(mesh, mat, 3.0)
    A0 = O.assemble(d)
    shifted = O.Discretisation(**{**d.__dict__, "pts": d.pts + np.array([0.3, -1.7, 2.2])})
    assert np.max(np.abs(O.assemble(shifted) - A0)) <= 1e-12 * np.max(np.abs(A0))
    # plane wave picks up the phase exp(i k0 d.t)
    t = np.array([0.3, -1.7, 2.2])
    dd = np.array([0.0, 0.6, 0.8])
    ratio = O.plane_wave(d.pts + t, 3.0, dd) / O.plane_wave(d.pts, 3.0, dd)
    assert np.allclose(ratio, np.exp(3j * dd @ t), rtol=1e-12)
    # rotating coordinates (x, y, z) -> (y, z, x) permutes nothing in A
    perm = O.Discretisation(**{**d.__dict__, "pts": d.pts[:, [1, 2, 0]],
                               "gT": d.gT[:, [1, 2, 0]], "nrm": d.nrm[:, [1, 2, 0]]})
    assert np.max(np.abs(O.assemble(perm) - A0)) <= 1e-12 * np.max(np.abs(A0))


# ---------------------------------------------------------------------------
# midpoint entries against the exact element integrals (brute force)

@pytest.mark.parametrize("h", [0.2, 0.1, 0.05])
def test_volume_entry_vs_exact_cell_integral(h):
    k0 = 3.0
    y = np.array([0.0, 0.0, 0.0])
    x = np.array([0.41, 0.23, -0.17])
    d = _tiny_disc(k0, [y], sV=[-h ** 3])          # -G * sV = G |cell|
    mid = _kappa(d, x)

    def f(zz, yy, xx, part):
        r = math.sqrt((x[0] - xx) ** 2 + (x[1] - yy) ** 2 + (x[2] - zz) ** 2)
        v = np.exp(1j * k0 * r) / (4 * math.pi * r)
        return v.real if part == 0 else v.imag
    ex = [integrate.tplquad(f, -h / 2, h / 2, -h / 2, h / 2, -h / 2, h / 2, args=(p,),
                            epsabs=1e-13, epsrel=1e-11)[0] for p in (0, 1)]
    exact = ex[0] + 1j * ex[1]
    r = np.linalg.norm(x - y)
    assert abs(mid - exact) <= 0.1 * (h / r) ** 2 * abs(exact)


@pytest.mark.parametrize("h", [0.2, 0.1, 0.05])
def test_surface_entry_vs_exact_face_integral(h):
    k0 = 3.0
    y = np.array([0.0, 0.0, 0.0])
    n = np.array([0.0, 0.0, 1.0])
    x = np.array([0.31, -0.12, 0.27])
    d = _tiny_disc(k0, np.zeros((0, 3)), pts_srf=[y], nrm=[n], dK=[h * h])
    mid = _kappa(d, x)

    def f(yy, xx, part):
        dv = x - np.array([xx, yy, 0.0])
        r = np.linalg.norm(dv)
        # dG/dn_y for n = +z: d/dy_z of exp(ikr)/(4 pi r) with r = |x - y|
        dGdr = np.exp(1j * k0 * r) * (1j * k0 * r - 1) / (4 * math.pi * r ** 2)
        v = dGdr * (-(dv[2]) / r)
        return v.real if part == 0 else v.imag
    ex = [integrate.dblquad(f, -h / 2, h / 2, -h / 2, h / 2, args=(p,), epsabs=1e-13,
                            epsrel=1e-11)[0] for p in (0, 1)]
    exact = ex[0] + 1j * ex[1]
    r = np.linalg.norm(x - y)
    assert abs(mid - exact) <= 0.2 * (h / r) ** 2 * abs(exact)


# ---------------------------------------------------------------------------
# closed forms on a ball

def test_ball_potential_closed_form_vs_quadrature():
    """u(r) = int_0^R rho^2 (e^{ik(r+rho)} - e^{ik|r-rho|}) / (2 i k r rho) drho."""
    R, k = 0.8, 3.0
    for r in (0.1, 0.5, 0.79, 1.3, 2.5):
        def f(rho):
            return rho ** 2 * (mp.exp(1j * k * (r + rho)) - mp.exp(1j * k * abs(r - rho))) / (
                2j * k * r * rho)
        mp.mp.dps = 25
        ref = complex(mp.quad(f, [0, min(r, R), R] if r < R else [0, R]))
        got = A.ball_potential(np.array([[r, 0, 0]]), R, k)[0]
        assert abs(got - ref) <= 1e-12 * abs(ref)
    # centre value is the self-term, gradient by central differences
    assert abs(A.ball_potential(np.zeros((1, 3)), R, k)[0]
               - O.ball_centre_integral(np.array([R]), k)[0]) < 1e-14
    x = np.array([[0.2, -0.3, 0.1]])
    eps = 1e-6
    g = [(A.ball_potential(x + eps * e, R, k) - A.ball_potential(x - eps * e, R, k))[0] / (2 * eps)
         for e in np.eye(3)]
    assert np.allclose(g, A.ball_potential_grad_inside(x, R, k)[0], rtol=1e-7, atol=1e-9)


def _ball_errors(kind, Ns=(8, 12, 16)):
    errs = []
    k0 = 2.5
    for N in Ns:
        mesh = W.nested_balls(N, R1=1.0, R2=0.0)
        Re = (3 * mesh.vol_w.sum() / (4 * math.pi)) ** (1 / 3)
        inner = np.linalg.norm(mesh.vol_xyz, axis=1) < 0.6
        if kind == "V":
            # rho = rho0 and (k^2 - k0^2) = -1: sV = -|cell|, so (A 1)_i - 1 = V[1](x_i)
            c = k0 / math.sqrt(k0 ** 2 - 1.0)
            d = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 1.0, c, 1.0, c), k0)
            got = O.matvec(d, np.ones(d.n))[:mesh.n_vol] - 1.0
            ref = A.ball_potential(mesh.vol_xyz, Re, k0)
        else:
            # c = c0, rho = rho0 with a prescribed constant grad alpha = g:
            # (A 1)_i - 1 = g . grad u(x_i)
            g = np.array([0.3, -0.5, 0.7])
            d = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0), k0,
                             grad_alpha=np.tile(g, (mesh.n_vol, 1)))
            got = O.matvec(d, np.ones(d.n))[:mesh.n_vol] - 1.0
            ref = A.ball_potential_grad_inside(mesh.vol_xyz, Re, k0) @ g
        errs.append(O.rel_error(got[inner], ref[inner]))
    return errs


def test_single_layer_matches_ball_potential():
    e = _ball_errors("V")
    assert e[-1] < 0.01 and e[0] > e[1] > e[2], e


def test_adjoint_double_layer_matches_ball_potential_gradient():
    e = _ball_errors("T")
    assert e[-1] < 0.05 and e[0] > e[2], e


def test_double_layer_green_identity():
    """For x inside a domain D: int_{dD} dG/dn_y dS = -1 - k^2 int_D G dy.  The
    staircase ball is such a domain, so on the same mesh the discrete K[1]
    must approach -1 - k^2 V[1] at interior points as the grid is refined."""
    k0 = 2.0
    errs = []
    for N in (8, 12, 16, 24):
        mesh = W.nested_balls(N, R1=1.0, R2=0.0)
        inner = np.linalg.norm(mesh.vol_xyz, axis=1) < 0.5
        # K only: c = c0 (no V), rho1 = rho0 / 2 -> alpha_1 = 1 on Gamma_1
        dK = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 0.5, 1.0, 0.5, 1.0), k0)
        dK.gT[:] = 0.0
        K1 = O.offdiag_apply(dK, np.concatenate([np.zeros(mesh.n_vol), np.ones(mesh.n_srf)]))
        # V[1] on the same cells
        c = k0 / math.sqrt(k0 ** 2 - 1.0)
        dV = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 1.0, c, 1.0, c), k0)
        V1 = O.matvec(dV, np.ones(dV.n))[:mesh.n_vol] - 1.0
        lhs = K1[:mesh.n_vol][inner]
        rhs = -1.0 - k0 ** 2 * V1[inner]
        errs.append(O.rel_error(lhs, rhs))
    assert errs[-1] < 0.01 and errs[0] > errs[-1], errs


# ---------------------------------------------------------------------------
# the layered-sphere series solution itself

def test_mie_series_satisfies_the_transmission_problem():
    k0, rho, c = 2.0, (1.0, 1.2, 2.0), (1.0, 1.5, 0.8)
    R1, R2 = 1.0, 0.5
    d = np.array([0.0, 0.0, 1.0])

    def p(P):
        return A.mie_layered(P, d, k0, rho[0], c[0], R1, rho[1], c[1], R2, rho[2], c[2])
    xhat = np.array([0.48, 0.6, 0.64])
    eps = 1e-5
    for R, ri, ro in ((R1, rho[1], rho[0]), (R2, rho[2], rho[1])):
        pin, pout = p([(R - eps) * xhat])[0], p([(R + eps) * xhat])[0]
        assert abs(pin - pout) < 1e-4 * abs(pin)
        h = 1e-4
        din = (p([(R - eps) * xhat])[0] - p([(R - eps - h) * xhat])[0]) / h
        dout = (p([(R + eps + h) * xhat])[0] - p([(R + eps) * xhat])[0]) / h
        assert abs(din / ri - dout / ro) < 2e-3 * abs(din / ri)
    # Helmholtz equation with the local wavenumber, by a 7-point Laplacian
    hh = 1e-3
    for x0, cj in (([0.1, 0.2, 0.15], c[2]), ([0.5, 0.4, 0.3], c[1]), ([1.2, -0.4, 0.5], c[0])):
        x0 = np.array(x0)
        pts = [x0] + [x0 + s * hh * e for e in np.eye(3) for s in (1, -1)]
        v = p(np.array(pts))
        lap = (np.sum(v[1:]) - 6 * v[0]) / hh ** 2
        k = k0 * c[0] / cj
        assert abs(lap + k ** 2 * v[0]) < 1e-4 * k ** 2 * abs(v[0])
    # no scatterer: plane wave
    P = np.random.default_rng(0).uniform(-1.5, 1.5, (20, 3))
    pw = A.mie_layered(P, d, k0, 1.0, 1.0, R1, 1.0, 1.0, R2, 1.0, 1.0)
    assert np.allclose(pw, np.exp(1j * k0 * P @ d), atol=1e-12)


# ---------------------------------------------------------------------------
# the whole oracle operator + solve against the series solution

def _mie_case(N, rho1, rho2):
    mesh = W.nested_balls(N)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, rho1, 1.5, rho2, 0.8)
    k0 = 2.0
    d = O.discretise(mesh, mat, k0)
    p = O.solve_lu(d, O.plane_wave(d.pts, k0, [0, 0, 1.0]))
    # compare against spheres of the staircase volumes
    R1e = (3 * mesh.vol_w.sum() / (4 * math.pi)) ** (1 / 3)
    R2e = (3 * mesh.vol_w[mesh.vol_dom == 2].sum() / (4 * math.pi)) ** (1 / 3)
    args = (k0, 1.0, 1.0, R1e, rho1, 1.5, R2e, rho2, 0.8)
    vol = O.rel_error(p[:mesh.n_vol], A.mie_layered(mesh.vol_xyz, [0, 0, 1.0], *args))
    ext_pts = W.fibonacci_sphere(200, 2.0)
    ext = O.rel_error(O.exterior_field(d, ext_pts, p, [0, 0, 1.0]),
                      A.mie_layered(ext_pts, [0, 0, 1.0], *args))
    return vol, ext


def test_lippmann_schwinger_case_converges_to_mie():
    errs = [_mie_case(N, 1.0, 1.0) for N in (8, 12, 16)]
    vol = [e[0] for e in errs]
    assert vol[0] > vol[1] > vol[2] and vol[2] < 2e-3, errs
    assert all(e[1] < 1e-3 for e in errs), errs


def test_density_jump_case_converges_to_mie():
    errs = [_mie_case(N, 1.2, 2.0) for N in (8, 12, 16)]
    vol = [e[0] for e in errs]
    ext = [e[1] for e in errs]
    assert vol[0] > vol[1] > vol[2] and vol[2] < 0.09, errs
    assert ext[0] > ext[1] > ext[2] and ext[2] < 3e-3, errs


def test_gmres_matches_lu():
    mesh, mat, k0s, dirs, _ = W.config_problem("c0", N=12)
    d = O.discretise(mesh, mat, k0s[0])
    b = O.plane_wave(d.pts, k0s[0], dirs[0])
    p_lu = O.solve_lu(d, b)
    p_gm, it, res = O.solve_gmres(d, b, tol=1e-12)
    assert res <= 1e-12 and O.rel_error(p_gm, p_lu) < 1e-10


def test_gmres_single_cycle_on_random_complex_system():
    """One GMRES cycle on a random complex system: the Givens residual estimate
    must equal the true residual of the returned iterate (exact arithmetic
    identity of GMRES), and the solve must agree with a dense solve."""
    rng = np.random.default_rng(5)
    n = 80
    Am = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    est = []
    x, it, res = O.gmres(lambda v: Am @ v, b, tol=1e-12, restart=200,
                         callback=lambda i, r: est.append(r))
    assert it == len(est) and res <= 1e-12
    assert abs(est[-1] - res) <= 1e-12
    assert np.linalg.norm(x - np.linalg.solve(Am, b)) <= 1e-10 * np.linalg.norm(x)
    # a truncated single cycle: estimate and true residual agree too
    est = []
    x5, it5, res5 = O.gmres(lambda v: Am @ v, b, tol=1e-30, restart=15, maxiter=15,
                            callback=lambda i, r: est.append(r))
    assert it5 == 15 and abs(est[-1] - res5) <= 1e-12 * max(1.0, res5) + 1e-14
