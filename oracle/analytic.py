"""Closed-form references for pinning the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* Newton potential of a constant unit source on a ball, u(x) = int_B G_k(x,y) dy,
  and its gradient inside the ball (used to pin the single-layer V block and
  the adjoint-double-layer T block of the discretised operator).
* Scattering of a plane wave by two concentric homogeneous spheres: the
  spherical-harmonic series solution the paper compares against in its
  first benchmark (section 3.2), written here for the nested case with
  transmission conditions p and (1/rho) dp/dr continuous (eqs.
  eq_transmission_pressure, eq_transmission_velocity) and the outgoing
  radiation condition (eq_sommerfeld), time convention exp(-i omega t).
* The far-field pattern of that series: the leading term of the exterior
  scattered field as r -> infinity.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special as sp


def ball_potential(x, R, k):
    """u(x) = int_{|y|<R} exp(i k |x-y|)/(4 pi |x-y|) dy for points x (n, 3)."""
    r = np.sqrt(np.sum(np.asarray(x, dtype=np.float64) ** 2, axis=-1))
    out = np.empty(r.shape, dtype=np.complex128)
    inside = r < R
    ri = r[inside]
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(ri > 0, np.sin(k * ri) / np.where(ri > 0, k * ri, 1.0), 1.0)
    out[inside] = ((1 - 1j * k * R) * np.exp(1j * k * R) * sinc - 1.0) / k ** 2
    ro = r[~inside]
    out[~inside] = np.exp(1j * k * ro) * (math.sin(k * R) - k * R * math.cos(k * R)) / (k ** 3 * ro)
    return out


def ball_potential_grad_inside(x, R, k):
    """grad u inside the ball: -(1 - i k R) exp(i k R) / k * j1(k r) * x/r."""
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(np.sum(x ** 2, axis=-1))
    amp = -(1 - 1j * k * R) * np.exp(1j * k * R) / k * sp.spherical_jn(1, k * r)
    with np.errstate(invalid="ignore", divide="ignore"):
        xhat = np.where(r[:, None] > 0, x / np.where(r > 0, r, 1.0)[:, None], 0.0)
    return amp[:, None] * xhat


def mie_truncation(kR: float) -> int:
    """Series length: ceil(kR + 4 (kR)^(1/3)) + 10 terms beyond n = 0."""
    return int(math.ceil(kR + 4.0 * kR ** (1.0 / 3.0))) + 10


def mie_coefficients(k0, rho0, k1, rho1, R1, k2, rho2, R2, nmax):
    """Per-degree coefficients (A_n, B_n, C_n, D_n) of

        p0 = sum i^n (2n+1) [j_n(k0 r) + A_n h_n(k0 r)] P_n      r > R1
        p1 = sum i^n (2n+1) [B_n j_n(k1 r) + C_n y_n(k1 r)] P_n  R2 < r < R1
        p2 = sum i^n (2n+1) D_n j_n(k2 r) P_n                    r < R2

    from continuity of p and of (1/rho) dp/dr at r = R1 and r = R2."""
    coef = np.zeros((nmax + 1, 4), dtype=np.complex128)
    for n in range(nmax + 1):
        ja, dja = sp.spherical_jn(n, k0 * R1), sp.spherical_jn(n, k0 * R1, derivative=True)
        ya, dya = sp.spherical_yn(n, k0 * R1), sp.spherical_yn(n, k0 * R1, derivative=True)
        ha, dha = ja + 1j * ya, dja + 1j * dya
        j11, dj11 = sp.spherical_jn(n, k1 * R1), sp.spherical_jn(n, k1 * R1, derivative=True)
        y11, dy11 = sp.spherical_yn(n, k1 * R1), sp.spherical_yn(n, k1 * R1, derivative=True)
        j12, dj12 = sp.spherical_jn(n, k1 * R2), sp.spherical_jn(n, k1 * R2, derivative=True)
        y12, dy12 = sp.spherical_yn(n, k1 * R2), sp.spherical_yn(n, k1 * R2, derivative=True)
        j22, dj22 = sp.spherical_jn(n, k2 * R2), sp.spherical_jn(n, k2 * R2, derivative=True)
        # unknown C_n is rescaled by y11 to keep the system balanced for large n
        s = 1.0 / y11
        M = np.array([
            [ha, -j11, -y11 * s, 0.0],
            [k0 / rho0 * dha, -k1 / rho1 * dj11, -k1 / rho1 * dy11 * s, 0.0],
            [0.0, j12, y12 * s, -j22],
            [0.0, k1 / rho1 * dj12, k1 / rho1 * dy12 * s, -k2 / rho2 * dj22],
        ], dtype=np.complex128)
        rhs = np.array([-ja, -k0 / rho0 * dja, 0.0, 0.0], dtype=np.complex128)
        sol = np.linalg.solve(M, rhs)
        sol[2] *= s
        coef[n] = sol
    return coef


def mie_layered(points, direction, k0, rho0, c0, R1, rho1, c1, R2, rho2, c2, nmax=None):
    """Total pressure at points (n, 3) for the plane wave exp(i k0 x.d) on the
    concentric spheres; omega = k0 c0, k_j = omega / c_j."""
    P = np.asarray(points, dtype=np.float64)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    omega = k0 * c0
    k1, k2 = omega / c1, omega / c2
    if nmax is None:
        nmax = mie_truncation(max(k0, k1, k2) * R1)
    coef = mie_coefficients(k0, rho0, k1, rho1, R1, k2, rho2, R2, nmax)
    r = np.sqrt(np.sum(P ** 2, axis=1))
    with np.errstate(invalid="ignore", divide="ignore"):
        ct = np.where(r > 0, (P @ d) / np.where(r > 0, r, 1.0), 1.0)
    out = np.zeros(r.shape, dtype=np.complex128)
    reg0, reg1, reg2 = r >= R1, (r < R1) & (r >= R2), r < R2
    for n in range(nmax + 1):
        A, B, C, D = coef[n]
        Pn = sp.eval_legendre(n, ct)
        f = (1j ** n) * (2 * n + 1)
        if np.any(reg0):
            x = k0 * r[reg0]
            out[reg0] += f * (sp.spherical_jn(n, x) + A * (sp.spherical_jn(n, x) + 1j * sp.spherical_yn(n, x))) * Pn[reg0]
        if np.any(reg1):
            x = k1 * r[reg1]
            out[reg1] += f * (B * sp.spherical_jn(n, x) + C * sp.spherical_yn(n, x)) * Pn[reg1]
        if np.any(reg2):
            x = k2 * r[reg2]
            out[reg2] += f * D * sp.spherical_jn(n, x) * Pn[reg2]
    return out


def mie_far_field(directions, incidence, k0, rho0, c0, R1, rho1, c1, R2, rho2, c2, nmax=None):
    """Far-field pattern f(xhat) of the scattered field of mie_layered,
    p - p_inc = exp(i k0 r)/r f(xhat) + O(r^-2) in the exterior.  With the
    large-argument form h_n(z) ~ (-i)^(n+1) exp(i z)/z of the outgoing
    spherical Hankel function, each term i^n (2n+1) A_n h_n(k0 r) P_n
    contributes (-i/k0) (2n+1) A_n P_n(xhat . d)."""
    X = np.atleast_2d(np.asarray(directions, dtype=np.float64))
    X = X / np.linalg.norm(X, axis=1, keepdims=True)
    d = np.asarray(incidence, dtype=np.float64)
    d = d / np.linalg.norm(d)
    omega = k0 * c0
    k1, k2 = omega / c1, omega / c2
    if nmax is None:
        nmax = mie_truncation(max(k0, k1, k2) * R1)
    coef = mie_coefficients(k0, rho0, k1, rho1, R1, k2, rho2, R2, nmax)
    ct = X @ d
    out = np.zeros(X.shape[0], dtype=np.complex128)
    for n in range(nmax + 1):
        out += (2 * n + 1) * coef[n, 0] * sp.eval_legendre(n, ct)
    return (-1j / k0) * out
