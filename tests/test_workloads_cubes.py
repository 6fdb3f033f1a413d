"""The nested-cube cuboid mesher and the heterogeneous-density medium of the
paper's fourth benchmark (section 3.4 of the paper, its 3D run), and the
oracle's grad alpha of an analytic density.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def test_paper_grid_of_the_3d_run():
    """9 + 43 + 9 cuboids per axis: the 226,981-voxel grid of the paper's 3D
    run at 10 voxels per interior wavelength (1.4 mm / 1.2), fitted to both
    cube interfaces."""
    mesh, mat, k0, dirs, grad = W.benchmark4_problem()
    c = mesh.counts()
    assert c["omega1"] + c["omega2"] == 61 ** 3 == 226981
    assert c["omega2"] == 43 ** 3
    assert c["gamma1"] == 6 * 61 ** 2 and c["gamma2"] == 6 * 43 ** 2
    assert mesh.h <= 1.4 / 1.2 / 10
    assert abs(k0[0] - 2 * math.pi / 1.4) < 1e-15
    assert np.allclose(dirs, [[math.sqrt(0.5), math.sqrt(0.5), 0.0]])


@pytest.mark.parametrize("ns,ni", [(1, 2), (2, 5), (3, 4)])
def test_nested_cubes_geometry(ns, ni):
    mesh = W.nested_cubes(ns, ni, 7.0, 5.0)
    N = 2 * ns + ni
    assert mesh.n_vol == N ** 3
    assert abs(mesh.vol_w.sum() - 343.0) < 1e-10
    inner = mesh.vol_dom == 2
    assert abs(mesh.vol_w[inner].sum() - 125.0) < 1e-10
    assert np.all(np.abs(mesh.vol_xyz[inner]) < 2.5) and np.all(np.max(np.abs(mesh.vol_xyz[~inner]), axis=1) > 2.5)
    g1, g2 = mesh.srf_iface == 1, mesh.srf_iface == 2
    assert abs(mesh.srf_area[g1].sum() - 6 * 49.0) < 1e-10
    assert abs(mesh.srf_area[g2].sum() - 6 * 25.0) < 1e-10
    # faces on the interface planes, normals out of the inside subdomain
    for sel, half in ((g1, 3.5), (g2, 2.5)):
        x, n = mesh.srf_xyz[sel], mesh.srf_n[sel]
        assert np.allclose(np.sum(x * n, axis=1), half)
        assert np.allclose(np.abs(n).sum(axis=1), 1.0)
    # each face sits on a face of its inside cell, and Gamma_2 faces have an Omega_1 cell outside
    cin = mesh.vol_xyz[mesh.srf_cell_in]
    assert np.all(np.sum((mesh.srf_xyz - cin) * mesh.srf_n, axis=1) > 0)
    assert np.all(mesh.srf_cell_out[g1] == -1)
    assert np.all(mesh.vol_dom[mesh.srf_cell_out[g2]] == 1)
    assert np.all(mesh.vol_dom[mesh.srf_cell_in[g2]] == 2)


def test_density_gradient_is_the_derivative_of_the_density():
    rng = np.random.default_rng(7)
    x = rng.uniform(-2.5, 2.5, (200, 3))
    g = W.benchmark4_density_gradient(x)
    h = 1e-5
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        fd = (W.benchmark4_density(x + e) - W.benchmark4_density(x - e)) / (2 * h)
        assert np.max(np.abs(fd - g[:, ax])) < 1e-8


def test_oracle_grad_alpha_of_an_analytic_density():
    """alpha = rho0/rho - 1 (eq_alpha): the oracle's grad alpha from grad rho
    against central differences of alpha itself."""
    rng = np.random.default_rng(8)
    x = rng.uniform(-2.5, 2.5, (200, 3))
    rho0 = 1.3
    ga = O.grad_alpha_from_density_gradient(W.benchmark4_density(x), W.benchmark4_density_gradient(x), rho0)
    h = 1e-5
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        fd = (rho0 / W.benchmark4_density(x + e) - rho0 / W.benchmark4_density(x - e)) / (2 * h)
        assert np.max(np.abs(fd - ga[:, ax])) < 1e-8


def test_analytic_and_stencil_grad_alpha_agree_under_refinement():
    """On the inner cube, the neighbour stencil of per-cell alpha approaches
    the analytic grad alpha as the grid is refined (second order inside)."""
    errs = []
    for ni in (8, 16, 32):
        mesh = W.nested_cubes(1, ni, 7.0, 5.0)
        inner = mesh.vol_dom == 2
        rho = np.ones(mesh.n_vol)
        rho[inner] = W.benchmark4_density(mesh.vol_xyz[inner])
        grad = np.zeros((mesh.n_vol, 3))
        grad[inner] = W.benchmark4_density_gradient(mesh.vol_xyz[inner])
        ga = O.grad_alpha_from_density_gradient(rho, grad, 1.0)
        gs = O.grad_alpha_stencil(mesh, 1.0 / rho - 1.0)
        # cells of a fixed region well inside the inner cube
        far = inner & np.all(np.abs(mesh.vol_xyz) < 1.5, axis=1)
        errs.append(np.sqrt(np.mean((ga[far] - gs[far]) ** 2)))
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3


@pytest.mark.parametrize("mesh_kind", ["balls", "cubes"])
def test_grad_alpha_stencil_exact_for_linear_alpha(mesh_kind):
    """A density with alpha = rho0/rho - 1 linear in x: every branch of the
    neighbour stencil (central, one-sided up, one-sided down) differentiates a
    linear function exactly, on uniform and nonuniform grids, so grad alpha
    must equal the constant gradient on every cell and axis with a neighbour in
    the same subdomain -- including the one-sided cells next to Gamma_1 and
    Gamma_2 -- and be zero where the axis has none."""
    if mesh_kind == "balls":
        mesh = W.nested_balls(10)
    else:
        mesh = W.nested_cubes(2, 5, 7.0, 5.0)
    rho0 = 1.3
    g = np.array([0.11, -0.07, 0.05])
    a0 = np.where(mesh.vol_dom == 2, 0.4, 0.2)     # a jump between the subdomains
    a = a0 + mesh.vol_xyz @ g
    rho = rho0 / (1.0 + a)
    assert np.all(rho > 0)
    ga = O.grad_alpha_stencil(mesh, O.alpha(rho, rho0))
    dom = mesh.vol_dom
    seen = {"central": 0, "up": 0, "down": 0, "none": 0}
    for ax in range(3):
        lo = mesh.vol_nb[:, 2 * ax].astype(np.int64)
        hi = mesh.vol_nb[:, 2 * ax + 1].astype(np.int64)
        lo_ok = (lo >= 0) & (dom[np.maximum(lo, 0)] == dom)
        hi_ok = (hi >= 0) & (dom[np.maximum(hi, 0)] == dom)
        has = lo_ok | hi_ok
        np.testing.assert_allclose(ga[has, ax], g[ax], rtol=0, atol=1e-12)
        assert np.all(ga[~has, ax] == 0.0)
        seen["central"] += int(np.sum(lo_ok & hi_ok))
        seen["up"] += int(np.sum(hi_ok & ~lo_ok))
        seen["down"] += int(np.sum(lo_ok & ~hi_ok))
        seen["none"] += int(np.sum(~has))
    # every branch ran, the one-sided ones at the interfaces
    assert min(seen["central"], seen["up"], seen["down"]) > 0, seen
