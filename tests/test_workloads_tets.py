"""Conforming tetrahedral meshes (the paper's section 2.3.1 leaves tetrahedra
and triangles to future implementations): the Kuhn split of cuboid grids,
with planar interfaces (nested cubes) and curved ones (nested balls mapped
from nested cubes), and the oracle on them.  CPU only.

* the mesher: volumes and interface areas, conformity and orientation of the
  interface triangles, the curved interfaces approaching the spheres;
* the oracle on tetrahedra: Green's identity for the double layer on a
  tetrahedral domain, discrete reciprocity for constant density (exact for
  any mesh), and the solution converging to the layered-sphere series.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.analytic as A
import workloads as W


@pytest.mark.parametrize("ns,ni", [(1, 3), (2, 5)])
def test_kuhn_split_of_nested_cubes(ns, ni):
    mesh = W.nested_cubes_tets(ns, ni, 7.0, 5.0)
    vox = W.nested_cubes(ns, ni, 7.0, 5.0)
    assert mesh.n_vol == 6 * vox.n_vol and mesh.n_srf == 2 * vox.n_srf
    assert abs(mesh.vol_w.sum() - 343.0) < 1e-10
    assert abs(mesh.vol_w[mesh.vol_dom == 2].sum() - 125.0) < 1e-10
    # each cuboid splits into six tetrahedra of a sixth of its volume
    assert np.allclose(np.sort(mesh.vol_w), np.sort(np.repeat(vox.vol_w, 6) / 6.0), rtol=1e-12)
    g1, g2 = mesh.srf_iface == 1, mesh.srf_iface == 2
    assert abs(mesh.srf_area[g1].sum() - 6 * 49.0) < 1e-10 and abs(mesh.srf_area[g2].sum() - 6 * 25.0) < 1e-10
    # planar interfaces: normals along an axis, pointing out of the inside
    # tetrahedron and into the outside one
    assert np.allclose(np.sort(np.abs(mesh.srf_n), axis=1), [0, 0, 1])
    cin = mesh.vol_xyz[mesh.srf_cell_in]
    assert np.all(np.einsum("ij,ij->i", mesh.srf_n, mesh.srf_xyz - cin) > 0)
    out = mesh.srf_cell_out[g2]
    assert np.all(out >= 0) and np.all(mesh.vol_dom[out] == 1) and np.all(mesh.vol_dom[mesh.srf_cell_in[g2]] == 2)
    assert np.all(np.einsum("ij,ij->i", mesh.srf_n[g2], mesh.vol_xyz[out] - mesh.srf_xyz[g2]) > 0)
    assert np.all(mesh.srf_cell_out[g1] == -1) and np.all(mesh.vol_dom[mesh.srf_cell_in[g1]] == 1)
    # conforming: every interface triangle occurs once; the two triangles of a
    # face have the face's centroid as the mean of their centroids
    key = np.round(mesh.srf_xyz, 9)
    assert np.unique(key, axis=0).shape[0] == mesh.n_srf
    assert np.allclose(np.sort(mesh.srf_area[g1]), np.sort(np.repeat(vox.srf_area[vox.srf_iface == 1], 2) / 2))


def test_mapped_balls_approach_the_spheres():
    """The curved interfaces are inscribed polyhedra of the spheres: volumes
    and areas converge to the balls' at O(h^2)."""
    errs = []
    for N in (4, 8, 16):
        mesh = W.nested_balls_tets(N)
        g1, g2 = mesh.srf_iface == 1, mesh.srf_iface == 2
        ev = abs(mesh.vol_w.sum() / (4 * math.pi / 3) - 1)
        ev2 = abs(mesh.vol_w[mesh.vol_dom == 2].sum() / (4 * math.pi / 3 * 0.125) - 1)
        ea1 = abs(mesh.srf_area[g1].sum() / (4 * math.pi) - 1)
        ea2 = abs(mesh.srf_area[g2].sum() / (4 * math.pi * 0.25) - 1)
        errs.append((ev, ev2, ea1, ea2))
        # the triangle centroids lie just inside the spheres (vertices on them)
        r = np.linalg.norm(mesh.srf_xyz, axis=1)
        assert np.all(r[g1] < 1.0) and np.all(r[g1] > 1.0 - 2.0 / N)
        assert np.all(r[g2] < 0.5) and np.all(r[g2] > 0.5 - 2.0 / N)
        cin = mesh.vol_xyz[mesh.srf_cell_in]
        assert np.all(np.einsum("ij,ij->i", mesh.srf_n, mesh.srf_xyz - cin) > 0)
        # outward normals, close to the radial direction
        assert np.all(np.einsum("ij,ij->i", mesh.srf_n, mesh.srf_xyz / r[:, None]) > 0.5)
    for q in range(4):
        assert errs[0][q] > errs[1][q] > errs[2][q], errs
        assert errs[1][q] / errs[2][q] > 3.0, errs    # about 4 per halving of h
    with pytest.raises(ValueError):
        W.nested_balls_tets(6)


def test_double_layer_green_identity_on_tetrahedra():
    """int_{dD} dG/dn_y dS = -1 - k^2 int_D G dy for x inside D, on a
    tetrahedral ball (the mapped grid with one subdomain): the discrete K[1]
    on its triangles approaches -1 - k^2 V[1] on its tetrahedra."""
    k0 = 2.0
    errs = []
    for N in (4, 8, 12):
        e = np.linspace(-1.0, 1.0, N + 1)
        mesh = W.kuhn_tet_mesh(e, lambda i, j, k: np.ones_like(i), W.cube_to_ball)
        inner = np.linalg.norm(mesh.vol_xyz, axis=1) < 0.5
        dK = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 0.5, 1.0, 0.5, 1.0), k0)
        K1 = O.offdiag_apply(dK, np.concatenate([np.zeros(mesh.n_vol), np.ones(mesh.n_srf)]))
        c = k0 / math.sqrt(k0 ** 2 - 1.0)
        dV = O.discretise(mesh, W.materials_piecewise(mesh, 1.0, 1.0, 1.0, c, 1.0, c), k0)
        V1 = O.matvec(dV, np.ones(dV.n))[:mesh.n_vol] - 1.0
        errs.append(O.rel_error(K1[:mesh.n_vol][inner], -1.0 - k0 ** 2 * V1[inner]))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.02, errs


@pytest.mark.parametrize("kind", ["cubes", "balls"])
def test_reciprocity_exact_on_tetrahedra_for_constant_density(kind):
    """diag(s) A is complex-symmetric on any mesh when the density is
    constant, so the discrete far field is reciprocal to rounding."""
    mesh = W.nested_cubes_tets(1, 3, 2.0, 1.2) if kind == "cubes" else W.nested_balls_tets(4)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.0, 1.5, 1.0, 0.8)
    d = O.discretise(mesh, mat, 2.0)
    D = W.fibonacci_sphere(4)
    X = W.fibonacci_sphere(3) @ np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    P = O.solve_lu(d, O.plane_wave(d.pts, 2.0, np.vstack([D, -X])))
    e = O.rel_error(O.far_field(d, X, P[:, :4]), O.far_field(d, -D, P[:, 4:]).T)
    assert e < 1e-12, e


def _series_errors(N, rho1, rho2):
    mesh = W.nested_balls_tets(N)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, rho1, 1.5, rho2, 0.8)
    d = O.discretise(mesh, mat, 2.0)
    b = O.plane_wave(d.pts, 2.0, [0, 0, 1.0])
    p = O.solve_lu(d, b) if d.n < 6000 else O.solve_gmres(d, b, tol=1e-10)[0]
    args = (2.0, 1.0, 1.0, 1.0, rho1, 1.5, 0.5, rho2, 0.8)
    vol = O.rel_error(p[:mesh.n_vol], A.mie_layered(mesh.vol_xyz, [0, 0, 1.0], *args))
    X = W.fibonacci_sphere(64)
    far = O.rel_error(O.far_field(d, X, p), A.mie_far_field(X, [0, 0, 1.0], *args))
    return vol, far


def test_tetrahedral_balls_converge_to_the_series():
    """The layered-sphere series (exact spheres; the meshes are inscribed
    polyhedra) against the oracle's solution on the mapped tetrahedra, with
    density jumps at both interfaces: volume values 5.7%, 4.4%, 3.4% and far
    field 4.3%, 1.2%, 0.61% for N = 4, 8, 12 (the voxel staircase at N = 8,
    12, 16: 11.0%, 9.6%, 7.7% and 2.3%, 1.8%, 1.2%)."""
    errs = [_series_errors(N, 1.2, 2.0) for N in (4, 8, 12)]
    vol = [e[0] for e in errs]
    far = [e[1] for e in errs]
    assert vol[0] > vol[1] > vol[2] and vol[2] < 0.04, errs
    assert far[0] > far[1] > far[2] and far[2] < 0.008, errs
