"""The GPU path on conforming tetrahedral meshes (Kuhn split of cuboid grids;
section 2.3.1 leaves tetrahedra to future implementations): the kernels take
any element centroids, measures and normals, so the operator, the solver and
the far field run unchanged.  Parity against the oracle on planar (nested
cubes) and curved (mapped nested balls) interfaces, convergence of the GPU
solution to the layered-sphere series, and tetrahedra against voxels on the
paper's nested-cube geometry."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.analytic as A
import workloads as W
from gpu_cases import dev, host, parity_err, say

pytestmark = pytest.mark.gpu

TOL64, TOL32, TOL_SOLVE = 1e-12, 1e-5, 1e-8


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2607_06429_amd as V
    return V


def _case(name):
    """(mesh, materials, k0, grad_rho or None)"""
    if name == "balls":          # curved interfaces, density jumps, smooth core sound speed
        mesh = W.nested_balls_tets(8)
        mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.2, 1.5, 2.0,
                                    lambda x: 0.8 * (1 + 0.2 * np.exp(-np.sum(x * x, axis=1) / 0.05)))
        return mesh, mat, 4.0, None
    if name == "cubes_lognormal":  # planar interfaces, per-tetrahedron log-normal c
        mesh = W.nested_cubes_tets(2, 4, 7.0, 5.0)
        mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.0, 1 / 1.2, 0.5, 1 / 1.2)
        mat.vol_c = mat.vol_c * W.lognormal_voxel_field(mesh.vol_xyz, -3.5, 3.5, 16, 0.1, 0)
        return mesh, mat, 2 * math.pi / 3.0, None
    if name == "cubes_graded":     # analytic density with its gradient: T terms on tetrahedra
        mesh = W.nested_cubes_tets(2, 4, 7.0, 5.0)
        mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.0, 1 / 1.2, W.benchmark4_density, 1 / 1.2)
        grad = np.zeros((mesh.n_vol, 3))
        inner = mesh.vol_dom == 2
        grad[inner] = W.benchmark4_density_gradient(mesh.vol_xyz[inner])
        return mesh, mat, 2 * math.pi / 1.4, grad
    raise KeyError(name)


CASES = ["balls", "cubes_lognormal", "cubes_graded"]


@pytest.mark.parametrize("name", CASES)
def test_tet_products_against_oracle(V, name):
    mesh, mat, k0, grad = _case(name)
    d = O.discretise(mesh, mat, k0, grad_rho=grad)
    P = V.Problem.from_mesh(mesh, mat, [k0], grad_rho=grad)
    for R in (1, 3):
        x = W.seeded_complex((d.n, R), seed=200 + R)
        xin = dev(x[:, 0]) if R == 1 else dev(x).contiguous()
        ref, refa = O.matvec(d, x), O.adjoint_matvec(d, x)
        for prec, tol in ((V.VSIE_FP64, TOL64), (V.VSIE_FP32, TOL32)):
            y = host(P.matvec(xin, prec=prec)).reshape(d.n, R)
            ya = host(P.matvec_adjoint(xin, prec=prec)).reshape(d.n, R)
            e, ea = parity_err(y, ref), parity_err(ya, refa)
            say("  %s n %d R %d prec %d: forward %.2e adjoint %.2e" % (name, d.n, R, prec, e, ea))
            assert e <= tol and ea <= tol
    P.close()


@pytest.mark.parametrize("name", CASES)
def test_tet_solves_against_oracle_lu(V, name):
    mesh, mat, k0, grad = _case(name)
    d = O.discretise(mesh, mat, k0, grad_rho=grad)
    b = O.plane_wave(d.pts, k0, W.fibonacci_sphere(2))
    ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, [k0], grad_rho=grad)
    for prec in (V.VSIE_FP64, V.VSIE_FP32):
        x, info = P.solve(dev(b).contiguous(), prec=prec, tol=1e-11)
        e = parity_err(host(x), ref)
        say("  %s solve prec %d: %s, vs LU %.2e" % (name, prec, info, e))
        assert info["status"] == V.VSIE_OK and e <= TOL_SOLVE
    P.close()


def test_tet_balls_converge_to_the_series(V):
    """GPU solutions (FP32 operator in FP64 refinement) on the mapped
    tetrahedral balls against the layered-sphere series, density jumps at both
    interfaces: volume values and far field improve with every refinement."""
    errs = []
    for N in (8, 12, 16, 20):
        if N % 4:
            continue
        mesh = W.nested_balls_tets(N)
        mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8)
        P = V.Problem.from_mesh(mesh, mat, [2.0])
        x, info = P.solve(P.plane_wave([0.0, 0.0, 1.0]), prec=V.VSIE_FP32, tol=1e-10)
        args = (2.0, 1.0, 1.0, 1.0, 1.2, 1.5, 0.5, 2.0, 0.8)
        X = W.fibonacci_sphere(64)
        vol = O.rel_error(host(x)[:mesh.n_vol], A.mie_layered(mesh.vol_xyz, [0, 0, 1.0], *args))
        far = O.rel_error(host(P.far_field(X, x)), A.mie_far_field(X, [0, 0, 1.0], *args))
        say("  tetrahedral balls N %d: n %d, %d iterations, vs series: volume %.4f far field %.4f"
            % (N, P.n, info["iterations"], vol, far))
        errs.append((vol, far))
        P.close()
    for q in range(2):
        assert all(errs[i][q] > errs[i + 1][q] for i in range(len(errs) - 1)), errs
    assert errs[-1][1] < 0.005, errs


def test_tets_and_voxels_agree_on_nested_cubes(V):
    """The paper's nested cubes with a density jump (7 and 5 mm, rho2 = 0.5,
    c = c0/1.2, wavelength 3 mm): the exterior fields of the tetrahedral and
    the cuboid discretisations of the same geometry approach each other under
    refinement (both converge to the continuous solution)."""
    k0 = 2 * math.pi / 3.0
    rec = W.fibonacci_sphere(64, 8.0)
    diffs = []
    for ns, ni in ((1, 5), (2, 10), (3, 15)):
        fields = []
        for mesh in (W.nested_cubes(ns, ni, 7.0, 5.0), W.nested_cubes_tets(ns, ni, 7.0, 5.0)):
            mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.0, 1 / 1.2, 0.5, 1 / 1.2)
            P = V.Problem.from_mesh(mesh, mat, [k0])
            x, info = P.solve(P.plane_wave([1.0, 0.0, 0.0]), prec=V.VSIE_FP32, tol=1e-10)
            assert info["status"] == V.VSIE_OK
            fields.append(host(P.plane_wave_at(rec, [1.0, 0.0, 0.0]) - P.field(rec, x)).reshape(-1))
            P.close()
        diffs.append(O.rel_error(fields[1], fields[0]))
        say("  nested cubes %d + %d + %d cells per axis: tetrahedra vs cuboids, exterior field %.4f"
            % (ns, ni, ns, diffs[-1]))
    assert diffs[0] > diffs[1] > diffs[2], diffs
