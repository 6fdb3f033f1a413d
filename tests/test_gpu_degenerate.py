"""Degenerate and boundary-sized meshes on the GPU against the oracle: one
cell, two cells, a mesh with no surface elements, and cell counts one past and
one short of a 64-point tile, in both precisions (products, adjoint products,
the one-column kernels, a solve and the far field)."""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_cases import dev, host, say, parity_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available()
    import paper_2607_06429_amd as V
    return V


def _box(nx, ny, nz, h=0.3):
    """nx x ny x nz unit cells of width h, all in Omega_1 (one subdomain)."""
    edges = [np.arange(m + 1) * h for m in (nx, ny, nz)]
    m = max(nx, ny, nz)
    e = np.arange(m + 1) * h
    mesh = W.tensor_mesh(e, lambda i, j, k: np.where((i < nx) & (j < ny) & (k < nz), 1, 0))
    assert mesh.n_vol == nx * ny * nz, edges
    return mesh


def _no_faces(mesh):
    z3, zi = np.zeros((0, 3)), np.zeros(0, np.int32)
    return dataclasses.replace(mesh, srf_xyz=z3, srf_n=z3, srf_area=np.zeros(0), srf_iface=zi,
                               srf_cell_in=zi, srf_cell_out=zi)


def _lognormal(mesh, seed):
    rng = np.random.default_rng(seed)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.3, 1.2, 1.3, 1.2)
    mat.vol_rho = mat.vol_rho * np.exp(0.2 * rng.standard_normal(mesh.n_vol))
    mat.vol_c = mat.vol_c * np.exp(0.2 * rng.standard_normal(mesh.n_vol))
    return mat


def _cases():
    one = _box(1, 1, 1)
    two = _box(2, 1, 1)
    balls = W.nested_balls(6)
    return {
        "one_cell": (one, _lognormal(one, 1)),
        "two_cells": (two, _lognormal(two, 2)),
        "no_faces": (_no_faces(balls), W.materials_piecewise(balls, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8)),
        "tile_plus_one": (_box(5, 13, 1), _lognormal(_box(5, 13, 1), 3)),      # 65 cells
        "tile_minus_one": (_box(7, 9, 1), _lognormal(_box(7, 9, 1), 4)),       # 63 cells
    }


CASES = list(_cases())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", CASES)
def test_degenerate_mesh(V, name, prec):
    mesh, mat = _cases()[name]
    k0 = 2.5
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr, tol = (V.VSIE_FP64, 1e-12) if prec == "fp64" else (V.VSIE_FP32, 1e-5)
    x = W.seeded_complex((d.n, 3), seed=90)
    e_fwd = parity_err(host(P.matvec(dev(x), prec=pr)), O.matvec(d, x))
    e_adj = parity_err(host(P.matvec_adjoint(dev(x), prec=pr)), O.adjoint_matvec(d, x))
    e_one = parity_err(host(P.matvec(dev(x[:, 0]), prec=pr)), O.matvec(d, x[:, :1])[:, 0])
    b = O.plane_wave(d.pts, k0, [0.0, 0.6, 0.8])
    xs, info = P.solve(dev(b).contiguous(), prec=pr, tol=1e-12)
    e_sol = parity_err(host(xs), O.solve_lu(d, b))
    X = W.fibonacci_sphere(20)
    e_ff = parity_err(host(P.far_field(X, dev(x[:, 0]), prec=pr)), O.far_field(d, X, x[:, 0]))
    say("  %s %s: n %d (%d cells, %d faces) fwd %.1e adj %.1e one %.1e solve %.1e (%d it) far %.1e"
        % (name, prec, d.n, mesh.n_vol, mesh.n_srf, e_fwd, e_adj, e_one, e_sol, info["iterations"], e_ff))
    assert max(e_fwd, e_adj, e_one, e_ff) <= tol
    assert info["status"] == V.VSIE_OK and e_sol <= 1e-8
    P.close()
