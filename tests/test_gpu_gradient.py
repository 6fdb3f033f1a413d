"""Adjoint-state gradient of a receiver misfit on the GPU against finite
differences of the FP64 oracle's misfit (dense LU solves), and the adjoint
pieces against the oracle's own sums."""
import copy
import sys

import numpy as np
import pytest

import oracle as O
from gpu_cases import host, oracle_residual, parity_err, sample_rows, say
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available()
    import paper_2607_06429_amd as V
    return V


def medium(N, seed_shift=0):
    mesh = W.nested_balls(N)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8)
    mat.vol_c = mat.vol_c * W.lognormal_voxel_field(mesh.vol_xyz, -1, 1, 32, 0.1, 0)
    mat.vol_rho = mat.vol_rho * W.lognormal_voxel_field(mesh.vol_xyz, -1, 1, 32, 0.1, 1)
    return mesh, mat


def gpu_gradient(V, mesh, mat, k0, dirs, rec, data, prec=0, tol=1e-13):
    import torch
    from paper_2607_06429_amd.autograd import receiver_pressure
    P = V.Problem.from_mesh(mesh, mat, [k0])
    c = torch.tensor(mat.vol_c, device="cuda", requires_grad=True)
    rho = torch.tensor(mat.vol_rho, device="cuda", requires_grad=True)
    pr = receiver_pressure(P, mesh.n_vol, c, rho, dirs, rec, prec=prec, tol=tol)
    dt = torch.as_tensor(np.ascontiguousarray(data.T), device="cuda")
    loss = 0.5 * (pr - dt).abs().pow(2).sum()
    loss.backward()
    return float(loss.detach()), c.grad.cpu().numpy(), rho.grad.cpu().numpy(), pr.detach().cpu().numpy().T


def fd(mesh, mat, k0, dirs, rec, data, which, cells, eps=1e-5):
    out = []
    for j in cells:
        vals = []
        for sgn in (1, -1):
            m2 = copy.deepcopy(mat)
            arr = m2.vol_c if which == "c" else m2.vol_rho
            h = eps * arr[j]
            arr[j] += sgn * h
            vals.append(O.receiver_misfit(mesh, m2, k0, dirs, rec, data))
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)


def test_receiver_pressures_match_oracle(V):
    mesh, mat = medium(7)
    k0, dirs, rec = 4.0, W.fibonacci_sphere(2), W.fibonacci_sphere(12, 2.0)
    ref = O.receiver_pressures(mesh, mat, k0, dirs, rec)
    data = np.zeros_like(ref)
    _, _, _, pr = gpu_gradient(V, mesh, mat, k0, dirs, rec, data)
    assert parity_err(pr, ref) < 1e-11


def test_gradient_all_parameters_tiny_mesh(V):
    """Every cell's c and rho on a 6^3 staircase mesh (T terms, both
    interfaces): the full oracle finite-difference gradient."""
    mesh, mat = medium(6)
    k0, dirs, rec = 3.0, W.fibonacci_sphere(2), W.fibonacci_sphere(10, 2.0)
    data = 0.5 * W.seeded_complex((10, 2), seed=41)
    say("tiny gradient: cells", mesh.n_vol, "faces", mesh.n_srf)
    J, gc, gr, _ = gpu_gradient(V, mesh, mat, k0, dirs, rec, data)
    J0 = O.receiver_misfit(mesh, mat, k0, dirs, rec, data)
    assert abs(J - J0) <= 1e-11 * abs(J0)
    cells = np.arange(mesh.n_vol)
    fc = fd(mesh, mat, k0, dirs, rec, data, "c", cells)
    fr = fd(mesh, mat, k0, dirs, rec, data, "rho", cells)
    ec, er = O.rel_error(gc, fc), O.rel_error(gr, fr)
    say("  rel err grad c %.2e  grad rho %.2e" % (ec, er))
    assert ec < 1e-6 and er < 1e-6


@pytest.mark.parametrize("prec", [0, 1])
def test_gradient_random_cells(V, prec):
    """16 seeded cells of a 10^3 mesh; FP64 and FP32+refinement solves."""
    mesh, mat = medium(10)
    k0, dirs, rec = 5.0, W.fibonacci_sphere(3), W.fibonacci_sphere(24, 2.5)
    data = 0.3 * W.seeded_complex((24, 3), seed=42)
    J, gc, gr, _ = gpu_gradient(V, mesh, mat, k0, dirs, rec, data, prec=prec, tol=1e-12)
    cells = np.random.default_rng(43).choice(mesh.n_vol, 16, replace=False)
    fc = fd(mesh, mat, k0, dirs, rec, data, "c", cells)
    fr = fd(mesh, mat, k0, dirs, rec, data, "rho", cells)
    ec, er = O.rel_error(gc[cells], fc), O.rel_error(gr[cells], fr)
    say("  prec %d rel err grad c %.2e  grad rho %.2e" % (prec, ec, er))
    assert ec < 1e-6 and er < 1e-6


def test_adjoint_rhs_and_source_sums_match_oracle(V):
    import torch
    mesh, mat = medium(8)
    k0, rec = 4.0, W.fibonacci_sphere(16, 2.0)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    rho = W.seeded_complex((16, 2), seed=44)
    zR, ZR = P.source_sums(torch.as_tensor(np.ascontiguousarray(rho.T), device="cuda"), targets=rec)
    rhs = P.adjoint_rhs(zR, ZR).cpu().numpy().T
    # oracle: (E^H rho)_j = sum_r conj(E_rj) rho_r with E_rj = -kappa(x_r, j), by columns of the
    # off-diagonal operator at the receivers
    E = -np.stack([O.offdiag_apply(d, np.eye(d.n)[:, j], targets=rec, exclude_self=False)
                   for j in range(d.n)], axis=1)
    ref = E.conj().T @ rho
    assert parity_err(rhs, ref) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c3_forward_block_solves_oracle_residual(V, prec):
    """The c3 forward problem at full size (n = 71,368, log-normal c and rho,
    k0 = 10, 8 incidences) by block GMRES, plain FP64 and FP32 operator inside
    FP64 refinement; the oracle computes the residual of all 8 GPU solutions
    on sampled rows."""
    mesh, mat, k0s, dirs, rec = W.config_problem("c3")
    d = O.discretise(mesh, mat, k0s[0])
    P = V.Problem.from_mesh(mesh, mat, k0s)
    b = P.plane_wave(dirs)
    x, info = P.solve(b, prec=V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32, tol=1e-10, block=True)
    res = oracle_residual(d, host(x), host(b), sample_rows(d.n, d.n_vol, 256, 27))
    say("c3 forward block solve %s: %s, oracle residual on sampled rows %.2e" % (prec, info, res))
    assert info["status"] == V.VSIE_OK and res <= 1e-9
    P.close()


def test_c3_gradient_full_size_finite_differences(V):
    """The c3 workload at full size (c1 mesh, n = 71,368, log-normal c and rho,
    k0 = 10, 8 incidences, 256 receivers on |x| = 3; data = receiver pressures
    of the unperturbed c1 medium).  The adjoint gradient against central
    differences of the misfit on 16 seeded cells x {c, rho}; every misfit
    evaluation is an FP64 GPU solve to relative residual 1e-13, and the step is
    1e-3 of the parameter (truncation ~1e-6 relative, solve noise ~1e-6)."""
    import torch
    from paper_2607_06429_amd.autograd import receiver_pressure
    mesh, mat, k0s, dirs, rec = W.config_problem("c3")
    mesh1, mat1, _, _, _ = W.config_problem("c1")
    k0 = k0s[0]
    P = V.Problem.from_mesh(mesh, mat, [k0])
    say("c3 gradient: n", P.n, "incidences", len(dirs), "receivers", len(rec))

    def pressures(c, rho, tol=1e-13):
        P.set_materials(torch.as_tensor(rho, device="cuda"), torch.as_tensor(c, device="cuda"))
        b = P.plane_wave(dirs)
        x, info = P.solve(b, prec=V.VSIE_FP64, tol=tol, block=True)
        assert info["status"] == V.VSIE_OK
        return P.plane_wave_at(rec, dirs) - P.field(rec, x)

    data = pressures(mat1.vol_c, mat1.vol_rho)
    c = torch.tensor(mat.vol_c, device="cuda", requires_grad=True)
    rho = torch.tensor(mat.vol_rho, device="cuda", requires_grad=True)
    pr = receiver_pressure(P, mesh.n_vol, c, rho, dirs, rec, tol=1e-13, block=True)
    loss = 0.5 * (pr - data).abs().pow(2).sum()
    loss.backward()
    gc, gr = c.grad.cpu().numpy(), rho.grad.cpu().numpy()

    def misfit(cv, rv):
        return float(0.5 * (pressures(cv, rv) - data).abs().pow(2).sum())

    cells = np.random.default_rng(2607).choice(mesh.n_vol, 16, replace=False)
    out = {}
    for which, g in (("c", gc), ("rho", gr)):
        fdv = []
        for j in cells:
            vals = []
            for sgn in (1, -1):
                cv, rv = mat.vol_c.copy(), mat.vol_rho.copy()
                arr = cv if which == "c" else rv
                h = 1e-3 * arr[j]
                arr[j] += sgn * h
                vals.append(misfit(cv, rv))
            fdv.append((vals[0] - vals[1]) / (2 * h))
        fdv = np.array(fdv)
        out[which] = O.rel_error(g[cells], fdv)
        say("  grad %s: rel err vs central differences %.2e (|fd| max %.3e)" % (which, out[which], np.abs(fdv).max()))
    assert out["c"] < 1e-4 and out["rho"] < 1e-4
    P.close()
