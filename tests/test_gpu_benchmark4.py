"""The paper's fourth benchmark (nested cubes, analytic heterogeneous density
in the inner cube with a jump across Gamma_2, wavespeed jump across Gamma_1;
its 3D run on 61^3 cuboids) on the GPU against the FP64 oracle, with
grad alpha from the analytic density gradient (vsie_geometry.vgrad_rho)."""
import copy

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_cases import dev, host, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
TOL_SOLVE = 1e-8


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available()
    import paper_2607_06429_amd as V
    return V


def small():
    """The benchmark on a coarse fitted grid (2 + 6 + 2 cuboids per axis)."""
    return W.benchmark4_problem(n_shell=2, n_inner=6, lam0=4.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_grid_products_against_oracle(V, prec):
    mesh, mat, k0, dirs, grad = small()
    d = O.discretise(mesh, mat, k0[0], grad_rho=grad)
    assert np.count_nonzero(d.gT) > 0            # the T term is active
    P = V.Problem.from_mesh(mesh, mat, k0, grad_rho=grad)
    x = W.seeded_complex((d.n, 3), seed=401)
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    tol = TOL64 if prec == "fp64" else TOL32
    y = host(P.matvec(dev(x), prec=pr))
    ya = host(P.matvec_adjoint(dev(x), prec=pr))
    e, ea = O.rel_error(y, O.matvec(d, x)), O.rel_error(ya, O.adjoint_matvec(d, x))
    # one column: the once-per-pair cell-cell kernel
    y1 = host(P.matvec(dev(x[:, 0]), prec=pr))
    e1 = O.rel_error(y1, O.matvec(d, x[:, :1])[:, 0])
    say("  b4 small %s: n %d rel err %.2e adjoint %.2e one column %.2e" % (prec, d.n, e, ea, e1))
    assert e <= tol and ea <= tol and e1 <= tol
    P.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_grid_solve_against_lu(V, prec):
    mesh, mat, k0, dirs, grad = small()
    d = O.discretise(mesh, mat, k0[0], grad_rho=grad)
    b = O.plane_wave(d.pts, k0[0], dirs)
    ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, k0, grad_rho=grad)
    x, info = P.solve(dev(b).contiguous(), prec=V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32, tol=1e-11)
    e = O.rel_error(host(x), ref)
    say("  b4 small solve %s: %s rel err %.2e" % (prec, info, e))
    assert info["status"] == V.VSIE_OK and e <= TOL_SOLVE
    P.close()


def test_density_gradient_through_the_adjoint(V):
    """Receiver-misfit gradient w.r.t. per-cell rho and c with the analytic
    density gradient held fixed (grad alpha = -rho0 grad(rho)/rho^2 moves with
    rho), against finite differences of the oracle misfit."""
    import torch
    from paper_2607_06429_amd.autograd import receiver_pressure
    mesh, mat, k0, dirs, grad = small()
    rec = W.fibonacci_sphere(12, 5.0)
    data = 0.4 * W.seeded_complex((12, 1), seed=402)
    P = V.Problem.from_mesh(mesh, mat, k0, grad_rho=grad)
    c = torch.tensor(mat.vol_c, device="cuda", requires_grad=True)
    rho = torch.tensor(mat.vol_rho, device="cuda", requires_grad=True)
    pr = receiver_pressure(P, mesh.n_vol, c, rho, dirs, rec, prec=V.VSIE_FP64, tol=1e-13)
    loss = 0.5 * (pr - torch.as_tensor(np.ascontiguousarray(data.T), device="cuda")).abs().pow(2).sum()
    loss.backward()
    gc, gr = c.grad.cpu().numpy(), rho.grad.cpu().numpy()
    inner = np.nonzero(mesh.vol_dom == 2)[0]
    cells = np.concatenate([np.random.default_rng(403).choice(inner, 8, replace=False),
                            np.random.default_rng(404).choice(np.nonzero(mesh.vol_dom == 1)[0], 4, replace=False)])
    out = {}
    for which, g in (("c", gc), ("rho", gr)):
        fd = []
        for j in cells:
            vals = []
            for sgn in (1, -1):
                m2 = copy.deepcopy(mat)
                arr = m2.vol_c if which == "c" else m2.vol_rho
                h = 1e-5 * arr[j]
                arr[j] += sgn * h
                vals.append(O.receiver_misfit(mesh, m2, k0[0], dirs, rec, data, grad_rho=grad))
            fd.append((vals[0] - vals[1]) / (2 * h))
        out[which] = O.rel_error(g[cells], np.array(fd))
    say("  b4 gradient vs oracle FD: c %.2e rho %.2e" % (out["c"], out["rho"]))
    assert out["c"] < 1e-6 and out["rho"] < 1e-6
    P.close()


def test_paper_grid_sampled_rows(V):
    """The 3D run's grid (61^3 cuboids, n = 260,401): sampled rows of the FP64
    and FP32 one-column products against the oracle."""
    mesh, mat, k0, dirs, grad = W.benchmark4_problem()
    d = O.discretise(mesh, mat, k0[0], grad_rho=grad)
    P = V.Problem.from_mesh(mesh, mat, k0, grad_rho=grad)
    b = P.plane_wave(dirs)
    rows = np.unique(np.concatenate([np.random.default_rng(405).choice(d.n, 128, replace=False),
                                     [0, mesh.n_vol - 1, mesh.n_vol, d.n - 1]]))
    xb = host(b)
    ref = O.matvec(d, xb.reshape(-1, 1), rows=rows)[:, 0]
    for pr, tol in ((V.VSIE_FP64, TOL64), (V.VSIE_FP32, TOL32)):
        y = host(P.matvec(b, prec=pr)).reshape(-1)
        e = O.rel_error(y[rows], ref)
        say("  b4 n %d prec %d: sampled-row rel err %.2e" % (d.n, pr, e))
        assert e <= tol
    P.close()
