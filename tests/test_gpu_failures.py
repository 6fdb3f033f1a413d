"""Failure paths of the C ABI on the GPU: non-finite right-hand sides and
initial guesses, rejected materials (which must leave the problem untouched),
material arrays of the wrong length, and the autograd wrapper when another
forward has changed the problem's materials before a backward."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_cases import case, dev, host, parity_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2607_06429_amd as V
    return V


@pytest.mark.parametrize("block", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("where", ["b_nan", "b_inf", "x0_nan"])
def test_non_finite_inputs_return_nan_status(V, where, prec, block):
    import torch
    mesh, mat, k0 = case("ragged")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    b = P.plane_wave(W.fibonacci_sphere(2))
    x0 = torch.zeros_like(b)
    if where == "b_nan":
        b[1, 5] = complex(float("nan"), 0.0)
    elif where == "b_inf":
        b[0, 0] = complex(0.0, float("inf"))
    else:
        x0[0, 7] = complex(float("nan"), 1.0)
    with pytest.raises(V.VsieError) as e:
        P.solve(b, prec=pr, x0=x0, block=block)
    say("  %s %s block=%s: %s" % (where, prec, block, e.value))
    assert e.value.status == V.VSIE_E_NAN
    P.close()


@pytest.mark.parametrize("bad", ["rho_zero", "rho_negative", "c_zero", "c_nan", "rho_inf"])
def test_rejected_materials_leave_the_problem_unchanged(V, bad):
    """vsie_set_materials with rho <= 0, c <= 0 or a non-finite value returns
    VSIE_E_INVALID, and the forward product, the adjoint product and the
    parameter gradient afterwards are bitwise those of before."""
    import torch
    mesh, mat, k0 = case("lognormal")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x = dev(W.seeded_complex(mesh.n, seed=141))
    lam = dev(W.seeded_complex((mesh.n, 1), seed=142)).reshape(1, -1).contiguous()
    xs = x.reshape(1, -1).contiguous()

    def snapshot():
        y = P.matvec(x, prec=V.VSIE_FP64)
        y32 = P.matvec(x, prec=V.VSIE_FP32)
        ya = P.matvec_adjoint(x, prec=V.VSIE_FP64)
        z, Z = P.source_sums(lam)
        g = P.param_gradient(xs, lam, z, Z, z, Z, mesh.n_vol)
        torch.cuda.synchronize()
        return [y, y32, ya, g[0], g[1]]

    before = snapshot()
    rho = torch.as_tensor(mat.vol_rho * 1.1, device="cuda")
    c = torch.as_tensor(mat.vol_c * 0.9, device="cuda")
    j = mesh.n_vol // 2
    if bad == "rho_zero":
        rho[j] = 0.0
    elif bad == "rho_negative":
        rho[j] = -1.0
    elif bad == "c_zero":
        c[j] = 0.0
    elif bad == "c_nan":
        c[j] = float("nan")
    else:
        rho[j] = float("inf")
    with pytest.raises(V.VsieError) as e:
        P.set_materials(rho, c)
    assert e.value.status == V.VSIE_E_INVALID and "positive" in str(e.value)
    after = snapshot()
    for a, b in zip(before, after):
        assert torch.equal(a, b)
    # still the oracle's operator of the original materials
    d = O.discretise(mesh, mat, k0)
    assert parity_err(host(after[0]), O.matvec(d, host(x)[:, None])[:, 0]) <= 1e-12
    # a short material array is refused by the binding before the call
    with pytest.raises(ValueError):
        P.set_materials(rho[:-1].contiguous(), c[:-1].contiguous())
    P.close()


def test_backward_after_another_forward_uses_its_own_materials(V):
    """Two receiver-pressure forwards with different materials on one problem,
    then the backward of the first: its gradient must equal that of the same
    forward and backward run alone."""
    import torch
    from paper_2607_06429_amd.autograd import receiver_pressure
    mesh, mat, k0 = case("lognormal")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    dirs = W.fibonacci_sphere(2)
    rec = W.fibonacci_sphere(16, 2.5)
    data = torch.as_tensor(W.seeded_complex((2, 16), seed=143), device="cuda")

    def leaf(a):
        return torch.tensor(a, device="cuda", requires_grad=True)

    c1, r1 = leaf(mat.vol_c), leaf(mat.vol_rho)
    loss = 0.5 * (receiver_pressure(P, mesh.n_vol, c1, r1, dirs, rec) - data).abs().pow(2).sum()
    loss.backward()
    ref = (c1.grad.clone(), r1.grad.clone())

    c1, r1 = leaf(mat.vol_c), leaf(mat.vol_rho)
    loss1 = 0.5 * (receiver_pressure(P, mesh.n_vol, c1, r1, dirs, rec) - data).abs().pow(2).sum()
    c2, r2 = leaf(mat.vol_c * 1.05), leaf(mat.vol_rho * 0.95)
    loss2 = 0.5 * (receiver_pressure(P, mesh.n_vol, c2, r2, dirs, rec) - data).abs().pow(2).sum()
    loss1.backward()
    e_c = float((c1.grad - ref[0]).norm() / ref[0].norm())
    e_r = float((r1.grad - ref[1]).norm() / ref[1].norm())
    say("  interleaved backward vs alone: c %.2e rho %.2e" % (e_c, e_r))
    assert e_c < 1e-10 and e_r < 1e-10
    loss2.backward()
    assert torch.isfinite(c2.grad).all()
    P.close()


@pytest.mark.parametrize("bad", [dict(krylov_gib=-1), dict(krylov_gib=5000), dict(restart=0),
                                 dict(inner_tol=1.0), dict(max_outer=0)])
def test_invalid_solver_options_are_rejected(V, bad):
    """Solver options outside their documented ranges are refused with
    VSIE_E_INVALID before any work, by the one-frequency and the lockstep
    multi-frequency solves and by the workspace query; x is left as given."""
    import torch
    mesh, mat, k0 = case("ragged")
    P = V.Problem.from_mesh(mesh, mat, [k0, 1.5 * k0])
    b = P.plane_wave(W.fibonacci_sphere(2))
    x0 = torch.full_like(b, 0.25)
    for call in (lambda: P.solve(b, x0=x0, **bad),
                 lambda: P.solve_multi(torch.cat([b, b]).contiguous(), x0=torch.cat([x0, x0]), **bad),
                 lambda: P.workspace_size(V.VSIE_OP_SOLVE, nrhs=2, **bad)):
        with pytest.raises(V.VsieError) as e:
            call()
        assert e.value.status == V.VSIE_E_INVALID, bad
    assert torch.all(x0 == 0.25)
    P.close()
