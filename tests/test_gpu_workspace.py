"""Caller workspace at the C ABI: every product and solve given exactly
vsie_workspace_size bytes matches the same call on the problem's own buffers
bitwise (the same kernels in the same order, only other addresses), and one
byte less is refused with VSIE_E_WORKSPACE before any work is queued."""
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


def _ws(nbytes, short=False):
    import torch
    return torch.empty(max(1, nbytes - (1 if short else 0)), dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("name", ["c0", "lognormal", "cube"])
@pytest.mark.parametrize("R", [1, 3, 17])
def test_products_with_caller_workspace(V, name, R):
    import torch
    mesh, mat, k0 = case(name)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x = dev(W.seeded_complex((mesh.n, R), seed=151)).contiguous()
    if R == 1:
        x = x.reshape(-1)
    for prec in (V.VSIE_FP64, V.VSIE_FP32):
        for op, fn in ((V.VSIE_OP_MATVEC, P.matvec), (V.VSIE_OP_MATVEC_ADJOINT, P.matvec_adjoint)):
            nb = P.workspace_size(op, R, prec=prec)
            ref = fn(x, prec=prec)
            got = fn(x, prec=prec, workspace=_ws(nb))
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (name, R, prec, op)
            with pytest.raises(V.VsieError) as e:
                fn(x, prec=prec, workspace=_ws(nb, short=True))
            assert e.value.status == V.VSIE_E_WORKSPACE
            # library-owned buffers again after a workspace call
            assert torch.equal(fn(x, prec=prec), ref)
        say("  %s R=%d prec %d: matvec %d B, adjoint %d B" % (
            name, R, prec, P.workspace_size(V.VSIE_OP_MATVEC, R, prec=prec),
            P.workspace_size(V.VSIE_OP_MATVEC_ADJOINT, R, prec=prec)))
    P.close()


def test_multi_frequency_and_dense_with_caller_workspace(V):
    import torch
    mesh, mat, _ = case("lognormal")
    ks = [2.0, 5.0, 7.5]
    P = V.Problem.from_mesh(mesh, mat, ks)
    R = 16
    x = dev(W.seeded_complex((mesh.n, 3 * R), seed=152)).contiguous()
    nb = P.workspace_size(V.VSIE_OP_MATVEC_MULTI, R, prec=V.VSIE_FP32, nf=3)
    ref = P.matvec_multi(x, 0, 3, prec=V.VSIE_FP32)
    got = P.matvec_multi(x, 0, 3, prec=V.VSIE_FP32, workspace=_ws(nb))
    assert torch.equal(got, ref)
    with pytest.raises(V.VsieError) as e:
        P.matvec_multi(x, 0, 3, prec=V.VSIE_FP32, workspace=_ws(nb, short=True))
    assert e.value.status == V.VSIE_E_WORKSPACE
    # the assembled FP32 operator
    A = P.assemble_dense(1)
    x4 = x[:4].contiguous()
    nbd = P.workspace_size(V.VSIE_OP_MATVEC, 4, f=1, prec=V.VSIE_FP32)
    ref = P.matvec(x4, f=1, prec=V.VSIE_FP32)
    got = P.matvec(x4, f=1, prec=V.VSIE_FP32, workspace=_ws(nbd))
    assert torch.equal(got, ref)
    d = O.discretise(mesh, mat, ks[1])
    assert parity_err(host(got), O.matvec(d, host(x4))) <= 1e-5
    del A
    P.close()


@pytest.mark.parametrize("block", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_solves_with_caller_workspace(V, prec, block, adjoint):
    """Solves (restarted so that the deflated later cycles run) with a caller
    workspace: bitwise the library-owned solve, and the oracle's solution."""
    import torch
    mesh, mat, k0 = case("ragged")
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    b = P.plane_wave(W.fibonacci_sphere(3))
    kw = dict(prec=pr, adjoint=adjoint, tol=1e-11, restart=6, block=block, max_outer=200)
    op = V.VSIE_OP_SOLVE_ADJOINT if adjoint else V.VSIE_OP_SOLVE
    nb = P.workspace_size(op, 3, prec=pr, tol=1e-11, restart=6, block=block, max_outer=200)
    x0, i0 = P.solve(b, **kw)
    x1, i1 = P.solve(b, workspace=_ws(nb), **kw)
    torch.cuda.synchronize()
    say("  solve %s block=%s adjoint=%s: workspace %d B, %s" % (prec, block, adjoint, nb, i1))
    assert i0 == i1 and torch.equal(x0, x1)
    with pytest.raises(V.VsieError) as e:
        P.solve(b, workspace=_ws(nb, short=True), **kw)
    assert e.value.status == V.VSIE_E_WORKSPACE
    A = O.assemble(d)
    ref = np.linalg.solve(A.conj().T if adjoint else A, host(b))
    assert parity_err(host(x1), ref) <= 1e-8
    P.close()


def test_c1_solve_with_caller_workspace(V):
    """The headline solve (c1, one column, FP32 operator in FP64 refinement)
    with every work buffer in a torch allocation: bitwise the library-owned
    solve."""
    import torch
    mesh, mat, k0s, dirs, _ = W.config_problem("c1")
    P = V.Problem.from_mesh(mesh, mat, k0s)
    b = P.plane_wave(dirs[0])
    nb = P.workspace_size(V.VSIE_OP_SOLVE, 1, prec=V.VSIE_FP32, tol=1e-10)
    x0, i0 = P.solve(b, prec=V.VSIE_FP32, tol=1e-10)
    x1, i1 = P.solve(b, prec=V.VSIE_FP32, tol=1e-10, workspace=_ws(nb))
    say("  c1 FP32 + refinement: workspace %.1f MB, %s" % (nb / 1e6, i1))
    assert i0 == i1 and torch.equal(x0, x1)
    P.close()
