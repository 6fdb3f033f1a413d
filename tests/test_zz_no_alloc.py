"""vsie_matvec_noalloc -- the forward product with its work buffers in the
library's static device work area (for callers that cannot allocate) --
against vsie_matvec through the C ABI: two calls in a row, the second with a
smaller input, then a smaller problem, and a request beyond the area's size
refused with VSIE_E_WORKSPACE."""
import ctypes

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


def _noalloc(V, P, x, prec):
    """y = A x through vsie_matvec_noalloc; x (R, n) or (n,) complex128."""
    import torch
    y = torch.full_like(x, complex(float("nan"), float("nan")))
    R = 1 if x.dim() == 1 else x.shape[0]
    st = V.lib.vsie_matvec_noalloc(P.handle, 0, prec, R, ctypes.c_void_p(x.data_ptr()), P.n,
                                   ctypes.c_void_p(y.data_ptr()), P.n,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, y


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_matvec(V, prec):
    import torch
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    tol = 1e-12 if prec == "fp64" else 1e-5
    big = case("lognormal")
    small = case("c0")
    Pb = V.Problem.from_mesh(big[0], big[1], [big[2]])
    Ps = V.Problem.from_mesh(small[0], small[1], [small[2]])
    calls = [(Pb, big, 5), (Pb, big, 1), (Ps, small, 1)]   # the same problem with fewer columns, then a smaller one
    for i, (P, (mesh, mat, k0), R) in enumerate(calls):
        x = dev(W.seeded_complex((mesh.n, R), seed=160 + i)).contiguous()
        if R == 1:
            x = x.reshape(-1)
        st, y = _noalloc(V, P, x, pr)
        assert st == V.VSIE_OK, V.vsie_last_error()
        ref = P.matvec(x, prec=pr)
        torch.cuda.synchronize()
        d = O.discretise(mesh, mat, k0)
        e_api = parity_err(host(y), host(ref))
        e_orc = parity_err(host(y), O.matvec(d, host(x).reshape(mesh.n, -1)).reshape(host(x).shape))
        say("  call %d: n %d R %d %s: vs vsie_matvec %.1e (bitwise %s), vs oracle %.2e"
            % (i, mesh.n, R, prec, e_api, torch.equal(y, ref), e_orc))
        assert torch.equal(y, ref) and e_api <= tol and e_orc <= tol
    Pb.close()
    Ps.close()


def test_noalloc_refuses_more_than_its_area(V):
    """16 columns of the c1 problem in FP64 need about 1.1 GB of chunk
    partials, beyond the static area: refused with VSIE_E_WORKSPACE, no
    output written."""
    import torch
    mesh, mat, k0s, dirs, _ = W.config_problem("c1")
    P = V.Problem.from_mesh(mesh, mat, k0s)
    need = P.workspace_size(V.VSIE_OP_MATVEC, 16, prec=V.VSIE_FP64)
    assert need > (256 << 20)
    x = torch.zeros((16, P.n), dtype=torch.complex128, device="cuda")
    st, y = _noalloc(V, P, x, V.VSIE_FP64)
    assert st == V.VSIE_E_WORKSPACE and "static work area" in V.vsie_last_error()
    assert torch.isnan(torch.view_as_real(y)).all()
    # one column fits (once-per-pair kernels, FP32 slot partials)
    x1 = dev(W.seeded_complex(P.n, seed=170))
    st, y1 = _noalloc(V, P, x1, V.VSIE_FP32)
    assert st == V.VSIE_OK and torch.equal(y1, P.matvec(x1, prec=V.VSIE_FP32))
    P.close()


def test_noalloc_with_assembled_operator(V):
    """With an assembled FP32 operator the product runs on the matrix-core
    kernel, still without allocating: equal to vsie_matvec bitwise, twice in
    a row with fewer columns the second time."""
    import torch
    mesh, mat, k0 = case("cube")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    A = P.assemble_dense(0)
    d = O.discretise(mesh, mat, k0)
    for R in (6, 2):
        x = dev(W.seeded_complex((mesh.n, R), seed=180 + R)).contiguous()
        st, y = _noalloc(V, P, x, V.VSIE_FP32)
        assert st == V.VSIE_OK, V.vsie_last_error()
        assert torch.equal(y, P.matvec(x, prec=V.VSIE_FP32))
        assert parity_err(host(y), O.matvec(d, host(x))) <= 1e-5
    del A
    P.close()
