"""Far-field pattern of the scattered pressure on the GPU (vsie_far_field)
against the oracle's far field, the series far field and the GPU's own
exterior field at large distance; the exterior field (vsie_field) on a slice
of the paper's sphere benchmark against the oracle and the series."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.analytic as A
import workloads as W
from gpu_cases import CASES, case, dev, host, say, parity_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available()
    import paper_2607_06429_amd as V
    return V


def _dirs(m):
    # Fibonacci directions plus the six axis directions (ragged count)
    X = np.concatenate([W.fibonacci_sphere(m), np.eye(3), -np.eye(3)])
    return X / np.linalg.norm(X, axis=1, keepdims=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", CASES)
def test_far_field_against_oracle(V, name, prec):
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr, tol = (V.VSIE_FP64, TOL64) if prec == "fp64" else (V.VSIE_FP32, TOL32)
    X = _dirs(300)
    for R in (1, 3, 21):        # 21 = 16 + 4 + 1 right-hand-side blocks
        x = W.seeded_complex((d.n, R), seed=70 + R)
        xin = dev(x[:, 0]) if R == 1 else dev(x)
        got = host(P.far_field(X, xin, prec=pr))
        ref = O.far_field(d, X, x[:, 0] if R == 1 else x)
        e = parity_err(got, ref)
        say("  far field %s %s R=%d: rel err %.2e" % (name, prec, R, e))
        assert e <= tol
    P.close()


def test_far_field_of_the_sphere_solution_matches_the_series(V):
    """The paper's sphere benchmark at 8 cells per interior wavelength: the
    far field of the GPU solution against the series far field (the
    discretisation error; the same solution's cell values are within 2.2% of
    the series), and the optical theorem within the same margin."""
    mesh, mat, k0, dirs, _ = W.benchmark1_problem(29)
    P = V.Problem.from_mesh(mesh, mat, k0)
    x, info = P.solve(P.plane_wave(dirs), prec=V.VSIE_FP32, tol=1e-10)
    assert info["status"] == V.VSIE_OK
    mu, w = np.polynomial.legendre.leggauss(96)
    phi = np.arange(48) * (2 * math.pi / 48)
    # quadrature grid about the incidence axis x: (mu along x, phi around it)
    MU, PH = np.meshgrid(mu, phi, indexing="ij")
    S = np.sqrt(1 - MU ** 2)
    X = np.stack([MU.ravel(), (S * np.cos(PH)).ravel(), (S * np.sin(PH)).ravel()], axis=1)
    f = host(P.far_field(X, x, prec=V.VSIE_FP64)).reshape(-1)
    ref = A.mie_far_field(X, dirs[0], k0[0], 1.0, 1.0, 3.0, 1.0, 1.0, 2.5, 1.0, 5.0 / 6.0)
    e = parity_err(f, ref)
    scat = np.sum(np.repeat(w, 48) * (2 * math.pi / 48) * np.abs(f) ** 2)
    ext = 4 * math.pi / k0[0] * host(P.far_field(dirs, x, prec=V.VSIE_FP64)).reshape(-1)[0].imag
    say("  b1 far field vs series: rel err %.4f; optical theorem scat %.5f ext %.5f" % (e, scat, ext))
    assert e < 0.03 and abs(scat - ext) < 0.03 * ext
    P.close()


def test_far_field_is_the_limit_of_the_gpu_exterior_field(V):
    """R exp(-i k R) (p - p_inc)(R d) from vsie_field approaches vsie_far_field
    as O(1/R): a property of the two entry points at any size."""
    mesh, mat, k0 = case("lognormal")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x = dev(W.seeded_complex(mesh.n, seed=77))
    X = _dirs(64)
    f = host(P.far_field(X, x))
    errs = []
    for R in (1e3, 1e4):
        psc = -host(P.field(R * X, x))
        errs.append(O.rel_error(R * np.exp(-1j * k0 * R) * psc, f))
    say("  far field vs field at R = 1e3, 1e4: %.2e %.2e" % tuple(errs))
    assert errs[1] < 1e-3 and errs[0] / errs[1] > 8
    P.close()


@pytest.mark.parametrize("which", ["c4", "b4"])
def test_far_field_at_full_size_sampled_directions(V, which):
    """The largest meshes (c4: n = 1,076,336 at k0 = 40; the 3D run of the
    paper's fourth benchmark: n = 260,401): 24 sampled directions against the
    oracle, FP64 and FP32, with the plane wave as the vector."""
    if which == "c4":
        mesh, mat, k0s, dirs, _ = W.config_problem("c4")
        k0s = k0s[:1]
        grad = None
    else:
        mesh, mat, k0s, dirs, grad = W.benchmark4_problem()
    d = O.discretise(mesh, mat, k0s[0], grad_rho=grad)
    P = V.Problem.from_mesh(mesh, mat, k0s, grad_rho=grad)
    b = P.plane_wave(dirs[:1])
    X = _dirs(18)
    ref = O.far_field(d, X, host(b).reshape(-1))
    for pr, tol in ((V.VSIE_FP64, TOL64), (V.VSIE_FP32, TOL32)):
        e = parity_err(host(P.far_field(X, b, prec=pr)).reshape(-1), ref)
        say("  far field %s n %d prec %d: rel err %.2e" % (which, d.n, pr, e))
        assert e <= tol
    P.close()


def test_far_field_second_frequency_and_errors(V):
    mesh, mat, _ = case("ragged")
    P = V.Problem.from_mesh(mesh, mat, [2.0, 4.5])
    d = O.discretise(mesh, mat, 4.5)
    x = W.seeded_complex(d.n, seed=78)
    X = _dirs(10)
    got = host(P.far_field(X, dev(x), f=1))
    assert parity_err(got, O.far_field(d, X, x)) <= TOL64
    import torch
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.complex128, device="cuda")
    with pytest.raises(V.VsieError):
        V.vsie_far_field(P.handle, 2, V.VSIE_FP64, one, one, one, dev(x), out)   # no frequency 2
    with pytest.raises(ValueError):
        P.far_field([[1.0, 1.0, 0.0]], dev(x))                                  # not a unit vector
    P.close()


def _slice_outside(half, lo, hi, m):
    """m x m grid on z = 0 over [lo, hi]^2 without the points of [-half, half]^2."""
    g = np.linspace(lo, hi, m)
    X, Y = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    keep = np.max(np.abs(P[:, :2]), axis=1) > half + 1e-9
    return P[keep]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_exterior_field_on_a_slice(V, prec):
    """The sphere benchmark's slice z = 0 outside the cube (the representation
    formula, section 2.3.1, at 4,880 points): the GPU field of the GPU solution
    against the oracle's exterior field of the same vector, and the total field
    against the series."""
    mesh, mat, k0, dirs, _ = W.benchmark1_problem(29)
    d = O.discretise(mesh, mat, k0[0])
    P = V.Problem.from_mesh(mesh, mat, k0)
    x, info = P.solve(P.plane_wave(dirs), prec=V.VSIE_FP64, tol=1e-10)
    pts = _slice_outside(3.0, -6.0, 6.0, 81)
    pr, tol = (V.VSIE_FP64, TOL64) if prec == "fp64" else (V.VSIE_FP32, TOL32)
    xh = host(x).reshape(-1)
    got = O.plane_wave(pts, k0[0], dirs[0]) - host(P.field(pts, x.reshape(-1), prec=pr))
    ref = O.exterior_field(d, pts, xh, dirs[0])
    e = parity_err(got, ref)
    series = A.mie_layered(pts, dirs[0], k0[0], 1.0, 1.0, 3.0, 1.0, 1.0, 2.5, 1.0, 5.0 / 6.0)
    es, esm = O.rel_error(got, series), O.rel_error(got, series, ord=np.inf)
    say("  b1 slice %s: %d points, vs oracle %.2e, vs series L2 %.4f max %.4f" % (prec, len(pts), e, es, esm))
    assert e <= tol and es < 0.03 and esm < 0.03
    P.close()
