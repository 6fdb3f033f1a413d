"""Lockstep multi-frequency block GMRES (vsie_solve_multi) on reduced copies
of the cube-with-ellipsoid workload (log-normal sound speed, 8 wavenumbers x
16 plane waves), frequency by frequency against the FP64 oracle.  The
wavenumbers are those of the 100^3 grid scaled by N/100, so that k0 h (the
sampling per wavelength) matches the full-size problem.

Bars: solutions within 1e-8 of the oracle's LU solutions (relative, 2-norm
and max-norm); sampled-row oracle residuals within 1e-9."""
import re

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_cases import dev, host, oracle_residual, parity_err, sample_rows, say

pytestmark = pytest.mark.gpu

TOL_SOLVE = 1e-8


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available()
    import paper_2607_06429_amd as V
    return V


def reduced_c4(N):
    mesh, mat, k0s, dirs, _ = W.config_problem("c4", N=N)
    return mesh, mat, [k * N / 100.0 for k in k0s], dirs


def rhs(P, dirs, nf):
    import torch
    return torch.cat([P.plane_wave(dirs, f=f) for f in range(nf)], dim=0).contiguous()


def step_lines(err):
    """The lockstep progress lines, grouped by refinement step."""
    groups = []
    for line in err.splitlines():
        if "lockstep refinement step" in line:
            groups.append([])
        elif "lockstep block step" in line and groups:
            groups[-1].append(line)
    return groups


@pytest.fixture(scope="module")
def small(V):
    """N = 12: every frequency's oracle LU solution of the 16 plane waves."""
    mesh, mat, ks, dirs = reduced_c4(12)
    refs = []
    for k in ks:
        d = O.discretise(mesh, mat, k)
        refs.append(O.solve_lu(d, O.plane_wave(d.pts, k, dirs)))
    say("reduced c4, N = 12: n", mesh.n, "k0", ["%.2f" % k for k in ks])
    return mesh, mat, ks, dirs, refs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("restart", [500, 4])
def test_solve_multi_against_oracle_lu(V, small, capfd, prec, restart):
    """All 8 frequencies in one call, long cycles and 4-step cycles (restarts,
    deflation by the kept first cycle); every block step of the first
    refinement step is one operator launch for all frequencies, and the
    single-layer kernel runs once per lockstep step."""
    mesh, mat, ks, dirs, refs = small
    P = V.Problem.from_mesh(mesh, mat, ks)
    B = rhs(P, dirs, len(ks))
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    P.profile(True)
    X, infos = P.solve_multi(B, prec=pr, tol=1e-10, restart=restart, progress=True)
    st = P.kernel_stats()
    P.profile(False)
    err = capfd.readouterr().err
    R = dirs.shape[0]
    for f, (info, ref) in enumerate(zip(infos, refs)):
        e = parity_err(host(X[f * R:(f + 1) * R]), ref)
        say("  %s restart %d k0 %.2f: %s, rel err vs LU %.2e" % (prec, restart, ks[f], info, e))
        assert info["status"] == V.VSIE_OK and info["rel_residual"] <= 1e-10
        assert e <= TOL_SOLVE
    groups = step_lines(err)
    assert groups and groups[0], err[-2000:]
    assert all("in 1 multi-frequency product " in ln for ln in groups[0]), groups[0]
    steps = sum(len(g) for g in groups)
    if prec == "fp32":
        # the FP32 kernel runs only in block steps: exactly one launch per step
        assert st["mfma_fwd_single_layer_fp32"]["launches"] == steps, (st, steps)
    else:
        # the FP64 kernel also computes the residual after every cycle (the
        # last progress group is the final check, with no cycle): one launch
        # each when the live frequencies form one run of equal width
        cycles = len(groups) - 1
        launches = st["mfma_fwd_single_layer_fp64"]["launches"]
        assert steps + cycles <= launches <= steps + cycles * len(ks), (launches, steps, cycles)
    P.close()


def test_solve_multi_matches_single_frequency_solves_c4_24(V):
    """N = 24 (n ~ 19k), FP32 operator in FP64 refinement: every frequency's
    lockstep solution against the oracle on 256 sampled rows and against a
    one-frequency block solve of the same right-hand sides."""
    mesh, mat, ks, dirs = reduced_c4(24)
    P = V.Problem.from_mesh(mesh, mat, ks)
    B = rhs(P, dirs, len(ks))
    X, infos = P.solve_multi(B, prec=V.VSIE_FP32, tol=1e-10)
    R = dirs.shape[0]
    rows = sample_rows(mesh.n, mesh.n_vol, 256, 61)
    for f, k in enumerate(ks):
        d = O.discretise(mesh, mat, k)
        xf, bf = X[f * R:(f + 1) * R], B[f * R:(f + 1) * R]
        res = oracle_residual(d, host(xf), host(bf), rows)
        x1, i1 = P.solve(bf.contiguous(), f=f, prec=V.VSIE_FP32, tol=1e-10, block=True)
        diff = parity_err(host(xf), host(x1))
        say("  N 24 k0 %.2f: %s; oracle residual %.2e; vs one-frequency block solve %.2e (%s)"
            % (k, infos[f], res, diff, i1))
        assert infos[f]["status"] == V.VSIE_OK and res <= 1e-9 and diff <= TOL_SOLVE
    P.close()


def test_solve_multi_caller_workspace_bitwise(V, small):
    """A caller workspace of vsie_workspace_size bytes gives bitwise the same
    solutions as the library-owned buffers; one byte less is refused."""
    import torch
    mesh, mat, ks, dirs, _ = small
    P = V.Problem.from_mesh(mesh, mat, ks)
    B = rhs(P, dirs, len(ks))
    kw = dict(prec=V.VSIE_FP32, tol=1e-10)
    X0, _ = P.solve_multi(B, **kw)
    nb = P.workspace_size(V.VSIE_OP_SOLVE_MULTI, nrhs=dirs.shape[0], nf=len(ks), prec=V.VSIE_FP32)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    X1, _ = P.solve_multi(B, workspace=ws, **kw)
    assert torch.equal(X0, X1)
    with pytest.raises(V.VsieError) as e:
        P.solve_multi(B, workspace=ws[:nb - 256], **kw)
    assert e.value.status == V.VSIE_E_WORKSPACE
    P.close()


def test_solve_multi_uneven_frequencies(V, small):
    """A sub-range of three frequencies where they do not move alike: the
    first has a zero column (width 15 against 16: separate launches), the
    second starts from its exact solution (no iterations), the third is
    ordinary."""
    mesh, mat, ks, dirs, refs = small
    P = V.Problem.from_mesh(mesh, mat, ks)
    R = dirs.shape[0]
    B = rhs(P, dirs, len(ks))[2 * R:5 * R].clone()
    B[3] = 0
    X0 = dev(np.zeros((mesh.n, 3 * R), dtype=complex)).contiguous()
    X0[R:2 * R] = dev(refs[3]).contiguous()
    X, infos = P.solve_multi(B, f0=2, nf=3, prec=V.VSIE_FP64, x0=X0, tol=1e-10)
    for t in range(3):
        ref = refs[2 + t].copy()
        if t == 0:
            ref[:, 3] = 0
        e = parity_err(host(X[t * R:(t + 1) * R]), ref)
        say("  f %d: %s, rel err %.2e" % (2 + t, infos[t], e))
        assert infos[t]["status"] == V.VSIE_OK and e <= TOL_SOLVE
    assert infos[1]["iterations"] == 0 and infos[1]["matvecs_fp64"] == R
    assert np.all(host(X[3]) == 0)
    P.close()


def test_solve_multi_rejects_bad_input(V, small):
    import torch
    mesh, mat, ks, dirs, _ = small
    P = V.Problem.from_mesh(mesh, mat, ks[:2])
    B = rhs(P, dirs[:2], 2)
    with pytest.raises(V.VsieError) as e:
        P.solve_multi(B, f0=1, nf=2)
    assert e.value.status == V.VSIE_E_INVALID
    B[1, 5] = float("nan")
    with pytest.raises(V.VsieError) as e:
        P.solve_multi(B)
    assert e.value.status == V.VSIE_E_NAN
    P.close()
    del torch
