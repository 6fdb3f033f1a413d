"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: FP64 operator <= 1e-12 relative (2-norm over all entries), FP32 operator
<= 1e-5, solutions of the refined FP32 path and of the FP64 path <= 1e-8
against the oracle solution.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_cases import CASES, case, dev, host, oracle_residual, parity_err, sample_rows, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
TOL_SOLVE = 1e-8


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2607_06429_amd as V
    return V



@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("R", [1, 3, 17])
def test_matvec_parity(V, name, R):
    say("matvec parity", name, "R", R)
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x = W.seeded_complex((d.n, R), seed=11)
    ref = O.matvec(d, x)
    y64 = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP64)).reshape(d.n, R)
    y32 = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP32)).reshape(d.n, R)
    e64, e32 = parity_err(y64, ref), parity_err(y32, ref)
    say("  rel err fp64 %.3e fp32 %.3e" % (e64, e32))
    assert e64 <= TOL64
    assert e32 <= TOL32


@pytest.mark.parametrize("name", ["c0", "lognormal", "cube"])
def test_adjoint_parity(V, name):
    say("adjoint parity", name)
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    lam = W.seeded_complex((d.n, 2), seed=12)
    ref = O.adjoint_matvec(d, lam)
    y64 = host(P.matvec_adjoint(dev(lam).contiguous(), prec=V.VSIE_FP64))
    y32 = host(P.matvec_adjoint(dev(lam).contiguous(), prec=V.VSIE_FP32))
    e64, e32 = parity_err(y64, ref), parity_err(y32, ref)
    say("  rel err fp64 %.3e fp32 %.3e" % (e64, e32))
    assert e64 <= TOL64 and e32 <= TOL32


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", CASES)
def test_adjoint_one_column(V, name, prec):
    """One-column adjoint products on the once-per-pair kernels (the symmetric
    kernel with charges conj(lambda) and, with grad-alpha cells (lognormal),
    the targets' weights inside; the cell-face kernel's adjoint variant; faces
    without a double-layer weight (single) enter with v' = 0), against the
    oracle and against the one-sided kernels."""
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    tol = TOL64 if prec == "fp64" else TOL32
    lam = W.seeded_complex(d.n, seed=13)
    ref = O.adjoint_matvec(d, lam[:, None])[:, 0]
    P.set_tuning(cell_face=0)
    y0 = host(P.matvec_adjoint(dev(lam), prec=pr))
    P.set_tuning(cell_face=1)
    P.profile(True)
    y = host(P.matvec_adjoint(dev(lam), prec=pr))
    st = P.kernel_stats()
    P.profile(False)
    pairs = ("cell_face_" + prec) in st
    e, e0 = parity_err(y, ref), parity_err(y, y0)
    say("  adjoint one column %s %s: once per pair %s, rel err %.2e, vs one-sided %.2e" % (name, prec, pairs, e, e0))
    assert pairs
    assert e <= tol and e0 <= 2 * tol
    # groups of 8 tiles (what the library picks for the largest meshes)
    P.set_tuning(sym_groups=8)
    y8 = host(P.matvec_adjoint(dev(lam), prec=pr))
    P.set_tuning(sym_groups=4)
    assert parity_err(y8, ref) <= tol
    if name in ("c0", "lognormal"):
        # an adjoint solve through the same path, against LU
        import scipy.linalg as sla
        b = W.seeded_complex(d.n, seed=14)
        xs, info = P.solve(dev(b), prec=pr, adjoint=True, tol=1e-11)
        es = parity_err(host(xs), sla.solve(O.assemble(d).conj().T, b))
        say("  adjoint solve %s %s: %d iterations, rel err %.2e" % (name, prec, info["iterations"], es))
        assert info["status"] == V.VSIE_OK and es <= TOL_SOLVE
    P.close()


def test_homogeneous_medium_is_identity(V):
    say("homogeneous medium")
    mesh = W.nested_balls(8)
    mat = W.materials_piecewise(mesh, 1.3, 0.7, 1.3, 0.7, 1.3, 0.7)
    P = V.Problem.from_mesh(mesh, mat, [3.0])
    x = W.seeded_complex(mesh.n, seed=3)
    for prec in (V.VSIE_FP64, V.VSIE_FP32):
        assert np.array_equal(host(P.matvec(dev(x), prec=prec)), x)


def test_multi_frequency_weights(V):
    say("multi-frequency problem")
    mesh, mat, _ = case("lognormal")
    ks = [2.0, 5.0, 7.5]
    P = V.Problem.from_mesh(mesh, mat, ks)
    x = W.seeded_complex(mesh.n, seed=4)
    for f, k in enumerate(ks):
        ref = O.matvec(O.discretise(mesh, mat, k), x)
        assert parity_err(host(P.matvec(dev(x), f=f)), ref) <= TOL64


def test_field_and_source_sums(V):
    say("field and source sums")
    mesh, mat, k0 = case("lognormal")
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    p = W.seeded_complex((d.n, 2), seed=5)
    rec = W.fibonacci_sphere(64, 2.5)
    ref = O.offdiag_apply(d, p, targets=rec, exclude_self=False)
    got = host(P.field(rec, dev(p).contiguous()))
    assert parity_err(got, ref) <= TOL64
    # collocation targets
    z, Z = P.source_sums(dev(p).contiguous())
    zr, Zr = O.source_sums(d, p)
    assert parity_err(host(z), zr) <= TOL64
    Zg = Z.cpu().numpy().transpose(2, 1, 0)   # (n, 3, R)
    assert parity_err(Zg, Zr) <= TOL64
    # receiver targets
    rho = W.seeded_complex((64, 2), seed=6)
    z, Z = P.source_sums(dev(rho).contiguous(), targets=rec)
    zr, Zr = O.source_sums(d, rho, targets=rec, exclude_self=False)
    assert parity_err(host(z), zr) <= TOL64
    assert parity_err(Z.cpu().numpy().transpose(2, 1, 0), Zr) <= TOL64


def test_plane_wave(V):
    mesh, mat, k0 = case("c0")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    dirs = W.fibonacci_sphere(5)
    b = host(P.plane_wave(dirs))
    ref = O.plane_wave(mesh.points(), k0, dirs)
    assert parity_err(b, ref) <= 1e-14


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_c0_against_oracle_lu(V, prec):
    say("solve c0", prec)
    mesh, mat, k0s, dirs, _ = W.config_problem("c0")
    d = O.discretise(mesh, mat, k0s[0])
    b = O.plane_wave(d.pts, k0s[0], dirs[0])
    p_ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, k0s)
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    x, info = P.solve(dev(b), prec=pr, tol=1e-10)
    err = parity_err(host(x), p_ref)
    say("  info", info, "err %.3e" % err)
    assert info["status"] == V.VSIE_OK and info["rel_residual"] <= 1e-10
    assert err <= TOL_SOLVE


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_solve(V, prec):
    say("adjoint solve", prec)
    mesh, mat, k0 = case("lognormal")
    d = O.discretise(mesh, mat, k0)
    b = W.seeded_complex(d.n, seed=8)
    import scipy.linalg as sla
    ref = sla.solve(O.assemble(d).conj().T, b)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    x, info = P.solve(dev(b), prec=pr, adjoint=True, tol=1e-10)
    assert info["status"] == V.VSIE_OK
    assert parity_err(host(x), ref) <= TOL_SOLVE


def test_multi_rhs_solve_and_restart(V):
    say("multi-rhs solve with short restarts")
    mesh, mat, k0 = case("ragged")
    d = O.discretise(mesh, mat, k0)
    dirs = W.fibonacci_sphere(3)
    b = O.plane_wave(d.pts, k0, dirs)
    ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x, info = P.solve(dev(b).contiguous(), prec=V.VSIE_FP64, tol=1e-11, restart=5)
    assert info["status"] == V.VSIE_OK
    assert parity_err(host(x), ref) <= TOL_SOLVE


def test_solver_reports_nonconvergence(V):
    mesh, mat, k0 = case("c0")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    b = P.plane_wave([0.0, 0.0, 1.0])
    x, info = P.solve(b, tol=1e-12, max_iter=2, restart=2, allow_noconv=True)
    assert info["status"] == V.VSIE_E_NOCONV and info["iterations"] == 2
    import torch
    assert torch.isfinite(torch.view_as_real(x)).all()


# ---------------------------------------------------------------------------
# full-size c1 (n = 71,368): sampled rows and the stored oracle solution

GOLD = os.path.join(os.path.dirname(__file__), "golden", "c1_oracle_solution.npz")


@pytest.fixture(scope="module")
def c1(V):
    mesh, mat, k0s, dirs, _ = W.config_problem("c1")
    return mesh, mat, k0s, dirs, V.Problem.from_mesh(mesh, mat, k0s)


def test_c1_matvec_sampled_rows(V, c1):
    mesh, mat, k0s, dirs, P = c1
    say("c1 matvec, sampled rows, n", P.n)
    d = O.discretise(mesh, mat, k0s[0])
    x = W.seeded_complex((d.n, 2), seed=21)
    rows = np.sort(np.random.default_rng(22).choice(d.n, 384, replace=False))
    rows = np.unique(np.concatenate([rows, [0, d.n_vol - 1, d.n_vol, d.n - 1]]))
    ref = O.matvec(d, x, rows=rows)
    y64 = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP64))[rows]
    y32 = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP32))[rows]
    e64, e32 = parity_err(y64, ref), parity_err(y32, ref)
    say("  rel err fp64 %.3e fp32 %.3e" % (e64, e32))
    assert e64 <= TOL64 and e32 <= TOL32


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c1_one_column_sampled_rows(V, c1, prec):
    """One random column at full c1 size: the once-per-pair kernels the
    headline solve runs (symmetric cell-cell single layer, cell-face pairs,
    face-face double layers), against the oracle on sampled rows."""
    mesh, mat, k0s, dirs, P = c1
    d = O.discretise(mesh, mat, k0s[0])
    x = W.seeded_complex(d.n, seed=24)
    rows = sample_rows(d.n, d.n_vol, 512, 25)
    ref = O.matvec(d, x[:, None], rows=rows)[:, 0]
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    P.profile(True)
    y = host(P.matvec(dev(x), prec=pr))[rows]
    st = P.kernel_stats()
    P.profile(False)
    e = parity_err(y, ref)
    say("c1 one column %s, %d sampled rows: rel err %.3e, kernels %s" % (prec, rows.size, e, sorted(st)))
    for kind in ("sym_single_layer_", "cell_face_", "face_face_"):
        assert (kind + prec) in st
    assert e <= (TOL64 if prec == "fp64" else TOL32)


@pytest.mark.skipif(not os.path.exists(GOLD), reason="c1 oracle solution not generated")
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_c1_solve_against_oracle_solution(V, c1, prec):
    mesh, mat, k0s, dirs, P = c1
    say("c1 solve", prec)
    g = np.load(GOLD)
    b = P.plane_wave(dirs[0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    x, info = P.solve(b, prec=pr, tol=1e-10)
    err = parity_err(host(x), g["p"])
    d = O.discretise(mesh, mat, k0s[0])
    res = oracle_residual(d, host(x), host(b), sample_rows(d.n, d.n_vol, 256, 26))
    say("  info", info, "err vs oracle %.3e, oracle residual on sampled rows %.2e" % (err, res))
    assert info["status"] == V.VSIE_OK
    assert err <= TOL_SOLVE and res <= 1e-9


# ---------------------------------------------------------------------------
# the other full-size workloads: sampled rows of the operator

def _sampled_rows(V, name, R, n_rows, f=0, seed=51):
    mesh, mat, k0s, dirs, _ = W.config_problem(name)
    say(name, "sampled rows: n", mesh.n, "R", R, "k0", k0s[f])
    d = O.discretise(mesh, mat, k0s[f])
    P = V.Problem.from_mesh(mesh, mat, k0s)
    x = W.seeded_complex((d.n, R), seed=seed)
    rng = np.random.default_rng(seed + 1)
    rows = np.unique(np.concatenate([rng.choice(d.n, n_rows, replace=False),
                                     [0, d.n_vol - 1, d.n_vol, d.n - 1]]))
    ref = O.matvec(d, x, rows=rows)
    out = {}
    for nm, pr in (("fp64", V.VSIE_FP64), ("fp32", V.VSIE_FP32)):
        y = host(P.matvec(dev(x).contiguous(), f=f, prec=pr)).reshape(d.n, R)[rows]
        out[nm] = parity_err(y, ref)
    say("  rel err fp64 %.3e fp32 %.3e" % (out["fp64"], out["fp32"]))
    P.close()
    return out


def test_c2_matvec_sampled_rows(V):
    e = _sampled_rows(V, "c2", 4, 256)
    assert e["fp64"] <= TOL64 and e["fp32"] <= TOL32


@pytest.mark.parametrize("f", [0, 7])
def test_c4_matvec_sampled_rows(V, f):
    """Cube + ellipsoid on a 100^3 grid, n = 1,076,336, at k0 = 40 and 26."""
    e = _sampled_rows(V, "c4", 2, 192, f=f)
    assert e["fp64"] <= TOL64 and e["fp32"] <= TOL32


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_solve_mixed_columns(V, prec):
    """One batch holding two plane waves, a zero column and a random column,
    with a nonzero initial guess in one column and short restarts."""
    import torch
    say("batched solve, mixed columns", prec)
    mesh, mat, k0 = case("lognormal")
    d = O.discretise(mesh, mat, k0)
    b = np.concatenate([O.plane_wave(d.pts, k0, W.fibonacci_sphere(2)),
                        np.zeros((d.n, 1)), W.seeded_complex((d.n, 1), seed=61)], axis=1)
    ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x0 = np.zeros_like(b)
    x0[:, 1] = 0.9 * ref[:, 1] + 0.01
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    x, info = P.solve(dev(b).contiguous(), prec=pr, tol=1e-11, restart=12, x0=dev(x0).contiguous())
    say("  info", info)
    got = host(x)
    assert info["status"] == V.VSIE_OK
    assert np.all(got[:, 2] == 0)
    for c in (0, 1, 3):
        assert parity_err(got[:, c], ref[:, c]) <= TOL_SOLVE


# ---------------------------------------------------------------------------
# assembled FP32 operator (complex GEMM path)

@pytest.mark.parametrize("name", ["c0", "lognormal", "cube"])
def test_dense_fp32_operator(V, name):
    say("dense FP32 operator", name)
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    A = P.assemble_dense(0, ld=d.n + 5)          # padded leading dimension
    x = W.seeded_complex((d.n, 3), seed=71)
    e = parity_err(host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP32)), O.matvec(d, x))
    ea = parity_err(host(P.matvec_adjoint(dev(x).contiguous(), prec=V.VSIE_FP32)),
                     O.adjoint_matvec(d, x))
    # FP64 products keep using the matrix-free kernels
    e64 = parity_err(host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP64)), O.matvec(d, x))
    say("  rel err dense fp32 %.3e adjoint %.3e fp64 %.3e" % (e, ea, e64))
    assert e <= TOL32 and ea <= TOL32 and e64 <= TOL64
    b = O.plane_wave(d.pts, k0, W.fibonacci_sphere(3))
    xs, info = P.solve(dev(b).contiguous(), prec=V.VSIE_FP32, tol=1e-10)
    assert info["status"] == V.VSIE_OK
    assert parity_err(host(xs), O.solve_lu(d, b)) <= TOL_SOLVE
    del A


def test_c2_dense_sampled_rows(V):
    """The c2 operator assembled in FP32 (n = 116,445: 108.5 GB), 4 columns."""
    import torch
    mesh, mat, k0s, dirs, _ = W.config_problem("c2")
    d = O.discretise(mesh, mat, k0s[0])
    P = V.Problem.from_mesh(mesh, mat, k0s)
    say("c2 dense: n", d.n, "bytes %.1f GB" % (8.0 * d.n * d.n / 1e9))
    A = P.assemble_dense(0)
    x = W.seeded_complex((d.n, 4), seed=72)
    rows = np.unique(np.concatenate([np.random.default_rng(73).choice(d.n, 256, replace=False),
                                     [0, d.n_vol - 1, d.n_vol, d.n - 1]]))
    ref = O.matvec(d, x, rows=rows)
    y = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP32))[rows]
    e = parity_err(y, ref)
    say("  rel err dense fp32 %.3e" % e)
    assert e <= TOL32
    # the batched form of the workload: 128 Fibonacci directions by block
    # GMRES on the assembled FP32 operator inside FP64 refinement; the oracle
    # computes the residual of 4 of the solutions on sampled rows
    b = P.plane_wave(dirs)
    assert b.shape[0] == 128
    xs, info = P.solve(b, prec=V.VSIE_FP32, tol=1e-10, block=True)
    say("  c2 block solve, 128 directions:", info)
    assert info["status"] == V.VSIE_OK
    cols = [0, 41, 86, 127]
    res = oracle_residual(d, host(xs[cols].contiguous()), host(b[cols].contiguous()), rows)
    say("  oracle residual of directions %s on %d rows: %.2e" % (cols, rows.size, res))
    assert res <= 1e-9
    P.release_dense(0)
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("restart", [2, 100])
def test_block_gmres(V, prec, restart):
    """Block GMRES over 6 columns (plane waves, a random column, a zero column)
    against LU; restart=2 forces several block cycles."""
    say("block gmres", prec, "restart", restart)
    mesh, mat, k0 = case("lognormal")
    d = O.discretise(mesh, mat, k0)
    b = np.concatenate([O.plane_wave(d.pts, k0, W.fibonacci_sphere(4)),
                        W.seeded_complex((d.n, 1), seed=81), np.zeros((d.n, 1))], axis=1)
    ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    # every short FP32 cycle is one refinement step: allow as many as the FP64 run needs cycles
    x, info = P.solve(dev(b).contiguous(), prec=pr, tol=1e-11, restart=restart, block=True,
                      max_outer=400)
    say("  info", info)
    got = host(x)
    assert info["status"] == V.VSIE_OK
    assert np.all(got[:, 5] == 0)
    assert parity_err(got[:, :5], ref[:, :5]) <= TOL_SOLVE


@pytest.mark.parametrize("R", [12, 24, 40])
def test_block_gmres_widths(V, R):
    """Block widths on each path of the tall block products: 12 and 24
    columns on the hand-written kernels (two and four groups of 8 columns,
    ragged), 40 on rocBLAS; FP32 + refinement with short cycles (restarts and
    block deflation) against LU, on c0 (n = 3,736: 14 row slabs)."""
    mesh, mat, k0 = case("c0")
    d = O.discretise(mesh, mat, k0)
    b = np.concatenate([O.plane_wave(d.pts, k0, W.fibonacci_sphere(R - 2)),
                        W.seeded_complex((d.n, 2), seed=83)], axis=1)
    ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x, info = P.solve(dev(b).contiguous(), prec=V.VSIE_FP32, tol=1e-11, restart=6, block=True, max_outer=400)
    e = parity_err(host(x), ref)
    say("  block width %d: %s, rel err vs LU %.2e" % (R, info, e))
    assert info["status"] == V.VSIE_OK
    assert e <= TOL_SOLVE
    P.close()


@pytest.mark.parametrize("R", [8, 40])
def test_block_lookahead_keeps_results(V, capfd, R):
    """Far from convergence the block solver queues the next product before
    the host QR; progress mode turns that off.  Both runs must give the same
    iterations and bit-identical solutions (8 columns: device CholeskyQR; 40:
    the host's)."""
    import torch
    mesh, mat, k0 = case("c0")
    d = O.discretise(mesh, mat, k0)
    b = np.concatenate([O.plane_wave(d.pts, k0, W.fibonacci_sphere(R - 1)),
                        W.seeded_complex((d.n, 1), seed=84)], axis=1)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    runs = []
    for progress in (False, True):
        x, info = P.solve(dev(b).contiguous(), prec=V.VSIE_FP32, tol=1e-11, block=True, progress=progress)
        runs.append((x, info))
    err = capfd.readouterr().err
    assert "block step" in err
    (x0, i0), (x1, i1) = runs
    say("  width %d: %s / %s" % (R, i0, i1))
    assert i0 == i1
    assert torch.equal(x0, x1)
    assert parity_err(host(x0), O.solve_lu(d, b)) <= TOL_SOLVE
    P.close()


def test_block_gmres_dense_adjoint(V):
    say("block gmres, assembled FP32, adjoint")
    mesh, mat, k0 = case("cube")
    d = O.discretise(mesh, mat, k0)
    b = W.seeded_complex((d.n, 3), seed=82)
    import scipy.linalg as sla
    ref = sla.solve(O.assemble(d).conj().T, b)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    A = P.assemble_dense(0)
    x, info = P.solve(dev(b).contiguous(), prec=V.VSIE_FP32, adjoint=True, tol=1e-11, block=True)
    assert info["status"] == V.VSIE_OK
    assert parity_err(host(x), ref) <= TOL_SOLVE
    del A


# ---------------------------------------------------------------------------
# hipGraph replay of the operator applications inside the solver

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_solve(V, prec):
    """With tuning graph=1 every operator application of the solve after the
    first is a replay of a captured hipGraph, with the solver's own eager
    kernels and host synchronisations between replays.  The graph holds the
    same kernels in the same order, so solves must match the eager ones
    bitwise, over several solves in a row (forward, adjoint, the matrix-core
    path); new materials and tuning changes must retire the graphs."""
    import time
    import torch
    say("graph replay", prec)
    mesh, mat, k0 = case("lognormal")
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    b = P.plane_wave(W.fibonacci_sphere(3))
    P.set_tuning(graph=0)
    t0 = time.perf_counter()
    x0, i0 = P.solve(b, prec=pr, tol=1e-11, restart=20)
    a0, j0 = P.solve(b, prec=pr, adjoint=True, tol=1e-11)
    torch.cuda.synchronize()
    te = time.perf_counter() - t0
    P.set_tuning(graph=1)
    for rep in range(3):
        t0 = time.perf_counter()
        x1, i1 = P.solve(b, prec=pr, tol=1e-11, restart=20)
        a1, j1 = P.solve(b, prec=pr, adjoint=True, tol=1e-11)
        torch.cuda.synchronize()
        say("  replay %d: eager %.1f ms, graph %.1f ms" % (rep, te * 1e3, (time.perf_counter() - t0) * 1e3))
        assert i1 == i0 and j1 == j0
        assert torch.equal(x1, x0) and torch.equal(a1, a0)
    # one column: the once-per-pair kernels with the cells' adjoint double
    # layers (every cell has grad alpha here), captured and replayed
    b1 = b[0].contiguous()
    P.set_tuning(graph=0)
    s0, l0 = P.solve(b1, prec=pr, tol=1e-11)
    P.set_tuning(graph=1)
    for rep in range(3):
        s1, l1 = P.solve(b1, prec=pr, tol=1e-11)
        assert l1 == l0 and torch.equal(s1, s0)
    assert parity_err(host(s1), O.solve_lu(d, host(b1))) <= TOL_SOLVE
    # new materials: graphs captured for the old sources must not be replayed
    mat2 = W.materials_piecewise(mesh, 1.0, 1.0, 1.3, 1.4, 1.9, 0.9)
    P.set_materials(torch.as_tensor(mat2.vol_rho, device="cuda"), torch.as_tensor(mat2.vol_c, device="cuda"))
    d2 = O.discretise(mesh, mat2, k0)
    x2, _ = P.solve(b, prec=pr, tol=1e-11)
    assert parity_err(host(x2), O.solve_lu(d2, host(b))) <= TOL_SOLVE
    # blocks of 8 columns: the matrix-core path on FP32, captured as well
    b8 = P.plane_wave(W.fibonacci_sphere(8))
    P.set_tuning(graph=0)
    y0, k_0 = P.solve(b8, prec=pr, tol=1e-11)
    P.set_tuning(graph=1)
    for rep in range(2):
        y1, k_1 = P.solve(b8, prec=pr, tol=1e-11)
        assert k_1 == k_0 and torch.equal(y1, y0)
    assert parity_err(host(y1), O.solve_lu(d2, host(b8))) <= TOL_SOLVE
    P.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graphs_survive_material_updates_of_the_same_structure(V, prec):
    """New per-cell materials with the same source structure (every cell a
    single-layer source, every cell with grad alpha, every face weighted)
    rewrite the weights in place and keep the captured operator graphs.  The
    replayed solves after each update must equal, bitwise, the eager solves of
    a second problem given the same updates, and match the oracle's LU
    solution of the new materials."""
    import copy
    import torch
    mesh, mat, k0 = case("lognormal")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    Q = V.Problem.from_mesh(mesh, mat, [k0])
    Q.set_tuning(graph=0)
    b1 = P.plane_wave(W.fibonacci_sphere(1))[0].contiguous()
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    P.solve(b1, prec=pr, tol=1e-11)           # captures the operator graphs
    for scale in (1.05, 0.97):
        m2 = copy.deepcopy(mat)
        m2.vol_c = m2.vol_c * scale
        m2.vol_rho = m2.vol_rho * (2.0 - scale)
        for prob in (P, Q):
            prob.set_materials(torch.as_tensor(m2.vol_rho, device="cuda"), torch.as_tensor(m2.vol_c, device="cuda"))
        x, info = P.solve(b1, prec=pr, tol=1e-11)
        xe, ie = Q.solve(b1, prec=pr, tol=1e-11)
        d2 = O.discretise(mesh, m2, k0)
        e = parity_err(host(x), O.solve_lu(d2, host(b1)))
        say("  %s scale %.2f: %s, vs LU %.2e" % (prec, scale, info, e))
        assert info == ie and torch.equal(x, xe)
        assert e <= TOL_SOLVE
    P.close()
    Q.close()


def test_material_updates_keep_or_rebuild_sources(V):
    """A sequence of material updates on one problem: grad-alpha cells
    disappear (the double-layer sources are rebuilt), come back (rebuilt), then
    change value with the same pattern (the sources keep their arrays and take
    the new v'), then only the sound speed changes.  After every update the
    one-column forward product in both precisions and the FP64 adjoint match
    the oracle built from the same materials."""
    import dataclasses
    import torch
    mesh, mat, k0 = case("lognormal")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x = W.seeded_complex(mesh.n, seed=131)
    flat = W.materials_piecewise(mesh, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8)
    steps = [("initial", mat), ("piecewise constant", flat),
             ("log-normal again", dataclasses.replace(mat, vol_rho=mat.vol_rho * 1.05)),
             ("same pattern, new rho", dataclasses.replace(mat, vol_rho=mat.vol_rho * 1.1)),
             ("new c only", dataclasses.replace(mat, vol_rho=mat.vol_rho * 1.1, vol_c=mat.vol_c * 1.07))]
    for label, m in steps:
        if m is not mat:
            P.set_materials(torch.as_tensor(m.vol_rho, device="cuda"), torch.as_tensor(m.vol_c, device="cuda"))
        d = O.discretise(mesh, m, k0)
        ref = O.matvec(d, x[:, None])[:, 0]
        ref_adj = O.adjoint_matvec(d, x)
        e64 = parity_err(host(P.matvec(dev(x), prec=V.VSIE_FP64)), ref)
        e32 = parity_err(host(P.matvec(dev(x), prec=V.VSIE_FP32)), ref)
        say("  %s: fp64 %.2e fp32 %.2e" % (label, e64, e32))
        assert e64 <= TOL64 and e32 <= TOL32
        ea = parity_err(host(P.matvec_adjoint(dev(x), prec=V.VSIE_FP64)), ref_adj)
        say("    adjoint fp64 %.2e" % ea)
        assert ea <= TOL64
    P.close()


def test_graph_small_problem_timing(V):
    """c0 (n = 3,736), FP64 and FP32: solve time with and without graphs
    (reported), identical solutions."""
    import time
    import torch
    mesh, mat, k0s, dirs, _ = W.config_problem("c0")
    P = V.Problem.from_mesh(mesh, mat, k0s)
    b = P.plane_wave(dirs[0])
    for pr in (V.VSIE_FP64, V.VSIE_FP32):
        res = {}
        for g in (0, 1):
            P.set_tuning(graph=g)
            x, info = P.solve(b, prec=pr, tol=1e-10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                x, info = P.solve(b, prec=pr, tol=1e-10)
            torch.cuda.synchronize()
            res[g] = ((time.perf_counter() - t0) / 3, x)
        say("  c0 prec %d: eager %.2f ms, graph %.2f ms (%d iterations)"
            % (pr, res[0][0] * 1e3, res[1][0] * 1e3, info["iterations"]))
        assert torch.equal(res[0][1], res[1][1])
    P.close()


# ---------------------------------------------------------------------------
# cell-cell single layer evaluated once per unordered pair (one column)

@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_symmetric_single_layer(V, name, prec):
    """One-column products with the symmetric cell-cell kernel, for every group
    size, against the oracle and against the one-sided kernels; ragged tiles
    (no case has a multiple of 64 cells) and the padding lanes included."""
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    tol = TOL64 if prec == "fp64" else TOL32
    x = W.seeded_complex(d.n, seed=95)
    ref = O.matvec(d, x[:, None])[:, 0]
    P.set_tuning(sym_groups=0)
    y0 = host(P.matvec(dev(x), prec=pr))
    for g in (2, 4, 8):
        P.set_tuning(sym_groups=g)
        P.profile(True)
        y = host(P.matvec(dev(x), prec=pr))
        st = P.kernel_stats()
        P.profile(False)
        e, e0 = parity_err(y, ref), parity_err(y, y0)
        say("  %s %s groups %d: n_vol %d rel err %.2e, vs one-sided %.2e" % (name, prec, g, mesh.n_vol, e, e0))
        assert ("sym_single_layer_" + prec) in st
        assert e <= tol and e0 <= 2 * tol
    P.close()


def test_symmetric_kernel_falls_back_when_some_cells_have_no_single_layer(V):
    """Shell sound speed equal to c0: its cells carry no single-layer weight, so
    the cells are not all single-layer sources and the one-sided kernels run."""
    mesh = W.nested_balls(9)
    mat = W.materials_piecewise(mesh, 1.0, 1.0, 1.3, 1.0, 2.0, 0.8)
    d = O.discretise(mesh, mat, 3.0)
    assert np.any(d.sV == 0) and np.any(d.sV != 0)
    P = V.Problem.from_mesh(mesh, mat, [3.0])
    x = W.seeded_complex(d.n, seed=96)
    P.profile(True)
    y = host(P.matvec(dev(x), prec=V.VSIE_FP64))
    st = P.kernel_stats()
    P.profile(False)
    assert not any(k.startswith("sym_") for k in st)
    assert parity_err(y, O.matvec(d, x[:, None])[:, 0]) <= TOL64
    P.close()


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cell_face_pairs(V, name, prec):
    """One-column products with the cell-face pairs evaluated once per pair (the
    single layer and the adjoint double layer of the cell at the face, the
    double layer of the face at the cell), the cells' adjoint double layers
    alongside the cell-cell single layer (lognormal: every cell has grad
    alpha) and the face-face double layers once per pair (single: the Gamma_2
    faces carry no jump, so their v' is zero), against the oracle and against
    the separate one-sided kernels."""
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    tol = TOL64 if prec == "fp64" else TOL32
    x = W.seeded_complex(d.n, seed=97)
    ref = O.matvec(d, x[:, None])[:, 0]
    P.set_tuning(cell_face=0)
    y0 = host(P.matvec(dev(x), prec=pr))
    P.set_tuning(cell_face=1)
    P.profile(True)
    y = host(P.matvec(dev(x), prec=pr))
    st = P.kernel_stats()
    P.profile(False)
    fused = ("cell_face_" + prec) in st
    e, e0 = parity_err(y, ref), parity_err(y, y0)
    say("  %s %s fused %s: rel err %.2e, vs separate kernels %.2e" % (name, prec, fused, e, e0))
    assert fused
    # the face-face double layers run once per pair on the symmetric kernel
    # (ordered face pairs), with no one-sided double-layer launch
    assert st["face_face_" + prec]["pairs"] == float(mesh.n_srf) * (mesh.n_srf - 1)
    assert ("fwd_double_layers_" + prec) not in st
    assert e <= tol and e0 <= 2 * tol
    P.close()


@pytest.mark.parametrize("name", ["c0", "lognormal", "cube"])
def test_relaxed_products_solve(V, name):
    """FP32 solves with relaxed products (FP64 operator while the residual is
    high, FP32 after the switch point) reach the oracle's dense solution; both
    operators are used, and a looser relax switches to FP32 no later."""
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    b = O.plane_wave(d.pts, k0, W.fibonacci_sphere(2))
    ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    infos = []
    for relax in (1e-7, 1e-5):
        x, info = P.solve(dev(b).contiguous(), prec=V.VSIE_FP32, tol=1e-11, relax=relax)
        say("  %s relax %.0e: %s" % (name, relax, info))
        assert info["status"] == V.VSIE_OK
        assert info["matvecs_fp64"] > 2 and info["matvecs_fp32"] > 0
        assert parity_err(host(x), ref) <= TOL_SOLVE
        infos.append(info)
    assert infos[1]["matvecs_fp64"] >= infos[0]["matvecs_fp64"]
    P.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_block_solve_with_dependent_right_hand_sides(V, prec):
    """Block GMRES whose right-hand sides are linearly dependent: an exact
    duplicate (the first block's Gram matrix is singular, so the Cholesky
    factorisation of CholeskyQR needs its diagonal shift) and a column that
    differs from another by 1e-9.  Every column must still reach the oracle's
    LU solution."""
    mesh, mat, k0 = case("ragged")
    d = O.discretise(mesh, mat, k0)
    b0 = O.plane_wave(d.pts, k0, W.fibonacci_sphere(3))
    b = np.stack([b0[:, 0], b0[:, 1], b0[:, 0], b0[:, 2], b0[:, 1] + 1e-9 * W.seeded_complex(d.n, seed=96)], axis=1)
    ref = O.solve_lu(d, b)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    x, info = P.solve(dev(b).contiguous(), prec=pr, tol=1e-10, block=True)
    e = parity_err(host(x), ref)
    say("  dependent columns, %s: %s, vs LU %.2e" % (prec, info, e))
    assert info["status"] == V.VSIE_OK and e <= TOL_SOLVE
    P.close()
