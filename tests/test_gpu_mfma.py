"""Matrix-core (MFMA) FP32 forward products, the multi-frequency launch and the
autotuner, against the FP64 oracle and the vector pair kernel, through the C ABI.

Bar: FP32 operator <= 1e-5 relative to the oracle (2-norm over all entries).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_cases import CASES, case, dev, host, say, parity_err

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12
VARIANTS = [(2, 1), (4, 1), (2, 2), (4, 2)]


@pytest.fixture(scope="module")
def V():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2607_06429_amd as V
    return V


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("R", [8, 16, 33])
def test_mfma_matvec_parity(V, name, R):
    """Every kernel variant (four or three real products per complex
    multiply-add), ragged column counts (33 = two full blocks + 1) and ragged
    target tiles (every case has n not a multiple of 64)."""
    say("mfma matvec", name, "R", R)
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x = W.seeded_complex((d.n, R), seed=91)
    ref = O.matvec(d, x)
    P.set_tuning(mfma_min_rhs=0)
    yv = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP32)).reshape(d.n, R)
    ev = parity_err(yv, ref)
    for tg, nb in VARIANTS:
        for ipw, m3 in ((1, 0), (16, 0), (1, 1), (16, 1)):
            P.set_tuning(mfma_min_rhs=8, mfma_tg=tg, mfma_nb=nb, items_per_wave=ipw, mfma_3m=m3)
            P.profile(True)
            y = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP32)).reshape(d.n, R)
            st = P.kernel_stats()
            P.profile(False)
            e = parity_err(y, ref)
            say("  tg %d nb %d ipw %2d 3m %d: rel err %.3e (vector kernel %.3e), vs vector %.3e"
                % (tg, nb, ipw, m3, e, ev, parity_err(y, yv)))
            assert "mfma_fwd_single_layer_fp32" in st and "fwd_single_layer_fp32" not in st
            assert e <= TOL32
            assert parity_err(y, yv) <= 2 * TOL32
    P.close()


def test_mfma_zero_and_unit_columns(V):
    """A zero column gives exactly the zero vector; a unit vector e_j gives
    column j of A (oracle assembly) to the FP32 bar."""
    mesh, mat, k0 = case("lognormal")
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x = np.zeros((d.n, 8), dtype=complex)
    cols = [0, d.n_vol - 1, d.n_vol, d.n - 1]
    for c, j in enumerate(cols):
        x[j, c + 1] = 1.0
    y = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP32))
    assert np.all(y[:, 0] == 0)
    A = O.assemble(d)
    for c, j in enumerate(cols):
        assert parity_err(y[:, c + 1], A[:, j]) <= TOL32


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matvec_multi_frequency(V, prec):
    """Three frequencies in one call (one launch per source class
    on the FP32 path), each block against the oracle of its frequency."""
    mesh, mat, _ = case("cube")
    ks = [12.0, 9.5, 4.0]
    R = 16
    P = V.Problem.from_mesh(mesh, mat, ks)
    x = W.seeded_complex((mesh.n, R * len(ks)), seed=92)
    pr = V.VSIE_FP64 if prec == "fp64" else V.VSIE_FP32
    P.profile(True)
    y = host(P.matvec_multi(dev(x).contiguous(), f0=0, nf=len(ks), prec=pr))
    st = P.kernel_stats()
    P.profile(False)
    if prec == "fp32":
        assert st["mfma_fwd_single_layer_fp32"]["launches"] == 1
    for t, k in enumerate(ks):
        d = O.discretise(mesh, mat, k)
        blk = slice(t * R, (t + 1) * R)
        e = parity_err(y[:, blk], O.matvec(d, x[:, blk]))
        say("  %s k0 %.1f rel err %.3e" % (prec, k, e))
        assert e <= (1e-12 if prec == "fp64" else TOL32)
    # a sub-range of the frequencies
    y2 = host(P.matvec_multi(dev(x[:, R:]).contiguous(), f0=1, nf=2, prec=pr))
    assert np.allclose(y2, y[:, R:], rtol=0, atol=1e-12 * np.abs(y).max())


def test_c4_multi_frequency_sampled_rows(V):
    """Cube + ellipsoid on the 100^3 grid (n = 1,076,336): 8 frequencies x 16
    plane-wave incidences in one multi-frequency FP32 product; sampled rows of
    every frequency against the oracle.  Then one column in FP64 and FP32 on
    the once-per-pair kernels at this size."""
    import torch
    mesh, mat, k0s, dirs, _ = W.config_problem("c4")
    say("c4 multi-frequency: n", mesh.n, "k0", k0s)
    P = V.Problem.from_mesh(mesh, mat, k0s)
    R = dirs.shape[0]
    X = torch.cat([P.plane_wave(dirs, f=f) for f in range(len(k0s))], dim=0).contiguous()
    Y = P.matvec_multi(X, f0=0, nf=len(k0s), prec=V.VSIE_FP32)
    rows = np.unique(np.concatenate([np.random.default_rng(93).choice(mesh.n, 96, replace=False),
                                     [0, mesh.n_vol - 1, mesh.n_vol, mesh.n - 1]]))
    for f, k in enumerate(k0s):
        d = O.discretise(mesh, mat, k)
        xf = host(X[f * R:(f + 1) * R])
        ref = O.matvec(d, xf, rows=rows)
        e = parity_err(host(Y[f * R:(f + 1) * R])[rows], ref)
        say("  k0 %.0f: rel err %.3e" % (k, e))
        assert e <= TOL32
    # one column at this size in both precisions: the once-per-pair kernels,
    # with cell groups of 8 tiles so that their slot partials stay within
    # the cap (about 3.2e9 partials: 52 GB in FP64, against 83 GB with the
    # default groups of 4)
    d = O.discretise(mesh, mat, k0s[0])
    x1 = host(X[:1])
    ref1 = O.matvec(d, x1.reshape(-1, 1), rows=rows)[:, 0]
    ws = P.workspace_size(V.VSIE_OP_MATVEC, nrhs=1, prec=V.VSIE_FP64)
    say("  one-column FP64 workspace %.1f GB" % (ws / 1e9))
    assert 50e9 < ws < 56e9
    for prec, tol, key in ((V.VSIE_FP64, TOL64, "sym_single_layer_fp64"),
                           (V.VSIE_FP32, TOL32, "sym_single_layer_fp32")):
        P.profile(True)
        y1 = host(P.matvec(X[:1].contiguous(), f=0, prec=prec))
        st = P.kernel_stats()
        P.profile(False)
        e1 = parity_err(y1.reshape(-1)[rows], ref1)
        say("  %s, one column: rel err %.3e, cell-cell %.1f ms, kernels %s"
            % (key[-4:], e1, st[key]["ms"], sorted(st)))
        assert e1 <= tol
        assert not any(k.startswith("fwd_single_layer") for k in st)
    P.close()
    del X, Y
    torch.cuda.empty_cache()


def test_autotune(V):
    """The autotuner returns a valid configuration, installs it, and products
    under it stay within the FP32 bar."""
    mesh, mat, k0 = case("cube")
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    for R in (1, 16):
        t = P.autotune(R)
        say("  autotune R", R, t)
        assert t == P.tuning
        assert t["mfma_tg"] in (2, 4) and t["mfma_nb"] in (1, 2)
        x = W.seeded_complex((d.n, R), seed=94)
        y = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP32)).reshape(d.n, R)
        assert parity_err(y, O.matvec(d, x)) <= TOL32


def test_tuning_validation(V):
    mesh, mat, k0 = case("c0")
    P = V.Problem.from_mesh(mesh, mat, [k0])
    before = P.tuning
    for bad in (dict(mfma_tg=3), dict(mfma_nb=4), dict(items_per_wave=0), dict(vec_target_waves=10),
                dict(mfma_min_rhs=-1), dict(mfma_3m=2)):
        with pytest.raises(V.VsieError):
            P.set_tuning(**bad)
        assert P.tuning == before


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("R", [16, 33, 64])
def test_mfma64_matvec_parity(V, name, R):
    """FP64 products on the FP64 matrix cores (16, 32 or 64 columns per kernel
    evaluation by the width of the block; 33 leaves a ragged last block), with
    three and four real products per complex multiply-add, against the oracle
    at the FP64 bar and against the vector kernel."""
    mesh, mat, k0 = case(name)
    d = O.discretise(mesh, mat, k0)
    P = V.Problem.from_mesh(mesh, mat, [k0])
    x = W.seeded_complex((d.n, R), seed=93)
    ref = O.matvec(d, x)
    P.set_tuning(mfma64_min_rhs=0)
    yv = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP64)).reshape(d.n, R)
    for m3 in (0, 1):
        P.set_tuning(mfma64_min_rhs=16, mfma_3m=m3)
        P.profile(True)
        y = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP64)).reshape(d.n, R)
        st = P.kernel_stats()
        P.profile(False)
        e, ev = parity_err(y, ref), parity_err(y, yv)
        say("  %s R %d 3m %d: rel err %.2e, vs vector kernel %.2e" % (name, R, m3, e, ev))
        assert "mfma_fwd_single_layer_fp64" in st and "fwd_single_layer_fp64" not in st
        assert e <= TOL64 and ev <= TOL64
    P.close()


def test_mfma64_c2_sampled_rows_and_multi_frequency(V):
    """The c2 residual product (n = 116,445, 128 columns) in FP64 on the
    matrix cores against the oracle on sampled rows; and a multi-frequency
    FP64 launch (3 wavenumbers x 16 columns) against per-frequency products."""
    import torch
    mesh, mat, k0s, dirs, _ = W.config_problem("c2")
    d = O.discretise(mesh, mat, k0s[0])
    P = V.Problem.from_mesh(mesh, mat, k0s)
    x = W.seeded_complex((d.n, 128), seed=94)
    rows = np.unique(np.concatenate([np.random.default_rng(95).choice(d.n, 96, replace=False),
                                     [0, d.n_vol - 1, d.n_vol, d.n - 1]]))
    P.profile(True)
    y = host(P.matvec(dev(x).contiguous(), prec=V.VSIE_FP64))
    st = P.kernel_stats()
    P.profile(False)
    cols = [0, 63, 127]
    e = parity_err(y[rows][:, cols], O.matvec(d, x[:, cols], rows=rows))
    say("  c2 FP64 128 columns on the matrix cores: sampled rows rel err %.2e, single layer %.1f ms" %
        (e, st["mfma_fwd_single_layer_fp64"]["ms"]))
    assert e <= TOL64
    P.close()
    mesh, mat, _ = case("lognormal")
    ks = [2.0, 5.0, 7.5]
    P = V.Problem.from_mesh(mesh, mat, ks)
    X = dev(W.seeded_complex((mesh.n, 48), seed=96)).contiguous()
    Y = P.matvec_multi(X, 0, 3, prec=V.VSIE_FP64)
    for f in range(3):
        dd = O.discretise(mesh, mat, ks[f])
        e = parity_err(host(Y[16 * f:16 * (f + 1)].contiguous()), O.matvec(dd, host(X[16 * f:16 * (f + 1)].contiguous())))
        assert e <= TOL64, (f, e)
    P.close()
