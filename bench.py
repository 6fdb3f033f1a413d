"""Benchmark of the nested-VSIE hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Workload (the heterogeneous nested-sphere configuration): concentric balls of
radius 1 and 0.5 on a 48^3 voxel grid over [-1, 1]^3 -- 57,856 cells and
13,512 interface faces, n = 71,368 unknowns -- exterior rho0 = c0 = 1, shell
rho = 1.2, c = 1.5, core rho = 2, c(x) = 0.8 (1 + 0.2 exp(-|x|^2/0.05)),
plane wave along +z with k0 = 10.

One step = the whole hot path once: per-element weights from the per-cell
materials, the plane-wave right-hand side, and the GMRES solve with the FP32
operator inside FP64 iterative refinement to relative residual 1e-10.  The
plain FP64 solve is timed beside it.  Prints one JSON line.

Unless --no-batched is given, the line also carries the batched workloads
(outside the timed steps): 128 plane-wave directions at k0 = 16 on the 57^3
grid (n = 116,445) solved by block GMRES with the assembled FP32 operator,
matrix-free FP32 and matrix-free FP64; the receiver-misfit gradient of the
log-normal medium with FP32 and with FP64 solves; the paper's four benchmarks
at the resolutions of its figures, the largest its 3D run of nested cubes
(226,981 cuboids, n = 260,401), in both precisions; and one multi-frequency FP32
product of the cube-with-ellipsoid medium on the 100^3 grid (n = 1,076,336),
8 wavenumbers x 16 directions in one matrix-core launch per source class.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GMRES solve s and Gpair-evals/s at 1e-8 rel err: FP64 vs FP32+refine, 1 GPU"
GOLD = os.path.join(ROOT, "tests", "golden", "c1_oracle_solution.npz")
ISSUE_PEAK = 256 * 4 * 2.4e9   # SIMD issue cycles/s: 256 CUs x 4 SIMDs x 2.4 GHz


def note(msg):
    """One progress line on stderr as each part of the run ends."""
    print("[bench] " + msg, file=sys.stderr, flush=True)
TOL = 1e-10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workloads")
    ap.add_argument("--c4-solve", action="store_true",
                    help="instead of the steps: the lockstep multi-frequency block GMRES solve of the "
                         "100^3 cube-with-ellipsoid medium (n = 1,076,336), 16 plane waves at each of the "
                         "wavenumbers --c4-freqs, FP32 operator in FP64 refinement to rel. residual 1e-10, "
                         "with the oracle's residual on sampled rows of every frequency (the solver "
                         "prints a progress line per block step on stderr)")
    ap.add_argument("--c4-freqs", default="0-1", metavar="A-B",
                    help="frequency indices of --c4-solve (k0 = 40 - 2 i); default 0-1: two wavenumbers, "
                         "about 9 minutes (0-1, 2-3, 4-5 and 6-7 cover all eight)")
    ap.add_argument("--c4-fp64", action="store_true",
                    help="--c4-solve with the plain FP64 operator (the FP64 matrix cores) instead of the "
                         "FP32 operator in FP64 refinement")
    ap.add_argument("--krylov-gib", type=int, default=200,
                    help="device memory of the Krylov bases of --c4-solve in GiB (0: the library default, "
                         "96); the frequencies share it, so the cycle length per frequency falls with "
                         "their number: 200 GiB gives two wavenumbers 181 block steps per cycle, "
                         "enough for k0 = 40 without a restart")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle's full FP64 GMRES solve of the headline workload "
                         "(several minutes on the host cores)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the steps, copy MIB MiB device-to-device three times (a kernel of "
                         "known traffic for scaling HBM byte counters)")
    return ap.parse_args()


def measured_traffic(key):
    """HBM bytes per launch of a pair kernel from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs (scaled by the same counters' reading for a copy of known
    size), or None when no record exists or the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "measurement", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(key)
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def c3_gradient(V, W, n_cells=3):
    """Receiver-misfit gradient w.r.t. every cell's c and rho on the c3 workload
    (forward solve of 8 incidences, adjoint solve, source sums, chain rule),
    timed with the FP32 operator in FP64 refinement, then checked against
    central differences (step 1e-3 of the parameter) of the misfit on n_cells
    seeded cells x {c, rho}, every misfit from FP64 solves to 1e-13."""
    import torch
    from paper_2607_06429_amd.autograd import receiver_pressure
    mesh, mat, k0s, dirs, rec = W.config_problem("c3")
    _, mat1, _, _, _ = W.config_problem("c1")
    P = V.Problem.from_mesh(mesh, mat, k0s)

    def pressures(c, rho, prec=V.VSIE_FP64, tol=1e-13):
        P.set_materials(torch.as_tensor(rho, device="cuda"), torch.as_tensor(c, device="cuda"))
        x, info = P.solve(P.plane_wave(dirs), prec=prec, tol=tol, block=True)
        return P.plane_wave_at(rec, dirs) - P.field(rec, x)

    data = pressures(mat1.vol_c, mat1.vol_rho)
    c = torch.tensor(mat.vol_c, device="cuda", requires_grad=True)
    rho = torch.tensor(mat.vol_rho, device="cuda", requires_grad=True)
    times, grads = {}, {}
    for tag, prec in (("fp64", V.VSIE_FP64), ("fp32", V.VSIE_FP32)):
        c.grad = None
        rho.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pr = receiver_pressure(P, mesh.n_vol, c, rho, dirs, rec, prec=prec, tol=TOL, block=True)
        loss = 0.5 * (pr - data).abs().pow(2).sum()
        loss.backward()
        torch.cuda.synchronize()
        times[tag] = time.perf_counter() - t0
        grads[tag] = (c.grad.cpu().numpy(), rho.grad.cpu().numpy())
    dt = times["fp32"]
    gc, gr = grads["fp32"]
    g64 = np.concatenate(grads["fp64"])
    diff64 = float(np.linalg.norm(np.concatenate(grads["fp32"]) - g64) / np.linalg.norm(g64))
    cells = np.random.default_rng(2607).choice(mesh.n_vol, n_cells, replace=False)
    errs = {}
    for which, g in (("c", gc), ("rho", gr)):
        fd = []
        for j in cells:
            vals = []
            for sgn in (1, -1):
                cv, rv = mat.vol_c.copy(), mat.vol_rho.copy()
                arr = cv if which == "c" else rv
                h = 1e-3 * arr[j]
                arr[j] += sgn * h
                vals.append(float(0.5 * (pressures(cv, rv) - data).abs().pow(2).sum()))
            fd.append((vals[0] - vals[1]) / (2 * h))
        fd = np.array(fd)
        errs[which] = float(np.linalg.norm(g[cells] - fd) / np.linalg.norm(fd))
    P.close()
    return {"workload": "c1 mesh (n=%d) with log-normal c and rho, k0=10, %d incidences, %d receivers on "
                        "|x|=3, misfit to the unperturbed medium's pressures" % (mesh.n, len(dirs), len(rec)),
            "gradient_s": dt, "gradient_s_fp64": times["fp64"], "speedup_vs_fp64": times["fp64"] / dt,
            "rel_diff_vs_fp64_gradient": diff64, "loss": float(loss.detach()),
            "solver": "block GMRES, FP32 operator in FP64 refinement to 1e-10 (forward and adjoint); "
                      "the FP64 timing uses the FP64 operator",
            "fd_check": {"cells": [int(j) for j in cells], "step": "1e-3 relative, central",
                         "misfit_solves": "FP64 to 1e-13", "rel_err_grad_c": errs["c"],
                         "rel_err_grad_rho": errs["rho"]}}


def matrix_core_issue(st, tuning, widths):
    """Issue-cycle fraction of the matrix-core pair launches in the profiler
    stats st: cycles per pair and per column block from isa_counts.json (the
    variant the tuning and the column widths select) x pair-column
    evaluations / column-block width, over the launches' measured time,
    against 256 CUs x 4 SIMDs x 2.4 GHz."""
    counts = json.load(open(os.path.join(ROOT, "measurement", "isa_counts.json")))
    out = {}
    for name, v in st.items():
        if not name.startswith("mfma_fwd_"):
            continue
        mode = name[len("mfma_"):].rsplit("_", 1)[0]
        m3 = "_3m" if tuning["mfma_3m"] else ""
        if name.endswith("fp32"):
            key = "mfma_%s_fp32_tg%d_nb%d%s" % (mode, tuning["mfma_tg"], tuning["mfma_nb"], m3)
        else:
            w = max(widths)
            key = "mfma64_%s_fp64_nb%d%s" % (mode, 1 if w <= 16 else 2 if w <= 32 else 4, m3)
        c = counts.get(key)
        if c is None:
            continue
        cyc = c["cycles_per_pair"] * v["rhs_pairs"] / c["rhs_per_trip"]
        out[name] = {"isa_variant": key, "cycles_per_pair_block": c["cycles_per_pair"],
                     "issue_frac": cyc / (v["ms"] * 1e-3) / ISSUE_PEAK}
    return out


def c4_block_solve(V, W, freqs, checks, krylov_gib=0, fp64=False):
    """The largest configuration in its batched form: 16 plane waves at each
    wavenumber of freqs solved together by the lockstep multi-frequency block
    GMRES (FP32 operator on the matrix cores inside FP64 refinement, to
    relative residual 1e-10), one multi-frequency product per block step.
    Two columns of every frequency's solution are kept for the oracle's
    sampled-row residual."""
    import torch
    mesh, mat, k0s, dirs, _ = W.config_problem("c4")
    f0, f1 = freqs
    nf = f1 - f0 + 1
    P = V.Problem.from_mesh(mesh, mat, k0s)
    R = dirs.shape[0]
    B = torch.cat([P.plane_wave(dirs, f=f) for f in range(f0, f1 + 1)], dim=0).contiguous()
    torch.cuda.synchronize()
    P.profile(True)
    t0 = time.perf_counter()
    prec = V.VSIE_FP64 if fp64 else V.VSIE_FP32
    X, infos = P.solve_multi(B, f0=f0, nf=nf, prec=prec, tol=TOL, progress=True, krylov_gib=krylov_gib)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = P.kernel_stats()
    P.profile(False)
    note("c4 lockstep solve of %d frequencies: %.1f s" % (nf, dt))
    P_tuning = P.tuning
    mv32 = sum(i["matvecs_fp32"] for i in infos)
    mv64 = sum(i["matvecs_fp64"] for i in infos)
    for t in range(nf):
        checks.append({"label": "c4_k0_%g" % k0s[f0 + t], "problem": ("c4", None), "f": f0 + t,
                       "x": X[t * R:t * R + 2].cpu().numpy().T, "b": B[t * R:t * R + 2].cpu().numpy().T})
    P.close()
    return {"c4_lockstep_solve": {
        "workload": "cube with ellipsoid, 100^3 grid, n=%d, k0 = %s, %d plane waves each; lockstep "
                    "multi-frequency block GMRES, %s to rel. residual 1e-10; Krylov budget %s GiB"
                    % (mesh.n, k0s[f0:f1 + 1], R, "plain FP64 operator (FP64 matrix cores)" if fp64 else
                       "FP32 operator (matrix cores) in FP64 refinement", krylov_gib or 96),
        "solve_s": dt, "per_frequency": dict(zip(["%g" % k for k in k0s[f0:f1 + 1]], infos)),
        "gpair_col_evals_per_s": float(mesh.n) * mesh.n * (mv32 + mv64) / dt / 1e9,
        "pair_kernels": {k: {"launches": v["launches"], "ms": v["ms"]} for k, v in st.items()},
        "matrix_core_issue": matrix_core_issue(st, P_tuning, [R])}}


def c4_lockstep_reduced(V, W, N, checks):
    """The cube-with-ellipsoid workload on an N^3 grid with the wavenumbers
    scaled by N/100 (the sampling per wavelength of the 100^3 grid): all 8
    frequencies x 16 plane waves by the lockstep multi-frequency block GMRES,
    and the same systems frequency by frequency with the one-frequency block
    solver, both FP32 operator in FP64 refinement to 1e-10."""
    import torch
    mesh, mat, k0s, dirs, _ = W.config_problem("c4", N=N)
    ks = [k * N / 100.0 for k in k0s]
    nf, R = len(ks), dirs.shape[0]
    P = V.Problem.from_mesh(mesh, mat, ks)
    B = torch.cat([P.plane_wave(dirs, f=f) for f in range(nf)], dim=0).contiguous()
    # untimed short runs size the work buffers of both paths
    P.solve_multi(B, prec=V.VSIE_FP32, tol=TOL, max_iter=R, allow_noconv=True)
    P.solve(B[:R].contiguous(), f=0, prec=V.VSIE_FP32, tol=TOL, block=True, max_iter=R, allow_noconv=True)
    torch.cuda.synchronize()
    P.profile(True)
    t0 = time.perf_counter()
    X, infos = P.solve_multi(B, prec=V.VSIE_FP32, tol=TOL)
    torch.cuda.synchronize()
    t_lock = time.perf_counter() - t0
    st = P.kernel_stats()
    P.profile(False)
    t0 = time.perf_counter()
    seq = []
    for f in range(nf):
        x1, i1 = P.solve(B[f * R:(f + 1) * R].contiguous(), f=f, prec=V.VSIE_FP32, tol=TOL, block=True)
        seq.append((x1, i1))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    diff = max(float(torch.linalg.norm(X[f * R:(f + 1) * R] - seq[f][0]) / torch.linalg.norm(seq[f][0]))
               for f in range(nf))
    for f in range(nf):
        checks.append({"label": "c4_%d_k0_%.2f" % (N, ks[f]), "problem": ("c4", N), "f": f,
                       "x": X[f * R:f * R + 2].cpu().numpy().T, "b": B[f * R:f * R + 2].cpu().numpy().T})
    note("c4 at %d^3 (n = %d): lockstep %.2f s, frequency by frequency %.2f s" % (N, mesh.n, t_lock, t_seq))
    issue = matrix_core_issue(st, P.tuning, [R])
    P.close()
    return {"workload": "cube with ellipsoid, %d^3 grid, n=%d, k0 = %s (the 100^3 wavenumbers x %d/100), "
                        "%d plane waves each, FP32 operator in FP64 refinement to rel. residual 1e-10"
                        % (N, mesh.n, ["%.2f" % k for k in ks], N, R),
            "lockstep_solve_s": t_lock, "one_frequency_solves_s": t_seq, "speedup_lockstep": t_seq / t_lock,
            "per_frequency": dict(zip(["%.2f" % k for k in ks], infos)),
            "one_frequency_iterations": [i for _, i in seq],
            "max_rel_diff_lockstep_vs_one_frequency": diff,
            "lockstep_pair_kernels": {k: {"launches": v["launches"], "ms": v["ms"]} for k, v in st.items()},
            "matrix_core_issue": issue}


def far_field_pattern(V, P, x):
    """Far-field pattern of the solution x on a 1-degree grid of directions
    (180 polar x 360 azimuthal = 64,800), FP32 and FP64, with the per-kernel
    times and issue-cycle rates of the two source classes."""
    import torch
    th = (np.arange(180) + 0.5) * (math.pi / 180)
    ph = np.arange(360) * (2 * math.pi / 360)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    X = np.stack([(np.sin(TH) * np.cos(PH)).ravel(), (np.sin(TH) * np.sin(PH)).ravel(), np.cos(TH).ravel()], axis=1)
    counts = json.load(open(os.path.join(ROOT, "measurement", "isa_counts.json")))
    res = {"directions": int(X.shape[0])}
    pats = {}
    for name, prec in (("fp32", V.VSIE_FP32), ("fp64", V.VSIE_FP64)):
        P.far_field(X, x, prec=prec)          # untimed first call (work buffers)
        torch.cuda.synchronize()
        P.profile(True)
        t0 = time.perf_counter()
        pats[name] = P.far_field(X, x, prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = P.kernel_stats()
        P.profile(False)
        ker = {}
        for k, v in st.items():
            cyc = counts[k + "_R1"]["cycles_per_pair"]
            rate = v["pairs"] / (v["ms"] * 1e-3)
            ker[k] = {"ms": v["ms"], "gpairs_per_s": rate / 1e9, "cycles_per_pair": cyc,
                      "issue_frac": cyc * rate / ISSUE_PEAK}
        res[name] = {"pattern_s": dt, "kernels": ker}
    res["rel_diff_fp32_vs_fp64"] = float(torch.linalg.norm(pats["fp32"] - pats["fp64"])
                                         / torch.linalg.norm(pats["fp64"]))
    return res


def exterior_slice(V, P, x, dirs):
    """Exterior field of the solution x on the slice z = 0: a 512 x 512 grid
    over [-7, 7]^2 mm without the points inside the 7 mm cube (the
    representation formula at 196,608 points), FP32 and FP64."""
    import torch
    g = np.linspace(-7.0, 7.0, 512)
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    pts = pts[np.max(np.abs(pts[:, :2]), axis=1) > 3.5]
    counts = json.load(open(os.path.join(ROOT, "measurement", "isa_counts.json")))
    res = {"points": int(pts.shape[0])}
    for name, prec in (("fp32", V.VSIE_FP32), ("fp64", V.VSIE_FP64)):
        P.field(pts, x, prec=prec)
        torch.cuda.synchronize()
        P.profile(True)
        t0 = time.perf_counter()
        P.field(pts, x, prec=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = P.kernel_stats()
        P.profile(False)
        ker = {}
        for k, v in st.items():
            cyc = counts[k + "_R1"]["cycles_per_pair"]
            rate = v["pairs"] / (v["ms"] * 1e-3)
            ker[k] = {"ms": v["ms"], "gpairs_per_s": rate / 1e9, "cycles_per_pair": cyc,
                      "issue_frac": cyc * rate / ISSUE_PEAK}
        res[name] = {"slice_s": dt, "kernels": ker}
    return res


def paper_benchmark_solves(V, W, checks):
    """The paper's four benchmarks (section 3) at the resolutions of its
    figures, each solved with the FP32 operator in FP64 refinement and with
    the FP64 operator: the sphere in a cube at 8 cells per interior
    wavelength, the nested cubes with piecewise-constant density and the
    heterogeneous single cube at 10, and the largest system, the 3D run of the
    fourth benchmark (nested cubes with a heterogeneous density and a jump,
    61^3 = 226,981 cuboids, n = 260,401, exterior wavelength 1.4 mm, incidence
    (1,1,0)/sqrt 2)."""
    import torch
    cases = (("b1_sphere_in_cube", W.benchmark1_problem), ("b2_nested_cubes_piecewise", W.benchmark2_problem),
             ("b3_heterogeneous_cube", W.benchmark3_problem), ("b4_3d_run", W.benchmark4_problem))
    res = {}
    for label, make in cases:
        mesh, mat, k0s, dirs, grad = make()
        P = V.Problem.from_mesh(mesh, mat, k0s, grad_rho=grad)
        b = P.plane_wave(dirs)
        out, sols = {"n": mesh.n, "k0": k0s[0]}, {}
        if mesh.n < 100000:
            # untimed first solves (work buffers, captured graphs); the large
            # system's solves take seconds and are timed cold
            for prec in (V.VSIE_FP32, V.VSIE_FP64):
                P.solve(b, prec=prec, tol=TOL)
        for name, prec in (("fp32_refine", V.VSIE_FP32), ("fp64", V.VSIE_FP64)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = P.solve(b, prec=prec, tol=TOL)
            torch.cuda.synchronize()
            out[name] = {"solve_s": time.perf_counter() - t0, "iterations": info}
            sols[name] = x
        out["speedup_fp32_refine_vs_fp64"] = out["fp64"]["solve_s"] / out["fp32_refine"]["solve_s"]
        out["rel_diff_fp32_refine_vs_fp64_solution"] = float(
            torch.linalg.norm(sols["fp32_refine"] - sols["fp64"]) / torch.linalg.norm(sols["fp64"]))
        note("%s: FP32+refinement %.3f s, FP64 %.3f s" % (label, out["fp32_refine"]["solve_s"], out["fp64"]["solve_s"]))
        if label == "b4_3d_run":
            checks.append({"label": "b4_3d_run_fp32_refine", "problem": ("b4", None), "f": 0,
                           "x": sols["fp32_refine"].cpu().numpy().reshape(-1, 1),
                           "b": b.cpu().numpy().reshape(-1, 1)})
            out["far_field_pattern"] = far_field_pattern(V, P, sols["fp64"])
            out["exterior_field_slice"] = exterior_slice(V, P, sols["fp64"].reshape(-1), dirs)
        P.close()
        res[label] = out
    return res


def dense_roofline(st, tuning):
    """Matrix-core roofline of the product with the assembled FP32 operator:
    algorithmic FLOP per pass = 8 n^2 R (a complex multiply-add is 8 real
    FLOP) over the measured launch time, against the FP32 matrix peak; the
    FLOP the matrix cores execute (6 n^2 R with three real products per
    complex multiply-add, 8 n^2 R with four) reported beside it."""
    avg_ms = st["ms"] / st["launches"]
    macs = st["rhs_pairs"] / st["launches"]          # n^2 R complex multiply-adds per launch
    alg = 8.0 * macs / (avg_ms * 1e-3) / 1e12
    mfma = (6.0 if tuning["mfma_3m"] else 8.0) * macs / (avg_ms * 1e-3) / 1e12
    return {"bound": "mfma", "launches": st["launches"], "avg_launch_ms": avg_ms,
            "achieved": alg, "peak": 157.3, "unit": "TFLOP/s", "frac": alg / 157.3,
            "mfma_executed_tflops": mfma, "mfma_busy_frac": mfma / 157.3}


def batched_workloads(V, W, checks):
    """Block GMRES over 128 directions (assembled and matrix-free), the
    gradient workload, the paper's benchmarks, one multi-frequency product over
    8 wavenumbers x 16 directions and the lockstep multi-frequency solve on
    reduced grids.  Columns of the solutions go to checks for the oracle."""
    import torch
    out = {}
    mesh, mat, k0s, dirs, _ = W.config_problem("c2")
    P = V.Problem.from_mesh(mesh, mat, k0s)
    n = P.n
    B = P.plane_wave(dirs)
    R = B.shape[0]
    sols = {}
    for name, prec in (("assembled_fp32", V.VSIE_FP32), ("matrix_free_fp32", V.VSIE_FP32),
                       ("matrix_free_fp64", V.VSIE_FP64)):
        A = P.assemble_dense(0) if name == "assembled_fp32" else None
        if name == "matrix_free_fp32":
            P.autotune(R)
        torch.cuda.synchronize()
        P.profile(True)
        t0 = time.perf_counter()
        x, info = P.solve(B, prec=prec, tol=TOL, block=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = P.kernel_stats()
        P.profile(False)
        sols[name] = x
        if name != "matrix_free_fp64":
            cols = [0, 42, 85, 127]
            checks.append({"label": "c2_block_gmres_" + name, "problem": ("c2", None), "f": 0,
                           "x": x[cols].cpu().numpy().T, "b": B[cols].cpu().numpy().T})
        mv = info["matvecs_fp32"] + info["matvecs_fp64"]
        op = ("FP32 operator %s in FP64 refinement" % ("assembled (%.1f GB)" % (8.0 * n * n / 1e9)
                                                       if A is not None else "matrix-free")
              if prec == V.VSIE_FP32 else "FP64 operator matrix-free")
        note("c2 block GMRES %s: %.2f s" % (name, dt))
        out["c2_block_gmres_" + name] = {
            "workload": "nested balls, 57^3 grid, n=%d, k0=16, %d Fibonacci directions, block GMRES, "
                        "%s to rel. residual 1e-10" % (n, R, op),
            "solve_s": dt, "iterations": info, "gpair_col_evals_per_s": float(n) * n * mv / dt / 1e9,
            "tuning": P.tuning if name == "matrix_free_fp32" else None,
            "pair_kernels": {k: {"launches": v["launches"], "ms": v["ms"]} for k, v in st.items()},
            "matrix_core_issue": matrix_core_issue(st, P.tuning, [R])}
        if A is not None and "dense_product_fp32" in st:
            out["c2_block_gmres_" + name]["dense_product"] = dense_roofline(st["dense_product_fp32"], P.tuning)
        if A is not None:
            P.release_dense(0)
            del A
            torch.cuda.empty_cache()
    ref = sols["matrix_free_fp64"]
    for name in ("assembled_fp32", "matrix_free_fp32"):
        out["c2_block_gmres_" + name]["rel_diff_vs_fp64_solution"] = float(
            torch.linalg.norm(sols[name] - ref) / torch.linalg.norm(ref))
        out["c2_block_gmres_" + name]["speedup_vs_fp64"] = (out["c2_block_gmres_matrix_free_fp64"]["solve_s"]
                                                             / out["c2_block_gmres_" + name]["solve_s"])
    del sols, ref
    P.close()
    del B
    out["c3_adjoint_gradient"] = c3_gradient(V, W)
    note("c3 gradient done")
    out["paper_benchmarks"] = paper_benchmark_solves(V, W, checks)
    mesh, mat, k0s, dirs, _ = W.config_problem("c4")
    P = V.Problem.from_mesh(mesh, mat, k0s)
    n, nf, R = P.n, len(k0s), dirs.shape[0]
    X = torch.cat([P.plane_wave(dirs, f=f) for f in range(nf)], dim=0).contiguous()
    Y = torch.empty_like(X)
    V.vsie_matvec_multi(P.handle, 0, nf, V.VSIE_FP32, X, Y)
    torch.cuda.synchronize()
    P.profile(True)
    t0 = time.perf_counter()
    V.vsie_matvec_multi(P.handle, 0, nf, V.VSIE_FP32, X, Y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = P.kernel_stats()
    P.profile(False)
    note("c4 multi-frequency product: %.2f s" % dt)
    out["c4_multi_frequency_product"] = {
        "workload": "cube with ellipsoid, 100^3 grid, n=%d, k0 = %s, %d directions each, FP32 operator, "
                    "one matrix-core launch per source class" % (n, k0s, R),
        "product_s": dt, "gpair_col_evals_per_s": float(n) * n * nf * R / dt / 1e9,
        "tuning": P.tuning,
        "pair_kernels": {k: {"launches": v["launches"], "ms": v["ms"]} for k, v in st.items()},
        "matrix_core_issue": matrix_core_issue(st, P.tuning, [R])}
    P.close()
    del X, Y
    torch.cuda.empty_cache()
    out["c4_lockstep_reduced"] = {"N%d" % N: c4_lockstep_reduced(V, W, N, checks) for N in (32, 48)}
    return out


def cpu_baseline(mesh, mat, k0, n, target_s):
    """The FP64 oracle's direct summation on a bounded sample of rows of the
    headline workload: the reported CPU baseline."""
    import oracle as O
    import workloads as W
    d = O.discretise(mesh, mat, k0)
    x = W.seeded_complex(n, seed=31)
    rng = np.random.default_rng(32)
    rows = np.sort(rng.choice(n, 1024, replace=False))
    t = time.perf_counter()
    O.matvec(d, x, rows=rows)
    dt = time.perf_counter() - t
    m = int(min(n, max(1024, 1024 * target_s / max(dt, 1e-3))))
    rows = np.sort(rng.choice(n, m, replace=False))
    t = time.perf_counter()
    O.matvec(d, x, rows=rows)
    dt = time.perf_counter() - t
    pairs = float(m) * n
    return {"value": pairs / dt / 1e9, "unit": "Gpair-evals/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": "FP64 oracle matvec (C, OpenMP, compensated sums) on %d seeded rows of the "
                      "%d-row operator: %.3g pair evaluations in %.2f s" % (m, n, pairs, dt),
            "seconds": dt}


def cpu_baseline_discretisation(problem, f):
    """The oracle's discretisation of a workload named by a check record."""
    import oracle as O
    import workloads as W
    name, N = problem
    if name == "b4":
        mesh, mat, k0s, _, grad = W.benchmark4_problem()
        return O.discretise(mesh, mat, k0s[f], grad_rho=grad)
    mesh, mat, k0s, _, _ = W.config_problem(name, N=N)
    k = k0s[f] * (N / 100.0 if N is not None else 1.0)
    return O.discretise(mesh, mat, k)


def cpu_baseline_checks(checks, rows_per_check=256):
    """The oracle's residual ||(b - A x)[rows]|| / ||b[rows]|| of GPU solution
    columns on 256 seeded rows (plus the first and last cell and face) of the
    Theorem 3 system."""
    import oracle as O
    out = {}
    cache = {}
    for c in checks:
        key = (c["problem"], c["f"])
        if key not in cache:
            cache.clear()
            cache[key] = cpu_baseline_discretisation(*key)
        d = cache[key]
        rng = np.random.default_rng(71)
        rows = np.unique(np.concatenate([rng.choice(d.n, rows_per_check, replace=False),
                                         [0, d.n_vol - 1, d.n_vol, d.n - 1]]))
        X, B = np.asarray(c["x"]).reshape(d.n, -1), np.asarray(c["b"]).reshape(d.n, -1)
        r = B[rows] - O.matvec(d, X, rows=rows)
        out[c["label"]] = {"rel_residual": float(np.linalg.norm(r) / np.linalg.norm(B[rows])),
                           "rows": int(rows.size), "columns": int(X.shape[1])}
    return out


def cpu_baseline_plan(full_c1_gmres=False):
    """The oracle timed on the other workloads, each bounded: c0 solved by
    dense LU; c2's operator on 2,048 seeded rows with 1 and with 4 columns;
    c3's forward (8 incidences) and adjoint (256 receivers) problems on the
    24^3 grid by one dense LU; 4,096 seeded rows of c4's operator (the full
    product extrapolated); and, when asked, the full FP64 GMRES solve of c1."""
    import scipy.linalg as sla
    import oracle as O
    import workloads as W
    plan = {}

    def timed(fn):
        t = time.perf_counter()
        r = fn()
        return r, time.perf_counter() - t

    mesh, mat, k0s, dirs, _ = W.config_problem("c0")
    d = O.discretise(mesh, mat, k0s[0])
    b = O.plane_wave(d.pts, k0s[0], dirs[0])
    A, t_asm = timed(lambda: O.assemble(d))
    lu, t_lu = timed(lambda: sla.lu_factor(A))
    _, t_sol = timed(lambda: sla.lu_solve(lu, b))
    plan["c0_lu"] = {"n": d.n, "assemble_s": t_asm, "factor_s": t_lu, "solve_s": t_sol,
                     "total_s": t_asm + t_lu + t_sol}
    note("oracle c0 LU: %.2f s" % (t_asm + t_lu + t_sol))

    mesh, mat, k0s, dirs, _ = W.config_problem("c2")
    d = O.discretise(mesh, mat, k0s[0])
    rows = np.sort(np.random.default_rng(33).choice(d.n, 2048, replace=False))
    for R in (1, 4):
        x = W.seeded_complex((d.n, R), seed=34)
        _, t = timed(lambda: O.matvec(d, x, rows=rows))
        plan["c2_matvec_%drhs" % R] = {"rows": int(rows.size), "n": d.n, "seconds": t,
                                       "gpair_evals_per_s": rows.size * float(d.n) / t / 1e9,
                                       "gpair_col_evals_per_s": rows.size * float(d.n) * R / t / 1e9,
                                       "full_matvec_s_extrapolated": t * d.n / rows.size}
    note("oracle c2 rows done")

    mesh, mat, k0s, dirs, rec = W.config_problem("c3", N=24)
    d = O.discretise(mesh, mat, k0s[0])
    A, t_asm = timed(lambda: O.assemble(d))
    lu, t_lu = timed(lambda: sla.lu_factor(A))
    B = O.plane_wave(d.pts, k0s[0], dirs)
    _, t_fwd = timed(lambda: sla.lu_solve(lu, B))
    lam = W.seeded_complex((d.n, rec.shape[0]), seed=35)
    _, t_adj = timed(lambda: sla.lu_solve(lu, lam, trans=2))
    plan["c3_24"] = {"n": d.n, "assemble_s": t_asm, "factor_s": t_lu, "forward_solve_s": t_fwd,
                     "adjoint_solve_s": t_adj, "incidences": int(dirs.shape[0]), "receivers": int(rec.shape[0])}
    del A, lu
    note("oracle c3 at 24^3: %.1f s" % (t_asm + t_lu + t_fwd + t_adj))

    mesh, mat, k0s, dirs, _ = W.config_problem("c4")
    d = O.discretise(mesh, mat, k0s[0])
    rows = np.sort(np.random.default_rng(36).choice(d.n, 4096, replace=False))
    x = W.seeded_complex(d.n, seed=37)
    _, t = timed(lambda: O.matvec(d, x, rows=rows))
    plan["c4_rows"] = {"rows": int(rows.size), "n": d.n, "seconds": t,
                       "gpair_evals_per_s": rows.size * float(d.n) / t / 1e9,
                       "full_matvec_s_extrapolated": t * d.n / rows.size,
                       "note": "the full product time is an extrapolation from the sampled rows"}
    note("oracle c4 rows: %.1f s" % t)

    if full_c1_gmres:
        mesh, mat, k0s, dirs, _ = W.config_problem("c1")
        d = O.discretise(mesh, mat, k0s[0])
        b = O.plane_wave(d.pts, k0s[0], dirs[0])
        (_, its, rr), t = timed(lambda: O.solve_gmres(d, b, tol=1e-12))
        plan["c1_gmres"] = {"n": d.n, "tol": 1e-12, "iterations": its, "rel_residual": rr, "seconds": t,
                            "restart": 200}
        note("oracle c1 GMRES: %.1f s" % t)
    return plan


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2607_06429_amd as V
    import workloads as W

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    checks = []
    if args.c4_solve:
        f0, f1 = (int(v) for v in args.c4_freqs.split("-"))
        res = c4_block_solve(V, W, (f0, f1), checks, args.krylov_gib, args.c4_fp64)
        res["cpu_baseline"] = {"kind": "oracle", "oracle_checks": cpu_baseline_checks(checks)}
        print(json.dumps(res), flush=True)
        return
    mesh, mat, k0s, dirs, _ = W.config_problem("c1")
    k0 = k0s[0]
    P = V.Problem.from_mesh(mesh, mat, k0s)
    n = P.n
    rho = torch.as_tensor(mat.vol_rho, device="cuda")
    c = torch.as_tensor(mat.vol_c, device="cuda")

    def step(prec):
        P.set_materials(rho, c)                     # weights from the materials
        b = P.plane_wave(dirs[0])                   # right-hand side
        x, info = P.solve(b, prec=prec, tol=TOL)    # GMRES (+ refinement)
        return x, info

    if args.calibrate_copy > 0:
        src = torch.empty(args.calibrate_copy << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step(V.VSIE_FP32)
    torch.cuda.synchronize()

    # timed region: K steps of the FP32 + FP64-refinement path
    P.profile(True)
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x32, info = step(V.VSIE_FP32)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    P.profile(False)
    kstats = P.kernel_stats()
    ms_per_step = elapsed / args.steps * 1e3

    # the plain FP64 path, same steps
    ksteps64 = max(1, min(args.steps, 3))
    step(V.VSIE_FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(ksteps64):
        x64, info64 = step(V.VSIE_FP64)
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) / ksteps64 * 1e3
    note("c1 steps: FP32+refinement %.1f ms, FP64 %.1f ms" % (ms_per_step, ms64))

    # pair evaluations of one step (all operator applications, both precisions)
    mv32 = infos[-1]["matvecs_fp32"]
    mv64 = infos[-1]["matvecs_fp64"]
    pairs_step = float(n) * n * (mv32 + mv64)
    value = pairs_step * args.steps / elapsed / 1e9

    err = {}
    if os.path.exists(GOLD):
        g = np.load(GOLD)["p"]
        for nm, xv in (("fp32_refine", x32), ("fp64", x64)):
            xh = xv.cpu().numpy()
            err[nm] = float(np.linalg.norm(xh - g) / np.linalg.norm(g))

    # roofline of the dominant kernel (the FP32 single-layer pair kernel):
    # issue cycles per pair counted in its compiled inner loop x pairs per
    # launch / average launch time, against 256 CUs x 4 SIMDs x 2.4 GHz
    counts = json.load(open(os.path.join(ROOT, "measurement", "isa_counts.json")))
    dom = max(kstats.items(), key=lambda kv: kv[1]["ms"])
    dom_name, st = dom
    per_pair = counts[dom_name + "_R1"]["cycles_per_pair"]
    avg_ms = st["ms"] / st["launches"]
    pairs_launch = st["pairs"] / st["launches"]
    achieved = per_pair * pairs_launch / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": dom_name, "achieved": achieved,
                "peak": ISSUE_PEAK / 1e12, "unit": "T SIMD issue-cycles/s", "frac": achieved / (ISSUE_PEAK / 1e12),
                "traffic": measured_traffic(dom_name + "_R1"), "cycles_per_pair": per_pair,
                "valu_per_pair": counts[dom_name + "_R1"]["valu_per_pair"], "avg_launch_ms": avg_ms,
                "launches": st["launches"], "pairs_per_launch": pairs_launch,
                "gpairs_per_s": pairs_launch / (avg_ms * 1e-3) / 1e9}
    kernel_summary = {k: {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"],
                          "gpairs_per_s": v["pairs"] / v["ms"] * 1e-6} for k, v in kstats.items()}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gpair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "nested balls R=1/0.5, 48^3 voxel grid, n=71368, k0=10, "
                              "smooth core sound speed, plane wave +z; FP32 operator in "
                              "FP64 iterative refinement to rel. residual 1e-10",
                   "n": n, "k0": k0, "tol": TOL},
        "solve_s_fp32_refine": ms_per_step / 1e3,
        "solve_s_fp64": ms64 / 1e3,
        "speedup_fp32_refine_vs_fp64": ms64 / ms_per_step,
        "iterations": {"fp32_refine": infos[-1], "fp64": info64},
        "gpairs_per_s_fp64_solve": float(n) * n * (info64["matvecs_fp64"]) / (ms64 * 1e-3) / 1e9,
        "rel_err_vs_oracle": err or None,
        "kernels": kernel_summary,
        "roofline": roofline,
    }
    if not args.no_batched:
        out["batched"] = batched_workloads(V, W, checks)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(mesh, mat, k0, n, args.cpu_seconds)
        cb["solve_s_extrapolated_fp64"] = float(n) * n * info64["matvecs_fp64"] / (cb["value"] * 1e9)
        cb["plan"] = cpu_baseline_plan(args.cpu_full)
        cb["oracle_checks"] = cpu_baseline_checks(checks)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    P.close()


if __name__ == "__main__":
    main()
