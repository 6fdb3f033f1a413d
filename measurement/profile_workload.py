"""Run one workload's operator products for a profiler (rocprofv3
--kernel-trace --stats, or --pmc counters) and print the library's own
HIP-event timings of the same launches, so that the two can be compared.

    python measurement/profile_workload.py c2-dense      # assembled FP32 operator, 128 columns
    python measurement/profile_workload.py c2-fp64       # FP64 matrix-core product, 128 columns
    python measurement/profile_workload.py c4-product    # 8 frequencies x 16 columns, FP32
    python measurement/profile_workload.py c4-lockstep   # lockstep solve on the 48^3 grid

Each product runs once untimed (work buffers), then REPS times under the
library profiler.  Measurement tooling for the benchmark, not part of the
library.
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

REPS = 3


def say(*a):
    print(*a, flush=True)


def timed(P, fn, reps=REPS):
    import torch
    fn()
    torch.cuda.synchronize()
    P.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    st = P.kernel_stats()
    P.profile(False)
    return dt, {k: {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"]} for k, v in st.items()}


def main():
    import torch
    import paper_2607_06429_amd as V
    import workloads as W
    which = sys.argv[1] if len(sys.argv) > 1 else "c2-dense"
    torch.cuda.set_device(0)
    if which in ("c2-dense", "c2-fp64"):
        mesh, mat, k0s, dirs, _ = W.config_problem("c2")
        P = V.Problem.from_mesh(mesh, mat, k0s)
        X = P.plane_wave(dirs).contiguous()
        Y = torch.empty_like(X)
        if which == "c2-dense":
            A = P.assemble_dense(0)
            for name, fn in (("forward", lambda: V.vsie_matvec(P.handle, 0, V.VSIE_FP32, X, Y)),
                             ("adjoint", lambda: V.vsie_matvec_adjoint(P.handle, 0, V.VSIE_FP32, X, Y))):
                dt, st = timed(P, fn)
                say("c2 assembled FP32, 128 columns, %s: %.1f ms per product; library events %s"
                    % (name, dt * 1e3, json.dumps(st)))
            P.release_dense(0)
            del A
        else:
            dt, st = timed(P, lambda: V.vsie_matvec(P.handle, 0, V.VSIE_FP64, X, Y))
            say("c2 FP64 matrix cores, 128 columns: %.1f ms per product; library events %s"
                % (dt * 1e3, json.dumps(st)))
        P.close()
    elif which == "c4-product":
        mesh, mat, k0s, dirs, _ = W.config_problem("c4")
        P = V.Problem.from_mesh(mesh, mat, k0s)
        nf = len(k0s)
        X = torch.cat([P.plane_wave(dirs, f=f) for f in range(nf)], dim=0).contiguous()
        Y = torch.empty_like(X)
        dt, st = timed(P, lambda: V.vsie_matvec_multi(P.handle, 0, nf, V.VSIE_FP32, X, Y), reps=1)
        say("c4 multi-frequency FP32 product, 8 x 16 columns: %.2f s; library events %s" % (dt, json.dumps(st)))
        P.close()
    elif which == "c4-lockstep":
        N = 48
        mesh, mat, k0s, dirs, _ = W.config_problem("c4", N=N)
        ks = [k * N / 100.0 for k in k0s]
        P = V.Problem.from_mesh(mesh, mat, ks)
        B = torch.cat([P.plane_wave(dirs, f=f) for f in range(len(ks))], dim=0).contiguous()
        dt, st = timed(P, lambda: P.solve_multi(B, prec=V.VSIE_FP32, tol=1e-10), reps=1)
        say("c4 48^3 lockstep solve, 8 x 16 columns: %.2f s; library events %s" % (dt, json.dumps(st)))
        P.close()
    else:
        raise SystemExit("unknown workload " + which)


if __name__ == "__main__":
    main()
