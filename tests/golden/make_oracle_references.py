"""Write oracle reference solutions that are too slow to recompute in a test.

Calls only ``oracle`` and ``workloads``.  Usage:

    python tests/golden/make_oracle_references.py c1

writes tests/golden/c1_oracle_solution.npz holding the FP64 oracle solution of
the c1 workload (nested balls on a 48^3 grid, k0 = 10, plane wave along +z) by
unrestarted GMRES to relative residual 1e-12, with its iteration count and
final residual.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main(name):
    mesh, mat, k0s, dirs, _ = W.config_problem(name)
    d = O.discretise(mesh, mat, k0s[0])
    b = O.plane_wave(d.pts, k0s[0], dirs[0])
    t0 = time.time()

    def cb(it, res):
        print("iter %d rel.res %.3e  %.0fs" % (it, res, time.time() - t0), flush=True)
    p, it, res = O.solve_gmres(d, b, tol=1e-12, restart=3000, maxiter=3000, callback=cb)
    out = os.path.join(HERE, "%s_oracle_solution.npz" % name)
    np.savez(out, p=p, iterations=it, rel_residual=res, n=d.n, k0=k0s[0],
             direction=dirs[0], threads=O.num_threads())
    print("wrote", out, "iterations", it, "residual", res, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c1")
