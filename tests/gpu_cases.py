"""Seeded small cases and tensor helpers shared by the GPU tests."""
import sys

import numpy as np

import workloads as W


def dev(a):
    import torch
    a = np.asarray(a, dtype=np.complex128)
    if a.ndim == 1:
        return torch.as_tensor(a, device="cuda")
    return torch.as_tensor(np.ascontiguousarray(a.T), device="cuda")


def host(t):
    a = t.cpu().numpy()
    return a if a.ndim == 1 else a.T


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def case(name):
    """(mesh, materials, k0) of the small parity cases."""
    if name == "c0":
        m, mat, k0, _, _ = W.config_problem("c0")
        return m, mat, k0[0]
    if name == "ragged":          # 7^3 grid: n not a multiple of any tile
        m = W.nested_balls(7)
        return m, W.materials_piecewise(m, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8), 3.0
    if name == "lognormal":       # per-cell rho and c: grad alpha (T terms) active
        m = W.nested_balls(10)
        mat = W.materials_piecewise(m, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8)
        mat.vol_c = mat.vol_c * W.lognormal_voxel_field(m.vol_xyz, -1, 1, 32, 0.1, 0)
        mat.vol_rho = mat.vol_rho * W.lognormal_voxel_field(m.vol_xyz, -1, 1, 32, 0.1, 1)
        return m, mat, 5.0
    if name == "single":          # Omega_2 with Omega_1's material
        m = W.nested_balls(9)
        return m, W.materials_piecewise(m, 1.0, 1.0, 1.4, 1.3, 1.4, 1.3), 2.5
    if name == "cube":            # cube + ellipsoid, small grid
        m = W.cube_with_ellipsoid(12)
        mat = W.materials_piecewise(m, 1.0, 1.0, 1.1, 1.3, 2.0, 0.8)
        mat.vol_c = mat.vol_c * W.lognormal_voxel_field(m.vol_xyz, -0.5, 0.5, 32, 0.1, 0)
        return m, mat, 12.0
    raise KeyError(name)


CASES = ["c0", "ragged", "lognormal", "single", "cube"]


def parity_err(num, ref):
    """Relative error of a GPU result against the oracle (eq_error) in the
    2-norm and in the max-norm over all entries, max|num - ref| / max|ref|:
    the larger of the two, so that one bar bounds both (an error confined to a
    few entries cannot hide in the 2-norm of a long vector)."""
    import oracle as O
    return max(O.rel_error(num, ref), O.rel_error(num, ref, ord=np.inf))


def oracle_residual(d, x, b, rows):
    """Residual of a GPU solution x (n or n x R) on sampled rows, computed by
    the oracle from the Theorem 3 system: ||(b - A x)[rows]|| / ||b[rows]||,
    the 2-norm over the rows and columns."""
    import oracle as O
    X = np.asarray(x).reshape(d.n, -1)
    B = np.asarray(b).reshape(d.n, -1)
    r = B[rows] - O.matvec(d, X, rows=rows)
    return float(np.linalg.norm(r) / np.linalg.norm(B[rows]))


def sample_rows(n, n_vol, count, seed):
    """count seeded rows plus the first and last cell and face."""
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.choice(n, count, replace=False),
                                     [0, n_vol - 1, n_vol, n - 1]]))
