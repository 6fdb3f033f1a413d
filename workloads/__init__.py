"""Seeded, synthetic inputs for the nested VSIE problem.

This module builds *inputs only*: voxel meshes of two nested subdomains with
surface elements that coincide with voxel faces (the paper's cuboid mesh,
section "Computational domain"), per-cell material values, incidence
directions and receiver points.  It contains none of the method's arithmetic
(no alpha/beta, no Green's function, no weights): both the CPU oracle and the
GPU path consume these arrays and derive everything else on their own.

Conventions
-----------
* Unknown order: volume cells of Omega_1, then Omega_2, then surface elements
  of Gamma_1, then Gamma_2 (the paper's block order of the 4x4 system).
* Surface normals point out of the inside subdomain (Gamma_1: out of Omega_1,
  Gamma_2: out of Omega_2), as in the paper's geometry figure.
* ``srf_cell_in`` / ``srf_cell_out`` index the volume cells on the two sides
  of a face; ``-1`` marks the exterior Omega_0.
* ``vol_nb`` holds, per cell, the indices of the 6 face neighbours in the
  order (-x, +x, -y, +y, -z, +z) that lie in Omega_1 or Omega_2, else -1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Mesh", "Materials", "voxel_mesh", "tensor_mesh", "nested_balls", "cube_with_ellipsoid", "nested_cubes",
    "kuhn_tet_mesh", "nested_cubes_tets", "nested_balls_tets", "cube_to_ball",
    "benchmark1_problem", "benchmark2_problem", "benchmark3_density", "benchmark3_density_gradient",
    "benchmark3_problem", "benchmark4_density", "benchmark4_density_gradient", "benchmark4_problem",
    "materials_piecewise", "materials_config", "fibonacci_sphere",
    "lognormal_voxel_field", "seeded_complex", "CONFIGS", "config_problem",
]

SEED = 2607


@dataclasses.dataclass
class Mesh:
    h: float
    vol_xyz: np.ndarray      # (n_vol, 3) centroids
    vol_w: np.ndarray        # (n_vol,) volumes
    vol_dom: np.ndarray      # (n_vol,) int32 in {1, 2}
    vol_nb: np.ndarray       # (n_vol, 6) int32 neighbour indices or -1
    srf_xyz: np.ndarray      # (n_srf, 3) centroids
    srf_n: np.ndarray        # (n_srf, 3) unit normals
    srf_area: np.ndarray     # (n_srf,)
    srf_iface: np.ndarray    # (n_srf,) int32 in {1, 2}
    srf_cell_in: np.ndarray  # (n_srf,) int32
    srf_cell_out: np.ndarray  # (n_srf,) int32, -1 = exterior

    @property
    def n_vol(self) -> int:
        return int(self.vol_w.shape[0])

    @property
    def n_srf(self) -> int:
        return int(self.srf_area.shape[0])

    @property
    def n(self) -> int:
        return self.n_vol + self.n_srf

    def points(self) -> np.ndarray:
        """All collocation points, (n, 3), in unknown order."""
        return np.concatenate([self.vol_xyz, self.srf_xyz], axis=0)

    def counts(self) -> dict:
        return {
            "omega1": int(np.sum(self.vol_dom == 1)),
            "omega2": int(np.sum(self.vol_dom == 2)),
            "gamma1": int(np.sum(self.srf_iface == 1)),
            "gamma2": int(np.sum(self.srf_iface == 2)),
            "n": self.n,
        }


@dataclasses.dataclass
class Materials:
    rho0: float
    c0: float
    vol_rho: np.ndarray  # (n_vol,)
    vol_c: np.ndarray    # (n_vol,)


def voxel_mesh(lo, hi, N, domain_fn) -> Mesh:
    """Uniform voxel grid of N^3 cells on the box [lo, hi]^3.

    ``domain_fn(xyz) -> int array`` classifies cell centroids into 0 (exterior),
    1 or 2.  Faces between a cell of Omega_1/Omega_2 and an exterior cell (or
    the grid boundary) become Gamma_1 elements; faces between an Omega_2 cell
    and an Omega_1 cell become Gamma_2 elements.
    """
    h = (hi - lo) / N
    c1d = lo + (np.arange(N) + 0.5) * h
    X, Y, Z = np.meshgrid(c1d, c1d, c1d, indexing="ij")
    cen = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    dom = np.asarray(domain_fn(cen), dtype=np.int32).reshape(N, N, N)
    # volume cells: Omega_1 first, then Omega_2 (each in lexicographic ijk order)
    flat = dom.ravel()
    order = np.concatenate([np.nonzero(flat == 1)[0], np.nonzero(flat == 2)[0]])
    cell_of = -np.ones(N ** 3, dtype=np.int64)
    cell_of[order] = np.arange(order.size)
    vol_xyz = cen[order].copy()
    vol_dom = flat[order].astype(np.int32)
    vol_w = np.full(order.size, h ** 3)

    ijk = np.stack(np.unravel_index(order, (N, N, N)), axis=1)
    nb = -np.ones((order.size, 6), dtype=np.int32)
    for ax in range(3):
        for side, step in ((0, -1), (1, +1)):
            q = ijk.copy()
            q[:, ax] += step
            inside = (q[:, ax] >= 0) & (q[:, ax] < N)
            lin = np.full(order.size, -1, dtype=np.int64)
            lin[inside] = np.ravel_multi_index(q[inside].T, (N, N, N))
            idx = np.where(inside, cell_of[np.maximum(lin, 0)], -1)
            nb[:, 2 * ax + side] = idx

    # faces
    faces = {1: [], 2: []}
    for ax in range(3):
        for side, step in ((0, -1), (1, +1)):
            other = nb[:, 2 * ax + side]
            # exterior faces: this cell inside, neighbour missing (exterior or out of grid)
            ext = np.nonzero(other < 0)[0]
            g2 = np.nonzero((other >= 0) & (vol_dom == 2))[0]
            g2 = g2[vol_dom[other[g2]] == 1]
            nvec = np.zeros(3)
            nvec[ax] = float(step)
            for iface, cells, outs in ((1, ext, np.full(ext.size, -1)),
                                       (2, g2, other[g2])):
                if cells.size == 0:
                    continue
                if iface == 1 and np.any(vol_dom[cells] != 1):
                    raise ValueError("an Omega_2 cell touches the exterior; refine the grid")
                fx = vol_xyz[cells].copy()
                fx[:, ax] += step * 0.5 * h
                faces[iface].append((fx, np.tile(nvec, (cells.size, 1)), cells, outs))

    def cat(iface):
        if not faces[iface]:
            return (np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, np.int32), np.zeros(0, np.int32))
        fx = np.concatenate([f[0] for f in faces[iface]])
        fn = np.concatenate([f[1] for f in faces[iface]])
        ci = np.concatenate([f[2] for f in faces[iface]]).astype(np.int32)
        co = np.concatenate([f[3] for f in faces[iface]]).astype(np.int32)
        # deterministic order: sort by centroid (z, y, x)
        o = np.lexsort((fx[:, 0], fx[:, 1], fx[:, 2]))
        return fx[o], fn[o], ci[o], co[o]

    f1, f2 = cat(1), cat(2)
    srf_xyz = np.concatenate([f1[0], f2[0]])
    srf_n = np.concatenate([f1[1], f2[1]])
    srf_in = np.concatenate([f1[2], f2[2]])
    srf_out = np.concatenate([f1[3], f2[3]])
    srf_iface = np.concatenate([np.full(f1[0].shape[0], 1, np.int32),
                                np.full(f2[0].shape[0], 2, np.int32)])
    return Mesh(h=h, vol_xyz=vol_xyz, vol_w=vol_w, vol_dom=vol_dom, vol_nb=nb,
                srf_xyz=srf_xyz, srf_n=srf_n, srf_area=np.full(srf_xyz.shape[0], h * h),
                srf_iface=srf_iface, srf_cell_in=srf_in, srf_cell_out=srf_out)


def tensor_mesh(edges, domain_of_index) -> Mesh:
    """Cuboid mesh on the tensor grid edges x edges x edges (the same
    nonuniform 1D grid on every axis): cell (i, j, k) spans
    [e_i, e_i+1] x [e_j, e_j+1] x [e_k, e_k+1].

    ``domain_of_index(I, J, K) -> int array`` classifies cells by index into 0
    (exterior), 1 or 2, so that interfaces can sit exactly on grid planes.
    Faces are built as in voxel_mesh, with the areas and centroids of the
    cuboids.  ``Mesh.h`` is the largest cell width.
    """
    e = np.asarray(edges, dtype=np.float64)
    N = e.size - 1
    c1d = 0.5 * (e[:-1] + e[1:])
    w1d = np.diff(e)
    I, J, K = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    flat = np.asarray(domain_of_index(I.ravel(), J.ravel(), K.ravel()), dtype=np.int32)
    order = np.concatenate([np.nonzero(flat == 1)[0], np.nonzero(flat == 2)[0]])
    cell_of = -np.ones(N ** 3, dtype=np.int64)
    cell_of[order] = np.arange(order.size)
    ijk = np.stack(np.unravel_index(order, (N, N, N)), axis=1)
    vol_xyz = c1d[ijk]
    wid = w1d[ijk]
    vol_w = wid[:, 0] * wid[:, 1] * wid[:, 2]
    vol_dom = flat[order].astype(np.int32)

    nb = -np.ones((order.size, 6), dtype=np.int32)
    for ax in range(3):
        for side, step in ((0, -1), (1, +1)):
            q = ijk.copy()
            q[:, ax] += step
            inside = (q[:, ax] >= 0) & (q[:, ax] < N)
            lin = np.full(order.size, -1, dtype=np.int64)
            lin[inside] = np.ravel_multi_index(q[inside].T, (N, N, N))
            nb[:, 2 * ax + side] = np.where(inside, cell_of[np.maximum(lin, 0)], -1)

    faces = {1: [], 2: []}
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        for side, step in ((0, -1), (1, +1)):
            other = nb[:, 2 * ax + side]
            ext = np.nonzero(other < 0)[0]
            g2 = np.nonzero((other >= 0) & (vol_dom == 2))[0]
            g2 = g2[vol_dom[other[g2]] == 1]
            nvec = np.zeros(3)
            nvec[ax] = float(step)
            for iface, cells, outs in ((1, ext, np.full(ext.size, -1)), (2, g2, other[g2])):
                if cells.size == 0:
                    continue
                if iface == 1 and np.any(vol_dom[cells] != 1):
                    raise ValueError("an Omega_2 cell touches the exterior")
                fx = vol_xyz[cells].copy()
                fx[:, ax] += step * 0.5 * wid[cells, ax]
                area = wid[cells, o1] * wid[cells, o2]
                faces[iface].append((fx, np.tile(nvec, (cells.size, 1)), cells, outs, area))

    def cat(iface):
        if not faces[iface]:
            return (np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, np.int32), np.zeros(0, np.int32),
                    np.zeros(0))
        parts = [np.concatenate([f[t] for f in faces[iface]]) for t in range(5)]
        o = np.lexsort((parts[0][:, 0], parts[0][:, 1], parts[0][:, 2]))
        return (parts[0][o], parts[1][o], parts[2][o].astype(np.int32), parts[3][o].astype(np.int32),
                parts[4][o])

    f1, f2 = cat(1), cat(2)
    return Mesh(h=float(w1d.max()), vol_xyz=vol_xyz, vol_w=vol_w, vol_dom=vol_dom, vol_nb=nb,
                srf_xyz=np.concatenate([f1[0], f2[0]]), srf_n=np.concatenate([f1[1], f2[1]]),
                srf_area=np.concatenate([f1[4], f2[4]]),
                srf_iface=np.concatenate([np.full(f1[0].shape[0], 1, np.int32),
                                          np.full(f2[0].shape[0], 2, np.int32)]),
                srf_cell_in=np.concatenate([f1[2], f2[2]]), srf_cell_out=np.concatenate([f1[3], f2[3]]))


def nested_cubes(n_shell: int, n_inner: int, L1: float = 7.0, L2: float = 5.0) -> Mesh:
    """Concentric cubes of sides L1 (Omega_1) and L2 (Omega_2) centred at the
    origin, on a nonuniform cuboid grid fitted to both interfaces (the
    paper's cuboid mesh for nested cubes): per axis n_shell cells across each
    (L1 - L2)/2 shell slab and n_inner cells across the inner cube."""
    a, b = 0.5 * L1, 0.5 * L2
    edges = np.concatenate([np.linspace(-a, -b, n_shell + 1), np.linspace(-b, b, n_inner + 1)[1:],
                            np.linspace(b, a, n_shell + 1)[1:]])

    def dom(i, j, k):
        lo, hi = n_shell, n_shell + n_inner
        inner = (i >= lo) & (i < hi) & (j >= lo) & (j < hi) & (k >= lo) & (k < hi)
        return np.where(inner, 2, 1)
    return tensor_mesh(edges, dom)


# the 6 monotone lattice paths from corner (0,0,0) to (1,1,1) of a cuboid, one
# per Kuhn tetrahedron (the axis moved at each of the three steps)
KUHN_PATHS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_tet_mesh(edges, domain_of_index, vertex_map=None) -> Mesh:
    """Conforming tetrahedral mesh of the cells of the tensor grid
    edges x edges x edges that ``domain_of_index(I, J, K)`` puts in Omega_1 or
    Omega_2 (0 = exterior), for the "conforming tetrahedral meshes" the paper
    leaves to future implementations (section 2.3.1).

    Each cuboid is split into the 6 Kuhn tetrahedra around its main diagonal
    (corner (i,j,k) to (i+1,j+1,k+1); tetrahedron p has the vertices visited by
    the path KUHN_PATHS[p]).  Every cell uses the same diagonal direction, so
    each rectangular cell face is split by its (low, low)-(high, high) diagonal
    from both sides and the mesh is conforming.  ``vertex_map(V) -> V'``
    optionally moves the grid vertices (curved interfaces); elements stay
    straight-sided.

    Volume elements: the tetrahedra (centroid = vertex mean, volume), Omega_1
    first, each subdomain ordered by (path, cell).  Surface elements: the two
    triangles of every cell face between Omega_1 and the exterior (Gamma_1)
    and between Omega_2 and Omega_1 (Gamma_2), with the unit normal of the
    triangle pointing away from the inside tetrahedron, and the tetrahedra on
    both sides as srf_cell_in / srf_cell_out.  vol_nb is -1 everywhere (no
    face-neighbour stencil: densities are piecewise constant or come with an
    analytic gradient).
    """
    e = np.asarray(edges, dtype=np.float64)
    N = e.size - 1
    I, J, K = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    flat = np.asarray(domain_of_index(I.ravel(), J.ravel(), K.ravel()), dtype=np.int32)
    g = np.arange(N + 1)
    VI, VJ, VK = np.meshgrid(g, g, g, indexing="ij")
    V = np.stack([e[VI.ravel()], e[VJ.ravel()], e[VK.ravel()]], axis=1)
    if vertex_map is not None:
        V = np.asarray(vertex_map(V), dtype=np.float64)

    def vid(ijk):
        return (ijk[..., 0] * (N + 1) + ijk[..., 1]) * (N + 1) + ijk[..., 2]

    cells = {d: np.nonzero(flat == d)[0] for d in (1, 2)}
    rank = -np.ones(N ** 3, dtype=np.int64)
    for d in (1, 2):
        rank[cells[d]] = np.arange(cells[d].size)
    start = {1: 0, 2: 6 * cells[1].size}

    def tet_index(c, path):
        d = flat[c]
        cnt = np.where(d == 1, cells[1].size, cells[2].size)
        st = np.where(d == 1, start[1], start[2])
        return st + KUHN_PATHS.index(path) * cnt + rank[c]

    tv, tdom = [], []
    for d in (1, 2):
        ijk = np.stack(np.unravel_index(cells[d], (N, N, N)), axis=1)
        for path in KUHN_PATHS:
            cur = ijk.copy()
            vs = [vid(cur)]
            for ax in path:
                cur = cur.copy()
                cur[:, ax] += 1
                vs.append(vid(cur))
            tv.append(np.stack(vs, axis=1))
            tdom.append(np.full(cells[d].size, d, dtype=np.int32))
    T = np.concatenate(tv)
    P = V[T]
    cen = P.mean(axis=1)
    vol = np.abs(np.einsum("ij,ij->i", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))) / 6.0

    tris = {1: [], 2: []}
    for ax in range(3):
        a, b = [q for q in range(3) if q != ax]
        for step in (-1, 1):
            own = np.nonzero(flat > 0)[0]
            ijk = np.stack(np.unravel_index(own, (N, N, N)), axis=1)
            q = ijk.copy()
            q[:, ax] += step
            inside = (q[:, ax] >= 0) & (q[:, ax] < N)
            oc = np.full(own.size, -1, dtype=np.int64)
            oc[inside] = np.ravel_multi_index(q[inside].T, (N, N, N))
            od = np.where(oc >= 0, flat[np.maximum(oc, 0)], 0)
            d = flat[own]
            for iface, sel in ((1, (d == 1) & (od == 0)), (2, (d == 2) & (od == 1))):
                if not np.any(sel):
                    continue
                c_in, c_out, base = own[sel], oc[sel], ijk[sel].copy()
                if step > 0:
                    base[:, ax] += 1
                # the two triangles of the face: path a-then-b and b-then-a
                for first, second in ((a, b), (b, a)):
                    p1 = base.copy()
                    p1[:, first] += 1
                    p2 = p1.copy()
                    p2[:, second] += 1
                    tri = np.stack([vid(base), vid(p1), vid(p2)], axis=1)
                    # owning tetrahedra: on the low side of a cell the path ends
                    # along ax, on the high side it starts along ax
                    path_lo, path_hi = (first, second, ax), (ax, first, second)
                    t_in = tet_index(c_in, path_lo if step < 0 else path_hi)
                    t_out = np.full(c_in.size, -1, dtype=np.int64)
                    if iface == 2:
                        t_out = tet_index(c_out, path_hi if step < 0 else path_lo)
                    tris[iface].append((tri, t_in, t_out))

    out = []
    for iface in (1, 2):
        if not tris[iface]:
            out.append((np.zeros((0, 3), np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64)))
            continue
        tri = np.concatenate([t[0] for t in tris[iface]])
        ti = np.concatenate([t[1] for t in tris[iface]])
        to = np.concatenate([t[2] for t in tris[iface]])
        q = V[tri].mean(axis=1)
        o = np.lexsort((q[:, 0], q[:, 1], q[:, 2]))
        out.append((tri[o], ti[o], to[o]))
    tri = np.concatenate([o[0] for o in out])
    Q = V[tri]
    cr = np.cross(Q[:, 1] - Q[:, 0], Q[:, 2] - Q[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    sx = Q.mean(axis=1)
    t_in = np.concatenate([o[1] for o in out])
    flip = np.einsum("ij,ij->i", nrm, sx - cen[t_in]) < 0
    nrm[flip] = -nrm[flip]
    iface = np.concatenate([np.full(out[0][0].shape[0], 1, np.int32), np.full(out[1][0].shape[0], 2, np.int32)])
    return Mesh(h=float(np.max(np.diff(e))), vol_xyz=cen, vol_w=vol, vol_dom=np.concatenate(tdom),
                vol_nb=-np.ones((T.shape[0], 6), dtype=np.int32), srf_xyz=sx, srf_n=nrm, srf_area=area,
                srf_iface=iface, srf_cell_in=t_in.astype(np.int32),
                srf_cell_out=np.concatenate([o[2] for o in out]).astype(np.int32))


def nested_cubes_tets(n_shell: int, n_inner: int, L1: float = 7.0, L2: float = 5.0) -> Mesh:
    """The nested-cube grid of nested_cubes, every cuboid split into 6 Kuhn
    tetrahedra (planar interfaces: the tetrahedra are not distorted)."""
    a, b = 0.5 * L1, 0.5 * L2
    edges = np.concatenate([np.linspace(-a, -b, n_shell + 1), np.linspace(-b, b, n_inner + 1)[1:],
                            np.linspace(b, a, n_shell + 1)[1:]])

    def dom(i, j, k):
        lo, hi = n_shell, n_shell + n_inner
        inner = (i >= lo) & (i < hi) & (j >= lo) & (j < hi) & (k >= lo) & (k < hi)
        return np.where(inner, 2, 1)
    return kuhn_tet_mesh(edges, dom)


def cube_to_ball(V):
    """Radial map taking the cube surface of sup-norm s onto the sphere of
    radius s: x -> x |x|_inf / |x|_2 (the origin stays)."""
    V = np.asarray(V, dtype=np.float64)
    r2 = np.linalg.norm(V, axis=1)
    ri = np.max(np.abs(V), axis=1)
    s = np.where(r2 > 0, ri / np.where(r2 > 0, r2, 1.0), 1.0)
    return V * s[:, None]


def nested_balls_tets(N: int, R1: float = 1.0, R2: float = 0.5) -> Mesh:
    """Concentric balls with curved interfaces: the N^3 grid of [-R1, R1]^3
    (N a multiple of 4 when R2 = R1/2, so that the cube of sup-norm R2 lies on
    grid planes), split into Kuhn tetrahedra, vertices mapped by cube_to_ball:
    the cube shells of sup-norm R2 and R1 become the spheres of radii R2 and
    R1, triangulated by the mapped face triangles."""
    e = np.linspace(-R1, R1, N + 1)
    m = int(round(N * (1.0 - R2 / R1) / 2.0))
    if abs(e[m] + R2) > 1e-12 * R1:
        raise ValueError("the inner sphere must lie on a grid plane (N a multiple of 4 for R2 = R1/2)")

    def dom(i, j, k):
        inner = (i >= m) & (i < N - m) & (j >= m) & (j < N - m) & (k >= m) & (k < N - m)
        return np.where(inner, 2, 1)
    return kuhn_tet_mesh(e, dom, cube_to_ball)


def nested_balls(N: int, R1: float = 1.0, R2: float = 0.5) -> Mesh:
    """Staircase voxel mesh of two concentric balls on an N^3 grid over [-R1, R1]^3."""
    def dom(x):
        r = np.sqrt(np.sum(x * x, axis=1))
        return np.where(r < R2, 2, np.where(r < R1, 1, 0))
    return voxel_mesh(-R1, R1, N, dom)


def cube_with_ellipsoid(N: int, centre=(0.05, 0.10, -0.10), axes=(0.4, 0.3, 0.2)) -> Mesh:
    """Unit cube [-0.5, 0.5]^3 (Omega_1) holding an axis-aligned ellipsoid (Omega_2)."""
    c = np.asarray(centre)
    a = np.asarray(axes)

    def dom(x):
        q = np.sum(((x - c) / a) ** 2, axis=1)
        return np.where(q < 1.0, 2, 1)
    return voxel_mesh(-0.5, 0.5, N, dom)


def materials_piecewise(mesh: Mesh, rho0, c0, rho1, c1, rho2, c2) -> Materials:
    """Piecewise values per subdomain; c1/c2/rho1/rho2 may be callables of xyz."""
    x = mesh.vol_xyz
    d = mesh.vol_dom

    def ev(v, sel):
        if callable(v):
            return np.asarray(v(x[sel]), dtype=np.float64)
        return np.full(int(np.sum(sel)), float(v))

    rho = np.empty(mesh.n_vol)
    c = np.empty(mesh.n_vol)
    for dd, r_, c_ in ((1, rho1, c1), (2, rho2, c2)):
        sel = d == dd
        rho[sel] = ev(r_, sel)
        c[sel] = ev(c_, sel)
    return Materials(rho0=float(rho0), c0=float(c0), vol_rho=rho, vol_c=c)


def fibonacci_sphere(m: int, radius: float = 1.0) -> np.ndarray:
    """m nearly uniform points on a sphere (golden-angle spiral), (m, 3)."""
    i = np.arange(m) + 0.5
    z = 1.0 - 2.0 * i / m
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def lognormal_voxel_field(xyz: np.ndarray, lo, hi, grid: int, sigma: float, stream: int,
                          seed: int = SEED) -> np.ndarray:
    """exp(sigma * xi) with xi ~ N(0,1) i.i.d. on a grid^3 voxel field over [lo,hi]^3.

    Each point takes the voxel containing it.  ``stream`` selects an independent
    PCG64 stream (0 for sound speed, 1 for density).
    """
    rng = np.random.default_rng([seed, stream])
    xi = rng.standard_normal((grid, grid, grid))
    idx = np.clip(np.floor((xyz - lo) / (hi - lo) * grid).astype(np.int64), 0, grid - 1)
    return np.exp(sigma * xi[idx[:, 0], idx[:, 1], idx[:, 2]])


def seeded_complex(shape, seed: int = SEED) -> np.ndarray:
    """Complex128 array with i.i.d. standard normal real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# the paper's heterogeneous-density benchmark with a density jump (nested
# cubes of 7 mm and 5 mm, lengths in mm, density relative to the exterior's
# 1000 kg/m^3, speeds relative to c0)

def benchmark4_density(xyz: np.ndarray) -> np.ndarray:
    """The inner cube's density: 2 - 0.8 sin(pi x/2.5) sin(pi y/2.5) cos(pi z/5)."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return 2.0 - 0.8 * np.sin(np.pi * x / 2.5) * np.sin(np.pi * y / 2.5) * np.cos(np.pi * z / 5.0)


def benchmark4_density_gradient(xyz: np.ndarray) -> np.ndarray:
    """Analytic gradient of benchmark4_density, (n, 3)."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    sx, cx = np.sin(np.pi * x / 2.5), np.cos(np.pi * x / 2.5)
    sy, cy = np.sin(np.pi * y / 2.5), np.cos(np.pi * y / 2.5)
    sz, cz = np.sin(np.pi * z / 5.0), np.cos(np.pi * z / 5.0)
    return -0.8 * np.stack([(np.pi / 2.5) * cx * sy * cz, (np.pi / 2.5) * sx * cy * cz,
                            -(np.pi / 5.0) * sx * sy * sz], axis=1)


def benchmark4_problem(n_shell: int = 9, n_inner: int = 43, lam0: float = 1.4):
    """The paper's 3D run of its fourth benchmark: exterior wavelength lam0 mm,
    incidence (1, 1, 0)/sqrt(2), c1 = c2 = c0/1.2, density 1 in Omega_0 and
    Omega_1 and benchmark4_density in Omega_2.  The default grid, 9 + 43 + 9
    cells per axis (61^3 = 226,981 cuboids, at most lam0/1.2/10 wide), is the
    10-voxel-per-interior-wavelength mesh of that run.
    Returns (mesh, materials, [k0], directions (1, 3), grad rho per cell)."""
    mesh = nested_cubes(n_shell, n_inner)
    mat = materials_piecewise(mesh, 1.0, 1.0, 1.0, 1.0 / 1.2, benchmark4_density, 1.0 / 1.2)
    grad = np.zeros((mesh.n_vol, 3))
    inner = mesh.vol_dom == 2
    grad[inner] = benchmark4_density_gradient(mesh.vol_xyz[inner])
    dirs = np.array([[1.0, 1.0, 0.0]]) / math.sqrt(2.0)
    return mesh, mat, [2.0 * math.pi / lam0], dirs, grad


# the paper's other three benchmarks (its first: a sphere in a cube against the
# spherical-harmonic series; its second: nested cubes with piecewise-constant
# density; its third: one cube with a smooth heterogeneous density).  Incidence
# along +x, the paper's default.

def benchmark1_problem(N: int = 29, lam0: float = 2.0):
    """Sphere of radius 2.5 (Omega_2, c2 = 5/6) inside the cube [-3, 3]^3
    (Omega_1, the exterior's material), constant density 1, exterior
    wavelength lam0, on a uniform N^3 staircase grid.  N = 29 gives 8.06 cells
    per interior wavelength (2 * 5/6 / (6/29)); odd N puts a layer of
    centroids on z = 0.  Returns (mesh, materials, [k0], directions, None)."""
    def dom(x):
        return np.where(np.sum(x * x, axis=1) < 2.5 ** 2, 2, 1)
    mesh = voxel_mesh(-3.0, 3.0, N, dom)
    mat = materials_piecewise(mesh, 1.0, 1.0, 1.0, 1.0, 1.0, 5.0 / 6.0)
    return mesh, mat, [2.0 * math.pi / lam0], np.array([[1.0, 0.0, 0.0]]), None


def benchmark2_problem(n_shell: int = 4, n_inner: int = 20, lam0: float = 3.0):
    """Nested cubes of 7 and 5 mm with density 1 in Omega_0 and Omega_1 and
    0.5 in Omega_2 (500 over 1000 kg/m^3), c1 = c2 = c0/1.2, exterior
    wavelength lam0 mm.  The default 4 + 20 + 4 grid has 0.25 mm cells: 10 per
    interior wavelength (3/1.2 mm)."""
    mesh = nested_cubes(n_shell, n_inner)
    mat = materials_piecewise(mesh, 1.0, 1.0, 1.0, 1.0 / 1.2, 0.5, 1.0 / 1.2)
    return mesh, mat, [2.0 * math.pi / lam0], np.array([[1.0, 0.0, 0.0]]), None


def benchmark3_density(xyz: np.ndarray) -> np.ndarray:
    """1 - 0.8 sin(pi x/3.5) sin(pi y/3.5) cos(pi z/7): continuous with the
    exterior's 1 on the faces of [-3.5, 3.5]^3."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return 1.0 - 0.8 * np.sin(np.pi * x / 3.5) * np.sin(np.pi * y / 3.5) * np.cos(np.pi * z / 7.0)


def benchmark3_density_gradient(xyz: np.ndarray) -> np.ndarray:
    """Analytic gradient of benchmark3_density, (n, 3)."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    sx, cx = np.sin(np.pi * x / 3.5), np.cos(np.pi * x / 3.5)
    sy, cy = np.sin(np.pi * y / 3.5), np.cos(np.pi * y / 3.5)
    sz, cz = np.sin(np.pi * z / 7.0), np.cos(np.pi * z / 7.0)
    return -0.8 * np.stack([(np.pi / 3.5) * cx * sy * cz, (np.pi / 3.5) * sx * cy * cz,
                            -(np.pi / 7.0) * sx * sy * sz], axis=1)


def benchmark3_problem(N: int = 21, lam0: float = 4.0):
    """One heterogeneous domain Omega_1 = [-3.5, 3.5]^3 mm (no Omega_2), c1 =
    c0/1.2, density benchmark3_density with its analytic gradient, exterior
    wavelength lam0 mm, uniform N^3 grid (N = 21: 10 cells per interior
    wavelength).  Returns (mesh, materials, [k0], directions, grad rho)."""
    mesh = voxel_mesh(-3.5, 3.5, N, lambda x: np.ones(x.shape[0], dtype=np.int32))
    mat = materials_piecewise(mesh, 1.0, 1.0, benchmark3_density, 1.0 / 1.2, 1.0, 1.0)
    grad = benchmark3_density_gradient(mesh.vol_xyz)
    return mesh, mat, [2.0 * math.pi / lam0], np.array([[1.0, 0.0, 0.0]]), grad


# ---------------------------------------------------------------------------
# the five workloads (nested spheres, heterogeneous core, batched incidences,
# log-normal medium with receivers, large cube + ellipsoid)

def _c_core(x):
    return 0.8 * (1.0 + 0.2 * np.exp(-np.sum(x * x, axis=1) / 0.05))


CONFIGS = {
    "c0": dict(kind="balls", N=16, k0=[2.0], dirs="z", core="const"),
    "c1": dict(kind="balls", N=48, k0=[10.0], dirs="z", core="smooth"),
    "c2": dict(kind="balls", N=57, k0=[16.0], dirs=128, core="smooth"),
    "c3": dict(kind="balls", N=48, k0=[10.0], dirs=8, core="lognormal", receivers=256),
    "c4": dict(kind="cube", N=100, k0=[40.0 - 2.0 * i for i in range(8)], dirs=16, core="lognormal4"),
}


def config_problem(name: str, N: int | None = None):
    """Return (mesh, materials, k0 list, directions (R,3), receivers or None)."""
    cfg = dict(CONFIGS[name])
    if N is not None:
        cfg["N"] = N
    if cfg["kind"] == "balls":
        mesh = nested_balls(cfg["N"])
        if cfg["core"] == "const":
            mat = materials_piecewise(mesh, 1.0, 1.0, 1.2, 1.5, 2.0, 0.8)
        else:
            mat = materials_piecewise(mesh, 1.0, 1.0, 1.2, 1.5, 2.0, _c_core)
        if cfg["core"] == "lognormal":
            x = mesh.vol_xyz
            mat.vol_c = mat.vol_c * lognormal_voxel_field(x, -1.0, 1.0, 32, 0.1, 0)
            mat.vol_rho = mat.vol_rho * lognormal_voxel_field(x, -1.0, 1.0, 32, 0.1, 1)
    else:
        mesh = cube_with_ellipsoid(cfg["N"])
        mat = materials_piecewise(mesh, 1.0, 1.0, 1.1, 1.3, 2.0, 0.8)
        mat.vol_c = mat.vol_c * lognormal_voxel_field(mesh.vol_xyz, -0.5, 0.5, 32, 0.1, 0)
    if cfg["dirs"] == "z":
        dirs = np.array([[0.0, 0.0, 1.0]])
    else:
        dirs = fibonacci_sphere(int(cfg["dirs"]))
    rec = fibonacci_sphere(cfg["receivers"], 3.0) if cfg.get("receivers") else None
    return mesh, mat, list(cfg["k0"]), dirs, rec
