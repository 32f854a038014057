"""Seeded synthetic inputs: tetrahedral meshes and nodal magnetisation fields.

This module produces inputs only and holds none of the method's arithmetic.
Both the oracle side (tests) and the product side (tests, benchmark) take
their inputs from here.

Meshes are structured boxes of cubes, each cube cut into the 6 Kuhn
tetrahedra (one per permutation of the axes), with interior nodes optionally
jittered.  Node (i, j, k) has index i + (nx+1) (j + (ny+1) k).
"""
import itertools
import math

import numpy as np

_PERMS = list(itertools.permutations(range(3)))


def box_mesh(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), jitter=0.15, seed=0):
    """Box [lo, hi] cut into n = (nx, ny, nz) cubes (or an int), 6 Kuhn tets each.

    Interior nodes get i.i.d. U(-jitter h, +jitter h) per coordinate (h the
    cube side along that axis); boundary nodes stay on the box surface so the
    tets fill the box exactly.  Returns (nodes [N,3] f64, tets [T,4] i32).
    """
    if np.isscalar(n):
        n = (int(n),) * 3
    nx, ny, nz = (int(v) for v in n)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    h = (hi - lo) / np.array([nx, ny, nz], dtype=np.float64)
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    i, j, k = (a.transpose(2, 1, 0).ravel() for a in (i, j, k))  # node index i + (nx+1)(j + (ny+1)k)
    nodes = np.stack([lo[0] + i * h[0], lo[1] + j * h[1], lo[2] + k * h[2]], axis=1)
    if jitter:
        rng = np.random.default_rng(seed)
        interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
        dis = rng.uniform(-jitter, jitter, size=(nodes.shape[0], 3)) * h
        nodes = nodes + np.where(interior[:, None], dis, 0.0)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = (a.transpose(2, 1, 0).ravel() for a in (ci, cj, ck))

    def nid(a, b, c):
        return a + (nx + 1) * (b + (ny + 1) * c)

    tets = []
    for perm in _PERMS:
        corners = [np.zeros(3, dtype=np.int64)]
        cur = np.zeros(3, dtype=np.int64)
        for ax in perm:
            cur = cur.copy()
            cur[ax] += 1
            corners.append(cur)
        tets.append(np.stack([nid(ci + c[0], cj + c[1], ck + c[2]) for c in corners], axis=1))
    tets = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return np.ascontiguousarray(nodes), np.ascontiguousarray(tets)


def unit_vectors(n, seed):
    """n i.i.d. unit vectors, uniform on the sphere (normalised N(0, I3))."""
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((n, 3))
    return m / np.linalg.norm(m, axis=1, keepdims=True)


def random_fields(n_nodes, F=1, seed=1):
    """F i.i.d. unit nodal fields, field f drawn with seed `seed + f`: [F, n_nodes, 3]."""
    return np.stack([unit_vectors(n_nodes, seed + f) for f in range(F)])


def lumped_volumes(nodes, tets):
    """Per node a quarter of the volume of every tet around it (sums to the
    mesh volume): the weights that turn nodal magnetisation into the moments
    of a point-dipole cloud on the same nodes."""
    v = nodes[tets]
    vol = np.abs(np.einsum("ij,ij->i", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))) / 6.0
    w = np.zeros(nodes.shape[0])
    for c in range(4):
        np.add.at(w, tets[:, c], vol / 4.0)
    return w


def uniform_field(n_nodes, direction):
    d = np.asarray(direction, dtype=np.float64)
    return np.tile(d, (n_nodes, 1))


def vortex_field(nodes, centre, half_width, mz=0.1, noise=0.05, seed=1):
    """Vortex m ~ (-y', x', mz) + noise N(0, I) per node, renormalised.

    x', y' are the lateral coordinates about `centre`, divided by `half_width`.
    """
    rng = np.random.default_rng(seed)
    xp = (nodes[:, 0] - centre[0]) / half_width
    yp = (nodes[:, 1] - centre[1]) / half_width
    m = np.stack([-yp, xp, np.full_like(xp, mz)], axis=1)
    m = m + noise * rng.standard_normal(m.shape)
    return m / np.linalg.norm(m, axis=1, keepdims=True)


def sphere_mesh(n, radius=1.0, jitter=0.15, seed=0):
    """Jittered n^3 Kuhn grid on [-r, r]^3, keeping tets whose centroid has |c| < r.

    Unused nodes are dropped and the rest renumbered in order.
    """
    nodes, tets = box_mesh(n, lo=(-radius,) * 3, hi=(radius,) * 3, jitter=jitter, seed=seed)
    cen = nodes[tets].mean(axis=1)
    keep = np.linalg.norm(cen, axis=1) < radius
    tets = tets[keep]
    used = np.unique(tets)
    remap = -np.ones(nodes.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    return np.ascontiguousarray(nodes[used]), np.ascontiguousarray(remap[tets].astype(np.int32))


def film_mesh(nx=512, ny=512, nz=4, half=64.0, thickness=1.0):
    """Unjittered thin film [-half, half]^2 x [0, thickness] of Kuhn tets."""
    return box_mesh((nx, ny, nz), lo=(-half, -half, 0.0), hi=(half, half, thickness), jitter=0.0)


def ragged_sizes(count=32, tmin=2.0e3, tmax=2.0e5, seed=2):
    """Cube resolutions n_i = round((T_i/6)^(1/3)), T_i log-uniform in [tmin, tmax]."""
    rng = np.random.default_rng(seed)
    T = np.exp(rng.uniform(math.log(tmin), math.log(tmax), size=count))
    return [int(round((t / 6.0) ** (1.0 / 3.0))) for t in T]


# Named workloads (mesh sizes of the paper-style box experiment and its
# larger relatives).  Each entry: mesh builder + FMM parameters.
WORKLOADS = {
    "cube8": dict(n=8, p=6, leaf=32),
    "cube40": dict(n=40, p=8, leaf=64),
    "cube64": dict(n=64, p=8, leaf=64),
}


def cube_workload(name, jitter=0.15, seed=0):
    w = WORKLOADS[name]
    nodes, tets = box_mesh(w["n"], jitter=jitter, seed=seed)
    return nodes, tets, w["p"], w["leaf"]
