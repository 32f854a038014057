"""Pins of the oracle's point-dipole functions (the paper's second source
kind, its "Mag FMM" for point-like dipole clouds, Sec. 4).

* A tetrahedron of volume V with the uniform magnetisation m / V becomes a
  point dipole m at its centroid as it shrinks: its exact potential (the tet
  closed form of the oracle) and its multipole coefficients (quadrature P2M
  of the oracle) approach the dipole ones at second order in the size.
* The dipole FMM converges to the O(N^2) dipole sum as p grows.
* Brute force on a few dipoles: the sum at a dipole's own position leaves
  that dipole out.
* Physics: dipoles m = M h^3 on a simple cubic lattice inside the unit
  sphere; at the lattice's body centres (inversion centres, where the
  neighbouring dipoles cancel in pairs) the potential approaches the
  continuum value M . r / 3 of the uniformly magnetised sphere.
"""
import numpy as np

import oracle as orc


def _small_tet(scale, rng):
    v = rng.standard_normal((4, 3))
    v -= v.mean(axis=0)
    return v * scale


def _vol(v):
    return abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0


def test_dipole_potential_is_the_small_tet_limit():
    rng = np.random.default_rng(0)
    base = _small_tet(1.0, rng)
    m = np.array([0.3, -0.7, 0.5])
    x = np.array([0.9, 0.4, -0.6])
    y = np.array([0.05, -0.02, 0.01])
    # sizes above the closed form's far-pair cancellation floor (which grows
    # as the tet shrinks relative to the distance)
    eps = (1e-1, 3e-2, 1e-2)
    errs = []
    for e in eps:
        v = base * e + y
        M = np.tile(m / _vol(v), (4, 1))
        ut = orc.tet_potential(x, v, M)
        ud = orc.dipole_potential(x, v.mean(axis=0), m)
        errs.append(abs(ut - ud) / abs(ud))
    for k in range(2):  # second order: the error falls with the square of the size
        assert errs[k + 1] < errs[k] * (eps[k + 1] / eps[k]) ** 2 * 1.5, errs
    assert errs[2] < 1e-4


def test_dipole_p2m_is_the_small_tet_limit():
    rng = np.random.default_rng(1)
    base = _small_tet(1.0, rng)
    m = np.array([-0.2, 0.9, 0.4])
    c = np.array([0.2, -0.1, 0.3])
    p = 6
    eps = (1e-1, 1e-2, 1e-3)
    errs = []
    for e in eps:
        v = base * e
        M = np.tile(m / _vol(v), (4, 1))
        Qt = orc.p2m_tet(v, M, c, p)
        Qd = orc.p2m_dipole(v.mean(axis=0), m, c, p)
        errs.append(np.linalg.norm(Qt - Qd) / np.linalg.norm(Qd))
    for k in range(2):  # second order (the centroid cancels the first-order term)
        assert errs[k + 1] < errs[k] * (eps[k + 1] / eps[k]) ** 2 * 1.5, errs
    # the monopole term vanishes and the first-order terms are the moment itself
    Qd = orc.p2m_dipole(np.zeros(3), m, c, p)
    mi = orc.multi_indices(p)
    assert Qd[0] == 0.0
    for k in range(1, 4):
        axis = int(np.argmax(mi[k]))
        assert Qd[k] == m[axis]


def test_dipole_fmm_converges_to_the_direct_sum():
    rng = np.random.default_rng(2)
    pts = rng.uniform(-1, 1, (1500, 3)) * [1.0, 0.6, 0.3]
    M = rng.standard_normal((2, pts.shape[0], 3))
    ref = orc.dipole_direct(pts, M)
    errs = []
    for p in (2, 4, 6, 8):
        u = orc.DipoleFMM(pts, p, 16, 0.5).evaluate(M)
        errs.append(max(np.linalg.norm(u[f] - ref[f]) / np.linalg.norm(ref[f]) for f in range(2)))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4, errs
    assert errs[-1] < errs[0] / 50, errs


def test_dipole_sum_leaves_out_the_own_dipole():
    pts = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 2.0, 0]])
    m = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    u = orc.dipole_direct(pts, m)
    for i in range(3):
        s = 0.0
        for j in range(3):
            if j == i:
                continue
            d = pts[i] - pts[j]
            s += m[j] @ d / (4 * np.pi * np.linalg.norm(d) ** 3)
        assert abs(u[i] - s) <= 1e-15 * max(1.0, abs(s))
    # a target off the points takes all three
    x = np.array([[0.3, 0.4, 0.5]])
    ux = orc.dipole_direct(pts, m, targets=x)
    assert abs(ux[0] - sum(orc.dipole_potential(x[0], pts[j], m[j]) for j in range(3))) < 1e-15


def test_lattice_sphere_approaches_the_uniform_sphere():
    h = 0.1
    g = np.arange(-1.0, 1.0 + h / 2, h)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pts = pts[np.linalg.norm(pts, axis=1) < 1.0]
    Mz = 1.0
    m = np.tile([0.0, 0.0, Mz * h ** 3], (pts.shape[0], 1))
    rng = np.random.default_rng(3)
    cen = np.round(rng.uniform(-0.45, 0.45, (60, 3)) / h) * h + h / 2  # body centres, |r| < 0.8
    u = orc.dipole_direct(pts, m, targets=cen)
    exact = Mz * cen[:, 2] / 3.0
    assert np.linalg.norm(u - exact) / np.linalg.norm(exact) < 0.05
    # and the FMM over the same lattice agrees with the direct sum
    uf = orc.DipoleFMM(pts, 8, 32, 0.5, targets=cen).evaluate(m)
    assert np.linalg.norm(uf - u) / np.linalg.norm(u) < 1e-4
