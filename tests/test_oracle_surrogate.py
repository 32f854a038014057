"""Pins of the surrogate's training targets (oracle/mlp.py): the network
predicts the residual of the pair integral (Sec. 2.1) after the tet's own
quadrupole expansion (Sec. 2.2); rebuilding the pair from the exact targets
must give the exact integral on the unscaled geometry for any nodal M
(within 1e-13 of |M| V / (4 pi d^2)), and
the quadrupole part must be the tet's far field to the expected order."""
import numpy as np

import meshgen
from oracle import mlp


def _pairs(rng, n, lo=2.0, hi=6.0):
    nodes, tets = meshgen.box_mesh(5, seed=3)
    out = []
    for _ in range(n):
        v = nodes[tets[rng.integers(tets.shape[0])]]
        c = v.mean(0)
        d = max(np.linalg.norm(v[a] - v[b]) for a in range(4) for b in range(a + 1, 4))
        e = rng.standard_normal(3)
        x = c + rng.uniform(lo, hi) * d * e / np.linalg.norm(e)
        out.append((x, v))
    return out


def test_targets_rebuild_the_exact_pair(orc):
    rng = np.random.default_rng(17)
    for x, v in _pairs(rng, 40):
        dist = np.linalg.norm(x - v.mean(0))
        s = (v - x) / dist
        # the pair integral by the 12^3-point Gauss rule (at round-off from 2
        # diameters, where the closed forms keep only ~1e-12 of the pair)
        def exact(xx, vv, MM):
            return orc.tet_potential_gauss(xx, vv, MM, 12)
        y = mlp.surrogate_target(s, exact, orc.p2m_tet, orc.taylor_coeffs)
        M = rng.standard_normal((4, 3))
        u = mlp.pair_from_target(s, y, M, dist, orc.p2m_tet, orc.taylor_coeffs)
        ref = exact(x, v, M)
        vol = abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0
        scale = np.abs(M).max() * vol / (4 * np.pi * dist ** 2)
        assert abs(u - ref) <= 1e-13 * scale, (u, ref)


def test_features_round_trip():
    rng = np.random.default_rng(20)
    for x, v in _pairs(rng, 20):
        dist = np.linalg.norm(x - v.mean(0))
        s = (v - x) / dist
        f = mlp.surrogate_features(s)
        assert f.shape == (16,)
        assert abs(np.linalg.norm(f[:3]) - 1.0) < 1e-15
        assert 1.0 / 6.0 < f[15] <= 0.5
        assert np.abs(mlp.corners_from_features(f) - s).max() < 1e-14


def test_targets_are_order_one(orc):
    rng = np.random.default_rng(18)
    ys = []
    for x, v in _pairs(rng, 60):
        dist = np.linalg.norm(x - v.mean(0))
        ys.append(mlp.surrogate_target((v - x) / dist, orc.tet_potential, orc.p2m_tet, orc.taylor_coeffs))
    rms = np.sqrt(np.mean(np.square(ys)))
    assert 0.1 < rms < 10.0, rms


def test_quadrupole_part_is_the_far_field(orc):
    """The residual after the quadrupole expansion is the octupole term and
    beyond: relative to the pair's size |M| V / (4 pi r^2) it falls like
    (diam/r)^2, x4 per doubling of r."""
    rng = np.random.default_rng(19)
    nodes, tets = meshgen.box_mesh(4, seed=1)
    for t in (5, 77, 200):
        v = nodes[tets[t]]
        M = rng.standard_normal((4, 3))
        c = v.mean(0)
        vol = abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        d = max(np.linalg.norm(v[a] - v[b]) for a in range(4) for b in range(a + 1, 4))
        rel = []
        for r in (2.0, 4.0, 8.0, 16.0):
            x = c + r * d * e
            ex = orc.tet_potential_gauss(x, v, M, 12)
            q = mlp.quadrupole_potential(x, v, M, orc.p2m_tet, orc.taylor_coeffs)
            rel.append(abs(ex - q) / (np.abs(M).max() * vol / (4 * np.pi * (r * d) ** 2)))
        for a, b in zip(rel, rel[1:]):
            assert b < a / 3.5, rel
        assert rel[0] < 5e-2, rel
