"""Pins of the oracle's far-pair branch of the direct sum.

Far from a tet the closed-form pair integral (Sec. 2.1) adds face and edge
terms much larger than their sum, so the direct sum switches to a Gauss
product rule on the collapsed cube beyond 3 tet diameters.  The rule is
pinned by
 - its 1-D Gauss-Legendre nodes and weights against numpy's;
 - the independent cone-decomposition quadrature of Sec. 2.1.1 at 2-10
   diameters (the overlap band where both are accurate);
 - geometric convergence in the number of points;
 - the closed form where the latter is still accurate (3-4 diameters);
 - the point-dipole limit far away;
 - the uniform-box closed form of the whole direct sum (test_oracle_pair).
"""
import math

import numpy as np

from tests.test_oracle_pair import _well_shaped_tet, cone_quadrature


def _scale(v, M, d):
    vol = abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0
    return np.abs(M).max() * vol / (4.0 * math.pi * d * d)


def _target(rng, v, L, ratio):
    d = rng.standard_normal(3)
    return v.mean(0) + ratio * L * d / np.linalg.norm(d)


def test_gauss_legendre_rule_matches_numpy(orc):
    for n in (1, 2, 5, 8, 13, 24):
        t, w = orc.gauss_legendre01(n)
        x, wr = np.polynomial.legendre.leggauss(n)
        o = np.argsort(t)
        assert np.allclose(np.sort(0.5 * (x + 1.0)), t[o], rtol=0, atol=2e-16)
        assert np.allclose(0.5 * wr[np.argsort(0.5 * (x + 1.0))], w[o], rtol=0, atol=3e-16)


def test_distance_ratio(orc):
    rng = np.random.default_rng(5)
    for _ in range(10):
        v, L = _well_shaped_tet(rng)
        x = rng.standard_normal(3) * 3
        assert abs(orc.tet_distance_ratio(x, v) - np.linalg.norm(x - v.mean(0)) / L) <= 1e-15 * (1 + np.linalg.norm(x))


def test_gauss_vs_cone_quadrature_overlap_band(orc):
    """2-10 diameters: the degree-13 rule against the cone decomposition (whose
    face terms cancel like d/diam far away: it holds ~1e-13 of |M| V/(4 pi d^2)
    there, the rule ~3e-15, measured against its own 20-point form)."""
    rng = np.random.default_rng(160600247)
    med = []
    for _ in range(30):
        v, L = _well_shaped_tet(rng)
        M = rng.standard_normal((4, 3))
        for ratio in (2.0, 3.0, 4.0, 6.0, 8.0, 10.0):
            x = _target(rng, v, L, ratio)
            g = orc.tet_potential_gauss(x, v, M, 8)
            c = cone_quadrature(x, v, M)
            err = abs(g - c) / _scale(v, M, ratio * L)
            assert err < (1e-12 if ratio < 3.0 else 5e-13), (ratio, err)
            med.append(err)
    assert np.median(med) < 2e-14


def test_gauss_converges_geometrically(orc):
    """At 4 diameters the error falls by a large factor per added point up to round-off."""
    rng = np.random.default_rng(8)
    for _ in range(5):
        v, L = _well_shaped_tet(rng)
        M = rng.standard_normal((4, 3))
        x = _target(rng, v, L, 4.0)
        ref = orc.tet_potential_gauss(x, v, M, 20)
        s = _scale(v, M, 4.0 * L)
        e = [abs(orc.tet_potential_gauss(x, v, M, n) - ref) / s for n in (2, 3, 4, 5, 6)]
        for a, b in zip(e, e[1:]):
            assert b < a / 5.0 or b < 1e-14
        assert abs(orc.tet_potential_gauss(x, v, M, 8) - ref) / s < 1e-14


def test_gauss_vs_closed_form_where_both_hold(orc):
    """3-4 diameters, where the closed form still keeps ~12 digits."""
    rng = np.random.default_rng(9)
    for _ in range(40):
        v, L = _well_shaped_tet(rng)
        M = rng.standard_normal((4, 3))
        ratio = rng.uniform(3.0, 4.0)
        x = _target(rng, v, L, ratio)
        s = _scale(v, M, ratio * L)
        assert abs(orc.tet_potential_gauss(x, v, M, 8) - orc.tet_potential(x, v, M)) / s < 1e-10


def test_direct_pair_switch(orc):
    rng = np.random.default_rng(10)
    v, L = _well_shaped_tet(rng)
    M = rng.standard_normal((4, 3))
    for ratio, far in ((2.9, False), (3.1, True), (50.0, True)):
        x = _target(rng, v, L, ratio)
        want = orc.tet_potential_gauss(x, v, M, 8) if far else orc.tet_potential(x, v, M)
        assert orc.tet_potential_direct(x, v, M) == want


def test_gauss_far_field_is_dipole(orc):
    """u_T(x) -> m.(x - c)/(4 pi |x - c|^3), relative error O(diam/d), down to 1e-4."""
    rng = np.random.default_rng(7)
    v, L = _well_shaped_tet(rng)
    M = rng.standard_normal((4, 3))
    vol = abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0
    c = v.mean(0)
    m = vol * M.mean(0)
    direction = rng.standard_normal(3)
    direction /= np.linalg.norm(direction)
    errs = []
    for d in (16.0, 64.0, 256.0, 1024.0, 4096.0):
        x = c + d * L * direction
        r = x - c
        dip = np.dot(m, r) / np.linalg.norm(r) ** 3 / (4.0 * math.pi)
        errs.append(abs(orc.tet_potential_gauss(x, v, M, 8) - dip) / abs(dip))
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.3 * e0
    assert errs[-1] < 1e-4
