"""Pins of the oracle's exact tet-to-target potential and its direct sum.

The pair integral (Sec. 2.1, eq. approx1 for one tet) is checked against
 - closed forms of a box with uniform and with affine magnetisation, at every
   node of a Kuhn mesh that fills the box (targets at tet vertices, on edges,
   in face planes and inside): the summed tets must reproduce the box;
 - brute-force quadrature of the cone decomposition of Sec. 2.1.1 / 2.1.3
   (target as apex of four signed cones over the faces);
 - the point-dipole far field, linearity, rigid motions, scaling and corner
   permutations.
"""
import math

import numpy as np
import pytest

import meshgen
from tests import closed_forms as cf


def _gl_triangle(n):
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    S, T = np.meshgrid(x, x, indexing="ij")
    WS, WT = np.meshgrid(w, w, indexing="ij")
    return S.ravel(), (T * (1.0 - S)).ravel(), (WS * WT * (1.0 - S)).ravel()


def _composite_triangle(m, n):
    """Collapsed Gauss-Legendre (n x n) on each of the m^2 congruent sub-triangles."""
    s, t, w = _gl_triangle(n)
    S, T, W = [], [], []
    h = 1.0 / m
    for i in range(m):
        for j in range(m - i):
            S.append((i + s) * h)
            T.append((j + t) * h)
            W.append(w * h * h)
            if i + j < m - 1:
                S.append((i + 1 - s) * h)
                T.append((j + 1 - t) * h)
                W.append(w * h * h)
    return np.concatenate(S), np.concatenate(T), np.concatenate(W)


_RULE = _composite_triangle(8, 24)


def cone_quadrature(x, v, M, rule=_RULE):
    """u_T(x) from the cone decomposition with apex x:

        int_T f = sum_k h_k int_{F_k} int_0^1 lam^2 f(x + lam (y - x)) dlam dA_y,

    which for f = M . (x - r')/|x - r'|^3 with affine M gives
        u_T(x) = -1/(4 pi) sum_k h_k int_{F_k} M((x+y)/2) . (y-x)/|y-x|^3 dA_y
    (h_k = n_k.(y - x), outward n_k).  Faces are integrated with collapsed
    Gauss-Legendre on 64 sub-triangles; accurate to ~1e-14 when x keeps at
    least 3% of the longest edge away from the planes of faces with h_k != 0.
    """
    s, t, w = rule
    J = np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]], axis=1)
    Ji = np.linalg.inv(J)
    tot = 0.0
    for k in range(4):
        f = [i for i in range(4) if i != k]
        a, b, c = v[f[0]], v[f[1]], v[f[2]]
        nn = np.cross(b - a, c - a)
        area2 = np.linalg.norm(nn)
        nk = nn / area2
        if np.dot(nk, v[k] - a) > 0:
            nk = -nk
        h = np.dot(nk, a - x)
        if any(np.array_equal(x, p) for p in (a, b, c)) or h == 0.0:
            continue
        y = a[None] + s[:, None] * (b - a)[None] + t[:, None] * (c - a)[None]
        mid = 0.5 * (x[None] + y)
        lam = (mid - v[0][None]) @ Ji.T
        Mm = np.concatenate([1.0 - lam.sum(1, keepdims=True), lam], axis=1) @ M
        d = y - x[None]
        r = np.linalg.norm(d, axis=1)
        tot += h * np.sum(w * np.einsum("ij,ij->i", Mm, d) / r ** 3) * area2
    return -tot / (4.0 * math.pi)


def _well_shaped_tet(rng):
    while True:
        v = rng.uniform(-1.0, 1.0, (4, 3))
        vol = abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0
        L = max(np.linalg.norm(v[i] - v[j]) for i in range(4) for j in range(i))
        if vol / L ** 3 > 0.02:  # regular tet: 0.118
            return v, L


def _face_heights(x, v):
    hs = []
    for k in range(4):
        f = [i for i in range(4) if i != k]
        a, b, c = v[f[0]], v[f[1]], v[f[2]]
        nn = np.cross(b - a, c - a)
        hs.append(abs(np.dot(nn / np.linalg.norm(nn), a - x)))
    return np.array(hs)


def _placements(rng, v, L):
    """Targets: outside near/far, inside, at a corner, in a face plane, on an edge line."""
    out = []
    while len(out) < 6:
        kind = len(out)
        if kind == 0:
            x = v.mean(0) + rng.uniform(-2.5, 2.5, 3) * L
        elif kind == 1:
            x = rng.dirichlet(np.ones(4)) @ v
        elif kind == 2:
            x = v[rng.integers(4)].copy()
        elif kind == 3:
            f = rng.choice(4, 3, replace=False)
            l = rng.uniform(-0.8, 1.8, 2)
            x = v[f[0]] + l[0] * (v[f[1]] - v[f[0]]) + l[1] * (v[f[2]] - v[f[0]])
        elif kind == 4:
            i, j = rng.choice(4, 2, replace=False)
            t = rng.choice([-1.0, 1.0]) * rng.uniform(1.3, 2.5)
            x = v[i] + t * (v[j] - v[i])
        else:
            x = v.mean(0) + rng.uniform(-1.0, 1.0, 3) * 0.9 * L
        h = _face_heights(x, v)
        nz = h[h > 1e-12 * L]
        if nz.size and nz.min() < 0.03 * L:
            continue
        out.append((kind, x))
    return out


def test_pair_vs_cone_quadrature(orc):
    """Paper's own check (Sec. 4): random tets, random nodal M, vs numerical integration."""
    rng = np.random.default_rng(20160601)
    worst = 0.0
    count = 0
    for _ in range(40):
        v, L = _well_shaped_tet(rng)
        M = rng.standard_normal((4, 3))
        for kind, x in _placements(rng, v, L):
            a = orc.tet_potential(x, v, M)
            b = cone_quadrature(x, v, M)
            scale = np.abs(M).max() * L * L / max(np.linalg.norm(x - v.mean(0)), L)
            err = abs(a - b) / scale
            worst = max(worst, err)
            count += 1
            assert err < 1e-12, (kind, x, v, M, a, b)
    assert count == 240
    assert worst < 1e-12


def test_pair_far_field_is_dipole(orc):
    """u_T(x) -> 1/(4 pi) m.(x - c)/|x - c|^3 with m = int_T M, relative error O(diam/d)."""
    rng = np.random.default_rng(7)
    v, L = _well_shaped_tet(rng)
    M = rng.standard_normal((4, 3))
    vol = abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0
    c = v.mean(0)
    m = vol * M.mean(0)  # exact integral of an affine field
    direction = rng.standard_normal(3)
    direction /= np.linalg.norm(direction)
    errs = []
    for d in (4.0, 8.0, 16.0, 32.0, 64.0):
        x = c + d * L * direction
        r = x - c
        dip = np.dot(m, r) / np.linalg.norm(r) ** 3 / (4.0 * math.pi)
        errs.append(abs(orc.tet_potential(x, v, M) - dip) / abs(dip))
    # centred at the centroid the quadrupole term of a linear M is O((diam/d)^1):
    # the error must fall at least ~x2 for each doubling of d
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.6 * e0
    assert errs[-1] < 2e-2


def test_pair_structure(orc):
    """Linearity in M, rigid motions, scaling u(s x; s v) = s u, corner permutation."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        v, L = _well_shaped_tet(rng)
        M1 = rng.standard_normal((4, 3))
        M2 = rng.standard_normal((4, 3))
        x = v.mean(0) + rng.uniform(-2, 2, 3) * L
        # natural size of u for this pair (the potential can cancel far below it)
        scale = max(np.abs(M1).max(), np.abs(M2).max()) * L * L / max(np.linalg.norm(x - v.mean(0)), L)
        u1, u2 = orc.tet_potential(x, v, M1), orc.tet_potential(x, v, M2)
        u12 = orc.tet_potential(x, v, 2.0 * M1 - 3.0 * M2)
        assert abs(u12 - (2 * u1 - 3 * u2)) <= 1e-13 * scale
        # rotation + translation, M rotated with the body
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        tr = rng.standard_normal(3)
        ur = orc.tet_potential(Q @ x + tr, v @ Q.T + tr, M1 @ Q.T)
        assert abs(ur - u1) <= 1e-13 * scale
        # scaling by s: u is homogeneous of degree 1 in length
        s = 2.0 ** rng.integers(-3, 4) * 1.37
        us = orc.tet_potential(s * x, s * v, M1)
        assert abs(us - s * u1) <= 1e-13 * scale * s
        # corner permutation (either orientation)
        perm = rng.permutation(4)
        up = orc.tet_potential(x, v[perm], M1[perm])
        assert abs(up - u1) <= 1e-13 * scale


@pytest.mark.parametrize("direction", [(0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (0.3, -0.5, 0.8)])
def test_direct_uniform_box_closed_form(orc, direction):
    """Uniform M on a jittered Kuhn cube: the tets fill the box and M is affine,
    so the nodal direct sum equals the surface-charge closed form exactly."""
    nodes, tets = meshgen.box_mesh(6, jitter=0.15, seed=0)
    M = meshgen.uniform_field(nodes.shape[0], direction)
    u = orc.direct(nodes, tets, M)
    ue = np.array([cf.box_potential_uniform(p, np.asarray(direction)) for p in nodes])
    assert np.linalg.norm(u - ue) / np.linalg.norm(ue) < 1e-13
    assert np.abs(u - ue).max() < 1e-13


def test_direct_affine_box_closed_form(orc):
    """Affine M = A r + b on a jittered Kuhn box: surface charge linear on the
    faces plus the constant volume charge -tr A, all in closed form."""
    nodes, tets = meshgen.box_mesh((5, 4, 6), lo=(-0.3, 0.1, 0.0), hi=(0.9, 0.7, 1.5), jitter=0.15, seed=4)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    M = nodes @ A.T + b
    u = orc.direct(nodes, tets, M)
    ue = np.array([cf.box_potential_affine(p, A, b, (-0.3, 0.1, 0.0), (0.9, 0.7, 1.5)) for p in nodes])
    assert np.linalg.norm(u - ue) / np.linalg.norm(ue) < 1e-13
    # off-mesh targets too (outside and inside the box)
    tg = np.array([[1.7, 0.3, -0.4], [0.31, 0.42, 0.77], [-0.3, 0.1, 0.75], [0.9, 0.2, 1.5]])
    ut = orc.direct(nodes, tets, M, targets=tg)
    ute = np.array([cf.box_potential_affine(p, A, b, (-0.3, 0.1, 0.0), (0.9, 0.7, 1.5)) for p in tg])
    assert np.abs(ut - ute).max() < 1e-13 * np.abs(ute).max() * 10


def test_closed_form_box_newton_potential_numeric():
    """Pin of the pin: the box volume integral against adaptive cubature."""
    from scipy import integrate
    xe = np.array([1.7, 0.3, -0.4])
    num, _ = integrate.tplquad(lambda z, y, x: 1.0 / math.sqrt((x - xe[0]) ** 2 + (y - xe[1]) ** 2 + (z - xe[2]) ** 2),
                               0, 1, 0, 1, 0, 1, epsabs=1e-13, epsrel=1e-12)
    assert abs(cf.box_newton_potential(xe, (0, 0, 0), (1, 1, 1)) - num) < 1e-11


def test_direct_multi_field_and_targets(orc):
    nodes, tets = meshgen.box_mesh(3, seed=1)
    M = meshgen.random_fields(nodes.shape[0], F=3, seed=1)
    u = orc.direct(nodes, tets, M)
    for f in range(3):
        assert np.array_equal(u[f], orc.direct(nodes, tets, M[f]))
    with pytest.raises(ValueError):
        bad = tets.copy()
        bad[0, 0] = nodes.shape[0]
        orc.direct(nodes, bad, M[0])
