"""Pins of the oracle's expansion operators (Secs. 2.2-2.3).

 - Taylor coefficients a_n(x) of 1/|x - y| against symbolic derivatives.
 - P2M (eq. expCoeffs) against exact rational integration over the tet.
 - M2M and L2L are exact re-centrings: shifted == computed at the new centre.
 - P2M -> M2L -> L2P converges to the exact pair integrals as p grows, at the
   rate set by the opening angle (Sec. 2.2 truncation law).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp


def test_multi_index_order(orc):
    for p in (0, 1, 4, 8):
        mi = orc.multi_indices(p)
        assert mi.shape == (orc.ncoef(p), 3)
        deg = mi.sum(1)
        assert (np.diff(deg) >= 0).all() and deg.max() == p
        assert len({tuple(r) for r in mi}) == mi.shape[0]


def test_taylor_coefficients_vs_symbolic(orc):
    """a_n(x) = (-1)^|n|/n! d^n/dx^n (1/|x|), so 1/|x - y| = sum_n a_n(x) y^n."""
    X, Y, Z = sp.symbols("X Y Z", real=True)
    f = 1 / sp.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    p = 8
    mi = orc.multi_indices(p)
    rng = np.random.default_rng(1)
    pts = [rng.uniform(-2, 2, 3) for _ in range(2)] + [np.array([0.3, 0.0, 0.0]), np.array([0.0, -1.1, 0.4])]
    derivs = {}
    for n in mi:
        key = tuple(int(k) for k in n)
        d = f
        for var, k in zip((X, Y, Z), key):
            if k:
                d = sp.diff(d, var, k)
        derivs[key] = sp.lambdify((X, Y, Z), d, "math")
    for x in pts:
        a = orc.taylor_coeffs(x, p)
        for i, n in enumerate(mi):
            key = tuple(int(k) for k in n)
            nf = math.factorial(key[0]) * math.factorial(key[1]) * math.factorial(key[2])
            ref = (-1) ** sum(key) / nf * derivs[key](*x)
            scale = np.linalg.norm(x) ** (-sum(key) - 1)
            assert abs(a[i] - ref) <= 1e-14 * scale * 10, (key, a[i], ref)


def _exact_p2m(v, M, c, p, mi):
    """Q_n = int_T M . grad (y - c)^n dy in exact rational arithmetic.

    y = sum_i lam_i v_i over the tet; monomials of the barycentric coordinates
    integrate to 6|V| alpha!/(|alpha|+3)!.
    """
    l = sp.symbols("l0:4")
    v = [[Fraction(x) for x in row] for row in v]
    M = [[Fraction(x) for x in row] for row in M]
    c = [Fraction(x) for x in c]
    J = sp.Matrix([[v[j][d] - v[0][d] for j in (1, 2, 3)] for d in range(3)])
    vol6 = abs(J.det())
    y = [sum(l[i] * v[i][d] for i in range(4)) - c[d] for d in range(3)]
    Mk = [sum(l[i] * M[i][d] for i in range(4)) for d in range(3)]

    def integrate(expr):
        P = sp.Poly(sp.expand(expr), *l)
        s = sp.Rational(0)
        for mon, coef in P.terms():
            num = math.prod(math.factorial(a) for a in mon)
            s += coef * sp.Rational(num, math.factorial(sum(mon) + 3))
        return s * vol6

    out = []
    for n in mi:
        n = [int(k) for k in n]
        expr = 0
        for k in range(3):
            if n[k] == 0:
                continue
            m = list(n)
            m[k] -= 1
            expr += n[k] * Mk[k] * y[0] ** m[0] * y[1] ** m[1] * y[2] ** m[2]
        out.append(float(integrate(expr)) if expr != 0 else 0.0)
    return np.array(out)


def test_p2m_vs_exact_rational_moments(orc):
    rng = np.random.default_rng(3)
    p = 5
    mi = orc.multi_indices(p)
    v = np.round(rng.uniform(-1, 1, (4, 3)), 3)
    M = np.round(rng.standard_normal((4, 3)), 3)
    c = np.array([0.25, -0.125, 0.5])
    Q = orc.p2m_tet(v, M, c, p)
    Qe = _exact_p2m(v, M, c, p, mi)
    scale = np.abs(Qe).max()
    assert np.abs(Q - Qe).max() <= 1e-13 * scale
    assert Q[0] == 0.0
    # degree-1 coefficients are the total moment int_T M
    vol = abs(np.linalg.det(np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]))) / 6.0
    for k, e in enumerate(([1, 0, 0], [0, 1, 0], [0, 0, 1])):
        i = int(np.where((mi == e).all(1))[0][0])
        assert abs(Q[i] - vol * M[:, k].mean()) <= 1e-14 * np.abs(M).max()


@pytest.mark.parametrize("p", [2, 6, 8])
def test_p2m_exact_degree(orc, p):
    """The quadrature is exact for every |n| <= p: compare the top degree too
    (p=8 needs a rule of degree 8), at a far centre where rounding is benign."""
    rng = np.random.default_rng(p)
    mi = orc.multi_indices(p)
    v = np.round(rng.uniform(-1, 1, (4, 3)), 2)
    M = np.round(rng.standard_normal((4, 3)), 2)
    c = np.array([0.5, 0.5, 0.5])
    if p >= 6:  # the rational reference is slow: check the highest degrees only
        sel = np.where(mi.sum(1) >= p - 1)[0][:: (3 if p < 8 else 6)]
    else:
        sel = np.arange(mi.shape[0])
    Q = orc.p2m_tet(v, M, c, p)
    Qe = _exact_p2m(v, M, c, p, mi[sel])
    assert np.abs(Q[sel] - Qe).max() <= 1e-12 * max(np.abs(Qe).max(), 1e-300)


def test_m2m_exact(orc):
    rng = np.random.default_rng(5)
    p = 8
    v = rng.uniform(0.0, 0.2, (4, 3))
    M = rng.standard_normal((4, 3))
    cc = np.array([0.1, 0.1, 0.1])
    cp = np.array([0.2, 0.0, 0.15])
    Qc = orc.p2m_tet(v, M, cc, p)
    Qp = orc.p2m_tet(v, M, cp, p)
    Qs = orc.m2m(Qc, cc - cp, p)
    assert np.abs(Qs - Qp).max() <= 1e-13 * np.abs(Qp).max()


def test_l2l_exact_and_l2p(orc):
    """A local expansion shifted to a child evaluates to the same polynomial."""
    rng = np.random.default_rng(6)
    p = 8
    L = rng.standard_normal(orc.ncoef(p))
    cp = np.array([0.0, 0.0, 0.0])
    cc = np.array([0.25, -0.25, 0.25])
    Lc = orc.l2l(L, cc - cp, p)
    for _ in range(5):
        x = cc + rng.uniform(-0.25, 0.25, 3)
        u1 = orc.l2p(L, x, cp, p)
        u2 = orc.l2p(Lc, x, cc, p)
        assert abs(u1 - u2) <= 1e-13 * max(1.0, abs(u1))
    # L2P is the plain polynomial sum_m l_m (x - c)^m
    mi = orc.multi_indices(p)
    x = np.array([0.3, -0.2, 0.1])
    ref = sum(L[i] * np.prod((x - cp) ** mi[i]) for i in range(mi.shape[0]))
    assert abs(orc.l2p(L, x, cp, p) - ref) <= 1e-14 * np.abs(L).sum()


def test_m2l_chain_converges_to_exact(orc):
    """u(x) of a source cluster through P2M -> M2L -> L2P approaches the exact
    pair integrals as p grows; error ~ (opening angle)^(p+1)."""
    rng = np.random.default_rng(9)
    cB = np.array([0.0, 0.0, 0.0])
    cA = np.array([3.0, 1.0, -0.5])
    tets = []
    for _ in range(5):
        base = cB + rng.uniform(-0.3, 0.3, 3)
        tets.append((base + rng.uniform(-0.15, 0.15, (4, 3)), rng.standard_normal((4, 3))))
    xs = [cA + rng.uniform(-0.3, 0.3, 3) for _ in range(4)]
    exact = np.array([sum(orc.tet_potential(x, v, M) for v, M in tets) for x in xs])
    errs = []
    for p in (2, 4, 6, 8, 10, 12):
        Q = sum(orc.p2m_tet(v, M, cB, p) for v, M in tets)
        Lc = orc.m2l(Q, cA - cB, p)
        approx = np.array([orc.l2p(Lc, x, cA, p) for x in xs])
        errs.append(np.abs(approx - exact).max() / np.abs(exact).max())
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.2 * e0
    assert errs[-1] < 1e-8


def test_multipole_far_field_formula(orc):
    """u(x) ~ 1/(4 pi) sum_n a_n(x - c) Q_n (multipole evaluated directly)."""
    rng = np.random.default_rng(10)
    p = 10
    mi = orc.multi_indices(p)
    v = rng.uniform(-0.2, 0.2, (4, 3))
    M = rng.standard_normal((4, 3))
    c = np.zeros(3)
    Q = orc.p2m_tet(v, M, c, p)
    x = np.array([1.5, -1.2, 0.9])
    a = orc.taylor_coeffs(x - c, p)
    approx = np.dot(a, Q) / (4 * math.pi)
    exact = orc.tet_potential(x, v, M)
    assert abs(approx - exact) <= 1e-10 * abs(exact)
    assert len(mi) == len(Q)


def test_taylor_coefficients_harmonic_and_reduced_contraction(orc):
    """1/|x| is harmonic, so D_n = (-1)^|n| n! a_n satisfies
    D_{n+2e_x} + D_{n+2e_y} + D_{n+2e_z} = 0.  Hence the truncated M2L sum
    sum_n D_{n+m} q_n (|n| + |m| <= p) over all n equals the sum over n_z <= 1
    of a reduced q (each n_z >= 2 term folded onto same-degree n_z <= 1 terms),
    and the outputs with m_z >= 2 follow from those with m_z <= 1."""
    p = 8
    mi = [tuple(int(k) for k in n) for n in orc.multi_indices(p)]
    idx = {n: i for i, n in enumerate(mi)}
    fact = lambda n: math.factorial(n[0]) * math.factorial(n[1]) * math.factorial(n[2])
    rng = np.random.default_rng(5)
    x = rng.uniform(1.0, 2.0, 3) * rng.choice([-1, 1], 3)
    a = orc.taylor_coeffs(x, p)
    D = {n: (-1) ** sum(n) * fact(n) * a[idx[n]] for n in mi}
    for n in mi:
        if sum(n) + 2 <= p:
            s = sum(D[(n[0] + 2 * (k == 0), n[1] + 2 * (k == 1), n[2] + 2 * (k == 2))] for k in range(3))
            assert abs(s) <= 1e-13 * max(abs(D[(n[0] + 2, n[1], n[2])]), 1.0)
    q = {n: (rng.standard_normal() if sum(n) >= 1 else 0.0) for n in mi}
    full = {m: sum(D[tuple(a_ + b_ for a_, b_ in zip(n, m))] * q[n] for n in mi if sum(n) + sum(m) <= p) for m in mi}
    qr = {}
    for (nx, ny, nz) in mi:
        if nz > 1:
            continue
        v = 0.0
        for j in range((sum((nx, ny, nz)) - nz) // 2 + 1):
            for i in range(j + 1):
                src = (nx - 2 * i, ny - 2 * (j - i), nz + 2 * j)
                if min(src) >= 0:
                    v += (-1) ** j * math.comb(j, i) * q[src]
        qr[(nx, ny, nz)] = v
    red = {m: sum(D[tuple(a_ + b_ for a_, b_ in zip(n, m))] * qr[n] for n in qr if sum(n) + sum(m) <= p)
           for m in mi if m[2] <= 1}
    scale = max(abs(v) for v in full.values())
    for m in mi:
        j, c = m[2] // 2, m[2] % 2
        v = (-1) ** j * sum(math.comb(j, i) * red[(m[0] + 2 * i, m[1] + 2 * (j - i), c)] for i in range(j + 1))
        assert abs(v - full[m]) <= 1e-12 * scale, m


def test_reference_perceptron_gradient_by_finite_differences():
    """The oracle's surrogate network: its chain-rule gradient equals central
    finite differences of its loss (FP64), and the packing covers every
    parameter once."""
    from oracle import mlp
    H = 8
    _, n = mlp.layout(H)
    assert n == 16 * H + H + 2 * (H * H + H) + H * 12 + 12
    rng = np.random.default_rng(3)
    p = rng.standard_normal(n) * 0.5
    X = rng.standard_normal((7, 16))
    Tg = rng.standard_normal((7, 12))
    loss, g = mlp.loss_and_grad(p, H, X, Tg)
    eps = 1e-6
    for i in rng.choice(n, 40, replace=False):
        q = p.copy()
        q[i] += eps
        lp = mlp.loss_and_grad(q, H, X, Tg)[0]
        q[i] -= 2 * eps
        lm = mlp.loss_and_grad(q, H, X, Tg)[0]
        assert abs((lp - lm) / (2 * eps) - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i
