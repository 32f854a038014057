"""GPU test of the near field's own elementary functions (the edge
logarithms and face solid angles of the exact pair integral, Sec. 2.1, and
the reciprocals and square roots of the direct sum's far rules), called one
element at a time through tfmm_elementary and compared with mpmath at 120
bits over their reduced ranges and edge cases.

Stated bounds (in units of the last place of the correctly rounded result):
 log_ratio 4 ulp (0 exactly for equal arguments), atan2 2 ulp (exact signs
 and quadrant values at the axes), division 1 ulp, reciprocal square root 1 ulp.
"""
import sys

import mpmath
import numpy as np
import pytest

import paper_1606_00247_amd as T

pytestmark = pytest.mark.gpu

mpmath.mp.prec = 120


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return 0


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _ulps(got, ref):
    ref = np.asarray(ref)
    return np.abs(got - ref) / np.spacing(np.abs(ref))


def _ref(fn, *args):
    return np.array([float(fn(*[mpmath.mpf(float(x)) for x in xs])) for xs in zip(*args)])


def test_log_ratio(gpu):
    rng = np.random.default_rng(1)
    n = 4000
    # ratios in the reduced range [1/sqrt2, sqrt2) and across many binades
    a = np.concatenate([rng.uniform(0.5, 1.0, n), 10.0 ** rng.uniform(-30, 30, n), 2.0 ** rng.integers(-60, 60, 200)])
    r = np.concatenate([rng.uniform(2 ** -0.5, 2 ** 0.5, n), 10.0 ** rng.uniform(-30, 30, n), 2.0 ** rng.integers(-9, 9, 200)])
    b = a * r
    near = a[:500] * (1.0 + rng.integers(-50, 50, 500) * 2.0 ** -52)  # ratios within a few ulp of 1
    a = np.concatenate([a, a[:500]])
    b = np.concatenate([b, near])
    _say("log_ratio", a.size)
    got = T.tfmm_elementary("log_ratio", a, b)
    ref = _ref(lambda x, y: mpmath.log(x / y), a, b)
    eq = a == b
    assert np.all(got[eq] == 0.0)
    u = _ulps(got[~eq], ref[~eq])
    print("log_ratio max ulp", u.max())
    assert u.max() <= 4.0


def test_log_ratio_is_odd(gpu):
    """ln(a/b) = -ln(b/a) bit for bit: the edge logarithm of the shared-entity
    near field takes ln((R_a - l_a)/(R_b - l_b)) as -ln((R_b - l_b)/(R_a - l_a)),
    which is the same value only if the reduction (the factor 2 on one
    argument, the exponent difference) and the odd series flip sign exactly.
    Random ratios across binades and ratios at the reduction thresholds
    sqrt2 and 1/sqrt2 (where the factor 2 moves from one argument to the
    other)."""
    rng = np.random.default_rng(5)
    n = 4000
    a = 10.0 ** rng.uniform(-30, 30, n)
    b = a * 10.0 ** rng.uniform(-8, 8, n)
    s2 = np.sqrt(2.0)
    m = rng.uniform(0.5, 1.0, 400)
    edge = np.concatenate([m * s2 * (1.0 + k * 2.0 ** -52) for k in range(-3, 4)])
    a = np.concatenate([a, np.tile(m, 7), edge])
    b = np.concatenate([b, edge, np.tile(m, 7)])
    _say("log_ratio oddness", a.size)
    f = T.tfmm_elementary("log_ratio", a, b)
    g = T.tfmm_elementary("log_ratio", b, a)
    assert np.array_equal(f, -g)


def test_atan2(gpu):
    rng = np.random.default_rng(2)
    n = 6000
    y = rng.standard_normal(n) * 10.0 ** rng.uniform(-20, 20, n)
    x = rng.standard_normal(n) * 10.0 ** rng.uniform(-20, 20, n)
    # near the reduction points tan(pi/8) and the diagonal
    t = np.tan(np.pi / 8) * (1.0 + rng.uniform(-1e-3, 1e-3, 500))
    y = np.concatenate([y, t, np.ones(500), [0.0, 0.0, 1.0, -1.0, 0.0, 2.0, -3.0]])
    x = np.concatenate([x, np.ones(500), 1.0 + rng.uniform(-1e-9, 1e-9, 500), [1.0, -1.0, 0.0, 0.0, 0.0, 2.0, -3.0]])
    _say("atan2", y.size)
    got = T.tfmm_elementary("atan2", y, x)
    ref = _ref(mpmath.atan2, y, x)
    # axes and the origin exactly: 0, pi, +-pi/2
    assert got[-7] == 0.0 and got[-6] == np.pi and got[-5] == np.pi / 2 and got[-4] == -np.pi / 2 and got[-3] == 0.0
    nz = ref != 0.0
    u = _ulps(got[nz], ref[nz])
    print("atan2 max ulp", u.max())
    assert u.max() <= 2.0
    assert np.all(np.sign(got[nz]) == np.sign(ref[nz]))


def test_div(gpu):
    rng = np.random.default_rng(3)
    n = 6000
    a = rng.standard_normal(n) * 10.0 ** rng.uniform(-100, 100, n)
    b = rng.standard_normal(n) * 10.0 ** rng.uniform(-100, 100, n)
    a = np.concatenate([a, [1.0, 3.0, -7.0, 0.0]])
    b = np.concatenate([b, [3.0, 3.0, 2.0, 5.0]])
    _say("div", a.size)
    got = T.tfmm_elementary("div", a, b)
    ref = a / b  # IEEE division is correctly rounded
    assert got[-3] == 1.0 and got[-1] == 0.0
    nz = ref != 0.0
    u = _ulps(got[nz], ref[nz])
    print("div max ulp", u.max())
    assert u.max() <= 1.0


def test_rsqrt(gpu):
    rng = np.random.default_rng(4)
    n = 6000
    a = np.concatenate([10.0 ** rng.uniform(-200, 200, n), rng.uniform(0.25, 4.0, n), 4.0 ** rng.integers(-100, 100, 100)])
    _say("rsqrt", a.size)
    got = T.tfmm_elementary("rsqrt", a)
    ref = _ref(lambda x: 1 / mpmath.sqrt(x), a)
    u = _ulps(got, ref)
    print("rsqrt max ulp", u.max())
    assert u.max() <= 1.0
    pw = a[-100:]
    assert np.all(got[-100:] == 1.0 / np.sqrt(pw))  # exact for powers of four
