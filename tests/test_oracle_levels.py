"""Pins of the oracle's per-level expansion orders (orc_fmm_set_level_orders),
the accuracy knob beside the opening angle and the order (Secs. 2.2, 3.2).

 - the same order q on every level equals the uniform-order FMM of order q;
 - orders on levels that hold no translations and no shifts change nothing;
 - lowering the order on the finest levels gives an error between those of
   the two uniform orders, and each lowered level adds error.
"""
import numpy as np

import meshgen


def _mesh(n, seed=3):
    nodes, tets = meshgen.box_mesh(n, seed=seed)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=5)[0]
    return nodes, tets, M


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_uniform_level_orders_equal_the_uniform_fmm(orc):
    nodes, tets, M = _mesh(8)
    for q in (4, 6):
        A = orc.FMM(nodes, tets, 8, 16, 0.5)
        A.set_level_orders([q])
        B = orc.FMM(nodes, tets, q, 16, 0.5)
        ua, ub = A.evaluate(M), B.evaluate(M)
        assert _rel(ua, ub) <= 1e-13, q
    # and all levels at p is the default
    A = orc.FMM(nodes, tets, 6, 16, 0.5)
    u0 = A.evaluate(M)
    A.set_level_orders([6] * 5)
    assert np.array_equal(A.evaluate(M), u0)


def test_orders_of_unused_levels_change_nothing(orc):
    """Levels without translations (here 0 and 1: all their cells are
    adjacent) pass only zero local expansions down and their multipoles feed
    no M2L: their order has no effect."""
    nodes, tets, M = _mesh(8)
    A = orc.FMM(nodes, tets, 6, 16, 0.5)
    m2l = A.lists("m2l")
    assert m2l[:, 0].min() >= 2 and m2l[:, 4].min() >= 2
    u0 = A.evaluate(M)
    A.set_level_orders([1, 2, 6])
    assert np.array_equal(A.evaluate(M), u0)
    A.set_level_orders([6, 6, 3])  # level 2 holds translations: now it matters
    assert _rel(A.evaluate(M), u0) > 1e-8


def test_lowering_fine_levels_adds_error(orc):
    nodes, tets, M = _mesh(10)
    ud = orc.direct(nodes, tets, M)
    A = orc.FMM(nodes, tets, 8, 16, 0.5)
    depth = A.stats()["depth"]
    e8 = _rel(A.evaluate(M), ud)
    A.set_level_orders([8] * depth + [6])  # the finest level at 6
    e_fine = _rel(A.evaluate(M), ud)
    A.set_level_orders([8] * (depth - 1) + [6])  # the two finest at 6
    e_two = _rel(A.evaluate(M), ud)
    A.set_level_orders([6])
    e6 = _rel(A.evaluate(M), ud)
    assert e8 < e_fine <= e_two <= e6 * 1.0001, (e8, e_fine, e_two, e6)
