"""The operation count of the oracle's pair integral that prices the near
field per pair in the benchmark's roofline (Sec. 2.1: the exact potential of
one affinely magnetised tetrahedron)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import meshgen  # noqa: E402
from oracle import opcount  # noqa: E402


@pytest.fixture(scope="module")
def cube():
    nodes, tets = meshgen.box_mesh(4, seed=0)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=1)[0]
    return nodes, tets, M


def test_counted_build_computes_the_oracle_potential(cube, orc):
    """The counting build runs oracle.c unchanged: its potentials, summed over
    every pair of the 4^3 cube, equal the oracle library's bit for bit."""
    nodes, tets, M = cube
    pt = np.repeat(np.arange(nodes.shape[0]), tets.shape[0])
    pq = np.tile(np.arange(tets.shape[0]), nodes.shape[0])
    _, usum = opcount.count_pairs(nodes, tets, nodes, M, pt, pq)
    ref = 0.0
    for i, q in zip(pt, pq):
        ref += orc.tet_potential(nodes[i], nodes[tets[q]], M[tets[q]])
    assert usum == ref


def test_count_is_geometry_independent_off_the_singular_sets(cube):
    """Away from the face planes and edge lines every branch of the closed
    form is taken: two generic pairs cost the same; a target at a corner
    skips the singular logs and angles and costs less."""
    nodes, tets, M = cube
    x = np.array([[3.1, 2.7, 2.9], [-1.3, 0.4, 5.2]])
    c1, _ = opcount.count_pairs(nodes, tets, x, M, [0], [5])
    c2, _ = opcount.count_pairs(nodes, tets, x, M, [1], [17])
    assert c1 == c2
    assert c1["log"] == 12 and c1["atan"] == 24 and c1["sqrt"] == 40
    corner = int(tets[5][0])
    c3, _ = opcount.count_pairs(nodes, tets, nodes, M, [corner], [5])
    assert opcount.flops(c3) < opcount.flops(c1)


def test_benchmark_prices_pairs_at_the_counted_mean():
    """The per-pair price in the benchmark's roofline is the mean count over
    every pair of the jittered 8^3 cube."""
    import bench
    r = opcount.cube_pairs(8)
    assert round(r["flops_per_pair_mean"]) == bench.P2P_PAIR_FLOPS
