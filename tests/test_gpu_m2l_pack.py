"""M2L packed by key (Secs. 2.2-2.3: the local expansion at a target cell
sums the translated multipoles of its interaction list; Sec. 3.3: the
interaction list of the dual traversal).  The packed schedule groups the
FP64 translations of each key inside blocks of target cells; it must give
the oracle FMM's potentials, and the tiled schedule's up to summation
order, for every field width (below 16) and order it serves."""
import sys

import numpy as np
import pytest

import meshgen
import paper_1606_00247_amd as T

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _eval(torch, plan, M):
    Md = torch.from_numpy(np.ascontiguousarray(M)).to("cuda:0")
    u = T.tfmm_evaluate(plan, Md)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("F", [1, 3, 8])
def test_packed_matches_tiled_and_oracle_fp64(torch_dev, orc, F):
    """12^3 cube (10,368 tets), p = 8, leaf 16: the packed FP64 M2L against
    the oracle FMM (<= 1e-12 relative L2, element-wise <= 1e-11 of the
    largest |u|) and against the tiled schedule (same contraction, other
    summation order: <= 1e-13)."""
    nodes, tets = meshgen.box_mesh(12, seed=0)
    M = meshgen.random_fields(nodes.shape[0], F=F, seed=1)
    P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=16, theta=0.5)
    _say("packed fp64 F", F)
    T.tfmm_plan_set_schedule(P, 512, 0, 1, 256)
    up = _eval(torch_dev, P, M)
    st = T.tfmm_plan_stats(P)
    assert st["m2l_packed"] == 1
    T.tfmm_plan_set_schedule(P, 512, 0, 0, 256)
    ut = _eval(torch_dev, P, M)
    uo = orc.FMM(nodes, tets, 8, 16, 0.5).evaluate(M)
    for f in range(F):
        assert _rel(up[f], uo[f]) <= 1e-12, f
        assert np.abs(up[f] - uo[f]).max() <= 1e-11 * np.abs(uo[f]).max(), f
        assert _rel(up[f], ut[f]) <= 1e-13, f


def test_packed_group_fill(torch_dev):
    """On the 24^3 cube the packed groups carry one translation in at least
    80% of their matrix-core columns (the tiles of 16 target cells fill
    about half)."""
    nodes, tets = meshgen.box_mesh(24, seed=0)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=1)
    P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=64, theta=0.5)
    T.tfmm_plan_set_schedule(P, 512, 0, 1, 256)
    _eval(torch_dev, P, M)
    st = T.tfmm_plan_stats(P)
    fill = st["n_m2l"] / (16.0 * st["m2l_groups"])
    _say("packed fill", fill, st["m2l_groups"], st["n_m2l"])
    assert 0.8 <= fill <= 1.0


@pytest.mark.parametrize("p", [1, 2, 5, 9, 10])
def test_packed_orders_vs_oracle(torch_dev, orc, p):
    """Every order the packed kernels are built for (block size 128 slots up
    to p = 8, 64 above): 9^3 cube, two fields, against the oracle FMM."""
    nodes, tets = meshgen.box_mesh(9, seed=2)
    M = meshgen.random_fields(nodes.shape[0], F=2, seed=3)
    P = T.tfmm_plan_create(nodes, tets, p=p, leaf_size=16, theta=0.5)
    T.tfmm_plan_set_schedule(P, 512, 0, 1, 128)
    _say("packed order", p)
    u = _eval(torch_dev, P, M)
    uo = orc.FMM(nodes, tets, p, 16, 0.5).evaluate(M)
    for f in range(2):
        assert _rel(u[f], uo[f]) <= 1e-12, f


def test_packed_level_orders_vs_oracle(torch_dev, orc):
    """Per-level orders with the packed form: one packed launch per target
    level at that level's order (including one above 8, whose blocks are
    half as large), against the oracle's per-level FMM."""
    nodes, tets = meshgen.box_mesh(12, seed=0)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=1)
    orders = [10, 9, 8, 6, 5]
    P = T.tfmm_plan_create(nodes, tets, p=10, leaf_size=16, theta=0.5)
    T.tfmm_plan_set_level_orders(P, orders)
    T.tfmm_plan_set_schedule(P, 512, 0, 1, 256)
    _say("packed level orders", orders)
    u = _eval(torch_dev, P, M)
    O = orc.FMM(nodes, tets, 10, 16, 0.5)
    O.set_level_orders(orders)
    uo = O.evaluate(M)
    assert _rel(u[0], uo[0]) <= 1e-12


def test_packed_after_schedule_changes(torch_dev, orc):
    """Switching forms and item sizes back and forth on one plan (work
    lists rebuilt, old ones freed) keeps every evaluation equal to the
    oracle's."""
    nodes, tets = meshgen.box_mesh(8, seed=1)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=2)
    P = T.tfmm_plan_create(nodes, tets, p=6, leaf_size=8, theta=0.5)
    uo = orc.FMM(nodes, tets, 6, 8, 0.5).evaluate(M)
    for sch in ((256, 0, 1, 16), (256, 1, 0, 256), (128, 0, 1, 4096), (1024, 1, 1, 64)):
        _say("schedule", sch)
        T.tfmm_plan_set_schedule(P, *sch)
        u = _eval(torch_dev, P, M)
        assert _rel(u[0], uo[0]) <= 1e-12, sch

