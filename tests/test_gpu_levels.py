"""GPU tests of per-level expansion orders (tfmm_plan_set_level_orders) and
their tuner, against the oracle FMM with the same orders."""
import sys

import numpy as np
import pytest

import meshgen
import paper_1606_00247_amd as T

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _eval(torch, P, M):
    u = T.tfmm_evaluate(P, torch.from_numpy(np.ascontiguousarray(M)).to("cuda:0"))
    torch.cuda.synchronize()
    return u.cpu().numpy()


@pytest.mark.parametrize("orders", [[8, 8, 8, 6], [5, 5, 8], [6], [8, 7, 6, 5, 4], [3, 8]])
def test_level_orders_match_oracle(torch_dev, orc, orders):
    nodes, tets = meshgen.box_mesh(10, seed=2)
    M = meshgen.random_fields(nodes.shape[0], F=2, seed=3)
    _say("level orders", orders)
    P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=16, theta=0.5)
    T.tfmm_plan_set_level_orders(P, orders)
    st = T.tfmm_plan_stats(P)
    assert st["level_order"][:len(orders)] == orders and st["level_order"][-1] == orders[-1]
    u = _eval(torch_dev, P, M)
    O = orc.FMM(nodes, tets, 8, 16, 0.5)
    O.set_level_orders(orders)
    uo = O.evaluate(M)
    for f in range(2):
        assert _rel(u[f], uo[f]) <= TOL, f
    # one field takes the shared-entity near field and a separate M2L tile width
    u1 = _eval(torch_dev, P, M[0])
    assert _rel(u1, uo[0]) <= TOL


def test_uniform_level_order_equals_plan_of_that_order(torch_dev):
    nodes, tets = meshgen.box_mesh(9, seed=4)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=5)[0]
    _say("uniform level order")
    P8 = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=16, theta=0.5)
    T.tfmm_plan_set_level_orders(P8, [6])
    P6 = T.tfmm_plan_create(nodes, tets, p=6, leaf_size=16, theta=0.5)
    assert _rel(_eval(torch_dev, P8, M), _eval(torch_dev, P6, M)) <= TOL
    # back to the plan's own order
    u8 = _eval(torch_dev, P8, M)
    T.tfmm_plan_set_level_orders(P8, [8])
    assert T.tfmm_plan_stats(P8)["level_order"] == [8] * 22
    assert _rel(_eval(torch_dev, P8, M), u8) > 1e-9
    with pytest.raises(T.TetFMMError):
        T.tfmm_plan_set_level_orders(P8, [9])


def test_level_orders_mixed_precision(torch_dev):
    nodes, tets = meshgen.box_mesh(10, seed=6)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=7)[0]
    _say("level orders fp32 / bf16x3")
    P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=16, theta=0.5)
    T.tfmm_plan_set_level_orders(P, [8, 8, 8, 6])
    u64 = _eval(torch_dev, P, M)
    for prec, tol in ((T.M2L_FP32, 2e-6), (T.M2L_BF16X3, 5e-6)):
        T.tfmm_plan_set_m2l_precision(P, prec)
        assert _rel(_eval(torch_dev, P, M), u64) <= tol, prec


def test_tuned_level_orders_meet_the_tolerance(torch_dev, orc):
    nodes, tets = meshgen.box_mesh(14, seed=8)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=9)[0]
    _say("tune level orders")
    P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=32, theta=0.5)
    before = T.tfmm_plan_stats(P)["level_order"]
    r = T.tfmm_tune_level_orders(P, M, 1e-9, n_sample=256, seed=3)  # out of reach at p = 8, theta 0.5
    assert not r["met"] and r["orders"] == before and T.tfmm_plan_stats(P)["level_order"] == before
    for tol in (1e-4, 2e-5):
        r = T.tfmm_tune_level_orders(P, M, tol, n_sample=256, seed=3)
        _say("tol", tol, r)
        assert r["met"] and r["err"] <= tol / 2
        depth = T.tfmm_plan_stats(P)["depth"]
        O = orc.FMM(nodes, tets, 8, 32, 0.5)
        O.set_level_orders(r["orders"][:depth + 1])
        uo = O.evaluate(M)
        u = _eval(torch_dev, P, M)
        assert _rel(u, uo) <= TOL
        ud = T.tfmm_direct(P, torch_dev.from_numpy(M).to("cuda:0"))
        torch_dev.cuda.synchronize()
        assert _rel(uo, ud.cpu().numpy()) <= tol
