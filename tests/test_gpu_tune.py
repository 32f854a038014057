"""GPU tests of the (p, theta) choice for an accuracy target.

The configuration the tuner returns is checked independently: the oracle FMM
with that (p, theta) against the oracle's direct sum over every target must
be within the tolerance, and a tighter tolerance must not come back with a
cheaper pair of knobs.
"""
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


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_tuned_configuration_meets_the_tolerance(torch_dev, orc):
    nodes, tets = meshgen.box_mesh(9, seed=3)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=4)[0]
    ref = orc.direct(nodes, tets, M)
    picks = {}
    for tol in (1e-3, 1e-6):
        _say("tune box9 tol", tol)
        r = T.tfmm_tune_accuracy(nodes, tets, tol, M=M, leaf_size=16, n_sample=256, seed=7,
                                 p_list=(3, 4, 6, 8), theta_list=(0.35, 0.5, 0.65))
        assert r["met"] and r["ms"] > 0 and r["err"] <= tol / 2, r
        assert 1 <= r["n_tried"] <= 12
        tab = r["table"]
        row = tab[(tab[:, 0] == r["p"]) & np.isclose(tab[:, 1], r["theta"])][0]
        assert np.isclose(row[2], r["err"]) and np.isclose(row[3], r["ms"])
        # independent check: oracle FMM of the chosen knobs against the oracle direct sum
        u = orc.FMM(nodes, tets, r["p"], 16, r["theta"]).evaluate(M)
        assert _rel(u, ref) <= tol, (tol, r["p"], r["theta"])
        picks[tol] = r
    lo, hi = picks[1e-3], picks[1e-6]
    assert hi["p"] > lo["p"] or hi["theta"] < lo["theta"]


def test_unreachable_tolerance_reports_the_most_accurate(torch_dev):
    nodes, tets = meshgen.box_mesh(5, seed=1)
    _say("tune unreachable")
    r = T.tfmm_tune_accuracy(nodes, tets, 1e-15, leaf_size=8, n_sample=64, p_list=(2, 3), theta_list=(0.5, 0.6))
    assert not r["met"] and r["ms"] == -1.0
    assert r["n_tried"] == 4
    tried = r["table"][r["table"][:, 2] >= 0]
    assert r["err"] == pytest.approx(tried[:, 2].min())
    with pytest.raises(T.TetFMMError):
        T.tfmm_tune_accuracy(nodes, tets, -1.0, leaf_size=8)


def test_tuned_dipole_configuration(torch_dev, orc):
    """Point dipoles: the returned (p, theta) meets the tolerance in the
    oracle's dipole FMM against the oracle's dipole sum."""
    rng = np.random.default_rng(12)
    pts = rng.uniform(-1, 1, (1200, 3)) * [1.0, 0.8, 0.5]
    m = rng.standard_normal((pts.shape[0], 3))
    tol = 1e-4
    _say("tune dipoles tol", tol)
    r = T.tfmm_tune_accuracy(pts, None, tol, M=m, leaf_size=16, n_sample=256, seed=2,
                             p_list=(4, 6, 8), theta_list=(0.35, 0.5, 0.65))
    assert r["met"] and r["err"] <= tol / 2, r
    u = orc.DipoleFMM(pts, r["p"], 16, r["theta"]).evaluate(m)
    assert _rel(u, orc.dipole_direct(pts, m)) <= tol, (r["p"], r["theta"])
