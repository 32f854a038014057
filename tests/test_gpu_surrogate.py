"""GPU tests of the near-field surrogate: its training data against the exact
pair integral of the oracle, its training gradients against the oracle's
perceptron, and what a trained network gives on the band of near-field pairs
(2 <= |x - c|/d < 6) against the exact integral on the same pairs."""
import os
import sys
import time

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


def test_training_targets_match_oracle_pair_integral(torch_dev, orc):
    from oracle import mlp
    nodes, tets = meshgen.box_mesh(6, seed=2)
    P = T.tfmm_plan_create(nodes, tets, p=4, leaf_size=16, theta=0.5)
    _say("surrogate samples")
    X, Y = T.tfmm_surrogate_samples(P, 48, seed=11)
    for i in range(X.shape[0]):
        sv = X[i].astype(np.float64).reshape(4, 3)
        ref = mlp.surrogate_target(sv, orc.tet_potential)
        assert abs(np.linalg.norm(sv.mean(axis=0)) - 1.0) <= 1e-6  # unit distance to the centroid
        d = max(np.linalg.norm(sv[a] - sv[b]) for a in range(4) for b in range(a + 1, 4))
        assert 1.99 <= 1.0 / d < 6.01
        # inputs are rounded to FP32, targets computed from the unrounded pair
        assert np.abs(Y[i] - ref).max() <= 2e-5 * np.abs(ref).max(), i


def test_training_gradients_match_oracle(torch_dev):
    from oracle import mlp
    H = 32
    n = T.tfmm_surrogate_param_count(H)
    rng = np.random.default_rng(4)
    p = (rng.standard_normal(n) * 0.3).astype(np.float32)
    X = rng.standard_normal((200, 12)).astype(np.float32)
    Y = rng.standard_normal((200, 12)).astype(np.float32)
    _say("surrogate gradients")
    loss, g = T.tfmm_surrogate_grad(H, p, X, Y)
    lo, go = mlp.loss_and_grad(p.astype(np.float64), H, X.astype(np.float64), Y.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    assert np.linalg.norm(g - go) <= 1e-5 * np.linalg.norm(go)


def test_trained_surrogate_on_the_band(torch_dev, tmp_path):
    """Train a small network, write and reload it, and compare the band
    potential with the exact integral on the same pairs: the accuracy it
    reaches and the time each takes (the surrogate's gain, which may be a
    loss) are printed and bounded loosely."""
    torch = torch_dev
    nodes, tets = meshgen.box_mesh(16, seed=0)
    M = torch.from_numpy(meshgen.random_fields(nodes.shape[0], F=1, seed=1)[0]).to("cuda:0")
    P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=64, theta=0.5)
    path = os.path.join(tmp_path, "sur.bin")
    t0 = time.perf_counter()
    loss = T.tfmm_surrogate_train(P, hidden=32, steps=1500, batch=2048, lr=2e-3, seed=3, out_path=path)
    _say("trained", loss, time.perf_counter() - t0)
    Q = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=64, theta=0.5)
    T.tfmm_surrogate_load(Q, path)
    ue = T.tfmm_band_potential(Q, M, False)
    us = T.tfmm_band_potential(Q, M, True)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(us - ue) / torch.linalg.norm(ue))

    def timed(flag):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            T.tfmm_band_potential(Q, M, flag, ue if not flag else us)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / 3

    te, ts = timed(False), timed(True)
    _say(f"band rel-L2 {err:.3e}, exact {te * 1e3:.3f} ms, surrogate {ts * 1e3:.3f} ms, gain {te / ts:.2f}x")
    assert loss < 1e-2
    assert err < 0.2
