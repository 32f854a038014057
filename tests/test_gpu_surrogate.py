"""GPU tests of the near-field surrogate: its training data against the
oracle (the exact pair integral of Sec. 2.1 minus the tet's quadrupole
expansion of Sec. 2.2), its training gradients against the oracle's
perceptron, and the trained network on the evaluation path: the near-field
pairs 2-6 tet diameters apart taken by the network (the exact integral for
the rest), against the exact path, the quadrupole expansion alone (the
network's base: what the network adds) and a 27-point Gauss rule (a cheap
control), on the sphere of radius 1 (96^3 grid, ~2.78M tets)."""
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


def test_training_targets_match_oracle(torch_dev, orc):
    from oracle import mlp
    nodes, tets = meshgen.box_mesh(6, seed=2)
    P = T.tfmm_plan_create(nodes, tets, p=4, leaf_size=16, theta=0.5)
    _say("surrogate samples")
    X, Y = T.tfmm_surrogate_samples(P, 48, seed=11)
    assert X.shape == (48, 16) and Y.shape == (48, 12)
    for i in range(X.shape[0]):
        sv = mlp.corners_from_features(X[i])
        ref = mlp.surrogate_target(sv, orc.tet_potential, orc.p2m_tet, orc.taylor_coeffs)
        assert abs(np.linalg.norm(X[i, :3]) - 1.0) <= 1e-6  # unit direction
        assert 1.99 <= 1.0 / X[i, 15] < 6.01  # a band pair
        # inputs are rounded to FP32, targets computed from the unrounded pair
        assert np.abs(Y[i] - ref).max() <= 1e-3 * np.abs(ref).max(), i


def test_training_gradients_match_oracle(torch_dev):
    from oracle import mlp
    H = 32
    n = T.tfmm_surrogate_param_count(H)
    rng = np.random.default_rng(4)
    p = (rng.standard_normal(n) * 0.3).astype(np.float32)
    X = rng.standard_normal((200, 16)).astype(np.float32)
    Y = rng.standard_normal((200, 12)).astype(np.float32)
    _say("surrogate gradients")
    loss, g = T.tfmm_surrogate_grad(H, p, X, Y)
    lo, go = mlp.loss_and_grad(p.astype(np.float64), H, X.astype(np.float64), Y.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    assert np.linalg.norm(g - go) <= 1e-5 * np.linalg.norm(go)


def test_band_controls_against_exact(torch_dev):
    """The band potential by the quadrupole expansion and by the Gauss rule
    against the exact integral on the same pairs (no network needed)."""
    torch = torch_dev
    nodes, tets = meshgen.box_mesh(12, seed=0)
    M = torch.from_numpy(meshgen.random_fields(nodes.shape[0], F=1, seed=1)[0]).to("cuda:0")
    P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=64, theta=0.5)
    _say("band controls cube12")
    ue = T.tfmm_band_potential(P, M, False)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(ue)) > 0.0
    u0 = T.tfmm_evaluate(P, M)
    for mode, tol in ((T.SUR_QUAD, 3e-2), (T.SUR_GAUSS, 3e-5)):
        T.tfmm_plan_set_surrogate(P, mode)
        u = T.tfmm_evaluate(P, M)
        torch.cuda.synchronize()
        # the whole evaluation differs from the exact one by the band error only
        err = float(torch.linalg.norm(u - u0) / torch.linalg.norm(ue))
        _say(f"mode {mode}: band error relative to the band potential {err:.2e}")
        assert err <= tol, (mode, err)
    T.tfmm_plan_set_surrogate(P, T.SUR_OFF)
    u1 = T.tfmm_evaluate(P, M)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(u1 - u0) / torch.linalg.norm(u0)) <= 1e-13


def test_surrogate_on_the_sphere(torch_dev, tmp_path):
    """Sphere r=1 (96^3 grid, ~2.78M tets), uniform M=(0,0,1) and one random
    unit field: the FMM with the network on the band (3 x 128 hidden, BF16
    weights, FP32 accumulation) against the FP64 direct sum on 512 sampled
    inner nodes, next to the exact path and both controls.  Asserts the
    measured accuracy bound, that the network beats its own base (the
    quadrupole expansion alone), and prints every time."""
    torch = torch_dev
    nodes, tets = meshgen.sphere_mesh(96)
    F = 2
    M = np.stack([meshgen.uniform_field(nodes.shape[0], (0.0, 0.0, 1.0)),
                  meshgen.random_fields(nodes.shape[0], F=1, seed=1)[0]])
    Md = torch.from_numpy(M).to("cuda:0")
    _say("sphere96 surrogate", tets.shape)
    P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=64, theta=0.5)
    path = os.path.join(tmp_path, "sur.bin")
    t0 = time.perf_counter()
    loss = T.tfmm_surrogate_train(P, hidden=128, steps=6000, batch=8192, lr=2e-3, seed=3, out_path=path)
    t_train = time.perf_counter() - t0
    _say(f"trained: loss {loss:.3e} in {t_train:.1f}s")
    assert loss < 2e-2  # measured 1.3e-2 (targets O(1))
    # a reloaded copy gives the same evaluation
    Q = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=64, theta=0.5, surrogate=T.SUR_MLP)
    T.tfmm_surrogate_load(Q, path)
    inner = np.flatnonzero(np.linalg.norm(nodes, axis=1) < 0.8)
    idx = inner[np.sort(np.random.default_rng(6).choice(inner.size, 512, replace=False))]
    Pd = T.tfmm_plan_create(nodes, tets, targets=nodes[idx], p=2, leaf_size=64, theta=0.5)
    ud = T.tfmm_direct(Pd, Md).cpu().numpy()
    del Pd
    res = {}
    for name, mode in (("exact", T.SUR_OFF), ("network", T.SUR_MLP), ("quadrupole", T.SUR_QUAD),
                       ("gauss27", T.SUR_GAUSS)):
        T.tfmm_plan_set_surrogate(P, mode)
        u = T.tfmm_evaluate(P, Md)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            T.tfmm_evaluate(P, Md, u)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / 3 * 1e3
        un = u.cpu().numpy()[:, idx]
        errs = [float(np.linalg.norm(un[f] - ud[f]) / np.linalg.norm(ud[f])) for f in range(F)]
        res[name] = (max(errs), ms, errs)
        _say(f"{name}: rel-L2 vs direct {errs[0]:.3e} (uniform) {errs[1]:.3e} (random), {ms:.2f} ms for 2 fields")
    T.tfmm_plan_set_surrogate(P, T.SUR_MLP)
    u1 = T.tfmm_evaluate(P, Md)
    u2 = T.tfmm_evaluate(Q, Md)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(u1 - u2) / torch.linalg.norm(u1)) <= 1e-11  # atomics order only
    st = T.tfmm_plan_stats(P)
    _say("band pairs", st["n_band_pairs"], "of", st["n_p2p_pairs"], "near pairs")
    # measured (MI355X): exact 9.3e-7 (uniform M) / 1.3e-5 (random M) in 98 ms;
    # network 3.0e-6 / 6.5e-5 in 1142 ms; quadrupole alone 2.6e-5 / 1.2e-3;
    # 27-point Gauss 9.3e-7 / 1.3e-5 in 171 ms
    assert res["exact"][2][0] <= 1e-5 and res["exact"][0] <= 2e-5
    for f in range(F):  # the network takes the quadrupole base's error down at least 5x
        assert res["network"][2][f] <= 0.2 * res["quadrupole"][2][f], f
    assert res["network"][2][0] <= 1e-5  # uniform M: within the bar
    assert res["network"][0] <= 1e-4
    for f in range(F):  # the control is as accurate as the exact band
        assert res["gauss27"][2][f] <= res["exact"][2][f] + 1e-6, f
