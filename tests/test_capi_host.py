"""CPU tests of the product library: it loads, exports every function the
header declares, and its host-side plan (tree, radii, lists) equals the
oracle's exactly.  No compute call needs a GPU here."""
import os
import re

import numpy as np
import pytest

import meshgen
import paper_1606_00247_amd as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "tetfmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tfmm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_header_symbols():
    lib = T._load()
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n


def test_library_is_the_in_tree_build():
    assert os.path.dirname(T.library_path()) == os.path.join(ROOT, "paper_1606_00247_amd")


@pytest.mark.parametrize("n,p,leaf,theta", [(8, 6, 32, 0.5), (6, 4, 8, 0.4), (5, 3, 4, 0.7), ((7, 3, 5), 8, 16, 0.45)])
def test_plan_matches_oracle_exactly(orc, n, p, leaf, theta):
    nodes, tets = meshgen.box_mesh(n, jitter=0.15, seed=7)
    P = T.tfmm_plan_create(nodes, tets, p=p, leaf_size=leaf, theta=theta, device=-1)
    F = orc.FMM(nodes, tets, p, leaf, theta)
    st, so = T.tfmm_plan_stats(P), F.stats()
    for a, b in (("n_cells", "ncells"), ("n_leaves", "nleaves"), ("depth", "depth"), ("n_m2l", "n_m2l"),
                 ("n_p2p", "n_p2p"), ("n_p2p_pairs", "n_p2p_pairs"), ("ncoef", "ncoef")):
        assert st[a] == so[b], a
    assert st["m2l_keys_per_item"] == 256 and st["p2p_wide"] == 0  # default schedule, untuned
    for kind in ("m2l", "p2p"):
        a = T.tfmm_plan_lists(P, kind)
        b = F.lists(kind)
        assert a.shape == b.shape
        assert {tuple(r) for r in a} == {tuple(r) for r in b}
    cg, rg = T.tfmm_plan_cells(P)
    co, ro = F.cells()
    dg = {tuple(c[:4]): (tuple(c[4:]), tuple(r)) for c, r in zip(cg, rg)}
    do = {tuple(c[:4]): (tuple(c[4:]), tuple(r)) for c, r in zip(co, ro)}
    assert dg == do  # radii bit for bit


@pytest.mark.parametrize("n,leaf,theta", [(10, 8, 0.5), ((14, 6, 9), 16, 0.4), (6, 2, 0.6)])
def test_m2l_schedules_cover_every_pair_once(orc, n, leaf, theta):
    """Both matrix-core schedules translate every M2L pair of the oracle's
    list exactly once: the tiles (16 target cells, entries per key, work
    items spread over the XCDs) and the key-packed groups (blocks of target
    cells, the pairs of each key in groups of 16).  In the packed order a
    block's pairs come key by key: the translation vector (level difference,
    centre offset) changes only between keys."""
    nodes, tets = meshgen.box_mesh(n, jitter=0.15, seed=3)
    P = T.tfmm_plan_create(nodes, tets, p=4, leaf_size=leaf, theta=theta, device=-1)
    ref = orc.FMM(nodes, tets, 4, leaf, theta).lists("m2l")
    for kind in ("m2l_tiles", "m2l_packs"):
        sched = T.tfmm_plan_lists(P, kind)
        assert sched.shape == ref.shape, kind
        a = np.unique(sched, axis=0, return_counts=True)
        assert a[1].max() == 1 and a[0].shape[0] == ref.shape[0], kind
        assert {tuple(r) for r in a[0]} == {tuple(r) for r in ref}, kind
    # translation vector of each pair in units of the finer cell's half side
    sched = T.tfmm_plan_lists(P, "m2l_packs").astype(np.int64)
    la, lb = sched[:, 0], sched[:, 4]
    fine = np.maximum(la, lb)
    ca = (2 * sched[:, 1:4] + 1) << (fine - la)[:, None]
    cb = (2 * sched[:, 5:8] + 1) << (fine - lb)[:, None]
    key = np.concatenate([(lb - la)[:, None], ca - cb], axis=1)
    runs = 1 + int(np.any(key[1:] != key[:-1], axis=1).sum())
    assert runs <= sched.shape[0] and runs >= np.unique(key, axis=0).shape[0]
    # each (block, key) is one run: far fewer runs than pairs in a dense tree
    if sched.shape[0] > 2000:
        assert runs < sched.shape[0] / 2


def test_plan_explicit_targets_and_unjittered(orc):
    nodes, tets = meshgen.box_mesh((6, 6, 2), lo=(-3, -3, 0), hi=(3, 3, 1), jitter=0.0)
    rng = np.random.default_rng(3)
    tg = rng.uniform(-3.5, 3.5, (300, 3))
    P = T.tfmm_plan_create(nodes, tets, targets=tg, p=5, leaf_size=12, theta=0.5, device=-1)
    F = orc.FMM(nodes, tets, 5, 12, 0.5, targets=tg)
    for kind in ("m2l", "p2p"):
        assert {tuple(r) for r in T.tfmm_plan_lists(P, kind)} == {tuple(r) for r in F.lists(kind)}


@pytest.mark.parametrize("deg", [0, 1, 2, 5, 6, 8, 10, 13])
def test_simplex_rule_exact(deg):
    """Exact for every monomial of total degree <= deg: int over the unit simplex
    of l1^a l2^b l3^c = a! b! c! / (a+b+c+3)!."""
    from math import factorial
    r = T.tfmm_simplex_rule(deg)
    l1, l2, l3, w = r.T
    assert np.all(w > 0) and np.all(l1 >= 0) and np.all(l2 >= 0) and np.all(l3 >= 0)
    assert np.all(l1 + l2 + l3 <= 1.0 + 1e-15)
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            for c in range(deg + 1 - a - b):
                ex = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
                q = np.sum(w * l1 ** a * l2 ** b * l3 ** c)
                assert abs(q - ex) <= 1e-14 * ex * 10, (a, b, c)


def test_errors():
    nodes, tets = meshgen.box_mesh(2)
    cases = [
        (dict(p=0), -1), (dict(p=T.TFMM_PMAX + 1), -1), (dict(leaf_size=0), -1), (dict(theta=1.0), -1),
        (dict(theta=0.0), -1), (dict(m2l_precision=9), -7),
    ]
    for kw, code in cases:
        args = dict(p=4, leaf_size=8, theta=0.5, device=-1)
        args.update(kw)
        with pytest.raises(T.TetFMMError) as e:
            T.tfmm_plan_create(nodes, tets, **args)
        assert e.value.code == code, kw
    bad = tets.copy()
    bad[1, 2] = nodes.shape[0]
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_plan_create(nodes, bad, device=-1)
    assert e.value.code == -2
    flat = nodes.copy()
    deg = tets.copy()
    deg[0] = [0, 1, 2, 3]  # collinear corners 0,1,2 of the grid
    flat_nodes = flat.copy()
    flat_nodes[3] = flat_nodes[0] + 0.5 * (flat_nodes[1] - flat_nodes[0])
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_plan_create(flat_nodes, deg, device=-1)
    assert e.value.code == -3
    nan_nodes = nodes.copy()
    nan_nodes[5, 1] = np.nan
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_plan_create(nan_nodes, tets, device=-1)
    assert e.value.code == -4
    # empty inputs: no tet, fewer than 4 nodes, an empty explicit target list
    for nd, tt, tg in ((nodes, tets[:0], None), (nodes[:3], np.zeros((0, 4), np.int32), None),
                       (nodes, tets, np.zeros((0, 3)))):
        with pytest.raises(T.TetFMMError) as e:
            T.tfmm_plan_create(nd, tt, targets=tg, device=-1)
        assert e.value.code == -1
    P = T.tfmm_plan_create(nodes, tets, p=4, leaf_size=8, theta=0.5, device=-1)
    M = np.zeros((nodes.shape[0], 3))
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_evaluate_host(P, M)
    assert e.value.code == -1  # host-only plan cannot evaluate
    T.tfmm_plan_destroy(P)
    T.tfmm_plan_destroy(P)  # idempotent


def test_no_device_is_reported():
    """Without a visible GPU a device plan fails with EDEVICE (never a CPU fallback)."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible")
    nodes, tets = meshgen.box_mesh(2)
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_plan_create(nodes, tets, device=0)
    assert e.value.code == -6


def test_batch_errors_without_device():
    """Batch creation checks its arguments and needs a device; a bad mesh is
    reported with its index; never a CPU fallback."""
    import ctypes as C
    import torch
    lib = T._load()
    out = C.c_void_p()
    prm = T._Params(4, 8, 0.5, 0, 0)
    assert lib.tfmm_batch_create(0, None, None, None, None, C.byref(prm), C.byref(out)) == -1
    assert not out.value
    meshes = [meshgen.box_mesh(2), meshgen.box_mesh(3)]
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_batch_create(meshes, p=4, leaf_size=8, device=-1)
    assert e.value.code == -1
    bad = meshes[1][1].copy()
    bad[0, 0] = -5
    if torch.cuda.device_count() == 0:
        with pytest.raises(T.TetFMMError) as e:
            T.tfmm_batch_create(meshes, p=4, leaf_size=8, device=0)
        assert e.value.code == -6 and "mesh 0" in e.value.args[-1]
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_batch_create([meshes[0], (meshes[1][0], bad)], p=4, leaf_size=8, device=0)
    assert e.value.code in (-2, -6)
    assert lib.tfmm_batch_destroy(None) == 0


@pytest.mark.parametrize("n,p,leaf,theta", [(1500, 6, 16, 0.5), (400, 4, 4, 0.6), (60, 3, 1, 0.45)])
def test_point_plan_matches_oracle_exactly(orc, n, p, leaf, theta):
    """Point-dipole plans: the same tree, radii and lists as the oracle's
    dipole FMM, bit for bit (host-only plan, no device)."""
    rng = np.random.default_rng(n)
    pts = rng.uniform(-1, 1, (n, 3)) * [1.0, 0.6, 0.3]
    P = T.tfmm_plan_create_points(pts, p=p, leaf_size=leaf, theta=theta, device=-1)
    F = orc.DipoleFMM(pts, p, leaf, theta)
    st, so = T.tfmm_plan_stats(P), F.stats()
    for a, b in (("n_cells", "ncells"), ("depth", "depth"), ("n_m2l", "n_m2l"), ("n_p2p", "n_p2p"),
                 ("n_p2p_pairs", "n_p2p_pairs")):
        assert st[a] == so[b], a
    for kind in ("m2l", "p2p"):
        assert {tuple(r) for r in T.tfmm_plan_lists(P, kind)} == {tuple(r) for r in F.lists(kind)}
    # the matrix-core schedule translates every M2L pair once
    sched = T.tfmm_plan_lists(P, "m2l_tiles")
    assert sched.shape[0] == so["n_m2l"] and np.unique(sched, axis=0).shape[0] == so["n_m2l"]
    assert {tuple(r) for r in sched} == {tuple(r) for r in F.lists("m2l")}
    cg, rg = T.tfmm_plan_cells(P)
    co, ro = F.cells()
    assert {tuple(c[:4]): (tuple(c[4:]), tuple(r)) for c, r in zip(cg, rg)} == \
        {tuple(c[:4]): (tuple(c[4:]), tuple(r)) for c, r in zip(co, ro)}


def test_point_plan_and_tuner_errors():
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_plan_create_points(np.ones((4, 3)), device=-1)  # all points coincide
    assert e.value.code == -1
    pts = np.random.default_rng(1).standard_normal((10, 3))
    pts[3, 0] = np.inf
    with pytest.raises(T.TetFMMError) as e:
        T.tfmm_plan_create_points(pts, device=-1)
    assert e.value.code == -4
    nodes, tets = meshgen.box_mesh(2)
    for kw in (dict(tol=0.0), dict(tol=1e-3, n_sample=0), dict(tol=1e-3, p_list=(0,)),
               dict(tol=1e-3, theta_list=(1.0,)), dict(tol=1e-3, device=-1)):
        args = dict(leaf_size=8)
        args.update(kw)
        tol = args.pop("tol")
        with pytest.raises(T.TetFMMError) as e:
            T.tfmm_tune_accuracy(nodes, tets, tol, **args)
        assert e.value.code == -1, kw
