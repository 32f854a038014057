"""Pins of the oracle FMM (Secs. 3.1-3.3) against its definition.

 - theta -> 0: the MAC never accepts, every leaf pair is direct: FMM == direct.
 - The error against the direct sum falls with the order p and with theta
   (truncation law of Sec. 2.2).
 - Tree: every tet (by centroid) and every target in exactly one leaf; radii
   are the farthest tet corner / target from the cube centre (Sec. 3.2).
 - Lists: M2L pairs satisfy the MAC, P2P pairs are leaf pairs that fail it,
   and every (target, tet) pair is covered exactly once by P2P or by an M2L
   between an ancestor-or-self of each side (Listings 1-2).
"""
import numpy as np
import pytest

import meshgen


def _mesh(n=4, seed=0):
    nodes, tets = meshgen.box_mesh(n, jitter=0.15, seed=seed)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=1)[0]
    return nodes, tets, M


def test_theta_to_zero_equals_direct(orc):
    nodes, tets, M = _mesh(5)
    ud = orc.direct(nodes, tets, M)
    F = orc.FMM(nodes, tets, p=4, leaf=8, theta=1e-9)
    st = F.stats()
    assert st["n_m2l"] == 0
    assert st["n_p2p_pairs"] == nodes.shape[0] * tets.shape[0]
    u = F.evaluate(M)
    # every pair integrated directly; the direct sum takes far pairs (from 3
    # tet diameters) by its Gauss rule, the FMM's near field by the closed
    # form, which keeps ~1e-12 of a pair there: equal to that rounding
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-13


def test_error_falls_with_order_and_theta(orc):
    nodes, tets, M = _mesh(6)
    ud = orc.direct(nodes, tets, M)
    errs = []
    for p in (2, 4, 6, 8, 10):
        F = orc.FMM(nodes, tets, p=p, leaf=8, theta=0.5)
        u = F.evaluate(M)
        errs.append(np.linalg.norm(u - ud) / np.linalg.norm(ud))
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 < 0.5 * e0
    assert errs[-1] < 1e-5
    et = []
    for theta in (0.7, 0.5, 0.3):
        F = orc.FMM(nodes, tets, p=6, leaf=8, theta=theta)
        et.append(np.linalg.norm(F.evaluate(M) - ud) / np.linalg.norm(ud))
    assert et[0] > et[1] > et[2]


def _cell_maps(F):
    cells, rad = F.cells()
    key = {tuple(c[:4]): i for i, c in enumerate(cells)}
    parent = {}
    for i, c in enumerate(cells):
        lv, ix, iy, iz = c[:4]
        if lv > 0:
            parent[i] = key[(lv - 1, ix >> 1, iy >> 1, iz >> 1)]
    has_child = set(parent.values())
    return cells, rad, key, parent, has_child


def test_tree_and_radii(orc):
    nodes, tets, M = _mesh(5, seed=3)
    leaf = 10
    F = orc.FMM(nodes, tets, p=3, leaf=leaf, theta=0.5)
    cells, rad, key, parent, has_child = _cell_maps(F)
    # bounding cube as specified: box centre, side = extent * (1 + 2^-20)
    lo, hi = nodes.min(0), nodes.max(0)
    side = (hi - lo).max() * (1.0 + 2.0 ** -20)
    origin = 0.5 * (lo + hi) - 0.5 * side
    cen = ((nodes[tets[:, 0]] + nodes[tets[:, 1]]) + (nodes[tets[:, 2]] + nodes[tets[:, 3]])) * 0.25
    leaves = [i for i in range(len(cells)) if i not in has_child]
    assert sum(cells[i][4] for i in leaves) == tets.shape[0]
    assert sum(cells[i][5] for i in leaves) == nodes.shape[0]
    for i in leaves:
        assert cells[i][4] <= leaf and cells[i][5] <= leaf
    for i, c in enumerate(cells):
        lv, ix, iy, iz, nt, nx = c
        s = side / 2.0 ** lv
        cc = origin + (np.array([ix, iy, iz]) + 0.5) * s
        lo_c = origin + np.array([ix, iy, iz]) * s
        tin = np.all((np.floor((cen - origin) / side * 2.0 ** 21).astype(np.int64) >> (21 - lv)) == [ix, iy, iz], axis=1)
        xin = np.all((np.floor((nodes - origin) / side * 2.0 ** 21).astype(np.int64) >> (21 - lv)) == [ix, iy, iz], axis=1)
        assert tin.sum() == nt and xin.sum() == nx
        if nt:
            rs = np.linalg.norm(nodes[tets[tin]].reshape(-1, 3) - cc, axis=1).max()
            assert abs(rs - rad[i, 0]) <= 1e-15 * max(rs, 1.0)
        if nx:
            rt = np.linalg.norm(nodes[xin] - cc, axis=1).max()
            assert abs(rt - rad[i, 1]) <= 1e-15 * max(rt, 1.0)
        assert np.all(lo_c <= cen[tin] + 1e-12 * side)


@pytest.mark.parametrize("n,leaf,theta", [(4, 8, 0.5), (6, 16, 0.4), (5, 4, 0.7)])
def test_lists_cover_every_pair_once(orc, n, leaf, theta):
    nodes, tets, M = _mesh(n, seed=n)
    F = orc.FMM(nodes, tets, p=2, leaf=leaf, theta=theta)
    cells, rad, key, parent, has_child = _cell_maps(F)
    nc = len(cells)
    lists = {k: F.lists(k) for k in ("m2l", "p2p")}
    side = (nodes.max(0) - nodes.min(0)).max() * (1.0 + 2.0 ** -20)
    origin = 0.5 * (nodes.min(0) + nodes.max(0)) - 0.5 * side

    def centre(lv, ix, iy, iz):
        return origin + (np.array([ix, iy, iz]) + 0.5) * (side / 2.0 ** lv)

    cover = np.zeros((nc, nc), dtype=np.int64)
    for kind, L in lists.items():
        for row in L:
            a, b = key[tuple(row[:4])], key[tuple(row[4:])]
            ca, cb = centre(*row[:4]), centre(*row[4:])
            d2 = np.sum((ca - cb) ** 2)
            mac = (rad[a, 1] + rad[b, 0]) ** 2 < theta * theta * d2
            if kind == "m2l":
                assert mac
            else:
                assert not mac and a not in has_child and b not in has_child
            cover[a, b] += 1
    # every leaf pair with targets x tets covered exactly once along the ancestor chains
    leaves = [i for i in range(nc) if i not in has_child]

    def chain(i):
        out = [i]
        while out[-1] in parent:
            out.append(parent[out[-1]])
        return out

    chains = {i: chain(i) for i in leaves}
    for a in leaves:
        if cells[a][5] == 0:
            continue
        for b in leaves:
            if cells[b][4] == 0:
                continue
            tot = sum(cover[x, y] for x in chains[a] for y in chains[b])
            assert tot == 1, (a, b, tot)
    st = F.stats()
    assert st["n_m2l"] == lists["m2l"].shape[0] and st["n_p2p"] == lists["p2p"].shape[0]
    assert st["n_p2p_pairs"] == sum(cells[key[tuple(r[:4])]][5] * cells[key[tuple(r[4:])]][4] for r in lists["p2p"])


def test_sample_matches_full_and_fields(orc):
    nodes, tets, _ = _mesh(5, seed=2)
    M = meshgen.random_fields(nodes.shape[0], F=2, seed=4)
    F = orc.FMM(nodes, tets, p=5, leaf=8, theta=0.5)
    u = F.evaluate(M)
    rng = np.random.default_rng(0)
    sample = rng.choice(nodes.shape[0], 37, replace=False)
    us = F.evaluate_sample(M, sample)
    assert np.abs(us - u[:, sample]).max() <= 1e-15 * np.abs(u).max()
    u0 = F.evaluate(M[0])
    assert np.array_equal(u0, u[0])


def test_explicit_targets(orc):
    nodes, tets, M = _mesh(4, seed=5)
    rng = np.random.default_rng(1)
    tg = rng.uniform(-0.2, 1.2, (50, 3))
    F = orc.FMM(nodes, tets, p=8, leaf=8, theta=0.4, targets=tg)
    u = F.evaluate(M)
    ud = orc.direct(nodes, tets, M, targets=tg)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-4


def test_build_rejects_bad_input(orc):
    nodes, tets, M = _mesh(2)
    for kw in (dict(p=0, leaf=8, theta=0.5), dict(p=4, leaf=0, theta=0.5), dict(p=4, leaf=8, theta=1.0),
               dict(p=99, leaf=8, theta=0.5)):
        with pytest.raises(ValueError):
            orc.FMM(nodes, tets, **kw)
    bad = tets.copy()
    bad[3, 2] = -1
    with pytest.raises(ValueError):
        orc.FMM(nodes, bad, p=4, leaf=8, theta=0.5)
