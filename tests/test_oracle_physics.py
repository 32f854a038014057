"""Physical pins of the oracle's direct sum (Sec. 4 experiments and textbook facts).

 - Demagnetising factors of a uniformly magnetised cube are 1/3 each (the
   paper's E = mu0 Ms^2/6); with P1 nodal u on the boundary the estimate
   N_kk = (1/V) surface-int u n_k dS is biased by the discretisation and the
   bias must shrink under refinement.
 - Uniformly magnetised sphere: u = M.r/3 inside; the mesh is a staircase of
   tets, so the interior error must be small and shrink under refinement.
 - Reciprocity <m1, H(m2)> = <m2, H(m1)> with H = -grad(P1 u): exact for the
   continuous operator, here up to a discretisation error that shrinks with h.
"""
import json
import os

import numpy as np

import meshgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_constants.json")


def _boundary_faces(tets):
    faces = np.sort(np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]]),
                    axis=1)
    uf, cnt = np.unique(faces, axis=0, return_counts=True)
    return uf[cnt == 1]


def _demag_factors(orc, n):
    nodes, tets = meshgen.box_mesh(n, jitter=0.15, seed=0)
    bf = _boundary_faces(tets)
    bn = np.unique(bf)
    P = nodes[bf]
    a = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    area = 0.5 * np.linalg.norm(a, axis=1)
    nrm = a / np.linalg.norm(a, axis=1, keepdims=True)
    nrm *= np.sign(np.sum((P.mean(1) - 0.5) * nrm, axis=1))[:, None]
    N = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        M = meshgen.uniform_field(nodes.shape[0], e)
        u = np.zeros(nodes.shape[0])
        u[bn] = orc.direct(nodes, tets, M, targets=nodes[bn])
        N.append(np.sum(area * u[bf].mean(1) * nrm[:, k]))
    return np.array(N)


def test_cube_demag_factors(orc):
    with open(GOLDEN) as f:
        g = json.load(f)
    target = g["cube_demag_factor"]["value"]
    N4 = _demag_factors(orc, 4)
    N8 = _demag_factors(orc, 8)
    assert np.all(np.abs(N8 - target) <= 1e-2)
    assert np.all(np.abs(N8 - target) < 0.5 * np.abs(N4 - target))
    assert abs(N8.sum() - 1.0) <= 3e-2
    # energy E = mu0 Ms^2 N / 2 per unit volume: 1/6 for the cube
    assert abs(0.5 * N8[2] - g["cube_energy_over_mu0_ms2"]["value"]) <= 5e-3


def test_sphere_interior_potential(orc):
    errs = []
    for n in (8, 16):
        nodes, tets = meshgen.sphere_mesh(n, jitter=0.15, seed=0)
        M = meshgen.uniform_field(nodes.shape[0], (0.0, 0.0, 1.0))
        inner = np.linalg.norm(nodes, axis=1) < 0.8
        u = orc.direct(nodes, tets, M, targets=nodes[inner])
        ue = nodes[inner, 2] / 3.0
        errs.append(np.linalg.norm(u - ue) / np.linalg.norm(ue))
    assert errs[0] < 2e-2
    assert errs[1] < 0.5 * errs[0]


def _pair_energy(nodes, tets, Ma, ub):
    """<m_a, H(m_b)> = -sum_T int_T M_a . grad(P1 u_b)."""
    v = nodes[tets]
    J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)
    vol = np.abs(np.linalg.det(J)) / 6.0
    Ji = np.linalg.inv(J)
    g = np.concatenate([-Ji.sum(1, keepdims=True), Ji], axis=1)
    gradu = np.einsum("tij,ti->tj", g, ub[tets])
    return -np.sum(vol * np.einsum("tj,tj->t", Ma[tets].mean(1), gradu))


def test_reciprocity(orc):
    asym = []
    for n in (4, 8):
        nodes, tets = meshgen.box_mesh(n, jitter=0.15, seed=0)
        x, y, z = nodes.T
        S1 = np.stack([np.cos(2 * y), np.sin(3 * z), x ** 2], axis=1)
        S2 = np.stack([z, np.cos(2 * x), np.sin(y)], axis=1)
        w1 = orc.direct(nodes, tets, S1)
        w2 = orc.direct(nodes, tets, S2)
        e12 = _pair_energy(nodes, tets, S1, w2)
        e21 = _pair_energy(nodes, tets, S2, w1)
        e11 = _pair_energy(nodes, tets, S1, w1)
        e22 = _pair_energy(nodes, tets, S2, w2)
        assert e11 < 0 and e22 < 0  # <m, H(m)> = -2 E_stray / mu0 < 0
        asym.append(abs(e12 - e21) / np.sqrt(e11 * e22))
    assert asym[0] < 2e-3
    assert asym[1] < 0.25 * asym[0]
