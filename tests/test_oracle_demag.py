"""Pins of the oracle's demagnetising field and energy (orc_demag): the P1
field per tet, the lumped nodal field and E / mu0 = 1/2 int M . grad u, the
quantity the paper reports for the magnetised box (Sec. 4.1).

 - exact for a linear potential: H = -a on every tet and node, and the
   energy of an affine M in closed form over the box;
 - the lumped nodal field conserves the volume integral of H;
 - the uniformly magnetised cube: E -> mu0 Ms^2 / 6 under refinement (Sec. 4.1);
 - reciprocity <m1, H(m2)> = <m2, H(m1)> up to a discretisation error that
   shrinks with h.
"""
import json
import os

import numpy as np

import meshgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_constants.json")


def test_linear_potential_exact(orc):
    lo, hi = np.array([-0.3, 0.1, 0.0]), np.array([0.9, 0.7, 1.5])
    nodes, tets = meshgen.box_mesh((5, 4, 6), lo=lo, hi=hi, jitter=0.15, seed=4)
    rng = np.random.default_rng(1)
    a, b0 = rng.standard_normal(3), 0.7
    A, b = rng.standard_normal((3, 3)), rng.standard_normal(3)
    u = nodes @ a + b0
    M = nodes @ A.T + b
    E, Ht, Hn = orc.demag(nodes, tets, M, u)
    assert np.abs(Ht + a).max() <= 1e-12 * np.abs(a).max()
    assert np.abs(Hn + a).max() <= 1e-12 * np.abs(a).max()
    vol = np.prod(hi - lo)
    centre = 0.5 * (lo + hi)
    E_exact = 0.5 * vol * a @ (A @ centre + b)  # 1/2 int_box M . a, M affine
    assert abs(E - E_exact) <= 1e-12 * abs(E_exact)


def test_lumped_field_conserves_the_volume_integral(orc):
    nodes, tets = meshgen.box_mesh(5, jitter=0.15, seed=2)
    rng = np.random.default_rng(3)
    u = np.sin(3 * nodes[:, 0]) * nodes[:, 1] + nodes[:, 2] ** 2
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=4)[0]
    E, Ht, Hn = orc.demag(nodes, tets, M, u)
    v = nodes[tets]
    vol = np.abs(np.einsum("ij,ij->i", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))) / 6.0
    w = meshgen.lumped_volumes(nodes, tets)
    assert np.allclose((w[:, None] * Hn).sum(0), (vol[:, None] * Ht).sum(0), rtol=1e-12, atol=1e-14)
    # and E equals -1/2 sum_T V_T Mbar_T . H_T
    mbar = M[tets].mean(1)
    assert abs(E + 0.5 * np.sum(vol * np.einsum("ij,ij->i", mbar, Ht))) <= 1e-13 * abs(E)
    # every nodal value is a convex combination of its tets' values
    for j in rng.choice(nodes.shape[0], 20, replace=False):
        adj = np.flatnonzero((tets == j).any(1))
        assert np.all(Hn[j] <= Ht[adj].max(0) + 1e-12) and np.all(Hn[j] >= Ht[adj].min(0) - 1e-12)


def test_cube_energy_converges_to_one_sixth(orc):
    with open(GOLDEN) as f:
        target = json.load(f)["cube_energy_over_mu0_ms2"]["value"]
    errs = []
    for n in (6, 12):
        nodes, tets = meshgen.box_mesh(n, jitter=0.15, seed=0)
        M = meshgen.uniform_field(nodes.shape[0], (0.0, 0.0, 1.0))
        u = orc.direct(nodes, tets, M)
        E, _, _ = orc.demag(nodes, tets, M, u)
        errs.append(abs(E - target))
    assert errs[0] <= 1e-2
    assert errs[1] <= 5e-3
    assert errs[1] < 0.6 * errs[0]


def test_reciprocity(orc):
    """Smooth fields (random nodal fields make the cross term tiny); the
    asymmetry is normalised by the geometric mean of the self energies."""
    asym = []
    for n in (4, 8):
        nodes, tets = meshgen.box_mesh(n, jitter=0.15, seed=5)
        x, y, z = nodes.T
        M1 = np.stack([np.cos(2 * y), np.sin(3 * z), x ** 2], axis=1)
        M2 = np.stack([z, np.cos(2 * x), np.sin(y)], axis=1)
        u1, u2 = orc.direct(nodes, tets, np.stack([M1, M2]))
        e12, _, _ = orc.demag(nodes, tets, M1, u2)  # -1/2 <m1, H(m2)>
        e21, _, _ = orc.demag(nodes, tets, M2, u1)
        e11, _, _ = orc.demag(nodes, tets, M1, u1)
        e22, _, _ = orc.demag(nodes, tets, M2, u2)
        assert e11 > 0 and e22 > 0  # the stray-field energy is positive
        asym.append(abs(e12 - e21) / np.sqrt(e11 * e22))
    assert asym[0] < 2e-3
    assert asym[1] < 0.25 * asym[0]
