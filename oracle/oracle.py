"""ctypes binding of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark call it; the product library never does.

Arrays are numpy float64 / int32 / int64, C-contiguous.  Shapes:
  nodes [n_nodes, 3], tets [n_tets, 4] (0-based), M [F, n_nodes, 3],
  targets [n_targets, 3], u [F, n_targets].
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

_dp = C.POINTER(C.c_double)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(_HERE, "oracle.c")
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(src):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB)
    lib.orc_tet_potential.restype = C.c_double
    lib.orc_tet_potential.argtypes = [_dp, _dp, _dp]
    lib.orc_tet_potential_gauss.restype = C.c_double
    lib.orc_tet_potential_gauss.argtypes = [_dp, _dp, _dp, C.c_int]
    lib.orc_gauss_legendre01_rule.restype = C.c_int
    lib.orc_gauss_legendre01_rule.argtypes = [C.c_int, _dp, _dp]
    lib.orc_tet_potential_direct.restype = C.c_double
    lib.orc_tet_potential_direct.argtypes = [_dp, _dp, _dp]
    lib.orc_tet_distance_ratio.restype = C.c_double
    lib.orc_tet_distance_ratio.argtypes = [_dp, _dp]
    lib.orc_direct.restype = C.c_int
    lib.orc_direct.argtypes = [_dp, C.c_int64, _i32p, C.c_int64, _dp, C.c_int32, _dp, C.c_int64, _dp]
    lib.orc_ncoef.restype = C.c_int
    lib.orc_ncoef.argtypes = [C.c_int]
    lib.orc_multi_indices.restype = C.c_int
    lib.orc_multi_indices.argtypes = [C.c_int, _i32p]
    lib.orc_taylor_coeffs.restype = C.c_int
    lib.orc_taylor_coeffs.argtypes = [_dp, C.c_int, _dp]
    lib.orc_p2m_tet.restype = C.c_int
    lib.orc_p2m_tet.argtypes = [_dp, _dp, _dp, C.c_int, _dp]
    for name in ("orc_m2m", "orc_m2l", "orc_l2l"):
        f = getattr(lib, name)
        f.restype = C.c_int
        f.argtypes = [_dp, _dp, C.c_int, _dp]
    lib.orc_l2p_eval.restype = C.c_int
    lib.orc_l2p_eval.argtypes = [_dp, _dp, _dp, C.c_int, _dp]
    lib.orc_fmm_build.restype = C.c_void_p
    lib.orc_fmm_build.argtypes = [_dp, C.c_int64, _i32p, C.c_int64, _dp, C.c_int64, C.c_int32, C.c_int32, C.c_double]
    lib.orc_fmm_free.restype = None
    lib.orc_fmm_free.argtypes = [C.c_void_p]
    lib.orc_fmm_stats.restype = None
    lib.orc_fmm_stats.argtypes = [C.c_void_p, _i64p]
    lib.orc_fmm_lists.restype = C.c_int64
    lib.orc_fmm_lists.argtypes = [C.c_void_p, C.c_int32, _i32p]
    lib.orc_fmm_cells.restype = C.c_int64
    lib.orc_fmm_cells.argtypes = [C.c_void_p, _i32p, _dp]
    lib.orc_fmm_evaluate.restype = C.c_int
    lib.orc_fmm_evaluate.argtypes = [C.c_void_p, _dp, C.c_int32, _dp]
    lib.orc_fmm_evaluate_sample.restype = C.c_int
    lib.orc_fmm_evaluate_sample.argtypes = [C.c_void_p, _dp, C.c_int32, _i64p, C.c_int64, _dp]
    lib.orc_fmm_set_level_orders.restype = C.c_int
    lib.orc_fmm_set_level_orders.argtypes = [C.c_void_p, _i32p, C.c_int32]
    lib.orc_fmm_expansions.restype = C.c_int
    lib.orc_fmm_expansions.argtypes = [C.c_void_p, C.c_int32, _dp]
    lib.orc_dipole_potential.restype = C.c_double
    lib.orc_dipole_potential.argtypes = [_dp, _dp, _dp]
    lib.orc_p2m_dipole.restype = C.c_int
    lib.orc_p2m_dipole.argtypes = [_dp, _dp, _dp, C.c_int, _dp]
    lib.orc_dipole_direct.restype = C.c_int
    lib.orc_dipole_direct.argtypes = [_dp, C.c_int64, _dp, C.c_int32, _dp, C.c_int64, _dp]
    lib.orc_fmm_build_points.restype = C.c_void_p
    lib.orc_fmm_build_points.argtypes = [_dp, C.c_int64, _dp, C.c_int64, C.c_int32, C.c_int32, C.c_double]
    lib.orc_demag.restype = C.c_int
    lib.orc_demag.argtypes = [_dp, C.c_int64, _i32p, C.c_int64, _dp, _dp, _dp, _dp, _dp]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_num_threads.restype = None
    lib.orc_set_num_threads.argtypes = [C.c_int]
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(t)


def num_threads():
    return _load().orc_num_threads()


def set_num_threads(n):
    _load().orc_set_num_threads(int(n))


def ncoef(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def multi_indices(p):
    """Multi-indices |n| <= p in the oracle's graded order, [ncoef, 3]."""
    out = np.zeros((ncoef(p), 3), dtype=np.int32)
    assert _load().orc_multi_indices(p, _ptr(out, _i32p)) == 0
    return out


def tet_potential(x, v, M):
    """Exact u_T(x) for one tet: x [3], v [4,3] corners, M [4,3] nodal values."""
    x, v, M = _d(x), _d(v), _d(M)
    return _load().orc_tet_potential(_ptr(x, _dp), _ptr(v, _dp), _ptr(M, _dp))


def tet_potential_gauss(x, v, M, n=8):
    """u_T(x) by the n^3-point collapsed Gauss-Legendre product rule (exact for
    integrands of total degree 2n - 3); accurate only for targets far from the tet."""
    x, v, M = _d(x), _d(v), _d(M)
    return _load().orc_tet_potential_gauss(_ptr(x, _dp), _ptr(v, _dp), _ptr(M, _dp), int(n))


def gauss_legendre01(n):
    """The oracle's n-point Gauss-Legendre rule on [0, 1]: nodes, weights."""
    t, w = np.zeros(n), np.zeros(n)
    if _load().orc_gauss_legendre01_rule(int(n), _ptr(t, _dp), _ptr(w, _dp)) != 0:
        raise ValueError("1 <= n <= 24")
    return t, w


def tet_potential_direct(x, v, M):
    """u_T(x) as the direct sum takes it: closed form within 3 diameters, Gauss beyond."""
    x, v, M = _d(x), _d(v), _d(M)
    return _load().orc_tet_potential_direct(_ptr(x, _dp), _ptr(v, _dp), _ptr(M, _dp))


def tet_distance_ratio(x, v):
    """|x - centroid| / longest edge."""
    x, v = _d(x), _d(v)
    return _load().orc_tet_distance_ratio(_ptr(x, _dp), _ptr(v, _dp))


def direct(nodes, tets, M, targets=None):
    """O(N^2) direct sum (closed form within 3 tet diameters, a degree-13 Gauss
    rule beyond).  M [F, n_nodes, 3] or [n_nodes, 3] -> u [F, nt] or [nt]."""
    nodes = _d(nodes)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    M = _d(M)
    squeeze = M.ndim == 2
    if squeeze:
        M = M[None]
    targets = nodes if targets is None else _d(targets)
    F = M.shape[0]
    u = np.zeros((F, targets.shape[0]))
    rc = _load().orc_direct(_ptr(nodes, _dp), nodes.shape[0], _ptr(tets, _i32p), tets.shape[0], _ptr(M, _dp), F,
                            _ptr(targets, _dp), targets.shape[0], _ptr(u, _dp))
    if rc != 0:
        raise ValueError("orc_direct: bad input")
    return u[0] if squeeze else u


def demag(nodes, tets, M, u):
    """P1 demagnetising field and energy from nodal potentials u [n]:
    returns (E / mu0, H per tet [T, 3], lumped nodal H [n, 3])."""
    nodes = _d(nodes)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    M = _d(M)
    u = _d(u)
    if M.shape != (nodes.shape[0], 3) or u.shape != (nodes.shape[0],):
        raise ValueError("M must be [n, 3] and u [n]")
    Ht = np.zeros((tets.shape[0], 3))
    Hn = np.zeros((nodes.shape[0], 3))
    E = C.c_double(0.0)
    if _load().orc_demag(_ptr(nodes, _dp), nodes.shape[0], _ptr(tets, _i32p), tets.shape[0], _ptr(M, _dp),
                         _ptr(u, _dp), _ptr(Ht, _dp), _ptr(Hn, _dp), C.byref(E)) != 0:
        raise ValueError("orc_demag: bad input")
    return E.value, Ht, Hn


def taylor_coeffs(x, p):
    a = np.zeros(ncoef(p))
    x = _d(x)
    assert _load().orc_taylor_coeffs(_ptr(x, _dp), p, _ptr(a, _dp)) == 0
    return a


def p2m_tet(v, M, c, p):
    Q = np.zeros(ncoef(p))
    v, M, c = _d(v), _d(M), _d(c)
    assert _load().orc_p2m_tet(_ptr(v, _dp), _ptr(M, _dp), _ptr(c, _dp), p, _ptr(Q, _dp)) == 0
    return Q


def _shift(name, X, d, p):
    out = np.zeros(ncoef(p))
    X, d = _d(X), _d(d)
    assert getattr(_load(), name)(_ptr(X, _dp), _ptr(d, _dp), p, _ptr(out, _dp)) == 0
    return out


def m2m(Qc, delta, p):
    """Multipole shift, delta = c_child - c_parent."""
    return _shift("orc_m2m", Qc, delta, p)


def m2l(Qb, R, p):
    """Multipole at c_B -> local at c_A, R = c_A - c_B (includes 1/(4 pi))."""
    return _shift("orc_m2l", Qb, R, p)


def l2l(Lp, delta, p):
    """Local shift, delta = c_child - c_parent."""
    return _shift("orc_l2l", Lp, delta, p)


def l2p(L, x, c, p):
    u = np.zeros(1)
    L, x, c = _d(L), _d(x), _d(c)
    assert _load().orc_l2p_eval(_ptr(L, _dp), _ptr(x, _dp), _ptr(c, _dp), p, _ptr(u, _dp)) == 0
    return float(u[0])


class FMM:
    """Oracle FMM: tree + lists at construction, evaluate() per field set."""

    def __init__(self, nodes, tets, p, leaf, theta, targets=None):
        self.nodes = _d(nodes)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.targets = None if targets is None else _d(targets)
        self.p = int(p)
        lib = _load()
        tp = _ptr(self.targets, _dp) if self.targets is not None else None
        nt = self.targets.shape[0] if self.targets is not None else 0
        h = lib.orc_fmm_build(_ptr(self.nodes, _dp), self.nodes.shape[0], _ptr(self.tets, _i32p), self.tets.shape[0],
                              tp, nt, int(p), int(leaf), float(theta))
        if not h:
            raise ValueError("orc_fmm_build: bad input")
        self._h = C.c_void_p(h)
        self.n_targets = self.stats()["n_targets"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_fmm_free(h)
            self._h = None

    def set_level_orders(self, orders):
        """Expansion order per octree level (level l takes orders[min(l, len - 1)],
        clamped to [1, p]); the default is p everywhere."""
        o = np.ascontiguousarray(orders, dtype=np.int32)
        if _load().orc_fmm_set_level_orders(self._h, _ptr(o, _i32p), o.size) != 0:
            raise ValueError("bad level orders")

    def stats(self):
        out = np.zeros(8, dtype=np.int64)
        _load().orc_fmm_stats(self._h, _ptr(out, _i64p))
        keys = ["ncells", "nleaves", "depth", "n_m2l", "n_p2p", "n_p2p_pairs", "ncoef", "n_targets"]
        return dict(zip(keys, (int(x) for x in out)))

    def lists(self, kind):
        """kind 'm2l' or 'p2p' -> int32 [n, 8]: (levA, ixA, iyA, izA, levB, ixB, iyB, izB)."""
        k = 0 if kind == "m2l" else 1
        n = _load().orc_fmm_lists(self._h, k, None)
        out = np.zeros((n, 8), dtype=np.int32)
        _load().orc_fmm_lists(self._h, k, _ptr(out, _i32p))
        return out

    def cells(self):
        """(int32 [ncells, 6]: level, ix, iy, iz, ntets, ntgts ; float64 [ncells, 2]: rsrc, rtgt)."""
        n = _load().orc_fmm_cells(self._h, None, None)
        out = np.zeros((n, 6), dtype=np.int32)
        rad = np.zeros((n, 2))
        _load().orc_fmm_cells(self._h, _ptr(out, _i32p), _ptr(rad, _dp))
        return out, rad

    def evaluate(self, M):
        M = _d(M)
        squeeze = M.ndim == 2
        if squeeze:
            M = M[None]
        F = M.shape[0]
        u = np.zeros((F, self.n_targets))
        assert _load().orc_fmm_evaluate(self._h, _ptr(M, _dp), F, _ptr(u, _dp)) == 0
        return u[0] if squeeze else u

    def evaluate_sample(self, M, sample):
        M = _d(M)
        squeeze = M.ndim == 2
        if squeeze:
            M = M[None]
        sample = np.ascontiguousarray(sample, dtype=np.int64)
        F = M.shape[0]
        u = np.zeros((F, sample.shape[0]))
        rc = _load().orc_fmm_evaluate_sample(self._h, _ptr(M, _dp), F, _ptr(sample, _i64p), sample.shape[0],
                                             _ptr(u, _dp))
        if rc != 0:
            raise ValueError("orc_fmm_evaluate_sample: bad sample index")
        return u[0] if squeeze else u

    def expansions(self, which):
        """After evaluate(): 'Q' (multipole) or 'L' (local), [ncells, ncoef], last field."""
        st = self.stats()
        out = np.zeros((st["ncells"], st["ncoef"]))
        assert _load().orc_fmm_expansions(self._h, 0 if which == "Q" else 1, _ptr(out, _dp)) == 0
        return out


# ---------------------------------------------------------------------------
# Point dipoles (the paper's second source kind, its "Mag FMM", Sec. 4)
# ---------------------------------------------------------------------------
def dipole_potential(x, y, m):
    """m . (x - y) / (4 pi |x - y|^3); 0 at x = y."""
    x, y, m = _d(x), _d(y), _d(m)
    return _load().orc_dipole_potential(_ptr(x, _dp), _ptr(y, _dp), _ptr(m, _dp))


def p2m_dipole(y, m, c, p):
    """Multipole coefficients of one dipole about c: Q_n = sum_k n_k m_k (y - c)^(n - e_k)."""
    Q = np.zeros(ncoef(p))
    y, m, c = _d(y), _d(m), _d(c)
    assert _load().orc_p2m_dipole(_ptr(y, _dp), _ptr(m, _dp), _ptr(c, _dp), p, _ptr(Q, _dp)) == 0
    return Q


def dipole_direct(points, M, targets=None):
    """O(N^2) dipole sum.  M [F, n, 3] or [n, 3] moments -> u [F, nt] or [nt]."""
    points = _d(points)
    M = _d(M)
    squeeze = M.ndim == 2
    if squeeze:
        M = M[None]
    F = M.shape[0]
    if targets is None:
        tp, nt, nu = None, 0, points.shape[0]
    else:
        tgt = _d(targets)
        tp, nt, nu = _ptr(tgt, _dp), tgt.shape[0], tgt.shape[0]
    u = np.zeros((F, nu))
    assert _load().orc_dipole_direct(_ptr(points, _dp), points.shape[0], _ptr(M, _dp), F, tp, nt, _ptr(u, _dp)) == 0
    return u[0] if squeeze else u


class DipoleFMM(FMM):
    """Oracle FMM over point dipoles at `points` (same tree, lists and
    translations as FMM; dipole P2M and near field).  evaluate(M) takes the
    moments M [F, n, 3] or [n, 3]."""

    def __init__(self, points, p, leaf, theta, targets=None):
        self.nodes = _d(points)
        self.tets = None
        self.targets = None if targets is None else _d(targets)
        self.p = int(p)
        lib = _load()
        tp = _ptr(self.targets, _dp) if self.targets is not None else None
        nt = self.targets.shape[0] if self.targets is not None else 0
        h = lib.orc_fmm_build_points(_ptr(self.nodes, _dp), self.nodes.shape[0], tp, nt, int(p), int(leaf),
                                     float(theta))
        if not h:
            raise ValueError("orc_fmm_build_points: bad input")
        self._h = C.c_void_p(h)
        self.n_targets = self.stats()["n_targets"]
