"""Operation count of the oracle's pair integral (orc_tet_potential).

Test and measurement infrastructure: compiles oracle.c unchanged against a
counting scalar type (opcount.cpp) and counts the floating-point operations
of the exact potential of one affinely magnetised tetrahedron (Sec. 2.1) per
(target, tet) pair.  Pricing the elementary functions at the FP64
instruction counts of their ROCm device implementations turns the count into
the algorithmic flops per near-field pair.

    python -m oracle.opcount      # prints the per-pair count on the 8^3 cube
"""
import ctypes as C
import json
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "opcount.cpp")
LIB = os.path.join(HERE, "libopcount.so")
FIELDS = ("add", "mul", "div", "sqrt", "log", "atan", "cmp", "other")

# FP64 VALU instructions of one call of the ROCm device function (gfx950,
# hipcc -O3; counted in the assembly of a one-line kernel per function).
ELEMENTARY_F64_INSTRUCTIONS = {"div": 11, "sqrt": 14, "log": 76, "atan": 35}

_lib = None


def build(verbose=False):
    cmd = ["g++", "-O1", "-fpermissive", "-w", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                                                 os.path.getmtime(os.path.join(HERE, "oracle.c"))):
            build()
        lib = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        lib.opc_count_pairs.restype = None
        lib.opc_count_pairs.argtypes = [dp, C.POINTER(C.c_int32), dp, dp, C.POINTER(C.c_int64),
                                        C.POINTER(C.c_int64), C.c_int64, C.POINTER(C.c_longlong), dp]
        _lib = lib
    return _lib


def count_pairs(nodes, tets, targets, M, pair_tgt, pair_tet):
    """Summed operation counts of orc_tet_potential over the given pairs, and
    the summed potential (a check value)."""
    lib = _load()
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    targets = np.ascontiguousarray(targets, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    pt = np.ascontiguousarray(pair_tgt, dtype=np.int64)
    pq = np.ascontiguousarray(pair_tet, dtype=np.int64)
    out = (C.c_longlong * 8)()
    u = C.c_double(0.0)
    dp = C.POINTER(C.c_double)
    lib.opc_count_pairs(nodes.ctypes.data_as(dp), tets.ctypes.data_as(C.POINTER(C.c_int32)),
                        targets.ctypes.data_as(dp), M.ctypes.data_as(dp), pt.ctypes.data_as(C.POINTER(C.c_int64)),
                        pq.ctypes.data_as(C.POINTER(C.c_int64)), len(pt), out, C.byref(u))
    return dict(zip(FIELDS, (int(v) for v in out))), u.value


def flops(counts, per=1):
    """Algorithmic flops of a count: adds and multiplies one each, the
    divide, sqrt, log and atan at their FP64 instruction counts."""
    f = counts["add"] + counts["mul"] + sum(counts[k] * c for k, c in ELEMENTARY_F64_INSTRUCTIONS.items())
    return f / per


def cube_pairs(n=8, seed=0):
    """Every (node, tet) pair of the jittered n^3 Kuhn cube with one random
    unit field: the count per pair, its spread and its flops."""
    sys.path.insert(0, os.path.dirname(HERE))
    import meshgen
    nodes, tets = meshgen.box_mesh(n, seed=seed)
    M = meshgen.random_fields(nodes.shape[0], F=1, seed=1)[0]
    nt, nq = nodes.shape[0], tets.shape[0]
    pt = np.repeat(np.arange(nt, dtype=np.int64), nq)
    pq = np.tile(np.arange(nq, dtype=np.int64), nt)
    total, _ = count_pairs(nodes, tets, nodes, M, pt, pq)
    # one generic pair (the target off every face plane and edge line) and one
    # touching pair (the target a corner of the tet)
    far = int(np.argmax(np.linalg.norm(nodes - nodes.mean(0), axis=1)))
    c_far, _ = count_pairs(nodes, tets, nodes, M, [0], [int(np.argmax(
        np.linalg.norm(nodes[tets].mean(1) - nodes[0], axis=1)))])
    touch = int(np.nonzero((tets == far).any(1))[0][0])
    c_touch, _ = count_pairs(nodes, tets, nodes, M, [far], [touch])
    npairs = nt * nq
    return {"mesh": f"{n}^3 cube, {nq} tets, {nt} nodes, all {npairs} pairs",
            "per_pair_mean": {k: v / npairs for k, v in total.items()},
            "flops_per_pair_mean": flops(total, npairs),
            "generic_pair": c_far, "flops_generic_pair": flops(c_far),
            "touching_pair": c_touch, "flops_touching_pair": flops(c_touch),
            "elementary_f64_instructions": ELEMENTARY_F64_INSTRUCTIONS}


if __name__ == "__main__":
    print(json.dumps(cube_pairs(), indent=1))
