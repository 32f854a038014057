"""Python binding of libtetfmm.so, the MI355X (gfx950) tetrahedral FMM.

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of the library.  The names mirror the C ABI of include/tetfmm.h.
There is no fallback: if the library is not built, loading fails loudly.

Device arrays are torch tensors on the plan's GPU (float64, contiguous);
work is queued on torch's current stream of that device unless a stream is
given.
"""
import ctypes as C
import os

import numpy as np

__all__ = [
    "TetFMMError", "Plan", "tfmm_plan_create", "tfmm_evaluate", "tfmm_direct", "tfmm_evaluate_host",
    "tfmm_direct_host", "tfmm_plan_stats", "tfmm_plan_lists", "tfmm_plan_cells", "tfmm_plan_expansions",
    "tfmm_plan_destroy", "tfmm_last_error", "tfmm_simplex_rule", "tfmm_set_timing", "tfmm_kernel_times",
    "library_path", "TFMM_PMAX", "KERNEL_NAMES", "ERRORS", "tfmm_plan_set_m2l_precision", "tfmm_plan_set_surrogate", "tfmm_plan_set_level_orders", "tfmm_tune_level_orders", "SUR_OFF", "SUR_MLP", "SUR_GAUSS", "SUR_QUAD", "M2L_FP64", "M2L_FP32", "M2L_BF16X3", "M2L_BF16X6",
    "tfmm_plan_autotune", "tfmm_plan_set_schedule", "tfmm_elementary", "ELEMENTARY", "tfmm_batch_create", "tfmm_batch_evaluate", "tfmm_batch_autotune", "tfmm_batch_plan", "tfmm_batch_merged_plan", "tfmm_batch_set_merged",
    "tfmm_batch_destroy", "Batch", "tfmm_surrogate_param_count", "tfmm_surrogate_train", "tfmm_surrogate_load",
    "tfmm_surrogate_samples", "tfmm_surrogate_grad", "tfmm_band_potential", "tfmm_demag_energy", "tfmm_demag_energy_noalloc", "NOALLOC_MAX_TETS", "tfmm_demag_field_nodes",
    "tfmm_plan_store_near", "tfmm_tune_accuracy", "tfmm_plan_create_points",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libtetfmm.so")
_lib = None

TFMM_PMAX = 10
M2L_FP64 = 0
M2L_FP32 = 1
M2L_BF16X3 = 2
M2L_BF16X6 = 3
SUR_OFF = 0
SUR_MLP = 1
SUR_GAUSS = 2
SUR_QUAD = 3
KERNEL_NAMES = ("p2m", "m2m", "m2l", "l2l", "l2p", "p2p")
ERRORS = {-1: "EINVAL", -2: "EINDEX", -3: "EDEGEN", -4: "ENONFINITE", -5: "ENOMEM", -6: "EDEVICE", -7: "ENOTSUP"}

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


class _TrainCfg(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("seed", C.c_uint64)]


class _Params(C.Structure):
    _fields_ = [("p", C.c_int32), ("leaf_size", C.c_int32), ("theta", C.c_double), ("m2l_precision", C.c_int32),
                ("surrogate", C.c_int32), ("device", C.c_int32)]


class _TuneResult(C.Structure):
    _fields_ = [("p", C.c_int32), ("theta", C.c_double), ("err", C.c_double), ("ms", C.c_double),
                ("n_tried", C.c_int32), ("met", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_nodes", "n_tets", "n_targets", "n_cells", "n_leaves", "depth", "n_m2l",
                                        "n_p2p", "n_p2p_pairs", "ncoef", "device_bytes")] + [("setup_seconds",
                                                                                               C.c_double)] + [
        ("near_nnz", C.c_int64), ("near_bytes", C.c_int64),
        ("m2l_keys_per_item", C.c_int32), ("p2p_wide", C.c_int32),
        ("p2p_node_evals", C.c_int64), ("p2p_edge_evals", C.c_int64), ("p2p_face_evals", C.c_int64),
        ("n_band_pairs", C.c_int64), ("surrogate", C.c_int32), ("surrogate_hidden", C.c_int32),
        ("level_order", C.c_int32 * 22), ("m2l_packed", C.c_int32), ("m2l_groups_per_item", C.c_int32),
        ("m2l_groups", C.c_int64)]


class TetFMMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def library_path():
    return _LIBPATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise RuntimeError(f"libtetfmm.so is not built ({_LIBPATH}); run __graft_entry__.build() "
                           "or python -m paper_1606_00247_amd.build")
    lib = C.CDLL(_LIBPATH)
    sig = {
        "tfmm_plan_create": (C.c_int, [_dp, C.c_int64, _i32p, C.c_int64, _dp, C.c_int64, C.POINTER(_Params),
                                       C.POINTER(C.c_void_p)]),
        "tfmm_evaluate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
        "tfmm_direct": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
        "tfmm_evaluate_host": (C.c_int, [C.c_void_p, _dp, C.c_int32, _dp]),
        "tfmm_direct_host": (C.c_int, [C.c_void_p, _dp, C.c_int32, _dp]),
        "tfmm_plan_stats": (C.c_int, [C.c_void_p, C.POINTER(_Stats)]),
        "tfmm_plan_lists": (C.c_int64, [C.c_void_p, C.c_int32, _i32p]),
        "tfmm_plan_cells": (C.c_int64, [C.c_void_p, _i32p, _dp]),
        "tfmm_plan_expansions": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
        "tfmm_plan_destroy": (C.c_int, [C.c_void_p]),
        "tfmm_plan_set_m2l_precision": (C.c_int, [C.c_void_p, C.c_int32]),
        "tfmm_plan_set_surrogate": (C.c_int, [C.c_void_p, C.c_int32]),
        "tfmm_plan_set_level_orders": (C.c_int, [C.c_void_p, _i32p, C.c_int32]),
        "tfmm_tune_level_orders": (C.c_int, [C.c_void_p, _dp, C.c_double, C.c_int32, C.c_uint64, _i32p, _dp, _dp]),
        "tfmm_plan_store_near": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
        "tfmm_plan_create_points": (C.c_int, [_dp, C.c_int64, _dp, C.c_int64, C.c_void_p, C.POINTER(C.c_void_p)]),
        "tfmm_tune_accuracy": (C.c_int, [_dp, C.c_int64, _i32p, C.c_int64, C.c_void_p, _dp, C.c_double, C.c_int32,
                                         C.c_uint64, _i32p, C.c_int32, _dp, C.c_int32, C.POINTER(_TuneResult), _dp]),
        "tfmm_tune_accuracy_points": (C.c_int, [_dp, C.c_int64, C.c_void_p, _dp, C.c_double, C.c_int32, C.c_uint64,
                                                _i32p, C.c_int32, _dp, C.c_int32, C.POINTER(_TuneResult), _dp]),
        "tfmm_last_error": (C.c_char_p, []),
        "tfmm_simplex_rule": (C.c_int, [C.c_int32, _dp, _i32p]),
        "tfmm_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
        "tfmm_kernel_times": (C.c_int, [C.c_void_p, _dp, _i64p]),
        "tfmm_plan_autotune": (C.c_int, [C.c_void_p, C.c_void_p]),
        "tfmm_plan_set_schedule": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "tfmm_elementary": (C.c_int, [C.c_int32, _dp, _dp, _dp, C.c_int64, C.c_int32]),
        "tfmm_demag_field_nodes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
        "tfmm_demag_energy_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                                C.c_void_p]),
        "tfmm_batch_create": (C.c_int, [C.c_int32, C.POINTER(_dp), _i64p, C.POINTER(_i32p), _i64p,
                                        C.POINTER(_Params), C.POINTER(C.c_void_p)]),
        "tfmm_batch_evaluate": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_void_p]),
        "tfmm_batch_autotune": (C.c_int, [C.c_void_p, C.c_void_p]),
        "tfmm_batch_plan": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
        "tfmm_batch_merged_plan": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
        "tfmm_batch_set_merged": (C.c_int, [C.c_void_p, C.c_int32]),
        "tfmm_batch_destroy": (C.c_int, [C.c_void_p]),
        "tfmm_surrogate_param_count": (C.c_int, [C.c_int32]),
        "tfmm_demag_energy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, _dp, C.c_void_p]),
        "tfmm_surrogate_train": (C.c_int, [C.c_void_p, C.POINTER(_TrainCfg), C.c_char_p, _dp]),
        "tfmm_surrogate_load": (C.c_int, [C.c_void_p, C.c_char_p]),
        "tfmm_surrogate_samples": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int32, _fp, _fp]),
        "tfmm_surrogate_grad": (C.c_int, [C.c_int32, _fp, _fp, _fp, C.c_int32, _fp, _dp, C.c_int32]),
        "tfmm_band_potential": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def tfmm_last_error():
    return _load().tfmm_last_error().decode()


def _check(rc):
    if rc < 0:
        raise TetFMMError(int(rc), tfmm_last_error())
    return rc


def _ptr(a, t):
    return a.ctypes.data_as(t)


class Plan:
    """Owns a tfmm_plan handle (destroyed with the object or tfmm_plan_destroy)."""

    def __init__(self, handle, device, n_nodes, n_targets, params):
        self._h = C.c_void_p(handle)
        self.device = device
        self.n_nodes = n_nodes
        self.n_targets = n_targets
        self.params = params

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan already destroyed")
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.tfmm_plan_destroy(h)
            self._h = None


def tfmm_plan_create(nodes, tets, targets=None, p=8, leaf_size=64, theta=0.5, m2l_precision=0, device=0,
                     surrogate=0):
    """Build the octree, lists and device data of a mesh (copies the host arrays)."""
    lib = _load()
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    if nodes.ndim != 2 or nodes.shape[1] != 3 or tets.ndim != 2 or tets.shape[1] != 4:
        raise ValueError("nodes must be [N,3] and tets [T,4]")
    tp, nt = None, 0
    if targets is not None:
        targets = np.ascontiguousarray(targets, dtype=np.float64)
        if targets.ndim != 2 or targets.shape[1] != 3:
            raise ValueError("targets must be [n,3]")
        tp, nt = _ptr(targets, _dp), targets.shape[0]
    prm = _Params(int(p), int(leaf_size), float(theta), int(m2l_precision), int(surrogate), int(device))
    h = C.c_void_p()
    _check(lib.tfmm_plan_create(_ptr(nodes, _dp), nodes.shape[0], _ptr(tets, _i32p), tets.shape[0], tp, nt,
                                C.byref(prm), C.byref(h)))
    return Plan(h.value, int(device), nodes.shape[0], nt if targets is not None else nodes.shape[0],
                dict(p=int(p), leaf_size=int(leaf_size), theta=float(theta), m2l_precision=int(m2l_precision)))


def tfmm_plan_create_points(points, targets=None, p=8, leaf_size=64, theta=0.5, m2l_precision=0, device=0,
                            surrogate=0):
    """Plan for point dipoles at `points` [n, 3]; evaluations take the dipole
    moments as M [F, n, 3] (device) and give u at the targets (default: the
    points, each excluding its own dipole)."""
    lib = _load()
    points = np.ascontiguousarray(points, dtype=np.float64)
    if points.ndim != 2 or points.shape[1] != 3:
        raise ValueError("points must be [n,3]")
    tp, nt = None, 0
    if targets is not None:
        targets = np.ascontiguousarray(targets, dtype=np.float64)
        if targets.ndim != 2 or targets.shape[1] != 3:
            raise ValueError("targets must be [n,3]")
        tp, nt = _ptr(targets, _dp), targets.shape[0]
    prm = _Params(int(p), int(leaf_size), float(theta), int(m2l_precision), int(surrogate), int(device))
    h = C.c_void_p()
    _check(lib.tfmm_plan_create_points(_ptr(points, _dp), points.shape[0], tp, nt, C.byref(prm), C.byref(h)))
    return Plan(h.value, int(device), points.shape[0], nt if targets is not None else points.shape[0],
                dict(p=int(p), leaf_size=int(leaf_size), theta=float(theta), m2l_precision=int(m2l_precision),
                     points=True))


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return C.c_void_p(stream.cuda_stream)


def _dev_call(fn, plan, M, u, stream):
    import torch
    if not (isinstance(M, torch.Tensor) and M.is_cuda and M.dtype == torch.float64 and M.is_contiguous()):
        raise ValueError("M must be a contiguous float64 CUDA tensor [F, n_nodes, 3] or [n_nodes, 3]")
    squeeze = M.dim() == 2
    F = 1 if squeeze else M.shape[0]
    if tuple(M.shape[-2:]) != (plan.n_nodes, 3):
        raise ValueError(f"M must end in [{plan.n_nodes}, 3]")
    if M.device.index != plan.device:
        raise ValueError("M is not on the plan's device")
    if u is None:
        u = torch.empty((plan.n_targets,) if squeeze else (F, plan.n_targets), dtype=torch.float64, device=M.device)
    elif not (u.is_cuda and u.dtype == torch.float64 and u.is_contiguous() and u.numel() == F * plan.n_targets):
        raise ValueError("u must be a contiguous float64 CUDA tensor with F * n_targets elements")
    _check(fn(plan.handle, C.c_void_p(M.data_ptr()), F, C.c_void_p(u.data_ptr()), _stream_handle(stream, M.device)))
    return u


def tfmm_evaluate(plan, M, u=None, stream=None):
    """FMM potential at the targets (asynchronous on `stream`)."""
    return _dev_call(_load().tfmm_evaluate, plan, M, u, stream)


def tfmm_direct(plan, M, u=None, stream=None):
    """O(N^2) direct sum of the exact tet integrals (asynchronous on `stream`)."""
    return _dev_call(_load().tfmm_direct, plan, M, u, stream)


def _host_call(fn, plan, M):
    M = np.ascontiguousarray(M, dtype=np.float64)
    squeeze = M.ndim == 2
    if squeeze:
        M = M[None]
    if M.shape[1:] != (plan.n_nodes, 3):
        raise ValueError(f"M must be [F, {plan.n_nodes}, 3]")
    u = np.zeros((M.shape[0], plan.n_targets))
    _check(fn(plan.handle, _ptr(M, _dp), M.shape[0], _ptr(u, _dp)))
    return u[0] if squeeze else u


def tfmm_evaluate_host(plan, M):
    return _host_call(_load().tfmm_evaluate_host, plan, M)


def tfmm_direct_host(plan, M):
    return _host_call(_load().tfmm_direct_host, plan, M)


def tfmm_plan_autotune(plan, stream=None):
    """Pick the plan's schedule (M2L work item size, P2P workgroup shape) by timing."""
    import torch
    dev = torch.device("cuda", plan.device)
    _check(_load().tfmm_plan_autotune(plan.handle, _stream_handle(stream, dev)))


def tfmm_plan_set_schedule(plan, m2l_keys_per_item, p2p_wide, m2l_packed=1, m2l_groups_per_item=256):
    """Set the schedule knobs tfmm_plan_autotune picks (same results, other launch shapes)."""
    _check(_load().tfmm_plan_set_schedule(plan.handle, int(m2l_keys_per_item), int(p2p_wide), int(m2l_packed),
                                          int(m2l_groups_per_item)))


ELEMENTARY = {"log_ratio": 0, "atan2": 1, "div": 2, "rsqrt": 3}


def tfmm_elementary(fn, a, b=None, device=0):
    """The near field's elementary function `fn` (a key of ELEMENTARY) on host arrays."""
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    b = np.zeros_like(a) if b is None else np.ascontiguousarray(b, dtype=np.float64).ravel()
    if a.shape != b.shape:
        raise ValueError("a and b must have the same size")
    out = np.zeros_like(a)
    _check(_load().tfmm_elementary(ELEMENTARY[fn], _ptr(a, _dp), _ptr(b, _dp), _ptr(out, _dp), a.size, int(device)))
    return out


class _BorrowedPlan(Plan):
    """A plan owned by a batch (not destroyed with this object)."""

    def __del__(self):
        pass


class Batch:
    """Owns a tfmm_batch handle: one plan per mesh, one field each."""

    def __init__(self, handle, device, sizes, params):
        self._h = C.c_void_p(handle)
        self.device = device
        self.sizes = sizes  # [(n_nodes, n_tets)]
        self.params = params

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch was destroyed")
        return self._h

    def __len__(self):
        return len(self.sizes)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.tfmm_batch_destroy(h)
            self._h = None


def tfmm_batch_create(meshes, p=8, leaf_size=64, theta=0.5, m2l_precision=0, device=0, surrogate=0):
    """meshes: sequence of (nodes [N_i, 3], tets [T_i, 4]) host arrays."""
    lib = _load()
    nodes = [np.ascontiguousarray(m[0], dtype=np.float64) for m in meshes]
    tets = [np.ascontiguousarray(m[1], dtype=np.int32) for m in meshes]
    n = len(nodes)
    NP = (_dp * n)(*[_ptr(a, _dp) for a in nodes])
    TP = (_i32p * n)(*[_ptr(a, _i32p) for a in tets])
    nn = np.array([a.shape[0] for a in nodes], dtype=np.int64)
    nt = np.array([a.shape[0] for a in tets], dtype=np.int64)
    prm = _Params(int(p), int(leaf_size), float(theta), int(m2l_precision), int(surrogate), int(device))
    h = C.c_void_p()
    _check(lib.tfmm_batch_create(n, NP, _ptr(nn, _i64p), TP, _ptr(nt, _i64p), C.byref(prm), C.byref(h)))
    return Batch(h.value, int(device), list(zip(nn.tolist(), nt.tolist())),
                 dict(p=int(p), leaf_size=int(leaf_size), theta=float(theta), m2l_precision=int(m2l_precision)))


def tfmm_batch_evaluate(batch, M, u=None, stream=None):
    """M: list of contiguous float64 CUDA tensors [n_nodes_i, 3]; returns the list u of [n_nodes_i]."""
    import torch
    if len(M) != len(batch):
        raise ValueError("one M per mesh")
    if u is None:
        u = [torch.empty(n_i, dtype=torch.float64, device=m.device) for (n_i, _), m in zip(batch.sizes, M)]
    for (n_i, _), m, ui in zip(batch.sizes, M, u):
        if not (isinstance(m, torch.Tensor) and m.is_cuda and m.dtype == torch.float64 and m.is_contiguous()
                and tuple(m.shape) == (n_i, 3) and m.device.index == batch.device):
            raise ValueError("each M must be a contiguous float64 CUDA tensor [n_nodes_i, 3] on the batch's device")
        if not (ui.is_cuda and ui.dtype == torch.float64 and ui.is_contiguous() and ui.numel() == n_i):
            raise ValueError("each u must be a contiguous float64 CUDA tensor of n_nodes_i elements")
    n = len(M)
    MP = (C.c_void_p * n)(*[C.c_void_p(m.data_ptr()) for m in M])
    UP = (C.c_void_p * n)(*[C.c_void_p(x.data_ptr()) for x in u])
    _check(_load().tfmm_batch_evaluate(batch.handle, MP, UP, _stream_handle(stream, M[0].device)))
    return u


def tfmm_batch_autotune(batch, stream=None):
    import torch
    _check(_load().tfmm_batch_autotune(batch.handle, _stream_handle(stream, torch.device("cuda", batch.device))))


def tfmm_batch_plan(batch, i):
    """The plan of mesh i (owned by the batch)."""
    h = C.c_void_p()
    _check(_load().tfmm_batch_plan(batch.handle, int(i), C.byref(h)))
    n_nodes = batch.sizes[i][0]
    return _BorrowedPlan(h.value, batch.device, n_nodes, n_nodes, dict(batch.params))


def tfmm_batch_merged_plan(batch):
    """The merged plan over all meshes (owned by the batch): set its precision,
    stored near field or schedule with the plan calls."""
    h = C.c_void_p()
    _check(_load().tfmm_batch_merged_plan(batch.handle, C.byref(h)))
    n = int(sum(s[0] for s in batch.sizes))
    return _BorrowedPlan(h.value, batch.device, n, n, dict(batch.params))


def tfmm_batch_set_merged(batch, on):
    """1 (default): evaluate the batch as its merged plan; 0: per-mesh plans."""
    _check(_load().tfmm_batch_set_merged(batch.handle, int(on)))


def tfmm_batch_destroy(batch):
    if batch._h is not None:
        _check(_load().tfmm_batch_destroy(batch._h))
        batch._h = None


def tfmm_demag_energy(plan, M, u, with_field=False, stream=None):
    """Stray-field energy over mu0 (and H per tet [n_tets, 3] when with_field) from nodal u."""
    import torch
    for a, shape in ((M, (plan.n_nodes, 3)), (u, (plan.n_nodes,))):
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()
                and tuple(a.shape) == shape):
            raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")
    H = None
    if with_field:
        H = torch.empty((tfmm_plan_stats(plan)["n_tets"], 3), dtype=torch.float64, device=M.device)
    E = C.c_double(0.0)
    _check(_load().tfmm_demag_energy(plan.handle, C.c_void_p(M.data_ptr()), C.c_void_p(u.data_ptr()),
                                     None if H is None else C.c_void_p(H.data_ptr()), C.byref(E),
                                     _stream_handle(stream, M.device)))
    return (E.value, H) if with_field else E.value


NOALLOC_MAX_TETS = 65535 * 256


def tfmm_demag_energy_noalloc(plan, M, u, energy, H=None, stream=None):
    """tfmm_demag_energy without allocation: E / mu0 into the device tensor
    `energy` (float64, one element) and, when H is given, H per tet into H
    [n_tets, 3]; asynchronous, nothing allocated (the caller's tensors only)."""
    import torch
    for a, shape in ((M, (plan.n_nodes, 3)), (u, (plan.n_nodes,)), (energy, (1,))):
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()
                and tuple(a.shape) == shape):
            raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")
    if H is not None and not (H.is_cuda and H.dtype == torch.float64 and H.is_contiguous() and H.dim() == 2
                              and H.shape[1] == 3):
        raise ValueError("H must be a contiguous float64 CUDA tensor [n_tets, 3]")
    _check(_load().tfmm_demag_energy_noalloc(plan.handle, C.c_void_p(M.data_ptr()), C.c_void_p(u.data_ptr()),
                                             None if H is None else C.c_void_p(H.data_ptr()),
                                             C.c_void_p(energy.data_ptr()), _stream_handle(stream, M.device)))
    return energy


def tfmm_demag_field_nodes(plan, u, H=None, stream=None):
    """Mass-lumped nodal field H [n_nodes, 3] from the nodal potential u (device)."""
    import torch
    if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()
            and tuple(u.shape) == (plan.n_nodes,)):
        raise ValueError(f"u must be a contiguous float64 CUDA tensor of shape ({plan.n_nodes},)")
    if H is None:
        H = torch.empty((plan.n_nodes, 3), dtype=torch.float64, device=u.device)
    elif not (H.is_cuda and H.dtype == torch.float64 and H.is_contiguous() and tuple(H.shape) == (plan.n_nodes, 3)):
        raise ValueError("H must be a contiguous float64 CUDA tensor [n_nodes, 3]")
    _check(_load().tfmm_demag_field_nodes(plan.handle, C.c_void_p(u.data_ptr()), C.c_void_p(H.data_ptr()),
                                          _stream_handle(stream, u.device)))
    return H


def tfmm_surrogate_param_count(hidden):
    return _check(_load().tfmm_surrogate_param_count(int(hidden)))


def tfmm_surrogate_train(plan, hidden=128, steps=3000, batch=4096, lr=1e-3, seed=1, out_path=None):
    """Train the near-field surrogate on pairs from the plan's tets; returns the final loss."""
    cfg = _TrainCfg(int(hidden), int(steps), int(batch), float(lr), int(seed))
    loss = C.c_double(0.0)
    path = None if out_path is None else os.fsencode(out_path)
    _check(_load().tfmm_surrogate_train(plan.handle, C.byref(cfg), path, C.byref(loss)))
    return loss.value


def tfmm_surrogate_load(plan, path):
    _check(_load().tfmm_surrogate_load(plan.handle, os.fsencode(path)))


def tfmm_surrogate_samples(plan, n, seed=7):
    """n training samples: inputs X [n, 16] and targets Y [n, 12] (float32)."""
    X = np.zeros((n, 16), dtype=np.float32)
    Y = np.zeros((n, 12), dtype=np.float32)
    _check(_load().tfmm_surrogate_samples(plan.handle, int(seed), int(n), _ptr(X, _fp), _ptr(Y, _fp)))
    return X, Y


def tfmm_surrogate_grad(hidden, params, X, Y, device=0):
    """Loss and gradient of the training kernels (FP32) for one batch."""
    params = np.ascontiguousarray(params, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    g = np.zeros_like(params)
    loss = C.c_double(0.0)
    _check(_load().tfmm_surrogate_grad(int(hidden), _ptr(params, _fp), _ptr(X, _fp), _ptr(Y, _fp), X.shape[0],
                                       _ptr(g, _fp), C.byref(loss), int(device)))
    return loss.value, g


def tfmm_band_potential(plan, M, use_surrogate, u=None, stream=None):
    """Potential of the near-field pairs at 2 <= |x - c|/d < 6 only (one field)."""
    import torch
    if not (isinstance(M, torch.Tensor) and M.is_cuda and M.dtype == torch.float64 and M.is_contiguous()
            and tuple(M.shape) == (plan.n_nodes, 3)):
        raise ValueError("M must be a contiguous float64 CUDA tensor [n_nodes, 3]")
    if u is None:
        u = torch.empty(plan.n_targets, dtype=torch.float64, device=M.device)
    _check(_load().tfmm_band_potential(plan.handle, int(bool(use_surrogate)), C.c_void_p(M.data_ptr()),
                                       C.c_void_p(u.data_ptr()), _stream_handle(stream, M.device)))
    return u


def tfmm_plan_stats(plan):
    st = _Stats()
    _check(_load().tfmm_plan_stats(plan.handle, C.byref(st)))
    out = {n: getattr(st, n) for n, _ in _Stats._fields_}
    out["level_order"] = list(out["level_order"])
    return out


def tfmm_plan_lists(plan, kind):
    """kind 'm2l', 'p2p', 'm2l_tiles' or 'm2l_packs' (the M2L pairs as the
    matrix-core tiles or the key-packed groups schedule them) -> int32 [n, 8]
    (levA, ixA, iyA, izA, levB, ixB, iyB, izB)."""
    k = {"m2l": 0, "p2p": 1, "m2l_tiles": 2, "m2l_packs": 3}[kind]
    n = _check(_load().tfmm_plan_lists(plan.handle, k, None))
    out = np.zeros((n, 8), dtype=np.int32)
    _check(_load().tfmm_plan_lists(plan.handle, k, _ptr(out, _i32p)))
    return out


def tfmm_plan_cells(plan):
    n = _check(_load().tfmm_plan_cells(plan.handle, None, None))
    cells = np.zeros((n, 6), dtype=np.int32)
    radii = np.zeros((n, 2))
    _check(_load().tfmm_plan_cells(plan.handle, _ptr(cells, _i32p), _ptr(radii, _dp)))
    return cells, radii


def tfmm_plan_expansions(plan, which):
    """'Q' (multipole) or 'L' (local) of the last evaluation's last field: [n_cells, ncoef]."""
    st = tfmm_plan_stats(plan)
    out = np.zeros((st["n_cells"], st["ncoef"]))
    _check(_load().tfmm_plan_expansions(plan.handle, {"Q": 0, "L": 1}[which], _ptr(out, _dp)))
    return out


def tfmm_plan_set_level_orders(plan, orders):
    """Expansion order per octree level (level l takes orders[min(l, len - 1)],
    each in [1, p] of the plan)."""
    o = np.ascontiguousarray(orders, dtype=np.int32)
    _check(_load().tfmm_plan_set_level_orders(plan.handle, _ptr(o, _i32p), o.size))


def tfmm_tune_level_orders(plan, M, tol, n_sample=512, seed=1):
    """Fastest per-level order profile whose sampled error against the FP64
    direct sum is within tol / 2 (set on the plan).  M: host [n_nodes, 3].
    Returns dict(orders [22], err, ms, met)."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    if M.shape != (plan.n_nodes, 3):
        raise ValueError("M must be [n_nodes, 3]")
    orders = np.zeros(22, dtype=np.int32)
    err, ms = C.c_double(0.0), C.c_double(0.0)
    _check(_load().tfmm_tune_level_orders(plan.handle, _ptr(M, _dp), float(tol), int(n_sample), int(seed),
                                          _ptr(orders, _i32p), C.byref(err), C.byref(ms)))
    return dict(orders=orders.tolist(), err=err.value, ms=ms.value, met=ms.value >= 0.0)


def tfmm_plan_set_surrogate(plan, mode):
    """How the near-field pairs 2-6 tet diameters apart are evaluated: SUR_OFF
    (exact), SUR_MLP (the attached network), SUR_GAUSS or SUR_QUAD (controls)."""
    _check(_load().tfmm_plan_set_surrogate(plan.handle, int(mode)))
    plan.params["surrogate"] = int(mode)


def tfmm_plan_set_m2l_precision(plan, m2l_precision):
    """M2L arithmetic of an existing plan: M2L_FP64, M2L_FP32, M2L_BF16X3 or M2L_BF16X6."""
    _check(_load().tfmm_plan_set_m2l_precision(plan.handle, int(m2l_precision)))
    plan.params["m2l_precision"] = int(m2l_precision)


def tfmm_tune_accuracy(nodes, tets, tol, M=None, leaf_size=64, m2l_precision=M2L_FP64, device=0, n_sample=512,
                       seed=1, p_list=(4, 5, 6, 7, 8, 9, 10), theta_list=(0.3, 0.35, 0.4, 0.45, 0.5, 0.55, 0.6, 0.7)):
    """Fastest (p, theta) whose sampled error against the FP64 direct sum is at
    most tol / 2.  M: host [n_nodes, 3] probe field (default: seeded random unit
    vectors).  tets=None tunes a point-dipole plan at `nodes` (M = moments).
    Returns dict(p, theta, err, ms, met, n_tried, table[n_p*n_theta, 4])."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    if tets is not None:
        tets = np.ascontiguousarray(tets, dtype=np.int32)
    if M is None:
        g = np.random.default_rng(seed).standard_normal((nodes.shape[0], 3))
        M = g / np.linalg.norm(g, axis=1, keepdims=True)
    M = np.ascontiguousarray(M, dtype=np.float64)
    if M.shape != (nodes.shape[0], 3):
        raise ValueError("M must be [n_nodes, 3]")
    pl = np.ascontiguousarray(p_list, dtype=np.int32)
    tl = np.ascontiguousarray(theta_list, dtype=np.float64)
    table = np.zeros((pl.size * tl.size, 4))
    prm = _Params(8, int(leaf_size), 0.5, int(m2l_precision), SUR_OFF, int(device))
    res = _TuneResult()
    if tets is None:
        _check(_load().tfmm_tune_accuracy_points(_ptr(nodes, _dp), nodes.shape[0], C.byref(prm), _ptr(M, _dp),
                                                 float(tol), int(n_sample), int(seed), _ptr(pl, _i32p), pl.size,
                                                 _ptr(tl, _dp), tl.size, C.byref(res), _ptr(table, _dp)))
    else:
        _check(_load().tfmm_tune_accuracy(_ptr(nodes, _dp), nodes.shape[0], _ptr(tets, _i32p), tets.shape[0],
                                          C.byref(prm), _ptr(M, _dp), float(tol), int(n_sample), int(seed),
                                          _ptr(pl, _i32p), pl.size, _ptr(tl, _dp), tl.size, C.byref(res),
                                          _ptr(table, _dp)))
    return dict(p=res.p, theta=res.theta, err=res.err, ms=res.ms, met=bool(res.met), n_tried=res.n_tried,
                table=table)


def tfmm_plan_store_near(plan, on=True, stream=None):
    """Assemble (on) or free (off) the plan's stored near-field operator; the
    plan's evaluations then apply it instead of integrating the near pairs.
    Synchronises `stream` (default: torch's current stream)."""
    import torch
    _check(_load().tfmm_plan_store_near(plan.handle, 1 if on else 0,
                                        _stream_handle(stream, torch.device("cuda", plan.device))))
    plan.params["near_stored"] = bool(on)


def tfmm_plan_destroy(plan):
    if plan._h is not None:
        _check(_load().tfmm_plan_destroy(plan._h))
        plan._h = None


def tfmm_simplex_rule(degree):
    """[npts, 4] rows (lambda1, lambda2, lambda3, weight) of the P2M quadrature."""
    n = C.c_int32()
    _check(_load().tfmm_simplex_rule(int(degree), None, C.byref(n)))
    out = np.zeros((n.value, 4))
    _check(_load().tfmm_simplex_rule(int(degree), _ptr(out, _dp), C.byref(n)))
    return out


def tfmm_set_timing(plan, on=True):
    _check(_load().tfmm_set_timing(plan.handle, 1 if on else 0))


def tfmm_kernel_times(plan):
    """{kernel: (average ms per evaluation, number of evaluations timed)} of the timed evaluations."""
    ms = np.zeros(len(KERNEL_NAMES))
    n = np.zeros(len(KERNEL_NAMES), dtype=np.int64)
    _check(_load().tfmm_kernel_times(plan.handle, _ptr(ms, _dp), _ptr(n, _i64p)))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_NAMES)}
