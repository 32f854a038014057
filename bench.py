#!/usr/bin/env python3
"""Benchmark: FMM potential evaluations per second on one MI355X.

A step is one tfmm_evaluate of the whole hot path (P2M, M2M, M2L, L2L, L2P,
P2P) for the magnetisation fields of the workload, with the plan built and M
resident on the device before the timed region.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cube40]

The accuracy of the timed configuration is measured against the FP64 direct
sum of exact tet integrals (GPU, all targets) outside the timed region.
The CPU baseline is the oracle FMM on a bounded sample of targets on the
host's cores (the oracle is test infrastructure; only this leg calls it).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work of the near field (flops; FMA = 2; elementary functions
# priced at the FP64 instruction counts of their ROCm device implementations
# on gfx950: divide 11, sqrt 14, log 76, atan 35, atan2 44).
#  - per pair, as the exact pair integral is written (the oracle's
#    orc_tet_potential on an operation-counting scalar, mean over every pair of
#    the jittered 8^3 cube; oracle/opcount.py): each tet's 4 faces and 12
#    face-edges are evaluated on their own;
#  - per mesh entity, as the near field is regrouped over the shared nodes,
#    edges and faces of a source chunk (the form the GPU evaluates):
#    node: |x - v| (8 + sqrt); edge: the two end projections, the squared
#    distance to the line, ln of a ratio (divide + log) and the quadratic
#    field weight (67 + 11 + 76); face: the height and the solid angle's
#    numerator and denominator, atan2, the affine field weight (48 + 44).
P2P_PAIR_FLOPS = 5094
P2P_NODE_FLOPS = 22
P2P_EDGE_FLOPS = 154
P2P_FACE_FLOPS = 92
P2P_FIELD_FLOPS = 24  # each further field: the 12 per-pair coefficients dotted with nodal M (12 FMA)
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
METRIC = "potential evals/s at \u22641e-5 rel-L2 vs FP64 direct: plain FP64 FMM vs mixed/batched"

WORKLOADS = {
    # unit cube, 40^3 cells x 6 Kuhn tets, +-0.15h jitter, unit nodal M, p=8, leaf 64, FP64
    "cube40": dict(n=40, p=8, leaf=64, theta=0.5, F=1),
    # unit cube, 8^3 x 6 tets, p=6, leaf 32
    "cube8": dict(n=8, p=6, leaf=32, theta=0.5, F=1),
}


_T0 = time.perf_counter()


def _say(*a):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s]", *a, file=sys.stderr, flush=True)


def m2l_terms(p):
    """Multiply-adds of one translation as computed: the harmonic reduction
    keeps the indices with z-component <= 1 on both sides ((2d+1) of degree d),
    |n| >= 1, |m| <= p - 1, |n| + |m| <= p (1284 at p = 8)."""
    return sum((2 * dm + 1) * (2 * dn + 1) for dm in range(p) for dn in range(1, p - dm + 1))


def near_flops(st, F):
    """Algorithmic flops of one evaluation's near field: over the shared
    entities for one field (the form evaluated then), per pair otherwise;
    and the per-pair count for comparison."""
    per_pair = st["n_p2p_pairs"] * (P2P_PAIR_FLOPS + (F - 1) * P2P_FIELD_FLOPS)
    if F == 1 and st["p2p_edge_evals"] > 0:
        ent = (st["p2p_node_evals"] * P2P_NODE_FLOPS + st["p2p_edge_evals"] * P2P_EDGE_FLOPS
               + st["p2p_face_evals"] * P2P_FACE_FLOPS)
        return ent, per_pair
    return per_pair, per_pair


def path_roofline(st, p, F, ms_per_step, n_targets):
    """Whole-path bound: per phase the time its algorithmic work takes at the
    peak of the unit that bounds it (FP64 vector for the near field, P2M, the
    shifts and L2P; FP64 matrix cores for M2L), summed and divided by the
    measured time per evaluation.  The compulsory HBM traffic (M, the mesh, u:
    ~150 B per target) is far below any of these and is left out."""
    nc = (p + 1) * (p + 2) * (p + 3) // 6
    mi = [(a, b, d - a - b) for d in range(p + 1) for a in range(d, -1, -1) for b in range(d - a, -1, -1)]
    shift_terms = 3 * sum(n[0] + 1 for n in mi)  # one axis pass ~ sum (n_ax + 1) terms, three passes
    flops = {
        "p2p": near_flops(st, F)[0],
        "m2l": st["n_m2l"] * F * 2 * m2l_terms(p),
        "p2m": st["n_tets"] * F * 24 * nc,
        "m2m_l2l": 2 * st["n_cells"] * F * 2 * shift_terms,
        "l2p": n_targets * F * 2 * nc,
    }
    t = {k: v / (FP64_PEAK_TFLOPS * 1e12) * 1e3 for k, v in flops.items()}
    return {"phase_bound_ms": {k: round(v, 4) for k, v in t.items()}, "bound_ms": round(sum(t.values()), 4),
            "frac": round(sum(t.values()) / ms_per_step, 4),
            "note": "sum over phases of algorithmic flops / FP64 peak (78.6 TFLOP/s vector and matrix)"}


def kernel_source_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_1606_00247_amd", "csrc", "kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_cube40.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernels_sha256") != kernel_source_hash() or kernel not in t.get("bytes_per_launch", {}):
        return None
    return t["bytes_per_launch"][kernel]


def measured_counters(kernel):
    """Hardware utilisation of `kernel` from the committed rocprofv3 counter
    summary (FP64 VALU lane operations per second against the 39.3 T lane-op/s
    of the FP64 pipes, VALU issue), or None when the kernels changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_cube40.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernels_sha256") != kernel_source_hash():
        return None
    return t.get("counters", {}).get(kernel)


def kernel_breakdown(T, torch, plan, M, u, steps):
    """Per-phase times (HIP event pairs on the evaluation stream) from separate
    evaluations with timing on; the phases then run one after another, so the
    times are not shared with the concurrent near field of the timed steps."""
    torch.cuda.synchronize()
    T.tfmm_set_timing(plan, True)
    for _ in range(steps):
        T.tfmm_evaluate(plan, M, u)
    torch.cuda.synchronize()
    kt = T.tfmm_kernel_times(plan)
    T.tfmm_set_timing(plan, False)
    return kt


def ragged_batch(T, torch, steps):
    """32 jittered cubes with 2k-200k tets (log-uniform), one field each, p=8,
    leaf 64, theta 0.5, FP64: one eager evaluation per mesh, the per-mesh
    plans as one captured graph (4 branches), and the merged plan (every mesh
    in one launch per phase) as one graph, before and after schedule tuning;
    then the tuned merged graph with split-BF16 and FP32 translations and
    with the stored near field."""
    import meshgen
    ns = meshgen.ragged_sizes(32)
    meshes = [meshgen.box_mesh(int(n), seed=i) for i, n in enumerate(ns)]
    B = T.tfmm_batch_create(meshes, p=8, leaf_size=64, theta=0.5)
    M = [torch.from_numpy(meshgen.random_fields(m[0].shape[0], F=1, seed=1 + i)[0]).to("cuda:0")
         for i, m in enumerate(meshes)]
    u = [torch.empty(m[0].shape[0], dtype=torch.float64, device="cuda:0") for m in meshes]
    plans = [T.tfmm_batch_plan(B, i) for i in range(len(meshes))]
    merged = T.tfmm_batch_merged_plan(B)
    evals = sum(m[0].shape[0] for m in meshes)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # references first: the FP64 direct sum of every mesh
    uds = [T.tfmm_direct(p, m) for p, m in zip(plans, M)]
    torch.cuda.synchronize()

    def max_err():
        """Error of a fresh batch evaluation (new output tensors: a graph of
        its own) against the direct sums, max over meshes."""
        uf = T.tfmm_batch_evaluate(B, M)
        torch.cuda.synchronize()
        return max(float(torch.linalg.norm(x - ud) / torch.linalg.norm(ud)) for x, ud in zip(uf, uds))

    t_eager = timed(lambda: [T.tfmm_evaluate(p, m, x) for p, m, x in zip(plans, M, u)])
    T.tfmm_batch_set_merged(B, 0)
    t_graph = timed(lambda: T.tfmm_batch_evaluate(B, M, u))
    err_per_mesh = max_err()
    T.tfmm_batch_set_merged(B, 1)
    t_merged = timed(lambda: T.tfmm_batch_evaluate(B, M, u))
    T.tfmm_batch_autotune(B)
    t_tuned = timed(lambda: T.tfmm_batch_evaluate(B, M, u))
    err = max_err()
    # the same graph with mixed-precision translations, then with the stored near field
    forms = {}
    for name, prec, store in (("bf16x3", T.M2L_BF16X3, False), ("fp32", T.M2L_FP32, False),
                              ("fp32_near_stored", T.M2L_FP32, True)):
        T.tfmm_plan_set_m2l_precision(merged, prec)
        if store:
            T.tfmm_plan_store_near(merged)
        t = timed(lambda: T.tfmm_batch_evaluate(B, M, u))
        forms[name] = {"value": evals / t, "ms_per_step": t * 1e3, "rel_l2_vs_direct_max_over_meshes": max_err(),
                       "speedup_vs_fp64_graph": t_tuned / t}
    T.tfmm_batch_destroy(B)
    return {"meshes": len(meshes), "tets": int(sum(m[1].shape[0] for m in meshes)), "targets": int(evals),
            "value": evals / t_tuned, "unit": "evals/s", "ms_per_step": t_tuned * 1e3,
            "ms_eager_per_mesh_launches": t_eager * 1e3, "ms_graph_per_mesh_plans": t_graph * 1e3,
            "ms_graph_merged_plan": t_merged * 1e3, "ms_graph_merged_tuned": t_tuned * 1e3,
            "m2l": "fp64", "rel_l2_vs_direct_max_over_meshes": err,
            "rel_l2_vs_direct_max_over_meshes_per_mesh_plans": err_per_mesh, "forms": forms}


def _sampled_direct(T, torch, nodes, tets, M, idx):
    """FP64 direct sum (GPU) at the nodes idx for the fields M [F, n, 3]: a plan
    whose explicit targets are the sample."""
    P = T.tfmm_plan_create(nodes, tets, targets=nodes[idx], p=2, leaf_size=64, theta=0.5, device=0)
    ud = T.tfmm_direct(P, torch.from_numpy(np.ascontiguousarray(M)).to("cuda:0"))
    torch.cuda.synchronize()
    out = ud.cpu().numpy().reshape(M.shape[0], -1)
    del P
    return out


def _time_form(T, torch, plan, Md, steps):
    u = torch.empty((Md.shape[0], plan.n_targets), dtype=torch.float64, device="cuda:0")
    T.tfmm_evaluate(plan, Md, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        T.tfmm_evaluate(plan, Md, u)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kt = kernel_breakdown(T, torch, plan, Md, u, 1)
    return u, dt, {k: round(v[0], 4) for k, v in kt.items()}


def config_lines(T, torch, steps):
    """The other workloads of the benchmark family, each on its own mesh with
    its accuracy measured against the FP64 direct sum on seeded sampled
    targets (max over fields of the relative L2 error):
      film    512 x 512 x 4 cells x 6 tets (6.29M tets, 1.32M targets),
              unjittered, vortex field, FP32 M2L, theta 0.4; also with the
              stored near field
      cube64  64^3 cells x 6 tets (1.57M tets), 64 random unit fields in one
              evaluation, split-BF16 (x3) M2L, theta 0.45; also with the
              stored near field
      sphere  radius 1 on a jittered 96^3 grid (~2.78M tets), uniform
              M = (0, 0, 1), FP64, theta 0.5
    Plans are built and their schedules autotuned outside the timed region."""
    import meshgen
    lines = {}

    def run(name, nodes, tets, M, theta, prec, sample, store, desc, surrogate=False):
        _say("configuration", name)
        t0 = time.perf_counter()
        P = T.tfmm_plan_create(nodes, tets, p=8, leaf_size=64, theta=theta, m2l_precision=prec, device=0)
        T.tfmm_plan_autotune(P)
        setup = time.perf_counter() - t0
        Md = torch.from_numpy(np.ascontiguousarray(M)).to("cuda:0")
        idx = np.sort(np.random.default_rng(11).choice(nodes.shape[0], sample, replace=False))
        ud = _sampled_direct(T, torch, nodes, tets, M, idx)
        forms = [("", False)] + ([("_near_stored", True)] if store else [])
        if surrogate:
            # the learned near-field surrogate (3 x 128 hidden) for the pairs 2-6
            # tet diameters apart, trained on the plan's own band pairs, and
            # the two controls on the same pairs
            _say("training the surrogate")
            t1 = time.perf_counter()
            loss = T.tfmm_surrogate_train(P, hidden=128, steps=6000, batch=8192, lr=2e-3, seed=3)
            t_train = time.perf_counter() - t1
            forms += [("_surrogate_mlp128", T.SUR_MLP), ("_control_gauss27", T.SUR_GAUSS),
                      ("_control_quadrupole", T.SUR_QUAD)]
        for suffix, st in forms:
            _say("form", name + suffix)
            extra = {}
            if not isinstance(st, bool):
                T.tfmm_plan_set_surrogate(P, st)
                sn = T.tfmm_plan_stats(P)
                extra = {"surrogate": {T.SUR_MLP: "mlp 16-128-128-128-12, bf16 weights, fp32 accumulation",
                                       T.SUR_GAUSS: "27-point Gauss-Jacobi rule (degree 5)",
                                       T.SUR_QUAD: "quadrupole expansion of each tet"}[st],
                         "band_pairs": sn["n_band_pairs"], "near_pairs": sn["n_p2p_pairs"]}
                if st == T.SUR_MLP:
                    extra.update(train_s=t_train, train_loss=loss, train_steps=6000, train_batch=8192)
            elif st:
                t1 = time.perf_counter()
                T.tfmm_plan_store_near(P)
                sn = T.tfmm_plan_stats(P)
                extra = {"near_store_s": time.perf_counter() - t1, "near_bytes": sn["near_bytes"]}
            u, dt, kt = _time_form(T, torch, P, Md, steps)
            un = u.cpu().numpy()[:, idx]
            err = max(float(np.linalg.norm(un[f] - ud[f]) / np.linalg.norm(ud[f])) for f in range(M.shape[0]))
            lines[name + suffix] = dict(
                desc=desc, n_tets=int(tets.shape[0]), n_targets=int(nodes.shape[0]), fields=int(M.shape[0]),
                p=8, leaf=64, theta=theta, m2l={0: "fp64", 1: "fp32", 2: "bf16x3", 3: "bf16x6"}[prec],
                near_stored=st is True, value=nodes.shape[0] * M.shape[0] / dt, unit="evals/s", ms_per_step=dt * 1e3,
                rel_l2_vs_direct_max_over_fields=err, direct_sample=int(sample), setup_s=setup, kernel_ms=kt, **extra)
            del u
        del P, Md

    nodes, tets = meshgen.film_mesh()
    M = meshgen.vortex_field(nodes, (0.0, 0.0), 64.0, seed=1)[None]
    run("film_fp32", nodes, tets, M, 0.4, T.M2L_FP32, 512, True,
        "thin film 512x512x4 cells x 6 Kuhn tets, unjittered, vortex M (0.05 noise), FP32 M2L")
    del nodes, tets, M
    nodes, tets = meshgen.box_mesh(64, seed=0)
    M = meshgen.random_fields(nodes.shape[0], F=64, seed=1)
    run("cube64_fields64_bf16x3", nodes, tets, M, 0.45, T.M2L_BF16X3, 256, True,
        "unit cube 64^3 cells x 6 Kuhn tets, +-0.15h jitter, 64 random unit nodal fields, BF16x3 M2L")
    del nodes, tets, M
    nodes, tets = meshgen.sphere_mesh(96)
    M = meshgen.uniform_field(nodes.shape[0], (0.0, 0.0, 1.0))[None]
    run("sphere96_fp64", nodes, tets, M, 0.5, T.M2L_FP64, 512, False,
        "sphere r=1, jittered 96^3 Kuhn grid keeping tets with centroid inside, uniform M=(0,0,1), FP64",
        surrogate=True)
    return lines


def study_energy(T, torch, sizes=(10, 20, 40, 60, 80, 100), orders=(3, 4, 5, 6), theta=0.5, direct_max=40):
    """Stray-field energy of the uniformly magnetised unit cube (M = e_z, the
    paper's Sec. 4.1 box; exact E / (mu0 Ms^2) = 1/6) against mesh size and
    expansion order: E from the FMM potentials (P1 on every tet, leaf 64) and,
    up to direct_max^3 cells, from the FP64 direct sum, which separates the
    discretisation error (direct - 1/6) from the FMM's (fmm - direct)."""
    import meshgen
    rows = []
    exact = 1.0 / 6.0
    for n in sizes:
        nodes, tets = meshgen.box_mesh(n, seed=0)
        M = torch.from_numpy(meshgen.uniform_field(nodes.shape[0], (0.0, 0.0, 1.0))).to("cuda:0")
        e_dir = None
        for p in orders:
            t0 = time.perf_counter()
            P = T.tfmm_plan_create(nodes, tets, p=p, leaf_size=64, theta=theta, device=0)
            setup = time.perf_counter() - t0
            u = T.tfmm_evaluate(P, M)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            T.tfmm_evaluate(P, M, u)
            torch.cuda.synchronize()
            t_eval = time.perf_counter() - t1
            E = T.tfmm_demag_energy(P, M, u)
            if e_dir is None and n <= direct_max:
                ud = T.tfmm_direct(P, M)
                e_dir = T.tfmm_demag_energy(P, M, ud)
                del ud
            rows.append({"cells": n, "vertices": int(nodes.shape[0]), "tets": int(tets.shape[0]), "p": p,
                         "theta": theta, "E": E, "E_minus_exact": E - exact,
                         "E_direct_minus_exact": None if e_dir is None else e_dir - exact,
                         "E_fmm_minus_direct": None if e_dir is None else E - e_dir,
                         "ms_per_eval": t_eval * 1e3, "setup_s": setup})
            print(json.dumps({"energy_row": rows[-1]}), file=sys.stderr, flush=True)
            del P, u
        del M
    return {"study": "energy", "exact": exact, "units": "mu0 Ms^2 (unit cube, M = e_z)",
            "paper_context": "paper Sec. 4.1: Delta E ~ 1e-3 (order 4) and ~3e-4 (order 6) at > 1M vertices; the "
                             "paper's order O keeps O(O+1)(O+2)/6 terms, i.e. |n| <= O - 1 here",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube40", choices=sorted(WORKLOADS))
    ap.add_argument("--theta", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=512)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (calibrates HBM byte counters in a profile)")
    ap.add_argument("--variant-steps", type=int, default=5)
    ap.add_argument("--study", choices=("energy",), default=None,
                    help="run a study instead of the benchmark and print its JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                          "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)

    import torch

    import meshgen
    import paper_1606_00247_amd as T

    if args.study == "energy":
        print(json.dumps(study_energy(T, torch)), flush=True)
        return

    W = dict(WORKLOADS[args.workload])
    if args.theta is not None:
        W["theta"] = args.theta
    nodes, tets = meshgen.box_mesh(W["n"], jitter=0.15, seed=0)
    M = meshgen.random_fields(nodes.shape[0], F=W["F"], seed=1)
    dev = torch.device("cuda:0")
    Md = torch.from_numpy(M).to(dev)
    t0 = time.time()
    plan = T.tfmm_plan_create(nodes, tets, p=W["p"], leaf_size=W["leaf"], theta=W["theta"], device=0)
    # schedule (M2L keys per work item, P2P workgroup shape) picked by timing;
    # the arithmetic is the same for every choice
    T.tfmm_plan_autotune(plan)
    setup_s = time.time() - t0
    st = T.tfmm_plan_stats(plan)
    u = torch.empty((W["F"], nodes.shape[0]), dtype=torch.float64, device=dev)

    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # reference: FP64 direct sum over all targets (GPU), outside the timed region
    _say("plan built", f"{setup_s:.1f} s; direct sum")
    ud = T.tfmm_direct(plan, Md)
    torch.cuda.synchronize()
    _say("timed steps")

    for _ in range(args.warmup):
        T.tfmm_evaluate(plan, Md, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        T.tfmm_evaluate(plan, Md, u)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ktimes = kernel_breakdown(T, torch, plan, Md, u, args.steps)
    err = max(float(torch.linalg.norm(u[f] - ud[f]) / torch.linalg.norm(ud[f])) for f in range(W["F"]))

    evals = nodes.shape[0] * W["F"]
    value = evals / dt

    # roofline of the dominant kernel
    dom = max(("p2p", "m2l"), key=lambda k: ktimes[k][0])
    t_dom = ktimes[dom][0] * 1e-3
    if dom == "p2p":
        flops, flops_pair = near_flops(st, W["F"])
        bound = "alu"
    else:
        flops = flops_pair = st["n_m2l"] * W["F"] * 2 * m2l_terms(W["p"])
        bound = "mfma"
    achieved = flops / t_dom / 1e12
    roof = {"kernel": dom, "bound": bound, "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": measured_traffic(dom),
            "algorithmic_unit": ("(target, node/edge/face) evaluations over the shared entities of each source "
                                 f"chunk: {P2P_NODE_FLOPS}/{P2P_EDGE_FLOPS}/{P2P_FACE_FLOPS} flop"
                                 if dom == "p2p" else "translations x 2 x terms"),
            "launch_ms": round(t_dom * 1e3, 4)}
    if dom == "p2p":
        # the same work priced per (target, tet) pair at the op count of the
        # oracle's pair integral: each tet evaluated on its own, the sharing of
        # faces, edges and nodes between tets not credited as saved work
        ap = flops_pair / t_dom / 1e12
        roof["per_pair_opcount"] = {"flops_per_pair": P2P_PAIR_FLOPS, "achieved": round(ap, 3),
                                    "frac": round(ap / FP64_PEAK_TFLOPS, 4)}
        hw = measured_counters("p2p")
        if hw is not None:
            roof["hw_counters"] = hw
    # the second phase: M2L on the FP64 matrix cores (the phase time holds the
    # multipole reduction, the translations and the expansion of the reduced
    # locals)
    t_m2l = ktimes["m2l"][0] * 1e-3
    am = st["n_m2l"] * W["F"] * 2 * m2l_terms(W["p"]) / t_m2l / 1e12
    m2l_roof = {"kernel": "m2l", "bound": "mfma", "achieved": round(am, 3), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(am / FP64_PEAK_TFLOPS, 4), "traffic": measured_traffic("m2l"),
                "algorithmic_unit": f"translations x fields x 2 x {m2l_terms(W['p'])} multiply-adds of the "
                                    "harmonically reduced contraction",
                "launch_ms": round(t_m2l * 1e3, 4)}
    hw = measured_counters("m2l")
    if hw is not None:
        m2l_roof["hw_counters"] = hw

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: unit cube {W['n']}^3 cells x 6 Kuhn tets, +-0.15h jitter, "
                               f"random unit nodal M",
                   "n_tets": int(tets.shape[0]), "n_targets": int(nodes.shape[0]), "fields": W["F"],
                   "p": W["p"], "leaf": W["leaf"], "theta": W["theta"], "m2l": "fp64",
                   "schedule": {"autotuned": True, "m2l_packed": bool(st["m2l_packed"]),
                                "m2l_groups_per_item": st["m2l_groups_per_item"],
                                "m2l_keys_per_item": st["m2l_keys_per_item"], "p2p_wide": bool(st["p2p_wide"])}},
        "rel_l2_vs_direct": err,
        "setup_s": setup_s,
        "setup_includes": "plan build and schedule autotune",
        "kernel_ms": {k: round(v[0], 4) for k, v in ktimes.items()},
        "counts": {"n_p2p_pairs": st["n_p2p_pairs"], "n_m2l": st["n_m2l"], "n_cells": st["n_cells"],
                   "p2p_node_evals": st["p2p_node_evals"], "p2p_edge_evals": st["p2p_edge_evals"],
                   "p2p_face_evals": st["p2p_face_evals"]},
        "roofline": roof,
        "m2l_roofline": m2l_roof,
        "path_roofline": path_roofline(st, W["p"], W["F"], dt * 1e3, nodes.shape[0]),
    }

    if not args.no_variants:
        # the mixed-precision and field-batched forms on the same mesh
        variants = {}
        cases = [("m2l_fp32", T.M2L_FP32, 1, False), ("fields16_fp64", T.M2L_FP64, 16, False),
                 ("fields16_m2l_fp32", T.M2L_FP32, 16, False), ("fields16_m2l_bf16x3", T.M2L_BF16X3, 16, False),
                 ("near_stored", T.M2L_FP64, 1, True), ("near_stored_m2l_fp32", T.M2L_FP32, 1, True),
                 ("near_stored_fields16_m2l_fp32", T.M2L_FP32, 16, True)]
        for name, prec, F, stored in cases:
            _say("variant", name)
            if stored and "near_store" not in out:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                T.tfmm_plan_store_near(plan)
                t_store = time.perf_counter() - t1
                sn = T.tfmm_plan_stats(plan)
                out["near_store"] = {"assembly_s": t_store, "nnz": sn["near_nnz"], "bytes": sn["near_bytes"]}
            T.tfmm_plan_set_m2l_precision(plan, prec)
            Mv = torch.from_numpy(meshgen.random_fields(nodes.shape[0], F=F, seed=1)).to(dev)
            uv = torch.empty((F, nodes.shape[0]), dtype=torch.float64, device=dev)
            T.tfmm_evaluate(plan, Mv, uv)
            udv = T.tfmm_direct(plan, Mv) if F > 1 else ud
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.variant_steps):
                T.tfmm_evaluate(plan, Mv, uv)
            torch.cuda.synchronize()
            dv = (time.perf_counter() - t1) / args.variant_steps
            kv = kernel_breakdown(T, torch, plan, Mv, uv, 2)
            ev = max(float(torch.linalg.norm(uv[f] - udv[f]) / torch.linalg.norm(udv[f])) for f in range(F))
            variants[name] = {"value": nodes.shape[0] * F / dv, "unit": "evals/s", "ms_per_step": dv * 1e3,
                              "fields": F, "m2l": {T.M2L_FP64: "fp64", T.M2L_FP32: "fp32", T.M2L_BF16X3: "bf16x3",
                                                   T.M2L_BF16X6: "bf16x6"}[prec],
                              "rel_l2_vs_direct_max_over_fields": ev,
                              "speedup_vs_plain": (nodes.shape[0] * F / dv) / value,
                              "kernel_ms": {k: round(v[0], 4) for k, v in kv.items()}}
            if stored:
                # the near field is a sparse product: HBM bound; algorithmic bytes = the
                # coefficient blocks and column lists once, M gathered once per field, u
                # read and written once per field
                nb = out["near_store"]["bytes"] + F * nodes.shape[0] * (24 + 16)
                gbs = nb / (kv["p2p"][0] * 1e-3) / 1e9
                variants[name]["near_roofline"] = {"kernel": "near_apply", "bound": "hbm", "achieved": round(gbs, 1),
                                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                                   "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes": nb}
            del Mv, uv, udv
        T.tfmm_plan_store_near(plan, False)
        T.tfmm_plan_set_m2l_precision(plan, T.M2L_FP64)
        # (p, theta) picked for the 1e-5 target by the tuner, then checked on all targets
        _say("variant tuned (p, theta)")
        t1 = time.perf_counter()
        tr = T.tfmm_tune_accuracy(nodes, tets, 1e-5, M=M[0], leaf_size=W["leaf"], n_sample=512, seed=3,
                                  p_list=(7, 8, 9), theta_list=(0.45, 0.5, 0.55))
        t_tune = time.perf_counter() - t1
        if tr["met"]:
            tp = T.tfmm_plan_create(nodes, tets, p=tr["p"], leaf_size=W["leaf"], theta=tr["theta"], device=0)
            T.tfmm_plan_autotune(tp)
            for name, prec, F, stored in (("tuned_tol1e-5", T.M2L_FP64, 1, False),
                                          ("tuned_tol1e-5_near_stored_fields16_m2l_fp32", T.M2L_FP32, 16, True)):
                T.tfmm_plan_set_m2l_precision(tp, prec)
                if stored:
                    T.tfmm_plan_store_near(tp)
                Mv = torch.from_numpy(meshgen.random_fields(nodes.shape[0], F=F, seed=1)).to(dev)
                uv = torch.empty((F, nodes.shape[0]), dtype=torch.float64, device=dev)
                T.tfmm_evaluate(tp, Mv, uv)
                udv = T.tfmm_direct(tp, Mv) if F > 1 else ud
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                for _ in range(args.variant_steps):
                    T.tfmm_evaluate(tp, Mv, uv)
                torch.cuda.synchronize()
                dv = (time.perf_counter() - t1) / args.variant_steps
                kv = kernel_breakdown(T, torch, tp, Mv, uv, 2)
                ev = max(float(torch.linalg.norm(uv[f] - udv[f]) / torch.linalg.norm(udv[f])) for f in range(F))
                variants[name] = {"value": nodes.shape[0] * F / dv, "unit": "evals/s", "ms_per_step": dv * 1e3,
                                  "fields": F, "p": tr["p"], "theta": tr["theta"], "tune_s": t_tune,
                                  "tune_sampled_err": tr["err"], "rel_l2_vs_direct_max_over_fields": ev,
                                  "m2l": "fp32" if prec == T.M2L_FP32 else "fp64", "near_stored": stored,
                                  "speedup_vs_plain": (nodes.shape[0] * F / dv) / value,
                                  "kernel_ms": {k: round(v[0], 4) for k, v in kv.items()}}
                del Mv, uv, udv
            del tp
        else:
            variants["tuned_tol1e-5"] = {"met": False, "tune_s": t_tune, "closest": [tr["p"], tr["theta"], tr["err"]]}
        # per-level orders for the same target on a p = 9, theta = 0.5 plan
        _say("variant tuned level orders")
        t1 = time.perf_counter()
        lp = T.tfmm_plan_create(nodes, tets, p=9, leaf_size=W["leaf"], theta=W["theta"], device=0)
        T.tfmm_plan_autotune(lp)
        lr = T.tfmm_tune_level_orders(lp, M[0], 1e-5, n_sample=512, seed=3)
        t_lt = time.perf_counter() - t1
        if lr["met"]:
            u_l, d_l, k_l = _time_form(T, torch, lp, Md, args.variant_steps)
            e_l = float(torch.linalg.norm(u_l[0] - ud[0]) / torch.linalg.norm(ud[0]))
            variants["tuned_levels_tol1e-5"] = {
                "value": nodes.shape[0] / d_l, "unit": "evals/s", "ms_per_step": d_l * 1e3, "fields": 1,
                "p_max": 9, "theta": W["theta"], "level_orders": lr["orders"][:T.tfmm_plan_stats(lp)["depth"] + 1],
                "tune_s": t_lt, "tune_sampled_err": lr["err"], "rel_l2_vs_direct_max_over_fields": e_l, "m2l": "fp64",
                "speedup_vs_plain": (nodes.shape[0] / d_l) / value, "kernel_ms": k_l}
            del u_l
        else:
            variants["tuned_levels_tol1e-5"] = {"met": False, "tune_s": t_lt}
        del lp
        _say("variant ragged batch")
        variants["ragged32"] = ragged_batch(T, torch, args.variant_steps)
        _say("variant point dipoles")
        # point-dipole cloud on the same nodes (moments M_i V_i, V_i the lumped volume)
        md = torch.from_numpy(M[0] * meshgen.lumped_volumes(nodes, tets)[:, None]).to(dev)
        pd = T.tfmm_plan_create_points(nodes, p=W["p"], leaf_size=W["leaf"], theta=0.5, device=0)
        udd = T.tfmm_direct(pd, md)
        torch.cuda.synchronize()
        del pd
        for th in (0.5, 0.4):
            pd = T.tfmm_plan_create_points(nodes, p=W["p"], leaf_size=W["leaf"], theta=th, device=0)
            uv = torch.empty(nodes.shape[0], dtype=torch.float64, device=dev)
            T.tfmm_evaluate(pd, md, uv)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.variant_steps):
                T.tfmm_evaluate(pd, md, uv)
            torch.cuda.synchronize()
            dv = (time.perf_counter() - t1) / args.variant_steps
            kv = kernel_breakdown(T, torch, pd, md, uv, 2)
            variants[f"dipoles_theta{th}"] = {
                "value": nodes.shape[0] / dv, "unit": "evals/s", "ms_per_step": dv * 1e3, "sources": "point dipoles",
                "p": W["p"], "theta": th, "m2l": "fp64",
                "rel_l2_vs_direct": float(torch.linalg.norm(uv - udd) / torch.linalg.norm(udd)),
                "kernel_ms": {k: round(v[0], 4) for k, v in kv.items()}}
            del pd, uv
        out["variants"] = variants
        out["configs"] = config_lines(T, torch, max(2, args.variant_steps // 2))
        _say("configurations done")

    if not args.no_cpu_baseline:
        _say("cpu baseline (oracle)")
        import oracle
        ncores = oracle.num_threads()
        O = oracle.FMM(nodes, tets, W["p"], W["leaf"], W["theta"])
        rng = np.random.default_rng(2024)
        sample = np.sort(rng.choice(nodes.shape[0], args.cpu_sample, replace=False))
        t1 = time.perf_counter()
        O.evaluate_sample(M, sample[:1])  # upward pass + one target
        t_up = time.perf_counter() - t1
        t1 = time.perf_counter()
        us = O.evaluate_sample(M, sample)
        t_s = time.perf_counter() - t1
        per_target = max(t_s - t_up, 0.0) / len(sample)
        t_full = t_up + per_target * nodes.shape[0]
        ucheck = float(np.linalg.norm(us - u[:, sample].cpu().numpy()) / np.linalg.norm(us))
        # the same on one core (a smaller sample)
        oracle.set_num_threads(1)
        t1 = time.perf_counter()
        O.evaluate_sample(M, sample[:1])
        t_up1 = time.perf_counter() - t1
        t1 = time.perf_counter()
        O.evaluate_sample(M, sample[:64])
        per1 = max(time.perf_counter() - t1 - t_up1, 0.0) / 64
        oracle.set_num_threads(ncores)
        t_full1 = t_up1 + per1 * nodes.shape[0]
        # the oracle's direct sum on the 8^3 cube (3,072 tets, all 729 nodes)
        n8, t8 = meshgen.box_mesh(8, seed=0)
        M8 = meshgen.random_fields(n8.shape[0], F=1, seed=1)[0]
        t1 = time.perf_counter()
        oracle.direct(n8, t8, M8)
        t_d8 = time.perf_counter() - t1
        # the oracle's direct sum at 32 of the benchmark's own targets, beside
        # the GPU direct sum there
        sd = sample[:32]
        t1 = time.perf_counter()
        udc = oracle.direct(nodes, tets, M, targets=nodes[sd])
        t_dc = time.perf_counter() - t1
        udg = ud.cpu().numpy()[:, sd]
        dcheck = float(np.linalg.norm(udg - udc) / np.linalg.norm(udc))
        out["cpu_baseline"] = {
            "value": evals / t_full, "unit": "evals/s", "cores": ncores, "kind": "oracle",
            "sample": f"oracle FMM on {len(sample)} seeded targets of {nodes.shape[0]} (full upward pass, "
                      f"{t_up:.1f}s; downward+near per target {per_target * 1e3:.2f} ms), extrapolated to all "
                      f"targets: {t_full:.1f}s per evaluation",
            "gpu_vs_oracle_rel_l2_on_sample": ucheck,
            "direct_cube8": {"value": n8.shape[0] / t_d8, "unit": "evals/s", "cores": ncores,
                             "sample": f"oracle direct sum on the 8^3 cube (3,072 tets, all {n8.shape[0]} nodes): "
                                       f"{t_d8:.2f}s"},
            "direct_sample": {"value": len(sd) * W["F"] / t_dc, "unit": "evals/s", "cores": ncores,
                              "sample": f"oracle direct sum at {len(sd)} seeded targets of the benchmark mesh "
                                        f"({tets.shape[0]} tets): {t_dc:.1f}s",
                              "gpu_direct_vs_oracle_direct_rel_l2": dcheck},
            "single_core": {"value": evals / t_full1, "cores": 1,
                            "sample": f"64 targets (upward pass {t_up1:.1f}s, {per1 * 1e3:.2f} ms per target), "
                                      f"extrapolated: {t_full1:.1f}s per evaluation"},
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
