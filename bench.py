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

# Algorithmic work per unit ("Measurement").
# P2P: flops of the pair formula (FMA = 2) per (target, tet) pair and field-independent part,
# plus the elementary functions costed at the FP64 instruction counts of their ROCm device
# implementations in this build (log 76, atan2 44, sqrt 14, divide 11).
P2P_ARITH_FLOPS = 410
P2P_FIELD_FLOPS = 53
P2P_TRANS_FLOPS = 6 * 76 + 4 * 44 + 4 * 14 + 6 * 11
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
METRIC = "potential evals/s at \u22641e-5 rel-L2 vs FP64 direct: plain FP64 FMM vs mixed/batched"

WORKLOADS = {
    # unit cube, 40^3 cells x 6 Kuhn tets, +-0.15h jitter, unit nodal M, p=8, leaf 64, FP64
    "cube40": dict(n=40, p=8, leaf=64, theta=0.5, F=1),
    # unit cube, 8^3 x 6 tets, p=6, leaf 32
    "cube8": dict(n=8, p=6, leaf=32, theta=0.5, F=1),
}


def m2l_terms(p):
    """Multiply-adds of one translation as computed: the harmonic reduction
    keeps the indices with z-component <= 1 on both sides ((2d+1) of degree d),
    |n| >= 1, |m| <= p - 1, |n| + |m| <= p (1284 at p = 8)."""
    return sum((2 * dm + 1) * (2 * dn + 1) for dm in range(p) for dn in range(1, p - dm + 1))


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
        "p2p": st["n_p2p_pairs"] * (P2P_ARITH_FLOPS + P2P_TRANS_FLOPS + F * P2P_FIELD_FLOPS),
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
    leaf 64, theta 0.5, FP64: one eager evaluation per mesh vs the batch's
    captured graph, before and after schedule tuning; then the tuned graph
    with split-BF16 and FP32 translations and with the stored near field."""
    import meshgen
    ns = meshgen.ragged_sizes(32)
    meshes = [meshgen.box_mesh(int(n), seed=i) for i, n in enumerate(ns)]
    B = T.tfmm_batch_create(meshes, p=8, leaf_size=64, theta=0.5)
    M = [torch.from_numpy(meshgen.random_fields(m[0].shape[0], F=1, seed=1 + i)[0]).to("cuda:0")
         for i, m in enumerate(meshes)]
    u = [torch.empty(m[0].shape[0], dtype=torch.float64, device="cuda:0") for m in meshes]
    plans = [T.tfmm_batch_plan(B, i) for i in range(len(meshes))]
    evals = sum(m[0].shape[0] for m in meshes)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_eager = timed(lambda: [T.tfmm_evaluate(p, m, x) for p, m, x in zip(plans, M, u)])
    t_graph = timed(lambda: T.tfmm_batch_evaluate(B, M, u))
    T.tfmm_batch_autotune(B)
    t_tuned = timed(lambda: T.tfmm_batch_evaluate(B, M, u))
    uds = [T.tfmm_direct(p, m) for p, m in zip(plans, M)]

    def max_err():
        torch.cuda.synchronize()
        return max(float(torch.linalg.norm(x - ud) / torch.linalg.norm(ud)) for x, ud in zip(u, uds))

    err = max_err()
    # the same graph with mixed-precision translations, then with the stored near field
    forms = {}
    for name, prec, store in (("bf16x3", T.M2L_BF16X3, False), ("fp32", T.M2L_FP32, False),
                              ("fp32_near_stored", T.M2L_FP32, True)):
        for pl in plans:
            T.tfmm_plan_set_m2l_precision(pl, prec)
            if store:
                T.tfmm_plan_store_near(pl)
        t = timed(lambda: T.tfmm_batch_evaluate(B, M, u))
        forms[name] = {"value": evals / t, "ms_per_step": t * 1e3, "rel_l2_vs_direct_max_over_meshes": max_err(),
                       "speedup_vs_fp64_graph": t_tuned / t}
    T.tfmm_batch_destroy(B)
    return {"meshes": len(meshes), "tets": int(sum(m[1].shape[0] for m in meshes)), "targets": int(evals),
            "value": evals / t_tuned, "unit": "evals/s", "ms_per_step": t_tuned * 1e3,
            "ms_eager_per_mesh_launches": t_eager * 1e3, "ms_graph": t_graph * 1e3, "ms_graph_tuned": t_tuned * 1e3,
            "m2l": "fp64", "rel_l2_vs_direct_max_over_meshes": err, "forms": forms}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)

    import torch

    import meshgen
    import paper_1606_00247_amd as T

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
    ud = T.tfmm_direct(plan, Md)
    torch.cuda.synchronize()

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
    if dom == "p2p":
        flops = st["n_p2p_pairs"] * (P2P_ARITH_FLOPS + P2P_TRANS_FLOPS + W["F"] * P2P_FIELD_FLOPS)
        bound = "alu"
    else:
        flops = st["n_m2l"] * W["F"] * 2 * m2l_terms(W["p"])
        bound = "mfma"
    t_dom = ktimes[dom][0] * 1e-3
    achieved = flops / t_dom / 1e12
    roof = {"kernel": dom, "bound": bound, "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": measured_traffic(dom)}

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
                   "schedule": {"autotuned": True, "m2l_keys_per_item": st["m2l_keys_per_item"],
                                "p2p_wide": bool(st["p2p_wide"])}},
        "rel_l2_vs_direct": err,
        "setup_s": setup_s,
        "setup_includes": "plan build and schedule autotune",
        "kernel_ms": {k: round(v[0], 4) for k, v in ktimes.items()},
        "counts": {"n_p2p_pairs": st["n_p2p_pairs"], "n_m2l": st["n_m2l"], "n_cells": st["n_cells"]},
        "roofline": roof,
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
        t1 = time.perf_counter()
        tr = T.tfmm_tune_accuracy(nodes, tets, 1e-5, M=M[0], leaf_size=W["leaf"], n_sample=512, seed=3,
                                  p_list=(7, 8), theta_list=(0.45, 0.5, 0.55))
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
        variants["ragged32"] = ragged_batch(T, torch, args.variant_steps)
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

    if not args.no_cpu_baseline:
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
        out["cpu_baseline"] = {
            "value": evals / t_full, "unit": "evals/s", "cores": ncores, "kind": "oracle",
            "sample": f"oracle FMM on {len(sample)} seeded targets of {nodes.shape[0]} (full upward pass, "
                      f"{t_up:.1f}s; downward+near per target {per_target * 1e3:.2f} ms), extrapolated to all "
                      f"targets: {t_full:.1f}s per evaluation",
            "gpu_vs_oracle_rel_l2_on_sample": ucheck,
            "single_core": {"value": evals / t_full1, "cores": 1,
                            "sample": f"64 targets (upward pass {t_up1:.1f}s, {per1 * 1e3:.2f} ms per target), "
                                      f"extrapolated: {t_full1:.1f}s per evaluation"},
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
