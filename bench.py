#!/usr/bin/env python3
"""Benchmark of the IFGF apply on one MI355X.

Workload (default): unit-diameter cubed sphere, 6 x 256^2 = 393,216 points,
32 wavelengths (k = 64 pi), eta = k, depth 7 (finest boxes 0.5 wavelength),
one complex density N(0,1) + i N(0,1).  A step is one full apply (gather,
near field, leaf factors, coefficients, upward pass, cousin targets) with
every input resident in device memory; the plan is built once before the
timed region and its build time is reported separately.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IFGF apply time (s) at N=393k 32λ sphere, rel.err≤1e-4; FP32/batched vs FP64"
PEAK_FP32_VECTOR_TFLOPS = 157.3     # MI355X published dense FP32 vector rate
PEAK_HBM_GBS = 8000.0

# Algorithmic work per unit (documented in the design notes).
def interp_flops(ps, pa):
    # complex coefficients x real Chebyshev basis: 2 FMAs per coefficient in
    # the innermost sum, then the theta and s sums, then one complex
    # multiply-accumulate with the centred factor or the propagation ratio
    return 4 * (ps * pa * pa + ps * pa + ps) + 8


LEAF_FLOPS = 48        # one analytic-factor evaluation W_c and its complex multiply-accumulate
NEAR_FLOPS = 40        # one kernel evaluation K(x, y) and its complex multiply-accumulate


def coeff_flops(ps, pa):
    P = ps * pa * pa
    return 4 * P * (ps + 2 * pa)   # three separable real-matrix passes on complex data


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# HBM bytes per launch of the upward-pass kernel, from hardware byte counters
# (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter reads for a
# device copy of known size).  The summary records the SHA-256 of the kernel
# sources it was taken with; when the sources have changed since, the figure
# no longer describes this kernel and is not reported.
TRAFFIC_SUMMARY = {
    "prop": os.path.join(ROOT, "profiles", "k_upairs_sphere32_hbm_traffic.md"),
    "prop_cone": os.path.join(ROOT, "profiles", "k_prop_ti_sphere32_hbm_traffic.md"),
}
KERNEL_OF_STAGE = {"prop": "k_upairs + k_upsum_coeffs (pair list) or k_prop (node formulation)",
                   "prop_cone": "k_prop_ti (cone-major, MFMA)",
                   "targets": "k_targets", "leaf": "k_leaf", "near": "k_near", "coeffs": "k_coeffs"}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2112_06316_amd", "csrc", f) for f in ("apply.hip", "common.h", "plan.hip")]


def pair_row_use(st):
    """Per level, the pair-list row stage's passes per row of 16 pairs and its
    lane use (pairs / (16 x passes)); empty without pair lists."""
    out = {}
    for d, rows in st.get("pair_rows", {}).items():
        passes = st["pair_row_cones"][d]
        if rows and passes:
            pairs = st["cousin_pairs"][d]
            out[d] = {"rows": rows, "passes_per_row": passes / rows, "lane_use": pairs / (16.0 * passes)}
    return out


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def config_tag(args):
    return f"{args.workload} p_s={args.p_s} p_ang={args.p_ang} ns0={args.ns0} nc0={args.nc0}"


def measured_traffic(tag, stage):
    if stage not in TRAFFIC_SUMMARY:
        return None
    try:
        with open(TRAFFIC_SUMMARY[stage]) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        if ln.startswith("- ") and ": " in ln:
            key, val = ln[2:].split(": ", 1)
            kv[key.strip().strip("`")] = val.strip().strip("`")
    if kv.get("source_sha256") != kernel_source_sha() or kv.get("config") != tag:
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measure_peaks(log):
    """Rates this GPU sustains for the instructions the kernels use (MFMA FP32
    chains, FP32 and FP64 FMA chains, a 1 GiB 16-byte-vector copy), from the
    probe library; None where it is not built."""
    import ctypes
    path = os.path.join(ROOT, "paper_2112_06316_amd", "libifgf_probe.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    lib.ifgf_probe_run.restype = ctypes.c_int
    lib.ifgf_probe_run.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    names = ["mfma_f32_tflops", "valu_f32_tflops", "valu_f64_tflops", "hbm_copy_gbs"]
    out = {}
    for i, name in enumerate(names):
        v = ctypes.c_double(0.0)
        st = lib.ifgf_probe_run(i, ctypes.byref(v))
        out[name] = v.value if st == 0 else None
    log(f"measured peaks: {out}")
    return out


PEAK_FP64_VECTOR_TFLOPS = 78.6     # MI355X published dense FP64 vector rate


def fp64_hi_entry(r, err, steps, n, D):
    """The FP64 apply at (P_s, P_ang) = (8, 8): time, error and the roofline of
    its dominant kernel (FP64 vector ALUs, 78.6 TFLOP/s)."""
    st, prof = r["stats"], r["prof"]
    P = 8 * 8 * 8
    fi = interp_flops(8, 8)
    work = {
        "prop": sum(st["prop_evals"].values()) * fi,
        "targets": sum(st["cousin_pairs"].values()) * fi,
        "near": st["near_pairs"] * NEAR_FLOPS,
        "leaf": (st["cones"][D] * P * (n / st["boxes"][D]) * LEAF_FLOPS + st["cones"][D] * coeff_flops(8, 8))
        if D >= 3 else 0,
    }
    stages = {}
    for name, (ms, cnt) in prof.items():
        e = {"ms_per_apply": ms / steps, "launches_per_apply": cnt / steps}
        if name in work and ms > 0:
            e["achieved_tflops"] = work[name] / (ms / steps * 1e-3) / 1e12
        stages[name] = e
    roof = None
    cand = [s_ for s_ in prof if s_ in work and prof[s_][0] > 0]
    if cand:
        dom = max(cand, key=lambda s_: prof[s_][0])
        ms_dom, cnt_dom = prof[dom]
        per_launch = work[dom] / (cnt_dom / steps)
        ach = per_launch / (ms_dom / cnt_dom * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP64_VECTOR_TFLOPS, "kernel": KERNEL_OF_STAGE.get(dom, dom), "stage": dom,
                "avg_launch_ms": ms_dom / cnt_dom, "launches_per_apply": cnt_dom / steps,
                "algorithmic_flops_per_launch": per_launch}
    return {"ms_per_step": r["wall"] * 1e3 / steps, "event_ms_median": r["ev_median"], "event_ms_min": r["ev_min"],
            "rel_err": err, "setting": "P=(8,8,8), cones (n_s0,n_C0)=(1,4), FP64 throughout",
            "plan_create_s": r["t_plan"], "stages": stages, "roofline": roof,
            "cones": st["cones"], "device_bytes": st["device_bytes"], "consistency_flags": r["flags"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere32")
    ap.add_argument("--fp64-steps", type=int, default=10)
    ap.add_argument("--targets", type=int, default=4096, help="sampled targets for the error and the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--p-s", type=int, default=4)
    ap.add_argument("--p-ang", type=int, default=6)
    ap.add_argument("--ns0", type=int, default=2)
    ap.add_argument("--nc0", type=int, default=4)
    ap.add_argument("--batched-rhs", type=int, default=64, help="RHS of the batched leg (0 = skip)")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--adjoint-steps", type=int, default=5)
    ap.add_argument("--ragged-steps", type=int, default=5, help="applies of the ragged 8-geometry batch (0 = skip)")
    ap.add_argument("--no-peak-probe", action="store_true", help="skip the measured-peak probes")
    ap.add_argument("--autotune-reps", type=int, default=3,
                    help="passes per candidate of the plan's formulation autotuner (0 = the built-in heuristic)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the FP32 leg, copy a buffer of this many MiB three times with a plain device copy "
                         "(the reference point that scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: only --gpus 1 is supported: this build runs on one GPU "
              f"(asked for {args.gpus}); the multi-GPU decomposition is a design note only.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2112_06316_amd import Plan, inputs

    dev = torch.device("cuda:0")
    wl = inputs.workload(args.workload)
    p, nr, w = inputs.build_surface(wl)
    n = len(p)
    k, eta, D = wl["k"], wl["eta"], wl["depth"]
    seed = inputs.config_seed(wl["config"])
    sigma = inputs.random_density(n, seed=seed)
    tg = inputs.sample_targets(n, args.targets, seed=seed + 100)
    sig_d = torch.from_numpy(sigma).to(dev)
    opts = dict(p_s=args.p_s, p_ang=args.p_ang, ns0=args.ns0, nc0=args.nc0, depth=D)
    log(f"workload {args.workload}: N={n} k={k:.4f} D={D} opts={opts}")

    def run(precision, steps, warmup, profile, o=None):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = Plan(p, nr, w, k, eta, precision=precision, **(o or opts))
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        log(f"{precision}: plan built in {t_plan:.3f} s")
        tune, t_tune = None, 0.0
        if args.autotune_reps > 0:   # measured formulation choice, kept in the plan (plan-time work)
            t0 = time.perf_counter()
            tune = plan.autotune(reps=args.autotune_reps)
            t_tune = time.perf_counter() - t0
            log(f"{precision}: autotuned in {t_tune:.3f} s: "
                f"{ {d: e['choice'] for d, e in tune['prop'].items()} } targets {tune['targets']}")
        u = torch.empty_like(sig_d)
        for _ in range(warmup):
            plan.apply(sig_d, out=u[:, None])
        torch.cuda.synchronize()
        # timed region: the applies alone, one event pair per apply on the
        # stream the library launches on (no per-kernel events)
        stream = torch.cuda.current_stream(dev)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e0, e1 in ev:
            e0.record(stream)
            plan.apply(sig_d, out=u[:, None])
            e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        ev_ms = sum(per)
        prof = {}
        if profile:
            # the same applies again with every kernel launch bracketed by
            # events (stage times and the dominant kernel's launch duration)
            plan.set_profiling(64 * steps)
            for _ in range(steps):
                plan.apply(sig_d, out=u[:, None])
            torch.cuda.synchronize()
            prof = plan.read_profile()
            plan.set_profiling(0)
        flags = plan.check()
        st = plan.stats()
        uh = u.cpu().numpy()
        med = per[len(per) // 2] if len(per) % 2 else 0.5 * (per[len(per) // 2 - 1] + per[len(per) // 2])
        log(f"{precision}: {steps} applies, wall {wall * 1e3 / steps:.3f} ms/apply, events median {med:.3f} "
            f"min {per[0]:.3f} ms")
        return dict(plan=plan, t_plan=t_plan, wall=wall, ev_ms=ev_ms, ev_median=med, ev_min=per[0], prof=prof,
                    stats=st, u=uh, flags=flags, tune=tune, t_tune=t_tune)

    r32 = run("fp32", args.steps, args.warmup, True)
    st = r32["stats"]
    if args.copy_probe_mib > 0:
        src = torch.ones((args.copy_probe_mib << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 x {args.copy_probe_mib} MiB device copy")
        del src, dst

    # ---- transposed apply (autograd backward) at the same workload --------------
    adj = None
    if args.adjoint_steps > 0:
        plan = r32["plan"]
        v = torch.empty_like(sig_d)
        plan.apply_adjoint(sig_d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.adjoint_steps):
            plan.apply_adjoint(sig_d)
        torch.cuda.synchronize()
        adj = {"ms_per_step": (time.perf_counter() - t0) * 1e3 / args.adjoint_steps, "conjugate": True}
        plan.set_profiling(64)   # one more transposed apply with its stages timed
        plan.apply_adjoint(sig_d)
        torch.cuda.synchronize()
        adj["stages"] = {k2: {"ms_per_apply": v2[0], "launches_per_apply": v2[1]}
                         for k2, v2 in plan.read_profile().items()}
        plan.set_profiling(0)
        log(f"adjoint: {adj['ms_per_step']:.3f} ms/apply, stages "
            f"{ {k2: round(v2['ms_per_apply'], 2) for k2, v2 in adj['stages'].items()} }")
        del v, plan
    r32.pop("plan")
    r64 = run("fp64", args.fp64_steps, 2, False) if args.fp64_steps > 0 else None
    if r64 is not None:
        r64.pop("plan")
    # the FP64 form at the order that reaches 1e-6: (P_s, P_ang) = (8, 8), cones (1, 4)
    hi_opts = dict(p_s=8, p_ang=8, ns0=1, nc0=4, depth=D)
    r64h = run("fp64", args.fp64_steps, 2, True, hi_opts) if args.fp64_steps > 0 else None
    if r64h is not None:
        r64h.pop("plan")

    # ---- oracle: error and CPU baseline on the sampled targets ----------------
    err32 = err64 = err64h = None
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import direct
        log(f"oracle: direct sum at {len(tg)} targets x {n} sources ({direct.num_threads()} threads)")
        t0 = time.perf_counter()
        ref = direct.apply_c(p, nr, w, k, eta, sigma, targets=tg)
        t_cpu = time.perf_counter() - t0
        log(f"oracle: {t_cpu:.2f} s")
        err32 = float(np.linalg.norm(r32["u"][tg] - ref) / np.linalg.norm(ref))
        if r64 is not None:
            err64 = float(np.linalg.norm(r64["u"][tg] - ref) / np.linalg.norm(ref))
        if r64h is not None:
            err64h = float(np.linalg.norm(r64h["u"][tg] - ref) / np.linalg.norm(ref))
        cpu = {
            "value": t_cpu * n / len(tg), "unit": "s", "cores": direct.num_threads(), "kind": "oracle",
            "sample": (f"FP64 direct sum (C/OpenMP) at {len(tg)} seeded targets x {n} sources = "
                       f"{len(tg) * n:.3e} kernel evaluations in {t_cpu:.2f} s, extrapolated x N/{len(tg)} "
                       f"to one full apply"),
        }

    # ---- algorithmic work per stage ---------------------------------------------
    ps, pa = args.p_s, args.p_ang
    P = ps * pa * pa
    fi = interp_flops(ps, pa)
    prop_evals = sum(st["prop_evals"].values())
    cousin = sum(st["cousin_pairs"].values())
    cone_lv = [d for d, m in st["prop_kernel"].items() if m == "cone"]
    node_lv = [d for d, m in st["prop_kernel"].items() if m in ("node", "pairs")]   # both time as "prop"
    leaf_cones = st["cones"][D] if D >= 3 else 0
    pts_per_leaf = n / st["boxes"][D]
    # leaf factors: every relevant leaf cone node against every source of its box
    # (exact count: sum over leaf boxes of cones(b) * P * npts(b); estimated with the mean)
    work = {
        "near": st["near_pairs"] * NEAR_FLOPS,
        "leaf": leaf_cones * P * pts_per_leaf * LEAF_FLOPS,
        "coeffs": leaf_cones * coeff_flops(ps, pa),
        "prop": sum(st["prop_evals"][d] for d in node_lv) * fi,
        "prop_cone": sum(st["prop_evals"][d] for d in cone_lv) * fi,
        "targets": cousin * fi,
    }
    F_bytes = {d: st["cones"][d] * P * 8 for d in st["cones"]}
    traffic = {
        "prop": sum(F_bytes[d] + F_bytes[d - 1] for d in node_lv),
        "prop_cone": sum(F_bytes[d] + F_bytes[d - 1] for d in cone_lv),
        "targets": sum(F_bytes.values()) + n * (24 + 8 + 4 + 16),
        "leaf": n * (24 + 24 + 8) + F_bytes.get(D, 0),
        "near": n * (24 + 24 + 8 + 8),
        "coeffs": 2 * F_bytes.get(D, 0),
    }
    prof = r32["prof"]
    if "coeffs" not in prof:   # one RHS: the finest level's transform runs inside the leaf kernel
        work["leaf"] += work.pop("coeffs")
        traffic["leaf"] += F_bytes.get(D, 0)
        traffic.pop("coeffs")
    stages = {}
    for name, (ms, cnt) in prof.items():
        entry = {"ms_per_apply": ms / args.steps, "launches_per_apply": cnt / args.steps}
        if name in work and ms > 0:
            entry["achieved_tflops"] = work[name] / (ms / args.steps * 1e-3) / 1e12
        if name in traffic and ms > 0:   # algorithmic bytes: inputs read once, outputs written once
            entry["algorithmic_gbs"] = traffic[name] / (ms / args.steps * 1e-3) / 1e9
        stages[name] = entry
    dom = max((s for s in prof if s in work), key=lambda s: prof[s][0])
    ms_dom, cnt_dom = prof[dom]
    avg_launch_s = ms_dom / cnt_dom * 1e-3
    per_launch_flops = work[dom] / (cnt_dom / args.steps)
    achieved = per_launch_flops / avg_launch_s / 1e12
    measured = measured_traffic(config_tag(args), dom)
    # the cone-major upward pass runs its contraction on FP32 MFMA (dense peak
    # 157.3 TFLOP/s); the other kernels on the FP32 vector ALUs (157.3 TFLOP/s)
    roofline = {
        "bound": "mfma" if dom == "prop_cone" else "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
        "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": measured,
        "kernel": KERNEL_OF_STAGE.get(dom, dom), "stage": dom,
        "avg_launch_ms": avg_launch_s * 1e3, "launches_per_apply": cnt_dom / args.steps,
        "algorithmic_flops_per_launch": per_launch_flops,
        "algorithmic_bytes_per_launch": traffic[dom] / (cnt_dom / args.steps),
    }

    # ---- batched right-hand sides (MFMA) -----------------------------------------
    batched = None
    if args.batched_rhs > 0:
        wb = inputs.workload("sphere16")
        pb, nb_, wb_ = inputs.build_surface(wb)
        Rb = args.batched_rhs
        Sb = inputs.plane_wave_densities(pb, wb["k"], Rb, seed=inputs.config_seed(wb["config"]))
        Sb_d = torch.from_numpy(Sb.astype(np.complex64)).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        planb = Plan(pb, nb_, wb_, wb["k"], wb["eta"], precision="fp32", max_rhs=Rb,
                     **dict(opts, depth=wb["depth"]))
        torch.cuda.synchronize()
        t_planb = time.perf_counter() - t0
        Ub = planb.apply(Sb_d)
        torch.cuda.synchronize()
        planb.set_profiling(64 * args.batched_steps)
        t0 = time.perf_counter()
        for _ in range(args.batched_steps):
            planb.apply(Sb_d, out=Ub)
        torch.cuda.synchronize()
        wall_b = time.perf_counter() - t0
        profb = planb.read_profile()
        planb.set_profiling(0)
        stb = planb.stats()
        Ubh = Ub.cpu().numpy()
        log(f"batched: {Rb} RHS, {wall_b * 1e3 / args.batched_steps:.2f} ms/apply")
        errb = None
        if not args.no_cpu_baseline:
            from oracle import direct
            tgb = inputs.sample_targets(len(pb), 512, seed=inputs.config_seed(wb["config"]) + 100)
            cols = [0, Rb // 2, Rb - 1]
            refb = direct.apply_c(pb, nb_, wb_, wb["k"], wb["eta"], Sb[:, cols], targets=tgb)
            errb = float(np.linalg.norm(Ubh[tgb][:, cols] - refb) / np.linalg.norm(refb))
        pe = sum(stb["prop_evals"].values())
        flops_prop = pe * Rb * 4 * P          # complex coefficients x real basis, per RHS
        ms_p, cnt_p = profb.get("prop", (0.0, 0))
        ach = flops_prop / (ms_p / args.batched_steps * 1e-3) / 1e12 if ms_p else None
        batched = {
            "workload": (f"sphere16: cubed sphere 6x{wb['n']}^2, N={len(pb)}, k=32pi, eta=k, D={wb['depth']}, "
                         f"{Rb} plane-wave RHS, FP32, MFMA contraction over RHS groups of 16"),
            "ms_per_step": wall_b * 1e3 / args.batched_steps, "ms_per_rhs": wall_b * 1e3 / args.batched_steps / Rb,
            "rel_err": errb, "plan_create_s": t_planb,
            "stages": {k2: {"ms_per_apply": v2[0] / args.batched_steps, "launches_per_apply": v2[1] / args.batched_steps}
                       for k2, v2 in profb.items()},
            "roofline_prop": {"bound": "mfma", "achieved": ach, "peak": 157.3, "unit": "TFLOP/s",
                              "frac": (ach / 157.3) if ach else None, "kernel": "k_prop_mfma_cone",
                              "algorithmic_flops_per_apply": flops_prop},
        }
        # the same workload one right-hand side at a time (the single-RHS
        # kernels), for the gain of the batched contraction per RHS
        plan1 = Plan(pb, nb_, wb_, wb["k"], wb["eta"], precision="fp32", **dict(opts, depth=wb["depth"]))
        s1 = Sb_d[:, 0].contiguous()
        u1 = torch.empty_like(s1)
        for _ in range(3):
            plan1.apply(s1, out=u1[:, None])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps1 = 20
        for _ in range(reps1):
            plan1.apply(s1, out=u1[:, None])
        torch.cuda.synchronize()
        ms1 = (time.perf_counter() - t0) * 1e3 / reps1
        batched["single_rhs_ms_per_apply"] = ms1
        batched["gain_per_rhs_vs_single"] = ms1 / batched["ms_per_rhs"]
        log(f"batched: single-RHS apply {ms1:.3f} ms, per-RHS gain {ms1 / batched['ms_per_rhs']:.2f}x")
        del planb, Ub, Sb_d, plan1

    # ---- ragged batch: 8 geometries in one launch vs 8 separate applies ----------
    ragged = None
    if args.ragged_steps > 0:
        from paper_2112_06316_amd import Batch
        geoms = inputs.ragged_batch()
        plans_r = [Plan(g["points"], g["normals"], g["weights"], g["k"], g["eta"], precision="fp32",
                        leaf_h_lambda=0.5, **dict(opts, depth=0)) for g in geoms]
        sig_r = [torch.from_numpy(inputs.random_density(g["n"], seed=g["seed"]).astype(np.complex64)).to(dev)
                 for g in geoms]
        out_r = [torch.empty_like(x) for x in sig_r]
        bat = Batch(plans_r)
        stream = torch.cuda.current_stream(dev)

        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        def separate():
            for pl, x, o in zip(plans_r, sig_r, out_r):
                pl.apply(x, out=o[:, None])

        ms_sep = timed(separate, args.ragged_steps)
        ms_bat = timed(lambda: bat.apply(sig_r, outs=out_r), args.ragged_steps)
        log(f"ragged: batch {ms_bat:.3f} ms, separate {ms_sep:.3f} ms")
        errs = None
        if not args.no_cpu_baseline:
            from oracle import direct
            errs = []
            for g, geo in enumerate(geoms):
                tgr = inputs.sample_targets(geo["n"], 256, seed=geo["seed"] + 100)
                sg = inputs.random_density(geo["n"], seed=geo["seed"])
                ref = direct.apply_c(geo["points"], geo["normals"], geo["weights"], geo["k"], geo["eta"], sg,
                                     targets=tgr)
                errs.append(float(np.linalg.norm(out_r[g].cpu().numpy()[tgr] - ref) / np.linalg.norm(ref)))
        ragged = {
            "workload": ("8 geometries, 6 x n_b^2 points, n_b = 32..128 (N = 6,144..98,304, 410,112 in all); "
                         "spheres (even b) and ellipsoids (0.5, 0.375, 0.25) (odd b); n_b/8 wavelengths across; "
                         "FP32, one density each"),
            "N": [g["n"] for g in geoms], "depth": [pl.stats()["depth"] for pl in plans_r],
            "ms_batch_one_launch": ms_bat, "ms_separate_applies": ms_sep, "speedup": ms_sep / ms_bat,
            "queue": bat.info(), "rel_err": errs, "rel_err_targets_per_geometry": 256,
            "consistency_flags": bat.check(),
        }
        del bat, plans_r, sig_r, out_r

    peaks = None if args.no_peak_probe else measure_peaks(log)
    if peaks:
        key = "mfma_f32_tflops" if roofline["bound"] == "mfma" else "valu_f32_tflops"
        if peaks.get(key):
            roofline["measured_peak"] = peaks[key]
            roofline["frac_of_measured_peak"] = roofline["achieved"] / peaks[key]

    ms_per_step = r32["wall"] * 1e3 / args.steps
    out = {
        "metric": METRIC,
        "value": ms_per_step * 1e-3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: cubed sphere 6x{wl['n']}^2, N={n}, k={k / math.pi:.0f}pi, eta=k, "
                         f"D={D}, P=({ps},{pa},{pa}), cones (n_s0,n_C0)=({args.ns0},{args.nc0}), 1 RHS"),
            "N": n, "depth": D, "p_s": ps, "p_ang": pa, "ns0": args.ns0, "nc0": args.nc0,
            "precision": "fp32 interpolation, fp64 target phase", "nrhs": 1,
        },
        "applies_per_s": 1e3 / ms_per_step,
        "event_ms_per_step": r32["ev_ms"] / args.steps,
        "event_ms_median": r32["ev_median"],
        "event_ms_min": r32["ev_min"],
        "rel_err": err32,
        "rel_err_targets": len(tg),
        "plan_create_s": r32["t_plan"],
        "plan_autotune_s": r32["t_tune"],
        "autotune": r32["tune"],
        "stages": stages,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "peaks_measured": peaks,
        "plan": {"cones": st["cones"], "boxes": st["boxes"], "near_pairs": st["near_pairs"],
                 "upward_pass_formulation": st["prop_kernel"],
                 "cousin_pairs": cousin, "prop_evals": prop_evals, "device_bytes": st["device_bytes"],
                 "pair_row_stage": pair_row_use(st)},
        "consistency_flags": r32["flags"],
    }
    out["adjoint"] = adj
    out["batched"] = batched
    out["ragged"] = ragged
    if r64 is not None:
        out["fp64"] = {"ms_per_step": r64["wall"] * 1e3 / args.fp64_steps, "event_ms_median": r64["ev_median"],
                       "event_ms_min": r64["ev_min"], "rel_err": err64, "plan_create_s": r64["t_plan"],
                       "setting": f"P=({ps},{pa},{pa}), cones ({args.ns0},{args.nc0}), as the FP32 apply",
                       "consistency_flags": r64["flags"]}
    if r64h is not None:
        out["fp64_1e-6"] = fp64_hi_entry(r64h, err64h, args.fp64_steps, n, D)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
