#!/usr/bin/env python3
"""Benchmark of the stiff-chemistry hot path on one MI355X.

Workload (default): the bulk-sparse detonation patch, 256 x 256 x 32 =
2,097,152 cells of the 9-species / 21-reaction synthetic H2-air mechanism,
dt = 5e-9 s, rtol 1e-8 / atol 1e-14, FP64.  One step = one chem_integrate
call over the whole patch (screen, bulk rounds, compaction, sparse phase),
restarted from a pristine device copy of the initial state (the copy is
inside the timed region).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

R_GAS = 8.314462618
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (256 CU x 2.4 GHz x 128 FLOP/clk)
HBM_PEAK_GBS = 8000.0
METRIC = "chemistry cell-steps/s, plain FP64 vs batched/mixed/surrogate at fixed error"


# HBM traffic of the bulk-round kernel per call, from two rocprofv3 --pmc
# passes (FETCH_SIZE, WRITE_SIZE; KiB summed over the 72 launches of three
# identical calls, 24 launches each) on the detonation patch with the options
# below.  The counters are scaled by what they read for a device copy of
# known size (151 MB: FETCH_SIZE reads half, WRITE_SIZE reads it exactly).
# Valid only for the kernel sources they were taken on (hash below) and
# these options.
TRAFFIC_PMC = {
    "src_sha1": "4865819382cd8b249a2c0f5fbf69e4bf2c7d4577",
    "options": {"group": 0.0, "max_rounds": 24.0, "nactive_star": 100000.0, "kmax_bulk": 20.0},
    "fetch_kib": 1.85639e7 / 3, "fetch_factor": 2.0,
    "write_kib": 3.80748e7 / 3, "write_factor": 1.0,
}


def kernel_sources_sha1():
    """Hash of the sources the one-lane integration kernels and their launch
    are built from (the cooperative, network and surrogate kernels are not)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2510_23993_amd", "csrc")
    names = ["chem_device.hpp", "chem_host_mech.hpp", "chem_kernels.hpp", "chem_lib.hip",
             "chem_math.hpp", "chem_types.hpp", "gen_mech.py"]
    files = [os.path.join(csrc, f) for f in names] + [os.path.join(ROOT, "synth", "data", "m9.mech")]
    h = hashlib.sha1()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(options, kernel):
    """Bytes per call of the bulk-round kernel, or None when the sources, the
    options or the dominant kernel differ from the ones measured."""
    t = TRAFFIC_PMC
    if not kernel.startswith("bulk-round") or kernel_sources_sha1() != t["src_sha1"]:
        return None
    if any(options.get(k) != v for k, v in t["options"].items()):
        return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"])


def mech_flop_model(path):
    """Algorithmic FLOPs per RHS / Jacobian / LU / solve, counted from the
    mechanism's nonzeros (exp, log and divide count as one FLOP)."""
    sys.path.insert(0, os.path.join(ROOT, "paper_2510_23993_amd", "csrc"))
    import gen_mech
    names, rx = gen_mech.parse_structure(path)
    ns, nr = len(names), len(rx)
    n = ns + 1
    nnz_f = sum(len(r["re"]) for r in rx)
    nnz_r = sum(len(r["pr"]) for r in rx)
    nnz = nnz_f + nnz_r
    n_tb = sum(1 for r in rx if r["type"] in (1, 2))
    n_fo = sum(1 for r in rx if r["type"] == 2)
    f_thermo = 20 * ns                      # NASA-7 h and s (Horner) per species
    f_conc = 3 * ns                         # C, floor, ln C
    f_arr = 5 * nr                          # ln kf contraction with (1, ln T, -1/T)
    f_kc = 2 * nnz + 2 * nr                 # ln Kc row of nu against g/RT, + dnu ln(Pref/RT)
    f_lnq = 2 * nnz + 2 * nr                # nu' and nu'' contractions against ln C, exp
    f_tb = 2 * ns * n_tb + n_tb             # [M] sums and multiply
    f_fo = 30 * n_fo                        # falloff: Pr, Fcent, Troe broadening
    f_om = 2 * nnz + nr                     # production omega = nu (qf - qr)
    f_out = 6 * ns + 4                      # dY/dt, c_v, energy sum, dT/dt
    F_rhs = f_thermo + f_conc + f_arr + f_kc + f_lnq + f_tb + f_fo + f_om + f_out
    dep = [len(r["re"]) + len(r["pr"]) if r["type"] == 0 else ns for r in rx]
    F_jac = F_rhs + sum(2 * (len(r["re"]) + len(r["pr"])) * d for r, d in zip(rx, dep)) \
        + 6 * n * nr + 4 * n * n
    F_lu = (2 * n ** 3) // 3
    F_solve = 2 * n * n
    return {"F_rhs": F_rhs, "F_jac": F_jac, "F_lu": F_lu, "F_solve": F_solve, "n": n,
            "ns": ns, "nr": nr}


def algorithmic_flops(model, st):
    return (st["rhs_evals"] * model["F_rhs"] + st["jac_evals"] * model["F_jac"]
            + st["lu_facts"] * model["F_lu"] + st["lin_solves"] * model["F_solve"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nz", type=int, default=32)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--atol", type=float, default=1e-14)
    ap.add_argument("--algorithm", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle sample size (0 = the whole field)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--opt", action="append", default=[], help="key=value library option")
    ap.add_argument("--workload", default="detonation", choices=["detonation", "amr", "m53"],
                    help="detonation: the bench line (default); amr: 400 AMR boxes, persistent "
                         "graph vs per-box launches; m53: 53-species mechanism, FP64 and mixed")
    ap.add_argument("--cells", type=int, default=65536, help="m53 workload: cells")
    ap.add_argument("--no-tune", action="store_true", help="detonation workload: skip chem_autotune")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the chemistry step shards "
                          "by cells with no exchange inside it, so each GPU's work is this "
                          "single-GPU workload on its share of the cells",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2510_23993_amd as chem
    from synth import fields
    if args.workload == "amr":
        return bench_amr(args, torch, chem, fields)
    if args.workload == "m53":
        return bench_m53(args, torch, chem, fields)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mech = chem.Mechanism(fields.M9_PATH)
    ctx = chem.Context(mech, algorithm=args.algorithm)
    for kv in args.opt:
        k, v = kv.split("=")
        ctx.set_option(k, float(v))

    cells = fields.c2_field(256, 256, args.nz)
    n = cells.T.size
    T_d = torch.as_tensor(cells.T, device=dev)
    p_d = torch.as_tensor(cells.p, device=dev)
    Y0 = torch.as_tensor(cells.Y, device=dev).contiguous()
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    e = torch.empty(n, dtype=torch.float64, device=dev)
    ctx.prepare_state(T_d, p_d, Y0, rho, e)        # reactor inputs built on the device
    Y = torch.empty_like(Y0)
    T = torch.empty_like(T_d)
    status = torch.empty(n, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(stats):
        Y.copy_(Y0)
        T.copy_(T_d)
        return ctx.integrate(rho, e, Y, T, cells.dt, args.rtol, args.atol, status=status, stats=stats)

    # schedule chosen by the library's autotuner on this field (outside the
    # timed region, reported separately)
    tune = None
    if not args.no_tune and not args.opt:
        Y.copy_(Y0)
        T.copy_(T_d)
        t0 = time.perf_counter()
        opts, best_ms = ctx.autotune([dict(rho=rho, e=e, Y=Y, T=T, status=status, dt=cells.dt)],
                                     args.rtol, args.atol)
        tune = {"options": opts, "best_call_ms": best_ms, "seconds": time.perf_counter() - t0}

    # warmup (also yields the per-call counters used for the FLOP count)
    st = None
    for _ in range(max(1, args.warmup)):
        st = step(True)
    torch.cuda.synchronize()
    # timed region: K steps, no host synchronisation inside
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step(False)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    ev_ms = ev0.elapsed_time(ev1) / args.steps
    value = n * args.steps / wall

    # per-call device time of each phase (library events on the context
    # stream) and the algorithmic FLOPs of each phase
    st = step(True)
    torch.cuda.synchronize()
    status_h = status.cpu().numpy()
    model = mech_flop_model(fields.M9_PATH)
    flops = algorithmic_flops(model, st)
    bulk = {k: st["bulk_" + k] for k in ("rhs_evals", "jac_evals", "lu_facts", "lin_solves")}
    f_bulk = algorithmic_flops(model, bulk)
    f_sparse = flops - f_bulk
    group = ctx.get_option("group")
    sched = ("one lane per cell" if (group == 0 or (group < 0 and n >= 65536)) else
             f"{int(group) if group > 0 else 16} lanes per cell")
    if ctx.get_option("algorithm") == 1 and ctx.get_option("max_rounds") == 0:
        sched += ", no bulk rounds"
    if st["t_bulk_ms"] >= st["t_sparse_ms"]:
        kern, f_k, t_k = f"bulk-round integration kernel ({sched})", f_bulk, st["t_bulk_ms"]
    else:
        kern, f_k, t_k = f"sparse-phase integration kernel ({sched})", f_sparse, st["t_sparse_ms"]
    achieved = f_k / (t_k * 1e-3) / 1e12

    # the same patch on the plain path (every cell, no skip, no compaction)
    ctx_plain = chem.Context(mech, algorithm=0)
    Y.copy_(Y0)
    T.copy_(T_d)
    st_plain = ctx_plain.integrate(rho, e, Y, T, cells.dt, args.rtol, args.atol, status=status)
    # mixed precision (FP32 exponentials), same tolerances
    ctx_mixed = chem.Context(mech, precision=1)
    for _ in range(2):
        Y.copy_(Y0)
        T.copy_(T_d)
        st_mixed = ctx_mixed.integrate(rho, e, Y, T, cells.dt, args.rtol, args.atol, status=status)
    # the paper's explicit first-order scheme (1% step limit), same screen
    ctx_exp = chem.Context(mech, method=1, explicit_frac=0.01)
    for _ in range(2):
        Y.copy_(Y0)
        T.copy_(T_d)
        st_exp = ctx_exp.integrate(rho, e, Y, T, cells.dt, args.rtol, args.atol, status=status)
    torch.cuda.synchronize()
    out = {
        "metric": METRIC, "value": value, "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"bulk-sparse detonation patch 256x256x{args.nz} ({n} cells), "
                   "9-species/21-reaction synthetic H2-air mechanism, dt 5e-9 s",
                   "rtol": args.rtol, "atol": args.atol,
                   "algorithm": "bulk-sparse" if args.algorithm == 1 else "plain",
                   "options": {k: ctx.get_option(k) for k in (
                       "t_react_min", "kmax_bulk", "nactive_star", "kmax_sparse", "max_rounds",
                       "grid_waves", "group")}},
        "event_ms_per_step": ev_ms,
        "autotune": tune,
        "stats": {k: st[k] for k in ("n_active0", "n_active_after_bulk", "n_bulk_rounds",
                                     "steps_total", "attempts_total", "rhs_evals", "jac_evals",
                                     "lu_facts", "lin_solves", "max_steps_cell", "t_total_ms")},
        "status_counts": np.bincount(status_h, minlength=8).tolist(),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic({k: ctx.get_option(k) for k in TRAFFIC_PMC["options"]}, kern),
                     "traffic_unit": "bytes per call (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                     "algorithmic_bytes_per_call": 8 * (2 * mech.ns + 4) * st["n_active0"],
                     "kernel": kern, "kernel_ms_per_call": t_k, "flops_per_call": f_k,
                     "whole_call": {"flops": flops, "ms": st["t_total_ms"],
                                    "tflops": flops / (st["t_total_ms"] * 1e-3) / 1e12},
                     "phase_ms": {k: st[k] for k in ("t_screen_ms", "t_bulk_ms", "t_sparse_ms")},
                     "flop_model": model},
        "variants": {
            "plain_all_cells_fp64": {"ms_per_call": st_plain["t_total_ms"],
                                     "speedup_of_bulk_sparse": st_plain["t_total_ms"] / st["t_total_ms"]},
            "bulk_sparse_mixed_fp32_exp": {"ms_per_call": st_mixed["t_total_ms"],
                                           "speedup_vs_fp64": st["t_total_ms"] / st_mixed["t_total_ms"]},
            "explicit_first_order_frac_0.01": {"ms_per_call": st_exp["t_total_ms"],
                                               "steps_total": st_exp["steps_total"],
                                               "note": "not at the BDF path's error: see the fixed-error comparison"},
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cells, args, n)
    print(json.dumps(out))


def _opts(ctx):
    return {k: ctx.get_option(k) for k in ("t_react_min", "kmax_bulk", "nactive_star", "kmax_sparse",
                                            "max_rounds", "grid_waves", "group", "precision")}


def bench_amr(args, torch, chem, fields):
    """400 seeded AMR boxes over three levels (about 6M cells, dt 4e-8 / 2e-8 /
    1e-8 s by level), jet-in-crossflow-like field.  Times K steps of: one
    launch per box (chem_integrate per box), one chem_integrate_boxes replayed
    from a hipGraph with default options, and the same after chem_autotune;
    then the subcycled coarse step (level 0 once, level 1 twice, level 2 four
    times, each with its own dt).  Every step restarts from a pristine device
    copy (inside the timed region)."""
    boxes = fields.c3_boxes()
    mech = chem.Mechanism(fields.M9_PATH)
    stream = torch.cuda.Stream()
    ntot = 0
    dev_boxes = []
    with torch.cuda.stream(stream):
        ctx0 = chem.Context(mech, stream=stream)
        for i, b in enumerate(boxes):
            c = fields.c3_box_state(b, box_id=i)
            n = c.T.size
            T0 = torch.as_tensor(c.T, device="cuda")
            p = torch.as_tensor(c.p, device="cuda")
            Y0 = torch.as_tensor(c.Y, device="cuda").contiguous()
            rho = torch.empty(n, dtype=torch.float64, device="cuda")
            e = torch.empty_like(rho)
            ctx0.prepare_state(T0, p, Y0, rho, e)
            dev_boxes.append(dict(rho=rho, e=e, Y=torch.empty_like(Y0), T=torch.empty_like(T0), Y0=Y0, T0=T0,
                                  status=torch.empty(n, dtype=torch.uint8, device="cuda"), dt=b.dt,
                                  level=b.level))
            ntot += n
    torch.cuda.synchronize()

    def reset():
        for d in dev_boxes:
            d["Y"].copy_(d["Y0"])
            d["T"].copy_(d["T0"])

    def timed(fn):
        with torch.cuda.stream(stream):
            for _ in range(max(1, args.warmup)):
                reset()
                fn()
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            ev0.record(stream)
            for _ in range(args.steps):
                reset()
                fn()
            ev1.record(stream)
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - t0) / args.steps, ev0.elapsed_time(ev1) / args.steps

    res = {}
    with torch.cuda.stream(stream):
        per = chem.Context(mech, stream=stream, use_graph=0)
        res["per_box_launches"] = timed(lambda: [per.integrate(d["rho"], d["e"], d["Y"], d["T"], d["dt"], args.rtol,
                                                               args.atol, status=d["status"], stats=False)
                                                 for d in dev_boxes])
        g = chem.Context(mech, stream=stream, use_graph=1)
        res["graph_default"] = timed(lambda: g.integrate_boxes(dev_boxes, args.rtol, args.atol, stats=False))
        tuned = chem.Context(mech, stream=stream, use_graph=1)
        reset()
        t0 = time.perf_counter()
        tuned_opts, tune_ms = tuned.autotune(dev_boxes, args.rtol, args.atol)
        t_tune = time.perf_counter() - t0
        res["graph_autotuned"] = timed(lambda: tuned.integrate_boxes(dev_boxes, args.rtol, args.atol, stats=False))
        # subcycled: per coarse step, level 0 once, level 1 twice and level 2
        # four times, each with its own dt (one graph per box table)
        l12 = [d for d in dev_boxes if d["level"] >= 1]
        l2 = [d for d in dev_boxes if d["level"] == 2]
        c12 = chem.Context(mech, stream=stream, use_graph=1, **tuned_opts)
        c2 = chem.Context(mech, stream=stream, use_graph=1, **tuned_opts)

        def subcycled():
            tuned.integrate_boxes(dev_boxes, args.rtol, args.atol, stats=False)
            c12.integrate_boxes(l12, args.rtol, args.atol, stats=False)
            c2.integrate_boxes(l2, args.rtol, args.atol, stats=False)
            c2.integrate_boxes(l2, args.rtol, args.atol, stats=False)
        res["subcycled_graph_autotuned"] = timed(subcycled)
        sub_cells = sum(d["rho"].numel() * (1 << d["level"]) for d in dev_boxes)
        # counters and phase times of one eager call with the tuned options
        tuned.set_option("use_graph", 0)
        reset()
        st = tuned.integrate_boxes(dev_boxes, args.rtol, args.atol)
    torch.cuda.synchronize()
    wall_ms, ev_ms = res["graph_autotuned"]
    model = mech_flop_model(fields.M9_PATH)
    flops = algorithmic_flops(model, st)
    bulk = {k: st["bulk_" + k] for k in ("rhs_evals", "jac_evals", "lu_facts", "lin_solves")}
    f_bulk = algorithmic_flops(model, bulk)
    if st["t_bulk_ms"] >= st["t_sparse_ms"]:
        kern, f_k, t_k = "bulk-round integration kernel", f_bulk, st["t_bulk_ms"]
    else:
        kern, f_k, t_k = "sparse-phase integration kernel", flops - f_bulk, st["t_sparse_ms"]
    achieved = f_k / (t_k * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": ntot / (wall_ms * 1e-3), "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"AMR batching: 400 boxes over 3 levels ({ntot} cells), jet-in-crossflow-like "
                               "field, dt 4e-8/2e-8/1e-8 s by level, 9-species mechanism",
                   "rtol": args.rtol, "atol": args.atol, "tuned_options": tuned_opts,
                   "autotune_s": t_tune, "autotune_best_call_ms": tune_ms},
        "event_ms_per_step": ev_ms,
        "variants_ms_per_step": {k: {"wall": v[0], "events": v[1]} for k, v in res.items()},
        "speedup_graph_autotuned_vs_per_box": res["per_box_launches"][0] / wall_ms,
        "subcycled": {"cell_steps_per_coarse_step": sub_cells,
                      "ms_per_coarse_step": res["subcycled_graph_autotuned"][0],
                      "cell_steps_per_s": sub_cells / (res["subcycled_graph_autotuned"][0] * 1e-3)},
        "stats": {k: st[k] for k in ("n_active0", "n_active_after_bulk", "n_bulk_rounds", "steps_total",
                                     "attempts_total", "t_total_ms", "t_screen_ms", "t_bulk_ms", "t_sparse_ms")},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None, "kernel": kern,
                     "kernel_ms_per_call": t_k, "flops_per_call": f_k},
    }
    print(json.dumps(out))


def bench_m53(args, torch, chem, fields):
    """53-species / 325-reaction mechanism, n cells of the seeded T/p/progress
    distribution, dt 1e-7 s.  FP64 at rtol 1e-7 / atol 1e-20 (the loosest
    tolerance at which the FP64 oracle meets 1e-4 relative on species above
    1e-10), cooperative schedules of 32 and 64 lanes per cell, and the
    FP32-exponential mode at rtol 1e-6 for context (it does not reach the
    budget on this mechanism)."""
    mech = chem.Mechanism(fields.M53_PATH)
    cells = fields.c4_cells(args.cells, seed=1004)
    n = cells.T.size
    T0 = torch.as_tensor(cells.T, device="cuda")
    p = torch.as_tensor(cells.p, device="cuda")
    Y0 = torch.as_tensor(cells.Y, device="cuda").contiguous()
    ctx0 = chem.Context(mech)
    rho = torch.empty(n, dtype=torch.float64, device="cuda")
    e = torch.empty_like(rho)
    ctx0.prepare_state(T0, p, Y0, rho, e)
    Y, T = torch.empty_like(Y0), torch.empty_like(T0)
    status = torch.empty(n, dtype=torch.uint8, device="cuda")
    runs = {}
    for name, opts, rtol in (("fp64_g64", dict(group=64), 1e-7), ("fp64_g32", dict(group=32), 1e-7),
                             ("mixed_g64_rtol1e-6", dict(group=64, precision=1, kmax_sparse=20000), 1e-6),
                             ("fp64_g64_rtol1e-6", dict(group=64), 1e-6)):
        ctx = chem.Context(mech, **opts)
        Y.copy_(Y0)
        T.copy_(T0)
        st = ctx.integrate(rho, e, Y, T, cells.dt, rtol, 1e-20, status=status)
        runs[name] = {"ms": st["t_total_ms"], "rtol": rtol, "steps_total": st["steps_total"],
                      "max_steps_cell": st["max_steps_cell"],
                      "status_counts": np.bincount(status.cpu().numpy(), minlength=8).tolist(),
                      "cell_steps_per_s": n / (st["t_total_ms"] * 1e-3)}
        print(json.dumps({name: runs[name]}), file=sys.stderr, flush=True)
    best = min(("fp64_g64", "fp64_g32"), key=lambda k: runs[k]["ms"])
    out = {"metric": METRIC, "value": runs[best]["cell_steps_per_s"], "unit": "cell-steps/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": runs[best]["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"53-species/325-reaction synthetic mechanism, {n} cells, dt 1e-7 s",
                      "rtol": 1e-7, "atol": 1e-20, "schedule": best},
           "variants": runs}
    if not args.no_cpu:
        import oracle
        orc = oracle.Oracle(fields.M53_PATH)
        m = 256
        r, ee = orc.state_from_TPY(cells.T[:m], cells.p[:m], cells.Y[:, :m])
        threads = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        orc.integrate(r, ee, cells.Y[:, :m], cells.dt, 1e-7, 1e-20, T=cells.T[:m], nthreads=threads)
        wall = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m / wall, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
                               "sample": f"the first {m} cells, rtol 1e-7 / atol 1e-20, {wall:.2f} s wall"}
    print(json.dumps(out))


def cpu_baseline(cells, args, n_full):
    """The oracle (plain C + OpenMP, FP64, no skip) on a stratified sample of
    the same field at the same tolerances, scaled to the full field."""
    import oracle
    from synth import fields
    orc = oracle.Oracle(fields.M9_PATH)
    if args.cpu_sample <= 0 or args.cpu_sample >= n_full:
        idx = np.arange(n_full)
    else:
        rng = np.random.default_rng(1002)
        idx = []
        for c in np.unique(cells.cls):
            members = np.where(cells.cls == c)[0]
            k = max(1, int(round(args.cpu_sample * members.size / n_full)))
            idx.append(rng.choice(members, size=min(k, members.size), replace=False))
        idx = np.sort(np.concatenate(idx))
    rho, e = orc.state_from_TPY(cells.T[idx], cells.p[idx], cells.Y[:, idx])
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    orc.integrate(rho, e, cells.Y[:, idx], cells.dt, args.rtol, args.atol, T=cells.T[idx],
                  nthreads=threads)
    wall = time.perf_counter() - t0
    return {"value": idx.size / wall, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
            "sample": (f"the whole field ({idx.size} cells)" if idx.size == n_full else
                       f"{idx.size} cells stratified by class (cold/induction/burnt)")
                      + f", same rtol/atol, {wall:.2f} s wall"}


if __name__ == "__main__":
    main()
