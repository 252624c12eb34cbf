#!/usr/bin/env python3
"""Benchmark of the stiff-chemistry hot path on one MI355X.

Default workload: the bulk-sparse detonation patch, 256 x 256 x 32 =
2,097,152 cells of the 9-species / 21-reaction synthetic H2-air mechanism,
dt = 5e-9 s, FP64, at fixed error: the loosest rtol (of 1e-4 ... 1e-8, atol
1e-14) at which the path's result stays within 1e-4 relative on species above
1e-10 and 1 K of the oracle (rtol 1e-12 / atol 1e-20) on a stratified sample
of the field.  One step = one chem_integrate call over the whole patch
(screen, compaction, bulk rounds if the autotuner keeps any, sparse phase)
with the autotuned schedule;
every timed step starts from its own pristine copy of the initial state,
resident in HBM before the timed region.  Prints one JSON line with the
roofline of the dominant kernel, the comparison paths (plain all-cells FP64,
mixed precision, the explicit scheme, the AMR batching and the surrogate
configurations) and the CPU oracle timed beside it.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import shutil
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector (256 CU x 2.4 GHz x 128 FLOP/clk)
HBM_PEAK_GBS = 8000.0
METRIC = "chemistry cell-steps/s, plain FP64 vs batched/mixed/surrogate at fixed error"
BUDGET_REL, BUDGET_T, SPECIES_FLOOR = 1e-4, 1.0, 1e-10
RTOLS = (1e-4, 1e-5, 1e-6, 1e-7, 1e-8)
ATOL = 1e-14
C1_RTOL, C1_ATOL = 1e-8, 1e-14


# ------------------------------------------------------------ FLOP counts
def _structure(path):
    sys.path.insert(0, os.path.join(ROOT, "paper_2510_23993_amd", "csrc"))
    import gen_mech
    return gen_mech.parse_structure(path)


def flop_count(path):
    """Algorithmic FLOPs per RHS / Jacobian / LU / solve counted from the
    mechanism's nonzeros (exp, log and divide count as one):
      RHS      20 ns (thermo) + 3 nr + 2 nnz(nu) (ln Kc) + 2 (nnz(nu') + nnz(nu''))
               (ln q) + 2 nnz(nu) (production) + 4 ns
      Jacobian sum_j 2 (r_j + p_j)^2 + 6 n nr (temperature column)
      LU       2 n^3 / 3,  solve 2 n^2,  n = ns + 1."""
    names, rx = _structure(path)
    ns, nr = len(names), len(rx)
    n = ns + 1
    nnz_f = sum(len(r["re"]) for r in rx)
    nnz_r = sum(len(r["pr"]) for r in rx)
    nnz_nu = 0
    for r in rx:
        net = {}
        for k, v in r["re"]:
            net[k] = net.get(k, 0) - v
        for k, v in r["pr"]:
            net[k] = net.get(k, 0) + v
        nnz_nu += sum(1 for v in net.values() if v != 0)
    F_rhs = 20 * ns + 3 * nr + 2 * nnz_nu + 2 * (nnz_f + nnz_r) + 2 * nnz_nu + 4 * ns
    F_jac = sum(2 * (len(r["re"]) + len(r["pr"])) ** 2 for r in rx) + 6 * n * nr
    return {"F_rhs": F_rhs, "F_jac": F_jac, "F_lu": (2 * n ** 3) // 3, "F_solve": 2 * n * n,
            "n": n, "ns": ns, "nr": nr, "nnz_nu": nnz_nu, "nnz_fwd": nnz_f, "nnz_rev": nnz_r}


def flops_of(model, c):
    return (c["rhs_evals"] * model["F_rhs"] + c["jac_evals"] * model["F_jac"]
            + c["lu_facts"] * model["F_lu"] + c["lin_solves"] * model["F_solve"])


def phase_counts(st):
    bulk = {k: st["bulk_" + k] for k in ("rhs_evals", "jac_evals", "lu_facts", "lin_solves")}
    rest = {k: st[k] - bulk[k] for k in bulk}
    return bulk, rest


# ------------------------------------------------------------ error checks
def rel_errors(Yg, Tg, Yr, Tr):
    big = Yr > SPECIES_FLOOR
    rel = np.where(big, np.abs(Yg - Yr) / np.where(big, Yr, 1.0), 0.0)
    return float(rel.max()), float(np.abs(Tg - Tr).max())


def stratified_sample(cls, per_class, seed):
    rng = np.random.default_rng(seed)
    idx = []
    for k, m in per_class.items():
        members = np.where(cls == k)[0]
        if members.size:
            idx.append(rng.choice(members, size=min(m, members.size), replace=False))
    return np.sort(np.concatenate(idx))


def oracle_reference(orc, T, p, Y, dt):
    rho, e = orc.state_from_TPY(T, p, Y)
    Yr, Tr, st = orc.integrate(rho, e, Y, dt, 1e-12, 1e-20, T=T,
                               nthreads=len(os.sched_getaffinity(0)))
    return Yr, Tr, st


# ------------------------------------------------------------ device helpers
class Field:
    """A device-resident field: reactor inputs and a pristine initial state."""

    def __init__(self, torch, ctx0, cells):
        dev = torch.device("cuda")
        self.n = cells.T.size
        self.dt = cells.dt
        self.T0 = torch.as_tensor(cells.T, device=dev)
        p = torch.as_tensor(cells.p, device=dev)
        self.Y0 = torch.as_tensor(cells.Y, device=dev).contiguous()
        self.rho = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.e = torch.empty_like(self.rho)
        ctx0.prepare_state(self.T0, p, self.Y0, self.rho, self.e)   # reactor inputs built on the device
        self.Y = torch.empty_like(self.Y0)
        self.T = torch.empty_like(self.T0)
        self.status = torch.empty(self.n, dtype=torch.uint8, device=dev)

    def reset(self):
        self.Y.copy_(self.Y0)
        self.T.copy_(self.T0)


def timed_calls(torch, ctx, F, rtol, atol, reps=3, stream=None):
    """Median of `reps` calls, each from a pristine state restored outside
    the HIP-event interval around the call; returns (ms, last stats)."""
    stream = stream or torch.cuda.current_stream()
    ms, st = [], None
    for _ in range(reps):
        F.reset()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        st = ctx.integrate(F.rho, F.e, F.Y, F.T, F.dt, rtol, atol, status=F.status)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    return float(np.median(ms)), st


def sweep(torch, ctx, F, idx, Yr, Tr, rtols=RTOLS, atol=ATOL):
    """Loosest rtol meeting the budget on the sample; one row per rtol tried."""
    rows, chosen = [], None
    for r in rtols:
        F.reset()
        st = ctx.integrate(F.rho, F.e, F.Y, F.T, F.dt, r, atol, status=F.status)
        Yg = F.Y[:, idx].cpu().numpy()
        Tg = F.T[idx].cpu().numpy()
        rel, dT = rel_errors(Yg, Tg, Yr, Tr)
        ok = rel <= BUDGET_REL and dT <= BUDGET_T and st["n_incomplete"] == 0
        rows.append({"rtol": r, "max_rel": rel, "max_dT_K": dT, "ms": st["t_total_ms"], "meets_budget": ok})
        if ok:
            chosen = r
            break
    return chosen, rows


# ------------------------------------------------------------ HBM traffic
def _pmc_sum(outdir, counter, name_part):
    """Sum of a counter over the dispatches whose kernel name contains name_part;
    also the number of such dispatches."""
    total, disp = 0.0, 0
    for f in glob.glob(os.path.join(outdir, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter or name_part not in row.get("Kernel_Name", ""):
                    continue
                total += float(row["Counter_Value"])
                disp += 1
    return total, disp


def measure_traffic(args, opts, rtol, mode=1):
    """HBM bytes per call of the dominant integration kernel (mode 1: the
    bulk rounds, 2: the sparse phase) from two rocprofv3 counter passes
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) over a probe run of this
    script with the same options, each scaled by what the same counter reads
    for a device copy of known size in the same run."""
    prof = shutil.which("rocprofv3")
    if prof is None:
        return None, "rocprofv3 not found"
    res = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        d = tempfile.mkdtemp(prefix="chem_pmc_", dir="/tmp")
        cmd = ["timeout", "-s", "KILL", "300", prof, "--pmc", counter, "-d", d, "-o", "p", "-f", "csv", "--",
               sys.executable, os.path.abspath(__file__), "--traffic-probe", "--nz", str(args.nz),
               "--rtol", repr(rtol), "--probe-opts", json.dumps(opts)]
        env = dict(os.environ, TMPDIR="/tmp")
        p = subprocess.run(cmd, cwd="/tmp", env=env, capture_output=True, text=True)
        if p.returncode != 0:
            shutil.rmtree(d, ignore_errors=True)
            return None, f"rocprofv3 --pmc {counter} exited with {p.returncode}: {p.stderr[-300:]}"
        kern, nk = _pmc_sum(d, counter, f"k_integrate<Mech_m9, {mode}>")
        copy, nc = _pmc_sum(d, counter, "copyBuffer")
        if nk == 0:
            kern, nk = _pmc_sum(d, counter, "k_integrate_coop")
        probe = json.loads([ln for ln in p.stdout.splitlines() if ln.startswith("{")][-1])
        shutil.rmtree(d, ignore_errors=True)
        if nk == 0 or nc == 0:
            return None, f"{counter}: no integration or copy dispatches found in the counter output"
        res[counter] = {"kib_per_call": kern / probe["calls"], "dispatches": nk,
                        "copy_kib": copy, "copy_bytes": probe["copy_bytes"] * probe["copies"],
                        "scale": probe["copy_bytes"] * probe["copies"] / (copy * 1024.0)}
    traffic = sum(1024.0 * r["kib_per_call"] * r["scale"] for r in res.values())
    return traffic, res


def traffic_probe(args):
    """Child of measure_traffic (run under rocprofv3): two device copies of a
    known size, then two integration calls with the given options."""
    import torch
    import paper_2510_23993_amd as chem
    from synth import fields
    torch.cuda.set_device(0)
    nbytes = 256 << 20
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    mech = chem.Mechanism(fields.M9_PATH)
    ctx = chem.Context(mech, **json.loads(args.probe_opts))
    F = Field(torch, ctx, fields.c2_field(256, 256, args.nz))
    calls = 2
    for _ in range(calls):
        F.reset()
        ctx.integrate(F.rho, F.e, F.Y, F.T, F.dt, args.rtol, ATOL, status=F.status, stats=False)
    torch.cuda.synchronize()
    print(json.dumps({"calls": calls, "copy_bytes": nbytes, "copies": 2}))


# ------------------------------------------------------------ main workload
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nz", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-traffic", action="store_true", help="skip the rocprofv3 counter passes")
    ap.add_argument("--no-extra", action="store_true", help="skip the AMR and surrogate configurations")
    ap.add_argument("--opt", action="append", default=[], help="key=value library option (skips autotuning)")
    ap.add_argument("--rtol", type=float, default=0.0, help="fixed rtol (0: the fixed-error sweep)")
    ap.add_argument("--workload", default="detonation", choices=["detonation", "amr", "m53", "strang", "contract"])
    ap.add_argument("--cells", type=int, default=65536, help="m53 workload: cells")
    ap.add_argument("--chunks", type=int, default=1, help="m53 workload: calls the cells are split into")
    ap.add_argument("--traffic-probe", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--probe-opts", default="{}", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the chemistry step shards "
                          "by cells with no exchange inside it, so each GPU's work is this "
                          "single-GPU workload on its share of the cells",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.traffic_probe:
        return traffic_probe(args)

    import torch
    import paper_2510_23993_amd as chem
    import oracle
    from synth import fields
    torch.cuda.set_device(0)
    if args.workload == "amr":
        print(json.dumps(bench_amr(args, torch, chem, fields, oracle, rtol=args.rtol or 1e-5)))
        return
    if args.workload == "m53":
        return bench_m53(args, torch, chem, fields, oracle)
    if args.workload == "strang":
        return bench_strang(args, torch, chem, fields)
    if args.workload == "contract":
        return bench_contract(args, torch, chem, fields)

    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    mech = chem.Mechanism(fields.M9_PATH)
    orc = oracle.Oracle(fields.M9_PATH)
    cells = fields.c2_field(256, 256, args.nz)
    n = cells.T.size
    ctx0 = chem.Context(mech)
    F = Field(torch, ctx0, cells)
    # oracle reference on a stratified sample (cold, induction, burnt)
    idx = stratified_sample(cells.cls, {0: 64, 1: 400, 2: 400}, seed=1002)
    Yr, Tr, _ = oracle_reference(orc, cells.T[idx], cells.p[idx], cells.Y[:, idx], cells.dt)
    sample_desc = (f"{idx.size} cells stratified by class (64 cold, 400 induction, 400 burnt), "
                   "oracle at rtol 1e-12 / atol 1e-20")

    # fixed-error sweep of each path with default options
    paths = {"bulk_sparse_fp64": dict(algorithm=1), "plain_all_cells_fp64": dict(algorithm=0),
             "bulk_sparse_fp32_exp": dict(algorithm=1, precision=1)}
    sweeps, chosen = {}, {}
    for name, o in paths.items():
        c = chem.Context(mech, **o)
        chosen[name], sweeps[name] = sweep(torch, c, F, idx, Yr, Tr)
        log(name, "fixed-error rtol", chosen[name])
    rtol = args.rtol or chosen["bulk_sparse_fp64"] or C1_RTOL

    # the headline path: bulk-sparse FP64, schedule autotuned at that rtol
    ctx = chem.Context(mech)
    tune = None
    if args.opt:
        for kv in args.opt:
            k, v = kv.split("=")
            ctx.set_option(k, float(v))
    else:
        F.reset()
        t0 = time.perf_counter()
        opts, best_ms = ctx.autotune([dict(rho=F.rho, e=F.e, Y=F.Y, T=F.T, status=F.status, dt=F.dt)], rtol, ATOL)
        tune = {"options": opts, "best_call_ms": best_ms, "seconds": time.perf_counter() - t0}
    tuned_opts = {k: ctx.get_option(k) for k in ("group", "max_rounds", "nactive_star", "kmax_bulk", "grid_waves", "order")}
    _, tuned_rows = sweep(torch, ctx, F, idx, Yr, Tr, rtols=(rtol,))

    # K pristine copies resident in HBM before the timed region
    K = args.steps
    Ys = [F.Y0.clone() for _ in range(K)]
    Ts = [F.T0.clone() for _ in range(K)]
    for _ in range(max(1, args.warmup)):
        F.reset()
        ctx.integrate(F.rho, F.e, F.Y, F.T, F.dt, rtol, ATOL, status=F.status)
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    stats = []
    torch.cuda.synchronize()
    torch.cuda._sleep(1)   # marks the start of the timed calls in a kernel trace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        evs[i][0].record(stream)
        # stats: per-phase HIP events on the context stream (a host sync per call)
        stats.append(ctx.integrate(F.rho, F.e, Ys[i], Ts[i], F.dt, rtol, ATOL, status=F.status))
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    torch.cuda._sleep(1)   # marks the end of the timed calls in a kernel trace
    ev_ms = [a.elapsed_time(b) for a, b in evs]
    value = n * K / wall
    del Ys, Ts

    # roofline of the dominant kernel over the timed calls
    model = flop_count(fields.M9_PATH)
    t_bulk = float(np.mean([s["t_bulk_ms"] for s in stats]))
    t_sparse = float(np.mean([s["t_sparse_ms"] for s in stats]))
    f_bulk = float(np.mean([flops_of(model, phase_counts(s)[0]) for s in stats]))
    f_rest = float(np.mean([flops_of(model, phase_counts(s)[1]) for s in stats]))
    sched = "one lane per cell" if tuned_opts["group"] == 0 else f"{int(tuned_opts['group'])} lanes per cell"
    if t_bulk >= t_sparse:
        kern, f_k, t_k = f"bulk-round integration kernel ({sched})", f_bulk, t_bulk
    else:
        kern, f_k, t_k = f"sparse-phase integration kernel ({sched})", f_rest, t_sparse
    achieved = f_k / (t_k * 1e-3) / 1e12
    traffic, traffic_detail = (None, "skipped (--no-traffic)")
    if not args.no_traffic:
        probe_opts = dict(tuned_opts, algorithm=1)
        traffic, traffic_detail = measure_traffic(args, probe_opts, rtol, 1 if kern.startswith("bulk") else 2)
    s_last = stats[-1]
    roofline = {
        "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
        "kernel": kern, "kernel_ms_per_call": t_k, "flops_per_call": f_k,
        "flop_count": model,
        "traffic_detail": traffic_detail,
        "algorithmic_bytes_per_call": 8 * (2 * mech.ns + 4) * s_last["n_active0"],
        "whole_call": {"flops": f_bulk + f_rest, "ms": float(np.mean([s["t_total_ms"] for s in stats]))},
        "phase_ms": {"screen": float(np.mean([s["t_screen_ms"] for s in stats])), "bulk": t_bulk,
                     "sparse": t_sparse},
    }

    # comparison paths at their own fixed-error rtol (median of 3 calls)
    variants = {}
    for name, o in paths.items():
        r = chosen[name]
        if r is None:
            variants[name] = {"meets_budget_at": None, "sweep": sweeps[name]}
            continue
        c = chem.Context(mech, **o)
        ms, st = timed_calls(torch, c, F, r, ATOL)
        variants[name] = {"rtol": r, "ms_per_call": ms, "cell_steps_per_s": n / (ms * 1e-3),
                          "steps_total": st["steps_total"], "sweep": sweeps[name]}
    t_plain = variants["plain_all_cells_fp64"].get("ms_per_call")
    for v in variants.values():
        if "ms_per_call" in v and t_plain:
            v["speedup_vs_plain_fp64_at_fixed_error"] = t_plain / v["ms_per_call"]
    ms_c1, st_c1 = timed_calls(torch, ctx, F, C1_RTOL, C1_ATOL)
    Yg = F.Y[:, idx].cpu().numpy()
    Tg = F.T[idx].cpu().numpy()
    rel_c1, dT_c1 = rel_errors(Yg, Tg, Yr, Tr)
    variants["bulk_sparse_fp64_tuned_c1_tolerances"] = {
        "rtol": C1_RTOL, "atol": C1_ATOL, "ms_per_call": ms_c1, "cell_steps_per_s": n / (ms_c1 * 1e-3),
        "max_rel": rel_c1, "max_dT_K": dT_c1}
    cexp = chem.Context(mech, method=1, explicit_frac=0.01)
    ms_e, st_e = timed_calls(torch, cexp, F, C1_RTOL, C1_ATOL, reps=2)
    rel_e, dT_e = rel_errors(F.Y[:, idx].cpu().numpy(), F.T[idx].cpu().numpy(), Yr, Tr)
    variants["explicit_first_order_frac_0.01"] = {
        "ms_per_call": ms_e, "steps_total": st_e["steps_total"], "max_rel": rel_e, "max_dT_K": dT_e,
        "meets_budget": rel_e <= BUDGET_REL and dT_e <= BUDGET_T}

    out = {
        "metric": METRIC, "value": value, "unit": "cell-steps/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": 1e3 * wall / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"bulk-sparse detonation patch 256x256x{args.nz} ({n} cells), "
                   "9-species/21-reaction synthetic H2-air mechanism, dt 5e-9 s, FP64 at fixed error",
                   "rtol": rtol, "atol": ATOL, "algorithm": "bulk-sparse", "options": tuned_opts},
        "fixed_error": {"budget": {"max_rel_species": BUDGET_REL, "species_floor": SPECIES_FLOOR,
                                   "max_dT_K": BUDGET_T},
                        "sample": sample_desc, "rtols_tried": list(RTOLS), "chosen_rtol": chosen,
                        "headline_check": tuned_rows[0]},
        "event_ms_per_step": {"median": float(np.median(ev_ms)), "mean": float(np.mean(ev_ms))},
        "autotune": tune,
        "stats": {k: s_last[k] for k in ("n_active0", "n_active_after_bulk", "n_bulk_rounds", "steps_total",
                                         "attempts_total", "rhs_evals", "jac_evals", "lu_facts", "lin_solves",
                                         "max_steps_cell", "t_total_ms")},
        "roofline": roofline,
        "variants": variants,
    }
    if not args.no_extra:
        out["amr_batching"] = bench_amr(args, torch, chem, fields, oracle, rtol=rtol, quiet=True)
        out["surrogate"] = bench_surrogate(args, torch, chem, fields, oracle, rtol=rtol)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(orc, cells, rtol, ATOL)
    print(json.dumps(out))


def cpu_baseline(orc, cells, rtol, atol):
    """The oracle (plain C + OpenMP, FP64, no skip) on the whole field at the
    same tolerances as the headline path; median of 3 runs."""
    threads = len(os.sched_getaffinity(0))
    rho, e = orc.state_from_TPY(cells.T, cells.p, cells.Y)
    walls = []
    for _ in range(3):
        t0 = time.perf_counter()
        orc.integrate(rho, e, cells.Y, cells.dt, rtol, atol, T=cells.T, nthreads=threads)
        walls.append(time.perf_counter() - t0)
    w = float(np.median(walls))
    return {"value": cells.T.size / w, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole field ({cells.T.size} cells, every cell integrated), rtol {rtol:g} / "
                      f"atol {atol:g}, median of 3 runs: " + ", ".join(f"{x:.2f}" for x in walls) + " s"}


# ------------------------------------------------------------ AMR batching
def bench_amr(args, torch, chem, fields, oracle, rtol, quiet=False):
    """400 seeded AMR boxes over three levels (5,750,784 cells, dt 4e-8 /
    2e-8 / 1e-8 s by level), jet-in-crossflow-like field: one launch per box
    against one hipGraph-replayed pipeline over all boxes (default options and
    after chem_autotune), then the subcycled coarse step (level 0 once, level 1
    twice, level 2 four times).  Median of 3 steps each, the restore of the
    initial state outside the HIP-event interval.  At fixed error: starting
    from `rtol`, the loosest rtol of the sweep at which a sample of active
    cells (one per even box) meets the budget against the oracle."""
    boxes = fields.c3_boxes()
    mech = chem.Mechanism(fields.M9_PATH)
    orc = oracle.Oracle(fields.M9_PATH)
    stream = torch.cuda.Stream()
    ntot, dev_boxes, sample = 0, [], []
    rng = np.random.default_rng(1003)
    with torch.cuda.stream(stream):
        ctx0 = chem.Context(mech, stream=stream)
        for i, b in enumerate(boxes):
            c = fields.c3_box_state(b, box_id=i)
            F = Field(torch, ctx0, c)
            dev_boxes.append(dict(rho=F.rho, e=F.e, Y=F.Y, T=F.T, Y0=F.Y0, T0=F.T0, status=F.status, dt=b.dt,
                                  level=b.level))
            if i % 2 == 0:
                act = np.where(c.T >= 500.0)[0]
                if act.size:
                    j = int(rng.choice(act))
                    sample.append((i, j, c.T[j], c.p[j], c.Y[:, j].copy(), c.dt))
            ntot += F.n
    torch.cuda.synchronize()
    refs = [oracle_reference(orc, np.array([T]), np.array([p]), Y.reshape(-1, 1), dt)[:2]
            for (i, j, T, p, Y, dt) in sample]

    def reset():
        for d in dev_boxes:
            d["Y"].copy_(d["Y0"])
            d["T"].copy_(d["T0"])

    def sample_errors():
        errs = []
        for (i, j, T, p, Y, dt), (Yr, Tr) in zip(sample, refs):
            Yg = dev_boxes[i]["Y"][:, j].cpu().numpy().reshape(-1, 1)
            Tg = dev_boxes[i]["T"][j].cpu().numpy().reshape(1)
            errs.append(rel_errors(Yg, Tg, Yr, Tr))
        return max(e[0] for e in errs), max(e[1] for e in errs)

    sweep_rows = []
    with torch.cuda.stream(stream):
        probe = chem.Context(mech, stream=stream, use_graph=0)
        for r in [x for x in RTOLS if x <= rtol]:
            reset()
            st = probe.integrate_boxes(dev_boxes, r, ATOL)
            rel, dT = sample_errors()
            ok = rel <= BUDGET_REL and dT <= BUDGET_T and st["n_incomplete"] == 0
            sweep_rows.append({"rtol": r, "max_rel": rel, "max_dT_K": dT, "meets_budget": ok})
            if ok:
                rtol = r
                break

    def timed(fn, reps=3):
        with torch.cuda.stream(stream):
            reset()
            fn()
            ms = []
            for _ in range(reps):
                reset()
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
                fn()
                ev1.record(stream)
                torch.cuda.synchronize()
                ms.append(ev0.elapsed_time(ev1))
        return float(np.median(ms))

    res = {}
    with torch.cuda.stream(stream):
        per = chem.Context(mech, stream=stream, use_graph=0)
        res["per_box_launches"] = timed(lambda: [per.integrate(d["rho"], d["e"], d["Y"], d["T"], d["dt"], rtol,
                                                               ATOL, status=d["status"], stats=False)
                                                 for d in dev_boxes])
        g = chem.Context(mech, stream=stream, use_graph=1)
        res["graph_default"] = timed(lambda: g.integrate_boxes(dev_boxes, rtol, ATOL, stats=False))
        tuned = chem.Context(mech, stream=stream, use_graph=1)
        reset()
        t0 = time.perf_counter()
        tuned_opts, tune_ms = tuned.autotune(dev_boxes, rtol, ATOL)
        t_tune = time.perf_counter() - t0
        res["graph_autotuned"] = timed(lambda: tuned.integrate_boxes(dev_boxes, rtol, ATOL, stats=False))
        l12 = [d for d in dev_boxes if d["level"] >= 1]
        l2 = [d for d in dev_boxes if d["level"] == 2]
        c12 = chem.Context(mech, stream=stream, use_graph=1, **tuned_opts)
        c2 = chem.Context(mech, stream=stream, use_graph=1, **tuned_opts)

        def subcycled():
            tuned.integrate_boxes(dev_boxes, rtol, ATOL, stats=False)
            c12.integrate_boxes(l12, rtol, ATOL, stats=False)
            c2.integrate_boxes(l2, rtol, ATOL, stats=False)
            c2.integrate_boxes(l2, rtol, ATOL, stats=False)
        res["subcycled_graph_autotuned"] = timed(subcycled)
        sub_cells = sum(d["rho"].numel() * (1 << d["level"]) for d in dev_boxes)
        # one eager call for the statistics, then the sample against the oracle
        tuned.set_option("use_graph", 0)
        reset()
        st = tuned.integrate_boxes(dev_boxes, rtol, ATOL)
    torch.cuda.synchronize()
    rel, dT = sample_errors()
    ms = res["graph_autotuned"]
    out = {"workload": f"AMR batching: 400 boxes over 3 levels ({ntot} cells), jet-in-crossflow-like field, "
                       "dt 4e-8/2e-8/1e-8 s by level, 9-species mechanism",
           "rtol": rtol, "atol": ATOL, "value": ntot / (ms * 1e-3), "unit": "cell-steps/s",
           "ms_per_step": ms, "ms_per_step_variants": res,
           "speedup_graph_autotuned_vs_per_box": res["per_box_launches"] / ms,
           "tuned_options": tuned_opts, "autotune_s": t_tune, "autotune_best_call_ms": tune_ms,
           "subcycled": {"cell_steps_per_coarse_step": sub_cells,
                         "ms_per_coarse_step": res["subcycled_graph_autotuned"],
                         "cell_steps_per_s": sub_cells / (res["subcycled_graph_autotuned"] * 1e-3)},
           "oracle_sample": {"cells": len(sample), "max_rel": rel, "max_dT_K": dT,
                             "meets_budget": rel <= BUDGET_REL and dT <= BUDGET_T},
           "fixed_error_sweep": sweep_rows,
           "stats": {k: st[k] for k in ("n_active0", "n_active_after_bulk", "n_bulk_rounds", "steps_total",
                                        "t_total_ms", "t_screen_ms", "t_bulk_ms", "t_sparse_ms")}}
    if quiet:
        return out
    out.update({"metric": METRIC, "n_gpus": 1, "steps": 3, "warmup": 1, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                "config": {"workload": out["workload"], "rtol": rtol, "atol": ATOL}})
    return out


# ------------------------------------------------------------ surrogate
def bench_surrogate(args, torch, chem, fields, oracle, rtol):
    """The surrogate configuration: a detonation-style evaluation field of
    256 x 256 x 128 = 8,388,608 cells (seed 1005), implicit only against the
    surrogate pass with its default trust check and implicit fallback, same
    rtol; fallback rate, accepted cells checked against the oracle."""
    cells = fields.c2_field(256, 256, 128, seed=1005)
    mech = chem.Mechanism(fields.M9_PATH)
    orc = oracle.Oracle(fields.M9_PATH)
    ctx0 = chem.Context(mech)
    F = Field(torch, ctx0, cells)
    impl = chem.Context(mech)
    ms_i, st_i = timed_calls(torch, impl, F, rtol, ATOL)
    sur = chem.Context(mech)
    sur.load_surrogate(os.path.join(ROOT, "paper_2510_23993_amd", "data", "surrogate_m9.bin"))
    sur.set_option("surrogate", 1)
    ms_s, st_s = timed_calls(torch, sur, F, rtol, ATOL)
    status = F.status.cpu().numpy()
    acc = np.where(status == chem.ST_SURR_OK)[0]
    check = {"accepted_sampled": 0}
    if acc.size:
        pick = np.sort(np.random.default_rng(7).choice(acc, size=min(200, acc.size), replace=False))
        Yr, Tr, _ = oracle_reference(orc, cells.T[pick], cells.p[pick], cells.Y[:, pick], cells.dt)
        rel, dT = rel_errors(F.Y[:, pick].cpu().numpy(), F.T[pick].cpu().numpy(), Yr, Tr)
        check = {"accepted_sampled": int(pick.size), "max_rel": rel, "max_dT_K": dT,
                 "meets_budget": rel <= BUDGET_REL and dT <= BUDGET_T}
    n_act = st_s["n_active0"]
    return {"workload": f"surrogate evaluation field 256x256x128 ({cells.T.size} cells, seed 1005), dt 5e-9 s",
            "rtol": rtol, "atol": ATOL, "surr_rtol": sur.get_option("surr_rtol"),
            "implicit_only_ms": ms_i, "surrogate_ms": ms_s, "speedup_vs_implicit_only": ms_i / ms_s,
            "active_cells": n_act, "accepted": st_s["n_surrogate"], "fallback": st_s["n_fallback"],
            "fallback_rate": st_s["n_fallback"] / max(1, n_act), "surrogate_pass_ms": st_s["t_surrogate_ms"],
            "first_failed_check_counts": dict(zip(("envelope", "Y_floor", "T_consistency", "self_consistency"),
                                                  st_s["surr_reject"])),
            "accepted_vs_oracle": check}


# ------------------------------------------------------------ Strang coupling
def bench_strang(args, torch, chem, fields):
    """Strang-split reacting steps (flow dt/2, chemistry dt, flow dt/2) on a
    one-dimensional detonation-like tube of 2^21 = 2,097,152 cells: the
    detonation patch's profile along x (cold premixed H2-air at rest ahead,
    a shocked induction band moving at 300 m/s, burnt gas at 600 m/s behind),
    dx 2e-5 m, dt 4e-9 s (CFL about 0.35), chemistry FP64 bulk-sparse at
    rtol 1e-5 / atol 1e-14 (the detonation patch's fixed-error tolerance).
    Reports the device time of the flow half steps against the chemistry's,
    i.e. chemistry's share of the reacting step."""
    n = 1 << 21
    dx, dt, rtol = 2e-5, 4e-9, args.rtol or 1e-5
    mech = chem.Mechanism(fields.M9_PATH)
    ctx = chem.Context(mech)
    c = fields.c2_field(n, 1, 1)
    dev = torch.device("cuda")
    T0 = torch.as_tensor(c.T, device=dev)
    p = torch.as_tensor(c.p, device=dev)
    Y = torch.as_tensor(c.Y, device=dev).contiguous()
    u = torch.as_tensor(np.where(c.cls == 2, 600.0, np.where(c.cls == 1, 300.0, 0.0)), device=dev)
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    e = torch.empty_like(rho)
    ctx.prepare_state(T0, p, Y, rho, e)
    U0 = torch.empty((3 + mech.ns, n), dtype=torch.float64, device=dev)
    U0[0] = rho
    U0[1] = rho * u
    U0[2] = rho * (e + 0.5 * u * u)
    U0[3:] = rho * Y
    U, T = U0.clone(), T0.clone()
    ctx.strang_step(U, T, dx, dt, rtol, ATOL)          # warm-up
    K = args.steps
    rows = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        st = ctx.strang_step(U, T, dx, dt, rtol, ATOL)
        rows.append((st["t_flow_ms"], st["t_total_ms"], st["n_active0"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flow = float(np.mean([r[0] for r in rows]))
    chem_ms = float(np.mean([r[1] for r in rows]))
    bytes_half = 2 * 8 * (3 + mech.ns) * n          # read and write U once per flow half step
    out = {"metric": METRIC, "value": n * K / wall, "unit": "cell-steps/s", "n_gpus": 1, "steps": K,
           "warmup": 1, "ms_per_step": 1e3 * wall / K, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"Strang-split reacting steps on a 1-D detonation-like tube ({n} cells), "
                                  f"dx {dx} m, dt {dt} s, HLLC + MUSCL + SSP-RK2 flow, 9-species chemistry",
                      "rtol": rtol, "atol": ATOL},
           "flow_ms_per_step": flow, "chemistry_ms_per_step": chem_ms,
           "chemistry_share_of_device_time": chem_ms / (chem_ms + flow),
           "active_cells_per_step": [r[2] for r in rows],
           "flow_roofline": {"bound": "hbm", "achieved": bytes_half / (0.5 * flow * 1e-3) / 1e9,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": bytes_half / (0.5 * flow * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "algorithmic_bytes": "one read and one write of U per half step"}}
    print(json.dumps(out))


# ------------------------------------------------------------ 53 species
def bench_contract(args, torch, chem, fields):
    """The stoichiometric contractions of the matrix-form rates alone
    (chem_eval_contractions) on batches of states, FP64 and FP32 sparse loops
    against the BF16 matrix cores with the three-term split: 8,388,608
    states of the 9-species mechanism and 1,048,576 of the 53-species one,
    ln C uniform in [-45, 8]; median of 5 launches each (HIP events)."""
    out = {"workload": "stoichiometric contractions nu'^T ln C and nu''^T ln C", "runs": []}
    for path, n in ((fields.M9_PATH, 1 << 23), (fields.M53_PATH, 1 << 20)):
        mech = chem.Mechanism(path)
        ctx = chem.Context(mech)
        g = torch.Generator(device="cuda").manual_seed(7)
        lnC = torch.rand((mech.ns, n), dtype=torch.float64, device="cuda", generator=g) * 53.0 - 45.0
        zf = torch.empty((mech.nr, n), dtype=torch.float64, device="cuda")
        zr = torch.empty_like(zf)
        kt, nt = (mech.ns + 31) // 32, (2 * mech.nr + 15) // 16
        for prec in (0, 1, 2):
            ms = []
            for _ in range(6):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                ctx.eval_contractions(lnC, zf, zr, prec)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            t = float(np.median(ms[1:]))
            row = {"nspec": mech.ns, "nreac": mech.nr, "states": n, "precision": prec, "ms": t,
                   "ns_per_state": t * 1e6 / n,
                   "hbm_bytes": 8 * n * (mech.ns + 2 * mech.nr),
                   "hbm_GBps": 8 * n * (mech.ns + 2 * mech.nr) / (t * 1e-3) / 1e9}
            if prec == 2:
                issued = 2.0 * 16 * 16 * 32 * 3 * kt * nt * (n / 16)
                row["mfma_issued_TFLOPs"] = issued / (t * 1e-3) / 1e12
            out["runs"].append(row)
    print(json.dumps(out))


def bench_m53(args, torch, chem, fields, oracle):
    """53-species / 325-reaction mechanism, n cells of the seeded T/p/progress
    distribution, dt 1e-7 s, FP64 at rtol 1e-7 / atol 1e-20 (the loosest
    tolerance at which the FP64 oracle meets 1e-4 relative on species above
    1e-10 on this mechanism), 64 lanes per cell, no bulk rounds.  The cells
    may be split into `chunks` consecutive calls (each prints a progress
    line).  The CPU oracle runs on a stratified sample (by temperature
    decile) and its full-field time is extrapolated; a smaller stratified
    sample (4 cells per decile) is checked against the oracle at rtol 1e-10 /
    atol 1e-20 for the 1e-4 / 1 K budget."""
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    mech = chem.Mechanism(fields.M53_PATH)
    cells = fields.c4_cells(args.cells, seed=1004)
    n = cells.T.size
    ctx = chem.Context(mech, group=64, max_rounds=0)
    ctx0 = chem.Context(mech)
    chunk = (n + args.chunks - 1) // args.chunks
    total_ms, steps, incomplete = 0.0, 0, 0
    dec = np.minimum((cells.T - 800.0) / 180.0, 9).astype(int)
    chk = stratified_sample(dec, {k: 4 for k in range(10)}, seed=2004)
    Ychk, Tchk = np.zeros((mech.ns, chk.size)), np.zeros(chk.size)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        sub = fields.Cells(T=cells.T[c0:c1], p=cells.p[c0:c1], Y=np.ascontiguousarray(cells.Y[:, c0:c1]),
                           dt=cells.dt)
        F = Field(torch, ctx0, sub)
        F.reset()
        st = ctx.integrate(F.rho, F.e, F.Y, F.T, F.dt, 1e-7, 1e-20, status=F.status)
        total_ms += st["t_total_ms"]
        sel = np.where((chk >= c0) & (chk < c1))[0]
        if sel.size:
            loc = torch.as_tensor(chk[sel] - c0, device=F.Y.device)
            Ychk[:, sel] = F.Y[:, loc].cpu().numpy()
            Tchk[sel] = F.T[loc].cpu().numpy()
        steps += st["steps_total"]
        incomplete += st["n_incomplete"]
        log(json.dumps({"cells": [c0, c1], "ms": st["t_total_ms"], "incomplete": st["n_incomplete"]}))
        del F
    out = {"metric": METRIC, "value": n / (total_ms * 1e-3), "unit": "cell-steps/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": total_ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"53-species/325-reaction synthetic mechanism, {n} cells, dt 1e-7 s, "
                                  f"{args.chunks} call(s) of up to {chunk} cells",
                      "rtol": 1e-7, "atol": 1e-20, "schedule": "64 lanes per cell, no bulk rounds"},
           "steps_total": steps, "incomplete": incomplete}
    orc = oracle.Oracle(fields.M53_PATH)
    rho_c, e_c = orc.state_from_TPY(cells.T[chk], cells.p[chk], cells.Y[:, chk])
    Yr, Tr, so = orc.integrate(rho_c, e_c, cells.Y[:, chk], cells.dt, 1e-10, 1e-20, T=cells.T[chk],
                               nthreads=len(os.sched_getaffinity(0)))
    rel, dT = rel_errors(Ychk, Tchk, Yr, Tr)
    out["oracle_check"] = {"cells": int(chk.size), "reference": "oracle at rtol 1e-10 / atol 1e-20",
                           "max_rel": rel, "max_dT_K": dT, "meets_budget": rel <= BUDGET_REL and dT <= BUDGET_T}
    if not args.no_cpu:
        idx = stratified_sample(dec, {k: 26 for k in range(10)}, seed=1004)
        rho, e = orc.state_from_TPY(cells.T[idx], cells.p[idx], cells.Y[:, idx])
        threads = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        orc.integrate(rho, e, cells.Y[:, idx], cells.dt, 1e-7, 1e-20, T=cells.T[idx], nthreads=threads)
        wall = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": idx.size / wall, "unit": "cell-steps/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{idx.size} cells stratified by temperature decile, rtol 1e-7 / atol "
                                         f"1e-20, {wall:.2f} s wall; full-field time extrapolated: "
                                         f"{n * wall / idx.size:.0f} s"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
