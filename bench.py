#!/usr/bin/env python3
"""Benchmark: block-updates/s of the multiresolution step on one MI355X.

Workload: the 2D swirl set-up (three seeded Gaussian blobs, beta = 0.01, Bs = 33,
Jmax = 7, eps = 1e-4, dt = 2^-13, 500 steps).  A step is the whole hot path:
refine all blocks (safety zone), one RK4 step with ghost synchronisation on the
refined grid, and multiresolution analysis + coarsening until nothing merges.
value = sum over timed steps of the refined block count |G~| / wall time.

Forms timed: FP64 plain (stored ghosts, per-level launches), FP64 fused and
mixed fused (FP32 stencil and slopes, FP64 state).  The headline value is the
mixed fused form.  Per-kernel device times come from HIP events on the solver's
stream in a second, instrumented pass over the same steps.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "block-updates/s (RK4 step, all blocks) FP64 vs mixed; % HBM roofline"


def counter_traffic(key):
    """HBM bytes per stage launch from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE runs, scaled by a copy calibration), or None if the kernel source
    changed since the counters were taken."""
    import hashlib
    if key is None:
        return None
    path = os.path.join(ROOT, "profiles", "stage_traffic_counters.md")
    src = os.path.join(ROOT, "paper_1902_00088_amd", "csrc", "kernels.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("traffic_sha256:"):
            vals["sha"] = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch " + key + ":"):
            vals["bytes"] = float(line.split(":", 1)[1])
    if vals.get("sha") != sha or "bytes" not in vals:
        return None
    return vals["bytes"]


def traffic_key(wl, form, kind):
    """Key of the counter summary for the dominant kernel of a form's run (stage launches
    or the overlapped-tile step with what it folds in), or None."""
    if kind == "stage":
        return f"{wl} nsub {form['stage_tiles']}" + tkey(form)
    if kind == "rk4_tile":
        r = form.get("rk4_tile") or {}
        a = r.get("analysis_folded") or [0, 256]
        f = r.get("refine_folded") or [0, 0, 256]
        mo = r.get("mothers_folded") or [0, 256]
        if a[0] > 0 and f[0] and mo[0] > 0:
            return f"{wl} rk4_tile nsub {mo[0]} t{mo[1]} analysis refine mothers"
        if a[0] > 0 and f[0] and f[1] > 0:
            return f"{wl} rk4_tile nsub {f[1]} t{f[2]} analysis refine"
        if a[0] > 0:
            return f"{wl} rk4_tile nsub {a[0]} t{a[1]} analysis" + (" refine" if f[0] else "")
        return f"{wl} rk4_tile nsub {r.get('tiles')}"
    return None


def tkey(form):
    """Key suffix of the counter summary for the stage kernel's threads per workgroup."""
    t = form.get("stage_threads") or 256
    return "" if t == 256 else f" t{t}"


def run_form(M, W, torch, cfg, steps, warmup, tune=False):
    s = M.Solver(cfg)
    s.init_grid()
    lv0, co0 = s.read_forest()
    data0 = s.read_blocks()

    def reset():
        s.init_forest(lv0, co0)
        s.load_blocks(data0)
        torch.cuda.synchronize()

    if tune:
        # set-up, before the warm-up: the autotuner on the refined initial grid, then 20
        # steps for the library's choice between graph replay and direct launches (ten
        # each way), so that no probing happens inside the timed region
        s.refine_all()
        s.tune(reps=3)
        reset()
        s.step(0.0, cfg.dt, 20)
        reset()
    t = 0.0
    for _ in range(warmup):
        s.step(t, cfg.dt)
        t += cfg.dt

    # timed pass (no per-kernel instrumentation)
    reset()
    st0 = s.stats()
    b0 = st0["block_updates"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(0.0, cfg.dt, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = s.stats()
    tiles = st["stage_tiles"]
    host_us = {k: (v - st0["host_us"][k]) / steps for k, v in st["host_us"].items()}
    bu = st["block_updates"] - b0
    wall = t1 - t0
    final_blocks = st["blocks"]
    # instrumented pass: per-kernel device time from HIP events
    reset()
    s.timing(True)
    s.step(0.0, cfg.dt, steps)
    kst = s.stats()["kernels"]
    s.timing(False)
    s.close()
    # the RK4 sweep's kernels (the overlapped-tile launch also holds the refinement and
    # the first analysis where those are folded in)
    sweep_ms = sum(kst[k]["ms"] for k in ("stage", "ghost", "rhs_plain", "rk4_tile") if k in kst)
    return {
        "value": bu / wall,
        "ms_per_step": 1e3 * wall / steps,
        "block_updates": bu,
        "blocks_initial": int(len(lv0)),
        "blocks_final": final_blocks,
        "sweep_block_updates_per_s": bu / (sweep_ms * 1e-3) if sweep_ms > 0 else None,
        "kernels": kst,
        "host_us_per_step": host_us,
        "stage_tiles": tiles,
        "stage_threads": st.get("stage_threads"),
        "sweep_launch": st.get("sweep_launch"),
        "rk4_tile": {"tiles": st.get("rk4_tile_tiles"), "analysis_folded": st.get("rk4_tile_analysis"),
                     "refine_folded": st.get("rk4_tile_refine"), "mothers_folded": st.get("rk4_tile_mothers")},
        "tune_ms": st.get("tune_ms"),
        "graph_in_use": st.get("graph_in_use"),
        "memo_hits": st.get("memo_hits"),
        "spec_hits": st.get("spec_hits"),
        "spec_misses": st.get("spec_misses"),
    }


FIELD_NAMES = {1: ["phi"], 4: ["rho", "u", "v", "p"]}


def mixed_accuracy(M, W, cfg, steps):
    """Accuracy of the mixed fused form against the FP64 fused form (which equals the FP64
    oracle bit for bit in the parity tests), both started from the FP64 initial grid, with
    the FP64 run's coarsening flags replayed on the mixed run (same topology every step).
    Per field: max|mixed - fp64| / max|fp64| and the relative 2-norm after `steps` steps;
    also how many block flags the mixed state's own analyses set differently."""
    import numpy as np
    s64 = M.Solver(cfg.replace(precision=W.FP64, form=W.FORM_FUSED))
    s32 = M.Solver(cfg.replace(precision=W.MIXED, form=W.FORM_FUSED))
    s64.init_grid()
    lv, co = s64.read_forest()
    s32.init_forest(lv, co)
    s32.load_blocks(s64.read_blocks())
    t, flags_total, flags_differ, analyses = 0.0, 0, 0, 0
    for _ in range(steps):
        for s in (s64, s32):
            s.refine_all()
            s.rk4(t, cfg.dt)
        while True:
            f64, _ = s64.mr_pass()
            f32, _ = s32.mr_pass()
            analyses += 1
            flags_total += len(f64)
            flags_differ += int(np.sum(f64 != f32))
            n = s64.coarsen(f64)
            s32.coarsen(f64)
            if n == 0:
                break
        t += cfg.dt
    a, b = s32.read_blocks(), s64.read_blocks()
    same_forest = all(np.array_equal(x, y) for x, y in zip(s32.read_forest(), s64.read_forest()))
    s64.close()
    s32.close()
    names = FIELD_NAMES.get(cfg.nf, [f"f{i}" for i in range(cfg.nf)])
    inf = np.max(np.abs(a - b), axis=(0, 2)) / np.maximum(np.max(np.abs(b), axis=(0, 2)), 1e-300)
    l2 = np.sqrt(np.sum((a - b) ** 2, axis=(0, 2)) / np.maximum(np.sum(b * b, axis=(0, 2)), 1e-300))
    return {"steps": steps, "topology": "FP64 run's flags replayed", "same_forest": bool(same_forest),
            "rel_inf_per_field": {k: float(v) for k, v in zip(names, inf)},
            "rel_l2_per_field": {k: float(v) for k, v in zip(names, l2)},
            "max_rel_inf": float(np.max(inf)), "within_1e-5": bool(np.max(inf) <= 1e-5),
            "own_flags_differing": flags_differ, "flags_compared": flags_total, "analyses": analyses}


def speedup_entry(res, acc, fast="mixed_fused", base="fp64_plain"):
    """Speedup of one form over another on the same GPU, stated with the accuracy of the
    mixed form measured on the same workload."""
    if fast not in res or base not in res:
        return None
    return {"speedup": res[fast]["value"] / res[base]["value"], "of": fast, "over": base,
            "max_rel_inf_error_of_mixed": acc["max_rel_inf"] if acc else None,
            "within_1e-5": acc["within_1e-5"] if acc else None}


def _oracle_rate(oracle, cfg, budget_s):
    """Block-updates/s of the oracle's plain steps from the workload's initial grid."""
    o = oracle.Oracle(cfg)
    o.init_grid()
    t = 0.0
    nbu = 0
    nsteps = 0
    elapsed = 0.0
    while elapsed < budget_s or nsteps < 3:
        t0 = time.perf_counter()
        o.refine_all()
        nbu += o.num_blocks()
        o.rk4(t, cfg.dt)
        o.adapt()
        elapsed += time.perf_counter() - t0
        t += cfg.dt
        nsteps += 1
    return nbu / elapsed, (f"first {nsteps} steps of the same workload from the same initial grid "
                           f"({nbu} block-updates in {elapsed:.1f} s)")


def cpu_model():
    """The host CPU's model name, with its family, model and clock as /proc/cpuinfo gives them
    (a virtual machine may shorten the name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = line.split(":", 1)
                info.setdefault(k.strip(), v.strip())
    except OSError:
        pass
    name = info.get("model name")
    if not name:
        import platform
        return platform.processor() or None
    extra = [f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info]
    if "cpu MHz" in info:
        extra.append(f"{float(info['cpu MHz']):.0f} MHz")
    return name + (f" ({', '.join(extra)})" if extra else "")


def cpu_baseline(W, cfg, budget_s):
    import ctypes
    import oracle
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    value, sample = _oracle_rate(oracle, cfg, budget_s)
    out = {"value": value, "unit": "block-updates/s", "cores": cores, "kind": "oracle", "sample": sample,
           "cpu_model": cpu_model(), "host_threads_available": os.cpu_count()}
    # the same on one thread (OpenMP of the oracle's library set to 1 for the sample)
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        v1, s1 = _oracle_rate(oracle, cfg, budget_s / 3)
        gomp.omp_set_num_threads(cores)
        out["single_thread"] = {"value": v1, "cores": 1, "sample": s1}
    except (OSError, AttributeError):   # no separate OpenMP runtime to set: all-threads figure only
        pass
    return out


def headline(args, res, acc=None):
    """The JSON line's headline fields from the 2D swirl forms (acc: the mixed form's accuracy)."""
    head = res.get("mixed_fused") or next(iter(res.values()))
    head_name = "mixed_fused" if "mixed_fused" in res else next(iter(res))
    ks = head["kernels"]
    dom = max(ks, key=lambda k: ks[k]["ms"])
    ach = ks[dom]["bytes"] / (ks[dom]["ms"] * 1e-3) / 1e9 if ks[dom]["ms"] > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS,
                "traffic": counter_traffic(traffic_key("c2", head, dom)),
                "traffic_unit": "bytes per launch", "kernel": dom,
                "algorithmic_bytes_per_launch": ks[dom]["bytes"] / max(1, ks[dom]["launches"]),
                "launches": ks[dom]["launches"], "avg_launch_us": 1e3 * ks[dom]["ms"] / max(1, ks[dom]["launches"])}
    return {
        "metric": METRIC,
        "value": head["value"],
        "unit": "block-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-stencil/f64-state" if head_name.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": f"C2 2D swirl advection: 3 seeded Gaussian blobs (beta=0.01), Bs=33, Jmax=7, "
                               f"eps=1e-4, dt=2^-13; {args.steps} timed steps from the initial grid "
                               f"(the full run is 500 steps)", "form": head_name,
                   "blocks_initial": head["blocks_initial"], "parallelism": "single GPU"},
        "roofline": roofline,
        "forms": res,
        "speedup_mixed_fused_vs_fp64_plain": speedup_entry(res, acc),
        "mixed_accuracy": acc,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=24)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="first run a plain device copy of this many MiB five times (counter calibration)")
    ap.add_argument("--forms", default="fp64_plain,fp64_fused,mixed_fused")
    ap.add_argument("--c4-steps", type=int, default=20, help="steps of the 3D workload (0 = skip)")
    ap.add_argument("--c4-forms", default="fp64_plain,fp64_fused,mixed_fused")
    ap.add_argument("--acc-steps", type=int, default=40,
                    help="steps of the mixed-vs-FP64 accuracy runs (C2; C3 and C4 take half; 0 = skip)")
    ap.add_argument("--c3-steps", type=int, default=20, help="steps of the Navier-Stokes workload (0 = skip)")
    ap.add_argument("--c3-forms", default="fp64_plain,fp64_fused,mixed_fused")
    ap.add_argument("--no-tune", action="store_true", help="default tilings instead of the autotuner")
    ap.add_argument("--c5-steps", type=int, default=2000,
                    help="recorded steps of the learned-predictor study (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the multi-GPU path (sharding the block forest along the "
              f"space-filling curve) is not built, so --gpus {args.gpus} is not supported.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    import paper_1902_00088_amd as M

    if args.copy_calib > 0:
        n = args.copy_calib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    base = W.C2()
    forms = {"fp64_plain": (W.FP64, W.FORM_PLAIN), "fp64_fused": (W.FP64, W.FORM_FUSED),
             "mixed_fused": (W.MIXED, W.FORM_FUSED)}
    res = {}
    for name in [f for f in args.forms.split(",") if f and f != "none"]:
        prec, form = forms[name]
        print(f"bench: {name} steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
        res[name] = run_form(M, W, torch, base.replace(precision=prec, form=form), args.steps, args.warmup,
                             tune=form == W.FORM_FUSED and not args.no_tune)
    out = {}
    acc2 = None
    if args.acc_steps > 0:
        print(f"bench: C2 mixed accuracy steps={args.acc_steps}", file=sys.stderr, flush=True)
        acc2 = mixed_accuracy(M, W, base, args.acc_steps)
    if res:
        out = headline(args, res, acc2)
    if args.c4_steps > 0:
        # the 3D set-up: a ragged forest of ~3,000 blocks of 17^3 after refine-all, HBM bound
        c4 = {}
        for name in [f for f in args.c4_forms.split(",") if f]:
            prec, form = forms[name]
            print(f"bench: C4 {name} steps={args.c4_steps}", file=sys.stderr, flush=True)
            c4[name] = run_form(M, W, torch, W.C4().replace(precision=prec, form=form), args.c4_steps, 2,
                                tune=form == W.FORM_FUSED and not args.no_tune)
        acc4 = None
        if args.acc_steps > 0:
            print(f"bench: C4 mixed accuracy steps={max(1, args.acc_steps // 2)}", file=sys.stderr, flush=True)
            acc4 = mixed_accuracy(M, W, W.C4(), max(1, args.acc_steps // 2))
        out["c4"] = {"workload": f"C4 3D advection: 4 seeded blobs sigma=0.04, Bs=17^3, Jmax=6, eps=1e-4, "
                                 f"dt=2^-11; {args.c4_steps} timed steps from the initial grid",
                     "forms": c4, "mixed_accuracy": acc4,
                     "speedup_mixed_fused_vs_fp64_plain": speedup_entry(c4, acc4),
                     "speedup_mixed_fused_vs_fp64_fused": speedup_entry(c4, acc4, base="fp64_fused")}
        if "mixed_fused" in c4:
            ks4 = c4["mixed_fused"]["kernels"]["stage"]
            ach4 = ks4["bytes"] / (ks4["ms"] * 1e-3) / 1e9 if ks4["ms"] > 0 else 0.0
            out["c4"]["roofline_stage_mixed"] = {
                "bound": "hbm", "achieved": ach4, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach4 / PEAK_HBM_GBS,
                "traffic": counter_traffic(f"c4 nsub {c4['mixed_fused']['stage_tiles']}" + tkey(c4['mixed_fused'])),
                "traffic_unit": "bytes per launch",
                "algorithmic_bytes_per_launch": ks4["bytes"] / max(1, ks4["launches"]),
                "avg_launch_us": 1e3 * ks4["ms"] / max(1, ks4["launches"])}

    if args.c3_steps > 0:
        # compressible Navier-Stokes mixing layer: 4 fields, halo 4, nested derivatives
        c3 = {}
        for name in [f for f in args.c3_forms.split(",") if f]:
            prec, form = forms[name]
            print(f"bench: C3 {name} steps={args.c3_steps}", file=sys.stderr, flush=True)
            c3[name] = run_form(M, W, torch, W.C3().replace(precision=prec, form=form), args.c3_steps, 2,
                                tune=form == W.FORM_FUSED and not args.no_tune)
        acc3 = None
        if args.acc_steps > 0:
            print(f"bench: C3 mixed accuracy steps={max(1, args.acc_steps // 2)}", file=sys.stderr, flush=True)
            acc3 = mixed_accuracy(M, W, W.C3(), max(1, args.acc_steps // 2))
        out["c3"] = {"workload": f"C3 2D compressible Navier-Stokes temporal mixing layer (rho, u, v, p), Bs=33, "
                                 f"Jmax=8, eps=1e-3, Re=1000, Mach 0.4; {args.c3_steps} timed steps",
                     "forms": c3, "mixed_accuracy": acc3,
                     "speedup_mixed_fused_vs_fp64_plain": speedup_entry(c3, acc3),
                     "speedup_mixed_fused_vs_fp64_fused": speedup_entry(c3, acc3, base="fp64_fused")}
        if "mixed_fused" in c3:
            ks3 = c3["mixed_fused"]["kernels"]["stage"]
            ach3 = ks3["bytes"] / (ks3["ms"] * 1e-3) / 1e9 if ks3["ms"] > 0 else 0.0
            out["c3"]["roofline_stage_mixed"] = {
                "bound": "hbm", "achieved": ach3, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach3 / PEAK_HBM_GBS,
                "traffic": counter_traffic(f"c3 nsub {c3['mixed_fused']['stage_tiles']}" + tkey(c3['mixed_fused'])),
                "traffic_unit": "bytes per launch",
                "algorithmic_bytes_per_launch": ks3["bytes"] / max(1, ks3["launches"]),
                "avg_launch_us": 1e3 * ks3["ms"] / max(1, ks3["launches"])}

    if args.c5_steps > 0:
        from paper_1902_00088_amd import predictor as P
        c5 = {}
        for name, cfg in (("C5_mixing_layer", W.C3(precision=W.MIXED)), ("swirl_moving_fronts", base.replace(precision=W.MIXED))):
            print(f"bench: predictor study {name} steps={args.c5_steps}", file=sys.stderr, flush=True)
            s = M.Solver(cfg)
            s.init_grid()
            c5[name] = P.gain_study(s, W.mlp_init_params(64 * cfg.nf, 5), nsteps=args.c5_steps, guard=[0.0, 4.0])
            s.close()
            present = [int(v) > 0 for v in c5[name]["labels_train"]]
            c5[name]["degenerate"] = sum(present) < 2
            if c5[name]["degenerate"]:
                c5[name]["note"] = ("every training label is the same class (the recorded grid never changes), so the "
                                    "test accuracy says nothing about the predictor")
        out["predictor"] = c5
    if not args.no_cpu:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W, base, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
