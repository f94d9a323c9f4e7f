"""Throughput of the geodesic tracer on one MI355X.

One step = one full trace of the workload frame: every pixel, every
integration pass and the FP64 hit refinement, with the metric, scene and
output buffers already resident in HBM.  `value` is rays per second.

The JSON line also carries
  roofline      the integration-pass kernel against the FP32 vector peak:
                algorithmic FLOPs (counted per lane by the instrumented
                kernel variant, priced with the per-unit figures below)
                divided by the pass kernels' HIP-event time inside the
                timed region;
  cpu_baseline  the FP64 oracle timed on the host cores on a bounded,
                seeded pixel sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3      # MI355X FP32 vector, published (counts packed FMA)
FP32_PEAK_NONPACKED = 78.6    # 256 CU x 128 FP32 lanes-flops/clk x 2.4 GHz without packed math

# Algorithmic FLOPs per unit (FMA = 2, each transcendental = 1); derived
# from the formulas the kernels evaluate ("FLOP model").
FLOPS = {
    "graph_eval": 16,        # |y|^2, 1 + |grad f|^2, rcp, scale
    "graph_bump": 27,        # one bump inside its cut sphere (incl. exp2)
    "twist_eval": 208,       # J, D^2 phi[y,y], Sherman-Morrison solve (incl. 6 transcendentals)
    "ztwist_eval": 40,
    "rk4_step": 109,         # stage states, combination, TwoSum position update, chord length
    "euler_step": 35,
    "dp5_attempt": 460,      # 6 stages' states, 5th-order update, embedded error, control
    "obj_test": 20,          # one segment-object test
}


def algorithmic_flops(kind, step, st):
    ev = st["acc_evals"]
    if kind == 1:
        f = FLOPS["graph_eval"] * ev + FLOPS["graph_bump"] * st["bump_evals"]
    elif kind == 2:
        f = FLOPS["twist_eval"] * ev
    elif kind == 3:
        f = FLOPS["ztwist_eval"] * ev
    else:
        f = 0
    if step == 0:
        f += FLOPS["rk4_step"] * st["ray_steps"]
    elif step == 1:
        f += FLOPS["dp5_attempt"] * st["attempts"]
    else:
        f += FLOPS["euler_step"] * st["ray_steps"]
    f += FLOPS["obj_test"] * st["obj_tests"]
    return f


def cpu_baseline(wl, budget_s):
    """FP64 oracle on a seeded pixel sample, stopping after budget_s."""
    import numpy as np

    import oracle
    import workloads as W
    cam, rule = wl["camera"], wl["rule"]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    pix = W.pixel_sample(cam["width"], cam["height"], 200000, seed=11)
    done, steps, t0 = 0, 0, time.perf_counter()
    chunk = 16 * threads
    while done < len(pix) and time.perf_counter() - t0 < budget_s:
        r = orc.trace(cam, rule, pix[done:done + chunk], nthreads=threads)
        steps += int(r["steps"].sum())
        done += len(r["id"])
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "ray_steps_per_s": steps / dt,
            "sample": "%d seeded pixels (seed 11) of the %dx%d frame, FP64, no culling, %.1f s" % (
                done, cam["width"], cam["height"], dt)}


def bench_adjoint(args, wl, torch, rt):
    """One step = forward trace with the adjoint tape + masked L2 loss against
    the target map + the adjoint, for every set and pixel."""
    cam, rule = wl["camera"], dict(wl["rule"])
    ck = wl["ckpt_every"]
    tr = rt.Tracer(0)
    tr.set_scene(wl["scene"])
    tr.set_metric(dict(wl["metric"], bumps=wl["target_bumps"]))
    target = tr.trace(cam, rule)
    tr.set_metric(wl["metric"])
    nb = wl["metric"]["bumps"].shape[1]
    out, tape = tr.trace_fwd_ckpt(cam, rule, rule["max_steps"], ck)
    print("[bench] adjoint workload %s: %d sets x %dx%d, tape %.2f GB" % (
        args.workload, tr.n_sets, cam["width"], cam["height"], tape.numel() * 4 / 1e9), flush=True)

    def step():
        tr.trace_fwd_ckpt(cam, rule, rule["max_steps"], ck, out=out, tape=tape)
        e1.record()
        loss, gh = tr.loss_l2(cam, out["hit"], out["id"], target["hit"], target["id"])
        g = tr.trace_bwd(tape, gh, nb)
        return loss, g

    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fwd_ms = tot_ms = 0.0
    for _ in range(args.steps):
        e0.record()
        loss, g = step()
        e2.record()
        torch.cuda.synchronize()
        fwd_ms += e0.elapsed_time(e1)
        tot_ms += e0.elapsed_time(e2)
    st = tr.stats()
    n_rays = tr.n_sets * cam["width"] * cam["height"]
    ms = tot_ms / args.steps
    line = {
        "metric": "differentiable trace: rays/s for forward + adjoint (64 sets x 512^2, 8 bumps)",
        "value": n_rays / (ms / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "width": cam["width"], "height": cam["height"], "n_sets": tr.n_sets,
                   "bumps": nb, "h": rule["h"], "max_steps": rule["max_steps"], "ckpt_every": ck},
        "forward_ms": fwd_ms / args.steps, "backward_ms": (tot_ms - fwd_ms) / args.steps,
        "tape_gb": tape.numel() * 4 / 1e9, "ray_steps_forward": st["ray_steps"],
        "loss_mean": float(loss.mean()), "grad_abs_max": float(g.abs().max()),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bumps16_1080p")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); DESIGN.md describes how the trace "
              "would shard across GPUs, but no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2005_05386_amd import rt

    wl = W.get(args.workload)
    if "ckpt_every" in wl:
        return bench_adjoint(args, wl, torch, rt)
    cam, rule = wl["camera"], dict(wl["rule"])
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    out = tr.alloc_outputs(cam)
    ms_steps = rule["max_steps"]
    print("[bench] workload %s %dx%d x%d sets, warmup %d" % (args.workload, cam["width"], cam["height"],
                                                          tr.n_sets, args.warmup), flush=True)
    for _ in range(args.warmup):
        tr.trace_into(cam, rule, ms_steps, out)
    torch.cuda.synchronize()

    # instrumented run (untimed): per-lane algorithmic work
    tr.trace_into(cam, dict(rule, flags=rt.FLAG_COUNT_WORK), ms_steps, out)
    work = tr.stats()
    print("[bench] work counted: %s" % json.dumps(work), flush=True)

    # timed region: K traces, per-kernel HIP events on the trace stream
    stream = torch.cuda.current_stream()
    timed_rule = dict(rule, flags=rt.FLAG_TIMING)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    pass_ms = refine_ms = compact_ms = 0.0
    n_pass_launches = 0
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        tr.trace_into(cam, timed_rule, ms_steps, out)
        st = tr.stats()  # waits for this trace; reads its kernel times
        pass_ms += st["pass_ms"]
        refine_ms += st["refine_ms"]
        compact_ms += st["compact_ms"]
        n_pass_launches += st["passes"]
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    n_rays = tr.n_sets * cam["width"] * cam["height"]

    flops = algorithmic_flops(wl["metric"]["kind"], rule["kind"], work)
    pass_s = pass_ms / 1e3 / args.steps
    achieved = flops / pass_s / 1e12
    line = {
        "metric": "rays/s & RK4 ray-steps/s (1080p, 16 bumps); surrogate vs RK4 at equal error",
        "value": n_rays / (ms / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "width": cam["width"], "height": cam["height"],
                   "n_sets": tr.n_sets, "step_rule": ["RK4", "RK45", "Euler"][rule["kind"]], "h": rule["h"],
                   "max_steps": ms_steps, "bumps": int(wl["metric"]["bumps"].shape[1]),
                   "spheres": int(len(wl["scene"]["spheres"]))},
        "ray_steps_per_s": work["ray_steps"] / (ms / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_trace_pass", "flops_per_trace": flops,
                     "kernel_ms_per_launch": pass_ms / max(1, n_pass_launches),
                     "frac_of_nonpacked_peak": achieved / FP32_PEAK_NONPACKED},
        "kernel_ms": {"passes": pass_ms / args.steps, "refine": refine_ms / args.steps,
                      "compaction": compact_ms / args.steps},
        "work": {"ray_steps": work["ray_steps"], "acc_evals": work["acc_evals"],
                 "bump_evals": work["bump_evals"], "obj_tests": work["obj_tests"],
                 "mean_active_bumps_per_eval": work["bump_evals"] / max(1, work["acc_evals"]),
                 "wave_list_bumps_per_iter": work["bump_list_sum"] / max(1, work["wave_iters"]),
                 "wave_list_objects_per_iter": work["obj_list_sum"] / max(1, work["wave_iters"]),
                 "lane_occupancy": work["lane_iters"] / max(1, 64 * work["wave_iters"]),
                 "refined": work["refined"], "passes": work["passes"]},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host (%.0f s budget)" % args.cpu_budget, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
