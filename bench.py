"""Throughput of the geodesic tracer on one MI355X.

One step = one full trace of the workload frame: every pixel, every
integration pass and the FP64 hit refinement, with the metric, scene and
output buffers already resident in HBM.  `value` is rays per second with
--frames-in-flight frames (default 2) traced concurrently, each on its own
stream with its own context and outputs, K frames in all between two device
synchronisations; `frame_latency_ms` is one frame traced alone (a separate
serial loop of K frames, which also gives the kernel times).

The JSON line also carries
  roofline      the integration-pass kernel against the FP32 vector peak:
                algorithmic FLOPs (counted per lane by the instrumented
                kernel variant, priced with the per-unit figures below)
                divided by the pass kernels' HIP-event time in the serial
                loop (launches that do not overlap); frame_rate_tflops is
                the same FLOPs over the throughput's time per frame;
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

FP32_PEAK_TFLOPS = 157.3      # MI355X FP32 vector, published
# (measured on gfx950: a wave64 FP32 VALU instruction whose operands are all
# VGPRs or constants issues every 2 cycles, which reaches this peak without
# packed math; one that reads an SGPR takes 4 cycles, a transcendental 8)

# Algorithmic FLOPs per unit (FMA = 2, each transcendental = 1); derived
# from the formulas the kernels evaluate: FMA = 2, each transcendental = 1.
FLOPS = {
    "graph_eval": 16,        # |y|^2, 1 + |grad f|^2, rcp, scale
    "graph_bump": 27,        # one bump inside its cut sphere (incl. exp2)
    "twist_eval": 208,       # J, D^2 phi[y,y], Sherman-Morrison solve (incl. 6 transcendentals)
    "ztwist_eval": 40,
    # composed local deformations: per evaluation the 3x3 solve by the adjugate
    # (cofactors 27, determinant 5, reciprocal 1, product 15, scale 3); per
    # deformation inside its cut: d, S d, d.S d 11, exponent 2, f 1, grad f 3,
    # S d . u 5, u.S u 8, second-order term 3, grad f . w and . u 11, grad f^T M 15,
    # updates of w, u, q 18, M 18
    "deform_eval": 51,
    "deform_term": 95,
    # a deformation whose field also rotates, V = v + w x d: w x u, w x w and
    # w x (the columns of M) 45, V 12, the extra terms of w 13, u 6 and M 18
    "deform_term_rot": 189,
    # anisotropic bumps: per evaluation 1 + |grad f|^2 6, reciprocal 1, scale 4; per bump
    # inside its cut: d, S d, d.S d 11, exponent 2, w 1, grad f 6, S d . y 5, y.S y 8, q 4
    "ganiso_eval": 11,
    "ganiso_bump": 37,
    # quadratic: grad f 6, y^T H y 9, 1 + |grad f|^2 6, reciprocal and scale 5
    "gquad_eval": 26,
    # RK4: step 74 (3 stage states 36, stage sums 30, h/2 and h/6 scaling 8), x_hi + x_lo 3,
    # chord length 5, two-float position update 12 (Fast2Sum and the low part, 4 per
    # coordinate), velocity update 3
    "rk4_step": 97,
    # Euler: h y and h a 6, x_hi + x_lo 3, chord length 5, two-float update 12, velocity update 3
    "euler_step": 29,
    # DP5(4): stage states 280 (6 positions with their h^2 terms, 6 velocities), 5th-order
    # increments 66, embedded error 77, h^2 1; error norm and step control 58; x_hi + x_lo,
    # chord length, two-float position and time updates (12 + 4), velocity update 27
    "dp5_attempt": 509,
    "obj_test": 20,          # one segment-object test
    # adjoint (RK4, graph metric), per full step reversed: the stage sums
    # recomputed 4 x 16, the stage VJP overheads 4 x 32 (|y|^2 5, 1/(1 + |g|^2) 7,
    # g.abar 5, qbar 1, gbar 14) and the VJP of the RK4 combination 216;
    # per bump term inside its cut: 27 (its stage sum) + 87 (its VJP: d, |d|^2,
    # exp, w, d.y, Cw, the cotangents of d and y, and of a, c, sigma)
    "adj_rev_step": 408,
    "adj_term": 114,
    # per step recomputed from a checkpoint: one RK4 step with its 4 evaluations
    # (97 + 4 x 16) plus 27 per bump term inside its cut
    "adj_recomp_step": 161,
    # crossing generator (training data): one RK4 step in the canonical frame
    # with its single bump always inside the cut, 4 x (16 + 27) + 97
    "cross_step": 269,
    # FP64 hit refinement (graph metric): per evaluation and per bump inside
    # its cut as in FP32 (the exponential counted once, although FP64 exp is
    # a software routine); per RK4 step 80 (stage states 36, stage sums 30,
    # scaling 8, x + dx and y + dv 6); per implicit-function value 9
    "ref_eval": 16,
    "ref_bump": 27,
    "ref_rk4_step": 80,
    "ref_obj": 9,
}
FP64_PEAK_TFLOPS = 78.6       # MI355X FP64 vector, published


KERNEL_SOURCES = ["paper_2005_05386_amd/csrc/rt_trace.hip", "paper_2005_05386_amd/csrc/rt_device.hpp",
                  "paper_2005_05386_amd/csrc/rt_step.hpp", "paper_2005_05386_amd/csrc/rt_internal.hpp"]


def kernel_source_digest():
    """SHA-256 over the sources the pass kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, pass_steps):
    """HBM bytes per pass-kernel launch from the committed PMC summary of
    this workload, or None when there is none, or the kernel sources or the
    pass length changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_k_trace_pass_%s.md" % workload)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ":" in ln and ln.startswith("- "):
                k, v = ln[2:].split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_digest() or vals.get("pass_steps") != str(pass_steps):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(nbytes, reps=4):
    """Plain device-to-device copies of a known size (calibration of the
    FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def algorithmic_flops(kind, step, st, rotating=False):
    ev = st["acc_evals"]
    if kind == 1:
        f = FLOPS["graph_eval"] * ev + FLOPS["graph_bump"] * st["bump_evals"]
    elif kind == 2:
        f = FLOPS["twist_eval"] * ev
    elif kind == 3:
        f = FLOPS["ztwist_eval"] * ev
    elif kind == 4:
        f = FLOPS["deform_eval"] * ev + FLOPS["deform_term_rot" if rotating else "deform_term"] * st["bump_evals"]
    elif kind == 5:
        f = FLOPS["ganiso_eval"] * ev + FLOPS["ganiso_bump"] * st["bump_evals"]
    elif kind == 6:
        f = FLOPS["gquad_eval"] * ev
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
    # the same oracle on one thread, over the next pixels of the sample
    one, steps1, t1 = done, 0, time.perf_counter()
    while one < len(pix) and time.perf_counter() - t1 < budget_s / 3:
        r = orc.trace(cam, rule, pix[one:one + 16], nthreads=1)
        steps1 += int(r["steps"].sum())
        one += len(r["id"])
    dt1 = time.perf_counter() - t1
    return {"value": done / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "ray_steps_per_s": steps / dt,
            "sample": "%d seeded pixels (seed 11) of the %dx%d frame, FP64, no culling, %.1f s" % (
                done, cam["width"], cam["height"], dt),
            "single_thread": {"value": (one - done) / dt1, "ray_steps_per_s": steps1 / dt1,
                              "sample": "the next %d pixels of the same sample, 1 thread, %.1f s" % (
                                  one - done, dt1)}}


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
        e3.record()
        g = tr.trace_bwd(tape, gh, nb)
        return loss, g

    # HIP events on the stream every kernel of the step runs on (torch's current one)
    e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fwd_ms = tot_ms = bwd_ms = 0.0
    for _ in range(args.steps):
        e0.record()
        loss, g = step()
        e2.record()
        torch.cuda.synchronize()
        fwd_ms += e0.elapsed_time(e1)
        tot_ms += e0.elapsed_time(e2)
        bwd_ms += e3.elapsed_time(e2)
    st = tr.stats()
    # algorithmic FLOPs of one rt_trace_bwd from its work counters; the bump
    # terms of the recomputed steps are taken in proportion to the reversed
    # steps' (the two walk the same states, less each segment's last step)
    S, T, Rc = st["adj_steps"], st["adj_bump_terms"], st["adj_recomputed"]
    adj_flops = (FLOPS["adj_rev_step"] * S + FLOPS["adj_term"] * T +
                 Rc * (FLOPS["adj_recomp_step"] + FLOPS["graph_bump"] * (T / max(S, 1))))
    adj_ms = bwd_ms / args.steps
    achieved = adj_flops / (adj_ms * 1e-3) / 1e12
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None, "kernel": "k_adjoint",
                     "flops_per_launch": adj_flops, "kernel_ms_per_launch": adj_ms},
        "adjoint_work": {"steps_reversed": S, "steps_recomputed": Rc, "bump_terms": T,
                         "bump_terms_per_step": T / max(S, 1)},
    }
    print(json.dumps(line), flush=True)


def _frame_error(out, ref, tol=1e-3):
    """Pixels whose object id differs from the reference frame or whose hit
    point is farther than tol (Euclidean) from it; hit-error quantiles over
    pixels with the same id."""
    import numpy as np
    same = out["id"] == ref["id"]
    err = np.linalg.norm(out["hit"].astype(np.float64) - ref["hit"], axis=1)
    bad = (~same) | (err > tol)
    e = err[same]
    # over all pixels, an id mismatch counting as an infinite error
    e_all = np.where(same, err, np.inf)
    return {"frac_within_tol": float(1.0 - bad.mean()), "frac_id_equal": float(same.mean()),
            "p999_hit_err": float(np.quantile(e, 0.999)) if e.size else 0.0,
            "p999_err_all_pixels": float(np.quantile(e_all, 0.999)),
            "max_hit_err": float(e.max()) if e.size else 0.0}


def _timed_frames(tr, cam, rule, out, steps, torch):
    """Mean wall time (ms) of `steps` traces between two stream events, and
    the stats of the last one."""
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    agg = {"pass_ms": 0.0, "surr_ms": 0.0, "refine_ms": 0.0, "compact_ms": 0.0}
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        tr.trace_into(cam, dict(rule, flags=rule.get("flags", 0) | 1), rule["max_steps"], out)
        st = tr.stats()
        for k in agg:
            agg[k] += st[k] / steps
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, st, agg


def cross_gen_roofline(tr, kappa, torch, h=0.01, n_per=16384, reps=3):
    """The training-data kernel alone (k_cross_gen): `reps` launches of
    n_per crossings per shape (16 training steps' worth) with the training
    loop's stratified draws, timed with stream events; its RK4 steps follow
    from the arc lengths it returns (steps of h to the exit, then 30
    bisection steps and the final partial step)."""
    import numpy as np
    ones = np.ones(len(kappa), np.float32)
    tr.surrogate_gen(kappa, ones, n_per, h, mode=4, seed=11)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for r in range(reps):
        _, _, aux = tr.surrogate_gen(kappa, ones, n_per, h, mode=4, seed=12 + r)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    arc = aux[:, :, 1].double().cpu().numpy()
    kmax = float(np.abs(np.asarray(kappa, np.float64)).max())
    max_steps = int((20.0 + 10.0 * kmax) / h) + 16
    exited = arc >= 0
    lane = np.where(exited, np.floor(arc / h + 1e-6) + 31, max_steps)
    total = float(lane.sum())
    waves = lane.reshape(len(kappa), -1, 64)
    flops = FLOPS["cross_step"] * total
    achieved = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "kernel": "k_cross_gen", "ms_per_launch": ms,
            "crossings_per_launch": int(lane.size), "rk4_steps_per_launch": total,
            "flops_per_launch": flops, "lane_efficiency": total / float(64 * waves.max(axis=2).sum())}


def bench_surrogate(args, wl, torch, rt):
    """Learned crossings against plain RK4 on the same frame: train one
    network per bump shape, time the RK4-only frame (the reference) and the
    surrogate frame, measure acceptance and hit error against the RK4 frame,
    and find the largest RK4 step whose error is no larger (equal-error
    comparison)."""
    import numpy as np

    from paper_2005_05386_amd import surrogate as S
    # RK4 frames with the workload's own pass length; surrogate frames with
    # shorter passes (a parked ray resumes at the next pass)
    cam, rule = wl["camera"], dict(wl["rule"])
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    out = tr.alloc_outputs(cam)
    n_rays = cam["width"] * cam["height"]
    kappa, net = S.shapes_of(wl["metric"]["bumps"][0])
    print("[bench] surrogate workload %s: %d shapes, training %d crossings each" % (
        args.workload, len(kappa), args.surr_samples), flush=True)
    model = S.train(tr, kappa, samples=args.surr_samples, batch=1024, h=0.01, seed=0,
                    log=lambda m: print("[bench] " + m, flush=True))
    # MLP FLOPs per training row: forward 2*(6*256 + 2*256^2 + 256*6), backward about twice that
    fwd_flops = 2 * (6 * 256 + 2 * 256 * 256 + 256 * 6)
    train_tflops = 3 * fwd_flops * model.samples * len(kappa) / model.train_s / 1e12
    S.load(tr, model, net, tol=args.surr_tol)
    gen = cross_gen_roofline(tr, kappa, torch)
    print("[bench] crossing generator: %s" % json.dumps(gen), flush=True)

    for _ in range(args.warmup):
        tr.trace_into(cam, rule, rule["max_steps"], out)
    rk4_ms, rk4_st, rk4_k = _timed_frames(tr, cam, rule, out, args.steps, torch)
    ref = rt.to_numpy(out)
    srule = dict(rule, flags=rt.FLAG_SURROGATE, pass_steps=args.surr_pass_steps)
    tr.trace_into(cam, srule, rule["max_steps"], out)
    if tr.stats()["eligible"] == 0:
        # nothing eligible: the library runs the plain kernels, keep the plain pass length
        srule["pass_steps"] = rule["pass_steps"]
    for _ in range(args.warmup):
        tr.trace_into(cam, srule, rule["max_steps"], out)
    sur_ms, sur_st, sur_k = _timed_frames(tr, cam, srule, out, args.steps, torch)
    sur = rt.to_numpy(out)
    sur_err = _frame_error(sur, ref)
    print("[bench] rk4 %.2f ms, surrogate %.2f ms, crossings %d accepted %d, %s" % (
        rk4_ms, sur_ms, sur_st["crossings"], sur_st["accepted"], json.dumps(sur_err)), flush=True)

    # equal error: the largest RK4 step whose frame is at least as close to the h = 0.005 frame, by the
    # 99.9th percentile over all pixels of the hit error (an id mismatch counts as infinite); steps that
    # divide t_max, so that misses end at the same t
    eq = []
    for hh in (0.00625, 0.008, 0.01, 0.0125, 0.016, 0.02, 0.025, 0.04):
        r2 = dict(rule, h=float(np.float32(hh)), max_steps=int(round(rule["t_max"] / hh)))
        tr.trace_into(cam, r2, r2["max_steps"], out)
        ms2, st2, _ = _timed_frames(tr, cam, r2, out, max(1, args.steps // 2), torch)
        e2 = _frame_error(rt.to_numpy(out), ref)
        eq.append({"h": hh, "ms": ms2, **e2})
        print("[bench] rk4 h=%g: %.2f ms %s" % (hh, ms2, json.dumps(e2)), flush=True)
    ok = [e for e in eq if e["p999_err_all_pixels"] <= sur_err["p999_err_all_pixels"]]
    best = max(ok, key=lambda e: e["h"]) if ok else None

    mlp_flops = fwd_flops * sur_st["crossings"]
    line = {
        "metric": "surrogate vs RK4 at equal error (learned crossings, rays/s)",
        "value": n_rays / (sur_ms / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sur_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": args.workload, "width": cam["width"], "height": cam["height"], "h": rule["h"],
                   "max_steps": rule["max_steps"], "bumps": int(wl["metric"]["bumps"].shape[1]),
                   "pass_steps_rk4": rule["pass_steps"], "pass_steps_surrogate": srule["pass_steps"],
                   "probe_tol": args.surr_tol},
        "rk4_ms_per_frame": rk4_ms, "rk4_rays_per_s": n_rays / (rk4_ms / 1e3),
        "speedup_vs_rk4": rk4_ms / sur_ms,
        "crossings": sur_st["crossings"], "accepted": sur_st["accepted"],
        "acceptance": sur_st["accepted"] / max(1, sur_st["crossings"]),
        "eligible_bumps": sur_st["eligible"],
        "ray_steps": {"rk4": rk4_st["ray_steps"], "surrogate": sur_st["ray_steps"]},
        "error_vs_rk4": sur_err,
        "equal_error": {"rk4_h": best["h"] if best else None, "rk4_ms": best["ms"] if best else None,
                        "speedup_surrogate_vs_equal_error_rk4": (best["ms"] / sur_ms) if best else None,
                        "sweep": eq},
        "kernel_ms": {"rk4": rk4_k, "surrogate": sur_k},
        "mlp": {"inference_tflops_over_crossing_stages": mlp_flops / max(1e-9, sur_k["surr_ms"] / 1e3) / 1e12,
                "bf16_peak_tflops": 2500.0, "training_s": model.train_s, "training_steps": model.steps,
                "training_samples_per_shape": model.samples, "training_mlp_tflops": train_tflops,
                "final_loss": model.losses[-1][1] if model.losses else None},
        "cross_gen_roofline": gen,
    }
    print(json.dumps(line), flush=True)


def _finite(x):
    """JSON has no infinity: an infinite error (an id mismatch among the
    quantile's pixels) is written as null."""
    return None if x == float("inf") else x


EULER_H = (0.005, 0.0025, 0.00125, 0.000625, 0.0003125)
RK4_H = (0.005, 0.00625, 0.008, 0.01, 0.0125, 0.016, 0.02, 0.025, 0.04, 0.05, 0.0625, 0.08, 0.1)


def bench_euler(args, wl, torch, rt):
    """The paper's explicit Euler march (Eq. 4.1) against RK4 at equal hit
    error on the 1080p, 16-bump frame. The reference is the RK4 frame at
    h = 0.005 (its own error is below 1e-6 there). For each Euler step the
    frame is timed and its error taken (99.9th percentile over all pixels of
    the hit error, an id mismatch counting as infinite); the RK4 frame at the
    largest step whose error is no larger is the equal-error competitor.
    Every step divides t_max = 20, so misses end at the same t."""
    import numpy as np

    import workloads as W_
    cam = wl["camera"]
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    out = tr.alloc_outputs(cam)
    n_rays = cam["width"] * cam["height"]
    t_max = wl["rule"]["t_max"]

    def run(kind, hh):
        n = int(round(t_max / hh))
        r = dict(wl["rule"], kind=kind, h=float(np.float32(hh)), max_steps=n, pass_steps=n)
        for _ in range(max(1, args.warmup)):
            tr.trace_into(cam, r, n, out)
        ms, st, _ = _timed_frames(tr, cam, r, out, max(1, args.steps), torch)
        return ms, st, rt.to_numpy(out)

    _, _, ref = run(W_.RK4, 0.005)
    rk4 = []
    for hh in RK4_H:
        ms, st, o = run(W_.RK4, hh)
        e = _frame_error(o, ref)
        rk4.append({"h": hh, "ms": ms, "ray_steps": st["ray_steps"], **e})
        print("[bench] rk4 h=%g: %.2f ms %s" % (hh, ms, json.dumps(e)), flush=True)
    eul = []
    for hh in EULER_H:
        ms, st, o = run(W_.EULER, hh)
        e = _frame_error(o, ref)
        ok = [r for r in rk4 if r["p999_err_all_pixels"] <= e["p999_err_all_pixels"]]
        best = max(ok, key=lambda r: r["h"]) if ok else None
        eul.append({"h": hh, "ms": ms, "ray_steps": st["ray_steps"], **e,
                    "rk4_equal_error_h": best["h"] if best else None,
                    "rk4_equal_error_ms": best["ms"] if best else None,
                    "rk4_speedup_at_equal_error": (ms / best["ms"]) if best else None})
        print("[bench] euler h=%g: %.2f ms %s, RK4 at equal error: %s" % (
            hh, ms, json.dumps(e), json.dumps(best and {"h": best["h"], "ms": best["ms"]})), flush=True)
    for r in rk4 + eul:
        for k in ("p999_hit_err", "p999_err_all_pixels", "max_hit_err"):
            r[k] = _finite(r[k])
    head = eul[0]
    line = {
        "metric": "Euler (Eq. 4.1) vs RK4 at equal hit error (1080p, 16 bumps), rays/s of the Euler frame",
        "value": n_rays / (head["ms"] / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "width": cam["width"], "height": cam["height"],
                   "bumps": int(wl["metric"]["bumps"].shape[1]), "t_max": t_max,
                   "reference": "RK4 h=0.005", "euler_h": list(EULER_H), "rk4_h": list(RK4_H)},
        "euler": eul, "rk4": rk4,
    }
    print(json.dumps(line), flush=True)


def bench_batch(args, wl, torch, rt):
    """Batched multi-segment intersection (RT_FLAG_BATCH_SEGMENTS, the
    batching of polygon segments Sec. 4.1 proposes) against the per-step
    chord test, on the 1080p 16-bump frame and on the 4K twist scene (256
    spheres).  Both traces must give the same outputs bit for bit; `value`
    is the rays/s of the batched 1080p frame."""
    import numpy as np

    import workloads as W_
    res = {}
    for name, steps in (("bumps16_1080p", max(1, args.steps)), ("twist_4k", max(1, min(args.steps, 3)))):
        w = W_.get(name)
        cam, rule = w["camera"], dict(w["rule"])
        tr = rt.Tracer(0)
        tr.set_metric(w["metric"])
        tr.set_scene(w["scene"])
        n_rays = cam["width"] * cam["height"]
        r = {}
        outs = {}
        for mode, flags in (("per_step", 0), ("batched", rt.FLAG_BATCH_SEGMENTS)):
            rr = dict(rule, flags=flags)
            out = tr.alloc_outputs(cam)
            for _ in range(max(1, args.warmup)):
                tr.trace_into(cam, rr, rr["max_steps"], out)
            ms, st, agg = _timed_frames(tr, cam, rr, out, steps, torch)
            outs[mode] = rt.to_numpy(out)
            r[mode] = {"ms_per_frame": ms, "rays_per_s": n_rays / (ms / 1e3), "pass_ms": agg["pass_ms"],
                       "refine_ms": agg["refine_ms"], "windows": st["batch_windows"],
                       "windows_replayed": st["batch_replays"]}
            print("[bench] %s %s: %.2f ms/frame %s" % (name, mode, ms, json.dumps(r[mode])), flush=True)
        r["bitwise_equal"] = all(np.array_equal(outs["per_step"][k], outs["batched"][k])
                                 for k in ("hit", "t", "id", "dir", "steps"))
        r["batched_over_per_step"] = r["batched"]["ms_per_frame"] / r["per_step"]["ms_per_frame"]
        res[name] = r
    head = res["bumps16_1080p"]["batched"]
    cam = wl["camera"]
    line = {
        "metric": "batched multi-segment intersection (Sec. 4.1) vs per-step test, rays/s of the batched frame",
        "value": head["rays_per_s"], "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_frame"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "width": cam["width"], "height": cam["height"],
                   "window_steps": wl["rule"]["cull_every"], "scenes": list(res)},
        "scenes": res,
    }
    print(json.dumps(line), flush=True)


def bench_illum(args, wl, torch, rt):
    """Direct Riemannian illumination of the traced 1080p frame by a point
    light: shooting for the geodesic from every hit to the light, visibility
    along it and the Lambert term in the metric (rt_illuminate).  The trace
    is not timed; `value` is hit pixels shaded per second."""
    import numpy as np

    cam = wl["camera"]
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    out = tr.trace(cam, wl["rule"])
    for _ in range(max(1, args.warmup)):
        sh = tr.illuminate(cam, out, wl["light"])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        sh = tr.illuminate(cam, out, wl["light"])
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    st = sh["status"].cpu().numpy()
    n_hit = int((st != -3).sum())
    line = {
        "metric": "direct illumination: hit pixels shaded per second (1080p, 16 bumps, point light)",
        "value": n_hit / (ms / 1e3), "unit": "pixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "width": cam["width"], "height": cam["height"],
                   "light": list(wl["light"]["pos"]), "h": wl["light"]["h"], "tol": wl["light"]["tol"],
                   "max_iters": wl["light"]["max_iters"]},
        "pixels": {"hit": n_hit, "lit": int((st == 1).sum()), "shadowed": int((st == 0).sum()),
                   "facing_away": int((st == 2).sum()), "no_geodesic": int((st == -1).sum())},
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
    ap.add_argument("--surr-samples", type=int, default=10_000_000, help="training crossings per bump shape")
    ap.add_argument("--surr-tol", type=float, default=1e-3, help="probe tolerance on the hit error")
    ap.add_argument("--surr-pass-steps", type=int, default=1024, help="steps per pass in surrogate traces")
    ap.add_argument("--frames-in-flight", type=int, default=2,
                    help="frames traced concurrently on as many streams for the throughput figure")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run plain copies of this many bytes")
    args = ap.parse_args()
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.gpus != 1:
        print("bench.py: the tracer runs on one GPU only (--gpus 1); there is no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2005_05386_amd import rt

    wl = W.get(args.workload)
    if "ckpt_every" in wl:
        return bench_adjoint(args, wl, torch, rt)
    if args.workload.startswith("surrogate"):
        return bench_surrogate(args, wl, torch, rt)
    if args.workload == "euler_vs_rk4_1080p":
        return bench_euler(args, wl, torch, rt)
    if args.workload == "batch_segments_1080p":
        return bench_batch(args, wl, torch, rt)
    if "light" in wl:
        return bench_illum(args, wl, torch, rt)
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
    ms_serial = ev0.elapsed_time(ev1) / args.steps
    n_rays = tr.n_sets * cam["width"] * cam["height"]

    # Throughput: frames in flight on as many streams, each with a context
    # (workspace) and outputs of its own, so that the next frame's waves take
    # the SIMDs an ending pass leaves idle.  The serial loop above gives the
    # kernel times (no overlap) and one frame's latency.
    nf = max(1, args.frames_in_flight)
    ms = ms_serial
    if nf > 1:
        trs, outs, streams = [tr], [out], [stream]
        for _ in range(nf - 1):
            t2 = rt.Tracer(0)
            t2.set_metric(wl["metric"])
            t2.set_scene(wl["scene"])
            trs.append(t2)
            outs.append(t2.alloc_outputs(cam))
            streams.append(torch.cuda.Stream())
        for i in range(2 * nf):
            trs[i % nf].trace_into(cam, rule, ms_steps, outs[i % nf], stream=streams[i % nf])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            trs[i % nf].trace_into(cam, rule, ms_steps, outs[i % nf], stream=streams[i % nf])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        print("[bench] %d frames in flight: %.3f ms per frame (serial %.3f)" % (nf, ms, ms_serial), flush=True)

    import numpy as np
    dfm = wl["metric"].get("deforms")
    # the rotating model applies when every deformation rotates
    rotating = dfm is not None and dfm.shape[-1] == 13 and bool(np.all(np.any(dfm[..., 10:13] != 0, axis=-1)))
    flops = algorithmic_flops(wl["metric"]["kind"], rule["kind"], work, rotating)
    pass_s = pass_ms / 1e3 / args.steps
    achieved = flops / pass_s / 1e12
    # FP64 refinement (graph metric, RK4): counted evaluations, bump terms and
    # steps of the instrumented trace, priced by the FP64 model, over the
    # refine kernel's HIP-event time
    refine_roof = None
    if wl["metric"]["kind"] == 1 and rule["kind"] == 0 and work["refine_evals"] > 0:
        rf = (FLOPS["ref_eval"] * work["refine_evals"] + FLOPS["ref_bump"] * work["refine_bump_terms"] +
              (FLOPS["ref_rk4_step"] + FLOPS["ref_obj"]) * work["refine_steps"] + FLOPS["ref_obj"] * work["refined"])
        r_ms = refine_ms / args.steps
        r_ach = rf / (r_ms * 1e-3) / 1e12
        refine_roof = {"bound": "alu", "achieved": r_ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s (FP64)",
                       "frac": r_ach / FP64_PEAK_TFLOPS, "kernel": "k_refine", "flops_per_launch": rf,
                       "kernel_ms_per_launch": r_ms, "records": work["refined"], "evals": work["refine_evals"],
                       "bump_terms": work["refine_bump_terms"], "steps": work["refine_steps"]}
    line = {
        "metric": "rays/s & RK4 ray-steps/s (1080p, 16 bumps); surrogate vs RK4 at equal error",
        "value": n_rays / (ms / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "width": cam["width"], "height": cam["height"],
                   "n_sets": tr.n_sets, "step_rule": ["RK4", "RK45", "Euler"][rule["kind"]], "h": rule["h"],
                   "max_steps": ms_steps, "bumps": int(wl["metric"]["bumps"].shape[1]),
                   "deforms": int(wl["metric"]["deforms"].shape[1]) if "deforms" in wl["metric"] else 0,
                   "anisotropic_bumps": int(wl["metric"]["abumps"].shape[1]) if "abumps" in wl["metric"] else 0,
                   "spheres": int(len(wl["scene"]["spheres"]))},
        "ray_steps_per_s": work["ray_steps"] / (ms / 1e3),
        "frames_in_flight": nf, "frame_latency_ms": ms_serial,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": measured_traffic(args.workload, rule["pass_steps"]),
                     "kernel": "k_trace_pass", "flops_per_trace": flops,
                     "kernel_ms_per_launch": pass_ms / max(1, n_pass_launches),
                     "frame_rate_tflops": flops / (ms / 1e3) / 1e12,
                     },
        "kernel_ms": {"passes": pass_ms / args.steps, "refine": refine_ms / args.steps,
                      "compaction": compact_ms / args.steps},
        "refine_roofline": refine_roof,
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
