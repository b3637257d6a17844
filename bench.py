#!/usr/bin/env python3
"""Benchmark of the SVT-R4SVD hot path on one MI355X.

A step is one SVT iteration of Alg. 4 (R4SVD with recycling, projected SVD,
soft-threshold, fused sampled product and dual update) on the image-recovery
workload: a 1024 x 1024 matrix of 40 separable smooth patterns plus noise,
50% of the pixels observed, tau = ||P_Lambda A||_F, delta = sqrt(mn / |Lambda|).
Inputs are synthetic and seeded; they are resident on the GPU before timing.

Prints one JSON line with:
  * iterations/s over the timed steps (one library call) for the float32-storage
    form (the value) and the FP64 form;
  * the roofline of the dominant single-kernel phase: its kernel launched
    back to back on the operands the timed region ended with, between hipEvents
    on the library's stream (and the event average inside the timed region),
    with the HBM traffic of a committed counter summary taken at the same basis
    width when one exists for the current kernel source;
  * a per-phase breakdown of every phase over the following iterations (untimed):
    time per step, share of the step, algorithmic bytes and flops, and the
    fraction of the HBM and compute peaks each phase reaches;
  * the sample MAE and the MAE of Eq. 15 over all pixels (0..255 scale);
  * whole runs on the image workload, every form: to the paper's stop rule for
    images (sample MAE below 1 on the 0..255 scale, Sec. 3.1) and to relative
    residual 1e-3, with the whole-run iterations/s;
  * the time to relative residual 1e-4 on the planted 1000 x 1000 rank-10
    problem for five Omega seeds (median and range), every form;
  * the recycling ablation: per-iteration cost of R4SVD, R3SVD from a fresh
    t-block every iteration, and the fixed-rank randomized SVD of Alg. 1;
  * the FP64 CPU oracle on the host, on the same trajectory: it starts from the
    state the FP64 GPU run had when its timed iterations began and replays that
    run's growth and annealing decisions, for a bounded number of iterations.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6    # FP64 vector FMA and FP64 matrix cores (dense)
FP32_PEAK_TFS = 157.3   # FP32 vector FMA

METRIC = "SVT iters/sec + time-to-rel-residual 1e-4 (BF16/FP32 form vs FP64 plain)"
FORMS = {"mixed": 1, "bf16": 2, "fp64": 0}  # svt_params.precision of each form
FORM_NAME = {v: k for k, v in FORMS.items()}
# single-kernel phases whose device time is recorded inside the timed region
ROOF_PHASES = ["spmm_t", "gram", "sddmm", "densify"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance run")
    ap.add_argument("--forms", default="mixed,bf16,fp64",
                    help="precision forms to time (comma list of mixed = float32 storage, bf16 = bfloat16 basis "
                         "with the exact projector, fp64); the first gives the headline value")
    ap.add_argument("--ttt-seeds", default="11,12,13,14,15",
                    help="Omega seeds of the time-to-tolerance runs (median and range are reported)")
    ap.add_argument("--workload", default="image", choices=["image", "ratings", "large"],
                    help="image: the 1024x1024 image-recovery configuration (default); ratings: the 6040 x 3706 "
                         "recommendation shape (900k training ratings, power-law degrees, test MAE on the 10% held "
                         "out); large: the 100000 x 50000 "
                         "planted rank-20 matrix with 20M power-law entries (BF16-representable values), tol 1e-3, "
                         "r_max 4096, timed for a few iterations per form")
    ap.add_argument("--ablation-steps", type=int, default=30,
                    help="SVT iterations per operator variant in the recycling ablation (0 skips it)")
    ap.add_argument("--breakdown-steps", type=int, default=10,
                    help="iterations after the timed ones with every phase timed (per-phase breakdown)")
    ap.add_argument("--replay-reps", type=int, default=50,
                    help="back-to-back launches per single-kernel phase for the per-launch roofline time")
    ap.add_argument("--grad", action="store_true",
                    help="also time the derivative workload (image, 50 iterations, checkpoints every 10)")
    ap.add_argument("--ratings-run", action="store_true",
                    help="with --workload ratings: also run every form to the paper's train-MAE stop rule")
    ap.add_argument("--image-maxit", type=int, default=1500,
                    help="cap on the whole image runs to the sample-MAE stop rule")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size reference kernel for "
                         "hardware traffic counters)")
    return ap.parse_args()


def committed_traffic(phase, form, workload, r):
    """HBM bytes per launch of the roofline kernel from a committed counter summary
    (profiles/*_traffic.json), or None.  A summary counts only while the kernel source it was
    taken with is unchanged (SHA-256) and it describes this phase, form, workload and basis width."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json"))):
        try:
            with open(path) as f:
                t = json.load(f)
            with open(os.path.join(ROOT, t["source"]), "rb") as f:
                sha = hashlib.sha256(f.read()).hexdigest()
        except (OSError, ValueError, KeyError):
            continue
        if sha != t.get("source_sha256"):
            continue
        for e in t.get("entries", [t]):
            if e.get("phase") == phase and e.get("form") == form and e.get("workload") == workload and e.get("r") == r:
                return float(e["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def divmod_all(m, n):
    import numpy as np
    i, j = np.divmod(np.arange(m * n, dtype=np.int64), n)
    return i.astype(np.int32), j.astype(np.int32)


def host_cpu():
    """Model name and logical CPU count of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(w, start, decisions, params, budget_s=15.0):
    """The FP64 oracle, as it stands, on the host, on the GPU run's own trajectory: from the FP64
    GPU run's state when its timed iterations began (Y on Lambda, the basis, the annealing state),
    replaying that run's growth and annealing decisions, until about budget_s seconds of host work
    or the end of the recorded window (bounded so the default run stays short)."""
    from threadpoolctl import threadpool_info

    from oracle import Params, Problem, State, svt_step

    prob = Problem(w.m, w.n, w.rows, w.cols, w.a)
    p = Params(tau=w.tau, delta=w.delta, **params)
    state = State(it=start["iter"], y=start["y"].copy(), Q=start["Q"].copy() if start["r"] > 0 else None,
                  eps_thr=start["eps_thr"], eps_min=start["eps_min"])
    done, t0, el = 0, time.perf_counter(), 0.0
    rs = []
    for blocks, annealed in decisions:
        state, info = svt_step(prob, p, state, (blocks, annealed))
        done += 1
        rs.append(info.r)
        el = time.perf_counter() - t0
        if el > budget_s or info.stopped:
            break
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    model, ncpu = host_cpu()
    return {"value": done / el, "unit": "iters/s", "cores": int(threads), "kind": "oracle",
            "cpu_model": model, "nproc": ncpu,
            "sample": f"{done} oracle SVT iterations ({start['iter'] + 1}..{start['iter'] + done}) of the same image "
                      f"workload, from the FP64 GPU run's state when its timed window began, with that run's growth "
                      f"and annealing decisions replayed (basis width {min(rs)}..{max(rs)}); {el:.1f} s wall on the "
                      f"host ({model}, {ncpu} logical CPUs), BLAS threads={threads}, scipy sparse products "
                      f"single-threaded"}


def time_to_tolerance(svt, W, stream, seed, precision):
    import torch
    w = W.planted()
    h = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, stream=stream, tau=w.tau, delta=w.delta, seed=seed, maxit=1000,
                     tol=w.tol, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = h.iterate(1000)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"seconds": el, "iterations": st.iter, "converged": bool(st.stopped), "rel_res": st.rel_res,
            "r_final": st.r, "k_final": st.k}


def ttt_seeds(svt, W, stream, seeds, precision):
    runs = [time_to_tolerance(svt, W, stream, sd, precision) for sd in seeds]
    secs = sorted(r["seconds"] for r in runs)
    its = sorted(r["iterations"] for r in runs)
    return {"seeds": list(seeds), "median_seconds": secs[len(secs) // 2], "min_seconds": secs[0],
            "max_seconds": secs[-1], "median_iterations": its[len(its) // 2], "min_iterations": its[0],
            "max_iterations": its[-1], "all_converged": all(r["converged"] for r in runs), "runs": runs}


def whole_run(svt, w, stream, seed, precision, maxit, chunk=25, **kw):
    """One run from Y^(0) to a stop rule (or maxit), iterated in chunks of `chunk` iterations with the
    wall clock read after each: total time, iterations, the whole-run rate, and the time at which
    the relative residual first fell below 1e-1 and 1e-2 (the end of the chunk it happened in)."""
    import torch
    h = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, stream=stream, tau=w.tau, delta=w.delta, seed=seed, maxit=maxit,
                     precision=precision, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks, done, st = [], 0, None
    while done < maxit:
        st = h.iterate(min(chunk, maxit - done))
        torch.cuda.synchronize()
        done = st.iter
        marks.append((done, time.perf_counter() - t0))
        if st.stopped:
            break
    el = marks[-1][1]
    hist = h.history()
    below = {}
    for thr in (1e-1, 1e-2):
        it = next((x.iter for x in hist if x.rel_res < thr), None)
        sec = next((t for i, t in marks if it is not None and i >= it), None)
        below[f"{thr:g}"] = {"iteration": it, "seconds_at_chunk_end": sec}
    out = {"seconds": el, "iterations": st.iter, "iters_per_s": st.iter / el, "stopped": bool(st.stopped),
           "rel_res": st.rel_res, "sample_mae_255": 255.0 * st.mae, "r_final": st.r, "k_final": st.k,
           "rel_res_below": below}
    h.close()
    return out


def grad_workload(svt, W, stream, seed, T=50, ckpt=10):
    """The derivative workload: the image, T unrolled iterations (FP64 form) and the gradient of the
    held-out RMSE with respect to tau, delta and every observed value, checkpoints every ckpt
    iterations; GPU tensors across the boundary.  Wall time of the forward iterations and of each
    reverse sweep (exact and frozen-basis)."""
    import numpy as np
    import torch
    w = W.image_adjoint()
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")  # noqa: E731
    rows, cols, vals = dev(w.rows, torch.int32), dev(w.cols, torch.int32), dev(w.a, torch.float64)
    hi, hj = dev(w.held_rows, torch.int32), dev(w.held_cols, torch.int32)
    ref = dev(w.held_a, torch.float64)
    h = svt.svt_init(w.m, w.n, rows, cols, vals, stream=stream, tau=w.tau, delta=w.delta, seed=seed, maxit=T + 5,
                     tol=0.0, precision=svt.SVT_FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = h.iterate(T)
    x = h.sample(hi, hj)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    rmse = torch.sqrt(torch.mean((x - ref) ** 2))
    g = ((x - ref) / (x.numel() * rmse)).contiguous()
    out = {"workload": f"image 1024x1024, {T} iterations (FP64), gradient of the RMSE on {w.held_rows.size} held-out "
                       f"pixels w.r.t. tau, delta and the {w.nnz} observed values, checkpoints every {ckpt}",
           "forward_seconds": t_fwd, "r_final": st.r, "k_final": st.k, "rmse": float(rmse)}
    for name, frozen in (("exact", False), ("frozen_basis", True)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dtau, ddelta, da = h.grad(T, ckpt, hi, hj, g, frozen_basis=frozen)
        torch.cuda.synchronize()
        out[name] = {"seconds": time.perf_counter() - t0, "dtau": dtau, "ddelta": ddelta,
                     "da_norm": float(torch.linalg.norm(da))}
    h.close()
    return out


def ablation(svt, w, stream, steps, seed):
    """Per-iteration cost and progress of the operator variants over the same first SVT iterations
    (FP64 form): R4SVD (recycling, Alg. 3), R3SVD from a fresh t-block every iteration (Alg. 2), and
    the fixed-rank randomized SVD of Alg. 1 (rank 40 + 10 oversampling)."""
    import torch
    out = {}
    variants = [("r4svd", dict(mode=svt.SVT_MODE_R4SVD)), ("r3svd", dict(mode=svt.SVT_MODE_R3SVD)),
                ("rsvd_rank40_p10", dict(mode=svt.SVT_MODE_RSVD, rank=40, oversample=10))]
    for name, kw in variants:
        h = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, stream=stream, tau=w.tau, delta=w.delta, seed=seed,
                         maxit=steps + 1, tol=0.0, precision=svt.SVT_FP64, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = h.iterate(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        hist = h.history()
        rs, blocks = [x.r for x in hist], sum(x.blocks for x in hist)
        out[name] = {"iterations": steps, "seconds": el, "ms_per_iter": 1e3 * el / steps, "r_mean": sum(rs) / steps,
                     "r_last": rs[-1], "growth_blocks": blocks, "rel_res_last": st.rel_res, "mae_last": st.mae}
        h.close()
    return out


def run_form(svt, w, stream, args, precision, want_state=False, **extra):
    """Warm up, then time args.steps SVT iterations of one precision form with per-phase events."""
    import torch
    h = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, stream=stream, tau=w.tau, delta=w.delta, seed=args.seed,
                     maxit=args.warmup + args.steps + args.breakdown_steps + 1000, precision=precision, **extra)
    if args.warmup > 0:
        h.iterate(args.warmup)
    torch.cuda.synchronize()
    start_state = h.get_state() if want_state else None
    # Timed region: hipEvents only around the single-kernel phases that compete for the roofline
    # (each event is a marker the GPU processes between kernels, so timing every phase would
    # slow the iteration being measured).
    h.profile(True, phases=ROOF_PHASES)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.iterate(args.steps)  # one library call; it stops early only at convergence
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    window = h.history(first=args.warmup)
    stats = [(st.r, st.k, st.blocks, st.eig_iters, st.rel_res, st.mae) for st in window]
    decisions = [(st.blocks, st.annealed) for st in window]
    prof = h.profile_read()
    h.profile(False)
    # Per-launch time of each single-kernel phase on the operands the timed region ended with:
    # args.replay_reps back-to-back launches between two events on the library stream.  (Events
    # around the launches inside the iteration also count the GPU's wait for the host to enqueue
    # the kernel after each host decision point.)
    replay = {}
    if not h.history()[-1].stopped:
        for ph in ROOF_PHASES:
            if ph == "densify" and 4 * w.nnz < w.m * w.n:
                continue  # no dense copy of Y in this problem
            ms, by, fl = h.time_phase(ph, reps=args.replay_reps)
            replay[ph] = {"ms": ms, "bytes": by, "flops": fl}
    # Per-phase breakdown of every phase over the next few iterations (not timed).
    breakdown, n_bd = {}, 0
    if args.breakdown_steps > 0 and not h.history()[-1].stopped:
        h.profile(True)
        n0 = len(h.history())
        h.iterate(args.breakdown_steps)
        breakdown = h.profile_read()
        n_bd = len(h.history()) - n0
        h.profile(False)
    if w.A is not None:
        # recovery quality after the timed steps on the 0..255 scale of the paper's images (Sec. 3):
        # the sample MAE on Lambda and the MAE of Eq. 15 over all m n pixels
        all_i, all_j = divmod_all(w.m, w.n)
        quality = {"sample_mae_255": 255.0 * stats[-1][5],
                   "overall_mae_255": 255.0 * h.mae(all_i, all_j, w.A.ravel())}
    else:
        quality = {"sample_mae": stats[-1][5]}
    if w.held_rows is not None:
        # test MAE of Eq. 15 on the held-out ratings (the paper's recommendation metric)
        quality["test_mae"] = h.mae(w.held_rows, w.held_cols, w.held_a)
    h.close()
    n_it = len(stats)
    r_vals = [s[0] for s in stats]
    es = 4.0 if precision else 8.0  # the iterate and W (float32 in the mixed and BF16 forms)
    # Roofline of the dominant single-kernel phase.  Its bound is the resource whose peak time for
    # the phase's algorithmic work is larger: HBM bytes, or flops on the unit the kernel uses.  The
    # Gram runs on the FP64 matrix cores in both forms.  W = Y^T Q runs on the matrix cores in the
    # storage precision (FP32 in the mixed form, FP64 in the FP64 form) with a dense copy of Y when
    # at least a quarter of the entries are observed (the library's rule), else on the vector units;
    # its algorithmic flops are 2 nnz r either way.  The scatter that refreshes the dense copy is a
    # phase of its own (pure data movement).
    dense_y = 4 * w.nnz >= w.m * w.n
    store_peak = FP32_PEAK_TFS if precision else FP64_PEAK_TFS
    units = {"spmm_t": ("mfma" if dense_y else "alu", store_peak), "sddmm": ("alu", store_peak),
             "gram": ("mfma", FP64_PEAK_TFS), "densify": ("alu", store_peak)}
    # dominant phase: the longest kernel on the final operands (replay), else inside the region
    if replay:
        dom = max(replay, key=lambda ph: replay[ph]["ms"])
        pd = replay[dom]
        per_ms, per_bytes, per_flops = pd["ms"], pd["bytes"], pd["flops"]
    else:
        dom = max(units, key=lambda ph: prof[ph]["ms"])
        pd = prof[dom]
        nl = max(pd["launches"], 1)
        per_ms, per_bytes, per_flops = pd["ms"] / nl, pd["bytes"] / nl, pd["flops"] / nl
    unit, cpeak = units[dom]
    t_hbm = per_bytes / (HBM_PEAK_GBS * 1e9)
    t_cmp = per_flops / (cpeak * 1e12)
    if t_hbm >= t_cmp:
        achieved = per_bytes / (per_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    else:
        achieved = per_flops / (per_ms * 1e-3) / 1e12
        roof = {"bound": unit, "achieved": achieved, "peak": cpeak, "unit": "TFLOP/s",
                "frac": achieved / cpeak, "traffic": None}
    traffic, tsrc = (committed_traffic(dom, FORM_NAME[precision], args.workload, r_vals[-1])
                     if replay else (None, None))
    roof["traffic"] = traffic
    if tsrc:
        roof["traffic_source"] = tsrc
    ip = prof[dom]
    roof.update({"kernel": dom, "avg_launch_us": 1e3 * per_ms, "bytes_per_launch": per_bytes,
                 "flops_per_launch": per_flops,
                 "timing": (f"{args.replay_reps} back-to-back launches on the operands after iteration "
                            f"{args.warmup + n_it} (r = {r_vals[-1]})") if replay else "events in the timed region",
                 "in_region": {"launches": ip["launches"],
                               "avg_launch_us": 1e3 * ip["ms"] / max(ip["launches"], 1)}})
    # Per-phase breakdown with rooflines: the share of the step, and the fraction of the HBM peak and
    # of the compute peak of the unit the phase's work runs on (the Gram, the eigensolver's products
    # and the growth blocks' projections in FP64, the rest in the storage precision) that its
    # algorithmic bytes and flops reach over the phase's measured time.
    step_ms = sum(v["ms"] for v in breakdown.values())
    phase_peak = {"spmm_t": store_peak, "grow": store_peak, "gram": FP64_PEAK_TFS, "eig": FP64_PEAK_TFS,
                  "factors": store_peak, "sddmm": store_peak, "reduce": FP64_PEAK_TFS, "densify": store_peak}
    phases = {}
    for ph, v in breakdown.items():
        gbs = (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["bytes"] > 0 else None
        tfs = (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 and v["flops"] > 0 else None
        phases[ph] = {"ms_per_step": v["ms"] / max(n_bd, 1), "share": v["ms"] / step_ms if step_ms > 0 else None,
                      "launches": v["launches"], "GB_s": gbs, "hbm_frac": gbs / HBM_PEAK_GBS if gbs else None,
                      "TFLOP_s": tfs, "compute_peak_TFLOP_s": phase_peak.get(ph),
                      "compute_frac": tfs / phase_peak[ph] if tfs and ph in phase_peak else None}
    timed_phases = {ph: {"ms_per_step": prof[ph]["ms"] / max(n_it, 1), "launches": prof[ph]["launches"]}
                    for ph in ROOF_PHASES}
    return {"iters_per_s": n_it / el, "ms_per_step": 1e3 * el / max(n_it, 1), "steps": n_it,
            "_start_state": start_state, "_decisions": decisions,
            "iterations_timed": [args.warmup + 1, args.warmup + n_it], "r_range": [min(r_vals), max(r_vals)],
            "r_mean": float(sum(r_vals) / len(r_vals)), "k_last": stats[-1][1],
            "growth_blocks": int(sum(s[2] for s in stats)), "eig_products": int(sum(s[3] for s in stats)),
            "rel_res_last": stats[-1][4], "bytes_per_value": es, "quality": quality, "roofline": roof,
            "timed_phases": timed_phases, "replay_us_per_launch": {ph: 1e3 * v["ms"] for ph, v in replay.items()},
            "phases": phases,
            "phases_iterations": [args.warmup + n_it + 1, args.warmup + n_it + n_bd]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported (the multi-GPU column "
              f"sharding is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import paper_1704_05528_amd as svt
    import svt_workloads as W
    import torch

    svt.require_gpu()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    if not forms or any(f not in FORMS for f in forms):
        print(f"--forms takes mixed, bf16 and/or fp64, got {args.forms!r}", file=sys.stderr)
        sys.exit(2)
    extra = {}
    if args.workload == "large":
        w = W.large_sparse()
        # The step-size rule of Sec. 3 gives delta = sqrt(mn/|Lambda|) = 15.8 here, and the iteration then
        # diverges within two steps: the heaviest power-law rows are sampled in full, so the local step
        # exceeds the stable bound of 2.  The large measurement uses delta = 1.2.
        w.delta = 1.2
        extra = {"r_max": 4096, "tol": w.tol}
        desc = ("large sparse 100000x50000, planted rank 20 + N(0,0.1^2), 20M Chung-Lu power-law entries (Zipf 1.1), "
                "BF16-representable values, tau=||P_Lambda A||_F, delta=1.2, t=2500, r_max=4096")
        args.no_ttt, args.no_cpu, args.ablation_steps = True, True, 0
    elif args.workload == "ratings":
        w = W.ratings()
        # As for the large case, the step-size rule of Sec. 3 (delta = sqrt(mn/|Lambda|) = 5.0 here) diverges on
        # power-law degrees (the heaviest users' rows are sampled almost in full); delta = 1.9 converges and
        # reaches the paper's stop rule for ratings (train MAE < 0.1, Sec. 3.2) in about 210 iterations with a
        # basis of up to 2048 columns.
        w.delta = 1.9
        extra = {"r_max": 2048}
        desc = ("ratings 6040x3706, 1,000,209 power-law entries (Zipf 1.2, >= 20 per user), integer ratings 1-5 from a "
                "rank-10 factor model, 90/10 train/held-out split, tau=||P_Lambda A||_F, delta=1.9, r_max=2048")
        args.no_ttt, args.no_cpu, args.ablation_steps = True, True, 0
    else:
        w = W.image()
        desc = ("image 1024x1024, 40 separable cosine patterns + N(0,0.01^2), 50% observed, "
                "tau=||P_Lambda A||_F, delta=sqrt(mn/|Lambda|)")
    res = {f: run_form(svt, w, stream, args, FORMS[f], want_state=(f == "fp64" and not args.no_cpu), **extra)
           for f in forms}
    starts = {f: (r.pop("_start_state"), r.pop("_decisions")) for f, r in res.items()}
    head = res[forms[0]]
    dtypes = {"mixed": "f32 storage / f64 Gram+eig (mixed form)",
              "bf16": "bf16 basis, f32 iterate and factors / f64 Gram+Cholesky+eig (BF16 form)", "fp64": "f64"}
    out = {"metric": METRIC, "value": head["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": head["steps"],
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtypes[forms[0]],
           "data": "synthetic",
           "config": {"workload": desc, "m": w.m, "n": w.n, "nnz": w.nnz, "form": forms[0]},
           "roofline": head["roofline"]}
    out.update(res)
    fp64 = res.get("fp64")
    for f in forms:
        if f != "fp64" and fp64:
            out[f"speedup_{f}_vs_fp64"] = res[f]["iters_per_s"] / fp64["iters_per_s"]
    if not args.no_ttt:
        seeds = [int(x) for x in args.ttt_seeds.split(",") if x.strip()]
        ttt = {f: ttt_seeds(svt, W, stream, seeds, FORMS[f]) for f in forms}
        out["time_to_tol"] = {"workload": "planted 1000x1000 rank 10, 20% observed, tau=5 sqrt(mn), "
                                          "delta=1.2 mn/|Lambda|, tol 1e-4", **ttt}
        for f in forms:
            if f != "fp64" and "fp64" in ttt:
                out["time_to_tol"][f"speedup_{f}_vs_fp64_median"] = (ttt["fp64"]["median_seconds"] /
                                                                     ttt[f]["median_seconds"])
    if args.workload == "image" and not args.no_ttt:
        # whole runs from Y^(0) to the paper's stop rule for images (sample MAE < 1 on 0..255, Sec. 3.1);
        # the relative residual passes 1e-2 on the way (it does not reach 1e-4 within a few thousand)
        runs = {}
        for f in forms:
            prec = FORMS[f]
            runs[f] = whole_run(svt, w, stream, args.seed, prec, args.image_maxit, tol=0.0, mae_tol=1.0 / 255.0)
        out["image_whole_runs"] = {"workload": "image 1024x1024 (as above), from Y^(0) to sample MAE < 1 (0..255 "
                                               "scale, the stop rule of Sec. 3.1)", **runs}
        for f in forms:
            if f != "fp64" and "fp64" in runs:
                out["image_whole_runs"][f"speedup_{f}_vs_fp64"] = runs["fp64"]["seconds"] / runs[f]["seconds"]
    if args.workload == "ratings" and args.ratings_run:
        # whole runs to the paper's stop rule for ratings (train MAE < 0.1 on the 1..5 scale, Sec. 3.2), with
        # the test MAE of Eq. 15 on the held-out 10% at the end
        rr = {}
        for f in forms:
            import torch
            h = svt.svt_init(w.m, w.n, w.rows, w.cols, w.a, stream=stream, tau=w.tau, delta=w.delta, seed=args.seed,
                             maxit=600, tol=0.0, mae_tol=0.1, precision=FORMS[f], **extra)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = h.iterate(600)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            rr[f] = {"seconds": el, "iterations": st.iter, "iters_per_s": st.iter / el, "stopped": bool(st.stopped),
                     "train_mae": st.mae, "test_mae": h.mae(w.held_rows, w.held_cols, w.held_a), "r_final": st.r,
                     "k_final": st.k}
            h.close()
        out["ratings_whole_runs"] = {"stop": "train MAE < 0.1 (Sec. 3.2), at most 600 iterations", **rr}
    if args.grad:
        out["derivative_workload"] = grad_workload(svt, W, stream, args.seed)
    if args.ablation_steps > 0:
        out["recycling_ablation"] = {"workload": "image 1024x1024 (as above), first iterations from Y^(0), FP64",
                                     **ablation(svt, w, stream, args.ablation_steps, args.seed)}
    if not args.no_cpu and fp64 and starts["fp64"][0] is not None:
        st0, dec = starts["fp64"]
        cb = cpu_baseline(w, st0, dec, dict(seed=args.seed, maxit=args.warmup + args.steps + 1000))
        cb["gpu_fp64_speedup"] = fp64["iters_per_s"] / cb["value"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
