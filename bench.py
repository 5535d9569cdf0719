"""Throughput of the CollisionSplatting metric on one MI355X.

One step = one evaluation of the whole hot path (query preparation, the
float32 pair kernel with every per-query reduction for the m conservatism
values, the split combine, and the per-rollout epilogue: any collision and
summed cost over each rollout's 32 steps) over the MPPI-shaped navigation
workload:
1M Gaussians (room scene) x 32,768 robot spheres (1,024 rollouts x 32 steps,
r = 0.2 m), n_sigma in {0, 1, 2}, neighbourhood ball 1 m, k = 2, tau = 0.1.
Inputs are resident in HBM before the timed region.

Prints one JSON line.  The value is sphere-Gaussian pair evaluations per
second, counted as Q x N_kept per batch.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sphere-Gaussian pair evals/s + queries/s at stated label accuracy; p50/p99 latency"
PEAK_VALU = 256 * 4 * 16 * 2.4e9   # lane-ops/s: 256 CUs x 4 SIMD16 x 2.4 GHz (one VALU slot per lane-cycle)
COUNT_NOTE = ("frac: the method's operation count (a transcendental priced at 4 VALU slots), which can exceed "
              "the kernel's work (its transcendentals issue in 2 slots) and so pass 1; frac_tight_count: the "
              "kernel's own count; VALU issue by counters in profiles/")
PEAK_MFMA_BF16 = 2.5e15            # dense bf16/fp16 MFMA FLOP/s (published, no sparsity)


# The roofline's operation counts come from the method, not from the emitted
# instructions: FMA = 1, compare or count = 1, a transcendental (sqrt, exp) = 4.
def ops_full_in_ball(m):
    """All outputs, per pair inside the ball: shared d 3, |d|^2 3, M d 9, V 3,
    sqrt 4; per conservatism value about 30 (label 5, s~^2 with min and
    softmin 13, cost 10 and the sums): 22 + 30 m (110 for m = 3, 52 for m = 1)."""
    return 22 + 30 * m


def ops_labels(m):
    """Labels, per evaluated pair: d 3, D 3, M d 9, V 3; per value a, w, a|a|, cmp, count 5."""
    return 18 + 5 * m


OPS_MFMA_EPILOGUE = 7              # per pair of an evaluated 32 x 32 block: a, a|a|, f, cmp, count, bound, flag
FLOP_MFMA_PAIR = 64                # two contractions over K = 16 (padded from 10), 2 FLOP per MAC


# The tighter per-launch count of the kernels' own work (transcendentals at
# their measured half rate, 2 slots), reported beside the method's count.
OPS_ALL_PAIRS = 7                  # d (3), |d|^2 (3), ball test (1)
OPS_IN_BALL_SHARED = 15            # M d (9), V (3), sqrt (2 slots), ball count (1)
OPS_IN_BALL_PER_NSIGMA = 15        # s~^2 (2), label (2), min (1), softmin (exp 2 + 2), cost (exp 2 + 4)


# The pair kernel's HBM traffic comes from the rocprofv3 counter summary under
# profiles/ (FETCH_SIZE and WRITE_SIZE of the same command, scaled by what the
# counters read for a plain copy of known size).  It is reported only while
# the kernel sources still hash to the digest recorded with the counters.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pair_task_kernel_mppi_nav.md")
KERNEL_SOURCES = ("paper_2609_35619_amd/csrc/pair_core.h", "paper_2609_35619_amd/csrc/pair_fp32.hip",
                  "paper_2609_35619_amd/csrc/internal.h")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per pair-kernel launch from the committed counter summary, or
    None when the summary is missing or was taken on other kernel sources."""
    try:
        lines = open(TRAFFIC_PROFILE).read().splitlines()
    except OSError:
        return None
    rec = {}
    for ln in lines:
        if ln.startswith("traffic-record:"):
            for kv in ln.split(":", 1)[1].split():
                k, v = kv.split("=")
                rec[k] = v
    if rec.get("digest") != kernel_digest():
        return None
    return float(rec["fetch_bytes"]) + float(rec["write_bytes"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the CPU-oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision-form comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--no-ellipsoids", action="store_true", help="skip the ellipsoidal-body workload")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper-shaped context workload")
    ap.add_argument("--no-manip", action="store_true", help="skip the manipulation (sphere chain) workload")
    ap.add_argument("--no-tiny", action="store_true", help="skip the plain tiny configuration")
    ap.add_argument("--no-rrt", action="store_true", help="skip the batched RRT steps")
    ap.add_argument("--serving-requests", type=int, default=500)
    ap.add_argument("--serving-reduced", action="store_true",
                    help="serve a reduced request law (MPPI K <= 512 x 32 x <= 8 spheres; quick)")
    ap.add_argument("--section", choices=("all", "main", "precision", "precision-kernels", "serving", "ellipsoids",
                                          "manip", "paper", "tiny", "rrt", "copy", "digest", "sizes"), default="all",
                    help="run one part only (for profiling); 'copy' is a plain 1 GiB device copy "
                         "used to calibrate the HBM traffic counters")
    args = ap.parse_args()
    if args.section == "copy":
        return copy_calibration()
    if args.section == "digest":
        print(kernel_digest())
        return None
    if args.section == "precision-kernels":
        import paper_2609_35619_amd as cs
        cs.load_library()
        with cs.Engine(0) as eng:
            print(json.dumps(precision_kernels(cs, eng)), flush=True)
        return None
    if args.section == "sizes":
        import paper_2609_35619_amd as cs
        cs.load_library()
        with cs.Engine(0) as eng:
            print(json.dumps(sizes(cs, eng)), flush=True)
        return None
    if args.section != "all":
        args.no_precision = args.section not in ("precision",)
        args.no_serving = args.section not in ("serving",)
        args.no_ellipsoids = args.section not in ("ellipsoids",)
        args.no_paper = args.section not in ("paper",)
        args.no_manip = args.section not in ("manip",)
        args.no_tiny = args.section not in ("tiny",)
        args.no_rrt = args.section not in ("rrt",)
        args.no_cpu_baseline = True
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by queries with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2609_35619_amd as cs
    from workloads import config

    cs.load_library()
    log("bench: generating the mppi_nav workload")
    sc, qs, p = config("mppi_nav")
    dev = 0
    eng = cs.Engine(dev)
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    n_kept, scene_bytes = cs.csplat_scene_info(h)
    import hashlib
    dig = hashlib.sha256()
    for a in (sc.means, sc.quats, sc.scales, sc.opacity, qs.centers, qs.radii):
        dig.update(np.ascontiguousarray(a).tobytes())
    inputs_sha256 = dig.hexdigest()[:16]
    eng.set_conservatism(p["n_sigma"])
    m = len(p["n_sigma"])
    opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"],
                          s_min=p["s_min"])
    c = torch.from_numpy(qs.centers).to(f"cuda:{dev}")
    r = torch.from_numpy(qs.radii).to(f"cuda:{dev}")
    out = eng.alloc_outputs(qs.q)
    # planner epilogue of the step: per rollout (32 steps x 1 sphere), any
    # collision and the summed cost (Sec. II-D Eq. 11, Sec. II-E)
    n_roll = qs.q // 32
    seg_any = torch.empty((n_roll, m), dtype=torch.uint8, device=f"cuda:{dev}")
    seg_cost = torch.empty((n_roll, m), dtype=torch.float32, device=f"cuda:{dev}")
    torch.cuda.synchronize()

    def epilogue():
        cs.csplat_segment_reduce(eng.ctx, n_roll, label=out["label"], cost=out["cost"], seg_any=seg_any,
                                 seg_cost=seg_cost)

    log(f"bench: {n_kept} kept Gaussians, {qs.q} queries, m={m}; warmup {args.warmup}")
    for _ in range(args.warmup):
        eng.evaluate(h, c, r, opts, out=out)
        epilogue()
    torch.cuda.synchronize()

    # timed region: K steps bracketed by synchronisations
    t0 = time.perf_counter()
    for _ in range(args.steps):
        eng.evaluate(h, c, r, opts, out=out)
        epilogue()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps

    # per-step latency and the pair kernel's own duration (HIP events on the
    # context stream), outside the throughput window
    cs.csplat_ctx_set_timing(eng.ctx, True)
    lat, kms = [], []
    for _ in range(args.steps):
        s0 = time.perf_counter()
        eng.evaluate(h, c, r, opts, out=out)
        st = cs.csplat_last_stats(eng.ctx)
        epilogue()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
        kms.append(st["kernel_ms"])
    cs.csplat_ctx_set_timing(eng.ctx, False)
    kernel_s = float(np.mean(kms)) / 1e3
    # the same step from host arrays (inputs copied in, outputs copied back
    # over PCIe inside the call): reported beside the resident-input value
    host_out = eng.alloc_outputs(qs.q, like="host")
    eng.evaluate(h, qs.centers, qs.radii, opts, out=host_out)
    host_t = []
    for _ in range(max(3, args.steps // 4)):
        s0 = time.perf_counter()
        eng.evaluate(h, qs.centers, qs.radii, opts, out=host_out)
        host_t.append(time.perf_counter() - s0)
    gpu = {k: v.cpu().numpy() for k, v in out.items()}
    nbr_total = int(gpu["nbr"].astype(np.int64).sum())
    pairs = qs.q * n_kept
    # the roofline counts the pairs the kernel evaluated: pairs in chunks
    # skipped by the exact reach-bound test cost no arithmetic (every in-ball
    # pair is evaluated); the dense count is reported beside it
    evaluated = int(st["kernel_pairs"])
    ops = ops_full_in_ball(m) * nbr_total
    ops_tight = OPS_ALL_PAIRS * evaluated + (OPS_IN_BALL_SHARED + OPS_IN_BALL_PER_NSIGMA * m) * nbr_total
    achieved = ops / kernel_s
    res = {
        "metric": METRIC,
        "value": pairs / step_s,
        "unit": "pair evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mppi_nav: 1M-Gaussian room scene (80% walls/floor, 20% in 50 clusters), "
                               "1024 rollouts x 32 steps x 1 sphere r=0.2 m, n_sigma {0,1,2}, "
                               "neighbourhood ball 1 m, k=2, tau=0.1, d_max=1, gamma=1, s_min=1; "
                               "outputs label, count, min, softmin, cost, nbr",
                   "n_gaussians": int(sc.n), "n_kept": int(n_kept), "queries": int(qs.q), "m": m,
                   "global_batch": int(qs.q), "parallelism": "single GPU", "inputs_sha256": inputs_sha256},
        "value_definition": "dense-equivalent sphere-Gaussian pair evaluations per second: Q x N_kept per step; "
                            "exact culling answers most pairs without evaluating them (their contribution is "
                            "provably none), evaluated_pair_evals_per_s counts the pairs the kernel evaluated",
        "evaluated_pair_evals_per_s": evaluated / step_s,
        "queries_per_s": qs.q / step_s,
        "rollout_epilogue": {"rollouts": n_roll, "in_collision_per_n_sigma": seg_any.sum(0).tolist()},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                       "mean": float(np.mean(lat) * 1e3), "std": float(np.std(lat) * 1e3)},
        "host_arrays": {"ms_per_step_median": float(np.median(host_t) * 1e3),
                        "pair_evals_per_s": pairs / float(np.median(host_t)),
                        "note": "inputs from and outputs to host memory, PCIe copies inside the call"},
        "vram_bytes": {"scene": int(scene_bytes), "workspace": int(st["workspace_bytes"])},
        "roofline": {"bound": "alu", "achieved": achieved / 1e9, "peak": PEAK_VALU / 1e9, "unit": "Gop/s",
                     "frac": achieved / PEAK_VALU, "traffic": traffic_from_profile(), "traffic_unit": "bytes",
                     "kernel": "pair_task_kernel<3,cull,sphere>", "kernel_ms": kernel_s * 1e3,
                     "ops_per_unit": ops_full_in_ball(m), "unit_of_work": "pair inside the 1 m ball",
                     "units_per_launch": nbr_total, "ops_per_launch": ops, "evaluated_pairs": evaluated,
                     "tight_ops_per_launch": ops_tight, "frac_tight_count": ops_tight / kernel_s / PEAK_VALU, "count_note": COUNT_NOTE,
                     "dense_pairs": pairs},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"], res["label_accuracy"] = cpu_baseline(sc, qs, p, gpu, args.cpu_seconds, n_kept)
    if not args.no_precision:
        res["precision_form"] = precision_form(cs, eng, not args.no_cpu_baseline)
    if not args.no_tiny:
        res["tiny"] = tiny(cs, eng, args.steps)
    if not args.no_manip:
        res["manip"] = manip(cs, eng, args.steps)
    if not args.no_ellipsoids:
        res["ellipsoids"] = ellipsoids(cs, eng, args.steps)
    if not args.no_paper:
        res["paper_context"] = paper_context(cs, eng)
    if not args.no_rrt:
        res["rrt"] = rrt(cs, eng, h, 100)
    if not args.no_serving:
        res["serving"] = serving(cs, eng, sc, h, args.serving_requests, args.serving_reduced)
    cs.csplat_scene_free(h)
    eng.close()
    print(json.dumps(res), flush=True)


def copy_calibration():
    """One device-to-device copy of 1 GiB: the HBM bytes it moves are known
    (1 GiB read, 1 GiB written), which calibrates FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4}), flush=True)


def _time_eval(eng, h, c, r, opts, want, reps=3):
    import torch
    out = eng.alloc_outputs(c.shape[0], want)
    eng.evaluate(h, c, r, opts, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        eng.evaluate(h, c, r, opts, out=out)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, {k: v.cpu().numpy() for k, v in out.items()}


OPS_ELL_SHARED = 36   # L d (9), s^2 (3), L^T e (9), M h (9), W (3), sqrt (2), ball count (1)


def manip(cs, eng, steps):
    """The manipulation workload: the 500k-Gaussian tabletop against 256
    configurations x 32 steps x 48 spheres of a 7-link chain (393,216
    spheres), all outputs, n_sigma = 1, neighbourhood ball 0.3 m."""
    import torch
    from workloads import config
    log("bench: manipulation (500k Gaussians x 393,216 chain spheres)")
    sc, qs, p = config("manip")
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    n_kept, _ = cs.csplat_scene_info(h)
    eng.set_conservatism(p["n_sigma"])
    m = len(p["n_sigma"])
    opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"],
                          s_min=p["s_min"])
    c = torch.from_numpy(qs.centers).cuda()
    r = torch.from_numpy(qs.radii).cuda()
    out = eng.alloc_outputs(qs.q)
    for _ in range(2):
        eng.evaluate(h, c, r, opts, out=out)
    torch.cuda.synchronize()
    reps = max(5, steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        eng.evaluate(h, c, r, opts, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    cs.csplat_ctx_set_timing(eng.ctx, True)
    kms = []
    for _ in range(3):
        eng.evaluate(h, c, r, opts, out=out)
        st = cs.csplat_last_stats(eng.ctx)
        kms.append(st["kernel_ms"])
    cs.csplat_ctx_set_timing(eng.ctx, False)
    nbr = int(out["nbr"].cpu().numpy().astype(np.int64).sum())
    cs.csplat_scene_free(h)
    ops = ops_full_in_ball(m) * nbr
    tight = OPS_ALL_PAIRS * int(st["kernel_pairs"]) + (OPS_IN_BALL_SHARED + OPS_IN_BALL_PER_NSIGMA * m) * nbr
    kernel_s = float(np.mean(kms)) / 1e3
    return {"workload": "manip: 500k-Gaussian tabletop, 256 configurations x 32 steps x 48 chain spheres "
                        "(r 0.03-0.10 m), n_sigma 1, ball 0.3 m, all outputs",
            "n_kept": int(n_kept), "queries": int(qs.q), "ms_per_step": dt * 1e3,
            "pair_evals_per_s": qs.q * n_kept / dt, "queries_per_s": qs.q / dt,
            "roofline": {"bound": "alu", "achieved": ops / kernel_s / 1e9, "peak": PEAK_VALU / 1e9,
                         "unit": "Gop/s", "frac": ops / kernel_s / PEAK_VALU, "kernel_ms": kernel_s * 1e3,
                         "ops_per_unit": ops_full_in_ball(m), "unit_of_work": "pair inside the 0.3 m ball",
                         "units_per_launch": nbr, "frac_tight_count": tight / kernel_s / PEAK_VALU, "count_note": COUNT_NOTE,
                         "evaluated_pairs": int(st["kernel_pairs"])}}


def ellipsoids(cs, eng, steps):
    """Ellipsoidal links: the tabletop scene (500k Gaussians) against 256
    configurations x 32 steps x 7 chain links as ellipsoids, all outputs,
    n_sigma = 1, neighbourhood ball 0.4 m."""
    import torch
    from workloads import config
    log("bench: ellipsoidal links (500k Gaussians x 57,344 link ellipsoids)")
    sc, b, p = config("manip_ell")
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    n_kept, _ = cs.csplat_scene_info(h)
    eng.set_conservatism(p["n_sigma"])
    m = len(p["n_sigma"])
    opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"],
                          s_min=p["s_min"])
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (b.centers, b.quats, b.axes)]
    out = eng.alloc_outputs(b.q)
    for _ in range(2):
        eng.evaluate_ellipsoids(h, *t, opts, out=out)
    torch.cuda.synchronize()
    reps = max(5, steps // 2)
    t0 = time.perf_counter()
    for _ in range(reps):
        eng.evaluate_ellipsoids(h, *t, opts, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    cs.csplat_ctx_set_timing(eng.ctx, True)
    kms = []
    for _ in range(3):
        eng.evaluate_ellipsoids(h, *t, opts, out=out)
        st = cs.csplat_last_stats(eng.ctx)
        kms.append(st["kernel_ms"])
    cs.csplat_ctx_set_timing(eng.ctx, False)
    nbr = int(out["nbr"].cpu().numpy().astype(np.int64).sum())
    cs.csplat_scene_free(h)
    labels = ellipsoid_labels(cs, eng, sc, b, p)
    ops = (ops_full_in_ball(m) + 18) * nbr   # L d, L^T e: +18 over a sphere
    tight = OPS_ALL_PAIRS * int(st["kernel_pairs"]) + (OPS_ELL_SHARED + OPS_IN_BALL_PER_NSIGMA * m) * nbr
    kernel_s = float(np.mean(kms)) / 1e3
    return {"workload": "manip_ell: 500k-Gaussian tabletop, 256 configurations x 32 steps x 7 link ellipsoids "
                        "(semi-axes r, r, L/2 + r), n_sigma 1, ball 0.4 m, all outputs",
            "n_kept": int(n_kept), "bodies": int(b.q), "ms_per_step": dt * 1e3,
            "pair_evals_per_s": b.q * n_kept / dt, "queries_per_s": b.q / dt,
            "roofline": {"bound": "alu", "achieved": ops / kernel_s / 1e9, "peak": PEAK_VALU / 1e9,
                         "unit": "Gop/s", "frac": ops / kernel_s / PEAK_VALU, "kernel_ms": kernel_s * 1e3,
                         "ops_per_unit": ops_full_in_ball(m) + 18, "unit_of_work": "pair inside the 0.4 m ball",
                         "units_per_launch": nbr, "frac_tight_count": tight / kernel_s / PEAK_VALU, "count_note": COUNT_NOTE,
                         "evaluated_pairs": int(st["kernel_pairs"])},
            "labels_every_gaussian": labels}


# The ellipsoid MFMA kernel per 32 x 32 block: one MFMA for each f_k and three
# for each e_k (32 x 32 x 16 each), and per pair about 25 VALU operations of
# epilogue (the squares and sums of f~ and e~, the bounds, the test, the counts).
FLOP_MFMA_ELL_BLOCK = 12 * 32 * 32 * 16 * 2
OPS_MFMA_ELL_EPILOGUE = 25


def ellipsoid_labels(cs, eng, sc, b, p):
    """Labels and counts of the same link ellipsoids over every kept Gaussian
    (n_sigma 1, k 2) in float32, bf16 and fp16 (the MFMA forms: certified
    bound, fp64 recheck), their time, recheck rate and agreement with the
    FP64 oracle on 256 seeded bodies plus up to 256 rechecked ones."""
    import torch
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import compare
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"],
                       precision_features=cs.CSPLAT_FEATURES_ELL_BF16 | cs.CSPLAT_FEATURES_ELL_FP16)
    eng.set_conservatism([1.0])
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (b.centers, b.quats, b.axes)]
    res, outs = {}, {}
    for name, prec in (("fp32", cs.CSPLAT_PRECISION_FP32), ("bf16", cs.CSPLAT_PRECISION_BF16_RECHECK),
                       ("fp16", cs.CSPLAT_PRECISION_FP16_RECHECK)):
        opts = cs.reduce_opts(k=2, r_nbr=math.inf, precision=prec)
        out = eng.alloc_outputs(b.q, ("label", "count"))
        eng.evaluate_ellipsoids(h, *t, opts, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            eng.evaluate_ellipsoids(h, *t, opts, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        cs.csplat_ctx_set_timing(eng.ctx, True)
        eng.evaluate_ellipsoids(h, *t, opts, out=out)
        st = cs.csplat_last_stats(eng.ctx)
        rk = cs.csplat_last_rechecked(eng.ctx)
        cs.csplat_ctx_set_timing(eng.ctx, False)
        torch.cuda.synchronize()
        outs[name] = ({k: v.cpu().numpy() for k, v in out.items()}, rk)
        d = {"ms": dt * 1e3, "kernel_ms": st["kernel_ms"], "rechecked_bodies": int(rk.size)}
        # labels alone (the RRT's question): a body is certain once its
        # bracket of counts decides count > k
        lab = eng.alloc_outputs(b.q, ("label",))
        eng.evaluate_ellipsoids(h, *t, opts, out=lab)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            eng.evaluate_ellipsoids(h, *t, opts, out=lab)
        torch.cuda.synchronize()
        d["labels_only_ms"] = (time.perf_counter() - t0) / 5 * 1e3
        d["labels_only_rechecked_bodies"] = int(cs.csplat_last_rechecked(eng.ctx).size)
        assert np.array_equal(lab["label"].cpu().numpy(), outs[name][0]["label"])
        if prec == cs.CSPLAT_PRECISION_FP32:
            d["evaluated_pairs"] = int(st["kernel_pairs"])
        else:
            blocks = int(st["kernel_pairs"]) // 1024
            k_s = st["kernel_ms"] / 1e3
            d["mfma_blocks_32x32"] = blocks
            d["roofline_mfma"] = {"bound": "mfma", "achieved": FLOP_MFMA_ELL_BLOCK * blocks / k_s / 1e12,
                                  "peak": PEAK_MFMA_BF16 / 1e12, "unit": "TFLOP/s",
                                  "frac": FLOP_MFMA_ELL_BLOCK * blocks / k_s / PEAK_MFMA_BF16}
            d["roofline_valu"] = {"bound": "alu", "ops_per_unit": OPS_MFMA_ELL_EPILOGUE, "unit_of_work":
                                  "pair of an evaluated 32 x 32 block", "units_per_launch": blocks * 1024,
                                  "frac": OPS_MFMA_ELL_EPILOGUE * blocks * 1024 / k_s / PEAK_VALU}
        res[name] = d
    cs.csplat_scene_free(h)
    rng = np.random.default_rng(61)
    sample = np.sort(rng.choice(b.q, 256, replace=False))
    rk_all = np.unique(np.concatenate([outs["bf16"][1], outs["fp16"][1]]))
    if rk_all.size > 256:
        rk_all = np.sort(rng.choice(rk_all, 256, replace=False))
    idx = np.unique(np.concatenate([sample, rk_all])).astype(np.int64)
    ref = oracle.evaluate_ellipsoids(sc, b.subset(idx), [1.0], alpha_f=p["alpha_f"], extent_f=p["extent_f"], k=2)
    for name in res:
        got = {k: v[idx] for k, v in outs[name][0].items()}
        s = compare(got, ref, tau=0.0, gamma=1.0, where=f"ell-labels-{name}")
        amb = ref["ambiguous"].astype(bool)
        res[name]["oracle_sample"] = int(idx.size)
        res[name]["label_flips_vs_oracle_outside_band"] = int(((got["label"] != ref["label"]) & ~amb).sum())
        res[name]["count_exact_fraction"] = s.get("count_exact")
    res["workload"] = "the same link ellipsoids, labels and counts over every kept Gaussian, n_sigma 1, k 2"
    return res


def paper_context(cs, eng):
    """Shaped like the paper's own measurement (Table I): a 200k-Gaussian unit
    scene, grid points as spheres of radius 0.015, collision labels for
    batches of 4,096 and 32,768, n_sigma = 1.  The paper's numbers were taken on
    other hardware with its own scene: context only."""
    import torch
    from workloads import config, grid_queries
    log("bench: paper-shaped context (200k Gaussians, batches 4,096 and 32,768)")
    sc, _, p = config("paper_p0")
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    n_kept, nbytes = cs.csplat_scene_info(h)
    eng.set_conservatism(p["n_sigma"])
    opts = cs.reduce_opts(k=p["k"], r_nbr=math.inf)
    out = {"workload": "paper_p0: 200k-Gaussian unit scene (ring of columns and lintels, 20% clutter), "
                       "grid points r = 0.015, n_sigma 1, k = 2, labels",
           "n_kept": int(n_kept), "scene_bytes": int(nbytes),
           "paper_table_I_context": {"hardware": "RTX 6000 Pro (Warp)", "checks_per_s_4096": 215578.9,
                                     "checks_per_s_32768": 1638400.0, "vram_gb": 0.166}}
    for res_, name in ((16, "batch_4096"), (32, "batch_32768")):
        qs = grid_queries(res_, size=(1.0, 1.0, 0.6), radius_classes=(0.015,))
        c, r = torch.from_numpy(qs.centers).cuda(), torch.from_numpy(qs.radii).cuda()
        dt, _ = _time_eval(eng, h, c, r, opts, ("label",), reps=20)
        out[name] = {"ms": dt * 1e3, "checks_per_s": qs.q / dt, "pair_evals_per_s": qs.q * n_kept / dt}
    cs.csplat_scene_free(h)
    return out


def _timed(cs, eng, h, c, r, opts, want, reps=5):
    """Mean wall time per evaluation (after one warm-up) and the statistics
    of one more with the kernel timing on."""
    import torch
    out = eng.alloc_outputs(c.shape[0], want)
    eng.evaluate(h, c, r, opts, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        eng.evaluate(h, c, r, opts, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    cs.csplat_ctx_set_timing(eng.ctx, True)
    eng.evaluate(h, c, r, opts, out=out)
    st = cs.csplat_last_stats(eng.ctx)
    rk = cs.csplat_last_rechecked(eng.ctx)
    cs.csplat_ctx_set_timing(eng.ctx, False)
    torch.cuda.synchronize()
    return dt, st, rk, {k: v.cpu().numpy() for k, v in out.items()}


def precision_form(cs, eng, cpu_baseline_on):
    """The 4M-Gaussian x 262,144-sphere grid workload (and its stress variant,
    half the points near a surface): labels, and labels plus the hard minimum,
    in fp32, bf16 and fp16; rooflines of the float32 label kernel and the MFMA
    kernel; accuracy against the FP64 oracle on 1,024 seeded queries per
    radius class plus every query a precision form rechecked."""
    import torch
    import oracle
    from workloads import config, grid_queries
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import compare
    log("bench: precision form (4M Gaussians x 262,144 grid spheres)")
    sc, qs, p = config("precision")
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"],
                       precision_features=cs.CSPLAT_FEATURES_BF16 | cs.CSPLAT_FEATURES_FP16)
    n_kept, nbytes = cs.csplat_scene_info(h)
    eng.set_conservatism(p["n_sigma"])
    out = {"workload": "precision: 4M-Gaussian room scene, 64^3 grid spheres in 4 radius classes "
                       "{0.05,0.1,0.2,0.4} m, n_sigma 1, k=2; labels, and labels plus the hard minimum",
           "n_kept": int(n_kept), "queries": int(qs.q), "scene_bytes_with_features": int(nbytes)}
    dtypes = (("fp32", cs.CSPLAT_PRECISION_FP32), ("bf16", cs.CSPLAT_PRECISION_BF16_RECHECK),
              ("fp16", cs.CSPLAT_PRECISION_FP16_RECHECK))
    radii = np.unique(qs.radii)

    def run_set(queries, tag):
        c = torch.from_numpy(queries.centers).cuda()
        r = torch.from_numpy(queries.radii).cuda()
        res, lab, mins, rk_all = {}, {}, {}, []
        for name, prec in dtypes:
            opts = cs.reduce_opts(k=p["k"], r_nbr=math.inf, precision=prec)
            dt, st, rk, o = _timed(cs, eng, h, c, r, opts, ("label",))
            d = {"labels_ms": dt * 1e3, "labels_kernel_ms": st["kernel_ms"], "rechecked_queries": int(rk.size),
                 "rechecked_fraction_per_radius_class":
                     {f"r={rv:.2f}": float(np.isin(rk, np.nonzero(queries.radii == rv)[0]).sum() /
                                           max(1, (queries.radii == rv).sum())) for rv in radii}}
            k_s = st["kernel_ms"] / 1e3
            if prec == cs.CSPLAT_PRECISION_FP32:
                ev = int(st["kernel_pairs"])
                d["labels_roofline"] = {"bound": "alu", "kernel": "pair_task_kernel<1,labels,cull>",
                                        "ops_per_unit": ops_labels(1), "unit_of_work": "evaluated pair",
                                        "units_per_launch": ev, "achieved": ops_labels(1) * ev / k_s / 1e9,
                                        "peak": PEAK_VALU / 1e9, "unit": "Gop/s",
                                        "frac": ops_labels(1) * ev / k_s / PEAK_VALU, "kernel_ms": k_s * 1e3}
            else:
                blocks = int(st["kernel_pairs"]) // 1024
                bp = blocks * 1024
                d["labels_roofline"] = {"bound": "alu", "kernel": f"mfma_label_kernel<{name}>",
                                        "unit_of_work": "pair of an evaluated 32x32 block", "units_per_launch": bp,
                                        "blocks": blocks, "ops_per_unit": OPS_MFMA_EPILOGUE,
                                        "achieved": OPS_MFMA_EPILOGUE * bp / k_s / 1e9, "peak": PEAK_VALU / 1e9,
                                        "unit": "Gop/s", "frac": OPS_MFMA_EPILOGUE * bp / k_s / PEAK_VALU,
                                        "mfma_tflops": FLOP_MFMA_PAIR * bp / k_s / 1e12,
                                        "mfma_frac": FLOP_MFMA_PAIR * bp / k_s / PEAK_MFMA_BF16, "kernel_ms": k_s * 1e3}
                rk_all.append(rk)
            lab[name] = o["label"]
            want = ("label", "min") + (("err",) if prec != cs.CSPLAT_PRECISION_FP32 else ())
            dt2, st2, _, o2 = _timed(cs, eng, h, c, r, opts, want, reps=3)
            d.update({"labels_min_ms": dt2 * 1e3, "labels_min_kernel_ms": st2["kernel_ms"],
                      "min_passes": int(st2["min_passes"])})
            mins[name] = o2
            res[name] = d
            log(f"bench: precision {tag} {name}: labels {dt * 1e3:.2f} ms, labels+min {dt2 * 1e3:.2f} ms")
        for name in ("bf16", "fp16"):
            res[name]["labels_speedup_vs_fp32"] = res["fp32"]["labels_ms"] / res[name]["labels_ms"]
            res[name]["labels_min_speedup_vs_fp32"] = res["fp32"]["labels_min_ms"] / res[name]["labels_min_ms"]
        return res, lab, mins, rk_all

    def accuracy(queries, lab, mins, rk_all, per_class, seed, max_rechecked=None):
        rng = np.random.default_rng(seed)
        idx = [rng.choice(np.nonzero(queries.radii == rv)[0], per_class, replace=False) for rv in radii]
        rk = np.unique(np.concatenate(rk_all)) if rk_all else np.zeros(0, np.int64)
        if max_rechecked is not None and rk.size > max_rechecked:
            rk = np.sort(rng.choice(rk, max_rechecked, replace=False))
        idx = np.unique(np.concatenate(idx + [rk]))
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        oracle.build(force=False)
        _, mu, sig = oracle.prepare_scene(sc.means, sc.quats, sc.scales, sc.opacity,
                                          alpha_f=p["alpha_f"], extent_f=p["extent_f"])
        sub = queries.subset(idx)
        t0 = time.perf_counter()
        ref = oracle.evaluate(mu, sig, sub.centers, oracle.sphere_bodies(sub.radii), p["n_sigma"], k=p["k"],
                              nthreads=threads)
        o_s = time.perf_counter() - t0
        amb = ref["ambiguous"][:, 0].astype(bool)
        acc = {"sample_queries": int(idx.size), "ambiguous_queries": int(amb.sum()),
               "sample": f"{per_class} seeded queries per radius class plus {rk.size} of the "
                         f"{sum(x.size for x in rk_all)} queries the precision forms rechecked"}
        fin = np.isfinite(ref["min"][:, 0])
        for name in lab:
            flips = lab[name][idx, 0] != ref["label"][:, 0]
            g = mins[name]["min"][idx, 0].astype(np.float64)
            e = np.abs(g[fin] - ref["min"][fin, 0])
            rel = e / np.maximum(1.0, np.abs(ref["min"][fin, 0]))
            a = {"label_flips_outside_eps_band": int((flips & ~amb).sum()),
                 "label_flips_inside_eps_band": int((flips & amb).sum()),
                 "labels_min_label_flips_outside_eps_band": int(((mins[name]["label"][idx, 0] != ref["label"][:, 0])
                                                                  & ~amb).sum()),
                 "min_abs_error_max": float(e.max(initial=0)), "min_abs_error_p99": float(np.percentile(e, 99)),
                 "min_rel_error_max": float(rel.max(initial=0)), "min_rel_error_p99": float(np.percentile(rel, 99))}
            if "err" in mins[name]:
                eb = mins[name]["err"][idx, 0].astype(np.float64)[fin]
                a["min_outside_certified_err"] = int((e > eb).sum())
                a["certified_err_p50"] = float(np.median(eb))
                a["certified_err_p99"] = float(np.percentile(eb, 99))
            else:
                st_ = compare({"min": mins[name]["min"][idx]}, ref, tau=0.0, gamma=1.0, where="bench-precision")
                a["min_within_tolerance"] = True
                a.update(st_)
            acc[name] = a
        cpu = {"value": idx.size * n_kept / o_s, "unit": "pair evals/s", "cores": threads, "kind": "oracle",
               "sample": f"{idx.size} of {queries.q} queries against all {n_kept} kept Gaussians, labels and min, FP64",
               "seconds": o_s, "queries_per_s": idx.size / o_s}
        return acc, cpu

    res, lab, mins, rk_all = run_set(qs, "grid")
    out.update(res)
    out["accuracy_vs_oracle"], cpu = accuracy(qs, lab, mins, rk_all, 1024, 4)
    if cpu_baseline_on:
        out["cpu_baseline"] = cpu
    log("bench: precision stress variant (half the points near a surface)")
    qs2 = grid_queries(64, stress_scene=sc, seed=104)
    res2, lab2, mins2, rk2 = run_set(qs2, "stress")
    acc2, _ = accuracy(qs2, lab2, mins2, rk2, 256, 5, max_rechecked=2048)
    out["stress"] = {"workload": "stress: half of the 64^3 grid points replaced by points at 0.5-1.5 r from a mean",
                     **res2, "accuracy_vs_oracle": acc2}
    cs.csplat_scene_free(h)
    return out


def precision_kernels(cs, eng):
    """Config 4's kernels alone, for profiling: labels in fp32, bf16 and fp16
    (three evaluations each), then labels plus the minimum in fp32 and bf16
    (one each)."""
    import torch
    from workloads import config
    sc, qs, p = config("precision")
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"],
                       precision_features=cs.CSPLAT_FEATURES_BF16 | cs.CSPLAT_FEATURES_FP16)
    eng.set_conservatism(p["n_sigma"])
    c = torch.from_numpy(qs.centers).cuda()
    r = torch.from_numpy(qs.radii).cuda()
    res = {}
    for name, prec in (("fp32", cs.CSPLAT_PRECISION_FP32), ("bf16", cs.CSPLAT_PRECISION_BF16_RECHECK),
                       ("fp16", cs.CSPLAT_PRECISION_FP16_RECHECK)):
        opts = cs.reduce_opts(k=p["k"], r_nbr=math.inf, precision=prec)
        dt, st, _, _ = _timed(cs, eng, h, c, r, opts, ("label",), reps=3)
        res[name] = {"labels_ms": dt * 1e3, "kernel_ms": st["kernel_ms"], "kernel_pairs": st["kernel_pairs"]}
        if name != "fp16":
            want = ("label", "min") + (("err",) if name != "fp32" else ())
            dt2, st2, _, _ = _timed(cs, eng, h, c, r, opts, want, reps=1)
            res[name].update({"labels_min_ms": dt2 * 1e3, "labels_min_kernel_ms": st2["kernel_ms"]})
    cs.csplat_scene_free(h)
    return res


def rrt(cs, eng, h_nav, n_steps):
    """The batched RRT step (Sec. II-E) on the 1M navigation scene: a robot of
    three link spheres translating in the room, strides of 0.5 m checked every
    5 cm (10 states per edge), n_sigma 1, k = 2; the paper's 32 samples per
    step, and 1,024."""
    import torch
    log("bench: RRT steps on the navigation scene")
    links = np.array([[0.0, 0.0, 0.0], [0.15, 0.0, 0.0], [0.0, 0.0, 0.25]], np.float32)
    radii = np.array([0.12, 0.08, 0.06], np.float32)
    out = {"workload": "rrt: 1M-Gaussian room, 3-link robot (r 0.12, 0.08, 0.06 m) translating in "
                       "[0.3, 9.7]^2 x [0.2, 2.5], stride 0.5 m, checks every 0.05 m (10 states per edge), "
                       "n_sigma 1, k 2, root (3, 3, 1) m, samples drawn on the device"}
    for nb in (32, 1024):
        t = cs.Rrt(eng.ctx, h_nav, (0.3, 0.3, 0.2), (9.7, 9.7, 2.5), 0.5, 0.05, 1.0, 2, links, radii,
                   (3.0, 3.0, 1.0), 2_000_000, seed=3)
        for _ in range(3):
            t.step(nb)
        torch.cuda.synchronize()
        cs.csplat_synchronize(eng.ctx)
        t0 = time.perf_counter()
        for _ in range(n_steps):
            t.step(nb)
        cs.csplat_synchronize(eng.ctx)
        dt = (time.perf_counter() - t0) / n_steps
        nodes, _ = t.nodes()
        t.close()
        out[f"batch_{nb}"] = {"ms_per_step": dt * 1e3, "steps_per_s": 1 / dt, "edges_per_s": nb / dt,
                              "sphere_checks_per_s": nb * 10 * 3 / dt, "nodes_after": int(nodes.shape[0]),
                              "steps": n_steps + 3}
    return out


def tiny(cs, eng, steps):
    """The plain tiny configuration: 10,000 Gaussians in a 4 x 4 x 2 m box x
    4,096 spheres (r = 0.1), n_sigma 1, every output over every Gaussian."""
    import torch
    from workloads import config
    sc, qs, p = config("tiny")
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    n_kept, _ = cs.csplat_scene_info(h)
    eng.set_conservatism(p["n_sigma"])
    opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=math.inf, d_max=p["d_max"], gamma=p["gamma"],
                          s_min=p["s_min"])
    c = torch.from_numpy(qs.centers).cuda()
    r = torch.from_numpy(qs.radii).cuda()
    dt, st, _, _ = _timed(cs, eng, h, c, r, opts, ("label", "count", "min", "softmin", "cost", "nbr"),
                          reps=max(10, steps))
    cs.csplat_scene_free(h)
    return {"workload": "tiny: 10k Gaussians uniform in 4x4x2 m, 4,096 spheres r = 0.1 m, n_sigma 1, all outputs",
            "n_kept": int(n_kept), "queries": int(qs.q), "ms_per_step": dt * 1e3,
            "pair_evals_per_s": qs.q * n_kept / dt, "queries_per_s": qs.q / dt, "kernel_ms": st["kernel_ms"]}


def sizes(cs, eng):
    """The navigation workload's law at other sizes: room scenes of 250k, 1M
    and 4M Gaussians against 256, 1,024 and 4,096 rollouts x 32 steps (8,192
    to 131,072 spheres, r = 0.2 m), three n_sigma values, every output over
    the 1 m ball.  Per size: time per evaluation, the pair kernel's time and
    its roofline fraction by the method's count, dense-equivalent and
    evaluated pairs per second."""
    import torch
    from workloads import config, mppi_walk_queries, room_scene
    _, _, p = config("mppi_nav", 0.001)
    m = len(p["n_sigma"])
    opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"],
                          s_min=p["s_min"])
    res = []
    for n in (250_000, 1_000_000, 4_000_000):
        log(f"bench: sizes, {n} Gaussians")
        sc = room_scene(n, seed=2)
        h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
        n_kept, _ = cs.csplat_scene_info(h)
        eng.set_conservatism(p["n_sigma"])
        for rollouts in (256, 1024, 4096):
            qs = mppi_walk_queries(rollouts, 32, seed=102)
            c = torch.from_numpy(qs.centers).cuda()
            r = torch.from_numpy(qs.radii).cuda()
            dt, st, _, o = _timed(cs, eng, h, c, r, opts, ("label", "count", "min", "softmin", "cost", "nbr"),
                                  reps=10)
            k_s = st["kernel_ms"] / 1e3
            nbr = int(o["nbr"].astype(np.int64).sum())
            ev = int(st["kernel_pairs"])
            tight = OPS_ALL_PAIRS * ev + (OPS_IN_BALL_SHARED + OPS_IN_BALL_PER_NSIGMA * m) * nbr
            res.append({"n_kept": int(n_kept), "queries": int(qs.q), "splits": int(st["splits"]),
                        "ms_per_step": dt * 1e3, "kernel_ms": k_s * 1e3,
                        "roofline_frac": ops_full_in_ball(m) * nbr / k_s / PEAK_VALU,
                        "roofline_frac_tight_count": tight / k_s / PEAK_VALU, "evaluated_pairs": ev,
                        "dense_pair_evals_per_s": qs.q * n_kept / dt,
                        "evaluated_pair_evals_per_s": int(st["kernel_pairs"]) / dt,
                        "in_ball_pairs": nbr})
        cs.csplat_scene_free(h)
    return {"workload": "mppi_nav law at other sizes: room scenes x rollouts x 32 steps x 1 sphere r = 0.2 m, "
                        "n_sigma {0,1,2}, ball 1 m, every output",
            "note": "roofline_frac prices a transcendental at 4 VALU slots (the method's count); the kernels "
                    "issue them in 2, so by that count a launch dominated by in-ball pairs can exceed 1; "
                    "roofline_frac_tight_count is the kernel's own count",
            "runs": res}


def serving(cs, eng, sc_nav, h_nav, n_requests, reduced):
    """The serving form with the 1M (navigation) and 4M (room) scenes resident:
    a Poisson stream mixing MPPI batches (K in {256..4096} x 32 steps x 1-48
    spheres) and RRT edge checks (1-10,000 points x 1-48 spheres).  The
    saturated request rate is measured first (every request at t = 0); the
    same stream then arrives at half that rate.  Latency is reported from the
    library's submit entry to results in host memory, and from each request's
    scheduled arrival to the moment a client thread collected it."""
    import threading
    from workloads import config, serving_stream
    log("bench: serving (1M + 4M resident scenes)")
    sc4, _, p4 = config("precision")
    h4 = eng.load_scene(sc4, floater_opacity_max=p4["alpha_f"], floater_extent_min=p4["extent_f"])
    kw = dict(max_mppi_k=512, max_rrt_points=4000, max_spheres=8) if reduced else \
        dict(max_mppi_k=4096, max_rrt_points=10000, max_spheres=48)
    mppi_opts = cs.reduce_opts(k=2, tau=0.1, r_nbr=1.0, d_max=1.0, gamma=1.0, s_min=1.0)
    rrt_opts = cs.reduce_opts(k=2, r_nbr=math.inf)
    n_scene = [cs.csplat_scene_info(h_nav)[0], cs.csplat_scene_info(h4)[0]]

    def run(reqs, rate):
        # one thread submits at the arrival times, another collects finished
        # requests as they complete (a finished request holds its output
        # staging until it is collected)
        srv = cs.csplat_server_create(0, 4 << 30, 16)
        ids = [cs.csplat_server_add_scene(srv, h_nav), cs.csplat_server_add_scene(srv, h4)]
        pending, lock, submitted = {}, threading.Lock(), threading.Event()
        arrival_lat = {}

        def collect():
            last = time.perf_counter()
            while True:
                with lock:
                    items = list(pending.items())
                if not items and submitted.is_set():
                    return
                for t, (kind, q, t_arr, i) in items:
                    if cs.csplat_server_poll(srv, t, q, kind) is not None:
                        arrival_lat[i] = time.perf_counter() - t_arr
                        with lock:
                            del pending[t]
                if time.perf_counter() - last > 10.0:
                    last = time.perf_counter()
                    log(f"bench: serving: {len(arrival_lat)} of {len(reqs)} requests collected")
                time.sleep(0.001)

        th = threading.Thread(target=collect)
        t0 = time.perf_counter()
        th.start()
        for i, rq in enumerate(reqs):
            t_arr = t0 + (rq["t"] / rate if rate else 0.0)
            while time.perf_counter() < t_arr:
                time.sleep(0.0002)
            kind = cs.CSPLAT_SERVE_COST if rq["kind"] == "mppi" else cs.CSPLAT_SERVE_LABELS
            t = cs.csplat_server_submit(srv, ids[rq["scene"]], kind, rq["centers"], rq["radii"],
                                        mppi_opts if kind == 0 else rrt_opts, rq["n_sigma"])
            with lock:
                pending[t] = (kind, rq["centers"].shape[0], t_arr, i)
        t_last_submit = time.perf_counter() - t0
        submitted.set()
        th.join()
        wall = time.perf_counter() - t0
        st = cs.csplat_server_stats(srv)
        lat = cs.csplat_server_latencies(srv)
        cs.csplat_server_destroy(srv)
        arr = np.array([arrival_lat[i] for i in range(len(reqs))]) * 1e3
        return st, wall, lat, arr, t_last_submit

    def boot_ci(x, q, n=2000):
        # percentile bootstrap: resample the requests' latencies with replacement
        rng = np.random.default_rng(7)
        v = np.percentile(x[rng.integers(0, x.size, (n, x.size))], q, axis=1)
        return [float(np.percentile(v, 2.5)), float(np.percentile(v, 97.5))]

    log(f"bench: serving: generating {n_requests} requests")
    reqs = serving_stream(n_requests, seed=105, rate_hz=1.0, **kw)   # unit-rate arrival times, scaled below
    sizes = np.array([rq["centers"].shape[0] for rq in reqs])
    pairs = sum(int(sz) * n_scene[rq["scene"]] for sz, rq in zip(sizes, reqs))
    sat, wall, _, _, _ = run(reqs, 0)        # saturated: every request at t = 0
    sat_rate = len(reqs) / wall
    lam = 0.5 * sat_rate
    log(f"bench: serving: saturated {sat_rate:.1f} requests/s; stream at {lam:.1f} requests/s")
    st, wall2, lat, arr, t_sub = run(reqs, lam)
    cs.csplat_scene_free(h4)
    small = sizes < 100_000
    by_class = {}
    for name, sel in (("under_100k_spheres", small), ("100k_to_1M", (sizes >= 100_000) & (sizes < 1_000_000)),
                      ("1M_and_more", sizes >= 1_000_000)):
        if sel.any():
            by_class[name] = {"requests": int(sel.sum()), "p50_ms": float(np.percentile(arr[sel], 50)),
                              "p99_ms": float(np.percentile(arr[sel], 99))}
    return {"workload": ("reduced" if reduced else "config-5") + " serving law: 1M and 4M room scenes resident, "
            f"{n_requests} Poisson requests (MPPI K in {{256..{kw['max_mppi_k']}}} x 32 x 1-{kw['max_spheres']} "
            f"spheres, RRT 1-{kw['max_rrt_points']} points x 1-{kw['max_spheres']} spheres), HBM budget 4 GiB, "
            "16 slots",
            "spheres_total": int(sizes.sum()), "largest_request_spheres": int(sizes.max()),
            "saturated_requests_per_s": sat_rate, "saturated_pair_evals_per_s": pairs / wall,
            "rate_requests_per_s": lam, "achieved_rate_requests_per_s": len(reqs) / max(t_sub, 1e-9),
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "p50_ci95_ms": boot_ci(lat, 50),
            "p99_ci95_ms": boot_ci(lat, 99), "mean_ms": st["mean_ms"], "max_ms": st["max_ms"],
            "from_arrival": {"p50_ms": float(np.percentile(arr, 50)), "p99_ms": float(np.percentile(arr, 99)),
                             "p50_ci95_ms": boot_ci(arr, 50), "p99_ci95_ms": boot_ci(arr, 99)},
            "from_arrival_by_size": by_class,
            "pair_evals_per_s": st["pairs_per_s"], "steps": st["steps"], "completed": st["completed"]}


def cpu_baseline(sc, qs, p, gpu, target_s, n_kept):
    """The FP64 oracle on the host cores over a bounded sample of the same
    queries (full scene); also the label agreement of the GPU on that sample."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import compare

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.build(force=False)
    _, mu, sig = oracle.prepare_scene(sc.means, sc.quats, sc.scales, sc.opacity,
                                      alpha_f=p["alpha_f"], extent_f=p["extent_f"])
    rng = np.random.default_rng(11)
    order = rng.permutation(qs.q)
    kw = dict(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"], s_min=p["s_min"])
    n_s = 64
    while True:
        idx = np.sort(order[:n_s])
        sub = qs.subset(idx)
        t0 = time.perf_counter()
        ref = oracle.evaluate(mu, sig, sub.centers, oracle.sphere_bodies(sub.radii), p["n_sigma"],
                              nthreads=threads, **kw)
        dt = time.perf_counter() - t0
        if dt >= target_s or n_s >= qs.q:
            break
        n_s = min(qs.q, max(n_s * 2, int(n_s * target_s / max(dt, 1e-3) * 1.1)))
        log(f"bench: cpu baseline sample -> {n_s} queries")
    st = compare({k: v[idx] for k, v in gpu.items()}, ref, tau=p["tau"], gamma=p["gamma"], d_max=p["d_max"],
                 where="bench")
    amb = ref["ambiguous"].astype(bool)
    agree = float(((gpu["label"][idx] == ref["label"]) | amb).mean())
    cpu_model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu_model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    base = {"value": n_s * n_kept / dt, "unit": "pair evals/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model,
            "sample": f"{n_s} of {qs.q} queries (seeded) against all {n_kept} kept Gaussians, all outputs, FP64",
            "seconds": dt, "queries_per_s": n_s / dt}
    acc = {"labels_equal_outside_eps_band": agree, "ambiguous_queries": int(amb.sum()),
           "sample_queries": int(n_s), "eps": 1e-5, **st}
    return base, acc


if __name__ == "__main__":
    main()
