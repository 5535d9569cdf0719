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
# Transcendentals (v_sqrt, v_exp) issue at half the FMA rate on gfx950
# (measured: 0.5 against 0.9-1.0 wave instructions per CU per cycle), so each
# counts 2 VALU slots.
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
    ap.add_argument("--serving-requests", type=int, default=500)
    ap.add_argument("--serving-full", action="store_true",
                    help="serve the full-size request law (MPPI K up to 4096 x 32 x 48; long)")
    ap.add_argument("--section", choices=("all", "main", "precision", "serving", "ellipsoids", "manip", "paper", "copy",
                                          "digest"), default="all",
                    help="run one part only (for profiling); 'copy' is a plain 1 GiB device copy "
                         "used to calibrate the HBM traffic counters")
    args = ap.parse_args()
    if args.section == "copy":
        return copy_calibration()
    if args.section == "digest":
        print(kernel_digest())
        return None
    if args.section != "all":
        args.no_precision = args.section not in ("precision",)
        args.no_serving = args.section not in ("serving",)
        args.no_ellipsoids = args.section not in ("ellipsoids",)
        args.no_paper = args.section not in ("paper",)
        args.no_manip = args.section not in ("manip",)
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
    ops = OPS_ALL_PAIRS * evaluated + (OPS_IN_BALL_SHARED + OPS_IN_BALL_PER_NSIGMA * m) * nbr_total
    dense_ops = OPS_ALL_PAIRS * pairs + (OPS_IN_BALL_SHARED + OPS_IN_BALL_PER_NSIGMA * m) * nbr_total
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
                     "ops_per_launch": ops, "in_ball_pairs": nbr_total, "evaluated_pairs": evaluated,
                     "dense_pairs": pairs, "dense_ops_per_launch": dense_ops,
                     "dense_equivalent_frac": dense_ops / kernel_s / PEAK_VALU},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"], res["label_accuracy"] = cpu_baseline(sc, qs, p, gpu, args.cpu_seconds, n_kept)
    if not args.no_precision:
        res["precision_form"] = precision_form(cs, eng)
    if not args.no_manip:
        res["manip"] = manip(cs, eng, args.steps)
    if not args.no_ellipsoids:
        res["ellipsoids"] = ellipsoids(cs, eng, args.steps)
    if not args.no_paper:
        res["paper_context"] = paper_context(cs, eng)
    if not args.no_serving:
        res["serving"] = serving(cs, eng, sc, h, args.serving_requests, args.serving_full)
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
    ops = OPS_ALL_PAIRS * int(st["kernel_pairs"]) + (OPS_IN_BALL_SHARED + OPS_IN_BALL_PER_NSIGMA * m) * nbr
    kernel_s = float(np.mean(kms)) / 1e3
    return {"workload": "manip: 500k-Gaussian tabletop, 256 configurations x 32 steps x 48 chain spheres "
                        "(r 0.03-0.10 m), n_sigma 1, ball 0.3 m, all outputs",
            "n_kept": int(n_kept), "queries": int(qs.q), "ms_per_step": dt * 1e3,
            "pair_evals_per_s": qs.q * n_kept / dt, "queries_per_s": qs.q / dt,
            "roofline": {"bound": "alu", "achieved": ops / kernel_s / 1e9, "peak": PEAK_VALU / 1e9,
                         "unit": "Gop/s", "frac": ops / kernel_s / PEAK_VALU, "kernel_ms": kernel_s * 1e3,
                         "evaluated_pairs": int(st["kernel_pairs"]), "in_ball_pairs": nbr}}


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
    ops = OPS_ALL_PAIRS * int(st["kernel_pairs"]) + (OPS_ELL_SHARED + OPS_IN_BALL_PER_NSIGMA * m) * nbr
    kernel_s = float(np.mean(kms)) / 1e3
    return {"workload": "manip_ell: 500k-Gaussian tabletop, 256 configurations x 32 steps x 7 link ellipsoids "
                        "(semi-axes r, r, L/2 + r), n_sigma 1, ball 0.4 m, all outputs",
            "n_kept": int(n_kept), "bodies": int(b.q), "ms_per_step": dt * 1e3,
            "pair_evals_per_s": b.q * n_kept / dt, "queries_per_s": b.q / dt,
            "roofline": {"bound": "alu", "achieved": ops / kernel_s / 1e9, "peak": PEAK_VALU / 1e9,
                         "unit": "Gop/s", "frac": ops / kernel_s / PEAK_VALU, "kernel_ms": kernel_s * 1e3,
                         "evaluated_pairs": int(st["kernel_pairs"]), "in_ball_pairs": nbr}}


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


def precision_form(cs, eng):
    """Labels of the 4M-Gaussian x 262,144-sphere grid workload: float32 pair
    kernel vs the bf16 / fp16 MFMA forms (certified, rechecked in fp64)."""
    import torch
    from workloads import config
    log("bench: precision form (4M Gaussians x 262,144 grid spheres, labels)")
    sc, qs, p = config("precision")
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"],
                       precision_features=cs.CSPLAT_FEATURES_BF16 | cs.CSPLAT_FEATURES_FP16)
    n_kept, nbytes = cs.csplat_scene_info(h)
    eng.set_conservatism(p["n_sigma"])
    c = torch.from_numpy(qs.centers).cuda()
    r = torch.from_numpy(qs.radii).cuda()
    out = {"workload": "precision: 4M-Gaussian room scene, 64^3 grid spheres in 4 radius classes "
                       "{0.05,0.1,0.2,0.4} m, n_sigma 1, k=2, labels", "n_kept": int(n_kept),
           "queries": int(qs.q), "scene_bytes_with_features": int(nbytes)}
    labels = {}
    for name, prec in (("fp32", cs.CSPLAT_PRECISION_FP32), ("bf16", cs.CSPLAT_PRECISION_BF16_RECHECK),
                       ("fp16", cs.CSPLAT_PRECISION_FP16_RECHECK)):
        opts = cs.reduce_opts(k=p["k"], r_nbr=math.inf, precision=prec)
        dt, res = _time_eval(eng, h, c, r, opts, ("label",))
        cs.csplat_ctx_set_timing(eng.ctx, True)
        eng.evaluate(h, c, r, opts, want=("label",))
        st = cs.csplat_last_stats(eng.ctx)
        cs.csplat_ctx_set_timing(eng.ctx, False)
        labels[name] = res["label"][:, 0]
        flagged = int(st["flagged"])
        per_class = {}
        if prec != cs.CSPLAT_PRECISION_FP32:
            per_class = {"rechecked_fraction": flagged / qs.q}
        if prec == cs.CSPLAT_PRECISION_FP32:
            per_class = {"evaluated_pairs": int(st["kernel_pairs"])}
        out[name] = {"ms": dt * 1e3, "pair_evals_per_s": qs.q * n_kept / dt, "kernel_ms": st["kernel_ms"],
                     "rechecked_queries": flagged, **per_class}
        log(f"bench: precision {name}: {dt*1e3:.1f} ms")
    for name in ("bf16", "fp16"):
        out[name]["label_disagreements_vs_fp32"] = int((labels[name] != labels["fp32"]).sum())
        out[name]["speedup_vs_fp32"] = out["fp32"]["ms"] / out[name]["ms"]
    # the certified-bound flag rate per radius class (one extra launch per dtype
    # with counts off: the decide step lists the undecided queries)
    radii = np.unique(qs.radii)
    for name, prec in (("bf16", cs.CSPLAT_PRECISION_BF16_RECHECK), ("fp16", cs.CSPLAT_PRECISION_FP16_RECHECK)):
        cls = {}
        for rv in radii:
            sel = np.nonzero(qs.radii == rv)[0]
            cc, rr = c[torch.from_numpy(sel).cuda()], r[torch.from_numpy(sel).cuda()]
            eng.evaluate(h, cc.contiguous(), rr.contiguous(), cs.reduce_opts(k=p["k"], r_nbr=math.inf, precision=prec),
                         want=("label",))
            torch.cuda.synchronize()
            cls[f"r={rv:.2f}"] = cs.csplat_last_stats(eng.ctx)["flagged"] / sel.size
        out[name]["rechecked_fraction_per_radius_class"] = cls
    cs.csplat_scene_free(h)
    return out


def serving(cs, eng, sc_nav, h_nav, n_requests, full):
    """The serving form with the 1M (navigation) and 4M (room) scenes resident:
    a Poisson stream mixing MPPI batches and RRT edge checks.  The saturated
    request rate is measured first (all requests at once); the stream then
    arrives at half that rate and p50/p99 latency is reported."""
    from workloads import config, serving_stream
    log("bench: serving (1M + 4M resident scenes)")
    sc4, _, p4 = config("precision")
    h4 = eng.load_scene(sc4, floater_opacity_max=p4["alpha_f"], floater_extent_min=p4["extent_f"])
    kw = dict(max_mppi_k=4096, max_rrt_points=10000, max_spheres=48) if full else \
        dict(max_mppi_k=512, max_rrt_points=4000, max_spheres=8)
    mppi_opts = cs.reduce_opts(k=2, tau=0.1, r_nbr=1.0, d_max=1.0, gamma=1.0, s_min=1.0)
    rrt_opts = cs.reduce_opts(k=2, r_nbr=math.inf)
    n_scene = [cs.csplat_scene_info(h_nav)[0], cs.csplat_scene_info(h4)[0]]

    def run(reqs, rate_scale):
        # one thread submits at the arrival times, another collects finished
        # requests as they complete (a finished request holds its output
        # staging until it is collected)
        import threading
        srv = cs.csplat_server_create(0, 4 << 30, 16)
        ids = [cs.csplat_server_add_scene(srv, h_nav), cs.csplat_server_add_scene(srv, h4)]
        pending, lock, submitted = {}, threading.Lock(), threading.Event()
        n_done = [0]

        def collect():
            last = time.perf_counter()
            while True:
                with lock:
                    items = list(pending.items())
                if not items and submitted.is_set():
                    return
                for t, (kind, q) in items:
                    if cs.csplat_server_poll(srv, t, q, kind) is not None:
                        with lock:
                            del pending[t]
                        n_done[0] += 1
                if time.perf_counter() - last > 10.0:
                    last = time.perf_counter()
                    log(f"bench: serving: {n_done[0]} of {len(reqs)} requests collected")
                time.sleep(0.002)

        th = threading.Thread(target=collect)
        t0 = time.perf_counter()
        th.start()
        for rq in reqs:
            while rate_scale and time.perf_counter() - t0 < rq["t"] * rate_scale:
                time.sleep(0.0002)
            kind = cs.CSPLAT_SERVE_COST if rq["kind"] == "mppi" else cs.CSPLAT_SERVE_LABELS
            t = cs.csplat_server_submit(srv, ids[rq["scene"]], kind, rq["centers"], rq["radii"],
                                        mppi_opts if kind == 0 else rrt_opts, rq["n_sigma"])
            with lock:
                pending[t] = (kind, rq["centers"].shape[0])
        submitted.set()
        th.join()
        wall = time.perf_counter() - t0
        st = cs.csplat_server_stats(srv)
        lat = cs.csplat_server_latencies(srv)
        cs.csplat_server_destroy(srv)
        return st, wall, lat

    def boot_ci(x, q, n=2000):
        # percentile bootstrap: resample the requests' latencies with replacement
        rng = np.random.default_rng(7)
        v = np.percentile(x[rng.integers(0, x.size, (n, x.size))], q, axis=1)
        return [float(np.percentile(v, 2.5)), float(np.percentile(v, 97.5))]

    log(f"bench: serving: generating {n_requests} requests")
    reqs = serving_stream(n_requests, seed=105, rate_hz=1.0, **kw)
    pairs = sum(rq["centers"].shape[0] * n_scene[rq["scene"]] for rq in reqs)
    sat, wall, _ = run(reqs, 0)        # saturated: every request at t = 0
    sat_rate = len(reqs) / wall
    lam = 0.5 * sat_rate
    reqs2 = serving_stream(n_requests, seed=105, rate_hz=lam, **kw)
    st, wall2, lat = run(reqs2, 1.0)
    cs.csplat_scene_free(h4)
    return {"workload": ("full" if full else "reduced") + " serving law: 1M and 4M room scenes resident, "
            f"{n_requests} requests (MPPI K<={kw['max_mppi_k']} x 32 x <= {kw['max_spheres']} spheres, "
            f"RRT <= {kw['max_rrt_points']} points x <= {kw['max_spheres']} spheres), HBM budget 4 GiB, 16 slots",
            "saturated_requests_per_s": sat_rate, "saturated_pair_evals_per_s": pairs / wall,
            "rate_requests_per_s": lam, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "p50_ci95_ms": boot_ci(lat, 50), "p99_ci95_ms": boot_ci(lat, 99), "mean_ms": st["mean_ms"],
            "max_ms": st["max_ms"], "pair_evals_per_s": st["pairs_per_s"], "steps": st["steps"],
            "completed": st["completed"]}


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
