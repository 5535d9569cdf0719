"""Parity of the float32 HIP path (through the C ABI) with the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

from parity import compare
from workloads import Queries, Scene, common_attrs, config, uniform_box_scene, uniform_queries

pytestmark = pytest.mark.gpu

ALL = ("label", "count", "min", "softmin", "cost", "nbr")


@pytest.fixture(scope="module")
def cs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2609_35619_amd as cs
    cs.load_library()
    return cs


@pytest.fixture(scope="module")
def eng(cs):
    e = cs.Engine(0)
    yield e
    e.close()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(cs, eng, scene, queries, p, want=ALL, scene_handle=None, host=False, raw=False):
    import torch
    sc = scene_handle
    if sc is None:
        sc = eng.load_scene(scene, floater_opacity_max=p.get("alpha_f", 0.0),
                            floater_extent_min=p.get("extent_f", 0.0),
                            param_mode=cs.CSPLAT_PARAM_RAW_3DGS if raw else cs.CSPLAT_PARAM_ACTIVATED)
    eng.set_conservatism(p["n_sigma"])
    opts = cs.reduce_opts(k=p.get("k", 0), tau=p.get("tau", 0.0), r_nbr=p.get("r_nbr", math.inf),
                          d_max=p.get("d_max", 1.0), gamma=p.get("gamma", 1.0), s_min=p.get("s_min", 1.0))
    if host:
        out = eng.evaluate(sc, queries.centers, queries.radii, opts, want)
        res = {k: np.array(v) for k, v in out.items()}
    else:
        c = torch.from_numpy(queries.centers).cuda()
        r = torch.from_numpy(queries.radii).cuda()
        out = eng.evaluate(sc, c, r, opts, want)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items()}
    if scene_handle is None:
        cs.csplat_scene_free(sc)
    return res


def _oracle(oracle_mod, scene, queries, p, raw=False):
    return oracle_mod.evaluate_spheres(scene, queries, p["n_sigma"], raw_mode=raw,
                                       alpha_f=p.get("alpha_f", 0.0), extent_f=p.get("extent_f", 0.0),
                                       k=p.get("k", 0), tau=p.get("tau", 0.0),
                                       r_nbr=p.get("r_nbr", math.inf), d_max=p.get("d_max", 1.0),
                                       gamma=p.get("gamma", 1.0), s_min=p.get("s_min", 1.0))


def _check(gpu, ref, p, where):
    st = compare(gpu, ref, tau=p.get("tau", 0.0), gamma=p.get("gamma", 1.0), d_max=p.get("d_max", 1.0),
                 where=where)
    _say(f"{where}: {st}")
    return st


# --- the small configuration, every query, every output ----------------------

def test_tiny_every_output(cs, eng, oracle_mod):
    _say("case: tiny config, 10k Gaussians x 4096 queries, all outputs")
    sc, qs, p = config("tiny")
    gpu = _run(cs, eng, sc, qs, p)
    ref = _oracle(oracle_mod, sc, qs, p)
    _check(gpu, ref, p, "tiny")


@pytest.mark.parametrize("name,scale", [("mppi_nav", 0.02), ("manip", 0.004), ("precision", 0.002),
                                        ("paper_p0", 0.05)])
def test_scaled_configs(cs, eng, oracle_mod, name, scale):
    _say(f"case: {name} at scale {scale}")
    sc, qs, p = config(name, scale)
    gpu = _run(cs, eng, sc, qs, p)
    ref = _oracle(oracle_mod, sc, qs, p)
    _check(gpu, ref, p, f"{name}@{scale}")


@pytest.mark.parametrize("r_nbr", [math.inf, 0.4])
def test_labels_only_path(cs, eng, oracle_mod, r_nbr):
    _say(f"case: labels-only kernel, r_nbr={r_nbr}")
    sc = uniform_box_scene(3000, seed=201, box=(2, 2, 1))
    qs = uniform_queries(777, seed=202, box=(2, 2, 1), radius=0.12)
    p = dict(n_sigma=[0.0, 0.5, 1.0, 3.0], k=1, r_nbr=r_nbr)
    gpu = _run(cs, eng, sc, qs, p, want=("label", "count"))
    ref = _oracle(oracle_mod, sc, qs, p)
    _check(gpu, ref, p, "labels-only")


def test_host_and_device_pointers_agree(cs, eng):
    _say("case: host vs device pointers")
    sc, qs, p = config("mppi_nav", 0.01)
    a = _run(cs, eng, sc, qs, p)
    b = _run(cs, eng, sc, qs, p, host=True)
    for k in ALL:
        assert np.array_equal(a[k], b[k]), k


def test_bit_reproducible(cs, eng):
    _say("case: repeat runs are bit-identical")
    sc, qs, p = config("tiny", 0.5)
    a = _run(cs, eng, sc, qs, p)
    b = _run(cs, eng, sc, qs, p)
    for k in ALL:
        assert np.array_equal(a[k], b[k]), k


# --- edge cases ---------------------------------------------------------------

def _scene(means, quats, scales, opacity=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    if opacity is None:
        opacity = np.full(n, 0.9, np.float32)
    return Scene(means, np.asarray(quats, np.float32).reshape(n, 4),
                 np.asarray(scales, np.float32).reshape(n, 3), np.asarray(opacity, np.float32))


def test_empty_scene_and_filtered_scene(cs, eng, oracle_mod):
    _say("case: empty scene, fully filtered scene")
    qs = uniform_queries(300, seed=5)
    p = dict(n_sigma=[1.0], tau=0.1, k=0)
    empty = _scene(np.zeros((0, 3)), np.zeros((0, 4)), np.zeros((0, 3)), np.zeros(0))
    gpu = _run(cs, eng, empty, qs, p)
    assert np.all(gpu["count"] == 0) and np.all(gpu["label"] == 0) and np.all(gpu["nbr"] == 0)
    assert np.all(np.isinf(gpu["min"])) and np.all(np.isinf(gpu["softmin"])) and np.all(gpu["cost"] == 0)
    floaters = _scene(np.random.default_rng(0).uniform(0, 4, (50, 3)), np.tile([1, 0, 0, 0], (50, 1)),
                      np.full((50, 3), 0.5), np.full(50, 0.01))
    p2 = dict(p, alpha_f=0.05, extent_f=0.1)
    gpu = _run(cs, eng, floaters, qs, p2)
    ref = _oracle(oracle_mod, floaters, qs, p2)
    assert np.all(ref["nbr"] == 0)
    _check(gpu, ref, p2, "filtered")


def test_single_query_and_degenerate_pairs(cs, eng, oracle_mod):
    _say("case: one query; a query on a Gaussian mean; zero-scale axes; far queries")
    rng = np.random.default_rng(3)
    q, s, o = common_attrs(rng, 500)
    s[:100, 0] = 0.0          # flat (2DGS-like) Gaussians
    s[100:150] = 0.0          # point Gaussians
    m = rng.uniform(0, 1, (500, 3)).astype(np.float32)
    sc = Scene(m, q, s, o)
    centers = np.concatenate([m[:3], m[100:103], rng.uniform(0, 1, (5, 3)), [[50.0, 50.0, 50.0]]]).astype(np.float32)
    qs = Queries(centers, np.full(centers.shape[0], 0.07, np.float32))
    p = dict(n_sigma=[0.0, 1.0, 2.5], tau=0.05, k=0, gamma=2.0, d_max=3.0)
    gpu = _run(cs, eng, sc, qs, p)
    ref = _oracle(oracle_mod, sc, qs, p)
    _check(gpu, ref, p, "degenerate")
    one = qs.subset([4])
    gpu1 = _run(cs, eng, sc, one, p)
    _check(gpu1, _oracle(oracle_mod, sc, one, p), p, "single")


@pytest.mark.parametrize("variant", ["m8", "tau0", "gamma0", "tiny_ball", "raw", "big_tau"])
def test_parameter_variants(cs, eng, oracle_mod, variant):
    _say(f"case: variant {variant}")
    sc, qs, p = config("tiny", 0.1)
    p = dict(p)
    raw = False
    if variant == "m8":
        p["n_sigma"] = [0.0, 0.25, 0.5, 0.75, 1.0, 1.5, 2.0, 4.0]
    elif variant == "tau0":
        p["tau"] = 0.0
    elif variant == "gamma0":
        p["gamma"] = 0.0
    elif variant == "tiny_ball":
        p["r_nbr"] = 0.05
    elif variant == "big_tau":
        p["tau"] = 7.5
    elif variant == "raw":
        raw = True
        sc = Scene(sc.means, sc.quats, np.log(sc.scales.astype(np.float64)).astype(np.float32),
                   np.log(sc.opacity.astype(np.float64) / (1 - sc.opacity.astype(np.float64))).astype(np.float32))
    gpu = _run(cs, eng, sc, qs, p, raw=raw)
    ref = _oracle(oracle_mod, sc, qs, p, raw=raw)
    _check(gpu, ref, p, variant)


@pytest.mark.parametrize("n_sigma", [[0.0, 1.0, 3.0], [1.0]])
def test_task_walk_queue_edges(cs, eng, oracle_mod, n_sigma):
    """Full outputs over a ball run as (query, sub-chunk) tasks queued per
    wave (with one n_sigma value two queries share a queue entry): a cluster
    inside every query's ball queues up to 64 tasks per sub-chunk (the ring
    wraps many times; odd counts leave an entry's second slot empty),
    n = 1037 leaves a last sub-chunk of 13 Gaussians plus padding, q = 197 a
    partial last wave, and far queries have no task at all.  Parity with the
    oracle on every output and the same bits with culling off."""
    import torch
    _say(f"case: task walk, clustered 1037 Gaussians x 197 queries, ball 0.5, n_sigma {n_sigma}")
    rng = np.random.default_rng(11)
    q, s, o = common_attrs(rng, 1037)
    m = (0.5 + 0.1 * rng.standard_normal((1037, 3))).astype(np.float32)
    sc = Scene(m, q, s * 0.3, o)
    near = (0.5 + 0.15 * rng.standard_normal((190, 3))).astype(np.float32)
    near[:4] = near[0]                                    # coincident queries
    far = np.array([[5.0, 5.0, 5.0], [-4.0, 0.5, 0.5], [0.5, 9.0, 0.5]], np.float32)
    centers = np.concatenate([near[:100], far, near[100:], far[:1], m[:3]]).astype(np.float32)
    assert centers.shape[0] == 197
    qs = Queries(centers, rng.uniform(0.02, 0.08, 197).astype(np.float32))
    p = dict(n_sigma=n_sigma, tau=0.05, k=1, r_nbr=0.5, gamma=1.5, d_max=2.0)
    gpu = _run(cs, eng, sc, qs, p)
    _check(gpu, _oracle(oracle_mod, sc, qs, p), p, "task-walk")
    h = eng.load_scene(sc)
    eng.set_conservatism(p["n_sigma"])
    c = torch.from_numpy(qs.centers).cuda()
    r = torch.from_numpy(qs.radii).cuda()
    res = {}
    for cull in (0, 1):
        opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"],
                              s_min=1.0, cull=cull)
        out = eng.evaluate(h, c, r, opts, ALL)
        torch.cuda.synchronize()
        res[cull] = {k: v.cpu().numpy() for k, v in out.items()}
    cs.csplat_scene_free(h)
    for k in ALL:
        assert np.array_equal(res[0][k].view(np.uint8), res[1][k].view(np.uint8)), k
    assert np.all(res[1]["nbr"][[100, 101, 102, 193]] == 0)  # far queries: empty ball


def test_query_order_and_crowded_cells(cs, eng, oracle_mod):
    """Queries are evaluated in the scene's curve order and scattered back:
    2,000 queries at one point (equal keys), queries outside the scene's box
    (clamped to its edge cells), 1,200 far beyond its eight corners (clamped
    to the corner cells, one of which holds the curve's largest key; equal
    keys spread over the sort's runs) and uniform ones.  Parity with the
    oracle, the same bits for the queries given in a shuffled order (a
    query's results do not depend on which queries share its wave), and the
    same bits on a repeat."""
    _say("case: crowded cell, out-of-box, corner and shuffled queries")
    sc, qs0, p = config("tiny", 0.5)
    rng = np.random.default_rng(5)
    same = np.tile(np.array([[1.0, 2.0, 1.0]], np.float32), (2000, 1))
    out_box = rng.uniform(-3.0, 7.0, (300, 3)).astype(np.float32)
    signs = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float32)
    corners = np.repeat(signs * 50.0 + 2.0, 150, axis=0)
    corners = corners[rng.permutation(corners.shape[0])]
    centers = np.concatenate([same[:1000], corners[:600], out_box, same[1000:], qs0.centers[:700],
                              corners[600:]]).astype(np.float32)
    radii = rng.uniform(0.05, 0.3, centers.shape[0]).astype(np.float32)
    qs = Queries(centers, radii)
    p = dict(p, k=1, tau=0.1, r_nbr=0.6)
    a = _run(cs, eng, sc, qs, p)
    sub = np.arange(0, qs.q, 7)
    _check({k: v[sub] for k, v in a.items()}, _oracle(oracle_mod, sc, qs.subset(sub), p), p, "crowded")
    perm = rng.permutation(qs.q)
    b = _run(cs, eng, sc, qs.subset(perm), p)
    c = _run(cs, eng, sc, qs, p)
    for k in ALL:
        assert np.array_equal(a[k][perm].view(np.uint8), b[k].view(np.uint8)), k
        assert np.array_equal(a[k].view(np.uint8), c[k].view(np.uint8)), k


def test_invalid_inputs_are_rejected_without_writing(cs, eng):
    import torch
    _say("case: invalid inputs")
    sc, qs, p = config("tiny", 0.05)
    h = eng.load_scene(sc)
    eng.set_conservatism([1.0])
    opts = cs.reduce_opts(k=0)
    for bad in ("nan_center", "zero_radius", "neg_radius"):
        c = qs.centers.copy()
        r = qs.radii.copy()
        if bad == "nan_center":
            c[3, 1] = np.nan
        elif bad == "zero_radius":
            r[7] = 0
        else:
            r[0] = -1
        for dev in (False, True):
            lab = np.full((qs.q, 1), 7, np.uint8)
            if dev:
                cc, rr, ll = torch.from_numpy(c).cuda(), torch.from_numpy(r).cuda(), torch.from_numpy(lab).cuda()
            else:
                cc, rr, ll = c, r, lab
            with pytest.raises(cs.CsplatError) as ei:
                cs.csplat_eval_labels(eng.ctx, h, cc, rr, opts, ll)
            assert ei.value.status == cs.CSPLAT_E_INVALID
            got = ll.cpu().numpy() if dev else ll
            assert np.all(got == 7), "outputs written on error"
            if dev:
                # the device-side flag is cleared for the next evaluation
                good = torch.from_numpy(qs.centers).cuda(), torch.from_numpy(qs.radii).cuda()
                cs.csplat_eval_labels(eng.ctx, h, *good, opts, ll)
                torch.cuda.synchronize()
                assert np.all(ll.cpu().numpy() <= 1)
    for ns in ([-1.0], [float("nan")], [1.0] * 9):
        with pytest.raises(cs.CsplatError):
            cs.csplat_set_conservatism(eng.ctx, ns)
    with pytest.raises(cs.CsplatError):
        cs.csplat_eval_labels(eng.ctx, h, qs.centers, qs.radii, cs.reduce_opts(k=-1), np.zeros((qs.q, 1), np.uint8))
    with pytest.raises(cs.CsplatError):
        cs.csplat_eval_labels(eng.ctx, h, qs.centers, qs.radii, cs.reduce_opts(r_nbr=0.0), np.zeros((qs.q, 1), np.uint8))
    bad_q = sc.quats.copy()
    bad_q[5] = 0
    with pytest.raises(cs.CsplatError) as ei:
        cs.csplat_scene_load(eng.ctx, sc.means, bad_q, sc.scales, sc.opacity)
    assert ei.value.status == cs.CSPLAT_E_INVALID
    neg = sc.scales.copy()
    neg[2, 1] = -0.1
    with pytest.raises(cs.CsplatError):
        cs.csplat_scene_load(eng.ctx, sc.means, sc.quats, neg, sc.opacity)
    # q = 0 is a no-op
    cs.csplat_eval_labels(eng.ctx, h, np.zeros((0, 3), np.float32), np.zeros(0, np.float32), opts,
                          np.zeros((0, 1), np.uint8))
    cs.csplat_scene_free(h)


# --- full-size workloads in the launch configuration the benchmark times -------

@pytest.mark.parametrize("name,sample", [("mppi_nav", 1024), ("manip", 1024), ("precision", 96)])
def test_full_size_sampled(cs, eng, oracle_mod, name, sample):
    import torch
    _say(f"case: full-size {name}, oracle on {sample} sampled queries")
    sc, qs, p = config(name)
    want = ALL if name != "precision" else ("label", "count", "min")
    gpu = _run(cs, eng, sc, qs, p, want=want)
    idx = np.sort(np.random.default_rng(7).choice(qs.q, sample, replace=False))
    # the last query is always checked (ragged tail of the final tile)
    idx = np.unique(np.concatenate([idx, [qs.q - 1]]))
    ref = _oracle(oracle_mod, sc, qs.subset(idx), p)
    _check({k: v[idx] for k, v in gpu.items()}, ref, p, f"{name} full")
    # properties that hold for every query at any size
    if "count" in gpu:
        assert np.array_equal(gpu["label"], (gpu["count"] > p["k"]).astype(np.uint8))
        if gpu["count"].shape[1] > 1:
            assert np.all(np.diff(gpu["count"], axis=1) >= 0)   # monotone in n_sigma
    if "min" in gpu and gpu["min"].shape[1] > 1:
        assert np.all(np.diff(gpu["min"], axis=1) <= 0)
    del torch


# --- exact culling: the same bits as the dense evaluation ----------------------

@pytest.mark.parametrize("name,scale,want", [("mppi_nav", 0.05, ALL), ("manip", 0.02, ALL),
                                             ("tiny", 1.0, ("label", "count")),
                                             ("precision", 0.01, ("label", "count")),
                                             ("mppi_nav", 0.05, ("label", "count"))])
def test_cull_is_bit_identical_to_dense(cs, eng, name, scale, want):
    import torch
    _say(f"case: cull vs dense, {name}@{scale} {want}")
    sc, qs, p = config(name, scale)
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    eng.set_conservatism(p["n_sigma"])
    c = torch.from_numpy(qs.centers).cuda()
    r = torch.from_numpy(qs.radii).cuda()
    res = {}
    for cull in (0, 1):
        opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"],
                              s_min=p["s_min"], cull=cull)
        out = eng.evaluate(h, c, r, opts, want)
        torch.cuda.synchronize()
        res[cull] = {k: v.cpu().numpy() for k, v in out.items()}
        st = eng.stats()
        _say(f"cull={cull}: kernel pairs {st['kernel_pairs']} of {qs.q * sc.n}")
        if cull and (want != ALL or math.isfinite(p["r_nbr"])):
            assert st["kernel_pairs"] < qs.q * sc.n
    cs.csplat_scene_free(h)
    for k in want:
        assert np.array_equal(res[0][k].view(np.uint8), res[1][k].view(np.uint8)), k


def test_scene_free_behind_queued_work(cs, eng):
    """Freeing a scene right after queuing evaluations on it (no wait in
    between) releases its memory only after they have run, and the context's
    workspace, grown between the calls, is replaced in stream order: the
    queued results equal those of the same calls on a scene that is kept."""
    import torch
    _say("case: scene freed behind queued work, growing workspace")
    sc, qs, p = config("tiny")
    kw = dict(floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    eng.set_conservatism(p["n_sigma"])
    opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"],
                          s_min=p["s_min"])
    c = torch.from_numpy(qs.centers).cuda()
    r = torch.from_numpy(qs.radii).cuda()
    sizes = (qs.q // 8, qs.q // 2, qs.q)
    kept = eng.load_scene(sc, **kw)
    ref = []
    for n in sizes:
        o = eng.evaluate(kept, c[:n], r[:n], opts, ALL)
        torch.cuda.synchronize()
        ref.append({k: v.cpu().numpy() for k, v in o.items()})
    cs.csplat_scene_free(kept)
    # a fresh context: its workspace grows with each call
    e2 = cs.Engine(0)
    try:
        e2.set_conservatism(p["n_sigma"])
        h = e2.load_scene(sc, **kw)
        outs = [e2.evaluate(h, c[:n], r[:n], opts, ALL) for n in sizes]
        cs.csplat_scene_free(h)
        # new allocations right away may take the freed blocks, in stream order
        filler = e2.load_scene(uniform_box_scene(20_000, seed=9))
        junk = e2.evaluate(filler, c, r, opts, ALL)
        torch.cuda.synchronize()
        for n, o, rf in zip(sizes, outs, ref):
            for k in ALL:
                assert np.array_equal(o[k].cpu().numpy(), rf[k], equal_nan=True), (n, k)
        assert junk["label"].shape[0] == qs.q
        cs.csplat_scene_free(filler)
    finally:
        e2.close()
