"""The MFMA precision form (bf16/fp16 hi-lo features, certified bound, fp64
recheck) against the FP64 oracle and the float32 path."""
import math
import sys

import numpy as np
import pytest

from parity import compare
from workloads import (Queries, Scene, common_attrs, config, grid_queries, room_scene, uniform_box_scene,
                       uniform_queries)

pytestmark = pytest.mark.gpu

PRECISIONS = ("bf16", "fp16")


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


def _prec(cs, name):
    return cs.CSPLAT_PRECISION_BF16_RECHECK if name == "bf16" else cs.CSPLAT_PRECISION_FP16_RECHECK


def _load(cs, eng, scene, p):
    return eng.load_scene(scene, floater_opacity_max=p.get("alpha_f", 0.0),
                          floater_extent_min=p.get("extent_f", 0.0),
                          precision_features=cs.CSPLAT_FEATURES_BF16 | cs.CSPLAT_FEATURES_FP16)


def _eval(cs, eng, h, queries, p, precision, want=("label", "count"), cull=1):
    import torch
    eng.set_conservatism(p["n_sigma"])
    opts = cs.reduce_opts(k=p.get("k", 0), r_nbr=math.inf, precision=precision, cull=cull)
    c = torch.from_numpy(queries.centers).cuda()
    r = torch.from_numpy(queries.radii).cuda()
    out = eng.evaluate(h, c, r, opts, want)
    torch.cuda.synchronize()
    st = eng.stats()
    return {k: v.cpu().numpy() for k, v in out.items()}, st


def _oracle(oracle_mod, scene, queries, p):
    return oracle_mod.evaluate_spheres(scene, queries, p["n_sigma"], alpha_f=p.get("alpha_f", 0.0),
                                       extent_f=p.get("extent_f", 0.0), k=p.get("k", 0))


@pytest.mark.parametrize("prec", PRECISIONS)
def test_precision_small_scene(cs, eng, oracle_mod, prec):
    _say(f"case: precision {prec}, uniform box 20k x 3000, n_sigma 0/1/2")
    sc = uniform_box_scene(20_000, seed=301, box=(3, 3, 1.5))
    qs = uniform_queries(3000, seed=302, box=(3, 3, 1.5), radius=0.08)
    p = dict(n_sigma=[0.0, 1.0, 2.0], k=2)
    h = _load(cs, eng, sc, p)
    gpu, st = _eval(cs, eng, h, qs, p, _prec(cs, prec))
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, qs, p)
    s = compare(gpu, ref, tau=0.0, gamma=1.0, where=f"precision-{prec}")
    _say(f"{prec}: {s} rechecked={st['flagged']} of {qs.q * 3}")
    # counts were requested: every count must be exact (certified or rechecked in fp64)
    assert np.array_equal(gpu["count"], ref["count"]) or np.all(
        (gpu["count"] == ref["count"]) | ref["ambiguous"].astype(bool))


@pytest.mark.parametrize("prec", PRECISIONS)
def test_precision_labels_only_and_mix_with_fp32(cs, eng, oracle_mod, prec):
    _say(f"case: precision {prec} labels only vs float32 path, room scene")
    sc, qs, p = config("precision", 0.01)
    p = dict(p)
    h = _load(cs, eng, sc, p)
    gpu, st = _eval(cs, eng, h, qs, p, _prec(cs, prec), want=("label",))
    f32, _ = _eval(cs, eng, h, qs, p, cs.CSPLAT_PRECISION_FP32, want=("label", "count"))
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, qs, p)
    compare(gpu, ref, tau=0.0, gamma=1.0, where=f"labels-{prec}")
    amb = ref["ambiguous"].astype(bool)
    assert np.all((gpu["label"] == f32["label"]) | amb)
    _say(f"{prec}: rechecked {st['flagged']} of {qs.q}")


def _isotropic_threshold_scene(n_pairs, s_iso, r, n_sigma, rel, seed):
    """Gaussian i sits at rho*(1 + rel_i) from query i (far from the others)."""
    rng = np.random.default_rng(seed)
    rho = n_sigma * s_iso + math.sqrt(n_sigma ** 2 * s_iso ** 2 + r * r)
    # pairs 0.5 m apart on a compact grid: float32 keeps positions to ~5e-7 m
    i = np.arange(n_pairs)
    centers = np.stack([(i % 12) * 0.5, ((i // 12) % 12) * 0.5, (i // 144) * 0.5], 1)
    u = rng.normal(size=(n_pairs, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    means = centers + u * (rho * (1 + rel))[:, None]
    q, _, _ = common_attrs(rng, n_pairs)
    sc = Scene(means.astype(np.float32), q, np.full((n_pairs, 3), s_iso, np.float32),
               np.full(n_pairs, 0.9, np.float32))
    return sc, Queries(centers.astype(np.float32), np.full(n_pairs, r, np.float32))


@pytest.mark.parametrize("prec", PRECISIONS)
def test_precision_adversarial_near_threshold(cs, eng, oracle_mod, prec):
    _say(f"case: precision {prec}, queries at rho*(1 +- delta)")
    rels = np.concatenate([np.full(200, 1e-3), np.full(200, -1e-3), np.full(200, 1e-5), np.full(200, -1e-5),
                           np.full(200, 3e-7), np.full(200, -3e-7)])
    sc, qs = _isotropic_threshold_scene(rels.size, 0.03, 0.03, 1.0, rels, seed=5)
    p = dict(n_sigma=[1.0], k=0)
    h = _load(cs, eng, sc, p)
    gpu, st = _eval(cs, eng, h, qs, p, _prec(cs, prec))
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, qs, p)
    compare(gpu, ref, tau=0.0, gamma=1.0, where=f"adversarial-{prec}")
    # pairs displaced by 1e-3 of rho* lie clearly on their side of the threshold
    amb = ref["ambiguous"][:, 0].astype(bool)
    clear = np.abs(rels) >= 1e-4
    assert np.all(gpu["label"][clear, 0] == (rels[clear] < 0))
    _say(f"{prec}: rechecked {st['flagged']} of {qs.q}, ambiguous {amb.sum()}")
    assert st["flagged"] >= 200   # the 3e-7 pairs cannot be certified by the MFMA bound


@pytest.mark.parametrize("prec", PRECISIONS)
def test_precision_degenerate_gaussians(cs, eng, oracle_mod, prec):
    _say(f"case: precision {prec}, flat and point Gaussians, small radii")
    rng = np.random.default_rng(9)
    q, s, o = common_attrs(rng, 6000)
    s[:1500, 2] = 0.0
    s[1500:2000] = 0.0
    s[2000:2500] *= 8.0   # very large, anisotropic
    m = rng.uniform(0, 1.5, (6000, 3)).astype(np.float32)
    sc = Scene(m, q, s, o)
    qs = uniform_queries(1500, seed=10, box=(1.5, 1.5, 1.5), radius=0.03)
    qs = Queries(qs.centers, rng.choice(np.array([0.03, 0.05, 0.1], np.float32), qs.q))
    p = dict(n_sigma=[0.5, 2.0], k=1)
    h = _load(cs, eng, sc, p)
    gpu, st = _eval(cs, eng, h, qs, p, _prec(cs, prec))
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, qs, p)
    s_ = compare(gpu, ref, tau=0.0, gamma=1.0, where=f"degenerate-{prec}")
    _say(f"{prec}: {s_} rechecked {st['flagged']}")


@pytest.mark.parametrize("prec", PRECISIONS)
def test_precision_cull_matches_dense(cs, eng, prec):
    """Skipping tiles beyond the reach bound changes no label or count (both
    are certified or rechecked exactly), only the work done."""
    _say(f"case: precision {prec}, tile culling vs dense, room scene")
    sc, qs, p = config("precision", 0.01)
    p = dict(p, n_sigma=[0.0, 1.0, 2.0], k=2)
    h = _load(cs, eng, sc, p)
    dense, st0 = _eval(cs, eng, h, qs, p, _prec(cs, prec), cull=0)
    culled, st1 = _eval(cs, eng, h, qs, p, _prec(cs, prec), cull=1)
    cs.csplat_scene_free(h)
    _say(f"{prec}: rechecked dense {st0['flagged']} culled {st1['flagged']} of {qs.q * 3}")
    for k in dense:
        assert np.array_equal(dense[k], culled[k]), k


def test_group_dealt_walks_match_dense(cs, eng):
    """Over a large scene (more than 1024 culling chunks per split) the label
    walks, float32 tasks and the MFMA form, deal whole 16-chunk groups to
    their splits instead of single chunks or tiles: culled and dense
    evaluations give the same labels and counts."""
    _say("case: group-dealt label walks vs dense, 1M-Gaussian room, 64^3 and 81^3 grid spheres")
    sc = room_scene(1_000_000, seed=311)
    p = dict(n_sigma=[1.0], k=2, alpha_f=0.05, extent_f=0.1)
    h = _load(cs, eng, sc, p)
    n_kept, _ = cs.csplat_scene_info(h)
    n_chunks = (int(n_kept) + 63) // 64
    try:
        for prec, res in ((cs.CSPLAT_PRECISION_FP32, 64), (_prec(cs, "bf16"), 81)):
            qs = grid_queries(res)
            dense, _ = _eval(cs, eng, h, qs, p, prec, cull=0)
            culled, st = _eval(cs, eng, h, qs, p, prec, cull=1)
            _say(f"precision {prec}: {qs.q} queries, {st['splits']} splits of {n_chunks} chunks, "
                 f"{int(dense['label'].sum())} labels set")
            assert n_chunks > 1024 * st["splits"], "the walk under test deals groups only over long splits"
            assert dense["label"].any() and not dense["label"].all()
            for k in dense:
                assert np.array_equal(dense[k], culled[k]), k
    finally:
        cs.csplat_scene_free(h)


def test_precision_invalid_device_inputs(cs, eng):
    """Invalid device queries are refused with CSPLAT_E_INVALID and no output
    written, although the sort and the first MFMA pass are queued before the
    check has returned; the next valid call is unaffected."""
    import torch
    _say("case: precision form, invalid device inputs")
    sc, qs, p = config("tiny", 0.1)
    p = dict(p, n_sigma=[1.0], k=0)
    h = _load(cs, eng, sc, p)
    eng.set_conservatism([1.0])
    opts = cs.reduce_opts(k=0, r_nbr=math.inf, precision=_prec(cs, "bf16"))
    try:
        for bad in ("nan_center", "zero_radius", "neg_radius"):
            c, r = qs.centers.copy(), qs.radii.copy()
            if bad == "nan_center":
                c[5, 2] = np.nan
            elif bad == "zero_radius":
                r[9] = 0
            else:
                r[0] = -1
            ll = torch.full((qs.q, 1), 7, dtype=torch.uint8, device="cuda")
            with pytest.raises(cs.CsplatError) as ei:
                cs.csplat_eval_labels(eng.ctx, h, torch.from_numpy(c).cuda(), torch.from_numpy(r).cuda(), opts, ll)
            assert ei.value.status == cs.CSPLAT_E_INVALID
            assert torch.all(ll == 7).item(), "outputs written on error"
            cs.csplat_eval_labels(eng.ctx, h, torch.from_numpy(qs.centers).cuda(), torch.from_numpy(qs.radii).cuda(),
                                  opts, ll)
            torch.cuda.synchronize()
            assert torch.all(ll <= 1).item()
    finally:
        cs.csplat_scene_free(h)


def test_precision_requires_features(cs, eng):
    sc, qs, p = config("tiny", 0.05)
    h = eng.load_scene(sc)   # no precision features
    eng.set_conservatism([1.0])
    with pytest.raises(cs.CsplatError):
        cs.csplat_eval_labels(eng.ctx, h, qs.centers, qs.radii,
                              cs.reduce_opts(precision=cs.CSPLAT_PRECISION_BF16_RECHECK),
                              np.zeros((qs.q, 1), np.uint8))
    with pytest.raises(cs.CsplatError):   # softmin and cost are float32-path outputs
        h2 = _load(cs, eng, sc, p)
        try:
            cs.csplat_eval_distance(eng.ctx, h2, qs.centers, qs.radii,
                                    cs.reduce_opts(precision=cs.CSPLAT_PRECISION_BF16_RECHECK),
                                    np.zeros((qs.q, 1), np.float32), softmin=np.zeros((qs.q, 1), np.float32))
        finally:
            cs.csplat_scene_free(h2)
    with pytest.raises(cs.CsplatError):   # err is an output of the precision forms
        cs.csplat_eval(eng.ctx, h, qs.centers, qs.radii, cs.reduce_opts(),
                       min=np.zeros((qs.q, 1), np.float32), err=np.zeros((qs.q, 1), np.float32))
    cs.csplat_scene_free(h)


def test_precision_rejects_finite_ball(cs, eng):
    """The MFMA forms count over every kept Gaussian: a finite neighbourhood
    ball is refused (CSPLAT_E_INVALID) before any output is written, for host
    and device pointers alike; the float32 path accepts the same call."""
    import torch
    _say("case: precision forms with a finite neighbourhood ball")
    sc, qs, p = config("tiny", 0.05)
    h = _load(cs, eng, sc, p)
    eng.set_conservatism([1.0])
    for prec in (cs.CSPLAT_PRECISION_BF16_RECHECK, cs.CSPLAT_PRECISION_FP16_RECHECK):
        lab = np.full((qs.q, 1), 7, np.uint8)
        with pytest.raises(cs.CsplatError):
            cs.csplat_eval_labels(eng.ctx, h, qs.centers, qs.radii,
                                  cs.reduce_opts(k=0, r_nbr=0.3, precision=prec), lab)
        assert np.all(lab == 7)
        dlab = torch.full((qs.q, 1), 7, dtype=torch.uint8, device="cuda")
        with pytest.raises(cs.CsplatError):
            cs.csplat_eval_labels(eng.ctx, h, torch.from_numpy(qs.centers).cuda(),
                                  torch.from_numpy(qs.radii).cuda(),
                                  cs.reduce_opts(k=0, r_nbr=0.3, precision=prec), dlab)
        torch.cuda.synchronize()
        assert bool((dlab == 7).all())
    lab = np.zeros((qs.q, 1), np.uint8)
    cs.csplat_eval_labels(eng.ctx, h, qs.centers, qs.radii, cs.reduce_opts(k=0, r_nbr=0.3), lab)
    cs.csplat_scene_free(h)


@pytest.mark.parametrize("variant", ["grid", "stress"])
def test_precision_full_size_against_oracle(cs, eng, oracle_mod, variant):
    """4M Gaussians x 262,144 spheres (the 64^3 grid, or its stress variant with
    half the points near a surface): labels and minima of fp32, bf16 and fp16,
    each against the oracle on 1,024 seeded queries per radius class plus every
    query a precision form rechecked in fp64."""
    from workloads import grid_queries
    _say(f"case: full-size precision workload (4M x 262144), {variant}")
    sc, qs, p = config("precision")
    if variant == "stress":
        qs = grid_queries(64, stress_scene=sc, seed=104)
    h = _load(cs, eng, sc, p)
    res, rechecked = {}, {}
    for name, prec in (("fp32", cs.CSPLAT_PRECISION_FP32), ("bf16", cs.CSPLAT_PRECISION_BF16_RECHECK),
                       ("fp16", cs.CSPLAT_PRECISION_FP16_RECHECK)):
        want = ("label", "min") + (("err",) if name != "fp32" else ())
        res[name], st = _eval(cs, eng, h, qs, p, prec, want=want)
        if name != "fp32":
            rechecked[name] = cs.csplat_last_rechecked(eng.ctx)
        _say(f"{name}: rechecked {st['flagged']} of {qs.q}, min passes {st['min_passes']}")
    cs.csplat_scene_free(h)
    rng = np.random.default_rng(4)
    classes = np.unique(qs.radii)
    idx = [rng.choice(np.nonzero(qs.radii == rc)[0], 1024, replace=False) for rc in classes]
    idx = np.unique(np.concatenate(idx + list(rechecked.values()) + [[qs.q - 1]]))
    _say(f"oracle on {idx.size} queries ({sum(v.size for v in rechecked.values())} rechecked)")
    ref = _oracle(oracle_mod, sc, qs.subset(idx), p)
    compare({"label": res["fp32"]["label"][idx], "min": res["fp32"]["min"][idx]}, ref, tau=0.0, gamma=1.0,
            where=f"full-fp32-{variant}")
    for name in ("bf16", "fp16"):
        compare({"label": res[name]["label"][idx]}, ref, tau=0.0, gamma=1.0, where=f"full-{name}-{variant}")
        e = _min_err_check({k: v[idx] for k, v in res[name].items()}, ref, f"full-min-{name}-{variant}")
        amb = ref["ambiguous"][:, 0].astype(bool)
        flips = int(((res[name]["label"][idx, 0] != ref["label"][:, 0]) & amb).sum())
        _say(f"{name}: label flips inside the eps band {flips}, min error {e}")



def _min_err_check(gpu, ref, where):
    """The certified bar: |min - oracle| <= err on every query; returns the
    error distribution."""
    g, o, e = (np.asarray(gpu["min"], np.float64), ref["min"], np.asarray(gpu["err"], np.float64))
    inf = np.isinf(o)
    assert np.array_equal(np.isinf(g), inf), f"{where}: min infinities differ"
    assert np.all(np.isfinite(e[~inf])) and np.all(e >= 0), f"{where}: err not finite"
    d = np.abs(g[~inf] - o[~inf])
    bad = d > e[~inf]
    assert not bad.any(), f"{where}: {bad.sum()} minima outside their certified bound, e.g. {d[bad][:3]} > {e[~inf][bad][:3]}"
    rel = d / np.maximum(1.0, np.abs(o[~inf]))
    return dict(max_abs=float(d.max(initial=0)), p99_abs=float(np.percentile(d, 99)) if d.size else 0.0,
                max_rel=float(rel.max(initial=0)), max_err=float(e[~inf].max(initial=0)),
                p99_err=float(np.percentile(e[~inf], 99)) if d.size else 0.0)


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("want", [("label", "count", "min", "err"), ("min", "err")])
def test_precision_min_certified(cs, eng, oracle_mod, prec, want):
    _say(f"case: precision {prec} minimum, outputs {want}")
    sc = uniform_box_scene(20_000, seed=331, box=(3, 3, 1.5))
    qs = uniform_queries(3000, seed=332, box=(3, 3, 1.5), radius=0.08)
    qs = Queries(qs.centers, (qs.radii * np.random.default_rng(333).uniform(0.5, 3.0, qs.q)).astype(np.float32))
    p = dict(n_sigma=[0.0, 1.0, 2.0], k=2)
    h = _load(cs, eng, sc, p)
    gpu, st = _eval(cs, eng, h, qs, p, _prec(cs, prec), want=want)
    f32, _ = _eval(cs, eng, h, qs, p, cs.CSPLAT_PRECISION_FP32, want=("min",))
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, qs, p)
    if "label" in want:
        compare({k: gpu[k] for k in ("label", "count")}, ref, tau=0.0, gamma=1.0, where=f"min-labels-{prec}")
    e = _min_err_check(gpu, ref, f"min-{prec}")
    _say(f"{prec}: passes {st['min_passes']}, blocks {st['kernel_pairs'] // 1024}, {e}")
    # the float32 search lies inside the same certified interval (both bracket the exact value)
    fin = np.isfinite(ref["min"])
    assert np.all(np.abs(f32["min"][fin] - gpu["min"][fin]) <= gpu["err"][fin] * 1.001 + 1e-5 * np.maximum(1, ref["tstar"][fin]))


def test_precision_min_fp64_fallback(cs, eng, oracle_mod):
    """fp16 query features overflow for spheres 300 units from the scene: those
    minima come from the fp64 fallback, still within err of the oracle."""
    _say("case: fp16 minimum with queries far from the scene (fp64 fallback)")
    sc = uniform_box_scene(5_000, seed=341, box=(2, 2, 1))
    qs = uniform_queries(500, seed=342, box=(2, 2, 1), radius=0.1)
    far = np.array([[300.0, 1.0, 0.5], [1.0, -350.0, 0.5], [1.0, 1.0, 400.0]], np.float32)
    qq = Queries(np.concatenate([qs.centers, far]), np.concatenate([qs.radii, np.full(3, 0.2, np.float32)]))
    p = dict(n_sigma=[1.0], k=1)
    h = _load(cs, eng, sc, p)
    res = {}
    for prec in PRECISIONS:
        res[prec], st = _eval(cs, eng, h, qq, p, _prec(cs, prec), want=("label", "min", "err"))
        _say(f"{prec}: passes {st['min_passes']}")
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, qq, p)
    for prec in PRECISIONS:
        compare({"label": res[prec]["label"]}, ref, tau=0.0, gamma=1.0, where=f"far-{prec}")
        _say(f"{prec}: {_min_err_check(res[prec], ref, f'far-min-{prec}')}")
