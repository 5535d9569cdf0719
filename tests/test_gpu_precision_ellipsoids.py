"""The MFMA precision forms for ellipsoidal bodies (Eq. 5-6 with a general A):
labels and counts through the C ABI against the FP64 oracle and the float32
ellipsoid path; pairs placed at the closed-form threshold along a body's
principal axis; culled and dense walks; the calls the forms refuse."""
import math
import sys

import numpy as np
import pytest

from parity import compare
from workloads import Bodies, Scene, common_attrs, config, random_ellipsoids, room_scene, uniform_box_scene

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
                          precision_features=cs.CSPLAT_FEATURES_ELL_BF16 | cs.CSPLAT_FEATURES_ELL_FP16)


def _eval(cs, eng, h, bodies, p, precision, want=("label", "count"), cull=1):
    import torch
    eng.set_conservatism(p["n_sigma"])
    opts = cs.reduce_opts(k=p.get("k", 0), r_nbr=math.inf, precision=precision, cull=cull)
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (bodies.centers, bodies.quats, bodies.axes)]
    out = eng.evaluate_ellipsoids(h, *t, opts, want)
    torch.cuda.synchronize()
    st = eng.stats()
    return {k: v.cpu().numpy() for k, v in out.items()}, st


def _oracle(oracle_mod, scene, bodies, p):
    return oracle_mod.evaluate_ellipsoids(scene, bodies, p["n_sigma"], alpha_f=p.get("alpha_f", 0.0),
                                          extent_f=p.get("extent_f", 0.0), k=p.get("k", 0))


@pytest.mark.parametrize("prec", PRECISIONS)
def test_random_ellipsoids_against_oracle_and_fp32(cs, eng, oracle_mod, prec):
    _say(f"case: ellipsoids {prec}, uniform box 20k Gaussians x 3000 random bodies, n_sigma 0/1/2")
    sc = uniform_box_scene(20_000, seed=501, box=(3, 3, 1.5))
    b = random_ellipsoids(3000, seed=502, box=(3, 3, 1.5), axis_range=(0.02, 0.25))
    p = dict(n_sigma=[0.0, 1.0, 2.0], k=2)
    h = _load(cs, eng, sc, p)
    gpu, st = _eval(cs, eng, h, b, p, _prec(cs, prec))
    f32, _ = _eval(cs, eng, h, b, p, cs.CSPLAT_PRECISION_FP32)
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, b, p)
    s = compare(gpu, ref, tau=0.0, gamma=1.0, where=f"ell-{prec}")
    amb = ref["ambiguous"].astype(bool)
    assert np.all((gpu["label"] == f32["label"]) | amb)
    assert np.all((gpu["count"] == ref["count"]) | amb)
    _say(f"{prec}: {s}, rechecked {st['flagged']} of {b.q * 3}")


def _axis_threshold_case(n, s_iso, n_sigma, rel, seed):
    """Body i (random orientation and semi-axes) with one isotropic Gaussian
    (scale s) on its principal axis k_i at t*(1 + rel_i), where
    t* = n s + sqrt(n^2 s^2 + a_k^2) solves s~^2 = 1 along that axis (for
    d = t R e_k: s^2 = t^2 / a_k^2 and sigma^2 = 4 s^2 t^2 / a_k^4)."""
    import oracle
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    centers = np.stack([(i % 12) * 0.6, ((i // 12) % 12) * 0.6, (i // 144) * 0.6], 1)
    quats = rng.normal(size=(n, 4))
    axes = rng.uniform(0.03, 0.15, (n, 3))
    k = rng.integers(0, 3, n)
    R = oracle.quat_to_rot(quats)
    a_k = axes[i, k]
    t = n_sigma * s_iso + np.sqrt(n_sigma ** 2 * s_iso ** 2 + a_k ** 2)
    sign = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    means = centers + (R[i, :, k] * (sign * t * (1 + rel))[:, None])
    q, _, _ = common_attrs(rng, n)
    sc = Scene(means.astype(np.float32), q, np.full((n, 3), s_iso, np.float32), np.full(n, 0.9, np.float32))
    return sc, Bodies(centers.astype(np.float32), quats.astype(np.float32), axes.astype(np.float32))


@pytest.mark.parametrize("prec", PRECISIONS)
def test_axis_threshold_pairs(cs, eng, oracle_mod, prec):
    _say(f"case: ellipsoids {prec}, Gaussians at t*(1 +- delta) on a principal axis")
    rels = np.concatenate([np.full(200, 1e-3), np.full(200, -1e-3), np.full(200, 1e-5), np.full(200, -1e-5),
                           np.full(200, 3e-7), np.full(200, -3e-7)])
    sc, b = _axis_threshold_case(rels.size, 0.02, 1.0, rels, seed=7)
    p = dict(n_sigma=[1.0], k=0)
    h = _load(cs, eng, sc, p)
    gpu, st = _eval(cs, eng, h, b, p, _prec(cs, prec))
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, b, p)
    compare(gpu, ref, tau=0.0, gamma=1.0, where=f"ell-axis-{prec}")
    clear = np.abs(rels) >= 1e-4
    assert np.all(ref["label"][clear, 0] == (rels[clear] < 0))   # the closed form, through the oracle
    assert np.all(gpu["label"][clear, 0] == (rels[clear] < 0))
    _say(f"{prec}: rechecked {st['flagged']} of {b.q}, ambiguous {int(ref['ambiguous'].sum())}")
    assert st["flagged"] >= 200   # the 3e-7 pairs are beyond what the MFMA bound certifies


@pytest.mark.parametrize("prec", PRECISIONS)
def test_chain_links_culled_and_dense(cs, eng, oracle_mod, prec):
    _say(f"case: ellipsoids {prec}, manip_ell at scale 0.01, culled and dense")
    sc, b, p = config("manip_ell", 0.01)
    p = dict(p, k=1)
    h = _load(cs, eng, sc, p)
    cul, st = _eval(cs, eng, h, b, p, _prec(cs, prec))
    den, _ = _eval(cs, eng, h, b, p, _prec(cs, prec), cull=0)
    cs.csplat_scene_free(h)
    for k in cul:
        assert np.array_equal(cul[k], den[k]), k
    ref = _oracle(oracle_mod, sc, b, p)
    _say(f"{prec}: {compare(cul, ref, tau=0.0, gamma=1.0, where=f'ell-chain-{prec}')}, rechecked {st['flagged']}")


def test_group_dealt_ellipsoid_walks_match_dense(cs, eng):
    """Over a large scene (more than 1024 culling chunks per split) the
    ellipsoid label walks, float32 tasks and the MFMA form, deal whole
    16-chunk groups to their splits: culled and dense evaluations give the
    same labels and counts."""
    _say("case: group-dealt ellipsoid label walks vs dense, 1M-Gaussian room, 300k random bodies")
    sc = room_scene(1_000_000, seed=511)
    b = random_ellipsoids(300_000, seed=512, box=(10.0, 10.0, 3.0), axis_range=(0.02, 0.2))
    p = dict(n_sigma=[1.0], k=2, alpha_f=0.05, extent_f=0.1)
    h = _load(cs, eng, sc, p)
    n_kept, _ = cs.csplat_scene_info(h)
    n_chunks = (int(n_kept) + 63) // 64
    try:
        for prec in (cs.CSPLAT_PRECISION_FP32, _prec(cs, "bf16")):
            dense, _ = _eval(cs, eng, h, b, p, prec, cull=0)
            culled, st = _eval(cs, eng, h, b, p, prec, cull=1)
            _say(f"precision {prec}: {st['splits']} splits of {n_chunks} chunks, "
                 f"{int(dense['label'].sum())} of {b.q} labels set")
            assert n_chunks > 1024 * st["splits"], "the walk under test deals groups only over long splits"
            assert dense["label"].any() and not dense["label"].all()
            for k in dense:
                assert np.array_equal(dense[k], culled[k]), k
    finally:
        cs.csplat_scene_free(h)


def test_refusals(cs, eng):
    """Distances, a finite ball and a scene without the ellipsoid operands are
    refused before any output is written; labels with the sphere operands only
    are refused too."""
    import torch
    _say("case: ellipsoid precision forms refuse what they do not compute")
    sc = uniform_box_scene(2000, seed=503)
    b = random_ellipsoids(64, seed=504)
    h = _load(cs, eng, sc, {})
    h_sph = eng.load_scene(sc, precision_features=cs.CSPLAT_FEATURES_BF16)
    eng.set_conservatism([1.0])
    lab = np.full((64, 1), 7, np.uint8)
    mn = np.full((64, 1), 7.0, np.float32)
    bf = cs.CSPLAT_PRECISION_BF16_RECHECK
    for hh, kw, opts in ((h, dict(label=lab, min=mn), cs.reduce_opts(precision=bf)),
                         (h, dict(label=lab), cs.reduce_opts(precision=bf, r_nbr=0.5)),
                         (h_sph, dict(label=lab), cs.reduce_opts(precision=bf))):
        with pytest.raises(cs.CsplatError) as ei:
            cs.csplat_eval_ellipsoids(eng.ctx, hh, b.centers, b.quats, b.axes, opts, **kw)
        assert ei.value.status == cs.CSPLAT_E_INVALID
        assert np.all(lab == 7) and np.all(mn == 7.0)
    cs.csplat_eval_ellipsoids(eng.ctx, h, b.centers, b.quats, b.axes, cs.reduce_opts(precision=bf), label=lab)
    assert set(np.unique(lab)) <= {0, 1}
    cs.csplat_scene_free(h)
    cs.csplat_scene_free(h_sph)
    del torch
