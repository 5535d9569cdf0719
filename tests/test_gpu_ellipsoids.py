"""Ellipsoidal robot bodies (general A_j, Eq. 5-6) on the float32 HIP path,
through the C ABI, against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

from parity import compare
from workloads import Bodies, config, random_ellipsoids, uniform_box_scene

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


def _opts(cs, p, cull=1):
    return cs.reduce_opts(k=p.get("k", 0), tau=p.get("tau", 0.0), r_nbr=p.get("r_nbr", math.inf),
                          d_max=p.get("d_max", 1.0), gamma=p.get("gamma", 1.0), s_min=p.get("s_min", 1.0),
                          cull=cull)


def _run(cs, eng, h, bodies, p, want=ALL, host=False, cull=1):
    import torch
    eng.set_conservatism(p["n_sigma"])
    if host:
        out = eng.evaluate_ellipsoids(h, bodies.centers, bodies.quats, bodies.axes, _opts(cs, p, cull), want)
        return {k: np.array(v) for k, v in out.items()}
    t = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (bodies.centers, bodies.quats, bodies.axes)]
    out = eng.evaluate_ellipsoids(h, *t, _opts(cs, p, cull), want)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _oracle(oracle_mod, scene, bodies, p):
    return oracle_mod.evaluate_ellipsoids(scene, bodies, p["n_sigma"], alpha_f=p.get("alpha_f", 0.0),
                                          extent_f=p.get("extent_f", 0.0), k=p.get("k", 0),
                                          tau=p.get("tau", 0.0), r_nbr=p.get("r_nbr", math.inf),
                                          d_max=p.get("d_max", 1.0), gamma=p.get("gamma", 1.0),
                                          s_min=p.get("s_min", 1.0))


def _load(cs, eng, scene, p):
    return eng.load_scene(scene, floater_opacity_max=p.get("alpha_f", 0.0),
                          floater_extent_min=p.get("extent_f", 0.0))


@pytest.mark.parametrize("r_nbr,want", [(0.5, ALL), (math.inf, ("label", "count")), (0.3, ("label", "count"))])
def test_random_ellipsoids_every_output(cs, eng, oracle_mod, r_nbr, want):
    _say(f"case: 20k Gaussians x 3000 random ellipsoids, r_nbr={r_nbr}, {want}")
    sc = uniform_box_scene(20_000, seed=401, box=(3, 3, 1.5))
    b = random_ellipsoids(3000, seed=402, box=(3, 3, 1.5), axis_range=(0.02, 0.25))
    p = dict(n_sigma=[0.0, 1.0, 2.0], k=2, tau=0.1, r_nbr=r_nbr)
    h = _load(cs, eng, sc, p)
    gpu = _run(cs, eng, h, b, p, want)
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, b, p)
    st = compare(gpu, ref, tau=p["tau"], gamma=1.0, where=f"ellipsoids-{r_nbr}")
    _say(f"{st}")


def test_chain_ellipsoids_scaled(cs, eng, oracle_mod):
    _say("case: manip_ell at scale 0.01 (tabletop 5k x chain links)")
    sc, b, p = config("manip_ell", 0.01)
    h = _load(cs, eng, sc, p)
    gpu = _run(cs, eng, h, b, p)
    cs.csplat_scene_free(h)
    ref = _oracle(oracle_mod, sc, b, p)
    _say(f"{compare(gpu, ref, tau=p['tau'], gamma=p['gamma'], where='manip_ell')}")


def test_sphere_as_ellipsoid_matches_sphere_path(cs, eng, oracle_mod):
    """a = b = c = r with random orientations: the same labels as the sphere
    path (outside the oracle's ambiguity band) and distances within tolerance."""
    import torch
    _say("case: spheres written as ellipsoids")
    sc = uniform_box_scene(10_000, seed=403)
    rng = np.random.default_rng(404)
    q = 2000
    c = rng.uniform(0, 1, (q, 3)).astype(np.float32) * np.array([4, 4, 2], np.float32)
    r = rng.uniform(0.05, 0.2, q).astype(np.float32)
    b = Bodies(c, rng.normal(size=(q, 4)).astype(np.float32), np.repeat(r[:, None], 3, 1))
    p = dict(n_sigma=[0.5, 1.5], k=1, tau=0.05, r_nbr=0.6)
    h = _load(cs, eng, sc, p)
    ell = _run(cs, eng, h, b, p)
    eng.set_conservatism(p["n_sigma"])
    out = eng.evaluate(h, torch.from_numpy(c).cuda(), torch.from_numpy(r).cuda(), _opts(cs, p))
    torch.cuda.synchronize()
    sph = {k: v.cpu().numpy() for k, v in out.items()}
    cs.csplat_scene_free(h)
    from workloads import Queries
    ref = oracle_mod.evaluate_spheres(sc, Queries(c, r), p["n_sigma"], k=1, tau=0.05, r_nbr=0.6)
    compare(ell, ref, tau=0.05, gamma=1.0, where="sphere-as-ellipsoid")
    compare(sph, ref, tau=0.05, gamma=1.0, where="sphere")
    amb = ref["ambiguous"].astype(bool)
    assert np.all((ell["label"] == sph["label"]) | amb)
    assert np.array_equal(ell["nbr"], sph["nbr"])


def test_host_device_and_cull_agree(cs, eng):
    _say("case: ellipsoids host vs device pointers, culled vs dense")
    sc, b, p = config("manip_ell", 0.02)
    h = _load(cs, eng, sc, p)
    dev = _run(cs, eng, h, b, p)
    host = _run(cs, eng, h, b, p, host=True)
    dense = _run(cs, eng, h, b, p, cull=0)
    lab_c = _run(cs, eng, h, b, dict(p, r_nbr=math.inf), want=("label", "count"))
    lab_d = _run(cs, eng, h, b, dict(p, r_nbr=math.inf), want=("label", "count"), cull=0)
    cs.csplat_scene_free(h)
    for k in dev:
        assert np.array_equal(dev[k].view(np.uint8), host[k].view(np.uint8)), k
        assert np.array_equal(dev[k].view(np.uint8), dense[k].view(np.uint8)), k
    for k in lab_c:
        assert np.array_equal(lab_c[k], lab_d[k]), k


def test_invalid_bodies_rejected(cs, eng):
    _say("case: invalid ellipsoid inputs")
    sc = uniform_box_scene(1000, seed=405)
    h = eng.load_scene(sc)
    eng.set_conservatism([1.0])
    b = random_ellipsoids(16, seed=406)
    lab = np.full((16, 1), 7, np.uint8)
    for field, idx, val in (("quats", (3, slice(None)), 0.0), ("axes", (5, 1), -0.1), ("axes", (2, 0), 0.0),
                            ("centers", (1, 2), np.nan), ("quats", (0, 0), np.inf)):
        bad = Bodies(b.centers.copy(), b.quats.copy(), b.axes.copy())
        getattr(bad, field)[idx] = val
        with pytest.raises(cs.CsplatError) as ei:
            cs.csplat_eval_ellipsoids(eng.ctx, h, bad.centers, bad.quats, bad.axes, cs.reduce_opts(), label=lab)
        assert ei.value.status == cs.CSPLAT_E_INVALID
        assert np.all(lab == 7)
    with pytest.raises(cs.CsplatError):
        cs.csplat_eval_ellipsoids(eng.ctx, h, b.centers, b.quats, b.axes,
                                  cs.reduce_opts(precision=cs.CSPLAT_PRECISION_BF16_RECHECK), label=lab)
    cs.csplat_eval_ellipsoids(eng.ctx, h, b.centers[:0], b.quats[:0], b.axes[:0], cs.reduce_opts(),
                              label=lab[:0])
    cs.csplat_scene_free(h)


def test_full_size_sampled(cs, eng, oracle_mod):
    """manip_ell at full size (500k Gaussians x 57,344 links): a seeded sample
    of bodies against the oracle, in the launch configuration the bench times."""
    import torch
    _say("case: manip_ell full size, sampled")
    sc, b, p = config("manip_ell")
    h = _load(cs, eng, sc, p)
    gpu = _run(cs, eng, h, b, p)
    cs.csplat_scene_free(h)
    idx = np.sort(np.random.default_rng(7).choice(b.q, 256, replace=False))
    idx = np.unique(np.concatenate([idx, [0, b.q - 1]]))
    ref = _oracle(oracle_mod, sc, b.subset(idx), p)
    _say(f"{compare({k: v[idx] for k, v in gpu.items()}, ref, tau=p['tau'], gamma=p['gamma'], where='manip_ell-full')}")
    del torch
