"""The minimum of s~^2 over every kept Gaussian (Eq. 8; R_nbr = inf) by the
threshold passes of the task walk, through the C ABI, against the FP64
oracle; culled and dense searches give the same bits."""
import math
import sys

import numpy as np
import pytest

from parity import compare
from workloads import Queries, Scene, config, room_scene, uniform_queries

pytestmark = pytest.mark.gpu


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


def _eval(cs, eng, h, qs, n_sigma, k=2, cull=1, want=("label", "count", "min")):
    import torch
    eng.set_conservatism(n_sigma)
    opts = cs.reduce_opts(k=k, r_nbr=math.inf, cull=cull)
    c = torch.from_numpy(qs.centers).cuda()
    r = torch.from_numpy(qs.radii).cuda()
    out = eng.evaluate(h, c, r, opts, want)
    torch.cuda.synchronize()
    st = eng.stats()
    return {k_: v.cpu().numpy() for k_, v in out.items()}, st


def _oracle(oracle_mod, sc, qs, n_sigma, k=2, p=None):
    p = p or {}
    return oracle_mod.evaluate_spheres(sc, qs, n_sigma, k=k, alpha_f=p.get("alpha_f", 0.0),
                                       extent_f=p.get("extent_f", 0.0))


@pytest.mark.parametrize("name,scale,n_sigma", [("precision", 0.01, [1.0]), ("tiny", 1.0, [0.0, 1.0, 2.5]),
                                                ("mppi_nav", 0.02, [0.0, 1.0, 2.0])])
def test_min_search_matches_oracle(cs, eng, oracle_mod, name, scale, n_sigma):
    _say(f"case: min search {name} x{scale}, n_sigma {n_sigma}")
    sc, qs, p = config(name, scale)
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    gpu, st = _eval(cs, eng, h, qs, n_sigma)
    dense, _ = _eval(cs, eng, h, qs, n_sigma, cull=0)
    cs.csplat_scene_free(h)
    for k_ in gpu:
        assert np.array_equal(gpu[k_], dense[k_]), k_
    ref = _oracle(oracle_mod, sc, qs, n_sigma, p=p)
    s = compare(gpu, ref, tau=0.0, gamma=1.0, where=f"min-{name}")
    _say(f"{name}: passes {st['min_passes']}, evaluated pairs {st['kernel_pairs']} of {st['pairs']}, {s}")
    assert st["min_passes"] >= 1 and st["kernel_pairs"] < st["pairs"]


def test_min_search_far_queries_and_min_only(cs, eng, oracle_mod):
    """Queries far outside the scene: a short unresolved list is finished by
    one dense pass over every Gaussian; min alone (no labels)."""
    _say("case: min search with queries far outside the scene")
    sc = room_scene(30_000, seed=41)
    rng = np.random.default_rng(42)
    c = np.concatenate([rng.uniform(0, 1, (200, 3)) * [10, 10, 3],
                        rng.uniform(-1, 1, (40, 3)) * 60.0 + [5, 5, 1.5],
                        [[5.0, 5.0, 400.0], [-300.0, 2.0, 1.0]]]).astype(np.float32)
    r = rng.uniform(0.03, 0.4, c.shape[0]).astype(np.float32)
    qs = Queries(c, r)
    h = eng.load_scene(sc)
    gpu, st = _eval(cs, eng, h, qs, [1.0], want=("min",))
    dense, _ = _eval(cs, eng, h, qs, [1.0], cull=0, want=("min",))
    cs.csplat_scene_free(h)
    assert np.array_equal(gpu["min"], dense["min"])
    ref = _oracle(oracle_mod, sc, qs, [1.0])
    compare(gpu, ref, tau=0.0, gamma=1.0, where="min-far")
    _say(f"far: passes {st['min_passes']}")
    assert st["min_passes"] >= 2


def test_min_search_threshold_growth(cs, eng, oracle_mod):
    """A long list of queries far from every Gaussian (4,096 of them 20-80 m
    from a 1M-Gaussian room) keeps the culled passes, whose thresholds grow
    fourfold until a pair is in reach: the same bits as a dense search, and
    the oracle's minimum on a sample."""
    _say("case: min search threshold growth, 1M room, 4096 far + 4096 inner queries")
    sc = room_scene(1_000_000, seed=43)
    rng = np.random.default_rng(44)
    u = rng.normal(size=(4096, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    far = np.array([5.0, 5.0, 1.5]) + u * rng.uniform(20.0, 80.0, (4096, 1))
    inner = rng.uniform(0, 1, (4096, 3)) * [10, 10, 3]
    c = np.concatenate([far, inner]).astype(np.float32)
    r = rng.uniform(0.03, 0.4, c.shape[0]).astype(np.float32)
    qs = Queries(c, r)
    h = eng.load_scene(sc)
    gpu, st = _eval(cs, eng, h, qs, [1.0])
    dense, _ = _eval(cs, eng, h, qs, [1.0], cull=0)
    cs.csplat_scene_free(h)
    _say(f"growth: passes {st['min_passes']}")
    assert st["min_passes"] >= 4
    for k_ in gpu:
        assert np.array_equal(gpu[k_], dense[k_]), k_
    idx = np.concatenate([rng.choice(4096, 48, replace=False), 4096 + rng.choice(4096, 48, replace=False)])
    ref = _oracle(oracle_mod, sc, qs.subset(idx), [1.0])
    compare({k_: v[idx] for k_, v in gpu.items()}, ref, tau=0.0, gamma=1.0, where="min-growth")


def test_min_search_degenerate(cs, eng, oracle_mod):
    """Queries on a mean (minimum 0), an empty scene (+inf, counts 0), one query."""
    import torch
    _say("case: min search degenerate inputs")
    sc, qs, p = config("tiny", 0.1)
    on = Queries(sc.means[:5].copy(), np.full(5, 0.1, np.float32))
    qq = Queries(np.concatenate([qs.centers, on.centers]), np.concatenate([qs.radii, on.radii]))
    h = eng.load_scene(sc)
    gpu, _ = _eval(cs, eng, h, qq, [1.0])
    one, _ = _eval(cs, eng, h, qq.subset([3]), [1.0])
    cs.csplat_scene_free(h)
    assert np.all(gpu["min"][-5:] == 0.0)
    assert np.array_equal(one["min"][0], gpu["min"][3])
    compare(gpu, _oracle(oracle_mod, sc, qq, [1.0]), tau=0.0, gamma=1.0, where="min-degenerate")
    empty = Scene(np.zeros((0, 3), np.float32), np.zeros((0, 4), np.float32), np.zeros((0, 3), np.float32),
                  np.zeros(0, np.float32))
    h0 = eng.load_scene(empty)
    res, _ = _eval(cs, eng, h0, qs, [1.0, 2.0])
    cs.csplat_scene_free(h0)
    assert np.all(np.isinf(res["min"])) and np.all(res["count"] == 0) and np.all(res["label"] == 0)
    del torch
