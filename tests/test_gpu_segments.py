"""Planner epilogues (segment OR of labels, segment sums of costs) through the
C ABI against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

from workloads import config

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


def _sum_tol(cost, offsets):
    """Float32 bound of the kernel's order: each lane sums ceil(n/64) terms in
    sequence, then six butterfly levels merge the lanes:
    |err| <= (ceil(n/64) + 6) 2^-24 sum |x| (first order, plus slack)."""
    tol = np.zeros((offsets.size - 1, cost.shape[1]))
    for s in range(offsets.size - 1):
        a, b = offsets[s], offsets[s + 1]
        n = b - a
        tol[s] = (math.ceil(n / 64) + 7) * 2.0 ** -24 * np.abs(cost[a:b].astype(np.float64)).sum(0)
    return tol


def _random_case(seed, q, m, n_cuts):
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.integers(0, q + 1, n_cuts))
    offsets = np.concatenate([[0], cuts, [q]]).astype(np.int64)
    label = (rng.uniform(size=(q, m)) < 0.01).astype(np.uint8)
    cost = rng.uniform(0, 1, (q, m)).astype(np.float32) * rng.choice([1e-6, 1.0, 1e3], (q, 1)).astype(np.float32)
    return offsets, label, cost


@pytest.mark.parametrize("host", [False, True])
def test_random_segments(cs, eng, oracle_mod, host):
    import torch
    _say(f"case: 20,000 queries x m=3 in 500 random segments (some empty, one long), host={host}")
    offsets, label, cost = _random_case(11, 20_000, 3, 499)
    offsets[250] = offsets[249]                      # an empty segment
    n_seg = offsets.size - 1
    ref_any, ref_sum = oracle_mod.segment_reduce(label, cost, offsets)
    if host:
        seg_any = np.full((n_seg, 3), 9, np.uint8)
        seg_cost = np.full((n_seg, 3), np.nan, np.float32)
        cs.csplat_segment_reduce(eng.ctx, n_seg, label=label, cost=cost, seg_any=seg_any, seg_cost=seg_cost,
                                 offsets=offsets)
    else:
        d = [torch.from_numpy(a).cuda() for a in (label, cost, offsets)]
        a_t = torch.full((n_seg, 3), 9, dtype=torch.uint8, device="cuda")
        c_t = torch.full((n_seg, 3), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        cs.csplat_segment_reduce(eng.ctx, n_seg, label=d[0], cost=d[1], seg_any=a_t, seg_cost=c_t, offsets=d[2])
        eng.synchronize()
        seg_any, seg_cost = a_t.cpu().numpy(), c_t.cpu().numpy()
    assert np.array_equal(seg_any, ref_any)
    err = np.abs(seg_cost.astype(np.float64) - ref_sum)
    assert np.all(err <= _sum_tol(cost, offsets)), f"max err / tol {np.max(err / np.maximum(_sum_tol(cost, offsets), 1e-300))}"


def test_rollout_epilogue_of_a_real_evaluation(cs, eng, oracle_mod):
    """mppi_nav at 5%: per-rollout collision flags and cost sums (32 steps,
    equal segments) of the pair kernel's own outputs."""
    import torch
    _say("case: rollout epilogue of mppi_nav@0.05")
    sc, qs, p = config("mppi_nav", 0.05)
    h = eng.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
    eng.set_conservatism(p["n_sigma"])
    opts = cs.reduce_opts(k=p["k"], tau=p["tau"], r_nbr=p["r_nbr"], d_max=p["d_max"], gamma=p["gamma"])
    out = eng.evaluate(h, torch.from_numpy(qs.centers).cuda(), torch.from_numpy(qs.radii).cuda(), opts,
                       ("label", "cost"))
    n_roll = qs.q // 32
    a_t = torch.empty((n_roll, 3), dtype=torch.uint8, device="cuda")
    c_t = torch.empty((n_roll, 3), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    cs.csplat_segment_reduce(eng.ctx, n_roll, label=out["label"], cost=out["cost"], seg_any=a_t, seg_cost=c_t)
    eng.synchronize()
    lab, cost = out["label"].cpu().numpy(), out["cost"].cpu().numpy()
    ref_any, ref_sum = oracle_mod.segment_reduce(lab, cost, n_seg=n_roll)
    assert np.array_equal(a_t.cpu().numpy(), ref_any)
    offs = np.arange(n_roll + 1, dtype=np.int64) * 32
    assert np.all(np.abs(c_t.cpu().numpy() - ref_sum) <= _sum_tol(cost, offs))
    _say(f"rollouts in collision (n_sigma 0/1/2): {ref_any.sum(0).tolist()} of {n_roll}")
    cs.csplat_scene_free(h)


def test_segment_errors(cs, eng):
    _say("case: segment_reduce invalid arguments")
    lab = np.zeros((10, 1), np.uint8)
    out = np.full((3, 1), 7, np.uint8)
    for offs in ([0, 5, 4, 10], [1, 5, 8, 10], [0, 5, 8, 9]):
        with pytest.raises(cs.CsplatError):
            cs.csplat_segment_reduce(eng.ctx, 3, label=lab, seg_any=out, offsets=np.array(offs, np.int64))
        assert np.all(out == 7)
    with pytest.raises(cs.CsplatError):          # 10 queries in 3 equal segments
        cs.csplat_segment_reduce(eng.ctx, 3, label=lab, seg_any=out)
    with pytest.raises(cs.CsplatError):          # cost output without cost input
        cs.csplat_segment_reduce(eng.ctx, 3, label=lab, seg_cost=np.zeros((3, 1), np.float32),
                                 offsets=np.array([0, 3, 6, 10], np.int64))
