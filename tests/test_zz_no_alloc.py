"""csplat_eval_noalloc (the float32 evaluation without any allocation, its
workspace in the library's fixed per-GPU scratch array) against csplat_eval
on the same inputs, through the C ABI: two calls in a row, the second with a
smaller input, on a context that allocates no workspace of its own.

Counts, labels, minima and ball sizes are integer or exact-min results and
must be equal bit for bit; softmin and cost come from sums in another split
order and are held to the oracle's bars (both entry points), and to each
other within float32 rounding."""
import math
import sys

import numpy as np
import pytest

from parity import compare
from workloads import config, mppi_walk_queries, room_scene, uniform_queries

pytestmark = pytest.mark.gpu

ALL = ("label", "count", "min", "softmin", "cost", "nbr")


@pytest.fixture(scope="module")
def cs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2609_35619_amd as cs
    cs.load_library()
    return cs


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev_outputs(torch, q, m):
    return dict(label=torch.full((q, m), 9, dtype=torch.uint8, device="cuda"),
                count=torch.full((q, m), -1, dtype=torch.int32, device="cuda"),
                min=torch.full((q, m), -1.0, dtype=torch.float32, device="cuda"),
                softmin=torch.full((q, m), -1.0, dtype=torch.float32, device="cuda"),
                cost=torch.full((q, m), -1.0, dtype=torch.float32, device="cuda"),
                nbr=torch.full((q,), -1, dtype=torch.int32, device="cuda"))


def test_noalloc_equals_eval_twice(cs, oracle_mod):
    import torch
    sc = room_scene(120_000, seed=21)
    p = dict(n_sigma=[0.0, 1.0, 2.0], k=2, tau=0.1, r_nbr=1.0, d_max=1.0, gamma=1.0, s_min=1.0,
             alpha_f=0.05, extent_f=0.1)
    calls = [("mppi walks, 8,192 spheres, m=3, ball 1 m", mppi_walk_queries(256, 32, seed=22), p),
             ("uniform, 1,500 spheres, m=1, no ball", uniform_queries(1500, seed=23, box=(10, 10, 3), radius=0.2),
              dict(p, n_sigma=[1.0], r_nbr=math.inf))]
    e_na, e_ev = cs.Engine(0), cs.Engine(0)
    try:
        h = e_ev.load_scene(sc, floater_opacity_max=p["alpha_f"], floater_extent_min=p["extent_f"])
        for i, (what, qs, pp) in enumerate(calls):
            _say(f"case: noalloc call {i + 1}: {what}")
            m = len(pp["n_sigma"])
            opts = cs.reduce_opts(k=pp["k"], tau=pp["tau"], r_nbr=pp["r_nbr"], d_max=pp["d_max"],
                                  gamma=pp["gamma"], s_min=pp["s_min"])
            for e in (e_na, e_ev):
                e.set_conservatism(pp["n_sigma"])
            c = torch.from_numpy(qs.centers).cuda()
            r = torch.from_numpy(qs.radii).cuda()
            o_na, o_ev = _dev_outputs(torch, qs.q, m), _dev_outputs(torch, qs.q, m)
            torch.cuda.synchronize()
            cs.csplat_eval_noalloc(e_na.ctx, h, c, r, opts, **o_na)
            cs.csplat_synchronize(e_na.ctx)
            cs.csplat_eval(e_ev.ctx, h, c, r, opts, **o_ev)
            cs.csplat_synchronize(e_ev.ctx)
            st = cs.csplat_last_stats(e_na.ctx)
            assert st["workspace_bytes"] == 0, "the no-allocation context grew a workspace"
            a = {k: v.cpu().numpy() for k, v in o_na.items()}
            b = {k: v.cpu().numpy() for k, v in o_ev.items()}
            for k in ("label", "count", "min", "nbr"):
                assert np.array_equal(a[k], b[k]), k
            for k in ("softmin", "cost"):
                fin = np.isfinite(b[k])
                assert np.array_equal(fin, np.isfinite(a[k])), k
                assert np.allclose(a[k][fin], b[k][fin], rtol=2e-5, atol=2e-6), k
            ref = oracle_mod.evaluate_spheres(sc, qs, pp["n_sigma"], alpha_f=pp["alpha_f"],
                                              extent_f=pp["extent_f"], k=pp["k"], tau=pp["tau"],
                                              r_nbr=pp["r_nbr"], d_max=pp["d_max"], gamma=pp["gamma"],
                                              s_min=pp["s_min"])
            s1 = compare(a, ref, tau=pp["tau"], gamma=pp["gamma"], d_max=pp["d_max"], where=f"noalloc-{i}")
            compare(b, ref, tau=pp["tau"], gamma=pp["gamma"], d_max=pp["d_max"], where=f"eval-{i}")
            _say(f"noalloc call {i + 1}: splits {st['splits']}, {s1}")
        cs.csplat_scene_free(h)
    finally:
        e_na.close()
        e_ev.close()


def test_noalloc_refusals(cs):
    import torch
    sc, qs, p = config("tiny", 0.05)
    with cs.Engine(0) as e:
        h = e.load_scene(sc)
        e.set_conservatism([1.0])
        opts = cs.reduce_opts(k=0)
        lab = np.zeros((qs.q, 1), np.uint8)
        with pytest.raises(cs.CsplatError):       # host arrays
            cs.csplat_eval_noalloc(e.ctx, h, qs.centers, qs.radii, opts, label=lab)
        big = cs.CSPLAT_NOALLOC_MAX_Q + 1
        c = torch.zeros((big, 3), dtype=torch.float32, device="cuda")
        r = torch.ones((big,), dtype=torch.float32, device="cuda")
        dl = torch.zeros((big, 1), dtype=torch.uint8, device="cuda")
        with pytest.raises(cs.CsplatError):       # above the stated maximum
            cs.csplat_eval_noalloc(e.ctx, h, c, r, opts, label=dl)
        cd = torch.from_numpy(qs.centers).cuda()
        rd = torch.from_numpy(qs.radii).cuda()
        rd[3] = -1.0                               # invalid radius: refused, nothing written
        dl = torch.full((qs.q, 1), 7, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(cs.CsplatError):
            cs.csplat_eval_noalloc(e.ctx, h, cd, rd, opts, label=dl)
        cs.csplat_synchronize(e.ctx)
        assert bool((dl == 7).all())
        with pytest.raises(cs.CsplatError):       # the precision forms allocate their recheck lists
            cs.csplat_eval_noalloc(e.ctx, h, cd, torch.from_numpy(qs.radii).cuda(),
                                   cs.reduce_opts(k=0, precision=cs.CSPLAT_PRECISION_BF16_RECHECK), label=dl)
        cs.csplat_scene_free(h)
