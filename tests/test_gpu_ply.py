"""Scenes loaded from PLY files (3DGS and 2DGS layouts) evaluate like the
same parameters passed to csplat_scene_load, and agree with the oracle run on
the file's raw parameters."""
import math
import sys

import numpy as np
import pytest

from parity import compare
from plyio import write_gaussian_ply
from workloads import Scene, uniform_box_scene, uniform_queries

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


@pytest.mark.parametrize("dims", [3, 2])
def test_ply_scene_matches_arrays_and_oracle(cs, eng, oracle_mod, tmp_path, dims):
    print(f"case: PLY scene with {dims} scales per Gaussian", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(500 + dims)
    base = uniform_box_scene(20_000, seed=501)
    log_s = rng.normal(np.log(0.03), 0.5, (base.n, dims)).astype(np.float32)
    logit = rng.normal(0, 1.5, base.n).astype(np.float32)
    path = str(tmp_path / "scene.ply")
    write_gaussian_ply(path, base.means, base.quats, log_s, logit)
    qs = uniform_queries(2000, seed=502, radius=0.1)
    opts = cs.reduce_opts(k=1, tau=0.1, r_nbr=0.5)
    eng.set_conservatism([0.0, 1.0])
    h_ply = cs.csplat_scene_load_ply(eng.ctx, path, floater_opacity_max=0.05, floater_extent_min=0.1)
    m, q, s, o = cs.csplat_ply_read(path)
    h_arr = eng.load_scene(Scene(m, q, s, o), floater_opacity_max=0.05, floater_extent_min=0.1)
    a = eng.evaluate(h_ply, qs.centers, qs.radii, opts)
    b = eng.evaluate(h_arr, qs.centers, qs.radii, opts)
    assert cs.csplat_scene_info(h_ply) == cs.csplat_scene_info(h_arr)
    cs.csplat_scene_free(h_ply)
    cs.csplat_scene_free(h_arr)
    for k in a:
        assert np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8)), k
    # the oracle on the file's raw values (2DGS: a flat third axis)
    if dims == 3:
        ref = oracle_mod.evaluate_spheres(Scene(base.means, base.quats, log_s, logit), qs, [0.0, 1.0],
                                          raw_mode=True, alpha_f=0.05, extent_f=0.1, k=1, tau=0.1, r_nbr=0.5)
    else:
        ref = oracle_mod.evaluate_spheres(Scene(m, q, s, o), qs, [0.0, 1.0], alpha_f=0.05, extent_f=0.1, k=1,
                                          tau=0.1, r_nbr=0.5)
    print(compare({k: np.asarray(v) for k, v in a.items()}, ref, tau=0.1, gamma=1.0, where=f"ply{dims}"),
          flush=True)
