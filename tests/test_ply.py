"""The PLY scene reader on the CPU (no GPU needed): the 3DGS and 2DGS
layouts, property types, skipped elements and properties, and errors."""
import os

import numpy as np
import pytest

from plyio import write_gaussian_ply
from workloads import uniform_box_scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_35619_amd", "libcsplat.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcsplat.so not built")


@pytest.fixture(scope="module")
def cs():
    import paper_2609_35619_amd as cs
    cs.load_library()
    return cs


def _raw(n, seed, dims=3):
    rng = np.random.default_rng(seed)
    sc = uniform_box_scene(n, seed=seed)
    log_s = rng.normal(np.log(0.03), 0.5, (n, dims))
    logit = rng.normal(0, 1.5, n)
    return sc.means.astype(np.float64), sc.quats.astype(np.float64), log_s, logit


def _expect(means, quats, log_s, logit, dtype):
    cast = np.float32 if dtype == "float" else np.float64
    m, q, ls, lo = (np.asarray(a).astype(cast).astype(np.float64) for a in (means, quats, log_s, logit))
    sc = np.exp(ls)
    if sc.shape[1] == 2:
        sc = np.concatenate([sc, np.zeros((sc.shape[0], 1))], 1)
    return (m.astype(np.float32), q.astype(np.float32), sc.astype(np.float32),
            (1.0 / (1.0 + np.exp(-lo))).astype(np.float32))


@pytest.mark.parametrize("dims,dtype", [(3, "float"), (2, "float"), (3, "double")])
def test_reads_trainer_layout(cs, tmp_path, dims, dtype):
    raw = _raw(5000, seed=7 + dims, dims=dims)
    path = str(tmp_path / "scene.ply")
    write_gaussian_ply(path, *raw, dtype=dtype, extra_before=3, faces=2)
    got = cs.csplat_ply_read(path)
    want = _expect(*raw, dtype)
    for g, w, name in zip(got, want, ("means", "quats", "scales", "opacity")):
        assert g.shape == w.shape, name
        # both sides round a double exp/sigmoid to float32: equal to within one ulp
        assert np.all(np.abs(g - w) <= np.spacing(np.abs(w)) + 0), name
    if dims == 2:
        assert np.all(got[2][:, 2] == 0)


def test_empty_and_errors(cs, tmp_path):
    raw = _raw(10, seed=3)
    p0 = str(tmp_path / "empty.ply")
    write_gaussian_ply(p0, *[a[:0] for a in raw])
    assert all(a.shape[0] == 0 for a in cs.csplat_ply_read(p0))
    bad = {
        "ascii": dict(fmt="ascii"),
        "missing": dict(drop=("rot_3",)),
        "noscale": dict(drop=("scale_1",)),
    }
    for name, kw in bad.items():
        p = str(tmp_path / f"{name}.ply")
        write_gaussian_ply(p, *raw, **kw)
        with pytest.raises(cs.CsplatError):
            cs.csplat_ply_read(p)
    p = str(tmp_path / "trunc.ply")
    write_gaussian_ply(p, *raw)
    data = open(p, "rb").read()
    open(p, "wb").write(data[:-20])
    with pytest.raises(cs.CsplatError):
        cs.csplat_ply_read(p)
    with pytest.raises(cs.CsplatError):
        cs.csplat_ply_read(str(tmp_path / "does_not_exist.ply"))
    open(p, "wb").write(b"not a ply file\n")
    with pytest.raises(cs.CsplatError):
        cs.csplat_ply_read(p)
