"""Pins of the oracle's batched RRT step (Sec. II-E): nearest node against a
k-d tree (a library routine), steering in closed form, growth in free space,
the capacity, and collision of edges with one isotropic Gaussian decided by
the closed-form threshold distance rho* = n s + sqrt(n^2 s^2 + r^2)."""
import math

import numpy as np
from scipy.spatial import cKDTree

FAR = np.array([[100.0, 100.0, 100.0]])


def _iso(oracle_mod, centers, s):
    """Prepared isotropic Gaussians (scale s) at `centers`."""
    c = np.asarray(centers, np.float64).reshape(-1, 3)
    sig = np.repeat((np.eye(3) * s * s)[None], c.shape[0], 0)
    return c, sig


def test_rrt_nearest_and_steer(oracle_mod):
    rng = np.random.default_rng(401)
    nodes = rng.uniform(0, 1, (300, 3))
    parents = np.arange(300) - 1
    samples = rng.uniform(0, 1, (64, 3))
    mu, sig = _iso(oracle_mod, FAR, 0.01)
    step = 0.07
    out = oracle_mod.rrt_step(mu, sig, nodes, parents, samples, [[0, 0, 0]], [0.05], step, 0.01, 1.0, 0, 10_000)
    dist, idx = cKDTree(nodes).query(samples)
    assert np.allclose(np.linalg.norm(nodes[out["nearest"]] - samples, axis=1), dist, rtol=0, atol=1e-15)
    for b in range(64):
        assert idx[b] in out["ties"][b]
        base = nodes[out["nearest"][b]]
        e = out["end"][b]
        assert math.isclose(np.linalg.norm(e - base), min(step, dist[b]), rel_tol=1e-12)
        # on the segment from the node to the sample
        assert np.linalg.norm(np.cross(e - base, samples[b] - base)) <= 1e-12
        assert np.dot(e - base, samples[b] - base) >= 0
    assert out["n_strides"] == math.ceil(float(np.float32(0.07) / np.float32(0.01)))


def test_rrt_free_space_growth_and_capacity(oracle_mod):
    rng = np.random.default_rng(402)
    mu, sig = _iso(oracle_mod, FAR, 0.01)
    nodes, parents = np.array([[0.5, 0.5, 0.5]]), np.array([-1])
    for it in range(4):
        smp = rng.uniform(0, 1, (32, 3))
        out = oracle_mod.rrt_step(mu, sig, nodes, parents, smp, [[0, 0, 0], [0.02, 0, 0]], [0.03, 0.02], 0.1, 0.02,
                                  2.0, 0, 10_000)
        assert out["valid"].all()
        assert out["nodes"].shape[0] == nodes.shape[0] + 32
        new = out["nodes"][nodes.shape[0]:]
        par = out["parents"][nodes.shape[0]:]
        assert np.all(np.linalg.norm(new - out["nodes"][par], axis=1) <= 0.1 * (1 + 1e-12))
        assert np.array_equal(par, out["nearest"])            # batch order
        nodes, parents = out["nodes"], out["parents"]
    # the capacity stops the growth, keeping the first edges of the batch
    out = oracle_mod.rrt_step(mu, sig, nodes, parents, rng.uniform(0, 1, (32, 3)), [[0, 0, 0]], [0.03], 0.1, 0.02,
                              2.0, 0, nodes.shape[0] + 5)
    assert out["nodes"].shape[0] == nodes.shape[0] + 5
    assert np.array_equal(out["parents"][nodes.shape[0]:], out["nearest"][:5])
    # a sample on its nearest node gives an edge of length 0: not appended
    out = oracle_mod.rrt_step(mu, sig, nodes, parents, nodes[3:4], [[0, 0, 0]], [0.03], 0.1, 0.02, 2.0, 0, 10_000)
    assert not out["valid"][0] and out["nodes"].shape[0] == nodes.shape[0]


def test_rrt_single_obstacle_closed_form(oracle_mod):
    """Robot: one sphere of radius r (or a second link at an offset); obstacle:
    one isotropic Gaussian of scale s at mu.  A state collides iff its link
    centre lies within rho* of mu (k = 0); an edge is kept iff none of its
    check points does."""
    s, r, n = 0.02, 0.05, 1.0
    rho = n * s + math.sqrt(n * n * s * s + r * r)
    mu_c = np.array([0.5, 0.5, 0.5])
    mu, sig = _iso(oracle_mod, mu_c[None], s)
    root = np.array([[0.3, 0.5, 0.5]])
    rng = np.random.default_rng(403)
    step, res = 0.3, 0.01
    T = math.ceil(float(np.float32(step) / np.float32(res)))
    for offsets, radii in (([[0, 0, 0]], [r]), ([[0, 0, 0], [0, 0.12, 0]], [0.001, r])):
        off = np.asarray(offsets, np.float64)
        smp = root + np.column_stack([np.full(200, 0.3), rng.uniform(-0.25, 0.25, 200), rng.uniform(-0.25, 0.25, 200)])
        out = oracle_mod.rrt_step(mu, sig, root, [-1], smp, offsets, radii, step, res, n, 0, 10_000)
        checked = 0
        for b in range(200):
            pts = root[0] + (np.arange(1, T + 1) / T)[:, None] * (out["end"][b] - root[0])[None]
            near = np.inf
            for l in range(off.shape[0]):
                # a link of tiny radius collides only within n s + sqrt(n^2 s^2 + r_l^2)
                rl = radii[l]
                rho_l = n * s + math.sqrt(n * n * s * s + rl * rl)
                dd = np.linalg.norm(pts + off[l] - mu_c, axis=1)
                near = min(near, np.min(dd / rho_l))
            if abs(near - 1) < 1e-6:
                continue   # a check point on the threshold: either answer is allowed
            assert out["valid"][b] == (near > 1), (b, near)
            checked += 1
        assert checked > 190
        assert 10 < out["valid"].sum() < 190       # both outcomes occur
    assert rho > r
