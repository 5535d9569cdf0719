"""Synthetic 3DGS scenes and robot-sphere query batches, seeded with PCG64.

Every array is float32, row-major, ready for the C-ABI:
  means   (N, 3)  Gaussian centres
  quats   (N, 4)  rotation quaternion (w, x, y, z), NOT normalised (the method
                  normalises; drawing 4 iid normals gives uniform rotations)
  scales  (N, 3)  linear per-axis standard deviations
  opacity (N,)    in (0, 1)
  centers (Q, 3), radii (Q,) for the query spheres.

The scale/opacity law is the same for every workload: per-axis log-scale
~ N(ln 0.03, 0.5^2), opacity = sigmoid(N(0, 1.5^2)).  Scene geometry and query
shapes mimic the paper's use cases (MPPI rollouts of shape (K, T, N_link) and
RRT edge checks, Sec. II-D/II-E; grid-of-points evaluation, Sec. III-B).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LOG_SCALE_MEAN = math.log(0.03)
LOG_SCALE_STD = 0.5
OPACITY_LOGIT_STD = 1.5


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    quats: np.ndarray
    scales: np.ndarray
    opacity: np.ndarray

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx].copy(), self.quats[idx].copy(),
                     self.scales[idx].copy(), self.opacity[idx].copy())


@dataclasses.dataclass
class Queries:
    centers: np.ndarray
    radii: np.ndarray

    @property
    def q(self) -> int:
        return int(self.centers.shape[0])

    def subset(self, idx) -> "Queries":
        return Queries(self.centers[idx].copy(), self.radii[idx].copy())


@dataclasses.dataclass
class Bodies:
    """Ellipsoidal robot bodies: centre, orientation quaternion (w, x, y, z;
    not necessarily unit) and semi-axes along the body's local x, y, z."""
    centers: np.ndarray
    quats: np.ndarray
    axes: np.ndarray

    @property
    def q(self) -> int:
        return int(self.centers.shape[0])

    def subset(self, idx) -> "Bodies":
        return Bodies(self.centers[idx].copy(), self.quats[idx].copy(), self.axes[idx].copy())


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def common_attrs(rng: np.random.Generator, n: int):
    """Quaternions, linear scales and opacities drawn from the common law."""
    quats = rng.normal(size=(n, 4))
    # a draw of exactly zero norm has probability zero; keep the guard anyway
    bad = np.linalg.norm(quats, axis=1) == 0.0
    quats[bad, 0] = 1.0
    log_s = rng.normal(LOG_SCALE_MEAN, LOG_SCALE_STD, size=(n, 3))
    logit = rng.normal(0.0, OPACITY_LOGIT_STD, size=n)
    return (quats.astype(np.float32), np.exp(log_s).astype(np.float32),
            (1.0 / (1.0 + np.exp(-logit))).astype(np.float32))


def _finish(rng, means) -> Scene:
    q, s, o = common_attrs(rng, means.shape[0])
    return Scene(np.ascontiguousarray(means, dtype=np.float32), q, s, o)


def uniform_box_scene(n: int, seed: int, box=(4.0, 4.0, 2.0)) -> Scene:
    rng = _rng(seed)
    means = rng.uniform(0.0, 1.0, size=(n, 3)) * np.asarray(box)
    return _finish(rng, means)


def room_scene(n: int, seed: int, size=(10.0, 10.0, 3.0), surface_frac=0.8,
               n_clusters=50, cluster_sigma=0.3, normal_sigma=0.01) -> Scene:
    """Floor + 4 walls (chosen in proportion to area, offset along the normal by
    N(0, normal_sigma^2)) and Gaussian clutter clusters."""
    rng = _rng(seed)
    lx, ly, lz = size
    n_surf = int(round(surface_frac * n))
    n_clu = n - n_surf
    # faces: floor z=0, walls x=0, x=lx, y=0, y=ly
    areas = np.array([lx * ly, ly * lz, ly * lz, lx * lz, lx * lz])
    face = rng.choice(5, size=n_surf, p=areas / areas.sum())
    u = rng.uniform(size=(n_surf, 2))
    off = rng.normal(0.0, normal_sigma, size=n_surf)
    pts = np.empty((n_surf, 3))
    f0 = face == 0
    pts[f0] = np.stack([u[f0, 0] * lx, u[f0, 1] * ly, off[f0]], 1)
    f1 = face == 1
    pts[f1] = np.stack([off[f1], u[f1, 0] * ly, u[f1, 1] * lz], 1)
    f2 = face == 2
    pts[f2] = np.stack([lx - off[f2], u[f2, 0] * ly, u[f2, 1] * lz], 1)
    f3 = face == 3
    pts[f3] = np.stack([u[f3, 0] * lx, off[f3], u[f3, 1] * lz], 1)
    f4 = face == 4
    pts[f4] = np.stack([u[f4, 0] * lx, ly - off[f4], u[f4, 1] * lz], 1)
    centres = np.stack([rng.uniform(0.5, lx - 0.5, n_clusters),
                        rng.uniform(0.5, ly - 0.5, n_clusters),
                        rng.uniform(0.2, 2.5, n_clusters)], 1)
    which = np.repeat(np.arange(n_clusters), n_clu // n_clusters)
    which = np.concatenate([which, rng.integers(0, n_clusters, n_clu - which.size)])
    clu = centres[which] + rng.normal(0.0, cluster_sigma, size=(n_clu, 3))
    means = np.concatenate([pts, clu], 0)
    return _finish(rng, means)


def tabletop_scene(n: int, seed: int, n_boxes=15, n_cyl=15, normal_sigma=0.01) -> Scene:
    """A 1.5 x 1 m table plane at z=0 with box and cylinder objects (sizes
    5-30 cm, random yaw); splats on exposed surfaces in proportion to area."""
    rng = _rng(seed)
    objs = []
    for kind in ["box"] * n_boxes + ["cyl"] * n_cyl:
        if kind == "box":
            ex, ey, h = rng.uniform(0.05, 0.30, 3)
            rad = None
        else:
            dia, h = rng.uniform(0.05, 0.30, 2)
            ex = ey = None
            rad = dia / 2
        cx, cy = rng.uniform(0.15, 1.35), rng.uniform(0.15, 0.85)
        yaw = rng.uniform(0, 2 * math.pi)
        objs.append((kind, cx, cy, yaw, ex, ey, rad, h))
    # surface list: (area, sampler)
    surfs = [(1.5 * 1.0, "table", None)]
    for o in objs:
        kind, cx, cy, yaw, ex, ey, rad, h = o
        if kind == "box":
            surfs.append((ex * ey, "boxtop", o))
            surfs.append((2 * (ex + ey) * h, "boxside", o))
        else:
            surfs.append((math.pi * rad * rad, "cyltop", o))
            surfs.append((2 * math.pi * rad * h, "cylside", o))
    areas = np.array([s[0] for s in surfs])
    pick = rng.choice(len(surfs), size=n, p=areas / areas.sum())
    pts = np.empty((n, 3))
    nrm = np.empty((n, 3))
    for si, (_, kind, o) in enumerate(surfs):
        idx = np.nonzero(pick == si)[0]
        m = idx.size
        if m == 0:
            continue
        if kind == "table":
            p = np.stack([rng.uniform(0, 1.5, m), rng.uniform(0, 1.0, m), np.zeros(m)], 1)
            nv = np.tile([0.0, 0.0, 1.0], (m, 1))
        else:
            _, cx, cy, yaw, ex, ey, rad, h = o
            if kind == "boxtop":
                lp = np.stack([rng.uniform(-ex / 2, ex / 2, m), rng.uniform(-ey / 2, ey / 2, m),
                               np.full(m, h)], 1)
                ln = np.tile([0.0, 0.0, 1.0], (m, 1))
            elif kind == "boxside":
                per = 2 * (ex + ey)
                t = rng.uniform(0, per, m)
                z = rng.uniform(0, h, m)
                lp = np.empty((m, 3))
                ln = np.zeros((m, 3))
                a = t < ex
                lp[a] = np.stack([t[a] - ex / 2, np.full(a.sum(), -ey / 2), z[a]], 1); ln[a, 1] = -1
                b = (t >= ex) & (t < ex + ey)
                lp[b] = np.stack([np.full(b.sum(), ex / 2), t[b] - ex - ey / 2, z[b]], 1); ln[b, 0] = 1
                c = (t >= ex + ey) & (t < 2 * ex + ey)
                lp[c] = np.stack([t[c] - ex - ey - ex / 2, np.full(c.sum(), ey / 2), z[c]], 1); ln[c, 1] = 1
                d = t >= 2 * ex + ey
                lp[d] = np.stack([np.full(d.sum(), -ex / 2), t[d] - 2 * ex - ey - ey / 2, z[d]], 1); ln[d, 0] = -1
            elif kind == "cyltop":
                rr = rad * np.sqrt(rng.uniform(0, 1, m))
                th = rng.uniform(0, 2 * math.pi, m)
                lp = np.stack([rr * np.cos(th), rr * np.sin(th), np.full(m, h)], 1)
                ln = np.tile([0.0, 0.0, 1.0], (m, 1))
            else:
                th = rng.uniform(0, 2 * math.pi, m)
                lp = np.stack([rad * np.cos(th), rad * np.sin(th), rng.uniform(0, h, m)], 1)
                ln = np.stack([np.cos(th), np.sin(th), np.zeros(m)], 1)
            cyaw, syaw = math.cos(yaw), math.sin(yaw)
            p = np.stack([cx + cyaw * lp[:, 0] - syaw * lp[:, 1],
                          cy + syaw * lp[:, 0] + cyaw * lp[:, 1], lp[:, 2]], 1)
            nv = np.stack([cyaw * ln[:, 0] - syaw * ln[:, 1],
                           syaw * ln[:, 0] + cyaw * ln[:, 1], ln[:, 2]], 1)
        pts[idx] = p
        nrm[idx] = nv
    means = pts + nrm * rng.normal(0.0, normal_sigma, size=(n, 1))
    return _finish(rng, means)


def stone_circle_scene(n: int, seed: int, n_columns=12, clutter_frac=0.2, normal_sigma=0.003) -> Scene:
    """A scene shaped like the paper's normalised ring of standing stones, in
    the unit cube: a ground slab (z = 0), a ring of upright columns (radius
    U[0.02, 0.05], height U[0.25, 0.45]) with lintel slabs on pairs of them;
    (1 - clutter_frac) of the splats on the surfaces in proportion to area,
    offset along the normal by N(0, normal_sigma^2), the rest uniform clutter."""
    rng = _rng(seed)
    n_surf = int(round(n * (1 - clutter_frac)))
    ang = np.linspace(0, 2 * math.pi, n_columns, endpoint=False) + rng.uniform(0, 0.2, n_columns)
    cx, cy = 0.5 + 0.35 * np.cos(ang), 0.5 + 0.35 * np.sin(ang)
    rad = rng.uniform(0.02, 0.05, n_columns)
    hgt = rng.uniform(0.25, 0.45, n_columns)
    # surfaces: ground, column mantles, lintels (boxes between neighbours, every other pair)
    areas = [1.0] + list(2 * math.pi * rad * hgt)
    lintels = []
    for i in range(0, n_columns, 2):
        k = (i + 1) % n_columns
        p0 = np.array([cx[i], cy[i]]); p1 = np.array([cx[k], cy[k]])
        z = min(hgt[i], hgt[k])
        lintels.append((p0, p1, z))
        areas.append(2 * np.linalg.norm(p1 - p0) * 0.06)
    areas = np.asarray(areas)
    which = rng.choice(areas.size, n_surf, p=areas / areas.sum())
    pts = np.empty((n_surf, 3))
    u = rng.uniform(size=(n_surf, 2))
    off = rng.normal(0.0, normal_sigma, n_surf)
    g = which == 0
    pts[g] = np.stack([u[g, 0], u[g, 1], off[g]], 1)
    for c in range(n_columns):
        sel = which == 1 + c
        th = 2 * math.pi * u[sel, 0]
        rr = rad[c] + off[sel]
        pts[sel] = np.stack([cx[c] + rr * np.cos(th), cy[c] + rr * np.sin(th), u[sel, 1] * hgt[c]], 1)
    for li, (p0, p1, z) in enumerate(lintels):
        sel = which == 1 + n_columns + li
        t = u[sel, 0]
        side = np.where(u[sel, 1] < 0.5, 0.0, 0.06)
        xy = p0[None] + (p1 - p0)[None] * t[:, None]
        pts[sel] = np.stack([xy[:, 0], xy[:, 1], z + side + off[sel]], 1)
    clutter = rng.uniform(0, 1, (n - n_surf, 3)) * np.array([1.0, 1.0, 0.6])
    return _finish(rng, np.concatenate([pts, clutter], 0))


def uniform_queries(q: int, seed: int, box=(4.0, 4.0, 2.0), radius=0.1) -> Queries:
    rng = _rng(seed)
    c = rng.uniform(0.0, 1.0, size=(q, 3)) * np.asarray(box)
    return Queries(c.astype(np.float32), np.full(q, radius, np.float32))


def mppi_walk_queries(rollouts: int, steps: int, seed: int, radius=0.2, step_len=0.05,
                      heading_sigma=0.15, z_sigma=0.01, size=(10.0, 10.0, 3.0)) -> Queries:
    """Smooth random walks (one sphere per step), rollout-major order:
    query index = rollout * steps + step."""
    rng = _rng(seed)
    lx, ly, _ = size
    start = np.stack([rng.uniform(1, lx - 1, rollouts), rng.uniform(1, ly - 1, rollouts),
                      rng.uniform(0.3, 1.5, rollouts)], 1)
    th = rng.uniform(0, 2 * math.pi, rollouts)
    out = np.empty((rollouts, steps, 3))
    p = start.copy()
    for t in range(steps):
        out[:, t] = p
        th = th + rng.normal(0, heading_sigma, rollouts)
        p = p + np.stack([step_len * np.cos(th), step_len * np.sin(th),
                          rng.normal(0, z_sigma, rollouts)], 1)
        p[:, 2] = np.clip(p[:, 2], 0.2, 2.8)
    c = out.reshape(-1, 3).astype(np.float32)
    return Queries(c, np.full(c.shape[0], radius, np.float32))


_AXES = "zyyzyzy"
_SPHERES_PER_LINK = (7, 7, 7, 7, 7, 7, 6)


def _axis_rot(axis: str, ang: np.ndarray) -> np.ndarray:
    c, s = np.cos(ang), np.sin(ang)
    o, z = np.ones_like(ang), np.zeros_like(ang)
    if axis == "z":
        m = [[c, -s, z], [s, c, z], [z, z, o]]
    else:  # y
        m = [[c, z, s], [z, o, z], [-s, z, c]]
    return np.moveaxis(np.array(m), (0, 1), (-2, -1))


def chain_queries(configs: int, steps: int, seed: int, base=(0.75, 0.1, 0.1)) -> Queries:
    """A random 7-link revolute chain (axes z,y,y,z,y,z,y; link lengths
    U[0.1,0.2] along the local z axis) on a 10 cm pedestal near the table's
    near edge, with 48 spheres placed at equal fractions along the links;
    joint paths q0 ~ U(-pi/2, pi/2)^7,
    q_{t+1} = q_t + N(0, 0.05^2).  Index = (config * steps + step) * 48 + sphere."""
    rng = _rng(seed)
    lengths = rng.uniform(0.1, 0.2, 7)
    nsph = sum(_SPHERES_PER_LINK)
    radii = rng.uniform(0.03, 0.10, nsph)
    q = np.empty((configs, steps, 7))
    q[:, 0] = rng.uniform(-math.pi / 2, math.pi / 2, (configs, 7))
    for t in range(1, steps):
        q[:, t] = q[:, t - 1] + rng.normal(0, 0.05, (configs, 7))
    qf = q.reshape(-1, 7)
    B = qf.shape[0]
    Rw = np.tile(np.eye(3), (B, 1, 1))
    pw = np.tile(np.asarray(base, float), (B, 1))
    centers = np.empty((B, nsph, 3))
    k = 0
    for l in range(7):
        Rw = Rw @ _axis_rot(_AXES[l], qf[:, l])
        seg = Rw[:, :, 2] * lengths[l]
        ns = _SPHERES_PER_LINK[l]
        for i in range(ns):
            centers[:, k] = pw + seg * ((i + 0.5) / ns)
            k += 1
        pw = pw + seg
    c = centers.reshape(-1, 3).astype(np.float32)
    r = np.tile(radii, B).astype(np.float32)
    return Queries(c, r)


def _qmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product of (w, x, y, z) quaternions, broadcast over leading axes."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def _axis_quat(axis: str, ang: np.ndarray) -> np.ndarray:
    c, s = np.cos(ang / 2), np.sin(ang / 2)
    z = np.zeros_like(ang)
    return np.stack([c, z, z, s] if axis == "z" else [c, z, s, z], -1)


def chain_ellipsoids(configs: int, steps: int, seed: int, base=(0.75, 0.1, 0.1)) -> Bodies:
    """The 7-link chain of chain_queries with one ellipsoid per link: centred on
    the link, local z along it, semi-axes (r_l, r_l, L_l / 2 + r_l) with link
    radii r_l ~ U[0.04, 0.08].  Index = (config * steps + step) * 7 + link."""
    rng = _rng(seed)
    lengths = rng.uniform(0.1, 0.2, 7)
    link_r = rng.uniform(0.04, 0.08, 7)
    q = np.empty((configs, steps, 7))
    q[:, 0] = rng.uniform(-math.pi / 2, math.pi / 2, (configs, 7))
    for t in range(1, steps):
        q[:, t] = q[:, t - 1] + rng.normal(0, 0.05, (configs, 7))
    qf = q.reshape(-1, 7)
    B = qf.shape[0]
    Rw = np.tile(np.eye(3), (B, 1, 1))
    qw = np.tile(np.array([1.0, 0.0, 0.0, 0.0]), (B, 1))
    pw = np.tile(np.asarray(base, float), (B, 1))
    centers = np.empty((B, 7, 3))
    quats = np.empty((B, 7, 4))
    axes = np.empty((B, 7, 3))
    for l in range(7):
        Rw = Rw @ _axis_rot(_AXES[l], qf[:, l])
        qw = _qmul(qw, _axis_quat(_AXES[l], qf[:, l]))
        seg = Rw[:, :, 2] * lengths[l]
        centers[:, l] = pw + 0.5 * seg
        quats[:, l] = qw
        axes[:, l] = (link_r[l], link_r[l], 0.5 * lengths[l] + link_r[l])
        pw = pw + seg
    return Bodies(centers.reshape(-1, 3).astype(np.float32), quats.reshape(-1, 4).astype(np.float32),
                  axes.reshape(-1, 3).astype(np.float32))


def random_ellipsoids(q: int, seed: int, box=(4.0, 4.0, 2.0), axis_range=(0.02, 0.2)) -> Bodies:
    """Centres uniform in the box, orientations from 4 iid normals (left
    unnormalised), semi-axes uniform in axis_range."""
    rng = _rng(seed)
    c = rng.uniform(0, 1, (q, 3)) * np.asarray(box)
    quat = rng.normal(size=(q, 4))
    ax = rng.uniform(axis_range[0], axis_range[1], (q, 3))
    return Bodies(c.astype(np.float32), quat.astype(np.float32), ax.astype(np.float32))


def grid_queries(res: int, size=(10.0, 10.0, 3.0), radius_classes=(0.05, 0.10, 0.20, 0.40),
                 stress_scene: Scene | None = None, seed: int = 0, stress_frac=0.5) -> Queries:
    """Cell centres of a res^3 grid over the box (x fastest); radius class =
    index mod len(radius_classes).  With stress_scene, a fraction of points is
    replaced by near-surface points mu_i + u * r * U[0.5, 1.5]."""
    ax = [(np.arange(res) + 0.5) * (size[d] / res) for d in range(3)]
    zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    c = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
    rc = np.asarray(radius_classes)
    r = rc[np.arange(c.shape[0]) % rc.size]
    if stress_scene is not None:
        rng = _rng(seed)
        sel = rng.uniform(size=c.shape[0]) < stress_frac
        m = int(sel.sum())
        gi = rng.integers(0, stress_scene.n, m)
        u = rng.normal(size=(m, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        c[sel] = stress_scene.means[gi] + u * (r[sel] * rng.uniform(0.5, 1.5, m))[:, None]
    return Queries(c.astype(np.float32), r.astype(np.float32))


def serving_stream(n_requests: int, seed: int, rate_hz: float, scene_ids=(0, 1),
                   max_mppi_k=4096, max_rrt_points=10000, max_spheres=48, steps=32):
    """A Poisson request stream mixing MPPI batches (K in {256..4096} x steps x L
    spheres) and RRT edge checks (P in 1..10000 points x L spheres).  Returns a
    list of dicts with arrival time, scene, kind, centres, radii and n_sigma."""
    rng = _rng(seed)
    t = 0.0
    reqs = []
    ks = [k for k in (256, 512, 1024, 2048, 4096) if k <= max_mppi_k]
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        kind = "mppi" if rng.uniform() < 0.5 else "rrt"
        scene = int(scene_ids[rng.integers(0, len(scene_ids))])
        L = int(rng.integers(1, max_spheres + 1))
        if L == 1:
            offs = np.zeros((1, 3))
            rad = np.array([0.2])
        else:
            offs = rng.uniform(-0.3, 0.3, (L, 3))
            rad = rng.uniform(0.03, 0.10, L)
        if kind == "mppi":
            K = int(ks[rng.integers(0, len(ks))])
            sub = int(rng.integers(1 << 30))
            path = mppi_walk_queries(K, steps, seed=sub).centers.astype(np.float64)
        else:
            P = int(rng.integers(1, max_rrt_points + 1))
            a = np.array([rng.uniform(1, 9), rng.uniform(1, 9), rng.uniform(0.3, 1.5)])
            seg_len = rng.uniform(0, 1.0)
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            f = (np.arange(P) + 0.5) / P
            path = a[None, :] + f[:, None] * (seg_len * d)[None, :]
        c = (path[:, None, :] + offs[None, :, :]).reshape(-1, 3).astype(np.float32)
        r = np.tile(rad, path.shape[0]).astype(np.float32)
        reqs.append(dict(id=i, t=t, kind=kind, scene=scene, centers=c, radii=r,
                         n_sigma=float(rng.integers(0, 3))))
    return reqs


# Named workloads.  Reduction defaults: k=2, tau=0.1, d_max=1, gamma=1, s_min=1;
# floater filter alpha_f=0.05, extent_f=0.1 m.
CONFIG_NAMES = ("tiny", "mppi_nav", "manip", "precision", "manip_ell", "paper_p0")

REDUCE_DEFAULTS = dict(k=2, tau=0.1, d_max=1.0, gamma=1.0, s_min=1.0)
FLOATER = dict(alpha_f=0.05, extent_f=0.1)


def config(name: str, scale: float = 1.0):
    """Scene, queries and parameters of a named workload.  `scale` < 1 shrinks
    N and Q proportionally (for tests); the laws and seeds stay the same."""
    def sz(v):
        return max(1, int(round(v * scale)))
    if name == "tiny":
        sc = uniform_box_scene(sz(10_000), seed=1)
        qs = uniform_queries(sz(4096), seed=101)
        par = dict(n_sigma=[1.0], r_nbr=math.inf)
    elif name == "mppi_nav":
        sc = room_scene(sz(1_000_000), seed=2)
        qs = mppi_walk_queries(sz(1024), 32, seed=102)
        par = dict(n_sigma=[0.0, 1.0, 2.0], r_nbr=1.0)
    elif name == "manip":
        sc = tabletop_scene(sz(500_000), seed=3)
        qs = chain_queries(sz(256), 32, seed=103)
        par = dict(n_sigma=[1.0], r_nbr=0.3)
    elif name == "manip_ell":
        sc = tabletop_scene(sz(500_000), seed=3)
        qs = chain_ellipsoids(sz(256), 32, seed=106)
        par = dict(n_sigma=[1.0], r_nbr=0.4)
    elif name == "paper_p0":
        # shaped like the paper's own measurement: ~200k Gaussians in a unit
        # scene, grid points as robot spheres of radius 0.015, labels
        sc = stone_circle_scene(sz(200_000), seed=6)
        res = max(4, int(round(32 * scale ** (1 / 3))))
        qs = grid_queries(res, size=(1.0, 1.0, 0.6), radius_classes=(0.015,))
        par = dict(n_sigma=[1.0], r_nbr=math.inf)
    elif name == "precision":
        sc = room_scene(sz(4_000_000), seed=4)
        res = max(4, int(round(64 * scale ** (1 / 3))))
        qs = grid_queries(res)
        par = dict(n_sigma=[1.0], r_nbr=math.inf)
    else:
        raise KeyError(name)
    p = dict(REDUCE_DEFAULTS)
    p.update(par)
    p.update(FLOATER)
    return sc, qs, p
