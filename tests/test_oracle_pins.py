"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formula: each compares it with a closed
form, a library routine, a Monte-Carlo estimate, an invariant of the method,
or brute force in a different formulation.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from workloads import Queries, Scene, common_attrs, uniform_box_scene, uniform_queries


def _scene(means, quats, scales, opacity=None):
    means = np.asarray(means, np.float32).reshape(-1, 3)
    n = means.shape[0]
    if opacity is None:
        opacity = np.full(n, 0.9, np.float32)
    return Scene(means, np.asarray(quats, np.float32).reshape(n, 4),
                 np.asarray(scales, np.float32).reshape(n, 3), np.asarray(opacity, np.float32))


def _random_scene(n, seed, box=(1.0, 1.0, 1.0)):
    return uniform_box_scene(n, seed=seed, box=box)


def _lib_sigma(quat_wxyz, scales):
    """Sigma from scipy's rotation (scalar-last convention) — a library construction."""
    w, x, y, z = [float(v) for v in quat_wxyz]
    R = Rotation.from_quat([x, y, z, w]).as_matrix()
    return R @ np.diag(np.asarray(scales, np.float64) ** 2) @ R.T, R


# --- P1: covariance and rotation (Eq. 2) ------------------------------------

def test_sigma_matches_library_rotation(oracle_mod):
    rng = np.random.default_rng(5)
    q, s, o = common_attrs(rng, 64)
    sc = Scene(rng.uniform(size=(64, 3)).astype(np.float32), q, s, o)
    _, _, sig = oracle_mod.prepare_scene(sc.means, sc.quats, sc.scales, sc.opacity)
    for i in range(64):
        ref, R = _lib_sigma(q[i], s[i])
        assert np.allclose(sig[i], ref, rtol=0, atol=1e-14 * np.abs(ref).max())
        # eigenvalues are the squared scales (library eigen-decomposition)
        ev = np.linalg.eigvalsh(sig[i])
        assert np.allclose(np.sort(ev), np.sort(s[i].astype(np.float64) ** 2), rtol=1e-12)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12) and abs(np.linalg.det(R) - 1) < 1e-12


def test_quaternion_sign_and_norm_invariance(oracle_mod):
    rng = np.random.default_rng(6)
    q, s, o = common_attrs(rng, 16)
    m = rng.uniform(size=(16, 3)).astype(np.float32)
    _, _, a = oracle_mod.prepare_scene(m, q, s, o)
    _, _, b = oracle_mod.prepare_scene(m, -q, s, o)
    _, _, c = oracle_mod.prepare_scene(m, (q * np.float32(4.0)), s, o)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-18)
    assert np.allclose(a, c, rtol=1e-13, atol=1e-18)


def test_rotation_direction(oracle_mod):
    # rotation by +30 degrees about z maps the local x axis to (cos30, sin30, 0)
    th = math.radians(30.0)
    qz = [math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)]
    _, _, sig = oracle_mod.prepare_scene([[0, 0, 0]], [qz], [[0.3, 0.01, 0.02]], [0.9])
    w, v = np.linalg.eigh(sig[0])
    axis = v[:, np.argmax(w)]
    assert abs(abs(axis @ np.array([math.cos(th), math.sin(th), 0.0])) - 1.0) < 1e-12


# --- P2: n_sigma = 0 is a strict radius count (Sec. II-B, Sec. III-C) -------

def test_point_cloud_limit_is_radius_count(oracle_mod):
    sc = _random_scene(2000, seed=11)
    qs = uniform_queries(300, seed=12, box=(1, 1, 1), radius=0.08)
    out = oracle_mod.evaluate_spheres(sc, qs, [0.0], k=3)
    d = np.linalg.norm(sc.means.astype(np.float64)[None] - qs.centers.astype(np.float64)[:, None], axis=2)
    cnt = (d < qs.radii.astype(np.float64)[:, None]).sum(1)
    assert np.array_equal(out["count"][:, 0], cnt)
    assert np.array_equal(out["label"][:, 0], (cnt > 3).astype(np.uint8))
    # the minimum is the squared nearest distance over r^2
    assert np.allclose(out["min"][:, 0], (d.min(1) / qs.radii.astype(np.float64)) ** 2, rtol=1e-12)


# --- P3: the linearised variance and the factor 2 in the gradient (Eq. 7) ---

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_linearised_variance_identity_monte_carlo(oracle_mod, seed):
    """For p ~ N(mu, Sigma), Var[(p-c)^T A (p-c)] = sigma^2_lin + 2 tr((A Sigma)^2).
    sigma_lin is read off the oracle as min(n=0) - min(n=1)."""
    rng = np.random.default_rng(seed)
    q, s, o = common_attrs(rng, 1)
    s = (s * 3).astype(np.float32)
    mu = np.zeros((1, 3), np.float32)
    _, mu64, sig = oracle_mod.prepare_scene(mu, q, s, o)
    # an ellipsoidal body (Eq. 6) at a distance of a few scales
    R_E = Rotation.random(random_state=seed).as_matrix()
    axes = rng.uniform(0.1, 0.2, 3)
    A = oracle_mod.ellipsoid_bodies(R_E[None], axes[None])
    c = rng.normal(size=3)
    c = c / np.linalg.norm(c) * 0.6
    out = oracle_mod.evaluate(mu64, sig, c[None], A, [0.0, 1.0])
    s2, red = out["min"][0]
    assert red > 0
    sd = s2 - red
    Sig, _ = _lib_sigma(q[0], s[0])
    Am = A[0]
    exact = 2 * np.trace(Am @ Sig @ Am @ Sig) + sd * sd
    # exact moment of a Gaussian quadratic form, independent of Eq. 7's derivation
    d = -c
    moment = 2 * np.trace(Am @ Sig @ Am @ Sig) + 4 * d @ Am @ Sig @ Am @ d
    assert abs(exact - moment) <= 1e-9 * moment
    # Monte Carlo, in a different formulation again
    gen = np.random.default_rng(100 + seed)
    p = gen.multivariate_normal(np.zeros(3), Sig, size=400_000)
    y = np.einsum("ni,ij,nj->n", p - c, Am, p - c)
    var = y.var()
    se = var * math.sqrt(2.0 / (p.shape[0] - 1)) * 3.0  # generous: quadratic forms have heavier tails
    assert abs(var - exact) < 4 * se


# --- P4/P5: isotropic closed form and principal axes (Eq. 5, 7, 8) ---------

def _single(oracle_mod, quat, scales, center, radius, n_sigma, **kw):
    _, mu, sig = oracle_mod.prepare_scene([[0, 0, 0]], [quat], [scales], [0.9])
    return oracle_mod.evaluate(mu, sig, np.asarray(center, np.float64)[None],
                               oracle_mod.sphere_bodies([radius]), n_sigma, **kw)


def test_isotropic_threshold_closed_form(oracle_mod):
    """Sigma = s^2 I and a sphere of radius r: collision iff
    rho < rho* = n s + sqrt(n^2 s^2 + r^2)."""
    s = float(np.float32(0.03))
    r = float(np.float32(0.1))
    expect = {0.0: 0.1, 0.5: 0.116119, 1.0: 0.134403, 2.0: 0.176619}
    rng = np.random.default_rng(0)
    for n, rho_tab in expect.items():
        rho = n * s + math.sqrt(n * n * s * s + r * r)
        assert abs(rho - rho_tab) < 1e-6
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        q = rng.normal(size=4)
        inside = _single(oracle_mod, q, [s, s, s], u * rho * (1 - 1e-9), r, [n])
        outside = _single(oracle_mod, q, [s, s, s], u * rho * (1 + 1e-9), r, [n])
        assert inside["count"][0, 0] == 1 and outside["count"][0, 0] == 0
        # value of s~^2 at random distances
        for rr in rng.uniform(0.01, 0.5, 5):
            out = _single(oracle_mod, q, [s, s, s], u * rr, r, [n])
            ref = max(0.0, (rr * rr - 2 * n * s * rr) / (r * r))
            assert abs(out["min"][0, 0] - ref) <= 1e-12 * max(1.0, ref)


def test_principal_axis_and_zero_scale(oracle_mod):
    rng = np.random.default_rng(1)
    r = float(np.float32(0.1))
    for trial in range(6):
        q = rng.normal(size=4).astype(np.float32)
        sc = rng.uniform(0.005, 0.08, 3).astype(np.float32)
        if trial >= 3:
            sc[trial - 3] = 0.0  # a flat (2DGS-like) axis
        _, R = _lib_sigma(q, sc)
        for k in range(3):
            for rho in (0.05, 0.12, 0.3):
                c = -R[:, k] * rho   # query displaced along principal axis k
                out = _single(oracle_mod, q, sc, c, r, [1.5])
                sk = float(sc[k])
                ref = max(0.0, (rho * rho - 2 * 1.5 * sk * rho) / (r * r))
                # along a zero axis the true variance is 0 and the explicit Sigma
                # leaves a residual of a few ulps of s_max^2 rho^2, which the square
                # root amplifies: allow sqrt of that residual
                resid = 2 * 1.5 * math.sqrt(8e-16) * rho * float(sc.max()) / (r * r)
                assert abs(out["min"][0, 0] - ref) <= 1e-11 * max(1.0, rho * rho / r / r) + resid


# --- P6: rigid-transform invariance -----------------------------------------

def _quat_mul(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b.T
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], 1)


def test_rigid_invariance(oracle_mod):
    sc = _random_scene(400, seed=21)
    qs = uniform_queries(64, seed=22, box=(1, 1, 1), radius=0.1)
    rng = np.random.default_rng(23)
    rot = Rotation.random(random_state=24)
    Rg = rot.as_matrix()
    x, y, z, w = rot.as_quat()
    t = rng.normal(size=3)
    # ellipsoidal bodies with random orientation
    R_E = Rotation.random(64, random_state=25).as_matrix()
    axes = rng.uniform(0.05, 0.15, (64, 3))
    ns = [0.0, 0.7, 1.5]
    kw = dict(k=1, tau=0.05, r_nbr=0.4, d_max=2.0, gamma=0.5)
    _, mu, sig = oracle_mod.prepare_scene(sc.means, sc.quats, sc.scales, sc.opacity)
    base = oracle_mod.evaluate(mu, sig, qs.centers, oracle_mod.ellipsoid_bodies(R_E, axes), ns, **kw)
    # transform in double: mu -> R mu + t, Sigma via the rotated quaternion, c -> R c + t
    qn = sc.quats.astype(np.float64)
    q2 = _quat_mul(np.array([w, x, y, z]), qn)
    sc2 = Scene(sc.means, q2.astype(np.float32), sc.scales, sc.opacity)
    _, _, sig2 = oracle_mod.prepare_scene(sc2.means, sc2.quats, sc2.scales, sc2.opacity)
    # rounding the rotated quaternion to float32 perturbs Sigma slightly: use the
    # exactly rotated covariance instead, and check the rounded one agrees
    sig_rot = Rg @ sig @ Rg.T
    assert np.allclose(sig2, sig_rot, rtol=0, atol=1e-6 * np.abs(sig).max())
    mu2 = mu @ Rg.T + t
    c2 = qs.centers.astype(np.float64) @ Rg.T + t
    moved = oracle_mod.evaluate(mu2, sig_rot, c2, oracle_mod.ellipsoid_bodies(Rg @ R_E, axes), ns, **kw)
    for key in ("min", "softmin", "cost"):
        a, b = base[key], moved[key]
        fin = np.isfinite(a)
        assert np.array_equal(fin, np.isfinite(b))
        assert np.allclose(a[fin], b[fin], rtol=1e-9, atol=1e-12)
    ok = base["ambiguous"] == 0
    assert np.array_equal(base["count"][ok], moved["count"][ok])
    assert np.array_equal(base["nbr"], moved["nbr"])


# --- P7/P8: monotonicity in n_sigma and in the scales (Sec. III-C) ---------

def test_monotone_in_nsigma(oracle_mod):
    sc = _random_scene(1500, seed=31)
    qs = uniform_queries(200, seed=32, box=(1, 1, 1), radius=0.05)
    out = oracle_mod.evaluate_spheres(sc, qs, [0.0, 0.25, 0.5, 1.0, 2.0], k=1, tau=0.1, r_nbr=0.5)
    assert np.all(np.diff(out["count"], axis=1) >= 0)
    assert np.all(np.diff(out["label"].astype(int), axis=1) >= 0)
    assert np.all(np.diff(out["min"], axis=1) <= 0)
    assert np.all(np.diff(out["softmin"], axis=1) <= 1e-12)
    assert np.all(np.diff(out["cost"], axis=1) >= -1e-15)
    assert out["count"][:, -1].sum() > out["count"][:, 0].sum()


def test_monotone_in_scale(oracle_mod):
    sc = _random_scene(1500, seed=33)
    qs = uniform_queries(200, seed=34, box=(1, 1, 1), radius=0.05)
    big = Scene(sc.means, sc.quats, (sc.scales * np.float32(1.5)), sc.opacity)
    a = oracle_mod.evaluate_spheres(sc, qs, [1.0], k=0, tau=0.1)
    b = oracle_mod.evaluate_spheres(big, qs, [1.0], k=0, tau=0.1)
    assert np.all(b["count"] >= a["count"]) and np.all(b["min"] <= a["min"])
    assert np.all(b["softmin"] <= a["softmin"] + 1e-12) and np.all(b["cost"] >= a["cost"] - 1e-15)


# --- P9: the reach bound is an exact cull ------------------------------------

def test_reach_bound_cull_is_exact(oracle_mod):
    sc = _random_scene(3000, seed=41)
    qs = uniform_queries(300, seed=42, box=(1, 1, 1), radius=0.07)
    ns = 1.5
    smax = float(sc.scales.max())
    reach = ns * smax + math.sqrt(ns * ns * smax * smax + 0.07 ** 2)
    full = oracle_mod.evaluate_spheres(sc, qs, [ns], k=2)
    cut = oracle_mod.evaluate_spheres(sc, qs, [ns], k=2, r_nbr=reach * (1 + 1e-6))
    assert np.array_equal(full["count"], cut["count"])
    assert np.array_equal(full["label"], cut["label"])
    assert np.all(cut["nbr"] <= full["nbr"]) and cut["nbr"].sum() < full["nbr"].sum()


# --- P11: softmin -------------------------------------------------------------

def test_softmin_properties(oracle_mod):
    sc = _random_scene(300, seed=51)
    qs = uniform_queries(40, seed=52, box=(1, 1, 1), radius=0.1)
    tau = 0.2
    out = oracle_mod.evaluate_spheres(sc, qs, [1.0], tau=tau)
    mn, sm, nb = out["min"][:, 0], out["softmin"][:, 0], out["nbr"]
    assert np.all(sm <= mn + 1e-15) and np.all(sm >= mn - tau * np.log(nb) - 1e-12)
    hard = oracle_mod.evaluate_spheres(sc, qs, [1.0], tau=1e-7)
    assert np.allclose(hard["softmin"][:, 0], mn, atol=1e-6)
    zero = oracle_mod.evaluate_spheres(sc, qs, [1.0], tau=0.0)
    assert np.array_equal(zero["softmin"], zero["min"])
    # permutation invariance
    perm = np.random.default_rng(53).permutation(sc.n)
    p = oracle_mod.evaluate_spheres(sc.subset(perm), qs, [1.0], tau=tau)
    assert np.allclose(p["softmin"], out["softmin"], rtol=1e-13, atol=1e-13)
    # equals the pairwise recursive fold min(a,b) - tau log1p(exp(-|a-b|/tau))
    _, mu, sig = oracle_mod.prepare_scene(sc.means, sc.quats, sc.scales, sc.opacity)
    for j in range(5):
        vals = [oracle_mod.evaluate(mu[i:i + 1], sig[i:i + 1], qs.centers[j:j + 1],
                                    oracle_mod.sphere_bodies(qs.radii[j:j + 1]), [1.0])["min"][0, 0]
                for i in range(mu.shape[0])]
        acc = vals[0]
        for v in vals[1:]:
            acc = min(acc, v) - tau * math.log1p(math.exp(-abs(acc - v) / tau))
        assert abs(acc - sm[j]) <= 1e-10 * max(1.0, abs(acc))


def test_softmin_of_identical_splats(oracle_mod):
    n = 7
    sc = _scene(np.zeros((n, 3)), np.tile([1, 0, 0, 0], (n, 1)), np.full((n, 3), 0.02))
    q = Queries(np.array([[0.3, 0.0, 0.0]], np.float32), np.array([0.1], np.float32))
    out = oracle_mod.evaluate_spheres(sc, q, [1.0], tau=0.3)
    one = oracle_mod.evaluate_spheres(sc.subset([0]), q, [1.0], tau=0.3)
    assert one["softmin"][0, 0] == one["min"][0, 0]
    assert abs(out["softmin"][0, 0] - (one["min"][0, 0] - 0.3 * math.log(n))) < 1e-12


# --- P12: the MPPI collision cost (Eq. 11) -----------------------------------

def test_cost_properties(oracle_mod):
    s = float(np.float32(0.03))
    r = float(np.float32(0.1))
    rng = np.random.default_rng(61)
    q = rng.normal(size=4)
    for rho in (0.05, 0.2, 0.4):
        out = _single(oracle_mod, q, [s, s, s], [rho, 0, 0], r, [1.0], d_max=2.5, gamma=0.7)
        x = max(0.0, (rho * rho - 2 * s * rho) / (r * r))
        assert abs(out["cost"][0, 0] - 2.5 * math.exp(-0.7 * max(x - 1.0, 0.0))) < 1e-12
        g0 = _single(oracle_mod, q, [s, s, s], [rho, 0, 0], r, [1.0], d_max=2.5, gamma=0.0)
        assert g0["cost"][0, 0] == 2.5
    # the mean over the neighbourhood: two splats average their costs
    sc = _scene([[0.05, 0, 0], [0.3, 0, 0]], [[1, 0, 0, 0]] * 2, [[s] * 3] * 2)
    qq = Queries(np.zeros((1, 3), np.float32), np.array([r], np.float32))
    both = oracle_mod.evaluate_spheres(sc, qq, [1.0], gamma=0.7)
    each = [oracle_mod.evaluate_spheres(sc.subset([i]), qq, [1.0], gamma=0.7)["cost"][0, 0] for i in (0, 1)]
    assert abs(both["cost"][0, 0] - 0.5 * sum(each)) < 1e-15
    # every splat inside (s~^2 <= s_min): cost = d_max
    inside = oracle_mod.evaluate_spheres(sc.subset([0]), qq, [1.0], d_max=3.0, gamma=5.0)
    assert inside["cost"][0, 0] == 3.0


def test_empty_neighbourhood(oracle_mod):
    sc = _scene([[5, 5, 5]], [[1, 0, 0, 0]], [[0.03] * 3])
    qq = Queries(np.zeros((2, 3), np.float32), np.array([0.1, 0.2], np.float32))
    out = oracle_mod.evaluate_spheres(sc, qq, [1.0], r_nbr=1.0, tau=0.1)
    assert np.all(out["nbr"] == 0) and np.all(out["count"] == 0) and np.all(out["cost"] == 0)
    assert np.all(np.isinf(out["min"])) and np.all(np.isinf(out["softmin"]))
    empty = Scene(np.zeros((0, 3), np.float32), np.zeros((0, 4), np.float32),
                  np.zeros((0, 3), np.float32), np.zeros(0, np.float32))
    out = oracle_mod.evaluate_spheres(empty, qq, [1.0])
    assert np.all(out["count"] == 0) and np.all(np.isinf(out["min"]))


# --- Sec. II-C floater filter, raw 3DGS parameters, invalid inputs ----------

def test_floater_filter(oracle_mod):
    means = np.zeros((4, 3))
    quats = np.tile([1, 0, 0, 0], (4, 1))
    scales = [[0.2, 0.01, 0.01], [0.05, 0.05, 0.05], [0.2, 0.01, 0.01], [0.05, 0.05, 0.05]]
    alpha = [0.01, 0.01, 0.5, 0.5]
    kept, _, _ = oracle_mod.prepare_scene(means, quats, scales, alpha, alpha_f=0.05, extent_f=0.1)
    assert list(kept) == [1, 2, 3]   # only the low-opacity AND large splat goes
    kept, _, _ = oracle_mod.prepare_scene(means, quats, scales, alpha)
    assert list(kept) == [0, 1, 2, 3]


def test_raw_mode_equals_activated(oracle_mod):
    rng = np.random.default_rng(71)
    q, s, o = common_attrs(rng, 50)
    m = rng.uniform(size=(50, 3)).astype(np.float32)
    log_s = np.log(s.astype(np.float64)).astype(np.float32)
    logit = np.log(o.astype(np.float64) / (1 - o.astype(np.float64))).astype(np.float32)
    k1, mu1, sg1 = oracle_mod.prepare_scene(m, q, s, o, alpha_f=0.3, extent_f=0.03)
    k2, mu2, sg2 = oracle_mod.prepare_scene(m, q, log_s, logit, raw_mode=True, alpha_f=0.3, extent_f=0.03)
    assert np.array_equal(k1, k2)
    assert np.allclose(sg1, sg2, rtol=1e-6)


@pytest.mark.parametrize("bad", ["zero_quat", "nan_mean", "neg_scale", "inf_quat"])
def test_invalid_scene_rejected(oracle_mod, bad):
    m = np.zeros((2, 3), np.float32)
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (2, 1))
    s = np.full((2, 3), 0.03, np.float32)
    o = np.full(2, 0.5, np.float32)
    if bad == "zero_quat":
        q[1] = 0
    elif bad == "nan_mean":
        m[0, 1] = np.nan
    elif bad == "neg_scale":
        s[1, 2] = -0.01
    else:
        q[0, 2] = np.inf
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.prepare_scene(m, q, s, o)


# --- O5: ellipsoidal bodies at n_sigma = 0 are point-in-ellipsoid tests ------

def test_ellipsoid_point_membership(oracle_mod):
    sc = _random_scene(3000, seed=81)
    rng = np.random.default_rng(82)
    nq = 50
    c = rng.uniform(0.2, 0.8, (nq, 3))
    R_E = Rotation.random(nq, random_state=83).as_matrix()
    axes = rng.uniform(0.03, 0.2, (nq, 3))
    _, mu, sig = oracle_mod.prepare_scene(sc.means, sc.quats, sc.scales, sc.opacity)
    out = oracle_mod.evaluate(mu, sig, c, oracle_mod.ellipsoid_bodies(R_E, axes), [0.0])
    for j in range(nq):
        body = (mu - c[j]) @ R_E[j]          # body-frame coordinates
        inside = ((body / axes[j]) ** 2).sum(1) < 1.0
        assert out["count"][j, 0] == inside.sum()
    # a sphere written as an ellipsoid is the sphere
    sph = oracle_mod.evaluate(mu, sig, c, oracle_mod.ellipsoid_bodies(R_E, np.full((nq, 3), 0.1)), [1.0])
    ref = oracle_mod.evaluate(mu, sig, c, oracle_mod.sphere_bodies(np.full(nq, 0.1)), [1.0])
    assert np.array_equal(sph["count"], ref["count"])
    assert np.allclose(sph["min"], ref["min"], rtol=1e-12)


def test_body_quaternion_matches_library_rotation(oracle_mod):
    """Body frames: (w, x, y, z) of any nonzero norm, against scipy's rotation
    (scalar-last convention)."""
    rng = np.random.default_rng(84)
    q = rng.normal(size=(40, 4)) * rng.uniform(0.1, 5.0, (40, 1))
    R = oracle_mod.quat_to_rot(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    assert np.allclose(R, ref, atol=1e-14)
    assert np.allclose(oracle_mod.quat_to_rot(-q), R, atol=1e-14)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.quat_to_rot([[0.0, 0.0, 0.0, 0.0]])


def test_ellipsoid_bodies_from_quaternions_membership(oracle_mod):
    """n_sigma = 0: the count is the number of means strictly inside the body,
    tested in the body frame built by scipy from the same quaternion."""
    from workloads import random_ellipsoids
    sc = _random_scene(3000, seed=85)
    bodies = random_ellipsoids(40, seed=86, box=(1, 1, 1), axis_range=(0.03, 0.25))
    out = oracle_mod.evaluate_ellipsoids(sc, bodies, [0.0])
    mu = sc.means.astype(np.float64)
    for j in range(bodies.q):
        w, x, y, z = bodies.quats[j].astype(np.float64)
        Rj = Rotation.from_quat([x, y, z, w]).as_matrix()
        local = (mu - bodies.centers[j].astype(np.float64)) @ Rj   # body-frame coordinates
        inside = ((local / bodies.axes[j].astype(np.float64)) ** 2).sum(1) < 1.0
        assert out["count"][j, 0] == inside.sum()


def test_ellipsoid_principal_axis_closed_form(oracle_mod):
    """Sigma = s^2 I and d along the body's local axis k at distance rho:
    s^2 = rho^2 / a_k^2, sqrt(sigma^2) = 2 s rho / a_k^2, so collision iff
    rho < n s + sqrt(n^2 s^2 + a_k^2)."""
    from workloads import Bodies
    rng = np.random.default_rng(87)
    s = float(np.float32(0.02))
    for trial in range(4):
        quat = rng.normal(size=4)
        axes = rng.uniform(0.05, 0.3, 3)
        w, x, y, z = quat
        Rb = Rotation.from_quat([x, y, z, w]).as_matrix()
        for k in range(3):
            for n in (0.0, 1.0, 2.5):
                rho = n * s + math.sqrt(n * n * s * s + axes[k] ** 2)
                for fac, want in ((1 - 1e-7, 1), (1 + 1e-7, 0)):
                    c = -Rb[:, k] * rho * fac      # the mean sits at +rho along local axis k
                    sc = _scene([[0, 0, 0]], [[1, 0, 0, 0]], [[s, s, s]])
                    b = Bodies(c[None].astype(np.float64), quat[None], axes[None])
                    out = oracle_mod.evaluate_ellipsoids(sc, b, [n])
                    assert out["count"][0, 0] == want, (trial, k, n, fac)
                b = Bodies(-Rb[:, k][None] * 0.03, quat[None], axes[None])
                out = oracle_mod.evaluate_ellipsoids(sc, b, [n])
                ref = max(0.0, (0.03 ** 2 - 2 * n * s * 0.03) / axes[k] ** 2)
                assert abs(out["min"][0, 0] - ref) <= 1e-12 * max(1.0, ref)


# --- Brute force on tiny isotropic scenes, per-pair closed form --------------

def test_isotropic_scene_brute_force(oracle_mod):
    rng = np.random.default_rng(91)
    n, nq = 400, 60
    m = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    s_iso = rng.uniform(0.005, 0.06, n).astype(np.float32)
    sc = Scene(m, rng.normal(size=(n, 4)).astype(np.float32), np.repeat(s_iso[:, None], 3, 1),
               np.full(n, 0.9, np.float32))
    qs = uniform_queries(nq, seed=92, box=(1, 1, 1), radius=0.09)
    ns = [0.0, 1.0, 2.0]
    out = oracle_mod.evaluate_spheres(sc, qs, ns, k=1)
    rho = np.linalg.norm(m.astype(np.float64)[None] - qs.centers.astype(np.float64)[:, None], axis=2)
    r = qs.radii.astype(np.float64)[:, None]
    s64 = s_iso.astype(np.float64)[None]
    for v, nv in enumerate(ns):
        thr = nv * s64 + np.sqrt(nv * nv * s64 * s64 + r * r)
        assert np.array_equal(out["count"][:, v], (rho < thr).sum(1))
        val = np.maximum(0.0, (rho * rho - 2 * nv * s64 * rho) / (r * r)).min(1)
        assert np.allclose(out["min"][:, v], val, rtol=1e-12, atol=1e-15)


# --- P13: rounding error of the oracle itself (50-digit arithmetic) ---------

def test_oracle_rounding_vs_mpmath(oracle_mod):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(101)
    q, s, o = common_attrs(rng, 8)
    m = rng.uniform(0, 0.3, (8, 3)).astype(np.float32)
    c = np.array([0.1, 0.12, 0.09], np.float32)
    r = np.float32(0.1)
    _, mu, sig = oracle_mod.prepare_scene(m, q, s, o)
    out = oracle_mod.evaluate(mu, sig, c[None].astype(np.float64), oracle_mod.sphere_bodies([r]), [1.3])
    best = None
    for i in range(8):
        w, x, y, z = [mp.mpf(float(v)) for v in q[i]]
        nq = mp.sqrt(w * w + x * x + y * y + z * z)
        w, x, y, z = w / nq, x / nq, y / nq, z / nq
        R = mp.matrix([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                       [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                       [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        S = mp.diag([mp.mpf(float(v)) ** 2 for v in s[i]])
        Sig = R * S * R.T
        d = mp.matrix([mp.mpf(float(m[i, k])) - mp.mpf(float(c[k])) for k in range(3)])
        rr = mp.mpf(float(r))
        s2 = (d.T * d)[0] / rr ** 2
        g = d * (2 / rr ** 2)
        var = (g.T * Sig * g)[0]
        val = max(mp.mpf(0), s2 - mp.mpf(1.3) * mp.sqrt(var))
        best = val if best is None else min(best, val)
    assert abs(out["min"][0, 0] - float(best)) <= 1e-14 * max(1.0, float(best))


# --- tolerance band diagnostics ---------------------------------------------

def test_count_band_brackets_count(oracle_mod):
    sc = _random_scene(2000, seed=111)
    qs = uniform_queries(200, seed=112, box=(1, 1, 1), radius=0.06)
    out = oracle_mod.evaluate_spheres(sc, qs, [1.0], k=2, eps=1e-3)
    assert np.all(out["count_lo"] <= out["count"]) and np.all(out["count"] <= out["count_hi"])
    amb = out["ambiguous"].astype(bool)
    assert np.array_equal(amb, (out["count_lo"] > 2) != (out["count_hi"] > 2))
    # a splat exactly on the isotropic threshold makes its query ambiguous (k = 0)
    s = float(np.float32(0.03))
    r = float(np.float32(0.1))
    rho = s + math.sqrt(s * s + r * r)
    on = _single(oracle_mod, [1, 0, 0, 0], [s, s, s], [rho, 0, 0], r, [1.0], k=0)
    assert on["ambiguous"][0, 0] == 1


def test_strict_threshold_tie_is_free(oracle_mod):
    """s~^2 = 1 exactly (n_sigma = 0, distance = r in exact binary values) is not
    a collision: the test is strict (Sec. II-E)."""
    sc = _scene([[0.0, 0.0, 0.0]], [[1, 0, 0, 0]], [[0.03] * 3])
    qq = Queries(np.array([[0.5, 0.0, 0.0], [0.4375, 0.0, 0.0]], np.float32),
                 np.array([0.5, 0.5], np.float32))
    out = oracle_mod.evaluate_spheres(sc, qq, [0.0], k=0)
    assert out["min"][0, 0] == 1.0 and out["count"][0, 0] == 0
    assert out["count"][1, 0] == 1


def test_ball_band_brackets_ball(oracle_mod):
    sc = _random_scene(3000, seed=121)
    qs = uniform_queries(100, seed=122, box=(1, 1, 1), radius=0.05)
    out = oracle_mod.evaluate_spheres(sc, qs, [1.0], r_nbr=0.3, eps_ball=1e-2)
    d2 = ((sc.means.astype(np.float64)[None] - qs.centers.astype(np.float64)[:, None]) ** 2).sum(2)
    assert np.array_equal(out["nbr"], (d2 <= 0.09).sum(1))
    assert np.array_equal(out["nbr_lo"], (d2 <= 0.09 * (1 - 1e-2)).sum(1))
    assert np.array_equal(out["nbr_hi"], (d2 <= 0.09 * (1 + 1e-2)).sum(1))


# --- Planner epilogues (Sec. II-D Eq. 11, Sec. II-E) ---------------------------

def test_segment_reduce_against_membership_matrix(oracle_mod):
    """Segment OR and sums equal a 0/1 membership matrix applied with a matrix
    product (a library routine), including empty segments."""
    rng = np.random.default_rng(90)
    q, m = 300, 3
    cuts = np.sort(rng.integers(0, q + 1, 40))
    offsets = np.concatenate([[0], cuts, [q]]).astype(np.int64)
    label = (rng.uniform(size=(q, m)) < 0.05).astype(np.uint8)
    cost = rng.uniform(0, 1, (q, m)).astype(np.float32)
    seg_any, seg_sum = oracle_mod.segment_reduce(label, cost, offsets)
    S = np.zeros((offsets.size - 1, q))
    for s_ in range(offsets.size - 1):
        S[s_, offsets[s_]:offsets[s_ + 1]] = 1.0
    assert np.array_equal(seg_any, (S @ label.astype(np.float64) > 0).astype(np.uint8))
    assert np.allclose(seg_sum, S @ cost.astype(np.float64), rtol=1e-14, atol=0)
    # invariants: the segment sums add up to the total; empty segments give 0 and no collision
    assert math.isclose(seg_sum.sum(), cost.astype(np.float64).sum(), rel_tol=1e-13)
    empty = np.diff(offsets) == 0
    assert np.all(seg_sum[empty] == 0) and np.all(seg_any[empty] == 0)


def test_segment_reduce_equal_segments_and_errors(oracle_mod):
    rng = np.random.default_rng(91)
    cost = rng.uniform(size=(64, 2))
    a, s1 = oracle_mod.segment_reduce(cost=cost, n_seg=64)       # one query per segment: identity
    assert np.array_equal(s1, cost)
    _, s8 = oracle_mod.segment_reduce(cost=cost, n_seg=8)
    assert np.allclose(s8, cost.reshape(8, 8, 2).sum(1), rtol=1e-14)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.segment_reduce(cost=cost, n_seg=7)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.segment_reduce(cost=cost, offsets=[0, 40, 30, 64])
