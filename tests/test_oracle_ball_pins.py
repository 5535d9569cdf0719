"""Pins of the oracle's neighbourhood-ball reductions and of its tolerance
magnitudes T*, T_soft and T_cost.

The count, minimum, softmin and cost of a query run over the ball
|mu_i - c_j| <= R_nbr (Sec. II-B: softmin over the neighbouring splats;
Sec. II-D, Eq. 11: cost averaged over the neighbouring splats; Sec. II-E:
the count of splats in collision).  These tests compare the oracle with an
independent vectorised numpy computation (covariances from scipy's rotation,
quadratic forms by einsum, log-sum-exp from scipy, exactly rounded sums from
math.fsum) on scenes built so that the ball excludes colliding and
near-minimum pairs; each scene is checked to be discriminating, i.e. the
plausible mistakes (counting outside the ball, a minimum over all splats,
averaging the cost over every splat) give different answers on it.

T = s^2 + n sqrt(sigma^2) is the magnitude of a pair's metric before the
cancellation of Eq. 8; the parity bars scale with it.  For an isotropic
Gaussian (Sigma = s_g^2 I) and a sphere of radius r at distance rho,
T = (rho^2 + 2 n s_g rho) / r^2 in closed form (the same geometry as the
threshold pin rho* = n s + sqrt(n^2 s^2 + r^2)); the one- and two-Gaussian
cases below fix T*, T_soft and T_cost from it.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import logsumexp

from workloads import Scene, common_attrs

NS = [0.0, 1.0, 2.5]
TAU, D_MAX, GAMMA, S_MIN, K = 0.1, 1.5, 0.7, 1.0, 1


def _unit(rng, n):
    u = rng.normal(size=(n, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _lib_sigma(quats, scales):
    """Sigma = R diag(s^2) R^T with R from scipy (scalar-last quaternions)."""
    q = np.asarray(quats, np.float64)
    R = Rotation.from_quat(np.stack([q[:, 1], q[:, 2], q[:, 3], q[:, 0]], 1)).as_matrix()
    s2 = np.asarray(scales, np.float64) ** 2
    return np.einsum("nik,nk,njk->nij", R, s2, R)


def _body_matrices(n, seed, ellipsoid, r=0.1):
    """Sphere bodies A = I / r^2, or ellipsoids R diag(1/a^2) R^T with R and
    the semi-axes drawn here (scipy rotation)."""
    if not ellipsoid:
        return np.repeat((np.eye(3) / r ** 2)[None], n, 0)
    rng = np.random.default_rng(seed)
    R = Rotation.random(n, random_state=seed).as_matrix()
    ax = rng.uniform(0.05, 0.15, (n, 3))
    return np.einsum("nik,nk,njk->nij", R, 1.0 / ax ** 2, R)


def _brute(mu, sig, centers, A, ns, r_nbr):
    """Every output of the method over the ball, vectorised in float64."""
    d = mu[None, :, :] - centers[:, None, :]                          # (q, n, 3)
    s2 = np.einsum("qni,qij,qnj->qn", d, A, d)                        # Eq. 5
    g = 2.0 * np.einsum("qij,qnj->qni", A, d)                         # gradient of s^2 at X = mu
    var = np.einsum("qni,nij,qnj->qn", g, sig, g)                     # Eq. 7
    inball = (d * d).sum(-1) <= r_nbr * r_nbr
    nq = centers.shape[0]
    out = {k: np.zeros((nq, len(ns))) for k in ("count", "min", "softmin", "cost")}
    out["nbr"] = inball.sum(1)
    st_all = []
    for v, n in enumerate(ns):
        st = np.maximum(0.0, s2 - n * np.sqrt(np.maximum(var, 0.0)))  # Eq. 8
        st_all.append(st)
        out["count"][:, v] = ((st < 1.0) & inball).sum(1)
        out["min"][:, v] = np.where(inball, st, np.inf).min(1)
        for j in range(nq):
            x = st[j][inball[j]]
            if x.size == 0:
                out["softmin"][j, v] = np.inf
                out["cost"][j, v] = 0.0
                continue
            out["softmin"][j, v] = -TAU * logsumexp(-x / TAU)
            terms = D_MAX * np.exp(-GAMMA * np.maximum(x - S_MIN, 0.0))     # Eq. 11
            out["cost"][j, v] = math.fsum(terms.tolist()) / x.size
    return out, st_all, inball


def _ball_scene(seed, nq=16, r_nbr=0.3):
    """Per query: a dozen small Gaussians well inside the ball, and large
    Gaussians just outside it whose variance term makes them collide
    (s~^2 = 0 for n_sigma >= 1) -- they would also be the minimum."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(0.5, 2.5, (nq, 3))
    means, scales = [], []
    for j in range(nq):
        lo = rng.choice([0.04, 0.13])      # some queries with inner collisions, some without
        rho = rng.uniform(lo, 0.95, 12) * r_nbr if lo < 0.1 else rng.uniform(0.45, 0.95, 12) * r_nbr
        means.append(centers[j] + _unit(rng, 12) * rho[:, None])
        scales.append(np.exp(rng.normal(math.log(0.01), 0.3, (12, 3))))
        rho_out = rng.uniform(1.02, 1.2, 3) * r_nbr
        means.append(centers[j] + _unit(rng, 3) * rho_out[:, None])
        scales.append(np.full((3, 3), 0.3))
    means = np.concatenate(means).astype(np.float32)
    scales = np.concatenate(scales).astype(np.float32)
    n = means.shape[0]
    quats = rng.normal(size=(n, 4)).astype(np.float32)
    return (Scene(means, quats, scales, np.full(n, 0.9, np.float32)),
            centers.astype(np.float32).astype(np.float64), r_nbr)


@pytest.mark.parametrize("ellipsoid", [False, True])
@pytest.mark.parametrize("seed", [201, 202])
def test_finite_ball_reductions_brute_force(oracle_mod, ellipsoid, seed):
    sc, centers, r_nbr = _ball_scene(seed)
    _, mu, sig_or = oracle_mod.prepare_scene(sc.means, sc.quats, sc.scales, sc.opacity)
    sig = _lib_sigma(sc.quats, sc.scales)
    A = _body_matrices(centers.shape[0], seed + 7, ellipsoid)
    ref, st_all, inball = _brute(mu, sig, centers, A, NS, r_nbr)
    out = oracle_mod.evaluate(mu, sig_or, centers, A, NS, k=K, tau=TAU, r_nbr=r_nbr, d_max=D_MAX,
                              gamma=GAMMA, s_min=S_MIN)
    assert np.array_equal(out["nbr"], ref["nbr"])
    assert np.array_equal(out["count"], ref["count"].astype(np.int32))
    assert np.array_equal(out["label"], (ref["count"] > K).astype(np.uint8))
    for key in ("min", "softmin", "cost"):
        o, b = out[key], ref[key]
        assert np.array_equal(np.isinf(o), np.isinf(b)), key
        fin = np.isfinite(b)
        assert np.allclose(o[fin], b[fin], rtol=1e-12, atol=1e-14), key

    # the scene is discriminating: each plausible mistake changes some result
    coll = [(st < 1.0) for st in st_all]
    count_all = np.stack([c.sum(1) for c in coll], 1)
    assert np.any(count_all[:, 1:] > ref["count"][:, 1:]), "no colliding pair outside the ball"
    assert np.any((count_all[:, 1:] > K) != (ref["count"][:, 1:] > K)), "ball never decides a label"
    min_all = np.stack([st.min(1) for st in st_all], 1)
    assert np.any(min_all[:, 1:] < ref["min"][:, 1:] - 0.1), "no near-minimum pair outside the ball"
    n_tot = mu.shape[0]
    wrong_cost = ref["cost"] * ref["nbr"][:, None] / n_tot            # averaged over every splat
    assert np.all(np.abs(wrong_cost - ref["cost"]) > 1e-3 * ref["cost"])


def test_finite_ball_count_sqrt_free_form_matches(oracle_mod):
    """The sqrt-free label form (Appendix identity: s~^2 < 1 iff a|a| < n^2 sigma^2,
    a = s^2 - 1) gives the oracle's ball counts on the same scenes."""
    sc, centers, r_nbr = _ball_scene(203)
    _, mu, sig_or = oracle_mod.prepare_scene(sc.means, sc.quats, sc.scales, sc.opacity)
    sig = _lib_sigma(sc.quats, sc.scales)
    A = _body_matrices(centers.shape[0], 0, False)
    d = mu[None] - centers[:, None]
    s2 = np.einsum("qni,qij,qnj->qn", d, A, d)
    g = 2.0 * np.einsum("qij,qnj->qni", A, d)
    var = np.einsum("qni,nij,qnj->qn", g, sig, g)
    inball = (d * d).sum(-1) <= r_nbr * r_nbr
    out = oracle_mod.evaluate(mu, sig_or, centers, A, NS, k=K, r_nbr=r_nbr)
    for v, n in enumerate(NS):
        a = s2 - 1.0
        cnt = ((a * np.abs(a) < n * n * var) & inball).sum(1)
        assert np.array_equal(out["count"][:, v], cnt)


# --- tolerance magnitudes in closed form --------------------------------------

def _iso_case(oracle_mod, rhos, s_gs, r, n, direction=(1.0, 0.0, 0.0), **kw):
    """Isotropic Gaussians (scale s_g) at distances rho along `direction`
    from a sphere query of radius r at the origin."""
    u = np.asarray(direction, np.float64)
    u = u / np.linalg.norm(u)
    means = np.array([u * rh for rh in rhos], np.float64)
    nq = len(rhos)
    sig = np.array([np.eye(3) * s * s for s in s_gs])
    A = (np.eye(3) / r ** 2)[None]
    return oracle_mod.evaluate(means.reshape(nq, 3), sig, np.zeros((1, 3)), A, [n], **kw)


def _T(rho, s_g, r, n):
    return (rho * rho + 2.0 * n * s_g * rho) / (r * r)


def _x(rho, s_g, r, n):
    return max(0.0, (rho * rho - 2.0 * n * s_g * rho) / (r * r))


@pytest.mark.parametrize("rho,s_g,n", [(0.35, 0.05, 1.0), (0.12, 0.01, 2.0), (0.05, 0.08, 1.0), (0.2, 0.0, 0.0)])
def test_tolerance_magnitudes_one_gaussian(oracle_mod, rho, s_g, n):
    r = 0.1
    out = _iso_case(oracle_mod, [rho], [s_g], r, n, tau=0.1, gamma=2.0, d_max=1.0, s_min=1.0)
    T = _T(rho, s_g, r, n)
    assert math.isclose(out["min"][0, 0], _x(rho, s_g, r, n), rel_tol=1e-13, abs_tol=1e-15)
    for key in ("tstar", "tsoft", "tcost"):
        assert math.isclose(out[key][0, 0], max(1.0, T), rel_tol=1e-13), (key, out[key][0, 0], T)


def test_tstar_takes_the_minimising_pair(oracle_mod):
    """Two Gaussians far apart in s~^2: T* is the minimising pair's magnitude,
    not the larger magnitude of the other pair; T_soft and T_cost are the
    softmin- and cost-weighted means of the two magnitudes."""
    r, n, tau, gamma, d_max = 0.1, 1.0, 0.1, 0.2, 2.0
    rho1, s1 = 0.25, 0.02     # x1 = 5.25, T1 = 7.25
    rho2, s2 = 0.9, 0.35      # x2 = 18, T2 = 144
    out = _iso_case(oracle_mod, [rho1, rho2], [s1, s2], r, n, tau=tau, gamma=gamma, d_max=d_max)
    x1, x2 = _x(rho1, s1, r, n), _x(rho2, s2, r, n)
    T1, T2 = _T(rho1, s1, r, n), _T(rho2, s2, r, n)
    assert x1 < x2 and T1 < T2
    assert math.isclose(out["min"][0, 0], x1, rel_tol=1e-13)
    assert math.isclose(out["tstar"][0, 0], T1, rel_tol=1e-13)
    e1, e2 = 1.0, math.exp(-(x2 - x1) / tau)
    assert math.isclose(out["tsoft"][0, 0], max(T1, (e1 * T1 + e2 * T2) / (e1 + e2)), rel_tol=1e-12)
    c1 = d_max * math.exp(-gamma * max(x1 - 1.0, 0.0))
    c2 = d_max * math.exp(-gamma * max(x2 - 1.0, 0.0))
    tc = (c1 * T1 + c2 * T2) / (c1 + c2)
    assert math.isclose(out["tcost"][0, 0], max(1.0, tc), rel_tol=1e-12)
    # the cost weight of the far pair is small but not negligible here: the
    # weighted magnitude differs from both single magnitudes
    assert T1 * 1.01 < tc < T2 * 0.99


def test_tstar_of_tied_pairs_is_the_larger_magnitude(oracle_mod):
    """Two pairs with equal s~^2 (a Gaussian with a variance term and a point
    Gaussian at the distance that gives the same value) but different T:
    either may be the minimiser under rounding, so T* is the larger T."""
    r, n = 0.1, 1.0
    rho1, s1 = 0.3, 0.05
    x1 = _x(rho1, s1, r, n)
    rho2 = math.sqrt(x1) * r       # point Gaussian: x2 = rho2^2 / r^2 = x1
    out = _iso_case(oracle_mod, [rho1, rho2], [s1, 0.0], r, n)
    T1, T2 = _T(rho1, s1, r, n), _T(rho2, 0.0, r, n)
    assert T1 > 1.5 * T2
    assert math.isclose(out["tstar"][0, 0], T1, rel_tol=1e-13)
    # moving the point Gaussian out by 1% breaks the tie: T* is its own T no more
    out2 = _iso_case(oracle_mod, [rho1, rho2 * 0.99], [s1, 0.0], r, n)
    assert math.isclose(out2["tstar"][0, 0], _T(rho2 * 0.99, 0.0, r, n), rel_tol=1e-13)


def test_tolerance_magnitudes_over_the_ball_only(oracle_mod):
    """A pair outside the ball neither sets T* (even when it would be the
    minimiser) nor enters T_soft or T_cost."""
    r, n = 0.1, 1.0
    rho1, s1 = 0.2, 0.01       # inside a 0.5 ball
    rho2, s2 = 0.55, 0.3       # outside it, s~^2 = 0 (it would be the minimiser), T huge
    out = _iso_case(oracle_mod, [rho1, rho2], [s1, s2], r, n, r_nbr=0.5, tau=0.1)
    T1 = _T(rho1, s1, r, n)
    assert _x(rho2, s2, r, n) == 0.0
    for key in ("tstar", "tsoft", "tcost"):
        assert math.isclose(out[key][0, 0], T1, rel_tol=1e-13), key
    assert out["nbr"][0] == 1 and out["count"][0, 0] == 0


def test_empty_ball_magnitudes(oracle_mod):
    out = _iso_case(oracle_mod, [0.8], [0.01], 0.1, 1.0, r_nbr=0.5)
    assert out["nbr"][0] == 0 and math.isinf(out["min"][0, 0]) and out["cost"][0, 0] == 0.0
    for key in ("tstar", "tsoft", "tcost"):
        assert out[key][0, 0] == 1.0


# --- 50-digit arithmetic: softmin and cost over a finite ball -----------------

def test_softmin_and_cost_vs_mpmath(oracle_mod):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(211)
    n = 14
    q, s, o = common_attrs(rng, n)
    c = np.array([0.2, 0.21, 0.19], np.float32)
    m = (c[None] + _unit(rng, n) * rng.uniform(0.03, 0.45, n)[:, None]).astype(np.float32)
    r, ns, r_nbr = np.float32(0.1), 1.3, 0.35
    tau, gamma, d_max, s_min = 0.2, 0.8, 1.7, 1.0
    _, mu, sig = oracle_mod.prepare_scene(m, q, s, o)
    out = oracle_mod.evaluate(mu, sig, c[None].astype(np.float64), oracle_mod.sphere_bodies([r]), [ns],
                              tau=tau, gamma=gamma, d_max=d_max, s_min=s_min, r_nbr=r_nbr)
    vals = []
    for i in range(n):
        w, x, y, z = [mp.mpf(float(v)) for v in q[i]]
        nq = mp.sqrt(w * w + x * x + y * y + z * z)
        w, x, y, z = w / nq, x / nq, y / nq, z / nq
        R = mp.matrix([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                       [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                       [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        Sig = R * mp.diag([mp.mpf(float(v)) ** 2 for v in s[i]]) * R.T
        d = mp.matrix([mp.mpf(float(m[i, k])) - mp.mpf(float(c[k])) for k in range(3)])
        if (d.T * d)[0] > mp.mpf(r_nbr) ** 2:
            continue
        rr = mp.mpf(float(r))
        s2 = (d.T * d)[0] / rr ** 2
        g = d * (2 / rr ** 2)
        vals.append(max(mp.mpf(0), s2 - mp.mpf(ns) * mp.sqrt((g.T * Sig * g)[0])))
    assert 3 <= len(vals) < n          # the ball excludes some splats and keeps several
    soft = -mp.mpf(tau) * mp.log(mp.fsum(mp.exp(-v / mp.mpf(tau)) for v in vals))
    cost = mp.fsum(mp.mpf(d_max) * mp.exp(-mp.mpf(gamma) * max(v - mp.mpf(s_min), 0)) for v in vals) / len(vals)
    assert out["nbr"][0] == len(vals)
    assert abs(out["softmin"][0, 0] - float(soft)) <= 1e-13 * max(1.0, abs(float(soft)))
    assert abs(out["cost"][0, 0] - float(cost)) <= 1e-13 * float(cost)
    assert abs(out["min"][0, 0] - float(min(vals))) <= 1e-14 * max(1.0, float(min(vals)))
