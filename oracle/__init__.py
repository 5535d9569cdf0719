"""FP64 CPU oracle of the CollisionSplatting metric — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It wraps `oracle.c` (plain C + OpenMP,
double precision) with ctypes and numpy; it shares nothing with the HIP
library.  See `oracle.c` for the definition and its citations of the paper.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_HDR = os.path.join(_HERE, "oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Reduce(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("tau", ctypes.c_double), ("r_nbr", ctypes.c_double),
                ("d_max", ctypes.c_double), ("gamma", ctypes.c_double),
                ("s_min", ctypes.c_double), ("eps", ctypes.c_double),
                ("eps_ball", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or \
                os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_prepare_scene.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_double, P, P, P, P]
        lib.oracle_prepare_scene.restype = ctypes.c_int
        lib.oracle_eval.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64, P, P, ctypes.c_int32,
                                    P, ctypes.POINTER(_Reduce)] + [P] * 14 + [ctypes.c_int]
        lib.oracle_eval.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def prepare_scene(means, quats, scales, opacity, raw_mode=False, alpha_f=0.0, extent_f=0.0):
    """Returns (kept_index, mu (n,3) f64, sigma (n,3,3) f64)."""
    lib = _load()
    means = np.ascontiguousarray(means, np.float32)
    quats = np.ascontiguousarray(quats, np.float32)
    scales = np.ascontiguousarray(scales, np.float32)
    opacity = np.ascontiguousarray(opacity, np.float32)
    n = means.shape[0]
    kept = np.empty(n, np.int64)
    mu = np.empty((max(n, 1), 3), np.float64)
    sig = np.empty((max(n, 1), 9), np.float64)
    nk = ctypes.c_int64(0)
    rc = lib.oracle_prepare_scene(n, _ptr(means), _ptr(quats), _ptr(scales), _ptr(opacity),
                                  int(bool(raw_mode)), float(alpha_f), float(extent_f),
                                  ctypes.byref(nk), _ptr(kept), _ptr(mu), _ptr(sig))
    if rc != 0:
        raise OracleError(f"oracle_prepare_scene failed ({rc})")
    k = nk.value
    return kept[:k].copy(), mu[:k].copy(), sig[:k].reshape(k, 3, 3).copy()


def sphere_bodies(radii):
    """A_j = I / r_j^2 (Eq. 6 with a = b = c = r), in double precision."""
    r = np.asarray(radii, np.float64)
    A = np.zeros((r.size, 3, 3))
    inv = 1.0 / (r * r)
    A[:, 0, 0] = inv
    A[:, 1, 1] = inv
    A[:, 2, 2] = inv
    return A


def ellipsoid_bodies(rot, semi_axes):
    """A_j = R_E diag(1/a^2, 1/b^2, 1/c^2) R_E^T (Eq. 5-6)."""
    rot = np.asarray(rot, np.float64)
    ax = np.asarray(semi_axes, np.float64)
    P = np.zeros(ax.shape[:-1] + (3, 3))
    for k in range(3):
        P[..., k, k] = 1.0 / (ax[..., k] ** 2)
    return rot @ P @ np.swapaxes(rot, -1, -2)


def quat_to_rot(quats):
    """Rotation matrices of (w, x, y, z) quaternions of any nonzero norm
    (normalised first), the Hamilton convention of 3DGS (Sec. II-A), in double
    precision."""
    qv = np.asarray(quats, np.float64).reshape(-1, 4)
    nrm = np.linalg.norm(qv, axis=1)
    if np.any(~np.isfinite(nrm)) or np.any(nrm == 0):
        raise OracleError("quaternions must be finite and nonzero")
    w, x, y, z = (qv / nrm[:, None]).T
    R = np.empty((qv.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def evaluate(mu, sigma, centers, A, n_sigma, k=0, tau=0.0, r_nbr=math.inf, d_max=1.0,
             gamma=1.0, s_min=1.0, eps=1e-5, eps_ball=1e-6, nthreads=0):
    """Evaluate all outputs.  Returns a dict of (q, m) arrays plus `nbr` (q,)."""
    lib = _load()
    mu = np.ascontiguousarray(mu, np.float64).reshape(-1, 3)
    sigma = np.ascontiguousarray(sigma, np.float64).reshape(-1, 9)
    centers = np.ascontiguousarray(centers, np.float64).reshape(-1, 3)
    A = np.ascontiguousarray(A, np.float64).reshape(-1, 9)
    ns = np.ascontiguousarray(np.atleast_1d(n_sigma), np.float64)
    n, q, m = mu.shape[0], centers.shape[0], ns.size
    if A.shape[0] != q:
        raise ValueError("one body matrix per query")
    out = dict(count=np.zeros((q, m), np.int32), label=np.zeros((q, m), np.uint8),
               min=np.zeros((q, m)), softmin=np.zeros((q, m)), cost=np.zeros((q, m)),
               nbr=np.zeros(q, np.int64), nbr_lo=np.zeros(q, np.int64),
               nbr_hi=np.zeros(q, np.int64), count_lo=np.zeros((q, m), np.int32),
               count_hi=np.zeros((q, m), np.int32), ambiguous=np.zeros((q, m), np.uint8),
               tstar=np.zeros((q, m)), tsoft=np.zeros((q, m)), tcost=np.zeros((q, m)))
    red = _Reduce(int(k), float(tau), float(r_nbr), float(d_max), float(gamma), float(s_min),
                  float(eps), float(eps_ball))
    rc = lib.oracle_eval(n, _ptr(mu), _ptr(sigma), q, _ptr(centers), _ptr(A), m, _ptr(ns),
                         ctypes.byref(red), _ptr(out["count"]), _ptr(out["label"]),
                         _ptr(out["min"]), _ptr(out["softmin"]), _ptr(out["cost"]),
                         _ptr(out["nbr"]), _ptr(out["nbr_lo"]), _ptr(out["nbr_hi"]),
                         _ptr(out["count_lo"]), _ptr(out["count_hi"]),
                         _ptr(out["ambiguous"]), _ptr(out["tstar"]), _ptr(out["tsoft"]),
                         _ptr(out["tcost"]), int(nthreads))
    if rc != 0:
        raise OracleError(f"oracle_eval failed ({rc})")
    return out


def segment_reduce(label=None, cost=None, offsets=None, n_seg=None):
    """Planner epilogues over segments of consecutive queries: an RRT state or
    edge is in collision when any of its bodies is (Sec. II-E); an MPPI
    rollout's collision cost sums its per-body costs over links and horizon
    (Sec. II-D, Eq. 11).  Segment s is queries offsets[s]:offsets[s+1]
    (offsets None: n_seg equal segments).  Returns (seg_any uint8 (n_seg, m),
    seg_sum float64 (n_seg, m)), exactly rounded sums (math.fsum)."""
    src = label if label is not None else cost
    q, m = np.asarray(src).shape
    if offsets is None:
        if n_seg is None or (n_seg > 0 and q % n_seg) or (n_seg == 0 and q):
            raise OracleError("equal segments need q to be a multiple of n_seg")
        offsets = np.arange(n_seg + 1, dtype=np.int64) * (q // n_seg if n_seg else 0)
    offsets = np.asarray(offsets, np.int64)
    if offsets[0] != 0 or offsets[-1] != q or np.any(np.diff(offsets) < 0):
        raise OracleError("offsets must rise from 0 to q")
    ns = offsets.size - 1
    seg_any = np.zeros((ns, m), np.uint8)
    seg_sum = np.zeros((ns, m), np.float64)
    for s_ in range(ns):
        a, b = int(offsets[s_]), int(offsets[s_ + 1])
        for v in range(m):
            if label is not None:
                seg_any[s_, v] = 1 if any(int(x) != 0 for x in np.asarray(label)[a:b, v]) else 0
            if cost is not None:
                seg_sum[s_, v] = math.fsum(float(x) for x in np.asarray(cost)[a:b, v])
    return seg_any, seg_sum


def evaluate_ellipsoids(scene, bodies, n_sigma, raw_mode=False, alpha_f=0.0, extent_f=0.0, **reduce):
    """Convenience: float32 scene against ellipsoidal bodies (centre, (w,x,y,z)
    quaternion of the body frame, semi-axes along its local x, y, z), with
    A_j = R_j diag(1/a^2, 1/b^2, 1/c^2) R_j^T (Eq. 5-6)."""
    _, mu, sig = prepare_scene(scene.means, scene.quats, scene.scales, scene.opacity,
                               raw_mode=raw_mode, alpha_f=alpha_f, extent_f=extent_f)
    A = ellipsoid_bodies(quat_to_rot(bodies.quats), bodies.axes)
    return evaluate(mu, sig, bodies.centers.astype(np.float64), A, n_sigma, **reduce)


def evaluate_spheres(scene, queries, n_sigma, raw_mode=False, alpha_f=0.0, extent_f=0.0,
                     **reduce):
    """Convenience: prepare a float32 scene and evaluate float32 query spheres."""
    _, mu, sig = prepare_scene(scene.means, scene.quats, scene.scales, scene.opacity,
                               raw_mode=raw_mode, alpha_f=alpha_f, extent_f=extent_f)
    return evaluate(mu, sig, queries.centers.astype(np.float64), sphere_bodies(queries.radii),
                    n_sigma, **reduce)


def rrt_step(mu, sigma, nodes, parents, samples, link_offsets, link_radii, step, resolution, n_sigma, k,
             max_nodes, eps=1e-5):
    """One batched RRT step (Sec. II-E) in float64.  For each sample: the
    nearest tree node (Euclidean, the lowest index among equal distances), the
    edge from it toward the sample of length at most `step`, the edge's states
    at n_strides = ceil(step / resolution) (the float32 quotient) evenly spaced points (the node
    excluded, the end included), each state placing the robot's link spheres
    (a rigid template: the state plus each link's offset), and the label of
    every sphere (more than k Gaussians with s~^2 < 1, every kept Gaussian).
    An edge is kept when no state is in collision and its length is positive;
    kept edges' ends are appended in batch order while room remains.

    Returns a dict: nearest (B,), ties (B, list of node indices within eps of
    the nearest distance), end (B, 3), length (B,), valid (B,), ambiguous (B,:
    some sphere of the edge is ambiguous for the label), nodes, parents (the
    grown tree)."""
    nodes = np.asarray(nodes, np.float64).reshape(-1, 3)
    parents = np.asarray(parents, np.int64).reshape(-1)
    smp = np.asarray(samples, np.float64).reshape(-1, 3)
    off = np.asarray(link_offsets, np.float64).reshape(-1, 3)
    rad = np.asarray(link_radii, np.float64).reshape(-1)
    B, L = smp.shape[0], rad.size
    d2 = ((smp[:, None, :] - nodes[None, :, :]) ** 2).sum(-1)
    nearest = np.argmin(d2, axis=1)                     # the first of equal minima
    dmin = d2[np.arange(B), nearest]
    ties = [np.nonzero(d2[b] <= dmin[b] * (1 + eps) + 1e-30)[0].tolist() for b in range(B)]
    base = nodes[nearest]
    dv = smp - base
    d = np.linalg.norm(dv, axis=1)
    f = np.where(d > step, step / np.where(d > 0, d, 1.0), 1.0)
    end = base + dv * f[:, None]
    length = d * f
    # the count of checks per edge from the float32 parameters, as the ABI
    # takes them (the ceiling of their float32 quotient)
    T = max(1, int(math.ceil(float(np.float32(step) / np.float32(resolution)))))
    w = np.arange(1, T + 1, dtype=np.float64) / T
    states = base[:, None, :] + w[None, :, None] * (end - base)[:, None, :]        # (B, T, 3)
    centers = (states[:, :, None, :] + off[None, None, :, :]).reshape(-1, 3)      # (B * T * L, 3)
    radii = np.broadcast_to(rad[None, None, :], (B, T, L)).reshape(-1)
    out = evaluate(mu, sigma, centers, sphere_bodies(radii), [n_sigma], k=k, eps=eps)
    lab = out["label"][:, 0].reshape(B, T * L)
    amb = out["ambiguous"][:, 0].reshape(B, T * L)
    valid = (length > 0) & ~lab.any(axis=1)
    new_nodes, new_par = [nodes], [parents]
    n = nodes.shape[0]
    for b in range(B):
        if valid[b] and n < max_nodes:
            new_nodes.append(end[b][None])
            new_par.append(np.array([nearest[b]]))
            n += 1
    return dict(nearest=nearest, ties=ties, end=end, length=length, valid=valid, ambiguous=amb.any(axis=1),
                nodes=np.concatenate(new_nodes), parents=np.concatenate(new_par), n_strides=T)
