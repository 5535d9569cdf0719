"""csplat: the CollisionSplatting robot-versus-3DGS metric on MI355X (gfx950).

A thin ctypes binding of the C ABI in include/csplat.h.  Functions keep the C
names (csplat_ctx_create, csplat_scene_load, csplat_set_conservatism,
csplat_eval, ...); they only marshal arguments.  Every step of the metric runs
in the HIP kernels of libcsplat.so; there is no CPU fallback: importing works
without the library, but every call raises if it is missing.

Device memory and streams come from PyTorch: pass torch CUDA tensors to run
asynchronously on the context's stream (by default torch's current stream),
or numpy arrays to run synchronously through staging buffers.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build (load_library(path) takes another build explicitly)
LIB_PATH = os.path.join(_HERE, "libcsplat.so")

CSPLAT_OK = 0
CSPLAT_E_INVALID = 1
CSPLAT_E_OOM = 2
CSPLAT_E_DEVICE = 3
CSPLAT_E_BUSY = 4
CSPLAT_E_NOT_FOUND = 5
CSPLAT_E_PENDING = 6
CSPLAT_E_CANCELLED = 7
CSPLAT_MAX_M = 8
CSPLAT_PARAM_ACTIVATED = 0
CSPLAT_PARAM_RAW_3DGS = 1
CSPLAT_PRECISION_FP32 = 0
CSPLAT_PRECISION_BF16_RECHECK = 1
CSPLAT_PRECISION_FP16_RECHECK = 2
CSPLAT_FEATURES_BF16 = 1
CSPLAT_FEATURES_FP16 = 2
CSPLAT_FEATURES_ELL_BF16 = 4
CSPLAT_FEATURES_ELL_FP16 = 8

# every symbol declared in include/csplat.h (checked by the test suite)
EXPORTS = (
    "csplat_ctx_create", "csplat_ctx_destroy", "csplat_scene_load", "csplat_scene_info",
    "csplat_scene_free", "csplat_set_conservatism", "csplat_eval", "csplat_eval_labels",
    "csplat_eval_distance", "csplat_eval_ellipsoids", "csplat_ply_read", "csplat_scene_load_ply", "csplat_segment_reduce", "csplat_ctx_set_timing", "csplat_last_stats", "csplat_synchronize",
    "csplat_last_error", "csplat_server_create", "csplat_server_destroy", "csplat_server_add_scene",
    "csplat_server_submit", "csplat_server_poll", "csplat_server_wait", "csplat_server_cancel",
    "csplat_server_stats", "csplat_server_latencies", "csplat_eval_noalloc", "csplat_last_rechecked",
    "csplat_rrt_create", "csplat_rrt_destroy", "csplat_rrt_step", "csplat_rrt_nodes", "csplat_rrt_last_edges",
    "csplat_server_submit_ellipsoids",
)
CSPLAT_SERVE_COST = 0
CSPLAT_SERVE_LABELS = 1


class CsplatError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"csplat error {status}: {msg}")
        self.status = status


class SceneOpts(ctypes.Structure):
    _fields_ = [("param_mode", ctypes.c_int32), ("floater_opacity_max", ctypes.c_float),
                ("floater_extent_min", ctypes.c_float), ("precision_features", ctypes.c_uint32)]


class ReduceOpts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("softmin_tau", ctypes.c_float),
                ("neighbor_radius", ctypes.c_float), ("d_max", ctypes.c_float),
                ("gamma", ctypes.c_float), ("s_min", ctypes.c_float), ("precision", ctypes.c_int32),
                ("cull", ctypes.c_int32)]


class Outputs(ctypes.Structure):
    _fields_ = [("label", ctypes.c_void_p), ("count", ctypes.c_void_p), ("min", ctypes.c_void_p),
                ("softmin", ctypes.c_void_p), ("cost", ctypes.c_void_p), ("nbr", ctypes.c_void_p),
                ("err", ctypes.c_void_p)]


class EvalStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("flagged", ctypes.c_int64),
                ("flagged_fp64", ctypes.c_int64), ("splits", ctypes.c_int32),
                ("queries_per_lane", ctypes.c_int32), ("kernel_pairs", ctypes.c_int64),
                ("kernel_ms", ctypes.c_float), ("workspace_bytes", ctypes.c_uint64),
                ("min_passes", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("refused", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("pairs_per_s", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("shared_steps", ctypes.c_int64), ("max_requests_per_step", ctypes.c_int32)]


_lib = None


def library_loaded() -> bool:
    return _lib is not None


def load_library(path: str = LIB_PATH):
    """Load libcsplat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise CsplatError(-1, f"{path} is missing: build it with paper_2609_35619_amd/build.py")
    # torch first: its HIP runtime must be the one the library binds to (a
    # runtime loaded by the library first makes torch's kernels unlaunchable)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "csplat_ctx_create": [I32, P, P],
        "csplat_ctx_destroy": [P],
        "csplat_scene_load": [P, I64, P, P, P, P, P, P],
        "csplat_ply_read": [ctypes.c_char_p, I64, P, P, P, P, P],
        "csplat_scene_load_ply": [P, ctypes.c_char_p, P, P],
        "csplat_scene_info": [P, P, P],
        "csplat_scene_free": [P],
        "csplat_set_conservatism": [P, P, I32],
        "csplat_eval": [P, P, I64, P, P, P, P],
        "csplat_eval_noalloc": [P, P, I64, P, P, P, P],
        "csplat_eval_labels": [P, P, I64, P, P, P, P, P],
        "csplat_eval_distance": [P, P, I64, P, P, P, P, P, P],
        "csplat_eval_ellipsoids": [P, P, I64, P, P, P, P, P],
        "csplat_segment_reduce": [P, I64, I32, I64, P, P, P, P, P],
        "csplat_ctx_set_timing": [P, I32],
        "csplat_last_stats": [P, P],
        "csplat_last_rechecked": [P, P, I64, P],
        "csplat_rrt_create": [P, P, P, I32, P, P],
        "csplat_rrt_destroy": [P],
        "csplat_rrt_step": [P, I32, P, P],
        "csplat_rrt_nodes": [P, P, P, I32, P],
        "csplat_rrt_last_edges": [P, P, P, P],
        "csplat_synchronize": [P],
        "csplat_server_create": [I32, ctypes.c_uint64, I32, P],
        "csplat_server_destroy": [P],
        "csplat_server_add_scene": [P, P, P],
        "csplat_server_submit": [P, I32, I32, I64, P, P, P, P, I32, P],
        "csplat_server_submit_ellipsoids": [P, I32, I32, I64, P, P, P, P, P, I32, P],
        "csplat_server_poll": [P, ctypes.c_uint64, P],
        "csplat_server_wait": [P, ctypes.c_uint64, P, I64],
        "csplat_server_cancel": [P, ctypes.c_uint64],
        "csplat_server_stats": [P, P],
        "csplat_server_latencies": [P, P, I64, P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    lib.csplat_last_error.argtypes = []
    lib.csplat_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status):
    if status != CSPLAT_OK:
        msg = _lib.csplat_last_error().decode(errors="replace")
        raise CsplatError(status, msg)


def _addr(x):
    """Address of a torch tensor or numpy array (None -> NULL)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    return x.ctypes.data_as(ctypes.c_void_p)


def _is_torch_cuda(x):
    return hasattr(x, "is_cuda") and x.is_cuda


# --- C names ---------------------------------------------------------------

def csplat_ctx_create(device: int = 0, stream=None):
    """Create a context on `device`.  `stream`: a torch.cuda.Stream or a raw
    hipStream_t integer to borrow, or None to let the library own a stream."""
    lib = load_library()
    handle = 0
    if stream is not None:
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    out = ctypes.c_void_p()
    _check(lib.csplat_ctx_create(device, ctypes.c_void_p(handle) if handle else None, ctypes.byref(out)))
    return out


def csplat_ctx_destroy(ctx):
    _check(load_library().csplat_ctx_destroy(ctx))


def csplat_scene_load(ctx, means, quats, scales, opacity, param_mode=CSPLAT_PARAM_ACTIVATED,
                      floater_opacity_max=0.0, floater_extent_min=0.0, precision_features=0):
    lib = load_library()
    arrs = [np.ascontiguousarray(a, np.float32) for a in (means, quats, scales, opacity)]
    n = arrs[0].shape[0]
    opts = SceneOpts(param_mode, floater_opacity_max, floater_extent_min, precision_features)
    out = ctypes.c_void_p()
    _check(lib.csplat_scene_load(ctx, n, *[_addr(a) if n else None for a in arrs], ctypes.byref(opts),
                                 ctypes.byref(out)))
    return out


def csplat_ply_read(path):
    """Parse a 3DGS/2DGS PLY file on the host: (means, quats, scales, opacity),
    activated (linear scales, opacity in [0, 1])."""
    lib = load_library()
    n = ctypes.c_int64()
    p = os.fsencode(path)
    _check(lib.csplat_ply_read(p, 0, ctypes.byref(n), None, None, None, None))
    k = n.value
    arrs = [np.empty((k, 3), np.float32), np.empty((k, 4), np.float32), np.empty((k, 3), np.float32),
            np.empty(k, np.float32)]
    _check(lib.csplat_ply_read(p, k, ctypes.byref(n), *[_addr(a) for a in arrs]))
    return tuple(arrs)


def csplat_scene_load_ply(ctx, path, floater_opacity_max=0.0, floater_extent_min=0.0, precision_features=0):
    opts = SceneOpts(CSPLAT_PARAM_ACTIVATED, floater_opacity_max, floater_extent_min, precision_features)
    out = ctypes.c_void_p()
    _check(load_library().csplat_scene_load_ply(ctx, os.fsencode(path), ctypes.byref(opts), ctypes.byref(out)))
    return out


def csplat_scene_info(scene):
    n = ctypes.c_int64()
    b = ctypes.c_uint64()
    _check(load_library().csplat_scene_info(scene, ctypes.byref(n), ctypes.byref(b)))
    return n.value, b.value


def csplat_scene_free(scene):
    _check(load_library().csplat_scene_free(scene))


def csplat_set_conservatism(ctx, n_sigma):
    ns = np.ascontiguousarray(np.atleast_1d(n_sigma), np.float32)
    _check(load_library().csplat_set_conservatism(ctx, _addr(ns), ns.size))


def reduce_opts(k=0, tau=0.0, r_nbr=math.inf, d_max=1.0, gamma=1.0, s_min=1.0,
                precision=CSPLAT_PRECISION_FP32, cull=1) -> ReduceOpts:
    return ReduceOpts(int(k), float(tau), float(r_nbr), float(d_max), float(gamma), float(s_min),
                      int(precision), int(cull))


def csplat_eval(ctx, scene, centers, radii, opts: ReduceOpts, label=None, count=None, min=None,
                softmin=None, cost=None, nbr=None, err=None):
    """Evaluate into caller-provided outputs (all torch CUDA tensors or all
    numpy arrays, matching centers/radii)."""
    q = int(centers.shape[0])
    o = Outputs(*[_addr(x) for x in (label, count, min, softmin, cost, nbr, err)])
    _check(load_library().csplat_eval(ctx, scene, q, _addr(centers), _addr(radii), ctypes.byref(opts),
                                      ctypes.byref(o)))


CSPLAT_NOALLOC_SCRATCH_MB = 64
CSPLAT_NOALLOC_MAX_Q = 262144


def csplat_eval_noalloc(ctx, scene, centers, radii, opts: ReduceOpts, label=None, count=None, min=None,
                        softmin=None, cost=None, nbr=None):
    """csplat_eval (float32 path) without any allocation: torch CUDA tensors
    only; the workspace is the library's fixed per-GPU scratch array."""
    q = int(centers.shape[0])
    o = Outputs(*[_addr(x) for x in (label, count, min, softmin, cost, nbr)])
    _check(load_library().csplat_eval_noalloc(ctx, scene, q, _addr(centers), _addr(radii), ctypes.byref(opts),
                                              ctypes.byref(o)))


def csplat_eval_labels(ctx, scene, centers, radii, opts: ReduceOpts, label, count=None):
    q = int(centers.shape[0])
    _check(load_library().csplat_eval_labels(ctx, scene, q, _addr(centers), _addr(radii),
                                             ctypes.byref(opts), _addr(label), _addr(count)))


def csplat_eval_distance(ctx, scene, centers, radii, opts: ReduceOpts, min, softmin=None, cost=None):
    q = int(centers.shape[0])
    _check(load_library().csplat_eval_distance(ctx, scene, q, _addr(centers), _addr(radii),
                                               ctypes.byref(opts), _addr(min), _addr(softmin),
                                               _addr(cost)))


def csplat_eval_ellipsoids(ctx, scene, centers, quats, axes, opts: ReduceOpts, label=None, count=None,
                           min=None, softmin=None, cost=None, nbr=None):
    """Ellipsoidal bodies: centres (q x 3), (w, x, y, z) quaternions (q x 4),
    semi-axes (q x 3); outputs as csplat_eval."""
    q = int(centers.shape[0])
    o = Outputs(*[_addr(x) for x in (label, count, min, softmin, cost, nbr)])
    _check(load_library().csplat_eval_ellipsoids(ctx, scene, q, _addr(centers), _addr(quats), _addr(axes),
                                                 ctypes.byref(opts), ctypes.byref(o)))


def csplat_segment_reduce(ctx, n_seg, label=None, cost=None, seg_any=None, seg_cost=None, offsets=None):
    """Segment OR of labels and segment sums of costs (arrays of shape (q, m);
    outputs (n_seg, m)); offsets (n_seg + 1, int64) or None for equal segments."""
    src = label if label is not None else cost
    q, m = int(src.shape[0]), int(src.shape[1])
    _check(load_library().csplat_segment_reduce(ctx, q, m, int(n_seg), _addr(offsets), _addr(label), _addr(cost),
                                                _addr(seg_any), _addr(seg_cost)))


def csplat_ctx_set_timing(ctx, enable: bool):
    _check(load_library().csplat_ctx_set_timing(ctx, 1 if enable else 0))


def csplat_last_stats(ctx) -> dict:
    st = EvalStats()
    _check(load_library().csplat_last_stats(ctx, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in EvalStats._fields_}


def csplat_last_rechecked(ctx) -> np.ndarray:
    """Indices (caller order) of the queries the last precision-form
    evaluation rechecked in fp64."""
    lib = load_library()
    n = ctypes.c_int64(0)
    _check(lib.csplat_last_rechecked(ctx, None, 0, ctypes.byref(n)))
    out = np.zeros(max(int(n.value), 1), np.int32)
    _check(lib.csplat_last_rechecked(ctx, out.ctypes.data_as(ctypes.c_void_p), int(n.value), ctypes.byref(n)))
    return out[:int(n.value)].copy()


class RrtOpts(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float * 3), ("hi", ctypes.c_float * 3), ("step", ctypes.c_float),
                ("resolution", ctypes.c_float), ("n_sigma", ctypes.c_float), ("k", ctypes.c_int32),
                ("n_links", ctypes.c_int32), ("link_offsets", ctypes.c_void_p), ("link_radii", ctypes.c_void_p),
                ("seed", ctypes.c_uint64)]


class Rrt:
    """A GPU-resident batched RRT (Sec. II-E) over a loaded scene: a rigid
    robot of link spheres translating in 3-D."""

    def __init__(self, ctx, scene, lo, hi, step, resolution, n_sigma, k, link_offsets, link_radii, root,
                 max_nodes, seed=0):
        lib = load_library()
        self._off = np.ascontiguousarray(link_offsets, np.float32).reshape(-1, 3)
        self._rad = np.ascontiguousarray(link_radii, np.float32).reshape(-1)
        o = RrtOpts((ctypes.c_float * 3)(*lo), (ctypes.c_float * 3)(*hi), float(step), float(resolution),
                    float(n_sigma), int(k), int(self._rad.size), self._off.ctypes.data_as(ctypes.c_void_p),
                    self._rad.ctypes.data_as(ctypes.c_void_p), int(seed))
        r = np.ascontiguousarray(root, np.float32).reshape(3)
        h = ctypes.c_void_p()
        _check(lib.csplat_rrt_create(ctx, scene, ctypes.byref(o), int(max_nodes), r.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.byref(h)))
        self.h = h
        self.max_nodes = int(max_nodes)

    def step(self, n_batch, samples=None, wait=False):
        """One step; samples: None (drawn on the device) or a torch CUDA
        tensor (n_batch x 3).  With wait, returns the nodes appended."""
        n = ctypes.c_int32(0)
        _check(load_library().csplat_rrt_step(self.h, int(n_batch), _addr(samples),
                                              ctypes.byref(n) if wait else None))
        return int(n.value) if wait else None

    def nodes(self):
        lib = load_library()
        n = ctypes.c_int32(0)
        _check(lib.csplat_rrt_nodes(self.h, None, None, 0, ctypes.byref(n)))
        pos = np.zeros((max(n.value, 1), 3), np.float32)
        par = np.zeros(max(n.value, 1), np.int32)
        _check(lib.csplat_rrt_nodes(self.h, pos.ctypes.data_as(ctypes.c_void_p), par.ctypes.data_as(ctypes.c_void_p),
                                    n.value, ctypes.byref(n)))
        return pos[:n.value].copy(), par[:n.value].copy()

    def last_edges(self, n_batch):
        near = np.zeros(n_batch, np.int32)
        end = np.zeros((n_batch, 3), np.float32)
        valid = np.zeros(n_batch, np.uint8)
        _check(load_library().csplat_rrt_last_edges(self.h, near.ctypes.data_as(ctypes.c_void_p),
                                                    end.ctypes.data_as(ctypes.c_void_p),
                                                    valid.ctypes.data_as(ctypes.c_void_p)))
        return near, end, valid

    def close(self):
        if self.h:
            load_library().csplat_rrt_destroy(self.h)
            self.h = None


def csplat_synchronize(ctx):
    _check(load_library().csplat_synchronize(ctx))


def csplat_last_error() -> str:
    return load_library().csplat_last_error().decode(errors="replace")


def csplat_server_create(device: int, hbm_budget: int, slots: int):
    out = ctypes.c_void_p()
    _check(load_library().csplat_server_create(device, int(hbm_budget), slots, ctypes.byref(out)))
    return out


def csplat_server_destroy(srv):
    _check(load_library().csplat_server_destroy(srv))


def csplat_server_add_scene(srv, scene) -> int:
    sid = ctypes.c_int32()
    _check(load_library().csplat_server_add_scene(srv, scene, ctypes.byref(sid)))
    return sid.value


def csplat_server_submit(srv, scene_id, kind, centers, radii, opts: ReduceOpts, n_sigma) -> int:
    c = np.ascontiguousarray(centers, np.float32)
    r = np.ascontiguousarray(radii, np.float32)
    ns = np.ascontiguousarray(np.atleast_1d(n_sigma), np.float32)
    t = ctypes.c_uint64()
    _check(load_library().csplat_server_submit(srv, scene_id, kind, c.shape[0], _addr(c) if c.size else None,
                                               _addr(r) if r.size else None, ctypes.byref(opts), _addr(ns),
                                               ns.size, ctypes.byref(t)))
    return t.value


def csplat_server_submit_ellipsoids(srv, scene_id, kind, centers, quats, axes, opts: ReduceOpts, n_sigma) -> int:
    """Ellipsoidal bodies (host arrays: centres q x 3, quaternions q x 4,
    semi-axes q x 3); otherwise as csplat_server_submit."""
    c = np.ascontiguousarray(centers, np.float32)
    qt = np.ascontiguousarray(quats, np.float32)
    ax = np.ascontiguousarray(axes, np.float32)
    ns = np.ascontiguousarray(np.atleast_1d(n_sigma), np.float32)
    t = ctypes.c_uint64()
    nz = c.shape[0] > 0
    _check(load_library().csplat_server_submit_ellipsoids(srv, scene_id, kind, c.shape[0], _addr(c) if nz else None,
                                                          _addr(qt) if nz else None, _addr(ax) if nz else None,
                                                          ctypes.byref(opts), _addr(ns), ns.size, ctypes.byref(t)))
    return t.value


def _server_outputs(q, kind):
    keys = ALL_OUTPUTS if kind == CSPLAT_SERVE_COST else ("label", "count")
    shapes = dict(label=np.uint8, count=np.int32, min=np.float32, softmin=np.float32, cost=np.float32,
                  nbr=np.int32)
    out = {k: np.empty((q, 1) if k != "nbr" else (q,), shapes[k]) for k in keys}
    return out, Outputs(*[_addr(out.get(k)) for k in ALL_OUTPUTS])


def csplat_server_poll(srv, ticket, q, kind):
    """Returns the outputs dict when done, None while pending."""
    out, o = _server_outputs(q, kind)
    st = load_library().csplat_server_poll(srv, ticket, ctypes.byref(o))
    if st == CSPLAT_E_PENDING:
        return None
    _check(st)
    return out


def csplat_server_wait(srv, ticket, q, kind, timeout_ms=-1):
    out, o = _server_outputs(q, kind)
    st = load_library().csplat_server_wait(srv, ticket, ctypes.byref(o), int(timeout_ms))
    if st == CSPLAT_E_PENDING:
        return None
    _check(st)
    return out


def csplat_server_cancel(srv, ticket):
    _check(load_library().csplat_server_cancel(srv, ticket))


def csplat_server_stats(srv) -> dict:
    st = ServerStats()
    _check(load_library().csplat_server_stats(srv, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in ServerStats._fields_}


def csplat_server_latencies(srv) -> np.ndarray:
    """Latencies in ms of the completed requests, in completion order."""
    lib = load_library()
    n = ctypes.c_int64(0)
    _check(lib.csplat_server_latencies(srv, None, 0, ctypes.byref(n)))
    out = np.zeros(max(n.value, 1), np.float64)
    _check(lib.csplat_server_latencies(srv, out.ctypes.data_as(ctypes.c_void_p), out.size, ctypes.byref(n)))
    return out[:min(n.value, out.size)].copy()


# --- convenience ------------------------------------------------------------

ALL_OUTPUTS = ("label", "count", "min", "softmin", "cost", "nbr")


class Engine:
    """One context on its own torch stream + its conservatism values.

    Evaluations on torch tensors are ordered after the work already queued on
    torch's current stream, and torch's current stream waits for them, so the
    results can be used like any other torch tensor."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.ctx = csplat_ctx_create(device, self.stream)
        self.m = 1

    def close(self):
        if self.ctx is not None:
            csplat_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def load_scene(self, scene, **kw):
        return csplat_scene_load(self.ctx, scene.means, scene.quats, scene.scales, scene.opacity, **kw)

    def set_conservatism(self, n_sigma):
        csplat_set_conservatism(self.ctx, n_sigma)
        self.m = int(np.atleast_1d(n_sigma).size)

    def alloc_outputs(self, q, want=ALL_OUTPUTS, like="cuda"):
        """Output buffers: torch CUDA tensors (like="cuda") or numpy arrays."""
        m = self.m
        shapes = dict(label=((q, m), "u8"), count=((q, m), "i32"), min=((q, m), "f32"),
                      softmin=((q, m), "f32"), cost=((q, m), "f32"), nbr=((q,), "i32"), err=((q, m), "f32"))
        out = {}
        if like == "cuda":
            import torch
            dt = dict(u8=torch.uint8, i32=torch.int32, f32=torch.float32)
            for k in want:
                s, t = shapes[k]
                out[k] = torch.empty(s, dtype=dt[t], device=f"cuda:{self.device}")
        else:
            dt = dict(u8=np.uint8, i32=np.int32, f32=np.float32)
            for k in want:
                s, t = shapes[k]
                out[k] = np.empty(s, dtype=dt[t])
        return out

    def evaluate(self, scene, centers, radii, opts: ReduceOpts, want=ALL_OUTPUTS, out=None):
        like = "cuda" if _is_torch_cuda(centers) else "host"
        if out is None:
            out = self.alloc_outputs(int(centers.shape[0]), want, like)
        if like == "cuda":
            cur = self.torch.cuda.current_stream(self.device)
            self.stream.wait_stream(cur)
            for t in (centers, radii, *out.values()):
                t.record_stream(self.stream)
        csplat_eval(self.ctx, scene, centers, radii, opts, **out)
        if like == "cuda":
            self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def evaluate_ellipsoids(self, scene, centers, quats, axes, opts: ReduceOpts, want=ALL_OUTPUTS, out=None):
        """Ellipsoidal bodies (arrays all torch CUDA tensors or all numpy)."""
        like = "cuda" if _is_torch_cuda(centers) else "host"
        if out is None:
            out = self.alloc_outputs(int(centers.shape[0]), want, like)
        if like == "cuda":
            cur = self.torch.cuda.current_stream(self.device)
            self.stream.wait_stream(cur)
            for t in (centers, quats, axes, *out.values()):
                t.record_stream(self.stream)
        csplat_eval_ellipsoids(self.ctx, scene, centers, quats, axes, opts, **out)
        if like == "cuda":
            self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def stats(self):
        return csplat_last_stats(self.ctx)

    def synchronize(self):
        csplat_synchronize(self.ctx)
