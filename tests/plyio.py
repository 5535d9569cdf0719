"""Writes PLY scene files in the trainers' layout, for the loader tests."""
import numpy as np


def write_gaussian_ply(path, means, quats, log_scales, opacity_logit, sh_rest=45, fmt="binary_little_endian",
                       dtype="float", extra_before=0, faces=0, drop=()):
    """3DGS layout: x y z nx ny nz f_dc_0..2 f_rest_* opacity scale_* rot_0..3.
    log_scales may have 2 columns (2DGS).  dtype: PLY scalar type of every
    property.  extra_before: an element of that many fixed-size records before
    the vertices; faces: a list element after them.  drop: property names left out."""
    n = means.shape[0]
    npdt = {"float": "<f4", "double": "<f8"}[dtype]
    cols = [("x", means[:, 0]), ("y", means[:, 1]), ("z", means[:, 2])]
    cols += [(f"n{a}", np.zeros(n)) for a in "xyz"]
    cols += [(f"f_dc_{i}", np.full(n, 0.5)) for i in range(3)]
    cols += [(f"f_rest_{i}", np.zeros(n)) for i in range(sh_rest)]
    cols += [("opacity", opacity_logit)]
    cols += [(f"scale_{i}", log_scales[:, i]) for i in range(log_scales.shape[1])]
    cols += [(f"rot_{i}", quats[:, i]) for i in range(4)]
    cols = [(k, v) for k, v in cols if k not in drop]
    head = ["ply", f"format {fmt} 1.0", "comment written by the csplat tests"]
    if extra_before:
        head += [f"element camera {extra_before}", "property float cx", "property uchar tag"]
    head += [f"element vertex {n}"] + [f"property {dtype} {k}" for k, _ in cols]
    if faces:
        head += [f"element face {faces}", "property list uchar int vertex_indices"]
    head += ["end_header"]
    with open(path, "wb") as f:
        f.write(("\n".join(head) + "\n").encode())
        if fmt != "binary_little_endian":
            return
        if extra_before:
            rec = np.zeros(extra_before, dtype=[("cx", "<f4"), ("tag", "u1")])
            f.write(rec.tobytes())
        arr = np.zeros(n, dtype=[(k, npdt) for k, _ in cols])
        for k, v in cols:
            arr[k] = v
        f.write(arr.tobytes())
        for _ in range(faces):
            f.write(np.array([3], "u1").tobytes() + np.array([0, 1, 2], "<i4").tobytes())
