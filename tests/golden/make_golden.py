"""Writes tests/golden/tiny_oracle.json: FP64 oracle outputs for a small seeded
case (400 Gaussians of the uniform-box law, 24 query spheres, three n_sigma
values).  It calls only the oracle and the input generators; the file guards
the oracle against unintended changes of its arithmetic."""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import uniform_box_scene, uniform_queries  # noqa: E402

CASE = dict(n=400, q=24, scene_seed=7, query_seed=8, box=[1.0, 1.0, 1.0], radius=0.1,
            n_sigma=[0.0, 1.0, 2.0], k=1, tau=0.1, r_nbr=0.5, d_max=1.0, gamma=1.0, s_min=1.0)


def compute(case=CASE):
    sc = uniform_box_scene(case["n"], seed=case["scene_seed"], box=case["box"])
    qs = uniform_queries(case["q"], seed=case["query_seed"], box=case["box"], radius=case["radius"])
    out = oracle.evaluate_spheres(sc, qs, case["n_sigma"], k=case["k"], tau=case["tau"],
                                  r_nbr=case["r_nbr"], d_max=case["d_max"], gamma=case["gamma"],
                                  s_min=case["s_min"])
    keys = ("count", "label", "min", "softmin", "cost", "nbr")
    return {k: out[k].tolist() for k in keys}


if __name__ == "__main__":
    res = compute()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_oracle.json")
    with open(path, "w") as f:
        json.dump({"case": CASE, "outputs": res}, f, indent=0, default=lambda x: None if math.isinf(x) else x)
    print("wrote", path)
