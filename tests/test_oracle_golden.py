"""The oracle reproduces its stored outputs (tests/golden/make_golden.py)."""
import json
import os

import numpy as np


def test_oracle_matches_golden(oracle_mod):
    import importlib.util
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(here, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    with open(os.path.join(here, "golden", "tiny_oracle.json")) as f:
        stored = json.load(f)
    assert stored["case"] == json.loads(json.dumps(mg.CASE))
    now = mg.compute(stored["case"])
    for k in ("count", "label", "nbr"):
        assert np.array_equal(np.asarray(now[k]), np.asarray(stored["outputs"][k])), k
    for k in ("min", "softmin", "cost"):
        a = np.asarray(now[k], float)
        b = np.asarray([[np.inf if v is None else v for v in row] for row in stored["outputs"][k]], float)
        assert np.allclose(a, b, rtol=1e-12, atol=0), k
