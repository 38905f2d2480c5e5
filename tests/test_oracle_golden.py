"""The oracle against its own stored outputs (guards against accidental change)."""
import json
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plain_fp64_gauss.json")


def test_oracle_matches_stored_outputs(ref):
    g = json.load(open(GOLDEN))
    c = W.cfg_plain_fp64()
    nodes = ref.layout_nodes(c["layout"], c["k"])
    assert np.array_equal(nodes, np.array(g["nodes"]))
    r = ref.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], per_path=True)
    # libm may differ by an ulp across hosts: compare to 1e-12, not bitwise
    assert np.max(np.abs(r["mean"] - np.array(g["mean"]))) < 1e-10
    assert np.max(np.abs(r["se"] - np.array(g["se"]))) < 1e-10
    assert abs(r["steps"] - g["steps"]) <= 4
    for p, q in zip(r["per_path"][0, :8], g["node0_paths"]):
        assert abs(p["exit_xi"] - q["exit"][0]) < 1e-12 and abs(p["exit_eta"] - q["exit"][1]) < 1e-12
        assert p["steps"] == q["steps"] and p["side"] == q["side"]
