"""Write the stored oracle outputs of this folder (calls only oracle/)."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def plain_fp64_gauss():
    c = workloads.cfg_plain_fp64()
    nodes = oracle.layout_nodes(c["layout"], c["k"])
    r = oracle.interface_estimate(c["density"], c["bmap"], nodes, c["paths"], c["dt"], c["seed"], per_path=True)
    pp = r["per_path"][0, :8]
    return {
        "workload": c["name"], "paths": c["paths"], "dt": c["dt"], "seed": c["seed"],
        "nodes": nodes.tolist(), "mean": r["mean"].tolist(), "se": r["se"].tolist(),
        "steps": r["steps"], "capped": r["capped"],
        "node0_paths": [{"exit": [float(p["exit_xi"]), float(p["exit_eta"])], "steps": int(p["steps"]),
                         "side": int(p["side"])} for p in pp],
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "plain_fp64_gauss.json"), "w") as f:
        json.dump(plain_fp64_gauss(), f, indent=1)
