"""Write the oracle's outputs for the 32x32 D=6 open-index workload (K=8).

Calls only the CPU oracle and the input generators; run from the repo root:
    python tests/golden/make_config5.py
Output: tests/golden/config5_oracle.json, one entry per separation d = 1..8.
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import pne_inputs as P  # noqa: E402


def main():
    out = {}
    for d in range(1, 9):
        net = P.config5_network(d)
        r = O.pne_contract(net, 8)
        out[str(d)] = {
            "log_scale": r.log_abs,
            "values": [[float(x) for x in row] for row in r.open_values],
            "bp_iters": r.bp_iters,
            "n_clusters": r.n_clusters,
            "n_configs": r.n_configs,
        }
        print(d, r.log_abs, r.n_clusters, flush=True)
    path = os.path.join(ROOT, "tests", "golden", "config5_oracle.json")
    with open(path, "w") as f:
        json.dump({"workload": "32x32 open-boundary U[0,1], D=6, open legs (dim 2) at x=12 and x=12+d, y=15; "
                               "seed 5000+d; K=8; FP64 oracle", "results": out}, f, indent=1)


if __name__ == "__main__":
    main()
