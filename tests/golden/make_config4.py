"""Write the oracle's outputs for a set of serving requests (K=6, FP64).

The requests cover the shapes of the serving mix that are hardest to check
live: 3D lattices with rank-6 sites at D = 4 (L = 4, 5, 8) and D = 3 (L = 8),
and large 2D lattices (L = 17, 30, 31).  Calls only the CPU oracle and the
input generators; run from the repo root:
    python tests/golden/make_config4.py
Output: tests/golden/config4_oracle.json, one entry per request index.
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import pne_inputs as P  # noqa: E402

# request index -> (dim, L, D, dist): 45 (3, 4, 4, normal), 47 (3, 4, 4, uniform),
# 104 (3, 5, 4, uniform), 4 (3, 8, 4, uniform), 34 (3, 8, 3, normal),
# 2 (2, 17, 2, normal), 19 (2, 30, 3, uniform), 62 (2, 31, 4, uniform)
REQUESTS = [45, 47, 104, 4, 34, 2, 19, 62]


def main():
    out = {}
    for i in REQUESTS:
        net = P.config4_request(i)
        r = O.pne_contract(net, 6)
        out[str(i)] = {
            "name": net.name,
            "sign": r.sign,
            "log_abs": r.log_abs,
            "log_abs_bp": r.log_abs_bp,
            "bp_iters": r.bp_iters,
            "n_clusters": r.n_clusters,
            "n_configs": r.n_configs,
            "dangling_max": r.dangling_max,
        }
        print(i, net.name, r.log_abs, r.bp_iters, r.n_clusters, flush=True)
    path = os.path.join(ROOT, "tests", "golden", "config4_oracle.json")
    with open(path, "w") as f:
        json.dump({"workload": "serving requests 40000+i (see pne_inputs.config4_request); K=6; FP64 oracle",
                   "results": out}, f, indent=1)


if __name__ == "__main__":
    main()
