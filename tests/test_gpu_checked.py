"""The checked build (libpne_checked.so, PNE_CHECKED=1): every cluster kernel
path with its index checks compiled in, against the plain build.

Each index of the cluster kernels (entry tables, LDS frontier, slices,
weights) is tested against its extent; a failed test suppresses the access
and reports PNE_ERR_CHECK for the network.  The workloads below drive each
path (frontier plans with and without entry tables, open outputs, cycles of
leg dimension 2 to 5, scalar products): every network must come back with
the plain build's status and bitwise the same value, in a process of its own
that loads the checked library.
"""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
assert torch.cuda.is_available()
import numpy as np
import paper_2512_10910_amd as pne, pne_inputs as P
ctx = pne.Context(0)
out = {"lib": pne.LIB_PATH}
def run(name, raws, K, prec="fp64", parts=None, **kw):
    nets = [ctx.network(x) for x in raws]
    if parts is not None:
        for x, n in zip(raws, nets):
            pp = parts(x)
            ps, subs = pp if isinstance(pp, tuple) else (pp, {})
            n.set_partitions(ps)
            for sx, inner in subs.items():
                n.set_subpartitions(sx, inner)
    b = ctx.batch(nets, K=K, precision=prec, **kw)
    r = b.run_arrays()
    ov = [b.open_values(i) for i in range(len(nets))]
    out[name] = {"status": [int(v) for v in r["status"]], "sign": [int(v) for v in r["sign"]],
                 "log_abs": [float(v).hex() for v in r["log_abs"]],
                 "open": [None if v is None else [float(x).hex() for x in np.ravel(v)] for v in ov]}
run("recursive_3x4", [P.small_network(3, 4, "random", 4, seed=70000 + i) for i in range(16)], 17,
    parts=P.grid3x4_recursive_partitions)
run("grid3_multi", [P.small_network(3, 3, "random", 4, seed=50000 + i) for i in range(16)], 12,
    parts=P.grid3_multi_partitions)
run("open_4x4_fp32", [P.random_2d(4, 4, 3, "uniform01", seed=30 + i, open_sites={5: 2, 6: 2}) for i in range(8)],
    6, "fp32")
run("aklt_4x4_launch", [P.aklt_2d(4, 4)] * 4, 8, persistent=False)
run("ising_4x4_launch", [P.ising_2d(4, 4, 0.3 + 0.01 * i) for i in range(8)], 4, persistent=False)
run("rand_d6_cycles", [P.random_2d(3, 3, 6, "uniform01", seed=90 + i) for i in range(8)], 4, "fp32",
    persistent=False)
run("rand_d3_cycles", [P.random_2d(4, 4, 3, "uniform01", seed=95 + i) for i in range(8)], 6, "bf16",
    persistent=False)
print("RESULT " + json.dumps(out), flush=True)
'''


def _run(checked: bool):
    env = dict(os.environ)
    env["PNE_CHECKED"] = "1" if checked else "0"
    p = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], env=env, capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-2000:]
    line = [x for x in p.stdout.splitlines() if x.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_checked_build_matches_plain_build():
    plain = _run(False)
    checked = _run(True)
    assert plain["lib"].endswith("libpne.so") and checked["lib"].endswith("libpne_checked.so")
    for name, a in plain.items():
        if name == "lib":
            continue
        b = checked[name]
        print(name, "status", b["status"][:4], flush=True)
        assert all(s >= 0 for s in b["status"]), (name, b["status"])
        assert a == b, name
