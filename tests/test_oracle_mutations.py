"""Plant plausible mistakes in the oracle (on the CPU) and check a pin catches each.

Each mutation replaces one oracle function with a subtly wrong variant; the
check recomputes a pinned quantity and asserts it no longer matches.
"""

import math

import numpy as np
import pytest

import oracle as O
import oracle.pne_oracle as PO
import pne_inputs as P


def _pins_hold():
    """True when both identity pins hold for the (possibly mutated) oracle."""
    net = P.random_2d(2, 3, 3, "uniform01", seed=5)
    r = PO.pne_contract(net, net.n_bonds)
    _, le = O.exact_log_contract(net)
    ok1 = abs(r.log_abs - le) < 1e-9
    beta = 0.44
    t = math.tanh(beta)
    ising = P.config1_network(beta)
    r2 = PO.pne_contract(ising, 8)
    ht = 16 * math.log(2) + 24 * math.log(math.cosh(beta)) + math.log(1 + 9 * t ** 4 + 12 * t ** 6 + 50 * t ** 8)
    ok2 = abs(r2.log_abs - ht) < 1e-9
    return ok1 and ok2


def test_unmutated_oracle_passes():
    assert _pins_hold()


def _transposed_projectors(net, inc):
    out = []
    for (u, lu, v, lv) in net.bonds:
        a, c = inc[int(u)][int(lu)], inc[int(v)][int(lv)]
        n = float(a @ c)
        Pm = np.outer(c, a) / n  # operands swapped
        out.append((Pm, np.eye(len(a)) - Pm, n))
    return out


def _wrong_sign_q(net, inc):
    return [(p, p - np.eye(p.shape[0]), n) for (p, q, n) in _ORIG["projectors"](net, inc)]


def _dropped_norm(net, inc):
    return [(p, q, 1.0) for (p, q, n) in _ORIG["projectors"](net, inc)]


def _singles_only(clusters, sizes, vsets, K):
    return [c for c in _ORIG["enumerate_collections"](clusters, sizes, vsets, K) if len(c) == 1]


def _one_sweep(net, tol=1e-13, max_iter=500, damping=0.0, stall=50):
    return _ORIG["bp_messages"](net, tol, 2)


def _index_shift(net, inc, proj, z, cluster):
    w = _ORIG["cluster_weight"](net, inc, proj, z, cluster)
    return w * (1.0 + 1e-3)


_ORIG = {k: getattr(PO, k) for k in ("projectors", "enumerate_collections", "bp_messages", "cluster_weight")}


@pytest.mark.parametrize("name,fn", [
    ("projectors", _transposed_projectors),
    ("projectors", _wrong_sign_q),
    ("projectors", _dropped_norm),
    ("enumerate_collections", _singles_only),
    ("bp_messages", _one_sweep),
    ("cluster_weight", _index_shift),
])
def test_planted_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(PO, name, fn)
    assert not _pins_hold()
