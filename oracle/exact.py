"""Exact references for the oracle (never used for GPU parity, only to pin the oracle).

TEST INFRASTRUCTURE ONLY.

* exact_contract: Eq. (1) evaluated by absorbing sites one at a time.
* ising_bruteforce_logz: the Ising partition function summed over all spin
  states, straight from the Boltzmann weights (independent of any tensor
  encoding).
* full_expansion_sum: the complete P/Q expansion, every one of the 2^M
  configurations contracted literally (Eqs. (4)/(7) are regroupings of it).
"""

from __future__ import annotations

import itertools
import math

import numpy as np


def exact_contract(net):
    """Exact contraction (Eq. (1)); returns (log_scale, tensor).

    Z = tensor * exp(log_scale); the tensor has one axis per open leg in the
    network's open-leg order (a 0-d array for a closed network).  Sites are
    absorbed in index order; after each absorption the running tensor is
    rescaled by its largest magnitude to avoid overflow.
    """
    M = net.n_bonds
    leg_label = {}
    for b, (u, lu, v, lv) in enumerate(net.bonds):
        leg_label[(int(u), int(lu))] = b
        leg_label[(int(v), int(lv))] = b
    for k, (s, l) in enumerate(net.open_legs):
        leg_label[(int(s), int(l))] = M + k
    state = np.array(1.0)
    labels = []
    log_scale = 0.0
    for s, t in enumerate(net.tensors):
        tl = [leg_label[(s, l)] for l in range(t.ndim)]
        common = [x for x in labels if x in tl]
        ax_state = [labels.index(x) for x in common]
        ax_t = [tl.index(x) for x in common]
        state = np.tensordot(state, t, axes=(ax_state, ax_t))
        labels = [x for x in labels if x not in common] + [x for x in tl if x not in common]
        m = float(np.max(np.abs(state))) if state.size else 0.0
        if m > 0:
            state = state / m
            log_scale += math.log(m)
    if net.n_open:
        perm = [labels.index(M + k) for k in range(net.n_open)]
        state = np.transpose(state, perm)
    return log_scale, state


def exact_log_contract(net):
    """(sign, ln|Z|) of a closed network by exact contraction."""
    ls, t = exact_contract(net)
    val = float(t)
    if val == 0.0:
        return 0, -math.inf
    return (1 if val > 0 else -1), ls + math.log(abs(val))


def ising_bruteforce_logz(n_sites, pairs, beta, J=1.0):
    """ln sum_{s in {+-1}^N} exp(beta J sum_{(u,v)} s_u s_v), vectorised over states."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    best = -math.inf
    acc = 0.0
    chunk = 1 << min(n_sites, 20)
    total = 1 << n_sites
    logs = []
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        spins = 1 - 2 * ((idx[:, None] >> np.arange(n_sites)[None, :]) & 1)
        e = np.sum(spins[:, pairs[:, 0]] * spins[:, pairs[:, 1]], axis=1)
        x = beta * J * e.astype(np.float64)
        mx = float(x.max())
        logs.append(mx + math.log(float(np.sum(np.exp(x - mx)))))
    del best, acc
    mx = max(logs)
    return mx + math.log(sum(math.exp(l - mx) for l in logs))


def full_expansion_sum(net, proj_pairs, filter_fn=None):
    """Sum of Z(y) over all 2^M configurations y (Q on y, P elsewhere).

    proj_pairs[b] = (P_b, Q_b).  Each term is a literal whole-network
    contraction.  filter_fn(y) may restrict the configurations.  Returns
    (log_scale, tensor) with a common scale.
    """
    from .pne_oracle import literal_term

    M = net.n_bonds
    terms = []
    for bits in itertools.product((0, 1), repeat=M):
        y = tuple(b for b in range(M) if bits[b])
        if filter_fn is not None and not filter_fn(y):
            continue
        ops = [proj_pairs[b][1] if bits[b] else proj_pairs[b][0] for b in range(M)]
        terms.append(literal_term(net, ops))
    if not terms:
        return 0.0, np.array(0.0)
    ref = max(ls for ls, _ in terms)
    total = sum(t * math.exp(ls - ref) for ls, t in terms)
    return ref, np.asarray(total)
