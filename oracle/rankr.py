"""Oracle: rank-r projectors from weight passing (Sec. V, Appendix C).

TEST INFRASTRUCTURE ONLY (see package docstring).  FP64 throughout.

Weight passing keeps a diagonal weight S_b on every bond, initially the
identity, and repeats sweeps over the bonds.  For a bond b joining leg lu of
site u (tensor A) and leg lv of site v (tensor B):

* A' is A with the weights of all its other bonds multiplied onto their legs,
  read as a matrix (other legs) x (leg lu); its SVD A' = U_A S_A V_A^T.
* B' likewise, read as (leg lv) x (other legs); its SVD B' = U_B S_B V_B^T.
* S_A V_A^T diag(S_b) U_B S_B = U_C S_C V_C^T (Eq. (C2)).
* A <- A x_lu (V_A S_A^-1 U_C S_C^((1-a)/2)), B <- (S_C^((1-a)/2) V_C^T
  S_B^-1 U_B^T) x_lv B, S_b <- S_C^a (Eq. (C3)): a pure change of gauge
  of the network with its weights.
* The new weight is rescaled to a largest entry of 1, the scale carried in a
  log-factor of the network value.

The exponent a ramps linearly from a / ramp to a over the first `ramp`
sweeps (the paper's annealing remark), then stays at a.  Sweeps stop when no
weight entry changed by more than tol.

With the weights sorted in decreasing order (the SVD order), the rank-r
projector of bond b is P_b = diag(1, .., 1, 0, ..) on its first r indices,
Q_b = I - P_b.  A term of the expansion contracts the gauged network with
diag(S_b) P_b, diag(S_b) Q_b or diag(S_b) on each bond.

Parity pins (tests): the network value is unchanged by weight passing; rank
r = chi gives P = I and the exact value; the expansion forms plus their
residue are exact; Ising below the critical temperature gets a large error
at rank 1 and a small one at rank 2 (Sec. V.B).
"""

from __future__ import annotations

import math

import numpy as np

from .exact import exact_contract
from .partitioned import _scaled_sum, subsets


def _svd(M):
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    return U, s, Vt


def _other_weighted(T, leg, weights_of_legs):
    out = T
    for l, w in enumerate(weights_of_legs):
        if l == leg or w is None:
            continue
        shape = [1] * T.ndim
        shape[l] = len(w)
        out = out * w.reshape(shape)
    return out


def weight_passing(net, alpha=0.8, ramp=10, tol=1e-12, max_sweeps=2000):
    """Returns (tensors, weights, log_scale, sweeps, converged)."""
    T = [np.array(t, dtype=np.float64) for t in net.tensors]
    bonds = [tuple(int(x) for x in b) for b in net.bonds]
    S = [np.ones(T[u].shape[lu]) for (u, lu, _, _) in bonds]
    leg_bond = {}
    for b, (u, lu, v, lv) in enumerate(bonds):
        leg_bond[(u, lu)] = b
        leg_bond[(v, lv)] = b
    log_scale = 0.0

    def weights_of(site):
        return [S[leg_bond[(site, l)]] if (site, l) in leg_bond else None for l in range(T[site].ndim)]

    for sweep in range(1, max_sweeps + 1):
        a = alpha * min(1.0, sweep / ramp) if ramp > 0 else alpha
        change = 0.0
        for b, (u, lu, v, lv) in enumerate(bonds):
            A, B = T[u], T[v]
            Ap = np.moveaxis(_other_weighted(A, lu, weights_of(u)), lu, -1)
            Bp = np.moveaxis(_other_weighted(B, lv, weights_of(v)), lv, 0)
            chi = A.shape[lu]
            _, sA, VAt = _svd(Ap.reshape(-1, chi))
            UB, sB, _ = _svd(Bp.reshape(chi, -1))
            M = (sA[:, None] * VAt) @ np.diag(S[b]) @ (UB * sB[None, :])
            UC, sC, VCt = _svd(M)
            WA = VAt.T @ np.diag(1.0 / sA) @ UC @ np.diag(sC ** ((1 - a) / 2))
            WB = np.diag(sC ** ((1 - a) / 2)) @ VCt @ np.diag(1.0 / sB) @ UB.T
            T[u] = np.moveaxis(np.tensordot(A, WA, axes=([lu], [0])), -1, lu)
            T[v] = np.moveaxis(np.tensordot(WB, B, axes=([1], [lv])), 0, lv)
            new = sC ** a
            m = float(new.max())
            log_scale += math.log(m)
            new = new / m
            change = max(change, float(np.abs(new - S[b]).max()))
            S[b] = new
        if change <= tol and sweep >= ramp:
            return T, S, log_scale, sweep, True
    return T, S, log_scale, max_sweeps, False


def _contract(net, T, ops):
    """(log, value) of the gauged network with a diagonal operator per bond."""
    from pne_inputs import Network

    tens = list(T)
    for b, (u, lu, _, _) in enumerate(net.bonds):
        u, lu = int(u), int(lu)
        shape = [1] * tens[u].ndim
        shape[lu] = len(ops[b])
        tens[u] = tens[u] * ops[b].reshape(shape)
    ls, t = exact_contract(Network(tens, net.bonds, net.open_legs))
    return ls, float(t)


def rank_expansion(net, partitions, r, form="combinatorial", wp=None, **wp_kw):
    """(sign, ln|Z|) of the partitioned expansion with rank-r weight-passing
    projectors, the residue dropped: Eq. (7) over the partitions, or Eq. (4)
    (single-index partitions, in the given order)."""
    if wp is None:
        wp = weight_passing(net, **wp_kw)
    T, S, log_scale = wp[0], wp[1], wp[2]
    parts = [sorted(int(b) for b in p) for p in partitions]
    P = [np.where(np.arange(len(s)) < r, s, 0.0) for s in S]
    Q = [np.where(np.arange(len(s)) < r, 0.0, s) for s in S]
    out = []
    if form == "combinatorial":
        for x in subsets(len(parts)):
            ops = list(S)
            for p in x:
                for b in parts[p]:
                    ops[b] = P[b]
            ls, v = _contract(net, T, ops)
            out.append((1 if len(x) % 2 == 1 else -1, ls + log_scale, v))
    else:
        for k in range(len(parts)):
            ops = list(S)
            for q in range(k):
                ops[parts[q][0]] = Q[parts[q][0]]
            ops[parts[k][0]] = P[parts[k][0]]
            ls, v = _contract(net, T, ops)
            out.append((1, ls + log_scale, v))
    return _scaled_sum(out)


def gauged_value(net, wp):
    """(sign, ln|Z|) of the gauged network with its weights (equals Z0)."""
    T, S, log_scale = wp[0], wp[1], wp[2]
    ls, v = _contract(net, T, S)
    return _scaled_sum([(1, ls + log_scale, v)])
