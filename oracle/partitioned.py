"""Oracle: partitioned expansions over user-chosen partitions (Sec. II.A-C).

TEST INFRASTRUCTURE ONLY (see package docstring).  FP64 throughout.

A partition p transects a set of bonds.  Its projector is the product of the
rank-1 BP projectors of those bonds (Eq. (9) with Eq. (11)); in the network's
own gauge the rank-1 projector of a bond is the oblique P_b = a c^T / (a . c)
built from the two fixed-point messages, which is the symmetrised projector of
Appendix B written back in the original gauge.  Bonds that no partition
transects carry the identity.

* ``combinatorial_terms`` writes out Eq. (7): for every non-empty subset x of
  the partitions, the whole network with P_b inserted on every bond
  transected by a partition in x, contracted exactly, with sign + for odd |x|
  and - for even |x|.  Where two partitions of x share a bond, P_b is
  inserted once (P_b P_b = P_b).
* ``linear_terms`` writes out Eq. (4) for single-index partitions taken in the
  given order: term r has Q on the bonds of partitions 0..r-1, P on the bond
  of partition r and the identity elsewhere.
* ``residue`` is Eq. res for single-index partitions: Q on every partitioned
  bond.

Both forms sum to the exact value minus the residue.  The approximation is
that sum (the residue dropped).  Values are returned as (sign, ln|value|)
with one common scale, so that terms of very different size add in FP64
without overflow.

Parity pins (tests): the exact identity Z0 = sum + residue for single-index
partitions, the two forms against each other, the residue of the double-loop
network against its single degree-seven loop term, the multi-index residue
against a brute-force sum over excitation patterns, and the subset count.
"""

from __future__ import annotations

import itertools
import math

import numpy as np

from .pne_oracle import bp_messages, literal_term, projectors


def _scaled_sum(parts):
    """sum_k sgn_k * exp(log_k) * val_k as (sign, ln|sum|), one common scale."""
    parts = [(s, lg, v) for (s, lg, v) in parts if v != 0.0]
    if not parts:
        return 0, -math.inf
    ref = max(lg + math.log(abs(v)) for (_, lg, v) in parts)
    tot = 0.0
    for s, lg, v in parts:
        tot += s * v * math.exp(lg - ref)
    if tot == 0.0:
        return 0, -math.inf
    return (1 if tot > 0 else -1), ref + math.log(abs(tot))


def _term(net, ops):
    ls, t = literal_term(net, ops)
    return ls, float(t)


def _check_partitions(net, partitions):
    parts = [sorted(int(b) for b in p) for p in partitions]
    for p in parts:
        if not p:
            raise ValueError("a partition transects no bond")
        if len(set(p)) != len(p):
            raise ValueError("bond listed twice in one partition")
        if p[0] < 0 or p[-1] >= net.n_bonds:
            raise ValueError("partition bond out of range")
    if net.n_open:
        raise ValueError("closed networks only")
    return parts


def bp_projectors(net, tol=1e-13, max_iter=500):
    """Per bond (P_b, Q_b, n_b) from the fixed-point BP messages."""
    inc, _, _, _ = bp_messages(net, tol, max_iter)
    return projectors(net, inc)


def subsets(n_parts):
    """Non-empty subsets of range(n_parts), as tuples, by size then order."""
    out = []
    for k in range(1, n_parts + 1):
        out.extend(itertools.combinations(range(n_parts), k))
    return out


def combinatorial_terms(net, partitions, proj=None):
    """Eq. (7) without its residue: list of (sign, log_scale, value, subset)."""
    parts = _check_partitions(net, partitions)
    if proj is None:
        proj = bp_projectors(net)
    eye = [np.eye(net.bond_dim(b)) for b in range(net.n_bonds)]
    terms = []
    for x in subsets(len(parts)):
        ops = list(eye)
        for p in x:
            for b in parts[p]:
                ops[b] = proj[b][0]
        ls, v = _term(net, ops)
        terms.append((1 if len(x) % 2 == 1 else -1, ls, v, x))
    return terms


def combinatorial_pne(net, partitions, proj=None):
    """(sign, ln|Z_PNE|): Eq. (7) with the residue dropped."""
    return _scaled_sum([(s, ls, v) for (s, ls, v, _) in combinatorial_terms(net, partitions, proj)])


def linear_pne(net, partitions, proj=None):
    """(sign, ln|Z_PNE|): Eq. (4) with the residue dropped (single-index partitions)."""
    parts = _check_partitions(net, partitions)
    if any(len(p) != 1 for p in parts):
        raise ValueError("the linear form is written for single-index partitions")
    if proj is None:
        proj = bp_projectors(net)
    eye = [np.eye(net.bond_dim(b)) for b in range(net.n_bonds)]
    out = []
    for r in range(len(parts)):
        ops = list(eye)
        for q in range(r):
            ops[parts[q][0]] = proj[parts[q][0]][1]
        ops[parts[r][0]] = proj[parts[r][0]][0]
        ls, v = _term(net, ops)
        out.append((1, ls, v))
    return _scaled_sum(out)


def residue(net, partitions, proj=None):
    """(sign, ln|R|): Q on every bond of single-index partitions (Eq. res)."""
    parts = _check_partitions(net, partitions)
    if any(len(p) != 1 for p in parts):
        raise ValueError("residue written for single-index partitions")
    if proj is None:
        proj = bp_projectors(net)
    ops = [np.eye(net.bond_dim(b)) for b in range(net.n_bonds)]
    for p in parts:
        ops[p[0]] = proj[p[0]][1]
    ls, v = _term(net, ops)
    return _scaled_sum([(1, ls, v)])


def count_retained(net, partitions, K):
    """Brute force over every bond subset: the dangling-free excitation
    patterns (no site with exactly one excited bond) of at most K bonds,
    other than the empty one, that leave some partition with no excited bond.
    With P built from a BP fixed point these are the loop configurations the
    expansion keeps (the others vanish or belong to the residue)."""
    parts = [set(int(b) for b in p) for p in partitions]
    M = net.n_bonds
    ends = [(int(u), int(v)) for (u, _, v, _) in net.bonds]
    count = 0
    for mask in range(1, 1 << M):
        S = [b for b in range(M) if mask >> b & 1]
        if len(S) > K:
            continue
        deg = [0] * net.n_sites
        for b in S:
            deg[ends[b][0]] += 1
            deg[ends[b][1]] += 1
        if any(d == 1 for d in deg):
            continue
        if parts and all(p & set(S) for p in parts):
            continue
        count += 1
    return count


def recursive_pne(net, partitions, subpartitions, proj=None):
    """(sign, ln|Z|): recursive partitioning (Sec. IV.A) written out.

    Eq. (7) over the first-level partitions, except that the term of each
    subset x that `subpartitions` maps (key: tuple of partition indices,
    ascending) to a list of sub-partitions is itself expanded: it becomes the
    combinatorial form, residue dropped, of the network with P on x's bonds,
    over those sub-partitions (P on their bonds as well, the identity
    elsewhere)."""
    parts = _check_partitions(net, partitions)
    subs = {tuple(sorted(k)): _check_partitions(net, v) for k, v in subpartitions.items()}
    if proj is None:
        proj = bp_projectors(net)
    eye = [np.eye(net.bond_dim(b)) for b in range(net.n_bonds)]
    out = []
    for x in subsets(len(parts)):
        sx = 1 if len(x) % 2 == 1 else -1
        base = set(b for p in x for b in parts[p])
        inner = subs.get(tuple(x))
        if not inner:
            ops = [proj[b][0] if b in base else eye[b] for b in range(net.n_bonds)]
            ls, v = _term(net, ops)
            out.append((sx, ls, v))
            continue
        for y in subsets(len(inner)):
            sy = 1 if len(y) % 2 == 1 else -1
            cut = base | set(b for r in y for b in inner[r])
            ops = [proj[b][0] if b in cut else eye[b] for b in range(net.n_bonds)]
            ls, v = _term(net, ops)
            out.append((sx * sy, ls, v))
    return _scaled_sum(out)
