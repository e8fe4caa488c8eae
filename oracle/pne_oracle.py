"""Oracle: the loop-truncated partitioned network expansion, written out plainly.

TEST INFRASTRUCTURE ONLY (see package docstring).  FP64 throughout.

What is computed (paper Sec. II and III):

* Every bond is its own single-index partition with P_b + Q_b = I (Eq. (2)).
  P_b is the rank-1 projector built from the two fixed-point BP messages on
  the bond (Eq. (8)).  With a_b the message arriving at the bond's first site
  u and c_b the one arriving at its second site v, the oblique form
  P_b = a_b c_b^T / (a_b . c_b) is the symmetrised projector of Appendix B
  written back in the original gauge, so no SVD is needed here.
* The complete P/Q expansion over all bonds is the sum over configurations y
  (the set of bonds carrying Q) of Z(y), the network with Q on y and P
  elsewhere (Eqs. (4)/(7) are regroupings of this sum).
* Retained terms: configurations of degree |y| <= K without dangling
  excitations (a site with exactly one excited bond), which vanish at a BP
  fixed point (Sec. III.A-B).  Sites with open legs are exempt from the
  dangling rule (Sec. III.D).
* Because P factorises its bond, Z(y) is the product of the BP-capped
  untouched sites, the factors 1/(a_b . c_b) of the P bonds, and one
  contraction per connected component of y with Q_b inserted explicitly.

Parity pins (tests): brute-force Ising sums and the high-temperature closed
form (configs with Ising tensors), the complete-expansion identity against
exact contraction for arbitrary projectors, the dangling-free identity at a
fixed point, ring/tree special cases, gauge invariance and cluster counts.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import _enum


# ----------------------------------------------------------------------------
# message passing (Sec. II.B; open legs reflected as in Sec. III.D)


def _partners(net):
    """Map each (site, leg) slot to the slot that receives its outgoing message."""
    partner = {}
    for (u, lu, v, lv) in net.bonds:
        u, lu, v, lv = int(u), int(lu), int(v), int(lv)
        if (u, lu) in partner or (v, lv) in partner:
            raise ValueError("leg used twice")
        if u == v:
            raise ValueError("bond joins a site to itself")
        if net.tensors[u].shape[lu] != net.tensors[v].shape[lv]:
            raise ValueError("bond dimension mismatch")
        partner[(u, lu)] = (v, lv)
        partner[(v, lv)] = (u, lu)
    for (s, l) in net.open_legs:
        s, l = int(s), int(l)
        if (s, l) in partner:
            raise ValueError("open leg also bonded")
        partner[(s, l)] = (s, l)  # reflection: incoming := outgoing
    for s, t in enumerate(net.tensors):
        for l in range(t.ndim):
            if (s, l) not in partner:
                raise ValueError(f"leg {l} of site {s} is neither bonded nor open")
    return partner


def _contract_except(t, msgs, keep):
    """Contract every leg of t except `keep` with its message (last leg first)."""
    out = t
    for l in range(t.ndim - 1, -1, -1):
        if l != keep:
            out = np.tensordot(out, msgs[l], axes=([l], [0]))
    return out


def bp_messages(net, tol=1e-13, max_iter=500, damping=0.0, stall=50):
    """Jacobi BP from uniform messages.

    Every directed message starts at 1/sqrt(d).  A sweep recomputes every
    outgoing message from the previous sweep's incoming messages, scales it
    to unit 2-norm and flips its sign so that its entries sum to >= 0.  The
    residual is the largest sign-insensitive infinity-norm change over all
    messages; sweeps stop once it is <= tol or after max_iter sweeps.

    Rounding floor (not part of the paper's method): with stall > 0, sweeps
    also stop, as converged, once `stall` sweeps in a row have not lowered
    the smallest residual so far and that residual is <= 100 * tol.  A
    residual that no longer decreases has reached the rounding noise of the
    messages, which an ill-conditioned bond gauge can lift above tol.

    Damping (not part of the paper's method; 0 by default): with
    0 <= damping < 1 the stored message is the mix
    (1 - damping) * m_new + damping * m_old of the normalised update and the
    same directed message of the previous sweep, normalised and sign-fixed
    again; the residual then compares the stored message with m_old.

    Returns (inc, iters, residual, converged), where inc[s][l] is the message
    arriving at leg l of site s.
    """
    if not (0.0 <= damping < 1.0):
        raise ValueError("damping must be in [0, 1)")
    partner = _partners(net)
    T = net.tensors
    inc = [[np.full(d, 1.0 / math.sqrt(d)) for d in t.shape] for t in T]
    residual = math.inf
    iters = 0
    best, best_at = math.inf, 0
    for it in range(1, max_iter + 1):
        new = [[None] * t.ndim for t in T]
        for s, t in enumerate(T):
            for l in range(t.ndim):
                m = np.asarray(_contract_except(t, inc[s], l), dtype=np.float64)
                nrm = float(np.sqrt(np.sum(m * m)))
                if not (nrm > 0.0) or not np.isfinite(nrm):
                    raise FloatingPointError(f"zero or non-finite message at site {s} leg {l}")
                m = m / nrm
                if m.sum() < 0:
                    m = -m
                s2, l2 = partner[(s, l)]
                if damping > 0.0:
                    m = (1.0 - damping) * m + damping * inc[s2][l2]
                    nrm = float(np.sqrt(np.sum(m * m)))
                    if not (nrm > 0.0) or not np.isfinite(nrm):
                        raise FloatingPointError(f"zero damped message at site {s} leg {l}")
                    m = m / nrm
                    if m.sum() < 0:
                        m = -m
                new[s2][l2] = m
        residual = 0.0
        for s, t in enumerate(T):
            for l in range(t.ndim):
                d1 = float(np.max(np.abs(new[s][l] - inc[s][l])))
                d2 = float(np.max(np.abs(new[s][l] + inc[s][l])))
                residual = max(residual, min(d1, d2))
        inc = new
        iters = it
        if residual <= tol:
            return inc, iters, residual, True
        if residual < best:
            best, best_at = residual, it
        elif stall > 0 and best <= 100.0 * tol and it - best_at >= stall:
            return inc, iters, residual, True
    return inc, iters, residual, False


# ----------------------------------------------------------------------------
# projectors (Eqs. (2), (8) and Appendix B in oblique form)


def projectors(net, inc):
    """Per bond: (P_b, Q_b, n_b) with P_b = a c^T / n_b, Q_b = I - P_b."""
    out = []
    for (u, lu, v, lv) in net.bonds:
        a = inc[int(u)][int(lu)]
        c = inc[int(v)][int(lv)]
        n = float(a @ c)
        if abs(n) < 1e-12 * np.linalg.norm(a) * np.linalg.norm(c):
            raise FloatingPointError("singular bond overlap")
        P = np.outer(a, c) / n
        out.append((P, np.eye(len(a)) - P, n))
    return out


def _open_slots(net):
    per_site = {}
    for k, (s, l) in enumerate(net.open_legs):
        per_site.setdefault(int(s), []).append((int(l), k))
    return per_site


def vacuum(net, inc):
    """z_v: site tensor with every bond leg capped by its arriving message.

    Scalars for closed sites; for sites with open legs, a tensor over the open
    legs (in leg order)."""
    open_site = _open_slots(net)
    out = []
    for s, t in enumerate(net.tensors):
        opens = {l for (l, _) in open_site.get(s, [])}
        z = t
        for l in range(t.ndim - 1, -1, -1):
            if l not in opens:
                z = np.tensordot(z, inc[s][l], axes=([l], [0]))
        out.append(np.asarray(z, dtype=np.float64))
    return out


def dangling_max(net, inc):
    """Size of the dropped dangling terms (Sec. III.A-B: a site with a single
    excited bond gives a term that vanishes at a BP fixed point).

    For every bond b = (u, v) with a = the message arriving at u, c = the one
    arriving at v and n = a . c, let y_u (y_v) be the site tensor of u (v)
    with every other leg capped by its arriving message.  The excited part of
    the single-leg term is measured in the excited basis of the symmetrising
    gauge (Appendix B): on the bond's first site the component of y_u
    orthogonal to c, on its second site Q y_v with Q = I - a c^T / n, each
    relative to the site's vacuum value (y_u . a / n, resp. y_v . c):

        d_u = |(I - c c^T / |c|^2) y_u| |n| / |y_u . a|,
        d_v = |y_v - a (c . y_v) / n| / |c . y_v|.

    Returns the largest d over every bond end at a site without open legs
    (0.0 for a network without such bonds).  It is 0 at a BP fixed point,
    where y_u is parallel to c and y_v to a.

    Parity: pinned by the fixed-point zero and by the bound
    |w_{b}| <= d_u d_v on the explicitly contracted single-bond term.
    """
    open_site = _open_slots(net)
    worst = 0.0
    for (u, lu, v, lv) in net.bonds:
        u, lu, v, lv = int(u), int(lu), int(v), int(lv)
        a = inc[u][lu]
        c = inc[v][lv]
        if len(a) < 2:
            continue  # a bond of dimension 1 has no excited index
        n = float(a @ c)
        if u not in open_site:
            y = np.asarray(_contract_except(net.tensors[u], inc[u], lu), dtype=np.float64)
            perp = y - c * (float(c @ y) / float(c @ c))
            worst = max(worst, float(np.linalg.norm(perp)) * abs(n) / abs(float(y @ a)))
        if v not in open_site:
            y = np.asarray(_contract_except(net.tensors[v], inc[v], lv), dtype=np.float64)
            q = y - a * (float(c @ y) / n)
            worst = max(worst, float(np.linalg.norm(q)) / abs(float(c @ y)))
    return worst


# ----------------------------------------------------------------------------
# term enumeration (Sec. III.A-B)


def enumerate_clusters(net, K, full=False):
    """Connected, dangling-free bond sets of size <= K (open sites exempt).

    full=True drops the dangling rule: every connected bond set of size <= K
    (the components of the complete expansion's configurations)."""
    exempt = np.zeros(net.n_sites, np.uint8)
    for (s, _) in net.open_legs:
        exempt[int(s)] = 1
    if full:
        exempt[:] = 1
    if net.n_bonds == 0 or K <= 0:
        return []
    return _enum.enum_clusters(net.n_sites, net.bonds[:, 0], net.bonds[:, 2], exempt, K)


def cluster_sites(net, cluster):
    vs = set()
    for b in cluster:
        vs.add(int(net.bonds[b, 0]))
        vs.add(int(net.bonds[b, 2]))
    return frozenset(vs)


def cluster_weight(net, inc, proj, z, cluster):
    """w_c = Z_c * prod_{b in c} n_b / prod_{closed v in V(c)} z_v.

    Z_c contracts the sites of c, each capped by BP messages on its bonds
    outside c, with Q_b inserted explicitly on every bond of c; open legs of
    the sites in c stay free (output axes in the network's open-leg order).
    """
    open_site = _open_slots(net)
    cl = list(cluster)
    idx = {b: i for i, b in enumerate(cl)}
    verts = sorted(cluster_sites(net, cl))
    n_open = net.n_open
    base_open = 2 * len(cl)
    operands = []
    out_labels = []
    for v in verts:
        t = net.tensors[v]
        labels = [None] * t.ndim
        for b in cl:
            u_, lu, v_, lv = (int(x) for x in net.bonds[b])
            if u_ == v:
                labels[lu] = 2 * idx[b]
            if v_ == v:
                labels[lv] = 2 * idx[b] + 1
        for (l, k) in open_site.get(v, []):
            labels[l] = base_open + k
            out_labels.append(base_open + k)
        # cap the remaining (bond) legs with their arriving messages
        capped = t
        keep = []
        for l in range(t.ndim - 1, -1, -1):
            if labels[l] is None:
                capped = np.tensordot(capped, inc[v][l], axes=([l], [0]))
        keep = [lab for lab in labels if lab is not None]
        operands += [capped, keep]
    for b in cl:
        operands += [proj[b][1], [2 * idx[b], 2 * idx[b] + 1]]
    out_labels.sort()
    Zc = np.einsum(*operands, sorted(out_labels), optimize="greedy")
    scale = 1.0
    for b in cl:
        scale *= proj[b][2]
    for v in verts:
        if v not in open_site:
            scale /= float(z[v])
    return np.asarray(Zc, dtype=np.float64) * scale


def enumerate_collections(clusters, sizes, vsets, K):
    """All non-empty sets of pairwise vertex-disjoint clusters with total size <= K.

    Explicit depth-first listing (no summation identities).  Returns a list
    of tuples of cluster indices.
    """
    order = sorted(range(len(clusters)), key=lambda i: (sizes[i], i))
    res = []

    def dfs(start, used, budget, chosen):
        for pos in range(start, len(order)):
            i = order[pos]
            if sizes[i] > budget:
                break  # sorted by size
            if used & vsets[i]:
                continue
            chosen.append(i)
            res.append(tuple(chosen))
            dfs(pos + 1, used | vsets[i], budget - sizes[i], chosen)
            chosen.pop()

    dfs(0, frozenset(), K, [])
    return res


def cumulant_sum(weights, sizes, vsets, K):
    """Exponentiated (cumulant) form of the retained-term sum.

    With the clusters as polymers, two of them incompatible when they share
    a site, the sum over vertex-disjoint collections is 1 + S =
    sum_collections prod w, and its logarithm is the Mayer cluster series
    ln(1 + S) = sum over ordered tuples of polymers whose incompatibility
    graph is connected, of phi(tuple) / n! prod w (phi = 1 for one polymer,
    -1 for two incompatible ones).  Truncated at total degree K < 3 * the
    smallest cluster, only one- and two-polymer tuples remain:

        F = sum_c w_c - 1/2 sum_{(c, c') incompatible, |c| + |c'| <= K} w_c w_c',

    the ordered pairs including c = c'.  Each term is local, so F is additive
    over disjoint parts of a network; ln Z ~ ln Z_BP + F.
    """
    n = len(weights)
    if n == 0:
        return 0.0
    if 3 * min(sizes) <= K:
        raise ValueError("the second-order cumulant form needs K < 3 * (smallest cluster size)")
    F = 0.0
    for i in range(n):
        F += float(weights[i])
    for i in range(n):
        for j in range(n):
            if sizes[i] + sizes[j] <= K and (i == j or vsets[i] & vsets[j]):
                F -= 0.5 * float(weights[i]) * float(weights[j])
    return F


# ----------------------------------------------------------------------------
# the full evaluation


@dataclass
class OracleResult:
    sign: int
    log_abs: float
    log_abs_bp: float
    bp_iters: int
    bp_residual: float
    converged: bool
    n_clusters: int
    n_configs: int
    open_values: np.ndarray | None = None
    dangling_max: float = 0.0
    clusters: list = field(default_factory=list)
    weights: list = field(default_factory=list)
    inc: list | None = None


def pne_contract(net, K, tol=1e-13, max_iter=500, keep_details=False, mode="loop", damping=0.0, stall=50):
    """Loop-truncated PNE of a closed or open network.

    Closed network: returns (sign, ln|Z|).  Open network: Out = open_values *
    exp(log_abs) with axes in the network's open-leg order.

    mode "loop": configurations of degree <= K without dangling sites (the
    retained terms).  mode "full": every configuration of degree <= K, the
    dangling ones included (closed networks); with K >= n_bonds this is the
    complete expansion of Eqs. (2)-(4), equal to the exact contraction for
    any rank-1 projectors, converged or not.  mode "cumulant": the same
    retained clusters in exponentiated form (see cumulant_sum), closed
    networks.
    """
    if mode not in ("loop", "full", "cumulant"):
        raise ValueError("mode must be 'loop', 'full' or 'cumulant'")
    if mode != "loop" and net.n_open:
        raise ValueError(f"{mode} mode is for closed networks")
    inc, iters, residual, converged = bp_messages(net, tol, max_iter, damping, stall)
    proj = projectors(net, inc)
    z = vacuum(net, inc)
    open_site = _open_slots(net)

    # scale = prod_{closed v} z_v / prod_b n_b, kept as (sign, log)
    log_scale = 0.0
    sign = 1
    for s, zs in enumerate(z):
        if s in open_site:
            continue
        zf = float(zs)
        if zf == 0.0:
            raise FloatingPointError("zero vacuum factor")
        log_scale += math.log(abs(zf))
        sign *= 1 if zf > 0 else -1
    for (_, _, n) in proj:
        log_scale -= math.log(abs(n))
        sign *= 1 if n > 0 else -1

    clusters = enumerate_clusters(net, K, full=(mode == "full"))
    weights = [cluster_weight(net, inc, proj, z, c) for c in clusters]
    sizes = [len(c) for c in clusters]
    vsets = [cluster_sites(net, c) for c in clusters]
    if mode == "cumulant":
        F = cumulant_sum(weights, sizes, vsets, K)
        res = OracleResult(sign=sign, log_abs=log_scale + F, log_abs_bp=log_scale, bp_iters=iters,
                           bp_residual=residual, converged=converged, n_clusters=len(clusters),
                           n_configs=len(clusters))
        res.dangling_max = dangling_max(net, inc)
        if keep_details:
            res.clusters, res.weights, res.inc = clusters, weights, inc
        return res
    colls = enumerate_collections(clusters, sizes, vsets, K)

    if net.n_open == 0:
        S = 0.0
        for col in colls:
            term = 1.0
            for i in col:
                term *= float(weights[i])
            S += term
        total = 1.0 + S
        res = OracleResult(sign=sign * (1 if total > 0 else -1) if total != 0 else 0,
                           log_abs=log_scale + (math.log(abs(total)) if total != 0 else -math.inf),
                           log_abs_bp=log_scale, bp_iters=iters, bp_residual=residual,
                           converged=converged, n_clusters=len(clusters), n_configs=len(colls))
    else:
        n_open = net.n_open
        site_of_leg = [int(s) for (s, _) in net.open_legs]
        open_sites = sorted(open_site)
        # clusters that touch an open site give tensors; others scalars
        touches = [tuple(sorted(set(vsets[i]) & set(open_sites))) for i in range(len(clusters))]
        acc = {(): 1.0}  # key: open-touching clusters in the collection
        for col in colls:
            key = tuple(sorted(i for i in col if touches[i]))
            term = 1.0
            for i in col:
                if not touches[i]:
                    term *= float(weights[i])
            acc[key] = acc.get(key, 0.0) + term
        out = np.zeros([net.tensors[s].shape[l] for (s, l) in net.open_legs])
        for key, scal in acc.items():
            covered = set()
            operands = []
            for i in key:
                labs = sorted(k for k in range(n_open) if site_of_leg[k] in vsets[i])
                operands += [weights[i], labs]
                covered |= set(touches[i])
            for s in open_sites:
                if s not in covered:
                    labs = sorted(k for k in range(n_open) if site_of_leg[k] == s)
                    operands += [z[s], labs]
            out += scal * np.einsum(*operands, list(range(n_open)))
        res = OracleResult(sign=sign, log_abs=log_scale, log_abs_bp=log_scale, bp_iters=iters,
                           bp_residual=residual, converged=converged,
                           n_clusters=len(clusters), n_configs=len(colls),
                           open_values=sign * out)
    res.dangling_max = dangling_max(net, inc)
    if keep_details:
        res.clusters = clusters
        res.weights = weights
        res.inc = inc
    return res


# ----------------------------------------------------------------------------
# literal whole-network terms (definition of Z(o_i, o_j, ...), Sec. II.A)


def literal_term(net, ops):
    """Contract the whole network with operator ops[b][i, j] on every bond b.

    i is the index at the bond's first site, j at its second.  Returns
    (log_scale, tensor) as exact.exact_contract does.
    """
    from .exact import exact_contract

    tensors = [t for t in net.tensors]
    for b, (u, lu, v, lv) in enumerate(net.bonds):
        u, lu = int(u), int(lu)
        t = np.tensordot(tensors[u], ops[b], axes=([lu], [0]))
        tensors[u] = np.moveaxis(t, -1, lu)
    from pne_inputs import Network

    mod = Network(tensors, net.bonds, net.open_legs)
    return exact_contract(mod)
