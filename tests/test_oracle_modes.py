"""Pins of the oracle's complete-expansion mode, its dangling-term measure and
BP damping, against what the mathematics fixes:

* the complete P/Q expansion (Eqs. (2)-(4)) reproduces the exact contraction
  for any rank-1 projectors, also from BP messages that have not converged;
* truncated to degree <= K it equals the sum of literal whole-network terms
  Z(y) over |y| <= K (a different computation: no cluster factorisation);
* the dangling measure vanishes at a BP fixed point (Sec. III.A-B), bounds
  every single-bond term by Cauchy-Schwarz and ignores the tensors' scale;
* damped BP reaches the undamped fixed point, and on a two-site ring its
  residual shrinks at the rate the linearised update predicts.
"""

import itertools
import math

import numpy as np
import pytest

import oracle as O
import pne_inputs as P


def _comb_count(M, K):
    return sum(math.comb(M, k) for k in range(1, K + 1))


@pytest.mark.parametrize("shape,D,dist,seed,iters", [
    ((3, 3), 3, "normal", 21, 2),
    ((3, 3), 2, "uniform01", 5, 3),
    ((2, 4), 3, ("uniform", -0.8, 1.2), 6, 1),
])
def test_full_mode_complete_expansion_is_exact(shape, D, dist, seed, iters):
    net = P.random_2d(shape[0], shape[1], D, dist, seed=seed)
    M = net.n_bonds
    r = O.pne_contract(net, M, max_iter=iters, mode="full")
    assert not r.converged
    s, le = O.exact_log_contract(net)
    assert r.sign == s
    assert abs(r.log_abs - le) < 1e-11
    assert r.n_configs == 2 ** M - 1
    # the dangling-free (loop) sum misses the dangling terms away from a fixed point
    loop = O.pne_contract(net, M, max_iter=iters)
    assert abs(loop.log_abs - le) > 1e-9


@pytest.mark.parametrize("K", [2, 3, 5])
def test_full_mode_truncated_equals_literal_terms(K):
    net = P.random_2d(2, 3, 3, "normal", seed=13)
    inc, _, _, _ = O.bp_messages(net, max_iter=2)
    proj = O.projectors(net, inc)
    pairs = [(p[0], p[1]) for p in proj]
    ls, tot = O.full_expansion_sum(net, pairs, filter_fn=lambda y: len(y) <= K)
    r = O.pne_contract(net, K, max_iter=2, mode="full")
    val = float(tot) * math.exp(ls - r.log_abs)
    assert abs(abs(val) - 1.0) < 1e-11 and np.sign(val) == r.sign
    assert r.n_configs == _comb_count(net.n_bonds, K)


def test_full_mode_rejects_open_networks():
    net = P.random_2d(3, 3, 2, "uniform01", seed=3, open_sites={4: 2})
    with pytest.raises(ValueError):
        O.pne_contract(net, 4, mode="full")


def test_dangling_measure_vanishes_at_fixed_point():
    net = P.random_2d(4, 4, 3, "normal", seed=31)
    r = O.pne_contract(net, 4)
    assert r.converged and r.dangling_max < 1e-11
    early = O.pne_contract(net, 4, max_iter=2)
    assert early.dangling_max > 1e-4
    # Ising at the paramagnetic point: BP is exact after one sweep
    assert O.pne_contract(P.ising_2d(3, 3, 0.4), 4).dangling_max < 1e-13


@pytest.mark.parametrize("iters", [1, 2, 4])
def test_dangling_measure_bounds_single_bond_terms(iters):
    net = P.random_2d(3, 4, 3, "uniform01", seed=17)
    inc, _, _, _ = O.bp_messages(net, max_iter=iters)
    proj = O.projectors(net, inc)
    z = O.vacuum(net, inc)
    d = O.dangling_max(net, inc)
    worst = max(abs(float(O.cluster_weight(net, inc, proj, z, [b]))) for b in range(net.n_bonds))
    assert worst > 0.0
    assert worst <= d * d * (1 + 1e-9)


def test_dangling_measure_ignores_tensor_scale():
    net = P.random_2d(3, 3, 3, "normal", seed=19)
    inc, _, _, _ = O.bp_messages(net, max_iter=2)
    d0 = O.dangling_max(net, inc)
    scaled = P.Network([t * (3.0 + s) for s, t in enumerate(net.tensors)], net.bonds, net.open_legs)
    inc2, _, _, _ = O.bp_messages(scaled, max_iter=2)
    assert abs(O.dangling_max(scaled, inc2) - d0) < 1e-12 * max(1.0, d0)


@pytest.mark.parametrize("lam", [0.3, 0.7])
def test_damped_bp_reaches_the_undamped_fixed_point(lam):
    net = P.random_2d(3, 4, 3, "uniform01", seed=23)
    a = O.pne_contract(net, 6, keep_details=True)
    b = O.pne_contract(net, 6, keep_details=True, damping=lam)
    assert a.converged and b.converged and b.bp_iters > a.bp_iters
    worst = max(float(np.max(np.abs(x - y))) for ra, rb in zip(a.inc, b.inc) for x, y in zip(ra, rb))
    assert worst < 1e-11
    assert abs(a.log_abs - b.log_abs) < 1e-12


def test_damped_bp_rate_on_two_site_ring():
    """Two sites joined by two bonds (matrices A, B): each of the two message
    chains is a power iteration of AB, whose linearised Jacobi sweep has
    eigenvalues +-sqrt(rho), rho = lambda_2 / lambda_1.  Damping by lam turns
    them into (1 - lam)(+-sqrt(rho)) + lam, so the residual shrinks by
    (1 - lam) sqrt(rho) + lam per sweep (by rho per two sweeps undamped)."""
    rng = np.random.default_rng(5)

    def spd():
        x = rng.random((2, 2))
        return x @ x.T + 0.3 * np.eye(2)

    A, B = spd(), spd()
    net = P.ring_network([A, B])
    ev = np.sort(np.linalg.eigvals(A @ B).real)[::-1]
    rho = ev[1] / ev[0]
    assert 0.05 < rho < 0.6
    res0 = [O.bp_messages(net, tol=0.0, max_iter=t)[2] for t in range(1, 16)]
    assert abs(res0[12] / res0[10] - rho) < 1e-4 * rho
    for lam in (0.4, 0.6):
        pred = (1.0 - lam) * math.sqrt(rho) + lam
        # sweeps until the residual is ~1e-8: the linear regime, far from rounding
        t = int(math.ceil(math.log(1e-8) / math.log(pred)))
        r1 = O.bp_messages(net, tol=0.0, max_iter=t, damping=lam)[2]
        r2 = O.bp_messages(net, tol=0.0, max_iter=t + 1, damping=lam)[2]
        assert abs(r2 / r1 - pred) < 1e-4 * pred, (r2 / r1, pred)


def test_damping_out_of_range_rejected():
    net = P.random_2d(2, 2, 2, "uniform01", seed=1)
    for bad in (-0.1, 1.0):
        with pytest.raises(ValueError):
            O.bp_messages(net, damping=bad)


def test_full_mode_planted_mistake_is_caught(monkeypatch):
    """Dropping the dangling configurations from the complete expansion (the
    loop rule applied by mistake) breaks the exactness pin."""
    net = P.random_2d(2, 3, 2, "normal", seed=29)
    s, le = O.exact_log_contract(net)
    good = O.pne_contract(net, net.n_bonds, max_iter=2, mode="full")
    assert abs(good.log_abs - le) < 1e-11
    from oracle import pne_oracle as PO

    real = PO.enumerate_clusters
    monkeypatch.setattr(PO, "enumerate_clusters", lambda n, K, full=False: real(n, K, full=False))
    bad = O.pne_contract(net, net.n_bonds, max_iter=2, mode="full")
    assert abs(bad.log_abs - le) > 1e-9


# ----------------------------------------------------------------------------
# exponentiated (cumulant) form


def _even_counts(Lx, Ly):
    """Size histogram of the even subgraphs of an Lx x Ly grid (XOR of plaquettes)."""
    idx = {}
    for y in range(Ly):
        for x in range(Lx):
            s = x + Lx * y
            if x + 1 < Lx:
                idx[(s, s + 1)] = len(idx)
            if y + 1 < Ly:
                idx[(s, s + Lx)] = len(idx)
    basis = []
    for y in range(Ly - 1):
        for x in range(Lx - 1):
            s = x + Lx * y
            basis.append((1 << idx[(s, s + 1)]) | (1 << idx[(s, s + Lx)]) | (1 << idx[(s + 1, s + 1 + Lx)])
                         | (1 << idx[(s + Lx, s + Lx + 1)]))
    counts = {}
    for bits in range(1 << len(basis)):
        m = 0
        for i in range(len(basis)):
            if bits >> i & 1:
                m ^= basis[i]
        k = bin(m).count("1")
        counts[k] = counts.get(k, 0) + 1
    return counts


def _log_series(counts, K):
    """Integer Taylor coefficients c_k, k <= K, of ln(1 + sum_k g_k t^k) when
    every g_k with k > 0 has k >= 4 and K < 12 (so P^3 is beyond t^K):
    ln(1 + P) = P - P^2 / 2 mod t^12."""
    P = {k: c for k, c in counts.items() if k > 0}
    out = {}
    for k, c in P.items():
        if k <= K:
            out[k] = out.get(k, 0) + c
    for a, ca in P.items():
        for b, cb in P.items():
            if a + b <= K:
                out[a + b] = out.get(a + b, 0) - 0.5 * ca * cb
    return out


@pytest.mark.parametrize("Lx,Ly,beta,K", [(4, 4, 0.44, 8), (5, 4, 0.3, 10), (5, 5, 0.4, 8), (4, 4, 0.25, 6)])
def test_cumulant_form_equals_the_log_of_the_ht_series(Lx, Ly, beta, K):
    """Ising at the paramagnetic point: every retained cluster weighs t^|c|
    (t = tanh beta), so the cumulant form must equal N ln 2 + M ln cosh beta
    plus the Taylor coefficients (to t^K) of ln(1 + sum_k g_k t^k), with g_k
    the brute-force even-subgraph counts."""
    net = P.ising_2d(Lx, Ly, beta)
    r = O.pne_contract(net, K, mode="cumulant")
    t = math.tanh(beta)
    c = _log_series(_even_counts(Lx, Ly), K)
    expect = net.n_sites * math.log(2.0) + net.n_bonds * math.log(math.cosh(beta)) + \
        sum(v * t ** k for k, v in c.items())
    assert r.sign == 1
    assert abs(r.log_abs - expect) < 1e-12 * expect


def _disjoint_union(a, b):
    tens = list(a.tensors) + list(b.tensors)
    bonds = np.concatenate([np.asarray(a.bonds), np.asarray(b.bonds) + np.array([a.n_sites, 0, a.n_sites, 0])])
    return P.Network(tens, bonds.astype(np.int32), np.zeros((0, 2), np.int32))


def test_cumulant_form_is_additive_over_disjoint_parts():
    a = P.random_2d(4, 4, 3, "normal", seed=41)
    b = P.random_2d(5, 3, 2, "uniform01", seed=42)
    ab = _disjoint_union(a, b)
    K = 8
    fa, fb, fab = (O.pne_contract(x, K, mode="cumulant") for x in (a, b, ab))
    assert abs(fab.log_abs - (fa.log_abs + fb.log_abs)) < 1e-11
    # the truncated sum over collections is not: products of clusters from
    # both parts beyond degree K are dropped
    la, lb, lab = (O.pne_contract(x, K) for x in (a, b, ab))
    assert abs(lab.log_abs - (la.log_abs + lb.log_abs)) > 1e-9


def test_cumulant_form_needs_small_K():
    with pytest.raises(ValueError):
        O.pne_contract(P.ising_2d(4, 4, 0.3), 12, mode="cumulant")
    with pytest.raises(ValueError):
        O.pne_contract(P.random_2d(3, 3, 2, "uniform01", seed=3, open_sites={4: 2}), 4, mode="cumulant")


def test_cumulant_planted_mistake_is_caught(monkeypatch):
    """Leaving out the self-pairs (c, c) breaks the HT pin."""
    from oracle import pne_oracle as PO

    def no_self(weights, sizes, vsets, K):
        F = sum(float(w) for w in weights)
        for i in range(len(weights)):
            for j in range(len(weights)):
                if i != j and sizes[i] + sizes[j] <= K and vsets[i] & vsets[j]:
                    F -= 0.5 * float(weights[i]) * float(weights[j])
        return F

    net = P.ising_2d(4, 4, 0.44)
    good = O.pne_contract(net, 8, mode="cumulant").log_abs
    monkeypatch.setattr(PO, "cumulant_sum", no_self)
    assert abs(O.pne_contract(net, 8, mode="cumulant").log_abs - good) > 1e-6


def test_bp_rounding_floor_stop():
    """The rounding-floor stop of BP: with tol (1e-17) below the FP64 noise of
    the messages, plain sweeps never reach tol; the floor stop ends them as
    converged once 50 sweeps have not lowered the smallest residual, at the
    messages a normal 1e-13 run reaches.  Above 100 * tol the floor does not
    count, and on a run that reaches tol the stop never fires."""
    net = P.apply_random_gauge(P.small_network(3, 3, "random", 3, seed=1), 11, scale=1.0)
    inc0, it0, _, c0 = O.bp_messages(net, tol=1e-13)
    assert c0 and O.bp_messages(net, tol=1e-13, stall=0)[1] == it0
    inc, it, r, c = O.bp_messages(net, tol=1e-17, max_iter=400)
    assert c and it0 < it < 400 and r < 1e-13
    for a, b in zip(inc, inc0):
        for x, y in zip(a, b):
            assert np.max(np.abs(x - y)) < 1e-12
    _, it, _, c = O.bp_messages(net, tol=1e-17, max_iter=400, stall=0)
    assert not c and it == 400
    _, it, _, c = O.bp_messages(net, tol=1e-20, max_iter=400)
    assert not c and it == 400
