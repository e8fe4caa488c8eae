"""Pins of the CPU oracle against values fixed by the mathematics, not by the oracle.

Every check here is independent of the oracle's own arithmetic: brute-force
spin sums, the high-temperature (HT) closed form with even-subgraph counts
taken from the cycle space, eigenvalues from LAPACK, exact contractions and
the complete-expansion identity (Eqs. (2)-(4): P + Q = I on every bond).
"""

import itertools
import math

import numpy as np
import pytest

import oracle as O
import pne_inputs as P


# ----------------------------------------------------------------------------
# helpers independent of the oracle


def _bond_index(net):
    return {(int(u), int(v)): b for b, (u, _, v, _) in enumerate(net.bonds)}


def _even_subgraph_counts_2d(Lx, Ly, net):
    """Size histogram of even subgraphs, from XOR combinations of plaquettes."""
    bi = _bond_index(net)
    basis = []
    for y in range(Ly - 1):
        for x in range(Lx - 1):
            s = x + Lx * y
            edges = [bi[(s, s + 1)], bi[(s, s + Lx)], bi[(s + 1, s + 1 + Lx)], bi[(s + Lx, s + Lx + 1)]]
            basis.append(sum(1 << e for e in edges))
    counts = {}
    for bits in range(1 << len(basis)):
        m = 0
        for i in range(len(basis)):
            if bits >> i & 1:
                m ^= basis[i]
        k = bin(m).count("1")
        counts[k] = counts.get(k, 0) + 1
    return counts


def _ht_logz(N, M, beta, counts, K):
    t = math.tanh(beta)
    s = 1.0 + sum(c * t ** k for k, c in counts.items() if 0 < k <= K)
    return N * math.log(2.0) + M * math.log(math.cosh(beta)) + math.log(s)


def _bruteforce_clusters(net, K, exempt=()):
    """All connected bond subsets of size <= K with the degree rule, by brute force."""
    M = net.n_bonds
    ends = [(int(u), int(v)) for (u, _, v, _) in net.bonds]
    found = set()
    for k in range(1, K + 1):
        for sub in itertools.combinations(range(M), k):
            deg = {}
            parent = {}

            def find(a):
                while parent[a] != a:
                    parent[a] = parent[parent[a]]
                    a = parent[a]
                return a

            for b in sub:
                u, v = ends[b]
                for x in (u, v):
                    deg[x] = deg.get(x, 0) + 1
                    parent.setdefault(x, x)
                ru, rv = find(u), find(v)
                if ru != rv:
                    parent[ru] = rv
            if len({find(x) for x in parent}) != 1:
                continue
            if all(d >= 2 or s in exempt for s, d in deg.items()):
                found.add(tuple(sorted(sub)))
    return found


# ----------------------------------------------------------------------------
# exact references


@pytest.mark.parametrize("Lx,Ly,beta", [(4, 4, 0.44), (3, 3, 0.3), (2, 5, 0.9)])
def test_ising_tensor_network_matches_bruteforce_spin_sum(Lx, Ly, beta):
    net = P.ising_2d(Lx, Ly, beta)
    sign, lz = O.exact_log_contract(net)
    bf = O.ising_bruteforce_logz(net.n_sites, net.bonds[:, [0, 2]], beta)
    assert sign == 1
    assert abs(lz - bf) < 1e-12 * max(1.0, abs(bf))


def test_config1_exact_value():
    # 4x4 open-boundary Ising at beta = 0.44: brute force over 2^16 states
    net = P.config1_network()
    bf = O.ising_bruteforce_logz(16, net.bonds[:, [0, 2]], 0.44)
    assert abs(bf - 13.667552384220082) < 1e-12


def test_ising_3d_cube_bruteforce():
    net = P.ising_3d(2, 0.25)
    sign, lz = O.exact_log_contract(net)
    bf = O.ising_bruteforce_logz(8, net.bonds[:, [0, 2]], 0.25)
    assert abs(lz - bf) < 1e-12


# ----------------------------------------------------------------------------
# high-temperature closed form (Ising at the paramagnetic BP fixed point)


def test_even_subgraph_histogram_4x4():
    net = P.config1_network()
    c = _even_subgraph_counts_2d(4, 4, net)
    assert c == {0: 1, 4: 9, 6: 12, 8: 50, 10: 92, 12: 158, 14: 116, 16: 69, 18: 4, 20: 1}


@pytest.mark.parametrize("K", [0, 4, 6, 8, 10])
def test_loop_series_equals_ht_series_2d(K):
    beta = 0.44
    net = P.config1_network(beta)
    counts = _even_subgraph_counts_2d(4, 4, net)
    r = O.pne_contract(net, K)
    expect = _ht_logz(16, 24, beta, counts, K)
    assert r.sign == 1
    assert abs(r.log_abs - expect) < 1e-13 * abs(expect)


def test_config1_k4_value():
    r = O.pne_contract(P.config1_network(), 4)
    assert abs(r.log_abs - 13.576120516902) < 1e-11
    assert r.n_clusters == 9


@pytest.mark.parametrize("beta", [0.18, 0.2217, 0.26])
def test_loop_series_equals_ht_series_3d(beta):
    # 6^3 open cube: 450 plaquettes (3 L (L-1)^2) and 2720 six-cycles
    # (6 L (L-1)(L-2) planar 1x2 rectangles + 16 per unit cube)
    L = 6
    net = P.config3_ising_network(beta)
    n4 = 3 * L * (L - 1) ** 2
    n6 = 6 * L * (L - 1) * (L - 2) + 16 * (L - 1) ** 3
    assert (n4, n6) == (450, 2720)
    r = O.pne_contract(net, 6)
    expect = _ht_logz(216, 540, beta, {4: n4, 6: n6}, 6)
    assert abs(r.log_abs - expect) < 1e-12 * expect


def test_3d_closed_form_values():
    table = {0.18: 158.852294287657, 0.2217: 163.721323202172, 0.26: 169.055513732165}
    for beta, val in table.items():
        t = math.tanh(beta)
        v = 216 * math.log(2) + 540 * math.log(math.cosh(beta)) + math.log(1 + 450 * t ** 4 + 2720 * t ** 6)
        assert abs(v - val) < 1e-9


# ----------------------------------------------------------------------------
# complete-expansion identities


def _random_oblique(D, rng):
    x = rng.standard_normal(D) + 2.0
    y = rng.standard_normal(D) + 2.0
    Pm = np.outer(x, y) / (x @ y)
    return Pm, np.eye(D) - Pm


def test_full_expansion_with_arbitrary_projectors_is_exact():
    rng = np.random.default_rng(7)
    net = P.random_2d(2, 3, 3, ("uniform", -0.8, 1.2), seed=11)
    pp = [_random_oblique(3, rng) for _ in range(net.n_bonds)]
    ls, tot = O.full_expansion_sum(net, pp)
    le, ex = O.exact_contract(net)
    assert abs(float(tot) * math.exp(ls - le) / float(ex) - 1.0) < 1e-11


@pytest.mark.parametrize("shape,D,seed", [((2, 3), 3, 5), ((3, 3), 2, 6), ((2, 4), 3, 8)])
def test_dangling_free_sum_at_fixed_point_is_exact(shape, D, seed):
    net = P.random_2d(shape[0], shape[1], D, "uniform01", seed=seed)
    r = O.pne_contract(net, net.n_bonds)
    s, le = O.exact_log_contract(net)
    assert r.converged
    assert r.sign == s
    assert abs(r.log_abs - le) < 1e-11


def test_cluster_factorisation_matches_literal_terms():
    # any rank-1 oblique projectors: Z(y) = scale * prod_components w_c
    net = P.random_2d(3, 3, 3, "normal", seed=21)
    inc, _, _, _ = O.bp_messages(net, max_iter=3)  # deliberately not converged
    proj = O.projectors(net, inc)
    z = O.vacuum(net, inc)
    log_scale = sum(math.log(abs(float(v))) for v in z) - sum(math.log(abs(p[2])) for p in proj)
    sgn = np.prod([np.sign(float(v)) for v in z]) * np.prod([np.sign(p[2]) for p in proj])
    clusters = O.enumerate_clusters(net, 8)
    assert clusters
    for c in clusters[:40]:
        w = float(O.cluster_weight(net, inc, proj, z, c))
        ops = [proj[b][1] if b in c else proj[b][0] for b in range(net.n_bonds)]
        ls, t = O.literal_term(net, ops)
        lit = float(t) * math.exp(ls - log_scale) * sgn
        assert abs(w - lit) < 1e-10 * max(1.0, abs(lit))


def test_ring_bp_gives_dominant_eigenvalue():
    rng = np.random.default_rng(3)
    mats = [rng.random((3, 3)) + 0.1 for _ in range(5)]
    net = P.ring_network(mats)
    prod = np.linalg.multi_dot(mats)
    ev = np.linalg.eigvals(prod)
    lmax = float(np.max(ev.real))
    r = O.pne_contract(net, 4)  # K < L: only the vacuum survives
    assert r.n_clusters == 0
    assert abs(r.log_abs - math.log(lmax)) < 1e-11
    r = O.pne_contract(net, 5)  # K = L: the whole ring is the only cluster
    assert r.n_clusters == 1
    assert abs(r.log_abs - math.log(float(np.trace(prod)))) < 1e-11


def test_tree_is_exact_at_bp():
    rng = np.random.default_rng(4)
    ts = [rng.random(3)] + [rng.random((3, 3)) for _ in range(4)] + [rng.random(3)]
    net = P.chain_network(ts)
    r = O.pne_contract(net, 6)
    s, le = O.exact_log_contract(net)
    assert r.n_clusters == 0
    assert abs(r.log_abs - le) < 1e-12


def test_gauge_invariance():
    net = P.random_2d(3, 4, 3, "uniform01", seed=9)
    r0 = O.pne_contract(net, 6)
    g = P.apply_random_gauge(net, 123)
    r1 = O.pne_contract(g, 6)
    assert abs(r0.log_abs - r1.log_abs) < 1e-10
    assert abs(O.exact_log_contract(net)[1] - O.exact_log_contract(g)[1]) < 1e-12


def test_aklt_bulk_message_is_su2_singlet():
    net = P.aklt_2d(4, 4)
    inc, it, res, conv = O.bp_messages(net)
    assert conv
    m = inc[5][0]  # site (1,1), -x leg
    assert np.allclose(m, np.array([1, 0, 0, 1]) / math.sqrt(2), atol=1e-10)


# ----------------------------------------------------------------------------
# open networks (Sec. III.D)


def test_open_network_dangling_free_sum_is_exact():
    net = P.random_2d(3, 3, 2, "uniform01", seed=31, open_sites={0: 2, 7: 2})
    r = O.pne_contract(net, net.n_bonds)
    le, ex = O.exact_contract(net)
    approx = r.open_values * math.exp(r.log_abs - le)
    assert np.allclose(approx, ex, rtol=1e-10, atol=1e-12 * np.abs(ex).max())


def test_open_network_low_order_error_is_small():
    net = P.random_2d(4, 4, 3, "uniform01", seed=32, open_sites={5: 2, 6: 2})
    r = O.pne_contract(net, 6)
    le, ex = O.exact_contract(net)
    approx = r.open_values * math.exp(r.log_abs - le)
    err = np.linalg.norm(approx - ex) / np.linalg.norm(ex)  # Eq. (14)
    assert err < 1e-3


# ----------------------------------------------------------------------------
# cluster enumeration


@pytest.mark.parametrize("shape,K,exempt", [((3, 3), 12, ()), ((3, 4), 8, ()),
                                            ((3, 3), 8, (0, 4)), ((2, 2, 2), 8, ())])
def test_enumerator_matches_bruteforce(shape, K, exempt):
    net = P.grid_from_tensors(shape, lambda s, r, o: np.ones((2,) * r + o),
                              open_sites={s: 2 for s in exempt})
    got = set(O.enumerate_clusters(net, K))
    assert got == _bruteforce_clusters(net, K, exempt)


@pytest.mark.parametrize("L", [4, 5, 6, 7])
def test_enumerator_counts_2d(L):
    net = P.grid_from_tensors((L, L), lambda s, r, o: np.ones((2,) * r))
    cl = O.enumerate_clusters(net, 8)
    h = {}
    for c in cl:
        h[len(c)] = h.get(len(c), 0) + 1
    assert h.get(4, 0) == (L - 1) ** 2
    assert h.get(6, 0) == 2 * (L - 1) * (L - 2)
    assert h.get(7, 0) == 2 * (L - 1) * (L - 2)
    n8 = (L - 2) ** 2 + 2 * (L - 1) * (L - 3) + 4 * (L - 2) ** 2 + 2 * (L - 2) ** 2
    assert h.get(8, 0) == n8
    assert set(h) <= {4, 6, 7, 8}


@pytest.mark.parametrize("L", [3, 4, 6])
def test_enumerator_counts_3d(L):
    net = P.grid_from_tensors((L, L, L), lambda s, r, o: np.ones((2,) * r))
    cl = O.enumerate_clusters(net, 6)
    h = {}
    for c in cl:
        h[len(c)] = h.get(len(c), 0) + 1
    assert h == {4: 3 * L * (L - 1) ** 2, 6: 6 * L * (L - 1) * (L - 2) + 16 * (L - 1) ** 3}


def test_collections_respect_disjointness_and_budget():
    net = P.config1_network()
    cl = O.enumerate_clusters(net, 8)
    vs = [frozenset(x for b in c for x in (int(net.bonds[b, 0]), int(net.bonds[b, 2]))) for c in cl]
    cols = O.enumerate_collections(cl, [len(c) for c in cl], vs, 8)
    pairs = [c for c in cols if len(c) == 2]
    # disjoint plaquette pairs on 4x4: 9 plaquettes, C(9,2)=36 pairs minus 20 sharing a site
    assert len(pairs) == 16
    assert len(cols) == len(cl) + 16
