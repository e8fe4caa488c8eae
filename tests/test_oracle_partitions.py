"""Pins of the partitioned-expansion oracle (user partitions, Sec. II.A-C).

The two forms (Eq. (4), Eq. (7)) are checked against facts that do not come from
the oracle's own inclusion-exclusion: the exact contraction (Eq. (1)), the
residue written out directly (Q on every partition, Eq. res), the double-loop
example whose residue is a single degree-seven loop term (Sec. III.A), a
brute-force spin sum for the Ising model, a brute-force sum over every
excitation pattern for multi-index partitions (Eq. (10)), and the term count of
the six-partition 3 x 3 expansion.  The host planner of the library is checked
against the oracle's brute-force count of retained configurations (no GPU
needed).
"""

import math

import numpy as np
import pytest

import oracle as O
import pne_inputs as P
from oracle import partitioned as PT
from oracle.exact import full_expansion_sum


def _val(sl):
    s, lg = sl
    return 0.0 if s == 0 else s * math.exp(lg)


def _z0(net):
    s, lg = O.exact_log_contract(net)
    return s * math.exp(lg)


def test_six_partition_term_count():
    # 2^6 - 1 non-empty subsets: 6 principal terms and 57 sub-leading ones
    subs = PT.subsets(6)
    assert len(subs) == 63
    assert sum(1 for x in subs if len(x) >= 2) == 57
    assert sum(1 for x in subs if len(x) == 1) == 6


@pytest.mark.parametrize("kind,D,bias,seed", [("random", 4, 1.0, 3), ("random", 3, 0.5, 4), ("aklt", 4, 0.0, 0)])
def test_double_loop_residue_is_the_degree_seven_term(kind, D, bias, seed):
    """Three vertical partitions of the double loop: the dropped part is the
    configuration with all seven bonds excited (every other dangling-free
    configuration misses a vertical bond)."""
    net = P.small_network(3, 2, kind, D, seed=seed, bias=bias)
    proj = PT.bp_projectors(net)
    z0 = _z0(net)
    comb = _val(PT.combinatorial_pne(net, P.double_loop_partitions(net), proj))
    ls, t = O.literal_term(net, [proj[b][1] for b in range(net.n_bonds)])
    r7 = float(t) * math.exp(ls)
    assert abs(z0 - comb - r7) <= 1e-12 * abs(z0)


def test_double_loop_ising_is_exact():
    """Ising: the degree-seven term has sites with three excited legs, which
    vanish by spin-flip symmetry, so both forms give the exact Z."""
    net = P.small_network(3, 2, "ising")
    parts = P.double_loop_partitions(net)
    lz = O.ising_bruteforce_logz(net.n_sites, [(int(u), int(v)) for (u, _, v, _) in net.bonds], P.ISING_BETA_C)
    s, lg = PT.combinatorial_pne(net, parts)
    assert s == 1 and abs(lg - lz) < 1e-12
    s, lg = PT.linear_pne(net, parts)
    assert s == 1 and abs(lg - lz) < 1e-12


@pytest.mark.parametrize("Lx,Ly,parts_of,seed", [(3, 2, P.double_loop_partitions, 5),
                                                  (3, 3, P.grid3_single_partitions, 6)])
def test_single_index_forms_plus_residue_are_exact(Lx, Ly, parts_of, seed):
    """Eq. (4) and Eq. (7) each add up, with the residue, to the exact value,
    for BP projectors and for arbitrary rank-1 projectors alike."""
    net = P.small_network(Lx, Ly, "random", 3, seed=seed, bias=0.7)
    parts = parts_of(net)
    z0 = _z0(net)
    rng = np.random.default_rng(seed)
    bp = PT.bp_projectors(net)
    arbitrary = []
    for b in range(net.n_bonds):
        d = net.bond_dim(b)
        a, c = rng.normal(size=d), rng.normal(size=d)
        Pm = np.outer(a, c) / float(a @ c)
        arbitrary.append((Pm, np.eye(d) - Pm, float(a @ c)))
    for proj in (bp, arbitrary):
        comb = _val(PT.combinatorial_pne(net, parts, proj))
        lin = _val(PT.linear_pne(net, parts, proj))
        res = _val(PT.residue(net, parts, proj))
        assert abs(comb + res - z0) <= 1e-12 * abs(z0)
        assert abs(lin + res - z0) <= 1e-12 * abs(z0)


def test_multi_index_residue_is_every_partition_excited():
    """Six multi-index partitions on 3 x 3: Z0 minus the combinatorial form
    equals the sum over all 2^12 excitation patterns that excite at least one
    bond of every partition (Eq. (10): Q_p is the sum of the patterns of p with
    an excited bond)."""
    net = P.small_network(3, 3, "random", 2, seed=8, bias=0.8)
    parts = [set(p) for p in P.grid3_multi_partitions(net)]
    proj = PT.bp_projectors(net)
    z0 = _z0(net)
    comb = _val(PT.combinatorial_pne(net, P.grid3_multi_partitions(net), proj))
    ls, t = full_expansion_sum(net, [(p[0], p[1]) for p in proj],
                               filter_fn=lambda y: all(p & set(y) for p in parts))
    res = float(t) * math.exp(ls)
    assert abs(z0 - comb - res) <= 1e-12 * abs(z0)


def test_partitions_sharing_bonds_insert_each_projector_once():
    """Two identical partitions: the expansion equals the one with a single
    copy (P P = P, and the subset with both cancels one of the singles)."""
    net = P.small_network(3, 2, "random", 3, seed=9, bias=0.9)
    one = PT.combinatorial_pne(net, [[1, 3]])
    two = PT.combinatorial_pne(net, [[1, 3], [3, 1]])
    assert one[0] == two[0] and abs(one[1] - two[1]) < 1e-12


def test_oracle_rejects_malformed_partitions():
    net = P.small_network(3, 2, "random", 2, seed=1)
    with pytest.raises(ValueError):
        PT.combinatorial_pne(net, [[]])
    with pytest.raises(ValueError):
        PT.combinatorial_pne(net, [[0, 0]])
    with pytest.raises(ValueError):
        PT.combinatorial_pne(net, [[99]])
    with pytest.raises(ValueError):
        PT.linear_pne(net, [[0, 1]])


# ----------------------------------------------------------------------------
# library host planner (no device) against the oracle's brute-force count


@pytest.fixture(scope="module")
def pne():
    import paper_2512_10910_amd as lib

    try:
        lib.load_library()
    except OSError as e:  # pragma: no cover
        pytest.skip(f"library not built: {e}")
    return lib


CASES = [(3, 2, P.double_loop_partitions), (3, 3, P.grid3_single_partitions),
         (3, 3, P.grid3_multi_partitions), (4, 3, lambda n: [[0, 1], [5, 9, 12]]), (4, 3, lambda n: [])]


@pytest.mark.parametrize("Lx,Ly,parts_of", CASES)
@pytest.mark.parametrize("K", [4, 6, 8, 12, 32])
def test_library_counts_retained_configurations(pne, Lx, Ly, parts_of, K):
    net = P.small_network(Lx, Ly, "random", 3, seed=1)
    parts = parts_of(net)
    _, n_cfg = pne.count_configurations(net, K, parts)
    assert n_cfg == PT.count_retained(net, parts, K)


def test_library_rejects_malformed_partitions(pne):
    net = P.small_network(3, 2, "random", 2, seed=1)
    for bad, code in (([[]], -1), ([[0, 0]], -1), ([[99]], -1), ([[0]] * 33, -2)):
        with pytest.raises(pne.PNEError) as e:
            pne.count_configurations(net, 8, bad)
        assert e.value.status == code
    opn = P.random_2d(3, 2, 2, seed=1, open_sites={0: 2})
    with pytest.raises(pne.PNEError) as e:
        pne.count_configurations(opn, 8, [[0]])
    assert e.value.status == -2


# ----------------------------------------------------------------------------
# planted mistakes in the partitioned forms are caught by the pins above


def _double_loop_pins_hold():
    """The degree-seven residue pin (random tensors) and the Ising exactness
    pin.  (Swapping P and Q leaves the first intact: with P on the three
    vertical bonds the network falls into two chains, on which BP is exact.)"""
    net = P.small_network(3, 2, "random", 4, seed=3, bias=1.0)
    proj = PT.bp_projectors(net)
    z0 = _z0(net)
    comb = _val(PT.combinatorial_pne(net, P.double_loop_partitions(net), proj))
    ls, t = O.literal_term(net, [proj[b][1] for b in range(net.n_bonds)])
    ok1 = abs(z0 - comb - float(t) * math.exp(ls)) <= 1e-12 * abs(z0)
    ising = P.small_network(3, 2, "ising")
    lz = O.ising_bruteforce_logz(6, [(int(u), int(v)) for (u, _, v, _) in ising.bonds], P.ISING_BETA_C)
    s, lg = PT.combinatorial_pne(ising, P.double_loop_partitions(ising))
    ok2 = s == 1 and abs(lg - lz) < 1e-12
    return ok1 and ok2


@pytest.mark.parametrize("mutation", ["even_sign_plus", "q_instead_of_p", "last_subset_dropped", "transposed_p"])
def test_planted_mistakes_fail_the_pins(monkeypatch, mutation):
    assert _double_loop_pins_hold()
    orig_terms = PT.combinatorial_terms
    orig_proj = PT.bp_projectors
    if mutation == "even_sign_plus":
        monkeypatch.setattr(PT, "combinatorial_terms",
                            lambda net, parts, proj=None: [(1, ls, v, x) for (_, ls, v, x) in
                                                           orig_terms(net, parts, proj)])
    elif mutation == "q_instead_of_p":
        monkeypatch.setattr(PT, "bp_projectors",
                            lambda net, *a: [(q, p, n) for (p, q, n) in orig_proj(net, *a)])
    elif mutation == "last_subset_dropped":
        monkeypatch.setattr(PT, "combinatorial_terms",
                            lambda net, parts, proj=None: orig_terms(net, parts, proj)[:-1])
    else:
        monkeypatch.setattr(PT, "bp_projectors",
                            lambda net, *a: [(p.T.copy(), np.eye(p.shape[0]) - p.T, n)
                                             for (p, q, n) in orig_proj(net, *a)])
    assert not _double_loop_pins_hold()


# ----------------------------------------------------------------------------
# recursive partitioning (Sec. IV.A)


def test_recursive_form_plus_residues_is_exact():
    """Single-index partitions refined by single-index sub-partitions: the
    exact value is the recursive expansion plus the first-level residue plus,
    for each refined subset x, its sub-residue (P on x's bonds, Q on the
    sub-partition bonds) with the sign of x."""
    net = P.small_network(3, 3, "random", 3, seed=14, bias=0.8)
    parts = P.grid3_single_partitions(net)
    subs = {(0,): [[0], [2], [9], [11]], (1, 2): [[5], [6]]}
    proj = PT.bp_projectors(net)
    z0 = _z0(net)
    rec = _val(PT.recursive_pne(net, parts, subs, proj))
    res1 = _val(PT.residue(net, parts, proj))
    total = rec + res1
    for x, inner in subs.items():
        base = set(b for p in x for b in parts[p])
        ops = [np.eye(net.bond_dim(b)) for b in range(net.n_bonds)]
        for b in base:
            ops[b] = proj[b][0]
        for r in inner:
            b = r[0]
            ops[b] = proj[b][0] @ proj[b][1] if b in base else proj[b][1]
        ls, t = O.literal_term(net, ops)
        total += (1 if len(x) % 2 == 1 else -1) * float(t) * math.exp(ls)
    assert abs(total - z0) <= 1e-12 * abs(z0)


def test_recursive_residue_by_brute_force_coefficients():
    """Multi-index partitions on 3 x 3 (the two vertical lines), the first
    principal term refined by lines inside columns 1-2.  Z0 minus the
    recursive expansion equals the sum over all 2^12 excitation patterns S of
    (1 - c(S)) Z(Q on S, P elsewhere), with c(S) the signed count of the
    first-level subsets x whose bonds S avoids and which, where refined, have
    a sub-partition that S avoids."""
    net = P.small_network(3, 3, "random", 2, seed=15, bias=0.8)
    multi = P.grid3_multi_partitions(net)
    parts = [multi[0], multi[1]]
    inner = [[b for b in multi[2] if b not in multi[0]], [b for b in multi[3] if b not in multi[0]], multi[5]]
    subs = {(0,): inner}
    proj = PT.bp_projectors(net)
    z0 = _z0(net)
    rec = _val(PT.recursive_pne(net, parts, subs, proj))
    psets = [set(p) for p in parts]
    isets = [set(r) for r in inner]

    def coef(S):
        S = set(S)
        c = 0
        for x in PT.subsets(len(parts)):
            if any(psets[p] & S for p in x):
                continue
            keep = 1
            if tuple(x) in subs:
                keep = 0 if all(r & S for r in isets) else 1
            c += keep if len(x) % 2 == 1 else -keep
        return c

    resid = 0.0
    M = net.n_bonds
    for mask in range(1 << M):
        y = [b for b in range(M) if mask >> b & 1]
        w = 1 - coef(y)
        if w == 0:
            continue
        ops = [proj[b][1] if (mask >> b & 1) else proj[b][0] for b in range(M)]
        lt, tt = O.literal_term(net, ops)
        resid += w * float(tt) * math.exp(lt)
    assert abs(z0 - rec - resid) <= 1e-12 * abs(z0)


def test_paper_three_by_four_example_geometry():
    """Three horizontal and two vertical lines on 3 x 4; the principal terms of
    the top and bottom cuts keep a 3 x 3 block whole and are refined by that
    block's six partitions (every sub-partition lies inside the block)."""
    net = P.small_network(3, 4, "random", 2, seed=1)
    parts, subs = P.grid3x4_recursive_partitions(net)
    assert [len(p) for p in parts] == [3, 3, 3, 4, 4]
    assert set(subs) == {(0,), (2,)}
    for x, inner in subs.items():
        y0 = 1 if x == (0,) else 0
        assert len(inner) == 6
        for r in inner:
            for b in r:
                u, _, v, _ = (int(q) for q in net.bonds[b])
                assert y0 <= u // 3 <= y0 + 2 and y0 <= v // 3 <= y0 + 2
