"""GPU parity for user partitions (Sec. II.A-C, Eqs. (4), (7), (9)-(11)).

The library evaluates a partitioned network as the BP vacuum times the sum of
the listed loop configurations that leave some partition unexcited; the
oracle evaluates Eq. (7) directly, as signed exact contractions of the network
with P inserted on the transected bonds.  The two share nothing but the
inputs.

Tolerances as in the other parity tests: FP64 |delta ln|Z|| <= 1e-10 with
equal signs; FP32 terms |delta ln|Z|| / max(1, |ln|Z||) <= 1e-5.
"""

import math

import numpy as np
import pytest

import oracle as O
import pne_inputs as P
from oracle import partitioned as PT
from oracle.exact import full_expansion_sum

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_10910_amd as pne

    c = pne.Context(0)
    yield c
    c.close()


def _net(Lx, Ly, kind, D=4, seed=0, bias=1.0):
    return lambda: P.small_network(Lx, Ly, kind, D, seed=seed, bias=bias)


CASES = [
    ("double_loop_rand_D4", _net(3, 2, "random", 4, 3, 1.0), P.double_loop_partitions),
    ("double_loop_rand_D3_bias05", _net(3, 2, "random", 3, 4, 0.5), P.double_loop_partitions),
    ("double_loop_rand_D6", _net(3, 2, "random", 6, 5, 1.0), P.double_loop_partitions),
    ("double_loop_aklt", _net(3, 2, "aklt"), P.double_loop_partitions),
    ("double_loop_ising", _net(3, 2, "ising"), P.double_loop_partitions),
    ("grid3_single_rand_D3", _net(3, 3, "random", 3, 6, 0.7), P.grid3_single_partitions),
    ("grid3_single_rand_D4", _net(3, 3, "random", 4, 7, 1.0), P.grid3_single_partitions),
    ("grid3_multi_rand_D4", _net(3, 3, "random", 4, 11, 1.0), P.grid3_multi_partitions),
    ("grid3_multi_rand_D3_bias05", _net(3, 3, "random", 3, 12, 0.5), P.grid3_multi_partitions),
    ("grid3_multi_aklt", _net(3, 3, "aklt"), P.grid3_multi_partitions),
    ("grid3_multi_ising", _net(3, 3, "ising"), P.grid3_multi_partitions),
    ("grid4x3_two_cuts", _net(4, 3, "random", 3, 13, 1.0), lambda n: [[0, 1], [5, 9, 12]]),
]


def _partitioned(ctx, net_in, parts):
    n = ctx.network(net_in)
    n.set_partitions(parts)
    return n


@pytest.mark.parametrize("name,make,parts_of", CASES)
def test_complete_expansion_matches_eq_a6_fp64(ctx, name, make, parts_of):
    net = make()
    parts = parts_of(net)
    n = _partitioned(ctx, net, parts)
    r = ctx.contract(n, K=32, precision="fp64")
    s, lg = PT.combinatorial_pne(net, parts)
    print(name, r.log_abs, lg, r.n_config_terms, flush=True)
    assert r.status == 0
    assert r.sign == s
    assert abs(r.log_abs - lg) <= 1e-10, f"|dlnZ|={abs(r.log_abs - lg):.3e}"
    assert r.n_config_terms == PT.count_retained(net, parts, 32)


@pytest.mark.parametrize("name,make,parts_of", [CASES[0], CASES[5], CASES[6]])
def test_single_index_partitions_match_eq_a4_fp64(ctx, name, make, parts_of):
    net = make()
    parts = parts_of(net)
    r = ctx.contract(_partitioned(ctx, net, parts), K=32, precision="fp64")
    s, lg = PT.linear_pne(net, parts)
    assert r.sign == s and abs(r.log_abs - lg) <= 1e-10


@pytest.mark.parametrize("K", [4, 6, 8])
def test_partitions_with_a_degree_cap(ctx, K):
    """Partitions and a degree cap together: the oracle sums the retained
    excitation patterns one literal contraction at a time."""
    net = P.small_network(3, 3, "random", 3, seed=21, bias=0.8)
    parts = P.grid3_multi_partitions(net)
    psets = [set(p) for p in parts]
    proj = PT.bp_projectors(net)
    ends = [(int(u), int(v)) for (u, _, v, _) in net.bonds]

    def keep(y):
        if len(y) > K:
            return False
        deg = [0] * net.n_sites
        for b in y:
            deg[ends[b][0]] += 1
            deg[ends[b][1]] += 1
        if any(d == 1 for d in deg):
            return False
        return not all(p & set(y) for p in psets)

    ls, t = full_expansion_sum(net, [(p[0], p[1]) for p in proj], filter_fn=keep)
    ref = ls + math.log(abs(float(t)))
    r = ctx.contract(_partitioned(ctx, net, parts), K=K, precision="fp64")
    assert r.sign == (1 if float(t) > 0 else -1)
    assert abs(r.log_abs - ref) <= 1e-10
    assert r.n_config_terms == PT.count_retained(net, parts, K)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_reduced_precision_terms(ctx, precision):
    net = P.small_network(3, 3, "random", 4, seed=31, bias=1.0)
    parts = P.grid3_multi_partitions(net)
    r = ctx.contract(_partitioned(ctx, net, parts), K=32, precision=precision)
    s, lg = PT.combinatorial_pne(net, parts)
    tol = 1e-5 if precision == "fp32" else 1e-2
    assert r.sign == s
    assert abs(r.log_abs - lg) / max(1.0, abs(lg)) <= tol, f"{abs(r.log_abs - lg):.3e}"


def test_mixed_batch_and_clearing(ctx):
    """One batch with partitioned and plain networks of the same geometry:
    the plain ones equal their own batch's results; clearing the partitions
    restores the plain expansion; the partitioned ones take the separate
    term launches (no in-block term path)."""
    import paper_2512_10910_amd as pne

    raw = [P.small_network(3, 3, "random", 3, seed=40 + i, bias=1.0) for i in range(6)]
    nets = [ctx.network(x) for x in raw]
    for i in (1, 3, 4):
        nets[i].set_partitions(P.grid3_multi_partitions(raw[i]))
    b = ctx.batch(nets, K=12, precision="fp64")
    res = b.run()
    paths = b.paths()
    for i in (1, 3, 4):
        s, lg = PT.combinatorial_pne(raw[i], P.grid3_multi_partitions(raw[i]))
        assert res[i].sign == s and abs(res[i].log_abs - lg) <= 1e-10
        assert not (paths[i] & pne.PATH_BLOCK_TERMS)
    plain = [ctx.network(raw[i]) for i in (0, 2, 5)]
    b2 = ctx.batch(plain, K=12, precision="fp64")
    res2 = b2.run()
    for k, i in enumerate((0, 2, 5)):
        assert abs(res[i].log_abs - res2[k].log_abs) <= 1e-12
    nets[3].set_partitions([])
    r3 = ctx.contract(nets[3], K=12, precision="fp64")
    ref = O.pne_contract(raw[3], 12)
    assert abs(r3.log_abs - ref.log_abs) <= 1e-10
    b.close()
    b2.close()


def test_invalid_partitions_are_errors(ctx):
    import paper_2512_10910_amd as pne

    net = ctx.network(P.small_network(3, 2, "random", 2, seed=1))
    for bad in ([[]], [[0, 0]], [[99]]):
        with pytest.raises(pne.PNEError):
            net.set_partitions(bad)
    opn = ctx.network(P.random_2d(3, 2, 2, seed=1, open_sites={0: 2}))
    with pytest.raises(pne.PNEError) as e:
        opn.set_partitions([[0]])
    assert e.value.status == -2


def test_workload_batch_sampled(ctx):
    """The benchmark's partition workload at its full size: 8192 3 x 3
    networks (D = 4, U[0, 2]) with six multi-index partitions, complete
    expansion, FP64 terms; sampled networks against Eq. (7)."""
    nb = 8192
    raw = [P.small_network(3, 3, "random", 4, seed=50000 + i, bias=1.0) for i in range(nb)]
    parts = P.grid3_multi_partitions(raw[0])
    nets = []
    for x in raw:
        n = ctx.network(x)
        n.set_partitions(parts)
        nets.append(n)
    b = ctx.batch(nets, K=12, precision="fp64")
    arr = b.run_arrays()
    assert (arr["status"] == 0).all()
    for i in (0, 1, 777, 4095, nb - 1):
        s, lg = PT.combinatorial_pne(raw[i], parts)
        assert arr["sign"][i] == s and abs(arr["log_abs"][i] - lg) <= 1e-10, i
    b.close()


# ----------------------------------------------------------------------------
# recursive partitioning (Sec. IV.A)


@pytest.mark.parametrize("kind,D,seed", [("random", 3, 1), ("random", 4, 2), ("ising", 2, 0), ("aklt", 4, 0)])
def test_recursive_three_by_four_matches_oracle(ctx, kind, D, seed):
    """The 3 x 4 example: five first-level lines, the two principal terms
    with a whole 3 x 3 block refined by its six partitions; complete
    expansion in FP64 against the oracle's literal recursion."""
    net = P.small_network(3, 4, kind, D, seed=seed)
    parts, subs = P.grid3x4_recursive_partitions(net)
    n = _partitioned(ctx, net, parts)
    for x, inner in subs.items():
        n.set_subpartitions(x, inner)
    r = ctx.contract(n, K=net.n_bonds, precision="fp64")
    s, lg = PT.recursive_pne(net, parts, subs)
    print(kind, r.log_abs, lg, r.n_config_terms, flush=True)
    assert r.status == 0 and r.sign == s
    assert abs(r.log_abs - lg) <= 1e-10, f"|dlnZ|={abs(r.log_abs - lg):.3e}"


def test_recursive_single_index_and_clearing(ctx):
    net = P.small_network(3, 3, "random", 3, seed=14, bias=0.8)
    parts = P.grid3_single_partitions(net)
    subs = {(0,): [[0], [2], [9], [11]], (1, 2): [[5], [6]]}
    n = _partitioned(ctx, net, parts)
    for x, inner in subs.items():
        n.set_subpartitions(x, inner)
    r = ctx.contract(n, K=12, precision="fp64")
    s, lg = PT.recursive_pne(net, parts, subs)
    assert r.sign == s and abs(r.log_abs - lg) <= 1e-10
    # removing one refinement, then resetting the partitions, restores the plain forms
    n.set_subpartitions((1, 2), [])
    r2 = ctx.contract(n, K=12, precision="fp64")
    s2, lg2 = PT.recursive_pne(net, parts, {(0,): subs[(0,)]})
    assert r2.sign == s2 and abs(r2.log_abs - lg2) <= 1e-10
    n.set_partitions(parts)
    r3 = ctx.contract(n, K=12, precision="fp64")
    s3, lg3 = PT.combinatorial_pne(net, parts)
    assert r3.sign == s3 and abs(r3.log_abs - lg3) <= 1e-10


def test_invalid_subpartitions_are_errors(ctx):
    import paper_2512_10910_amd as pne

    raw = P.small_network(3, 3, "random", 2, seed=1)
    n = ctx.network(raw)
    with pytest.raises(pne.PNEError):
        n.set_subpartitions((0,), [[1]])  # no partitions yet
    n.set_partitions(P.grid3_single_partitions(raw))
    for x, bad in (((7,), [[1]]), ((0,), [[]]), ((0,), [[99]]), ((0,), [[1, 1]])):
        with pytest.raises(pne.PNEError):
            n.set_subpartitions(x, bad)
