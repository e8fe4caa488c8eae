"""GPU parity of the complete-expansion mode, damped BP, the dangling-term
measure and the reduced-precision estimate, against the CPU oracle.

* PNE_MODE_FULL with K = n_bonds is the complete expansion of Eqs. (2)-(4):
  it equals the exact contraction for the projectors of unconverged BP
  messages (|delta ln|Z|| <= 1e-10), and matches the oracle's complete mode
  at smaller K.
* bp_damping: Jacobi sweeps with the damped mix, sweep for sweep as the
  oracle's (same iteration count, ln|Z| within 1e-10).
* dangling_max: the oracle's measure (relative 1e-9 away from a fixed point).
* term_err_est: BF16 results whose estimate exceeds err_bound carry
  PNE_WARN_PRECISION and lie within the estimate; FP64/FP32 never warn here.
"""

import math

import pytest

import oracle as O
import pne_inputs as P

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


@pytest.mark.parametrize("shape,D,dist,seed,iters", [
    ((3, 3), 3, "normal", 21, 2),
    ((3, 3), 2, "uniform01", 5, 3),
    ((2, 4), 3, ("uniform", -0.8, 1.2), 6, 1),
    ((2, 5), 2, "normal", 8, 2),
])
def test_full_mode_complete_expansion_is_exact(ctx, shape, D, dist, seed, iters):
    net_in = P.random_2d(shape[0], shape[1], D, dist, seed=seed)
    M = net_in.n_bonds
    print(f"full mode {shape} D={D} M={M} iters={iters}", flush=True)
    net = ctx.network(net_in)
    r = ctx.contract(net, K=M, max_iter=iters, mode="full")
    assert r.status == 1 and r.bp_iters == iters  # BP stopped at the cap: a warning, with a result
    s, le = O.exact_log_contract(net_in)
    assert r.sign == s
    assert abs(r.log_abs - le) <= 1e-10, abs(r.log_abs - le)
    assert r.n_config_terms == 2 ** M - 1
    assert r.n_cluster_terms == len(O.enumerate_clusters(net_in, M, full=True))
    ref = O.pne_contract(net_in, M, max_iter=iters, mode="full")
    assert abs(r.log_abs - ref.log_abs) <= 1e-10


@pytest.mark.parametrize("K", [3, 5, 6])
def test_full_mode_truncated_matches_oracle(ctx, K):
    net_in = P.random_2d(3, 4, 2, "uniform01", seed=31)
    net = ctx.network(net_in)
    # Jacobi sweeps, as the oracle's, so that the unconverged messages agree
    r = ctx.contract(net, K=K, max_iter=3, mode="full", jacobi=True)
    ref = O.pne_contract(net_in, K, max_iter=3, mode="full")
    assert r.sign == ref.sign and r.n_config_terms == ref.n_configs and r.n_cluster_terms == ref.n_clusters
    assert abs(r.log_abs - ref.log_abs) <= 1e-10
    # at a fixed point the dangling terms vanish: full and loop modes agree
    a = ctx.contract(net, K=K, mode="full")
    b = ctx.contract(net, K=K)
    assert abs(a.log_abs - b.log_abs) <= 1e-10


@pytest.mark.parametrize("lam", [0.3, 0.6])
@pytest.mark.parametrize("name,make,K", [
    ("rand_4x4_D3", lambda: P.random_2d(4, 4, 3, "uniform01", seed=7), 6),
    ("rand3d_3_D2", lambda: P.random_3d(3, 2, "normal", seed=10), 6),
    ("open_4x4", lambda: P.random_2d(4, 4, 3, "uniform01", seed=32, open_sites={5: 2, 6: 2}), 6),
])
def test_damped_bp_matches_oracle(ctx, name, make, K, lam):
    net_in = make()
    r = ctx.contract(ctx.network(net_in), K=K, damping=lam)
    ref = O.pne_contract(net_in, K, damping=lam)
    assert r.status == 0
    assert abs(r.bp_iters - ref.bp_iters) <= 1
    if net_in.n_open:
        import numpy as np

        g = r.open_values * math.exp(r.log_abs - ref.log_abs)
        assert np.linalg.norm(g - ref.open_values) <= 1e-10 * np.linalg.norm(ref.open_values)
    else:
        assert r.sign == ref.sign and abs(r.log_abs - ref.log_abs) <= 1e-10


def test_damping_rejected_out_of_range(ctx):
    import paper_2512_10910_amd as pne

    net = ctx.network(P.random_2d(3, 3, 2, "uniform01", seed=1))
    with pytest.raises(pne.PNEError):
        ctx.batch([net], K=4, damping=1.0)


@pytest.mark.parametrize("iters", [2, 3, 500])
def test_dangling_max_matches_oracle(ctx, iters):
    nets_in = [P.random_2d(4, 4, 3, "normal", seed=31), P.random_3d(3, 3, "uniform01", seed=12),
               P.random_2d(5, 4, 2, "uniform01", seed=33, open_sites={6: 2})]
    for net_in in nets_in:
        for persistent in (True, False):
            r = ctx.contract(ctx.network(net_in), K=4, max_iter=iters, persistent=persistent, jacobi=True)
            inc, _, _, conv = O.bp_messages(net_in, max_iter=iters)
            d = O.dangling_max(net_in, inc)
            if conv:
                assert r.dangling_max < 1e-10 and d < 1e-10
            else:
                assert abs(r.dangling_max - d) <= 1e-9 * d, (r.dangling_max, d)


@pytest.mark.parametrize("name,make,K", [
    ("aklt_4x4", lambda: P.aklt_2d(4, 4), 8),
    ("aklt_12x12", lambda: P.config3_aklt_network(), 8),
])
def test_bf16_on_aklt_warns_and_stays_within_its_estimate(ctx, name, make, K):
    """O(1) loop corrections: BF16 slices (8-bit mantissa) cannot give 1e-5
    on ln|Z|; the result comes with PNE_WARN_PRECISION and its error lies
    within the reported estimate.  FP32 terms meet the bound without warning."""
    import paper_2512_10910_amd as pne

    net_in = make()
    ref = O.pne_contract(net_in, K)
    net = ctx.network(net_in)
    r = ctx.contract(net, K=K, precision="bf16")
    d = abs(r.log_abs - ref.log_abs)
    print(f"{name} bf16: |dlnZ|={d:.3e} estimate={r.term_err_est:.3e}", flush=True)
    assert r.status == pne.PNE_WARN_PRECISION
    assert r.sign == ref.sign and d <= r.term_err_est
    r32 = ctx.contract(net, K=K, precision="fp32")
    d32 = abs(r32.log_abs - ref.log_abs)
    assert r32.status == 0 and d32 / max(1.0, abs(ref.log_abs)) <= 1e-5 and d32 <= r32.term_err_est
    # a looser bound accepts the BF16 result without the warning
    r2 = ctx.contract(net, K=K, precision="bf16", err_bound=1.0)
    assert r2.status == 0 and r2.log_abs == r.log_abs


def test_bf16_on_random_networks_meets_the_bound_without_warning(ctx):
    for D, seed in ((4, 2000), (3, 2001)):
        net_in = P.config2_network(D, seed)
        ref = O.pne_contract(net_in, 6)
        r = ctx.contract(ctx.network(net_in), K=6, precision="bf16")
        d = abs(r.log_abs - ref.log_abs)
        assert r.status == 0, (r.status, r.term_err_est)
        assert d / max(1.0, abs(ref.log_abs)) <= 1e-5
        assert d <= max(r.term_err_est, 1e-12)


@pytest.mark.parametrize("name,make,K", [
    ("ising_4x4", lambda: P.ising_2d(4, 4, 0.44), 8),
    ("rand_6x5_D3", lambda: P.random_2d(6, 5, 3, "normal", seed=44), 8),
    ("rand3d_3_D3", lambda: P.random_3d(3, 3, "uniform01", seed=11), 6),
    ("config2_D4", lambda: P.config2_network(4, 2000), 6),
    ("aklt_12x12", lambda: P.config3_aklt_network(), 8),
    ("ising3d_6", lambda: P.config3_ising_network(0.2217), 6),
])
def test_cumulant_form_matches_oracle(ctx, name, make, K):
    """PNE_MODE_CUMULANT on both combine paths (the persistent block's and the
    combine launch's) against the oracle's second-order Mayer series."""
    net_in = make()
    ref = O.pne_contract(net_in, K, mode="cumulant")
    net = ctx.network(net_in)
    for fused in (True, False):
        r = ctx.contract(net, K=K, mode="cumulant", fused_regauge=fused)
        assert r.status == 0 and r.sign == ref.sign
        assert abs(r.log_abs - ref.log_abs) <= 1e-10, (fused, r.log_abs - ref.log_abs)
        assert r.n_config_terms == r.n_cluster_terms == ref.n_clusters
    r32 = ctx.contract(net, K=K, mode="cumulant", precision="fp32")
    assert r32.status == 0 and abs(r32.log_abs - ref.log_abs) / max(1.0, abs(ref.log_abs)) <= 1e-5


def test_cumulant_form_refusals(ctx):
    import paper_2512_10910_amd as pne

    closed = ctx.network(P.ising_2d(4, 4, 0.3))
    with pytest.raises(pne.PNEError) as ei:
        ctx.batch([closed], K=12, mode="cumulant")
    assert ei.value.status == -2
    opened = ctx.network(P.random_2d(4, 4, 3, "uniform01", seed=32, open_sites={5: 2, 6: 2}))
    with pytest.raises(pne.PNEError) as ei:
        ctx.batch([opened], K=6, mode="cumulant")
    assert ei.value.status == -2
