"""GPU tests of the request server (continuous batching): every result equals
the same network contracted alone (bitwise: same kernels, same per-network
reduction order), admission under a small memory budget still completes
every request, and served results match the CPU oracle."""

import math
import time

import numpy as np
import pytest

import oracle as O
import pne_inputs as P

pytestmark = pytest.mark.gpu

# serving requests (seed 40000+i) with at most 64 sites: 2D L<=8 and 3D L=4
SMALL_REQUESTS = [7, 12, 13, 18, 23, 36, 37, 45, 47, 55, 63, 68, 69, 73, 94, 99, 106, 112]


@pytest.fixture(scope="module")
def pne():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_10910_amd as m

    return m


def _alone(pne, nets, K, precision):
    ctx = pne.Context(0)
    out = []
    for n in nets:
        out.append(ctx.contract(ctx.network(n), K=K, precision=precision))
    ctx.close()
    return out


def _serve(pne, nets, K, precision, **server_kw):
    ctx = pne.Context(0)
    sv = pne.Server(ctx, **server_kw)
    tickets = [sv.submit(n, K=K, precision=precision) for n in nets]
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                r = sv.poll(t)
                if r is not None:
                    res[t] = r
        assert time.time() - t0 < 120, "server did not finish"
        time.sleep(0.001)
    stats = sv.stats()
    sv.close()
    ctx.close()
    return [res[t] for t in tickets], stats


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_served_results_equal_alone(pne, precision):
    nets = [P.config4_request(i) for i in SMALL_REQUESTS]
    nets.append(P.random_2d(5, 4, 2, "uniform01", seed=60, open_sites={6: 2, 9: 2}))
    alone = _alone(pne, nets, 6, precision)
    served, stats = _serve(pne, nets, 6, precision, max_batch=7)
    assert stats["completed"] == len(nets) and stats["failed"] == 0
    assert stats["batches"] >= 3
    for a, s in zip(alone, served):
        assert s.status == a.status and s.sign == a.sign and s.bp_iters == a.bp_iters
        assert s.log_abs == a.log_abs, (s.log_abs, a.log_abs)
        assert s.n_cluster_terms == a.n_cluster_terms
    np.testing.assert_array_equal(served[-1].open_values, alone[-1].open_values)


def test_admission_under_small_budget(pne):
    nets = [P.config4_request(i) for i in SMALL_REQUESTS[:10]]
    alone = _alone(pne, nets, 6, "fp32")
    # a budget of a few requests' worth forces several admission rounds
    served, stats = _serve(pne, nets, 6, "fp32", mem_budget=2_000_000, pipeline_depth=2)
    assert stats["completed"] == len(nets) and stats["failed"] == 0
    assert stats["batches"] >= 3
    assert stats["device_bytes_admitted"] == 0
    assert stats["latency_p99_ms"] >= stats["latency_p50_ms"] > 0
    for a, s in zip(alone, served):
        assert s.log_abs == a.log_abs


def test_served_results_match_oracle(pne):
    nets = [P.config4_request(i) for i in (7, 12, 73)]
    served, _ = _serve(pne, nets, 6, "fp64")
    for n, s in zip(nets, served):
        ref = O.pne_contract(n, 6)
        assert s.sign == ref.sign
        assert abs(s.log_abs - ref.log_abs) <= 1e-10, (s.log_abs, ref.log_abs)


def test_submit_rejects_request_over_budget(pne):
    ctx = pne.Context(0)
    sv = pne.Server(ctx, mem_budget=10_000)
    with pytest.raises(pne.PNEError) as ei:
        sv.submit(P.config2_network(4, 2000), K=6)
    assert ei.value.status == -3
    sv.close()
    ctx.close()
    assert math.isfinite(0.0)


def test_completion_queue_with_prepared_requests(pne):
    nets = [P.config4_request(i) for i in SMALL_REQUESTS[:8]]
    alone = _alone(pne, nets, 6, "fp32")
    ctx = pne.Context(0)
    sv = pne.Server(ctx, completion_queue=True)
    reqs = [pne.Server.prepare(n, K=6, precision="fp32") for n in nets]
    tickets = [sv.submit(r) for r in reqs]
    seen = []
    t0 = time.time()
    while len(seen) < len(tickets):
        seen += sv.completed()
        assert time.time() - t0 < 120, "server did not finish"
        time.sleep(0.001)
    assert sorted(seen) == sorted(tickets)
    assert sv.completed() == []
    for t, a in zip(tickets, alone):
        r = sv.poll(t)
        assert r.status == a.status and r.log_abs == a.log_abs
    sv.close()
    ctx.close()


def test_cancel_queued_requests(pne):
    """Requests still queued when cancelled finish with PNE_ERR_CANCELLED;
    the others complete as if alone."""
    nets = [P.config4_request(i) for i in SMALL_REQUESTS[:12]]
    alone = _alone(pne, nets, 6, "fp32")
    ctx = pne.Context(0)
    # one request per batch, one batch in flight: the tail waits in the queue
    sv = pne.Server(ctx, max_batch=1, pipeline_depth=1, completion_queue=True)
    reqs = [pne.Server.prepare(n, K=6, precision="fp32") for n in nets]
    tickets = [sv.submit(r) for r in reqs]
    cancelled = {t for t in tickets[6:] if sv.cancel(t)}
    assert cancelled, "no request was still queued"
    seen = []
    t0 = time.time()
    while len(seen) < len(tickets):
        seen += sv.completed()
        assert time.time() - t0 < 120, "server did not finish"
        time.sleep(0.001)
    assert sorted(seen) == sorted(tickets)
    for t, a in zip(tickets, alone):
        r = sv.poll(t)
        if t in cancelled:
            assert r.status == pne.PNE_ERR_CANCELLED
        else:
            assert r.status == a.status and r.log_abs == a.log_abs
    with pytest.raises(pne.PNEError):
        sv.cancel(tickets[0])  # finished and polled: unknown ticket
    st = sv.stats()
    assert st["failed"] == len(cancelled) and st["completed"] == len(tickets)
    sv.close()
    ctx.close()
