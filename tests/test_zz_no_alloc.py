"""The allocation-free entry point (pne_contract_batch_noalloc) against
pne_contract_batch, through the C ABI: same kernels and per-network reduction
order, so every result must be bitwise equal, on two calls in a row (the
second with a smaller input, over the scratch the first call left)."""

import ctypes

import numpy as np
import pytest

import pne_inputs as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_10910_amd as pne
    from paper_2512_10910_amd import pne as B

    ctx = pne.Context(0)
    yield pne, B, ctx
    ctx.close()


def _call(B, ctx, fn, nets, K, precision, flags=0):
    o = B._options(K, precision, 1e-13, 500, 0)
    o.flags |= flags
    arr = (ctypes.c_void_p * len(nets))(*[n.handle.value for n in nets])
    res = (B.ResultStruct * len(nets))()
    bufs = []
    for i, n in enumerate(nets):
        m = int(np.prod(n.open_shape)) if n.n_open else 0
        buf = np.zeros(max(1, m))
        bufs.append(buf)
        res[i].open_values = buf.ctypes.data_as(B._f64p) if m else None
        res[i].open_capacity = m
    st = fn(ctx.handle, arr, len(nets), ctypes.byref(o), res)
    return st, res, bufs


def _same(r1, b1, r2, b2):
    for i in range(len(r1)):
        a, b = r1[i], r2[i]
        assert (a.status, a.sign, a.bp_iters, a.n_cluster_terms, a.n_config_terms) == \
            (b.status, b.sign, b.bp_iters, b.n_cluster_terms, b.n_config_terms), i
        assert a.log_abs == b.log_abs and a.log_abs_bp == b.log_abs_bp, (i, a.log_abs, b.log_abs)
        assert a.dangling_max == b.dangling_max and a.term_err_est == b.term_err_est
        np.testing.assert_array_equal(b1[i], b2[i])


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_noalloc_equals_contract_batch_twice(env, precision):
    pne, B, ctx = env
    lib = ctx.lib
    big = [P.config2_network(4, 2000), P.config2_network(3, 2001), P.random_3d(4, 4, "normal", seed=5),
           P.random_2d(5, 4, 2, "uniform01", seed=60, open_sites={6: 2, 9: 2}), P.config1_network()]
    small = [P.random_2d(4, 4, 3, "uniform01", seed=7)]
    for batch in (big, small):  # the second call is smaller and reuses the scratch
        nets = [ctx.network(n) for n in batch]
        print(f"noalloc {precision}: {[n.name for n in batch]}", flush=True)
        s1, r1, b1 = _call(B, ctx, lib.pne_contract_batch, nets, 6, precision)
        s2, r2, b2 = _call(B, ctx, lib.pne_contract_batch_noalloc, nets, 6, precision)
        assert s1 == s2 and s1 >= 0, (s1, s2, ctx.error())
        _same(r1, b1, r2, b2)


def test_noalloc_refuses_what_needs_allocation(env):
    pne, B, ctx = env
    lib = ctx.lib
    nets = [ctx.network(P.random_2d(4, 4, 3, "uniform01", seed=7))]
    st, _, _ = _call(B, ctx, lib.pne_contract_batch_noalloc, nets, 6, "fp64", flags=B.PNE_FLAG_PROFILE)
    assert st == B.PNE_ERR_INVALID_ARG
    # 256 16x16 D=4 networks (about 0.35 MB each with FP32 slices) need more
    # than the 64 MiB scratch
    many = [ctx.network(P.config2_network(4, 2000 + i)) for i in range(256)]
    st, _, _ = _call(B, ctx, lib.pne_contract_batch_noalloc, many, 6, "fp32")
    assert st == B.PNE_ERR_OUT_OF_MEMORY, ctx.error()
    assert "scratch" in ctx.error()
    # and the next call still works
    st, r, _ = _call(B, ctx, lib.pne_contract_batch_noalloc, nets, 6, "fp64")
    assert st == 0 and r[0].status == 0
