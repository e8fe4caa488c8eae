"""CPU-side checks of the C ABI: exports, struct layout, validation, host geometry.

No compute call reaches a GPU here; the host-only enumeration entry point is
compared with the oracle's independent enumerator.
"""

import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
import pne_inputs as P
import paper_2512_10910_amd as pne
from paper_2512_10910_amd import pne as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pne.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pne_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pne.LIB_PATH):
        from paper_2512_10910_amd import build

        build.build()
    return pne.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # and the binding knows each of them
    assert set(names) <= set(B._PROTOS), set(names) - set(B._PROTOS)


def test_checked_build_exports_the_same_symbols(lib):
    """libpne_checked.so (cluster index checks compiled in) is built beside
    libpne.so and exports every declared entry point too."""
    from paper_2512_10910_amd import build

    assert os.path.exists(build.LIB_CHECKED)
    chk = ctypes.CDLL(build.LIB_CHECKED)
    for n in _declared_functions():
        assert hasattr(chk, n), n
    assert B.PNE_ERR_CHECK == -8 and "PNE_ERR_CHECK = -8" in open(HEADER).read()


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "pne.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("desc %zu\nopt %zu\nres %zu\n", sizeof(pne_network_desc), sizeof(pne_options), sizeof(pne_result));
  P(pne_network_desc, site_rank) P(pne_network_desc, site_data)
  P(pne_options, bp_tol) P(pne_options, bp_max_iter) P(pne_options, flags)
  P(pne_options, mode) P(pne_options, bp_damping) P(pne_options, err_bound)
  P(pne_options, small_sites) P(pne_options, tiles_in_flight) P(pne_options, reg_budget)
  P(pne_result, log_abs) P(pne_result, bp_iters) P(pne_result, bp_residual)
  P(pne_result, n_config_terms) P(pne_result, open_values) P(pne_result, open_capacity)
  P(pne_result, dangling_max) P(pne_result, term_err_est)
  printf("sopt %zu\nsstat %zu\n", sizeof(pne_server_options), sizeof(pne_server_stats));
  P(pne_server_options, max_batch) P(pne_server_options, pipeline_depth) P(pne_server_options, completion_queue)
  P(pne_server_stats, device_bytes_admitted) P(pne_server_stats, latency_p50_ms) P(pne_server_stats, busy_s)
  P(pne_server_stats, launch_s)
  printf("stopt %zu\nstres %zu\n", sizeof(pne_strip_options), sizeof(pne_strip_result));
  P(pne_strip_options, bp_tol) P(pne_strip_options, power_max_iter) P(pne_strip_options, power_tol)
  P(pne_strip_options, check_every) P(pne_strip_result, f) P(pne_strip_result, cell_sum)
  P(pne_strip_result, power_iters) P(pne_strip_result, lam) P(pne_strip_result, iters)
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)]).decode().split("\n") if line)
    assert int(out["desc"]) == ctypes.sizeof(B.NetworkDesc)
    assert int(out["opt"]) == ctypes.sizeof(B.Options)
    assert int(out["res"]) == ctypes.sizeof(B.ResultStruct)
    assert int(out["sopt"]) == ctypes.sizeof(B.ServerOptions)
    assert int(out["sstat"]) == ctypes.sizeof(B.ServerStats)
    assert int(out["stopt"]) == ctypes.sizeof(B.StripOptions)
    assert int(out["stres"]) == ctypes.sizeof(B.StripResult)
    for key, val in out.items():
        if "." in key:
            T, f = key.split(".")
            cls = {"pne_network_desc": B.NetworkDesc, "pne_options": B.Options, "pne_result": B.ResultStruct,
                   "pne_server_options": B.ServerOptions, "pne_server_stats": B.ServerStats,
                   "pne_strip_options": B.StripOptions, "pne_strip_result": B.StripResult}[T]
            assert getattr(cls, f).offset == int(val), key


def test_options_default(lib):
    o = B.Options()
    assert lib.pne_options_default(ctypes.byref(o)) == 0
    assert o.max_excited == 4 and o.precision == 0 and o.bp_tol == 1e-13 and o.bp_max_iter == 500
    assert o.mode == 0 and o.bp_damping == 0.0 and o.err_bound == 1e-5


def test_server_options_default_and_null_context(lib):
    so = B.ServerOptions()
    assert lib.pne_server_options_default(ctypes.byref(so)) == 0
    assert so.mem_budget == 0 and so.max_batch == 1024 and so.pipeline_depth == 2 and so.completion_queue == 0
    h = ctypes.c_void_p()
    assert lib.pne_server_create(None, ctypes.byref(so), ctypes.byref(h)) == B.PNE_ERR_INVALID_ARG
    assert lib.pne_submit(None, None, None, None) == B.PNE_ERR_INVALID_ARG
    assert lib.pne_poll(None, ctypes.c_uint64(1), None) == B.PNE_ERR_INVALID_ARG
    n = ctypes.c_int32(0)
    assert lib.pne_server_completed(None, None, 0, ctypes.byref(n)) == B.PNE_ERR_INVALID_ARG


def test_context_without_gpu_reports_device_error(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pne.PNEError) as ei:
        pne.Context(0)
    assert ei.value.status == B.PNE_ERR_DEVICE


@pytest.mark.parametrize("make,K", [
    (lambda: P.config1_network(), 8),
    (lambda: P.random_2d(5, 6, 3, seed=1), 8),
    (lambda: P.random_3d(3, 2, seed=2), 6),
    (lambda: P.random_2d(4, 4, 2, seed=3, open_sites={5: 2, 10: 2}), 8),
    (lambda: P.random_2d(6, 3, 2, seed=4, open_sites={7: 2}), 7),
    (lambda: P.ring_network([np.ones((2, 2))] * 6), 6),
    (lambda: P.random_2d(3, 3, 2, seed=5), 12),
])
def test_library_enumerator_matches_oracle(lib, make, K):
    net = make()
    mine = pne.enumerate_clusters(net, K)
    assert len(mine) == len(set(mine))
    assert set(mine) == set(O.enumerate_clusters(net, K))


def test_library_cluster_order_is_type_then_size(lib):
    net = P.random_2d(4, 4, 2, seed=3, open_sites={5: 2, 10: 2})
    cl = pne.enumerate_clusters(net, 8)
    opens = {5, 10}
    key = []
    for c in cl:
        vs = {int(net.bonds[b, 0]) for b in c} | {int(net.bonds[b, 2]) for b in c}
        t = (1 if 5 in vs else 0) | (2 if 10 in vs else 0)
        key.append((t, len(c)))
    assert key == sorted(key)
    assert opens


def test_dimension_one_bonds_are_never_excited(lib):
    net = P.grid_from_tensors((3, 3), lambda s, r, o: np.ones((2,) * r))
    # shrink bond 0 (between sites 0 and 1) to dimension 1
    u, lu, v, lv = net.bonds[0]
    t0 = net.tensors[u].take([0], axis=lu)
    t1 = net.tensors[v].take([0], axis=lv)
    net.tensors[u], net.tensors[v] = t0, t1
    cl = pne.enumerate_clusters(net, 12)
    assert all(0 not in c for c in cl)
    ref = [c for c in O.enumerate_clusters(net, 12) if 0 not in c]
    assert set(cl) == set(ref)


def _desc_status(tensors, bonds, open_legs=None, K=4):
    lib = pne.load_library()
    da = B._DescArrays(tensors, bonds, open_legs, data_ptrs=[1] * len(tensors))
    nc = ctypes.c_int64(0)
    ne = ctypes.c_int64(0)
    return lib.pne_enumerate_clusters(ctypes.byref(da.desc), K, ctypes.byref(nc), ctypes.byref(ne), None, None)


def test_validation_rejects_malformed_networks(lib):
    a = np.ones((2, 2))
    assert _desc_status([a, a], [(0, 0, 1, 0), (0, 1, 1, 1)]) == 0
    assert _desc_status([a, a], [(0, 0, 1, 0), (0, 0, 1, 1)]) == B.PNE_ERR_INVALID_ARG  # leg used twice
    assert _desc_status([a, np.ones((3, 2))], [(0, 0, 1, 0), (0, 1, 1, 1)]) == B.PNE_ERR_INVALID_ARG  # dims
    assert _desc_status([a, a], [(0, 0, 0, 1), (1, 0, 1, 1)]) == B.PNE_ERR_INVALID_ARG  # self bond
    assert _desc_status([a, a], [(0, 0, 1, 0)]) == B.PNE_ERR_INVALID_ARG  # dangling leg
    assert _desc_status([a, a], [(0, 0, 1, 0), (0, 1, 5, 1)]) == B.PNE_ERR_INVALID_ARG  # site range
    assert _desc_status([a, a], [(0, 0, 1, 0)], [(0, 1), (1, 1)]) == 0  # open legs fine
    assert _desc_status([a, a], [(0, 0, 1, 0), (0, 1, 1, 1)], K=-1) in (0, B.PNE_ERR_INVALID_ARG)


def test_three_open_sites_unsupported(lib):
    t = [np.ones((2, 2, 2)), np.ones((2, 2, 2)), np.ones((2, 2, 2))]
    bonds = [(0, 0, 1, 0), (1, 1, 2, 0), (2, 1, 0, 1)]
    assert _desc_status(t, bonds, [(0, 2), (1, 2), (2, 2)]) == B.PNE_ERR_UNSUPPORTED


def test_strip_options_default_and_null_arguments(lib):
    opt = B.StripOptions()
    assert lib.pne_strip_options_default(ctypes.byref(opt)) == 0
    assert (opt.L, opt.two_d, opt.bp_max_iter, opt.power_max_iter, opt.check_every) == (2, 1, 10000, 20000, 4)
    assert opt.bp_tol == 1e-14 and opt.power_tol == 1e-13
    assert lib.pne_strip_options_default(None) == -1
    res = B.StripResult()
    assert lib.pne_strip_expand(None, None, 2, ctypes.byref(opt), ctypes.byref(res)) == -1


def test_rank_and_partition_entry_points_reject_null_arguments(lib):
    opt = B.RankOptions()
    assert lib.pne_rank_options_default(ctypes.byref(opt)) == 0
    assert (opt.rank, opt.form, opt.ramp_sweeps, opt.max_sweeps) == (2, 0, 10, 2000)
    assert opt.alpha == 0.8 and opt.tol == 1e-12
    assert lib.pne_rank_options_default(None) == -1
    res = (B.RankResult * 1)()
    begin = (ctypes.c_int32 * 2)(0, 1)
    bond = (ctypes.c_int32 * 1)(0)
    assert lib.pne_rank_expand(None, None, 1, 3, 3, 1, begin, bond, ctypes.byref(opt), res) == -1
    assert opt.profile == 0
    ms = (ctypes.c_double * 5)()
    assert lib.pne_rank_last_times(None, ms, 5) == -1
    assert lib.pne_cancel(None, ctypes.c_uint64(1)) == -1
    assert lib.pne_network_set_partitions(None, 1, begin, bond) == -1
    assert lib.pne_network_set_subpartitions(None, 1, 1, begin, bond) == -1


def test_rank_structs_match_header(tmp_path):
    src = tmp_path / "rank.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "pne.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(pne_rank_options), sizeof(pne_rank_result),
         offsetof(pne_rank_options, tol), offsetof(pne_rank_result, log_abs), offsetof(pne_rank_result, log_scale),
         offsetof(pne_rank_options, profile));
  return 0;
}
''')
    exe = tmp_path / "rank"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    a, b, c, d, e, f = (int(x) for x in subprocess.check_output([str(exe)]).split())
    assert a == ctypes.sizeof(B.RankOptions) and b == ctypes.sizeof(B.RankResult)
    assert c == B.RankOptions.tol.offset and d == B.RankResult.log_abs.offset and e == B.RankResult.log_scale.offset
    assert f == B.RankOptions.profile.offset


@pytest.mark.parametrize("shape,K", [((3, 3), 12), ((3, 3), 5), ((2, 4), 10), ((3, 4), 17)])
def test_full_mode_counts_match_oracle(lib, shape, K):
    """The complete-expansion mode lists every bond subset of size <= K as its
    connected components: sum_k C(M, k) configurations, and the oracle's
    connected sets (no dangling rule) as clusters."""
    import math

    net = P.random_2d(shape[0], shape[1], 2, "uniform01", seed=1)
    M = net.n_bonds
    nc, ncf = pne.count_configurations(net, K, mode="full")
    assert ncf == sum(math.comb(M, k) for k in range(1, min(K, M) + 1))
    assert nc == len(O.enumerate_clusters(net, K, full=True))
    loop_nc, _ = pne.count_configurations(net, K)
    assert loop_nc == len(O.enumerate_clusters(net, K)) < nc


def test_full_mode_envelope(lib):
    big = P.random_2d(5, 3, 2, "uniform01", seed=1)  # 22 bonds
    with pytest.raises(pne.PNEError) as ei:
        pne.count_configurations(big, 4, mode="full")
    assert ei.value.status == B.PNE_ERR_UNSUPPORTED
    opn = P.random_2d(3, 3, 2, "uniform01", seed=2, open_sites={4: 2})
    with pytest.raises(pne.PNEError) as ei:
        pne.count_configurations(opn, 4, mode="full")
    assert ei.value.status == B.PNE_ERR_UNSUPPORTED
    with pytest.raises(pne.PNEError) as ei:
        pne.count_configurations(P.random_2d(3, 3, 2, "uniform01", seed=2), 4, [[0]], mode="full")
    assert ei.value.status == B.PNE_ERR_UNSUPPORTED
