"""ctypes binding of libpne.so (include/pne.h).  Argument marshalling only:
every step of the expansion runs inside the library's HIP kernels.

PyTorch appears only as plumbing: device-resident inputs may be passed as
CUDA tensors (their data pointers are borrowed), and a torch stream can be
handed to the context.
"""

from __future__ import annotations

import ctypes
import os
import weakref
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PNE_CHECKED=1 in the environment selects the checked build (cluster
# kernel index checks compiled in, PNE_ERR_CHECK on a failed check)
LIB_PATH = os.path.join(_HERE, "libpne_checked.so" if os.environ.get("PNE_CHECKED") == "1" else "libpne.so")

PNE_OK = 0
PNE_WARN_BP_NOT_CONVERGED = 1
PNE_WARN_PRECISION = 2
PNE_ERR_INVALID_ARG = -1
PNE_ERR_UNSUPPORTED = -2
PNE_ERR_OUT_OF_MEMORY = -3
PNE_ERR_SINGULAR = -4
PNE_ERR_DEVICE = -5
PNE_ERR_NOT_READY = -6
PNE_ERR_CANCELLED = -7
PNE_ERR_CHECK = -8

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
MODES = {"loop": 0, "full": 1, "cumulant": 2}

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class NetworkDesc(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32),
        ("n_bonds", ctypes.c_int32),
        ("n_open", ctypes.c_int32),
        ("site_rank", _i32p),
        ("leg_dim", _i32p),
        ("bond_site", _i32p),
        ("bond_leg", _i32p),
        ("open_leg", _i32p),
        ("site_data", ctypes.POINTER(ctypes.c_void_p)),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("max_excited", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("bp_tol", ctypes.c_double),
        ("bp_max_iter", ctypes.c_int32),
        ("bp_check_every", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("profile_kernels", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("bp_stall_steps", ctypes.c_int32),
        ("bp_damping", ctypes.c_double),
        ("err_bound", ctypes.c_double),
        ("small_sites", ctypes.c_int32),
        ("tiles_in_flight", ctypes.c_int32),
        ("reg_budget", ctypes.c_int32),
        ("reserved1", ctypes.c_int32),
    ]


class ResultStruct(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("sign", ctypes.c_int32),
        ("log_abs", ctypes.c_double),
        ("log_abs_bp", ctypes.c_double),
        ("bp_iters", ctypes.c_int32),
        ("n_open_values", ctypes.c_int32),
        ("bp_residual", ctypes.c_double),
        ("n_cluster_terms", ctypes.c_int64),
        ("n_config_terms", ctypes.c_int64),
        ("open_values", _f64p),
        ("open_capacity", ctypes.c_int64),
        ("dangling_max", ctypes.c_double),
        ("term_err_est", ctypes.c_double),
    ]


class ServerOptions(ctypes.Structure):
    _fields_ = [
        ("mem_budget", ctypes.c_size_t),
        ("max_batch", ctypes.c_int32),
        ("pipeline_depth", ctypes.c_int32),
        ("completion_queue", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("batches", ctypes.c_int64),
        ("pending", ctypes.c_int64),
        ("device_bytes_admitted", ctypes.c_int64),
        ("latency_p50_ms", ctypes.c_double),
        ("latency_p99_ms", ctypes.c_double),
        ("latency_mean_ms", ctypes.c_double),
        ("latency_max_ms", ctypes.c_double),
        ("networks_per_s", ctypes.c_double),
        ("busy_s", ctypes.c_double),
        ("prep_s", ctypes.c_double),
        ("wait_s", ctypes.c_double),
        ("upload_s", ctypes.c_double),
        ("networks_s", ctypes.c_double),
        ("batch_s", ctypes.c_double),
        ("launch_s", ctypes.c_double),
    ]


# numpy view of pne_result (same field offsets as the C struct)
_RESULT_FIELDS = ["status", "sign", "log_abs", "log_abs_bp", "bp_iters", "n_open_values", "bp_residual",
                  "n_cluster_terms", "n_config_terms", "open_values", "open_capacity", "dangling_max",
                  "term_err_est"]
RESULT_DTYPE = np.dtype({
    "names": _RESULT_FIELDS,
    "formats": [np.int32, np.int32, np.float64, np.float64, np.int32, np.int32, np.float64, np.int64, np.int64,
                np.uint64, np.int64, np.float64, np.float64],
    "offsets": [getattr(ResultStruct, f).offset for f in _RESULT_FIELDS],
    "itemsize": ctypes.sizeof(ResultStruct),
})


class StripOptions(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("two_d", ctypes.c_int32),
        ("bp_tol", ctypes.c_double),
        ("bp_max_iter", ctypes.c_int32),
        ("power_max_iter", ctypes.c_int32),
        ("power_tol", ctypes.c_double),
        ("check_every", ctypes.c_int32),
        ("single_site_passes", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class StripResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("bp_iters", ctypes.c_int32),
        ("f", ctypes.c_double),
        ("f_bp", ctypes.c_double),
        ("bp_residual", ctypes.c_double),
        ("cell_sum", ctypes.c_double),
        ("power_iters", ctypes.c_int32),
        ("n_unconverged", ctypes.c_int32),
        ("lam", _f64p),
        ("gam", _f64p),
        ("patch", _f64p),
        ("iters", ctypes.POINTER(ctypes.c_int32)),
        ("reserved", ctypes.c_int64),
    ]


class RankOptions(ctypes.Structure):
    _fields_ = [
        ("rank", ctypes.c_int32),
        ("form", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("ramp_sweeps", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("profile", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class RankResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("sign", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("log_abs", ctypes.c_double),
        ("log_scale", ctypes.c_double),
    ]


# exported C symbols and their prototypes: (restype, argtypes)
_PROTOS = {
    "pne_options_default": (ctypes.c_int, [ctypes.POINTER(Options)]),
    "pne_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "pne_ctx_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pne_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "pne_network_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(NetworkDesc), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "pne_network_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pne_network_set_partitions": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _i32p, _i32p]),
    "pne_network_set_subpartitions": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32, _i32p,
                                                     _i32p]),
    "pne_rank_options_default": (ctypes.c_int, [ctypes.POINTER(RankOptions)]),
    "pne_rank_expand": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p,
                                       ctypes.POINTER(RankOptions), ctypes.POINTER(RankResult)]),
    "pne_rank_last_times": (ctypes.c_int, [ctypes.c_void_p, _f64p, ctypes.c_int32]),
    "pne_strip_options_default": (ctypes.c_int, [ctypes.POINTER(StripOptions)]),
    "pne_strip_expand": (ctypes.c_int, [ctypes.c_void_p, _f64p, ctypes.c_int32, ctypes.POINTER(StripOptions),
                                        ctypes.POINTER(StripResult)]),
    "pne_count_configurations": (ctypes.c_int, [ctypes.POINTER(NetworkDesc), ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int32, _i32p, _i32p, ctypes.POINTER(ctypes.c_int64),
                                                ctypes.POINTER(ctypes.c_int64)]),
    "pne_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                        ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_void_p)]),
    "pne_batch_launch": (ctypes.c_int, [ctypes.c_void_p]),
    "pne_batch_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ResultStruct)]),
    "pne_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ResultStruct)]),
    "pne_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pne_contract": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Options),
                                    ctypes.POINTER(ResultStruct)]),
    "pne_contract_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                          ctypes.POINTER(Options), ctypes.POINTER(ResultStruct)]),
    "pne_contract_batch_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                                  ctypes.POINTER(Options), ctypes.POINTER(ResultStruct)]),
    "pne_enumerate_clusters": (ctypes.c_int, [ctypes.POINTER(NetworkDesc), ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                              _i32p, _i32p]),
    "pne_batch_messages": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p, ctypes.c_int64]),
    "pne_batch_phase_times": (ctypes.c_int, [ctypes.c_void_p, _f64p, ctypes.c_int32]),
    "pne_batch_paths": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "pne_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                    ctypes.POINTER(Options), ctypes.c_int32, ctypes.POINTER(Options)]),
    "pne_tune_cache_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "pne_tune_cache_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
    "pne_server_options_default": (ctypes.c_int, [ctypes.POINTER(ServerOptions)]),
    "pne_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerOptions),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "pne_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "pne_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(NetworkDesc), ctypes.POINTER(Options),
                                  ctypes.POINTER(ctypes.c_uint64)]),
    "pne_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ResultStruct)]),
    "pne_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "pne_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "pne_server_completed": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "pne_batch_kernel_times": (ctypes.c_int, [ctypes.c_void_p, _f64p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                              ctypes.c_int32]),
    "pne_batch_cluster_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, _f64p, ctypes.c_int64,
                                                 ctypes.POINTER(ctypes.c_int64),
                                                 ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpne.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2512_10910_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class PNEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pne status {status}: {msg}")
        self.status = status


def _err(lib, ctx_handle):
    m = lib.pne_last_error(ctx_handle)
    return m.decode() if m else ""


def _check(lib, status, ctx_handle=None):
    if status < 0:
        raise PNEError(status, _err(lib, ctx_handle))
    return status


# ----------------------------------------------------------------------------
# descriptors


class _DescArrays:
    """Keeps the numpy arrays a NetworkDesc points into alive."""

    def __init__(self, tensors, bonds, open_legs, data_ptrs=None):
        self.ranks = np.ascontiguousarray([t.ndim for t in tensors], dtype=np.int32)
        self.dims = np.ascontiguousarray([d for t in tensors for d in t.shape], dtype=np.int32)
        b = np.asarray(bonds, dtype=np.int32).reshape(-1, 4)
        self.bond_site = np.ascontiguousarray(b[:, [0, 2]]).reshape(-1)
        self.bond_leg = np.ascontiguousarray(b[:, [1, 3]]).reshape(-1)
        o = np.asarray(open_legs if open_legs is not None else np.zeros((0, 2)), dtype=np.int32).reshape(-1, 2)
        self.open_leg = np.ascontiguousarray(o).reshape(-1)
        self.n_bonds = b.shape[0]
        self.n_open = o.shape[0]
        if data_ptrs is None:
            self.host = [np.ascontiguousarray(t, dtype=np.float64) for t in tensors]
            data_ptrs = [h.ctypes.data for h in self.host]
        self.ptrs = (ctypes.c_void_p * len(tensors))(*data_ptrs)
        self.desc = NetworkDesc(
            len(tensors), self.n_bonds, self.n_open,
            self.ranks.ctypes.data_as(_i32p), self.dims.ctypes.data_as(_i32p),
            self.bond_site.ctypes.data_as(_i32p) if self.n_bonds else None,
            self.bond_leg.ctypes.data_as(_i32p) if self.n_bonds else None,
            self.open_leg.ctypes.data_as(_i32p) if self.n_open else None,
            ctypes.cast(self.ptrs, ctypes.POINTER(ctypes.c_void_p)))


def _net_parts(obj):
    tensors = list(obj.tensors)
    bonds = np.asarray(obj.bonds)
    open_legs = getattr(obj, "open_legs", None)
    return tensors, bonds, open_legs


def _partition_arrays(partitions):
    parts = [np.asarray(p, dtype=np.int32).reshape(-1) for p in partitions]
    begin = np.zeros(len(parts) + 1, dtype=np.int32)
    for k, p in enumerate(parts):
        begin[k + 1] = begin[k] + p.size
    bonds = np.concatenate(parts).astype(np.int32) if parts else np.zeros(1, np.int32)
    return parts, np.ascontiguousarray(begin), np.ascontiguousarray(bonds)


def count_configurations(obj, K: int, partitions=(), mode="loop"):
    """Host-only: (retained clusters, retained configurations) at degree cap K
    in the given mode ("loop" or "full")."""
    lib = load_library()
    tensors, bonds, open_legs = _net_parts(obj)
    shapes = [np.empty(t.shape, dtype=np.float64) if isinstance(t, np.ndarray) else np.empty(tuple(t.shape))
              for t in tensors]
    da = _DescArrays(shapes, bonds, open_legs, data_ptrs=[1] * len(tensors))
    parts, begin, pb = _partition_arrays(partitions)
    nc = ctypes.c_int64(0)
    ncf = ctypes.c_int64(0)
    _check(lib, lib.pne_count_configurations(ctypes.byref(da.desc), K, MODES[mode], len(parts),
                                             begin.ctypes.data_as(_i32p),
                                             pb.ctypes.data_as(_i32p), ctypes.byref(nc), ctypes.byref(ncf)))
    return nc.value, ncf.value


def enumerate_clusters(obj, K: int):
    """Host-only: the library's retained clusters (tuples of bond ids) in its order."""
    lib = load_library()
    tensors, bonds, open_legs = _net_parts(obj)
    shapes = [np.empty(t.shape, dtype=np.float64) if isinstance(t, np.ndarray) else np.empty(tuple(t.shape))
              for t in tensors]
    da = _DescArrays(shapes, bonds, open_legs, data_ptrs=[1] * len(tensors))
    nc = ctypes.c_int64(0)
    ne = ctypes.c_int64(0)
    _check(lib, lib.pne_enumerate_clusters(ctypes.byref(da.desc), K, ctypes.byref(nc), ctypes.byref(ne), None, None))
    sizes = np.zeros(max(1, nc.value), np.int32)
    bl = np.zeros(max(1, ne.value), np.int32)
    _check(lib, lib.pne_enumerate_clusters(ctypes.byref(da.desc), K, ctypes.byref(nc), ctypes.byref(ne),
                                           sizes.ctypes.data_as(_i32p), bl.ctypes.data_as(_i32p)))
    out = []
    pos = 0
    for s in sizes[: nc.value]:
        out.append(tuple(int(x) for x in bl[pos:pos + s]))
        pos += s
    return out


# ----------------------------------------------------------------------------
# objects


@dataclass
class Result:
    status: int
    sign: int
    log_abs: float
    log_abs_bp: float
    bp_iters: int
    bp_residual: float
    n_cluster_terms: int
    n_config_terms: int
    open_values: np.ndarray | None = None
    dangling_max: float = 0.0
    term_err_est: float = 0.0

    @property
    def ok(self) -> bool:
        return self.status >= 0


KERNEL_NAMES = ["init", "bp_sweep", "bp_close", "bp_persistent", "gauge", "regauge", "clusters", "combine"]
PNE_FLAG_PROFILE = 1
PNE_FLAG_NO_PERSISTENT = 2
PNE_FLAG_BP_JACOBI = 4
PNE_FLAG_SEPARATE_REGAUGE = 8
PNE_FLAG_GRAPH = 16
PNE_FLAG_AUTOTUNE = 32
PATH_PERSISTENT, PATH_BLOCK_GAUGE, PATH_BLOCK_TERMS = 1, 2, 4


def _options(K, precision, tol, max_iter, check_every, profile=False, persistent=True, jacobi=False,
             fused_regauge=True, graph=False, autotune=False, mode="loop", damping=0.0, err_bound=1e-5,
             small_sites=0, tiles_in_flight=0, reg_budget=0, stall_steps=0):
    """profile: False, True (every kernel) or a list of KERNEL_NAMES to time."""
    lib = load_library()
    o = Options()
    lib.pne_options_default(ctypes.byref(o))
    o.max_excited = int(K)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.bp_tol = float(tol)
    o.bp_max_iter = int(max_iter)
    o.bp_check_every = int(check_every)
    if profile and not isinstance(profile, bool):
        o.profile_kernels = sum(1 << KERNEL_NAMES.index(k) for k in profile)
    o.flags = (PNE_FLAG_PROFILE if profile else 0) | (0 if persistent else PNE_FLAG_NO_PERSISTENT) | \
        (PNE_FLAG_BP_JACOBI if jacobi else 0) | (0 if fused_regauge else PNE_FLAG_SEPARATE_REGAUGE) | \
        (PNE_FLAG_GRAPH if graph else 0) | (PNE_FLAG_AUTOTUNE if autotune else 0)
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.bp_damping = float(damping)
    o.err_bound = float(err_bound)
    o.small_sites = int(small_sites)
    o.tiles_in_flight = int(tiles_in_flight)
    o.reg_budget = int(reg_budget)
    o.bp_stall_steps = int(stall_steps)
    return o


class Context:
    """A library context on one HIP device, enqueuing on one stream."""

    def __init__(self, device: int = 0, mem_budget: int = 0, stream=None):
        self.lib = load_library()
        h = ctypes.c_void_p()
        sp = None
        if stream is not None:
            sp = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        _check(self.lib, self.lib.pne_ctx_create(int(device), int(mem_budget), sp, ctypes.byref(h)))
        self.handle = h
        self._alive = True
        self._children = weakref.WeakSet()  # servers, batches and networks made on this context

    def close(self):
        """Destroy the context, after every server, batch and network made on it."""
        if self._alive:
            kids = list(self._children)
            for kind in (Server, Batch, Network):
                for k in kids:
                    if isinstance(k, kind):
                        k.close()
            self.lib.pne_ctx_destroy(self.handle)
            self._alive = False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return _err(self.lib, self.handle)

    def network(self, obj, on_device: bool = False) -> "Network":
        return Network(self, obj, on_device)

    def batch(self, nets, K=4, precision="fp64", tol=1e-13, max_iter=500, check_every=0,
              profile=False, persistent=True, jacobi=False, fused_regauge=True, graph=False,
              autotune=False, mode="loop", damping=0.0, err_bound=1e-5, small_sites=0, tiles_in_flight=0,
              reg_budget=0, stall_steps=0) -> "Batch":
        """persistent=False: BP launch by launch; jacobi=True: Jacobi sweeps
        in the persistent kernel even on bipartite networks; fused_regauge=
        False: gauge + slices in their own launch; graph=True: replay a
        captured HIP graph; autotune=True: pick the variant by measurement
        (cached per batch signature in the context); mode="full": every
        configuration of degree <= K, dangling ones included; damping: BP
        damping in [0, 1); err_bound: reduced-precision warning bound;
        small_sites, tiles_in_flight, reg_budget: the persistent kernel's tile
        shape (see pne_options); stall_steps: BP's rounding-floor stop (0:
        50 sweeps, < 0: off)."""
        return Batch(self, nets, K, precision, tol, max_iter, check_every, profile, persistent, jacobi,
                     fused_regauge, graph, autotune, mode, damping, err_bound, small_sites, tiles_in_flight,
                     reg_budget, stall_steps)

    def autotune(self, nets, K=4, precision="fp64", tol=1e-13, max_iter=500, trials=3) -> dict:
        """Time the tile-shape variants for this batch; returns the choice."""
        o = _options(K, precision, tol, max_iter, 0)
        best = Options()
        arr = (ctypes.c_void_p * len(nets))(*[n.handle.value for n in nets])
        _check(self.lib, self.lib.pne_autotune(self.handle, arr, len(nets), ctypes.byref(o), int(trials),
                                               ctypes.byref(best)), self.handle)
        return {"graph": bool(best.flags & PNE_FLAG_GRAPH),
                "fused_regauge": not bool(best.flags & PNE_FLAG_SEPARATE_REGAUGE), "flags": int(best.flags),
                "small_sites": int(best.small_sites), "tiles_in_flight": int(best.tiles_in_flight),
                "reg_budget": int(best.reg_budget)}

    def tune_cache_save(self, path: str):
        _check(self.lib, self.lib.pne_tune_cache_save(self.handle, os.fsencode(path)), self.handle)

    def tune_cache_load(self, path: str) -> int:
        n = ctypes.c_int32(0)
        _check(self.lib, self.lib.pne_tune_cache_load(self.handle, os.fsencode(path), ctypes.byref(n)), self.handle)
        return int(n.value)

    def rank_expand(self, nets, Lx: int, Ly: int, partitions, rank: int = 2, form: str = "combinatorial",
                    alpha: float = 0.8, ramp_sweeps: int = 10, max_sweeps: int = 2000, tol: float = 1e-12,
                    profile: bool = False):
        """Rank-r weight-passing projectors and the partitioned expansion on a
        batch of Lx x Ly lattice networks (Sec. V): per network (status,
        sweeps, sign, ln|Z|, log_scale) as a structured array."""
        nets = list(nets)
        opt = RankOptions()
        _check(self.lib, self.lib.pne_rank_options_default(ctypes.byref(opt)))
        opt.rank, opt.form = int(rank), {"combinatorial": 0, "linear": 1}[form]
        opt.alpha, opt.ramp_sweeps, opt.max_sweeps, opt.tol = float(alpha), int(ramp_sweeps), int(max_sweeps), float(tol)
        opt.profile = 1 if profile else 0
        parts, begin, bonds = _partition_arrays(partitions)
        arr = (ctypes.c_void_p * len(nets))(*[n.handle.value for n in nets])
        res = (RankResult * len(nets))()
        st = self.lib.pne_rank_expand(self.handle, arr, len(nets), int(Lx), int(Ly), len(parts),
                                      begin.ctypes.data_as(_i32p), bonds.ctypes.data_as(_i32p), ctypes.byref(opt), res)
        if st < 0 and st not in (PNE_ERR_SINGULAR,):
            _check(self.lib, st, self.handle)
        dt = np.dtype([("status", np.int32), ("sweeps", np.int32), ("sign", np.int32), ("pad", np.int32),
                       ("log_abs", np.float64), ("log_scale", np.float64)])
        return np.frombuffer(bytes(res), dtype=dt).copy()

    def rank_last_times(self) -> dict:
        """Phase device times (ms) of the last rank_expand(profile=True)."""
        ms = np.zeros(5)
        _check(self.lib, self.lib.pne_rank_last_times(self.handle, ms.ctypes.data_as(_f64p), 5), self.handle)
        return dict(zip(("gather", "weight_passing", "site_matrices", "terms", "combine"), ms.tolist()))

    def strip_expand(self, A, L: int, two_d: bool = True, bp_tol: float = 1e-14, power_tol: float = 1e-13,
                     power_max_iter: int = 20000, check_every: int = 4, single_site_passes: bool = False) -> dict:
        """Strip expansion of the infinite lattice of tensor A (legs -x, +x, -y, +y;
        Sec. IV.C): free energy per site and the per-width quantities."""
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
        if A.ndim != 4 or len(set(A.shape)) != 1:
            raise ValueError("A must be a rank-4 tensor with equal leg dimensions")
        chi = int(A.shape[0])
        opt = StripOptions()
        _check(self.lib, self.lib.pne_strip_options_default(ctypes.byref(opt)))
        opt.L, opt.two_d, opt.bp_tol = int(L), 1 if two_d else 0, float(bp_tol)
        opt.power_tol, opt.power_max_iter, opt.check_every = float(power_tol), int(power_max_iter), int(check_every)
        opt.single_site_passes = 1 if single_site_passes else 0
        lam = np.zeros(L)
        gam = np.zeros(L)
        patch = np.zeros((L, L))
        res = StripResult()
        res.lam = lam.ctypes.data_as(_f64p)
        res.gam = gam.ctypes.data_as(_f64p)
        res.patch = patch.ctypes.data_as(_f64p)
        iters = np.zeros(2 * L, np.int32)
        res.iters = iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        st = _check(self.lib, self.lib.pne_strip_expand(self.handle, A.ctypes.data_as(_f64p), chi, ctypes.byref(opt),
                                                        ctypes.byref(res)), self.handle)
        out = {"status": int(st), "f": res.f, "f_bp": res.f_bp, "bp_iters": res.bp_iters,
               "bp_residual": res.bp_residual, "cell_sum": res.cell_sum, "power_iters": res.power_iters,
               "n_unconverged": res.n_unconverged, "lam_ratio": lam, "iters": iters}
        if two_d:
            out["gam_ratio"] = gam
            out["patch_ratio"] = patch
        return out

    def contract(self, net, K=4, precision="fp64", tol=1e-13, max_iter=500, **kw) -> Result:
        b = self.batch([net], K, precision, tol, max_iter, **kw)
        try:
            return b.run()[0]
        finally:
            b.close()


class Network:
    """A validated network held by the library.

    on_device=False: tensors (numpy) are copied to device memory.
    on_device=True : tensors must be CUDA torch tensors (FP64, contiguous);
                     their memory is borrowed and kept referenced here.
    """

    def __init__(self, ctx: Context, obj, on_device: bool = False):
        self.ctx = ctx
        tensors, bonds, open_legs = _net_parts(obj)
        self.n_open = 0 if open_legs is None else int(np.asarray(open_legs).reshape(-1, 2).shape[0])
        self.open_shape = tuple(int(tensors[s].shape[l]) for (s, l) in np.asarray(open_legs).reshape(-1, 2)) \
            if self.n_open else ()
        if on_device:
            self._keep = [t for t in tensors]
            ptrs = [int(t.data_ptr()) for t in tensors]
            da = _DescArrays(tensors, bonds, open_legs, data_ptrs=ptrs)
        else:
            da = _DescArrays(tensors, bonds, open_legs)
        h = ctypes.c_void_p()
        _check(ctx.lib, ctx.lib.pne_network_create(ctx.handle, ctypes.byref(da.desc), 1 if on_device else 0,
                                                   ctypes.byref(h)), ctx.handle)
        self.handle = h
        self._desc = da
        self._alive = True
        ctx._children.add(self)

    def set_partitions(self, partitions):
        """Partitions as lists of bond indices (Eqs. (4), (7), (9)-(11)); [] clears.

        Batches made afterwards expand the network over these partitions
        (closed networks; see pne_network_set_partitions)."""
        parts, begin, bonds = _partition_arrays(partitions)
        _check(self.ctx.lib, self.ctx.lib.pne_network_set_partitions(
            self.handle, len(parts), begin.ctypes.data_as(_i32p), bonds.ctypes.data_as(_i32p)), self.ctx.handle)
        self.partitions = [p.tolist() for p in parts]

    def set_subpartitions(self, x, subpartitions):
        """Recursive partitioning: expand the term of first-level subset x (an
        iterable of partition indices) over its own sub-partitions (lists of
        bond indices); [] removes them."""
        mask = 0
        for p in x:
            mask |= 1 << int(p)
        parts, begin, bonds = _partition_arrays(subpartitions)
        _check(self.ctx.lib, self.ctx.lib.pne_network_set_subpartitions(
            self.handle, mask, len(parts), begin.ctypes.data_as(_i32p), bonds.ctypes.data_as(_i32p)), self.ctx.handle)

    def close(self):
        if self._alive:
            self.ctx.lib.pne_network_destroy(self.handle)
            self._alive = False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Prepared batch: plans and device tables built once, run many times."""

    def __init__(self, ctx: Context, nets, K, precision, tol, max_iter, check_every, profile=False,
                 persistent=True, jacobi=False, fused_regauge=True, graph=False, autotune=False, mode="loop",
                 damping=0.0, err_bound=1e-5, small_sites=0, tiles_in_flight=0, reg_budget=0, stall_steps=0):
        self.ctx = ctx
        self.nets = list(nets)
        self.opt = _options(K, precision, tol, max_iter, check_every, profile, persistent, jacobi, fused_regauge,
                            graph, autotune, mode, damping, err_bound, small_sites, tiles_in_flight, reg_budget,
                            stall_steps)
        arr = (ctypes.c_void_p * len(self.nets))(*[n.handle.value for n in self.nets])
        h = ctypes.c_void_p()
        _check(ctx.lib, ctx.lib.pne_batch_create(ctx.handle, arr, len(self.nets), ctypes.byref(self.opt),
                                                 ctypes.byref(h)), ctx.handle)
        self.handle = h
        self._alive = True
        ctx._children.add(self)
        n = len(self.nets)
        self._res = (ResultStruct * n)()
        self._open = []
        for i, net in enumerate(self.nets):
            m = int(np.prod(net.open_shape)) if net.n_open else 0
            buf = np.zeros(max(1, m), np.float64)
            self._open.append(buf)
            self._res[i].open_values = buf.ctypes.data_as(_f64p) if m else None
            self._res[i].open_capacity = m

    def close(self):
        if self._alive:
            self.ctx.lib.pne_batch_destroy(self.handle)
            self._alive = False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def launch(self):
        _check(self.ctx.lib, self.ctx.lib.pne_batch_launch(self.handle), self.ctx.handle)

    def wait(self, raise_on_error: bool = False):
        st = self.ctx.lib.pne_batch_wait(self.handle, self._res)
        if raise_on_error:
            _check(self.ctx.lib, st, self.ctx.handle)
        elif st < 0 and all(self._res[i].status >= 0 for i in range(len(self.nets))):
            _check(self.ctx.lib, st, self.ctx.handle)
        out = []
        for i, net in enumerate(self.nets):
            r = self._res[i]
            ov = None
            if net.n_open and r.n_open_values:
                ov = self._open[i][: r.n_open_values].copy().reshape(net.open_shape)
            out.append(Result(r.status, r.sign, r.log_abs, r.log_abs_bp, r.bp_iters, r.bp_residual,
                              r.n_cluster_terms, r.n_config_terms, ov, r.dangling_max, r.term_err_est))
        return out

    def run(self, raise_on_error: bool = False):
        self.launch()
        return self.wait(raise_on_error)

    def wait_arrays(self, raise_on_error: bool = False) -> np.ndarray:
        """Like wait(), but returns the per-network results as one numpy
        structured array (fields of RESULT_DTYPE), without building a Python
        object per network.  Open-index values stay in open_values(i)."""
        st = self.ctx.lib.pne_batch_wait(self.handle, self._res)
        arr = np.frombuffer(self._res, dtype=RESULT_DTYPE, count=len(self.nets)).copy()
        if raise_on_error or (st < 0 and not (arr["status"] < 0).any()):
            _check(self.ctx.lib, st, self.ctx.handle)
        return arr

    def run_arrays(self, raise_on_error: bool = False) -> np.ndarray:
        self.launch()
        return self.wait_arrays(raise_on_error)

    def open_values(self, i: int) -> np.ndarray | None:
        """Open-index output of network i from the last wait (rescaled: the
        contraction is open_values * exp(log_abs))."""
        net = self.nets[i]
        m = int(self._res[i].n_open_values)
        return self._open[i][:m].copy().reshape(net.open_shape) if net.n_open and m else None

    def kernel_times(self, reset: bool = False):
        """{kernel: (total ms, launches)} from HIP events (profile=True batches)."""
        n = len(KERNEL_NAMES)
        ms = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int64)
        _check(self.ctx.lib, self.ctx.lib.pne_batch_kernel_times(
            self.handle, ms.ctypes.data_as(_f64p), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n,
            1 if reset else 0), self.ctx.handle)
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_NAMES)}

    def paths(self) -> np.ndarray:
        """Per network: PATH_* bits (persistent block, in-block gauge, in-block terms)."""
        out = np.zeros(len(self.nets), np.int32)
        _check(self.ctx.lib, self.ctx.lib.pne_batch_paths(self.handle, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_int32)), len(self.nets)), self.ctx.handle)
        return out

    def phase_times(self) -> dict:
        """Persistent-block phase durations of the last run (microseconds)."""
        out = np.zeros(6, np.float64)
        _check(self.ctx.lib, self.ctx.lib.pne_batch_phase_times(self.handle, out.ctypes.data_as(_f64p), 6),
               self.ctx.handle)
        keys = ["bp_mean", "regauge_mean", "bp_max", "regauge_max", "bp_span", "total_span"]
        return {k: float(v) for k, v in zip(keys, out)}

    def messages(self, i: int) -> np.ndarray:
        """Final BP messages of network i: per bond, [a_b, c_b] concatenated."""
        net = self.nets[i]
        d = net._desc
        total = 0
        b = np.asarray(d.bond_site).reshape(-1, 2)
        legs = np.asarray(d.bond_leg).reshape(-1, 2)
        offs = np.concatenate([[0], np.cumsum(d.ranks)])
        for k in range(b.shape[0]):
            total += 2 * int(d.dims[offs[b[k, 0]] + legs[k, 0]])
        out = np.zeros(max(1, total), np.float64)
        _check(self.ctx.lib, self.ctx.lib.pne_batch_messages(self.handle, i, out.ctypes.data_as(_f64p), total),
               self.ctx.handle)
        return out[:total]

    def cluster_weights(self, i: int):
        """(values, offsets) of network i's cluster weights, library cluster order."""
        n = ctypes.c_int64(0)
        _check(self.ctx.lib, self.ctx.lib.pne_batch_cluster_weights(self.handle, i, None, 0, ctypes.byref(n), None),
               self.ctx.handle)
        vals = np.zeros(max(1, n.value), np.float64)
        # offsets sized by cluster count: upper bound = number of values
        offs = np.zeros(max(1, n.value), np.int64)
        _check(self.ctx.lib, self.ctx.lib.pne_batch_cluster_weights(
            self.handle, i, vals.ctypes.data_as(_f64p), n.value, ctypes.byref(n),
            offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), self.ctx.handle)
        return vals[: n.value], offs


PNE_ERR_NOT_READY = -6


class Prepared:
    """A request marshalled for Server.submit: descriptor arrays with every
    site tensor in one contiguous FP64 buffer, and its options."""

    def __init__(self, obj, opt):
        tensors, bonds, open_legs = _net_parts(obj)
        flat = [np.ascontiguousarray(t, dtype=np.float64).reshape(-1) for t in tensors]
        self.buf = np.concatenate(flat) if flat else np.zeros(0)
        offs = np.concatenate([[0], np.cumsum([f.size for f in flat])])[:-1]
        base = self.buf.ctypes.data
        self.da = _DescArrays(tensors, bonds, open_legs, data_ptrs=[base + 8 * int(o) for o in offs])
        self.opt = opt
        self.open_shape = tuple(int(tensors[a].shape[b]) for a, b in np.asarray(open_legs).reshape(-1, 2)) \
            if self.da.n_open else ()


class Server:
    """Continuous-batching request server on a context (see pne_server_* in
    pne.h).  While it exists, its worker thread is the context's only user."""

    def __init__(self, ctx: Context, mem_budget: int = 0, max_batch: int = 1024, pipeline_depth: int = 2,
                 completion_queue: bool = False):
        self.ctx = ctx
        self.lib = ctx.lib
        so = ServerOptions()
        self.lib.pne_server_options_default(ctypes.byref(so))
        so.mem_budget = int(mem_budget)
        so.max_batch = int(max_batch)
        so.pipeline_depth = int(pipeline_depth)
        so.completion_queue = 1 if completion_queue else 0
        self._cq = np.zeros(4096, np.uint64)
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.pne_server_create(ctx.handle, ctypes.byref(so), ctypes.byref(h)))
        self.handle = h
        self._alive = True
        self._open_shape = {}
        ctx._children.add(self)

    @staticmethod
    def prepare(obj, K=6, precision="fp64", tol=1e-13, max_iter=500, persistent=True) -> "Prepared":
        """Marshal a request once (descriptor arrays and options), so that
        submit() only hands it to the server."""
        return Prepared(obj, _options(K, precision, tol, max_iter, 0, False, persistent))

    def submit(self, obj, K=6, precision="fp64", tol=1e-13, max_iter=500, persistent=True) -> int:
        """Queue a network (or a Prepared request, whose own options apply)."""
        pr = obj if isinstance(obj, Prepared) else Server.prepare(obj, K, precision, tol, max_iter, persistent)
        t = ctypes.c_uint64(0)
        _check(self.lib, self.lib.pne_submit(self.handle, ctypes.byref(pr.da.desc), ctypes.byref(pr.opt),
                                             ctypes.byref(t)))
        if pr.open_shape:
            self._open_shape[t.value] = pr.open_shape
        return int(t.value)

    def completed(self) -> list:
        """Tickets finished since the last call (servers made with
        completion_queue=True), oldest first."""
        out = []
        n = ctypes.c_int32(0)
        while True:
            _check(self.lib, self.lib.pne_server_completed(
                self.handle, self._cq.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(self._cq),
                ctypes.byref(n)))
            out.extend(int(x) for x in self._cq[: n.value])
            if n.value < len(self._cq):
                return out

    def poll(self, ticket: int):
        """Result for `ticket`, or None while it is pending or running."""
        shape = self._open_shape.get(ticket)
        m = int(np.prod(shape)) if shape else 0
        buf = np.zeros(max(1, m), np.float64)
        r = ResultStruct()
        r.open_values = buf.ctypes.data_as(_f64p) if m else None
        r.open_capacity = m
        st = self.lib.pne_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(r))
        if st == PNE_ERR_NOT_READY:
            return None
        if st == -1 and r.status >= 0:
            raise PNEError(st, "unknown ticket or open buffer too small")
        self._open_shape.pop(ticket, None)
        ov = buf[: r.n_open_values].copy().reshape(shape) if (m and r.n_open_values) else None
        return Result(r.status, r.sign, r.log_abs, r.log_abs_bp, r.bp_iters, r.bp_residual, r.n_cluster_terms,
                      r.n_config_terms, ov, r.dangling_max, r.term_err_est)

    def cancel(self, ticket: int) -> bool:
        """Cancel a queued request: True when it left the queue (its poll then
        reports PNE_ERR_CANCELLED), False when it is already running."""
        st = self.lib.pne_cancel(self.handle, ctypes.c_uint64(ticket))
        if st == PNE_ERR_NOT_READY:
            return False
        _check(self.lib, st)
        return True

    def stats(self) -> dict:
        st = ServerStats()
        _check(self.lib, self.lib.pne_server_get_stats(self.handle, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if self._alive:
            self.lib.pne_server_destroy(self.handle)
            self._alive = False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
