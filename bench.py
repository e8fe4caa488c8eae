"""Benchmark: PNE networks/s (and terms/s) on one MI355X.

Workload (one step): the 16x16 open-boundary random-tensor networks with
i.i.d. U[0,1] entries, 256 networks at bond dimension D=4 (seeds 2000-2255)
plus the same 256 seeds at D=3, expanded to clusters of up to K=6 excited
bonds.  Term contractions in FP32 (default) with FP64 BP, gauge, vacuum
log-norms and cross-term sum; every network runs the whole path (BP from
uniform messages, gauge, slices, clusters, sum) every step.  Tensors are
resident in device memory before timing; the batch's geometry plan and
device tables are prepared once (they depend only on the lattice).

Then (unless --serving 0) the serving loop on the serving requests: the
saturated capacity, Poisson arrivals at 0.3, 0.5, 0.7 and 0.9 x that capacity
(p50/p99 latency and networks/s, the 0.7 point reported at the top of
"serving"), and a sample of served results against their FP64 form.

Prints one JSON line.  Kernel durations come from HIP events the library
records on its own stream around each launch during the timed steps.
Results come back as one numpy structured array per step (no Python object
per network).
"""

from __future__ import annotations

import argparse
import contextlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PNE terms/s and networks/s at <=1e-5 rel err vs FP64 oracle; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6  # dense FP64 matrix-core peak


def site_colours(net):
    """Two-colouring of the site graph (site 0 has colour 0), or None when the
    graph is not bipartite."""
    import collections

    adj = collections.defaultdict(list)
    for (u, _, v, _) in net.bonds:
        adj[int(u)].append(int(v))
        adj[int(v)].append(int(u))
    col = {}
    for s0 in range(len(net.tensors)):
        if s0 in col:
            continue
        col[s0] = 0
        q = [s0]
        for x in q:
            for y in adj[x]:
                if y not in col:
                    col[y] = 1 - col[x]
                    q.append(y)
                elif col[y] == col[x]:
                    return None
    return col


def bp_bytes(net, steps: int, messages_in_lds: bool = False, red_black: bool = True) -> int:
    """Algorithmic bytes of the BP of one network over `steps` steps: network
    sweeps under Jacobi; under red-black (bipartite networks in the
    persistent kernel), step k updates the sites of colour k mod 2 only.  Per
    updated site: the FP64 tensor read once, and, when the messages live in
    memory, every incoming message read twice (contraction and residual) and
    every outgoing message written once.  With messages_in_lds (the
    persistent block keeps its network's messages in LDS) only the tensors
    stream, plus one write of the final messages."""
    msg = 0 if messages_in_lds else 3 * 8
    per = [8 * t.size + msg * sum(t.shape) for t in net.tensors]
    col = site_colours(net) if (red_black and len(net.tensors) > 1) else None
    if col is None:
        b = steps * sum(per)
    else:
        cb = [0, 0]
        for i, x in enumerate(per):
            cb[col[i]] += x
        b = ((steps + 1) // 2) * cb[0] + (steps // 2) * cb[1]
    if messages_in_lds:
        b += sum(8 * sum(t.shape) for t in net.tensors)
    return b


_CLUSTER_BYTES = {}


def cluster_bytes(pne, net, K: int, slice_bytes: int) -> int:
    """Algorithmic bytes of the cluster contractions and term sum of one
    network: every cluster reads, at each of its sites, the excited block of
    that site's slice (e^(cluster legs at the site) entries) and writes one
    FP64 weight, which the sum reads back.  Depends only on the lattice."""
    key = (tuple(t.shape for t in net.tensors), K, slice_bytes)
    if key not in _CLUSTER_BYTES:
        bonds = np.asarray(net.bonds).reshape(-1, 4)
        total = 0
        for cl in pne.enumerate_clusters(net, K):
            deg = {}
            for b in cl:
                u, lu, v, _ = (int(x) for x in bonds[b])
                e = net.tensors[u].shape[lu] - 1
                deg.setdefault(u, []).append(e)
                deg.setdefault(v, []).append(e)
            for es in deg.values():
                total += slice_bytes * int(np.prod(es))
            total += 16
        _CLUSTER_BYTES[key] = total
    return _CLUSTER_BYTES[key]


def regauge_bytes(net, slice_bytes: int, messages_in_lds: bool = False) -> int:
    """Site tensors read once (FP64), slices written once, one FP64 vacuum
    log-factor written per site and, unless they are already in LDS, the two
    FP64 messages of every bond slot read (the gauge is built from them)."""
    msg = 0 if messages_in_lds else 2 * 8
    b = 0
    for t in net.tensors:
        b += 8 * t.size + slice_bytes * t.size + msg * sum(t.shape) + 12
    return b


# sources compiled into the persistent BP kernel; a committed HBM-traffic
# profile counts only while their hash matches the one it records
KERNEL_SOURCES = ["paper_2512_10910_amd/csrc/bp_persistent.hip", "paper_2512_10910_amd/csrc/regauge.h",
                  "paper_2512_10910_amd/csrc/terms.h", "paper_2512_10910_amd/csrc/gmem.h",
                  "paper_2512_10910_amd/csrc/kernels.h", "paper_2512_10910_amd/csrc/pne_internal.h"]
TRAFFIC_PROFILE = "profiles/hbm_traffic_16x16_D4D3_K6_fp32.md"


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration), or
    None when the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("<!-- ") and "=" in line:
                k, v = line[5:].split("-->")[0].strip().split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return None
    v = vals.get(f"traffic_bytes_per_launch.{kernel}")
    return int(float(v)) if v else None


def serving_bench(pne, P, n_req: int, budget: int, precision: str, K: int, depth: int = 2,
                  rates=(0.3, 0.5, 0.7, 0.9), n_check: int = 32):
    """Serving requests i = 0..n_req-1 (seed 40000+i): saturated capacity
    (all submitted at once), then Poisson arrivals (seed 4) at a sweep of
    fractions of that capacity (0.7 is the reported point); latency is
    submit -> result ready, measured by the server.  A sample of n_check
    served results is compared with the same requests run in FP64."""
    nets = [P.config4_request(i) for i in range(n_req)]
    # requests are marshalled by the client before they arrive (descriptor
    # arrays, one contiguous tensor buffer each); the server copies them at submit
    reqs = [pne.Server.prepare(n, K=K, precision=precision) for n in nets]
    ctx = pne.Context(0)

    def drain(sv, tickets, keep=None, deadline=300.0):
        left = set(tickets)
        t0 = time.perf_counter()
        while left:
            for t in sv.completed():
                if t in left:
                    r = sv.poll(t)
                    if r.status < 0:
                        raise RuntimeError(f"request failed with status {r.status}")
                    if keep is not None and t in keep:
                        keep[t] = r
                    left.discard(t)
            if time.perf_counter() - t0 > deadline:
                raise RuntimeError("serving run did not finish")
            time.sleep(0.0002)

    # warm the context's plan cache: one request per distinct lattice (plans
    # depend only on the geometry and K, and a server keeps them across requests)
    seen, warm = set(), []
    for n, r in zip(nets, reqs):
        key = (n.info["dim"], n.info["L"], n.info["D"])
        if key not in seen:
            seen.add(key)
            warm.append(r)
    sv = pne.Server(ctx, mem_budget=budget, completion_queue=True)
    drain(sv, [sv.submit(r) for r in warm])
    sv.close()
    sv = pne.Server(ctx, mem_budget=budget, pipeline_depth=depth, completion_queue=True)
    t0 = time.perf_counter()
    tickets = [sv.submit(r) for r in reqs]
    check_idx = list(range(0, n_req, max(1, n_req // n_check)))[:n_check]
    kept = {tickets[i]: None for i in check_idx}
    drain(sv, tickets, kept)
    cap = n_req / (time.perf_counter() - t0)
    sat = sv.stats()
    sv.close()
    # accuracy of the served results against the FP64 form of the same requests
    errs, warned = [], 0
    ref_nets = [ctx.network(nets[i]) for i in check_idx]
    ref = ctx.batch(ref_nets, K=K, precision="fp64").run_arrays()
    for j, i in enumerate(check_idx):
        r = kept[tickets[i]]
        warned += int(r.status == 2)
        errs.append(abs(r.log_abs - float(ref["log_abs"][j])) / max(1.0, abs(float(ref["log_abs"][j]))))
    for x in ref_nets:
        x.close()
    sweep = []
    for frac in rates:
        rate = frac * cap
        arrivals = P.config4_arrivals(n_req, rate)
        sv = pne.Server(ctx, mem_budget=budget, pipeline_depth=depth, completion_queue=True)
        tickets = []
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            while time.perf_counter() - t0 < arrivals[i]:
                pass
            tickets.append(sv.submit(r))
        drain(sv, tickets)
        st = sv.stats()
        sv.close()
        sweep.append({"fraction_of_capacity": frac, "rate_per_s": round(rate, 1),
                      "networks_per_s": round(st["networks_per_s"], 1),
                      "latency_p50_ms": round(st["latency_p50_ms"], 3),
                      "latency_p99_ms": round(st["latency_p99_ms"], 3),
                      "latency_mean_ms": round(st["latency_mean_ms"], 3), "batches": st["batches"]})
        print(f"bench: serving at {frac:.1f} x capacity: p50 {st['latency_p50_ms']:.2f} ms, "
              f"p99 {st['latency_p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    ctx.close()
    at07 = next((x for x in sweep if abs(x["fraction_of_capacity"] - 0.7) < 1e-9), sweep[-1])
    return {
        "workload": f"{n_req} serving requests (seed 40000+i: 2D L~U{{4..32}} or 3D L~U{{4..8}}, D~U{{2,3,4}}, "
                    f"U[0,1] or N(1,0.3)), K={K}, {precision} terms, device budget {budget / 1e9:.1f} GB",
        "capacity_networks_per_s": round(cap, 1),
        "saturated_batches": sat["batches"],
        "saturated_host_prep_s": round(sat["prep_s"], 3),
        "saturated_wait_s": round(sat["wait_s"], 3),
        "saturated_prep_split_s": {k: round(sat[k + "_s"], 3) for k in ("upload", "networks", "batch", "launch")},
        "rate_per_s": at07["rate_per_s"],
        "networks_per_s": at07["networks_per_s"],
        "latency_p50_ms": at07["latency_p50_ms"],
        "latency_p99_ms": at07["latency_p99_ms"],
        "latency_mean_ms": at07["latency_mean_ms"],
        "batches": at07["batches"],
        "rate_sweep": sweep,
        "sampled_max_rel_err_log_vs_fp64_form": max(errs) if errs else None,
        "sampled_requests": len(errs),
        "sampled_precision_warnings": warned,
    }


def kernel_bytes(pne, nets_in, paths, iters, n_clusters, K: int, slice_bytes: int) -> dict:
    """Algorithmic HBM bytes per kernel for one run of a batch, each network's
    share going to the kernel that runs that step of it (paths: the
    library's PATH_* bits per network)."""
    alg = {}

    def add(k, v):
        alg[k] = alg.get(k, 0) + v

    for net, path, s, nc in zip(nets_in, paths, iters, n_clusters):
        pers = bool(path & pne.PATH_PERSISTENT)
        cl = cluster_bytes(pne, net, K, slice_bytes) - 8 * nc
        if pers:
            add("bp_persistent", bp_bytes(net, s, True))
        else:
            add("bp_sweep", bp_bytes(net, s, False, red_black=False))
        if path & pne.PATH_BLOCK_GAUGE:
            add("bp_persistent", regauge_bytes(net, slice_bytes, True))
        else:
            add("regauge", regauge_bytes(net, slice_bytes, False))
        if path & pne.PATH_BLOCK_TERMS:
            add("bp_persistent", cl + 8 * nc)
        else:
            add("clusters", cl)
            add("combine", 8 * nc)
    return alg


def strip_bytes(chi: int, k: int, paired: bool = True) -> int:
    """Algorithmic HBM bytes of one width-k transfer-matrix application: the
    first pass reads chi^k and writes chi^(k+1) entries, each middle pass
    reads and writes chi^(k+1), the last reads chi^(k+1) plus the input
    vector and writes chi^k (FP64).  Paired passes (chi <= 4) apply two sites
    each, so a width-k application makes about k/2 passes instead of k."""
    if k == 1 or (k == 2 and paired and chi <= 4):
        return 8 * 3 * chi ** k
    if paired and chi <= 4:
        n_mid = (k - 4) // 2 if k % 2 == 0 else (k - 3) // 2
        return 8 * (3 * chi ** k + 2 * (1 + n_mid) * chi ** (k + 1))
    return 8 * (3 * chi ** k + 2 * (k - 1) * chi ** (k + 1))


def strips_bench(pne, P, L: int = 12, betas=(0.3, 0.4, 0.4407, 0.5, 0.6)):
    """Infinite 2D Ising, 2x2 blocked (chi = 4, four spins per tensor), width-L
    strips in both directions (Sec. IV.C): wall time per coupling, the free
    energy per spin against Onsager's, and the streaming passes' algorithmic
    bytes over that wall time."""
    import torch

    from oracle import strips as S

    ctx = pne.Context(0)
    ctx.strip_expand(P.ising_blocked_tensor(0.3), 2)
    for beta in betas:
        A = P.ising_blocked_tensor(beta)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.strip_expand(A, L)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        its = [int(x) for x in r["iters"]]
        alg = sum(its[d * L + k - 1] * strip_bytes(4, k) for d in (0, 1) for k in range(1, L + 1))
        gbs = alg / (ms * 1e-3) / 1e9
        exact = S.onsager_f(beta)
        out = {"workload": f"infinite 2D Ising, 2x2 blocked (chi=4), width-{L} strips both directions, fp64",
               "beta": beta, "ms": round(ms, 2), "f_per_spin": r["f"] / 4, "f_bp_per_spin": r["f_bp"] / 4,
               "onsager_f_per_spin": exact, "abs_err_per_spin": abs(r["f"] / 4 - exact),
               "bp_abs_err_per_spin": abs(r["f_bp"] / 4 - exact), "status": r["status"],
               "power_iters": r["power_iters"], "power_iters_width_L": [its[L - 1], its[2 * L - 1]],
               "alg_bytes": alg, "achieved_GBps_over_wall": round(gbs, 1),
               "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        print(json.dumps(out), flush=True)
    ctx.close()


def rank_bench(pne, P, n: int = 4096):
    """Rank-r projectors from weight passing (Sec. V.B's setting, reduced):
    n coarse-grained 6x6 Ising lattices (3x3 blocks of 2x2 spins, chi = 4)
    with beta spread over [0.6, 0.9] (below T_c), four single-index
    partitions (the centre's bonds), linear form, rank 1 and rank 2: wall
    time and networks/s, and sampled errors against the exact contraction."""
    import torch

    import oracle as O

    betas = np.linspace(0.6, 0.9, n)
    raws = [P.ising_blocked_lattice(6, 2, float(b)) for b in betas]
    ctx = pne.Context(0)
    nets = [ctx.network(x) for x in raws]
    parts = P.grid3_single_partitions(raws[0])
    ctx.rank_expand(nets[:8], 3, 3, parts, rank=2, form="linear")
    samples = [0, n // 2, n - 1]
    exact = [O.exact_log_contract(raws[i])[1] for i in samples]
    for r in (1, 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.rank_expand(nets, 3, 3, parts, rank=r, form="linear")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        errs = [abs(float(out["log_abs"][i]) - e) for i, e in zip(samples, exact)]
        print(json.dumps({"workload": f"coarse-grained 6x6 Ising below T_c (3x3, chi=4), rank-{r} weight-passing "
                          "projectors, four centre bonds, Eq. (4), fp64", "networks": n, "ms": round(ms, 2),
                          "networks_per_s": round(n / (ms * 1e-3), 1), "mean_sweeps": float(out["sweeps"].mean()),
                          "status_min": int(out["status"].min()),
                          "abs_err_lnZ_vs_exact_samples": errs}), flush=True)
    for x in nets:
        x.close()
    ctx.close()


def measured_copy_gbps(torch, mib: int = 1024, reps: int = 5) -> float:
    """Achieved HBM bandwidth of a plain device copy of `mib` MiB (bytes read
    plus bytes written over the copy's time, HIP events on torch's stream):
    the practical ceiling beside the published 8 TB/s."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.synchronize()
    return 2 * mib * (1 << 20) / (ms * 1e-3) / 1e9


def rank_terms_flops(chi: int, Lx: int, Ly: int) -> int:
    """Algorithmic FP64 flops of one term of the bond-dimension-8/16 path: the
    lattice contracted row by row, site (x, y) absorbed as a dense GEMM of
    chi^(Lx-1) other-column rows by its present incoming legs (-x, -y) by its
    present outgoing legs (+x, +y), 2 flops per multiply-add."""
    tot = 0
    for y in range(Ly):
        for x in range(Lx):
            k = (chi if x > 0 else 1) * (chi if y > 0 else 1)
            n = (chi if x < Lx - 1 else 1) * (chi if y < Ly - 1 else 1)
            tot += 2 * chi ** (Lx - 1) * k * n
    return tot


def rank_large_bench(pne, P, n: int = 256, reps: int = 3) -> dict:
    """Rank-r projectors at the paper's bond dimension (Sec. V.B): n 12x12
    Ising lattices blocked into 3x3 sites of 4x4 spins (chi = 16), beta spread
    over [0.5, 0.9] (below T_c), rank 2, the four single-index partitions of
    the centre's bonds in the combinatorial form (Eq. (7), 15 terms): the
    phase device times (HIP events), networks/s, the term kernel's FP64
    matrix-core rate against its roofline, and sampled errors against the
    exact contraction."""
    import torch

    import oracle as O

    betas = np.linspace(0.5, 0.9, n)
    raws = [P.ising_blocked_lattice(12, 4, float(b)) for b in betas]
    ctx = pne.Context(0)
    nets = [ctx.network(x) for x in raws]
    parts = P.grid3_single_partitions(raws[0])
    n_terms = 2 ** len(parts) - 1
    ctx.rank_expand(nets[:4], 3, 3, parts, rank=2)
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.rank_expand(nets, 3, 3, parts, rank=2, profile=True)
        ms = (time.perf_counter() - t0) * 1e3
        ph = ctx.rank_last_times()
        if best is None or ms < best[0]:
            best = (ms, ph, out)
    ms, ph, out = best
    samples = [0, n // 2, n - 1]
    errs = [abs(float(out["log_abs"][i]) - O.exact_log_contract(raws[i])[1]) for i in samples]
    flops = rank_terms_flops(16, 3, 3) * n_terms * n
    tf = flops / (ph["terms"] * 1e-3) / 1e12 if ph["terms"] > 0 else 0.0
    for x in nets:
        x.close()
    ctx.close()
    return {"workload": "12x12 Ising in 3x3 blocks (chi=16), beta in [0.5, 0.9], rank-2 weight-passing projectors, "
                        "four centre-bond partitions, Eq. (7) (15 terms), fp64",
            "networks": n, "ms": round(ms, 2), "networks_per_s": round(n / (ms * 1e-3), 1),
            "phase_ms": {k: round(v, 3) for k, v in ph.items()}, "mean_sweeps": float(out["sweeps"].mean()),
            "status_min": int(out["status"].min()), "status_max": int(out["status"].max()),
            "terms_roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": FP64_MFMA_PEAK_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(tf / FP64_MFMA_PEAK_TFLOPS, 4),
                               "alg_flops_per_term": rank_terms_flops(16, 3, 3)},
            "abs_err_lnZ_vs_exact_samples": errs}


def _cpu_worker(job):
    """One oracle evaluation of a benchmark network in a single-threaded
    worker process; returns its wall time."""
    D, seed, K = job
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import oracle as O
    import pne_inputs as P

    net = P.config2_network(D, seed)
    with (threadpool_limits(1) if threadpool_limits else contextlib.nullcontext()):
        t0 = time.perf_counter()
        O.pne_contract(net, K)
        return time.perf_counter() - t0


def cpu_baseline(K: int, per_core: int, n_seeds: int) -> dict:
    """The FP64 CPU oracle on the host's cores, one single-threaded process
    per core (at most 16, the machine's CPU share), over a bounded sample of the
    benchmark workload (per_core networks per process, alternating D = 4 and
    D = 3, seeds 2000+i).  Runs before anything initialises the GPU, so the
    worker processes are plain forks of a CPU-only interpreter."""
    import multiprocessing as mp

    cores = max(1, min(os.cpu_count() or 1, 16))
    jobs = [((4, 3)[i % 2], 2000 + (i // 2) % n_seeds, K) for i in range(cores * per_core)]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        times = pool.map(_cpu_worker, jobs, chunksize=per_core)
        wall = time.perf_counter() - t0
    return {
        "value": round(len(jobs) / wall, 4),
        "unit": "networks/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{len(jobs)} networks of this workload (half D=4, half D=3, seeds 2000+), FP64 oracle, "
                  f"{cores} single-threaded processes x {per_core} networks, {wall:.1f}s wall, "
                  f"{sum(times):.1f}s of CPU work; host nproc={os.cpu_count()}",
        "latency_s_per_network_1thread": round(float(np.mean(times)), 4),
    }


def measure_batch(pne, ctx, nets_in, nets, K: int, prec: str, steps: int, **tile) -> dict:
    """Step time of one batch (whole path, results back each step), then a
    separate pass with HIP events around every launch for the per-kernel
    split and each kernel's algorithmic bytes over its device time."""
    import torch

    sb = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
    b = ctx.batch(nets, K=K, precision=prec, **tile)
    res = b.run_arrays()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = b.run_arrays()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    paths = b.paths()
    b.close()
    pb = ctx.batch(nets, K=K, precision=prec, profile=True, **tile)
    pb.run_arrays()
    pb.kernel_times(reset=True)
    for _ in range(steps):
        pb.run_arrays()
    kt = pb.kernel_times(reset=True)
    pb.close()
    iters = [int(x) for x in res["bp_iters"]]
    alg = kernel_bytes(pne, nets_in, paths, iters, [int(x) for x in res["n_cluster_terms"]], K, sb)
    kernels = {}
    for k, (tms, cnt) in kt.items():
        if cnt == 0:
            continue
        d = {"ms_per_step": round(tms / steps, 4), "launches_per_step": cnt / steps}
        if k in alg and tms > 0:
            gbs = alg[k] / (tms / steps * 1e-3) / 1e9
            d.update({"alg_bytes_per_step": alg[k], "achieved_GBps": round(gbs, 1),
                      "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)})
        kernels[k] = d
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"]) if kernels else None
    n = len(nets)
    return {"networks": n, "precision": prec, "K": K, "ms_per_step": round(ms, 4),
            "networks_per_s": round(n / (ms * 1e-3), 1),
            "terms_per_s": round(float(res["n_cluster_terms"].sum()) / (ms * 1e-3), 1),
            "bp_iters_mean": float(np.mean(iters)), "status_counts": {int(s): int((res["status"] == s).sum())
                                                                        for s in np.unique(res["status"])},
            "dominant_kernel": dom, "dominant_frac_of_hbm_peak": kernels[dom].get("frac_of_hbm_peak") if dom else None,
            "kernels": kernels, "_res": res}


def other_configs(pne, P, steps: int) -> dict:
    """The remaining benchmark configurations at batch scale, each with its
    per-kernel rooflines and an accuracy check: 4x4 Ising (16384 betas),
    6^3 Ising (three betas x 1365), 12x12 AKLT (4096 copies), and the 32x32
    D=6 open-index networks at d = 1..8 (x16) in FP64, FP32 and BF16 terms
    against the stored oracle outputs."""
    import oracle as O

    out = {}
    ctx = pne.Context(0)

    def run(label, nets_in, K, prec, reuse=None):
        objs = reuse if reuse is not None else [ctx.network(x) for x in nets_in]
        m = measure_batch(pne, ctx, nets_in, objs, K, prec, steps)
        m = {"workload": label, **m}
        print(f"bench: {label}, {prec}: {m['networks_per_s']} networks/s", file=sys.stderr, flush=True)
        return m, objs

    # config 1
    betas = P.config1_betas(16384)
    c1_in = [P.ising_2d(4, 4, float(bb)) for bb in betas]
    m, objs = run("4x4 Ising, beta_i = 0.44(1 + 0.01 u_i), 16384 networks, K=4", c1_in, 4, "fp64")
    res = m.pop("_res")
    errs = [abs(float(res["log_abs"][i]) - O.pne_contract(c1_in[i], 4).log_abs) for i in (0, 1, 16383)]
    m["max_abs_err_log_vs_oracle_samples"] = max(errs)
    out["config1_ising_4x4"] = m
    for x in objs:
        x.close()
    # config 3, Ising
    base = {bb: P.config3_ising_network(bb) for bb in (0.18, 0.2217, 0.26)}
    c3_in = [base[bb] for bb in (0.18, 0.2217, 0.26) for _ in range(1365)]
    m, objs = run("6x6x6 Ising, beta in {0.18, 0.2217, 0.26} x 1365, K=6", c3_in, 6, "fp32")
    res = m.pop("_res")
    errs = []
    for j, bb in enumerate((0.18, 0.2217, 0.26)):
        tt = math.tanh(bb)
        closed = 216 * math.log(2.0) + 540 * math.log(math.cosh(bb)) + math.log1p(450 * tt ** 4 + 2720 * tt ** 6)
        errs.append(abs(float(res["log_abs"][j * 1365]) - closed) / closed)
    m["max_rel_err_log_vs_closed_form"] = max(errs)
    out["config3_ising_6cube"] = m
    for x in objs:
        x.close()
    # config 3, AKLT
    aklt = P.config3_aklt_network()
    ref = O.pne_contract(aklt, 8)
    for prec in ("fp32", "bf16"):
        m, objs = run(f"12x12 AKLT double layer, 4096 copies, K=8", [aklt] * 4096, 8, prec)
        res = m.pop("_res")
        m["rel_err_log_vs_oracle"] = abs(float(res["log_abs"][0]) - ref.log_abs) / abs(ref.log_abs)
        out[f"config3_aklt_12x12_{prec}"] = m
        for x in objs:
            x.close()
    # config 5
    with open(os.path.join(ROOT, "tests", "golden", "config5_oracle.json")) as fh:
        gold = json.load(fh)["results"]
    c5_uniq = [P.config5_network(d) for d in range(1, 9)]
    c5_in = c5_uniq * 16
    objs = [ctx.network(x) for x in c5_in]
    c5 = {}
    for prec in ("fp64", "fp32", "bf16"):
        m = measure_batch(pne, ctx, c5_in, objs, 8, prec, max(1, steps // 2))
        res = m.pop("_res")
        b = ctx.batch(objs[:8], K=8, precision=prec)
        r8 = b.run()
        b.close()
        eps = []
        for d in range(1, 9):
            g = gold[str(d)]
            o = np.asarray(g["values"])
            v = r8[d - 1].open_values * math.exp(r8[d - 1].log_abs - g["log_scale"])
            eps.append(float(np.linalg.norm(v - o) / np.linalg.norm(o)))
        m["eps2_vs_oracle_d1_to_8"] = eps
        c5[prec] = m
        print(f"bench: 32x32 D=6 open, {prec}: {m['networks_per_s']} networks/s", file=sys.stderr, flush=True)
    for x in objs:
        x.close()
    c5["speedup_fp32_over_fp64"] = round(c5["fp64"]["ms_per_step"] / c5["fp32"]["ms_per_step"], 3)
    c5["speedup_bf16_over_fp64"] = round(c5["fp64"]["ms_per_step"] / c5["bf16"]["ms_per_step"], 3)
    c5["workload"] = "32x32 D=6 U[0,1], open dim-2 legs at separation d = 1..8, x16 each (128 networks), K=8"
    out["config5_open_32x32"] = c5
    ctx.close()
    return out


def beyond_mall(pne, P, steps: int, precision: str, K: int) -> dict:
    """The benchmark kernel on a batch whose concurrently resident tensors
    exceed the 256 MB MALL: 512 networks of 18x18 U[0,1] at D = 4 (663 KB of
    FP64 tensors each, 340 MB for the 512 blocks resident at once), so the
    BP re-reads come from DRAM rather than the last-level cache."""
    nets_in = [P.random_2d(18, 18, 4, "uniform01", seed=9000 + i) for i in range(512)]
    ctx = pne.Context(0)
    objs = [ctx.network(x) for x in nets_in]
    m = measure_batch(pne, ctx, nets_in, objs, K, precision, steps)
    m.pop("_res")
    # the tuned tile shape (the 256-VGPR kernel leaves room in LDS for the
    # in-block gauge of these larger networks)
    choice = ctx.autotune(objs, K=K, precision=precision, trials=3)
    tuned = measure_batch(pne, ctx, nets_in, objs, K, precision, steps, **{k: choice[k] for k in (
        "small_sites", "tiles_in_flight", "reg_budget")})
    tuned.pop("_res")
    m["autotuned"] = {"choice": choice, "ms_per_step": tuned["ms_per_step"],
                      "networks_per_s": tuned["networks_per_s"], "dominant_kernel": tuned["dominant_kernel"],
                      "kernels": tuned["kernels"]}
    for x in objs:
        x.close()
    ctx.close()
    m["workload"] = f"512 networks of 18x18 U[0,1] D=4 (seeds 9000+i), K={K}, {precision} terms"
    m["resident_tensor_bytes"] = int(sum(x.nbytes() for x in nets_in))
    return m


def workloads_bench(pne, P, steps: int, only: str = ""):
    """The other workloads at batch scale, one JSON line each: step time,
    networks/s, per-kernel device time (HIP events around every launch) with
    its algorithmic HBM bytes and roofline fraction, and a sampled check
    against the FP64 oracle (skipped for the 32x32 D=6 networks, whose oracle
    takes minutes; the parity tests cover them)."""
    import torch

    import oracle as O

    cases = [
        ("4x4 Ising, beta_i = 0.44(1 + 0.01 u_i), K=4, fp64",
         lambda: [P.ising_2d(4, 4, float(b)) for b in P.config1_betas(65536)], 4, "fp64", True, None, 500),
        ("6x6x6 Ising, beta in {0.18, 0.2217, 0.26} x 1365 each, K=6, fp32",
         lambda: [P.config3_ising_network(b) for b in (0.18, 0.2217, 0.26) for _ in range(1365)], 6, "fp32", True,
         None, 500),
        # a random gauge makes the uniform start a generic one: BP then also
        # has to damp the slow non-singlet modes (about 0.95 per step), and
        # the copies take 500-750 red-black steps to reach 1e-13
        ("12x12 AKLT double layer, random bond gauge per copy (seed 3000+i), K=8, fp32",
         lambda: [P.config3_aklt_network(gauge_seed=3000 + i) for i in range(4096)], 8, "fp32", True, None, 1500),
        ("32x32 D=6 U[0,1], two open dim-2 legs d = 1..8 apart, x16 each, K=8, fp32",
         lambda: [P.config5_network(d) for d in range(1, 9)] * 16, 8, "fp32", False, None, 500),
    ]
    # user partitions (Eqs. (4), (7)): complete expansion over the partitions
    parted = [
        ("3x3 U[0,2] D=4 (seed 50000+i), six multi-index partitions, Eq. (7) complete (K=12), fp64",
         lambda: [P.small_network(3, 3, "random", 4, seed=50000 + i) for i in range(8192)], 12, "fp64", True,
         P.grid3_multi_partitions, 500),
        ("3x2 double loop U[0,2] D=6 (seed 60000+i), three vertical partitions, Eq. (4) complete (K=7), fp64",
         lambda: [P.small_network(3, 2, "random", 6, seed=60000 + i) for i in range(16384)], 7, "fp64", True,
         P.double_loop_partitions, 500),
        ("3x4 U[0,2] D=4 (seed 70000+i), five lines with the two 3x3 principal terms refined by six partitions "
         "(recursive, Sec. IV.A), complete (K=17), fp64",
         lambda: [P.small_network(3, 4, "random", 4, seed=70000 + i) for i in range(8192)], 17, "fp64", True,
         P.grid3x4_recursive_partitions, 500),
    ]
    sb = {"fp64": 8, "fp32": 4, "bf16": 2}
    for label, make, K, prec, check, parts_of, max_iter in cases + parted:
        if only and only not in label:
            continue
        nets_in = make()
        ctx = pne.Context(0)
        nets = [ctx.network(n) for n in nets_in]
        if parts_of is not None:
            for n, x in zip(nets, nets_in):
                pp = parts_of(x)
                parts, subs = pp if isinstance(pp, tuple) else (pp, {})
                n.set_partitions(parts)
                for sx, inner in subs.items():
                    n.set_subpartitions(sx, inner)
        b = ctx.batch(nets, K=K, precision=prec, max_iter=max_iter, profile=True)
        b.run_arrays()
        b.kernel_times(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            res = b.run_arrays()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        kt = b.kernel_times(reset=True)
        iters = [int(x) for x in res["bp_iters"]]
        alg = kernel_bytes(pne, nets_in, b.paths(), iters, [int(x) for x in res["n_cluster_terms"]], K,
                           sb[prec])
        nclu = int(res["n_cluster_terms"].sum())
        kernels = {}
        for k, (tms, cnt) in kt.items():
            if cnt == 0:
                continue
            d = {"ms_per_step": round(tms / steps, 4), "launches_per_step": cnt / steps}
            if k in alg and tms > 0:
                gbs = alg[k] / (tms / steps * 1e-3) / 1e9
                d.update({"alg_bytes_per_step": alg[k], "achieved_GBps": round(gbs, 1),
                          "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)})
            kernels[k] = d
        out = {"workload": label, "networks": len(nets), "ms_per_step": round(ms, 4),
               "networks_per_s": round(len(nets) / (ms * 1e-3), 1), "precision": prec, "K": K,
               "bp_iters_mean": float(np.mean(iters)), "bp_iters_max": max(iters), "bp_max_iter": max_iter,
               "status_min": int(res["status"].min()), "status_max": int(res["status"].max()),
               "cluster_terms_per_step": nclu, "kernels": kernels}
        if check and parts_of is not None:
            from oracle import partitioned as PT

            pp = parts_of(nets_in[0])
            parts, subs = pp if isinstance(pp, tuple) else (pp, {})
            _, lg = PT.recursive_pne(nets_in[0], parts, subs)
            out["rel_err_log_vs_oracle_sample0"] = abs(float(res["log_abs"][0]) - lg) / max(1.0, abs(lg))
        elif check:
            ref = O.pne_contract(nets_in[0], K, max_iter=3 * max_iter)
            out["rel_err_log_vs_oracle_sample0"] = abs(float(res["log_abs"][0]) - ref.log_abs) / max(
                1.0, abs(ref.log_abs))
        print(json.dumps(out), flush=True)
        b.close()
        for n in nets:
            n.close()
        ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--nets", type=int, default=256, help="networks per bond dimension")
    ap.add_argument("--K", type=int, default=6)
    ap.add_argument("--check", type=int, default=2, help="networks per D checked against the oracle")
    ap.add_argument("--cpu-sample", type=int, default=24,
                    help="oracle networks per 8 cores in the CPU baseline (0: skip)")
    ap.add_argument("--fp64-steps", type=int, default=10, help="steps timed with FP64 terms (0: skip)")
    ap.add_argument("--profile-run", action="store_true", help="short run for rocprofv3 (no checks)")
    ap.add_argument("--no-events", action="store_true", help="time without per-kernel HIP events")
    ap.add_argument("--serving", type=int, default=4096, metavar="N",
                    help="also run the serving loop on N requests (capacity, then a sweep of Poisson arrival rates); 0: skip")
    ap.add_argument("--serving-budget", type=float, default=2.0, help="serving device budget, GB")
    ap.add_argument("--workloads", action="store_true",
                    help="instead: the other workloads at batch scale with per-kernel rooflines")
    ap.add_argument("--workload-filter", default="", metavar="TEXT",
                    help="with --workloads: only the batch workloads whose label contains TEXT")
    ap.add_argument("--rank-large", type=int, default=0, metavar="N",
                    help="instead: only the chi = 16 rank-r workload (12x12 Ising, 3x3 blocks) on N lattices")
    ap.add_argument("--rank", type=int, default=0, metavar="N",
                    help="instead: only the rank-r weight-passing workload on N lattices")
    ap.add_argument("--strips", type=int, default=0, metavar="L",
                    help="instead: only the infinite-lattice strip expansion at width L")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the workload, run plain device copies of MIB MiB (HBM counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other configurations and the beyond-MALL batch in the default line")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    # the CPU oracle baseline first: worker processes forked before anything
    # touches the GPU
    cpu = None
    default_run = not (args.workloads or args.strips or args.rank or args.rank_large or args.profile_run)
    if default_run and args.cpu_sample > 0:
        cpu = cpu_baseline(args.K, max(1, args.cpu_sample // 8), args.nets)
        print(f"bench: cpu baseline {cpu['value']} networks/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import torch

    import pne_inputs as P
    import paper_2512_10910_amd as pne

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.workloads:
        workloads_bench(pne, P, max(1, min(args.steps, 5)), args.workload_filter)
        if args.workload_filter:
            return
        strips_bench(pne, P)
        rank_bench(pne, P)
        print(json.dumps(rank_large_bench(pne, P)), flush=True)
        return
    if args.strips:
        strips_bench(pne, P, L=args.strips)
        return
    if args.rank:
        rank_bench(pne, P, n=args.rank)
        return
    if args.rank_large:
        print(json.dumps(rank_large_bench(pne, P, n=args.rank_large)), flush=True)
        return

    if args.copy_calibration:
        # a plain copy kernel of known size: reads and writes exactly MIB MiB
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    t_setup = time.time()
    nets_in = []
    for D in (4, 3):
        for i in range(args.nets):
            nets_in.append(P.config2_network(D, 2000 + i))
    print(f"bench: built {len(nets_in)} networks in {time.time() - t_setup:.1f}s", file=sys.stderr, flush=True)
    ctx = pne.Context(0)
    nets = [ctx.network(n) for n in nets_in]
    slice_bytes = {"fp64": 8, "fp32": 4, "bf16": 2}[args.precision]
    bp_kernels = ("bp_persistent", "bp_sweep")

    # Breakdown pass (outside the timed region): every kernel bracketed by HIP
    # events, to name the dominant kernel and report the per-kernel split.
    pb = ctx.batch(nets, K=args.K, precision=args.precision, profile=True)
    for _ in range(max(1, args.warmup)):
        pb.run_arrays(raise_on_error=True)
    pb.kernel_times(reset=True)
    bd_steps = max(3, min(args.steps, 10))
    for _ in range(bd_steps):
        pb.run_arrays(raise_on_error=True)
    kt_all = pb.kernel_times(reset=True)
    phases = pb.phase_times()
    pb.close()
    breakdown = {k: round(v[0] / bd_steps, 4) for k, v in kt_all.items()}
    dom = max(("bp_persistent", "bp_sweep", "regauge", "clusters", "combine"), key=lambda k: kt_all[k][0])
    if dom == "bp_sweep" and kt_all["bp_persistent"][0] > 0:
        dom = "bp_persistent"
    timed_kernels = list(bp_kernels) if dom in bp_kernels else [dom]

    # Timed region: HIP events only around the dominant kernel(s) on the
    # library's stream (events around every launch would add gaps).
    prof = False if args.no_events else timed_kernels
    batch = ctx.batch(nets, K=args.K, precision=args.precision, profile=prof)
    print(f"bench: prepared batches in {time.time() - t_setup:.1f}s", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        batch.run_arrays(raise_on_error=True)
    batch.kernel_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = None
    for _ in range(args.steps):
        results = batch.run_arrays(raise_on_error=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = batch.kernel_times(reset=True)
    ms_step = (t1 - t0) * 1e3 / args.steps
    n_nets = len(nets)
    terms = int(results["n_cluster_terms"].sum())
    nets_per_s = n_nets / (ms_step * 1e-3)
    print(f"bench: {ms_step:.3f} ms/step, {nets_per_s:.1f} networks/s", file=sys.stderr, flush=True)

    # roofline of the dominant kernel: algorithmic bytes of the steps it ran
    sweeps = [int(x) for x in results["bp_iters"]]
    paths = batch.paths()
    ncl = [int(x) for x in results["n_cluster_terms"]]
    alg = kernel_bytes(pne, nets_in, paths, sweeps, ncl, args.K, slice_bytes)
    in_lds = bool((paths & pne.PATH_PERSISTENT).all())
    dom_ms = sum(kt[k][0] for k in timed_kernels) / args.steps
    dom_launches = sum(kt[k][1] for k in timed_kernels)
    alg_bytes = sum(alg.get(k, 0) for k in timed_kernels) or None
    alg_split = {}
    if "bp_persistent" in timed_kernels:
        # the persistent kernel's share: BP, in-block gauge and slices, in-block terms
        for net, pth, st, nc in zip(nets_in, paths, sweeps, ncl):
            if not pth & pne.PATH_PERSISTENT:
                continue
            alg_split["bp"] = alg_split.get("bp", 0) + bp_bytes(net, st, True)
            if pth & pne.PATH_BLOCK_GAUGE:
                alg_split["gauge_slices"] = alg_split.get("gauge_slices", 0) + regauge_bytes(net, slice_bytes, True)
            if pth & pne.PATH_BLOCK_TERMS:
                alg_split["clusters_sum"] = alg_split.get("clusters_sum", 0) + cluster_bytes(pne, net, args.K,
                                                                                             slice_bytes)
    achieved = None
    if alg_bytes is not None and dom_ms > 0:
        # bytes per launch / average launch duration == bytes per step / time per step
        achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    roofline = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": measured_traffic(dom),
        "launches_per_step": dom_launches / args.steps,
        "avg_launch_us": round(dom_ms * args.steps / max(1, dom_launches) * 1e3, 2),
        "alg_bytes_per_step": alg_bytes,
        "alg_bytes_split": alg_split,
        "messages_in_lds": in_lds,
    }

    out = {
        "metric": METRIC,
        "value": round(nets_per_s, 1),
        "unit": "networks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64 (BP, gauge, sums) + f32 (terms)",
                  "bf16": "f64 (BP, gauge, sums) + bf16/f32 (terms)"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"16x16 open-boundary U[0,1] random networks, D=4 and D=3, {args.nets} seeds each "
                        f"(2000+), K={args.K}, {args.precision} terms",
            "networks_per_step": n_nets,
            "K": args.K,
            "precision": args.precision,
        },
        "terms_per_s": round(terms / (ms_step * 1e-3), 1),
        "terms_per_step": terms,
        "bp_sweeps_mean": float(np.mean(sweeps)),
        "kernel_ms_per_step_breakdown_pass": breakdown,
        "persistent_block_phases_us": {k: round(v, 1) for k, v in phases.items()},
        "roofline": roofline,
    }

    if not args.profile_run:
        bw = measured_copy_gbps(torch)
        roofline["measured_copy_GBps"] = round(bw, 1)
        if roofline.get("achieved"):
            roofline["frac_of_measured_copy"] = round(roofline["achieved"] / bw, 4)

    if args.fp64_steps > 0 and not args.profile_run and args.precision != "fp64":
        # the same batch with FP64 term contractions (slices, clusters and
        # sums all FP64), timed the same way: the plain FP64 form
        fb = ctx.batch(nets, K=args.K, precision="fp64")
        for _ in range(args.warmup):
            fb.run_arrays(raise_on_error=True)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            r64 = fb.run_arrays(raise_on_error=True)
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        fb.close()
        fms = (f1 - f0) * 1e3 / args.fp64_steps
        d = np.abs(results["log_abs"] - r64["log_abs"]) / np.maximum(1.0, np.abs(r64["log_abs"]))
        out["fp64_form"] = {
            "networks_per_s": round(n_nets / (fms * 1e-3), 1),
            "ms_per_step": round(fms, 4),
            "steps": args.fp64_steps,
            "speedup_of_reduced_precision": round(fms / ms_step, 3),
            "max_rel_err_log_vs_fp64_form": float(d.max()),
            "signs_equal": bool((results["sign"] == r64["sign"]).all()),
        }
        # the other reduced precision on the same batch, against the FP64 form
        other = "bf16" if args.precision == "fp32" else "fp32"
        ob = ctx.batch(nets, K=args.K, precision=other)
        for _ in range(args.warmup):
            ob.run_arrays()
        torch.cuda.synchronize()
        o0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            ro = ob.run_arrays()
        torch.cuda.synchronize()
        o1 = time.perf_counter()
        ob.close()
        oms = (o1 - o0) * 1e3 / args.fp64_steps
        do = np.abs(ro["log_abs"] - r64["log_abs"]) / np.maximum(1.0, np.abs(r64["log_abs"]))
        st_o = {int(k): int(v) for k, v in zip(*np.unique(ro["status"], return_counts=True))}
        out[f"{other}_form"] = {
            "networks_per_s": round(n_nets / (oms * 1e-3), 1),
            "ms_per_step": round(oms, 4),
            "steps": args.fp64_steps,
            "speedup_over_fp64_form": round(fms / oms, 3),
            "max_rel_err_log_vs_fp64_form": float(do.max()),
            "status_counts": st_o,
        }

    if not args.profile_run:
        import oracle as O

        # accuracy against the FP64 oracle on sampled networks of this batch
        errs = []
        idx = list(range(min(args.check, args.nets))) + [args.nets + i for i in range(min(args.check, args.nets))]
        for i in idx:
            ref = O.pne_contract(nets_in[i], args.K)
            d = abs(float(results["log_abs"][i]) - ref.log_abs)
            errs.append(d / max(1.0, abs(ref.log_abs)))
            if int(results["sign"][i]) != ref.sign:
                errs.append(math.inf)
        out["max_rel_err_log_vs_oracle"] = float(max(errs)) if errs else None
        out["accuracy_ok"] = bool(errs and max(errs) <= 1e-5)

        if cpu is not None:
            out["cpu_baseline"] = cpu
    if not args.profile_run and not args.no_extras:
        # the autotuner on this batch: the persistent kernel's tile shapes
        # timed against the default, the choice kept in a JSON cache
        import tempfile

        choice = ctx.autotune(nets, K=args.K, precision=args.precision, trials=3)
        with tempfile.TemporaryDirectory() as td:
            ctx.tune_cache_save(os.path.join(td, "tune.json"))
            with open(os.path.join(td, "tune.json")) as fh:
                entries = json.load(fh)["entries"]
        ent = entries[0] if entries else {}
        out["autotune"] = {"choice": choice, "tuned_ms": ent.get("ms"), "default_ms": ent.get("default_ms")}
        del batch
        for x in nets:
            x.close()
        del nets
        try:
            out["beyond_mall"] = beyond_mall(pne, P, max(3, args.steps // 4), args.precision, args.K)
            print("bench: beyond-MALL batch done", file=sys.stderr, flush=True)
            out["other_configs"] = other_configs(pne, P, max(3, args.steps // 4))
            print("bench: other configurations done", file=sys.stderr, flush=True)
            out["rank_chi16"] = rank_large_bench(pne, P, n=256, reps=2)
            print("bench: chi = 16 rank-r workload done", file=sys.stderr, flush=True)
        except Exception as e:  # report, keep the throughput line
            out["other_configs_error"] = repr(e)
    if args.serving > 0 and not args.profile_run:
        batch = nets = None
        try:
            out["serving"] = serving_bench(pne, P, args.serving, int(args.serving_budget * 1e9), "bf16", args.K)
        except Exception as e:  # report, keep the throughput line
            out["serving"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
