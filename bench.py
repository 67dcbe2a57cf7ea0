#!/usr/bin/env python3
"""Throughput of the WAH index pipeline (radix sort of (value, row) pairs, then
the WAH encoder) on one MI355X: input elements/s over K requests of 2^26
Zipf(1.1) uint32 values already resident in HBM, built by the wah_index actor
with the 16-bit value hint (the paper sorts with a fixed cardinality of 16
bits), with the HBM roofline of the dominant kernel and of the whole pipeline,
the composition of the two stage actors timed beside it, and the CPU oracle
timed on the host.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import re
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
SORT_KERNELS = ("radix_upsweep0", "radix_plan", "radix_upsweep", "exclusive_scan_u32", "radix_scatter")
ENCODE_KERNELS = ("wah_write",)
KERNELS = SORT_KERNELS + ENCODE_KERNELS
# Counter summary of the dominant kernel (FETCH_SIZE / WRITE_SIZE runs of this
# script under rocprofv3), valid while the kernel's sources hash to what it names.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "radix_scatter_zipf_2p26_traffic.md")
SCATTER_SOURCES = ("paper_1709_07781_amd/csrc/k_sort.hip", "paper_1709_07781_amd/csrc/common.hpp")
METRIC = "input elements/s (and % HBM roofline) of composed pipeline; p50/p99 latency served"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def active_passes(v: np.ndarray) -> tuple[int, int]:
    """(radix passes the sort runs, index of the first one): a pass runs unless
    one 8-bit digit value is shared by every key (measurement bookkeeping)."""
    act = []
    for p in range(4):
        d = (v >> np.uint32(8 * p)) & np.uint32(0xFF)
        if d.size and not np.all(d == d[0]):
            act.append(p)
    if not act:
        act = [3]
    return len(act), act[0]


def sources_digest(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(n_log2: int):
    """HBM bytes per launch of k_radix_scatter from the committed counter
    summary, or None when there is none for this size or the kernel's sources
    changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"^traffic_json: (\{.*\})$", text, re.M)
    if not m:
        return None
    t = json.loads(m.group(1))
    if t.get("sources_sha256") != sources_digest(SCATTER_SOURCES) or t.get("n_log2") != n_log2:
        return None
    return t["hbm_bytes_per_launch"]


def host_info() -> dict:
    """The host's CPU count and model (for the CPU baseline)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "cpu_count": os.cpu_count(), "cpu_model": model}


def timed_oracle(o, v, runs: int):
    """The oracle's index of v, timed `runs` times with the calling thread
    pinned to one core (restored afterwards).  Returns (seconds per run, the
    last result)."""
    old = None
    try:
        old = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(old)})
    except (AttributeError, OSError):
        old = None
    times, res = [], None
    try:
        for _ in range(runs):
            c0 = time.perf_counter()
            res = o.wah_index(v)
            times.append(time.perf_counter() - c0)
    finally:
        if old is not None:
            os.sched_setaffinity(0, old)
    return times, res


def batched_oracle_leg(off, v, budget_s: float = 20.0) -> dict:
    """The oracle on the batch's requests, one request per host thread at a
    time (the oracle is a C library called through ctypes, which releases the
    GIL, so a thread pool runs requests in parallel), over the first requests
    of the batch up to about budget_s of work: elements/s and the threads used."""
    import concurrent.futures as cf

    import oracle

    o = oracle.default()
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    threads = max(1, min(threads, 64))
    nreq = len(off) - 1
    # size the sample from one request's rate (about 1.1e7 elements/s per core)
    per_core = 1.1e7
    cap = budget_s * per_core * threads
    k = 0
    while k < nreq and off[k + 1] <= cap:
        k += 1
    k = max(k, 1)
    parts = [v[off[j]:off[j + 1]] for j in range(k)]
    c0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(o.wah_index, parts))
    t = time.perf_counter() - c0
    elems = int(off[k])
    return {"value": elems / t, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {k} of {nreq} requests ({elems} elements), one request per thread at a time",
            "seconds": t, "host": host_info()}


def plain_request_leg(sess, args) -> dict:
    """The plain configuration: one request of 2^16 values uniform below 1024
    through ka_wah_index, host values in and host arrays out (the paper's
    timer includes the transfers), median over repeated requests; also the
    device-only time of the same request from HBM-resident input."""
    import ctypes

    import paper_1709_07781_amd as ka
    import workloads

    v = workloads.plain_request()
    hint = ka.KA_WAH_VALUE_BITS(10)  # values below 1024
    reps = 50
    e2e = []
    first = None
    for k in range(reps + 3):
        t0 = time.perf_counter()
        res = ka.ka_wah_result()
        ka.check(ka.lib.ka_wah_index(sess.sys, v.ctypes.data, v.size, hint, ctypes.byref(res)))
        dt = time.perf_counter() - t0
        D, W = res.D, res.W
        if first is None:
            first = (np.ctypeslib.as_array(res.keys, shape=(max(D, 1),))[:D].copy(),
                     np.ctypeslib.as_array(res.offsets, shape=(D + 1,)).copy(),
                     np.ctypeslib.as_array(res.words, shape=(max(W, 1),))[:W].copy())
        ka.check(ka.lib.ka_wah_result_free(ctypes.byref(res)))
        if k >= 3:
            e2e.append(dt)
    dv = sess.upload(v)
    dev = []
    import torch
    for k in range(reps + 3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ka.ka_wah_result()
        ka.check(ka.lib.ka_wah_index(sess.sys, ctypes.c_void_p(dv.data_ptr()), v.size,
                                     ka.KA_WAH_INPUT_DEVICE | ka.KA_WAH_OUTPUT_REFS | hint, ctypes.byref(res)))
        dt = time.perf_counter() - t0
        ka.check(ka.lib.ka_wah_result_free(ctypes.byref(res)))
        if k >= 3:
            dev.append(dt)
    # The same request through a batch plan of one request: its launches
    # recorded once into a HIP graph, then per request one upload, one replay
    # and one copy of the results back (host in, host out).
    from paper_1709_07781_amd.session import BatchPlan
    plan = BatchPlan(sess, [0, v.size], 10)
    graph = []
    try:
        for k in range(reps + 3):
            t0 = time.perf_counter()
            plan.run(v)
            (got,) = plan.result()
            dt = time.perf_counter() - t0
            if k == 0 and not all(np.array_equal(g, e) for g, e in zip(got, first)):
                raise RuntimeError("plain request: the batch plan's index differs from ka_wah_index's")
            if k >= 3:
                graph.append(dt)
    finally:
        plan.close()
    e2e_ms = float(np.median(e2e)) * 1e3
    dev_ms = float(np.median(dev)) * 1e3
    graph_ms = float(np.median(graph)) * 1e3
    log(f"[bench] plain 2^16 request: {e2e_ms:.3f} ms end to end (host in/out), {dev_ms:.3f} ms from HBM, "
        f"{graph_ms:.3f} ms end to end through a graph-replayed plan")
    return {"workload": "2^16 values uniform below 1024, one ka_wah_index call (10-bit value hint)", "n": int(v.size),
            "D": int(D),
            "W": int(W), "e2e_ms_median": e2e_ms, "e2e_elements_per_s": v.size / (e2e_ms * 1e-3),
            "device_resident_ms_median": dev_ms, "device_resident_elements_per_s": v.size / (dev_ms * 1e-3),
            "plan_graph_e2e_ms_median": graph_ms, "plan_graph_e2e_elements_per_s": v.size / (graph_ms * 1e-3),
            "requests": reps, "how": "wall time per call on the host (waits for the result), median; the plan "
                                     "form: a ka_batch_plan of this one request (host in, host out)"}


def pcie_inclusive_leg(sess, v, args) -> dict:
    """The large request with host input and host outputs (ka_wah_index: copy
    in, pipeline, copy the index back): the rate including the transfers over
    PCIe.  Context only; `value` is measured from HBM-resident input."""
    import ctypes

    import paper_1709_07781_amd as ka

    times = []
    for k in range(4):
        t0 = time.perf_counter()
        res = ka.ka_wah_result()
        ka.check(ka.lib.ka_wah_index(sess.sys, v.ctypes.data, v.size, ka.KA_WAH_VALUE_BITS(args.value_bits),
                                     ctypes.byref(res)))
        dt = time.perf_counter() - t0
        D, W = res.D, res.W
        ka.check(ka.lib.ka_wah_result_free(ctypes.byref(res)))
        if k:
            times.append(dt)
    ms = float(np.median(times)) * 1e3
    moved = 4 * v.size + 4 * (D + (D + 1) + W)
    log(f"[bench] PCIe-inclusive large request: {ms:.2f} ms")
    return {"ms_median": ms, "elements_per_s": v.size / (ms * 1e-3), "host_bytes_moved": int(moved),
            "runs": len(times), "how": "ka_wah_index with host input and host outputs (pageable), wall time"}


def bench_batched(args) -> int:
    """4096 index requests (sizes log-uniform in [2^10, 2^20], values below
    2^12): the batched actor wah_index_batch over all of them per step,
    against the plain composed actor sent each request in turn."""
    import ctypes

    import torch
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Session
    import workloads

    t0 = time.time()
    off, v = workloads.batched_requests()
    N, nreq = int(off[-1]), len(off) - 1
    log(f"[bench] batched input ready: {nreq} requests, {N} elements ({time.time() - t0:.1f}s)")
    torch.cuda.set_device(0)
    sess = Session(profile=True)
    dv = sess.upload(v)
    doff = sess.upload(off.astype(np.uint32))
    vin, oin = sess.wrap(dv), sess.wrap(doff)
    vb = (ctypes.c_uint32 * 1)(12)
    batch = sess.spawn("wah_index_batch", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN), ka.arg(ka.KA_PRIV, count=1, init=vb)]
                       + [ka.arg(ka.KA_OUT)] * 5)
    sort = sess.spawn("radix_sort_rows_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT), ka.arg(ka.KA_OUT)])
    enc = sess.spawn("wah_encode_sorted", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN)] + [ka.arg(ka.KA_OUT)] * 3)
    pipe = sess.compose(enc, sort)
    views = [sess.wrap(dv[int(off[j]):int(off[j + 1])]) for j in range(nreq)]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev0.record(stream)
        for k in range(steps):
            a = time.perf_counter()
            fn()
            log(f"[bench] step {k + 1}/{steps} ({1e3 * (time.perf_counter() - a):.2f} ms on the host)")
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps, (time.perf_counter() - w0) / steps

    def batched_step():
        for r in sess.request(batch, ka.ref(vin), ka.ref(oin), n_out=5):
            sess.release_ref(r)

    def plain_step():
        for j in range(nreq):
            for r in sess.request(pipe, ka.ref(views[j]), n_out=3):
                sess.release_ref(r)

    plain_step()  # warm-up of the per-request path (pool sizes)
    sess.profile_reset()
    for _ in range(args.warmup):  # then of the batched step: its blocks are cached when the timing starts
        batched_step()
    torch.cuda.synchronize()
    sess.profile_reset()
    b_ms, b_wall = timed(batched_step, args.steps)
    prof = {k: sess.profile(k) for k in KERNELS + ("batch_keys", "batch_split")}
    p_steps = max(1, min(3, args.steps))
    p_ms, p_wall = timed(plain_step, p_steps)

    # the same batch through a batch plan (the pipeline recorded into a HIP graph)
    from paper_1709_07781_amd.session import BatchPlan

    tuned = {}

    def graph_ms(off_, dv_, steps):
        plan = BatchPlan(sess, off_, 12, autotune=True)
        pstream = torch.cuda.ExternalStream(plan.stream_handle())
        plan.run(dv_)  # fills the plan's input and times every tile shape; later replays read it in place
        tuned[len(tuned)] = plan.shape()
        for _ in range(args.warmup):
            plan.run(None)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(pstream)
        for _ in range(steps):
            plan.run(None)
        e1.record(pstream)
        torch.cuda.synchronize()
        plan.close()
        return e0.elapsed_time(e1) / steps

    g_ms = graph_ms(off, dv, args.steps)

    def any_graph_ms(scale, steps):
        """The same batch through a plan recorded for any batch of up to
        scale x its values and requests (one graph for every batch)."""
        plan = BatchPlan(sess, None, 12, autotune=True, any_batch=(int(scale * N), int(scale * nreq), 0))
        pstream = torch.cuda.ExternalStream(plan.stream_handle())
        plan.run_batch(dv, off)  # table and values in, every sort variant timed
        for _ in range(args.warmup):
            plan.run(None)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(pstream)
        for _ in range(steps):
            plan.run(None)
        e1.record(pstream)
        torch.cuda.synchronize()
        plan.close()
        return e0.elapsed_time(e1) / steps

    ga_ms, ga2_ms = any_graph_ms(1, args.steps), any_graph_ms(1.5, args.steps)
    log(f"[bench] batched: actor {b_ms:.3f} ms, graph {g_ms:.3f} ms, any-batch graph {ga_ms:.3f} ms "
        f"(capacities 1.5x: {ga2_ms:.3f} ms), plain {p_ms:.1f} ms")
    # a batch of small requests (sizes 2^4..2^10), where launch work matters more
    soff, sv = workloads.batched_requests(seed=40, count=4096, lo_log2=4, hi_log2=10)
    sdv = sess.upload(sv)
    sdoff = sess.upload(soff.astype(np.uint32))
    svin, soin = sess.wrap(sdv), sess.wrap(sdoff)

    def small_step():
        for r in sess.request(batch, ka.ref(svin), ka.ref(soin), n_out=5):
            sess.release_ref(r)

    small_step()
    s_ms, _ = timed(small_step, args.steps)
    sg_ms = graph_ms(soff, sdv, args.steps)
    sviews = [sess.wrap(sdv[int(soff[j]):int(soff[j + 1])]) for j in range(len(soff) - 1)]

    def small_plain():
        for j in range(len(soff) - 1):
            for r in sess.request(pipe, ka.ref(sviews[j]), n_out=3):
                sess.release_ref(r)

    small_plain()
    sp_ms, _ = timed(small_plain, 1)
    for r in sviews + [svin, soin]:
        sess.release_ref(r)
    log(f"[bench] small batch ({int(soff[-1])} elements): actor {s_ms:.3f} ms, graph {sg_ms:.3f} ms, "
        f"plain {sp_ms:.1f} ms")

    outs = sess.request(batch, ka.ref(vin), ka.ref(oin), n_out=5)
    keys, offs, words, ks, ws = (sess.read(r) for r in outs)
    for r in outs:
        sess.release_ref(r)
    # Algorithmic bytes of the batch: the sum over its requests of one
    # request's bytes, 16 P_j n_j + 8 n_j + 4 W_j + 8 D_j + 4, with P_j the
    # 8-bit digit passes request j's own values need.
    sizes = np.diff(off)
    nonempty = sizes > 0
    starts = off[:-1][nonempty]
    P_j = np.zeros(nreq, dtype=np.int64)
    for p in range(4):
        d = ((v >> np.uint32(8 * p)) & np.uint32(0xFF)).astype(np.uint8)
        moves = np.minimum.reduceat(d, starts) != np.maximum.reduceat(d, starts)
        P_j[nonempty] += moves
    P_j[nonempty] = np.maximum(P_j[nonempty], 1)
    D_j = np.diff(ks.astype(np.int64))
    W_j = np.diff(ws.astype(np.int64))
    batch_bytes = int(np.sum(16 * P_j * sizes + 8 * sizes + 4 * W_j + 8 * D_j + 4 * nonempty))
    b_gbs = batch_bytes / (b_ms * 1e-3) / 1e9
    g_gbs = batch_bytes / (g_ms * 1e-3) / 1e9
    sc_launches, sc_ms = prof["radix_scatter"]
    # The batch's sort: values below 2^12 take the segmented sort (each
    # request sorted inside its own positions over 16-bit keys), 2 passes of
    # 8-bit digits; the method's pair-pass bytes per launch as for one request
    # (12 N for the first pass, 16 N for each later one).
    P_sort = 2
    sc_bytes = (12 * N + 16 * N * (P_sort - 1)) * args.steps
    sc_gbs = sc_bytes / max(sc_launches, 1) / (sc_ms / max(sc_launches, 1) * 1e-3) / 1e9
    log(f"[bench] batched: sum of per-request bytes {batch_bytes / 1e9:.2f} GB: actor {b_gbs:.0f} GB/s, "
        f"graph {g_gbs:.0f} GB/s")

    parity = None
    if not args.no_parity:
        import oracle
        o = oracle.default()
        ok = True
        for j in sorted({0, nreq - 1, int(np.argmax(sizes)), int(np.argmin(sizes))}):
            ek, eo, ew = o.wah_index(v[off[j]:off[j + 1]])
            k0, k1, w0, w1 = int(ks[j]), int(ks[j + 1]), int(ws[j]), int(ws[j + 1])
            ok &= (np.array_equal(keys[k0:k1], ek) and np.array_equal(offs[k0 + j:k1 + j + 1], eo)
                   and np.array_equal(words[w0:w1], ew))
        parity = "bit-exact (requests sampled)" if ok else "MISMATCH"
    for a in (batch, pipe, sort, enc):
        sess.release_actor(a)
    for r in views + [vin, oin]:
        sess.release_ref(r)
    sess.close()
    out = {
        "metric": METRIC, "value": N / (b_ms * 1e-3), "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": b_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"batched: {nreq} index requests, sizes log-uniform in [2^10, 2^20], values uniform "
                               "below 2^12, input resident in HBM; one wah_index_batch pass per step",
                   "n": N, "nreq": nreq},
        "plain": {"ms_per_step": p_ms, "value": N / (p_ms * 1e-3), "steps": p_steps, "wall_s_per_step": p_wall,
                  "how": "the composed sort->encode actor sent each request in turn (per-stage launches)"},
        "speedup_vs_plain": p_ms / b_ms,
        "graph": {"ms_per_step": g_ms, "value": N / (g_ms * 1e-3),
                  "how": "ka_batch_plan, autotuned: the same batch recorded into a HIP graph per sort tile "
                         "shape, the fastest on the first run replayed",
                  "shape": tuned[0][0], "first_run_ms_per_shape": tuned[0][1][:4]},
        "graph_any_batch": {"ms_per_step": ga_ms, "capacity_1p5x_ms_per_step": ga2_ms,
                            "how": "ka_batch_plan_create_any: one graph recorded for capacities (values, requests) "
                                   "that serves any batch within them; capacities equal to this batch, and 1.5 "
                                   "times it (the grids sized by the capacity, the counts read on the device)"},
        "small_batch": {"workload": "4096 requests, sizes log-uniform in [2^4, 2^10], values below 2^12",
                        "n": int(soff[-1]), "actor_ms": s_ms, "graph_ms": sg_ms, "plain_ms": sp_ms,
                        "shape": tuned[1][0], "first_run_ms_per_shape": tuned[1][1][:4]},
        "roofline": {"bound": "hbm", "kernel": "k_radix_scatter", "achieved": sc_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": sc_gbs / HBM_PEAK_GBS, "traffic": None,
                     "launches": sc_launches, "avg_launch_ms": sc_ms / max(sc_launches, 1),
                     "algorithmic_bytes_per_launch": sc_bytes / max(sc_launches, 1), "sort_passes": P_sort},
        "pipeline": {"algorithmic_bytes": batch_bytes,
                     "bytes_formula": "sum over requests of 16*P_j*n_j + 8*n_j + 4*W_j + 8*D_j + 4",
                     "actor_GBs": b_gbs, "actor_frac": b_gbs / HBM_PEAK_GBS, "graph_GBs": g_gbs,
                     "graph_frac": g_gbs / HBM_PEAK_GBS},
        "batched_wall_s_per_step": b_wall,
        "kernel_ms_per_step": {k: prof[k][1] / args.steps for k in prof if prof[k][0]},
        "parity": parity,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batched_oracle_leg(off, v)
        log(f"[bench] batched oracle: {out['cpu_baseline']['value']:.3g} elements/s on "
            f"{out['cpu_baseline']['cores']} threads ({out['cpu_baseline']['sample']})")
    print(json.dumps(out), flush=True)
    return 0 if parity in (None, "bit-exact (requests sampled)") else 1


def bench_served(args) -> int:
    """The served mix at each rate: request j arrives at its scheduled Poisson
    time (sizes log-uniform in [2^8, 2^22], 40% index of values below 2^12,
    30% scan, 30% 8-stage affine chain); latency runs from the scheduled
    arrival to completion seen on the host.  The batched server (continuous
    batching, 2 streams, 64 GiB budget) against the plain server (one request
    at a time, same kernels)."""
    import torch
    from paper_1709_07781_amd.session import Server, Session
    import workloads

    torch.cuda.set_device(0)
    sess = Session(n_streams=max(4, args.served_streams))
    a, b = workloads.chain_params()
    # payloads are slices of two pre-generated pools (values below 2^12 for
    # the index requests, full 32-bit values for the others)
    pool_n = 1 << 23
    pool_idx = workloads.uniform_values(workloads.derive(5, 10), pool_n, 1 << 12)
    pool_u32 = workloads.u32(workloads.derive(5, 11), pool_n)
    rates = [float(r) for r in args.rates.split(",") if r]
    rows = []
    check_every = 64  # every 64th timed request is checked against the oracle after its run
    parity_ok = True
    if not args.no_parity:
        import oracle
        ora = oracle.default()
    for rate in rates:
        count = int(min(args.served_max, max(50, rate * args.served_seconds)))
        warm = max(50, count // 8)
        t, sizes, kinds, dseeds = workloads.served_requests(seed=5, count=warm + count, rate_per_s=rate)
        sizes = np.minimum(sizes, pool_n)
        starts = (dseeds % np.uint64(pool_n)).astype(np.int64)
        starts = np.minimum(starts, pool_n - sizes)
        res = {"rate_per_s": rate, "requests": count, "warmup_requests": warm}
        batched_kw = dict(streams=args.served_streams, max_batch=1024, max_batch_bytes=args.served_batch_mb << 20,
                          copy_threads=args.served_copy_threads)
        plain_kw = dict(streams=1, max_batch=1, copy_threads=args.served_copy_threads)
        for form, kw in (("batched", batched_kw), ("plain", plain_kw)):
            srv = Server(sess, chain_a=a, chain_b=b, **kw)

            def run(lo, hi, keep=None):
                """Requests lo..hi-1 on their schedule; a client thread takes
                each result as it completes and releases it.  keep: a dict
                that receives a copy of the outputs of every
                check_every-th request, for the parity check after the run."""
                m = hi - lo
                handles = [None] * m
                submitted = threading.Semaphore(0)
                failures = []

                def consume():
                    for j in range(m):
                        submitted.acquire()
                        rc = srv.wait(handles[j])
                        if rc != 0:
                            failures.append(rc)
                        elif keep is not None and (lo + j) % check_every == 0:
                            nout = 3 if kinds[lo + j] == workloads.KIND_WAH else 1
                            keep[lo + j] = [srv.result(handles[j], i) for i in range(nout)]
                        srv.release(handles[j])

                consumer = threading.Thread(target=consume)
                consumer.start()
                t0 = Server.clock_us() + 20_000.0 - t[lo] * 1e6  # first arrival 20 ms from now
                for j in range(m):
                    due = t0 + t[lo + j] * 1e6
                    while True:
                        now = Server.clock_us()
                        if now >= due:
                            break
                        if due - now > 200:
                            time.sleep((due - now - 100) * 1e-6)
                    k = lo + j
                    pool = pool_idx if kinds[k] == workloads.KIND_WAH else pool_u32
                    handles[j] = srv.submit(int(kinds[k]), pool[starts[k]:starts[k] + sizes[k]], arrival_us=due)
                    submitted.release()
                consumer.join()
                if failures:
                    raise RuntimeError(f"served request failed: {failures[0]}")

            # warm-up: the first requests of the same schedule fill the pinned
            # and device caches; their statistics are dropped.  The client's
            # garbage collector is off while requests are submitted (its
            # pauses would be charged to the server as late arrivals).
            run(0, warm)
            srv.reset_stats()
            gc.collect()
            gc.disable()
            kept = {}
            try:
                w0 = time.perf_counter()
                run(warm, warm + count, kept)
                wall = time.perf_counter() - w0
            finally:
                gc.enable()
            st = srv.stats()
            srv.close()
            bad = 0
            if not args.no_parity:
                for k, outs in kept.items():
                    pool = pool_idx if kinds[k] == workloads.KIND_WAH else pool_u32
                    x = pool[starts[k]:starts[k] + sizes[k]]
                    if kinds[k] == workloads.KIND_WAH:
                        exp = ora.wah_index(x)
                    elif kinds[k] == workloads.KIND_SCAN:
                        exp = (ora.exclusive_scan(x),)
                    else:
                        exp = (ora.affine_chain(x, a, b),)
                    bad += not all(np.array_equal(g, e) for g, e in zip(outs, exp))
            span_s = max(wall - 0.02, 1e-9)
            res[form] = {"p50_ms": st["p50_us"] / 1e3, "p99_ms": st["p99_us"] / 1e3, "max_ms": st["max_us"] / 1e3,
                         "elements_per_s": st["elements"] / span_s, "requests_per_s": st["completed"] / span_s,
                         "mean_batch": st["mean_batch"], "batches": st["batches"],
                         "parity": None if args.no_parity else
                         (f"bit-exact ({len(kept)} requests checked)" if not bad else f"MISMATCH in {bad}")}
            parity_ok &= bad == 0
            log(f"[bench] served rate={rate:.0f}/s {form}: p50={res[form]['p50_ms']:.2f} ms "
                f"p99={res[form]['p99_ms']:.2f} ms, {res[form]['requests_per_s']:.0f} req/s, "
                f"batch={st['mean_batch']:.1f}")
        rows.append(res)
    sess.close()
    top = max(rows, key=lambda r: r["batched"]["elements_per_s"])
    out = {
        "metric": METRIC, "value": top["batched"]["elements_per_s"], "unit": "elements/s", "n_gpus": 1,
        "steps": len(rates), "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "served: Poisson arrivals, sizes log-uniform in [2^8, 2^22], 40% WAH index "
                               "(values below 2^12) / 30% exclusive scan / 30% 8-stage affine chain, host data, "
                               "latency from the scheduled arrival to completion on the host",
                   "rates": rates, "budget_bytes": 64 << 30, "batched_streams": args.served_streams,
                   "batch_mib": args.served_batch_mb, "copy_threads": args.served_copy_threads or 4},
        "served": rows,
    }
    print(json.dumps(out), flush=True)
    return 0 if parity_ok else 1


def bench_spawn(args) -> int:
    """The paper's first benchmark (Sec. 5.1): wall-clock time to create the
    runtime and spawn N actors, then to make sure they are usable by sending
    one message to the last one and waiting for its response; mean of R runs
    with 95% confidence intervals.  Kernel actors (affine_u32 of the built-in
    program; add_u32 of a gfx950 code object loaded per run) against host-only
    actors (composed actors over two affine stages: they run no kernel of their
    own, the closest thing here to CAF's event-based actors)."""
    import ctypes

    import paper_1709_07781_amd as ka

    hsaco = os.path.join(ROOT, "tests", "kernels", "user_kernels.hsaco")
    counts = [int(c) for c in args.spawn_counts.split(",")]
    runs = args.spawn_runs
    m = 1024
    x = np.arange(m, dtype=np.uint32)
    P = ctypes.c_void_p

    def one_run(kind: str, n: int) -> float:
        t0 = time.perf_counter()
        cfg = ka.ka_system_config()
        sysh, prog = P(), P()
        ka.check(ka.lib.ka_system_create(ctypes.byref(cfg), ctypes.byref(sysh)))
        if kind == "code_object":
            ka.check(ka.lib.ka_program_load(sysh, hsaco.encode(), ctypes.byref(prog)))
        else:
            ka.check(ka.lib.ka_program_builtin(sysh, ctypes.byref(prog)))
        ca, cb = (ctypes.c_uint32 * 1)(3), (ctypes.c_uint32 * 1)(1)
        aff_sig = ka.sig(ka.arg(ka.KA_IN_OUT, in_mode=ka.KA_VAL, out_mode=ka.KA_VAL),
                         ka.arg(ka.KA_PRIV, count=1, init=ca), ka.arg(ka.KA_PRIV, count=1, init=cb))
        add_sig = ka.sig(ka.arg(ka.KA_IN, in_mode=ka.KA_VAL), ka.arg(ka.KA_IN, in_mode=ka.KA_VAL),
                         ka.arg(ka.KA_OUT, out_mode=ka.KA_VAL))
        rng = ka.nd_range(global0=m)
        actors, stages = [], []
        if kind == "composed":
            for _ in range(2):
                st = P()
                ka.check(ka.lib.ka_spawn(sysh, prog, b"affine_u32", ctypes.byref(rng), aff_sig, 3, ctypes.byref(st)))
                stages.append(st)
        for _ in range(n):
            a = P()
            if kind == "builtin":
                ka.check(ka.lib.ka_spawn(sysh, prog, b"affine_u32", ctypes.byref(rng), aff_sig, 3, ctypes.byref(a)))
            elif kind == "code_object":
                ka.check(ka.lib.ka_spawn(sysh, prog, b"add_u32", ctypes.byref(rng), add_sig, 3, ctypes.byref(a)))
            else:
                ka.check(ka.lib.ka_compose(stages[0], stages[1], ctypes.byref(a)))
            actors.append(a)
        msg = [ka.val(x.ctypes.data, m)] * (2 if kind == "code_object" else 1)
        t = P()
        ka.check(ka.lib.ka_send(actors[-1], ka.values(*msg), len(msg), ctypes.byref(t)))
        out = np.empty(m, np.uint32)
        o = (ka.ka_value * 1)()
        o[0].ptr, o[0].count = out.ctypes.data, m
        ka.check(ka.lib.ka_receive(t, o, 1, -1))
        dt = time.perf_counter() - t0
        ka.check(ka.lib.ka_ticket_release(t))
        for a in actors + stages:
            ka.check(ka.lib.ka_actor_release(a))
        ka.check(ka.lib.ka_program_release(prog))
        ka.check(ka.lib.ka_system_destroy(sysh))
        return dt

    import torch
    torch.cuda.set_device(0)
    one_run("builtin", 1)  # the process's first HIP initialisation, not counted
    res = {}
    for kind in ("builtin", "code_object", "composed"):
        rows = []
        for n in counts:
            ts = [one_run(kind, n) for _ in range(runs)]
            mean = float(np.mean(ts))
            ci = 1.96 * float(np.std(ts, ddof=1)) / np.sqrt(len(ts)) if len(ts) > 1 else 0.0
            rows.append({"actors": n, "mean_ms": mean * 1e3, "ci95_ms": ci * 1e3})
            log(f"[bench] spawn {kind}: {n} actors {mean * 1e3:.3f} ms +- {ci * 1e3:.3f}")
        ns = np.array([r["actors"] for r in rows], float)
        ms = np.array([r["mean_ms"] for r in rows])
        slope, icept = np.polyfit(ns, ms, 1) if len(ns) > 1 else (0.0, float(ms[0]))
        res[kind] = {"runs": rows, "per_actor_us": slope * 1e3, "intercept_ms": icept}
    out = {"metric": "wall-clock time to create the runtime and spawn N actors (Sec. 5.1)", "unit": "ms",
           "higher_is_better": False, "runs_per_point": runs, "message": f"one request of {m} uint32 to the last actor",
           "kinds": res}
    print(json.dumps(out), flush=True)
    return 0


def bench_chain(args) -> int:
    """The actor-overhead chain: 8 affine actors composed with device-resident
    refs, the same stages with a host round trip per stage (values in and out),
    and the raw launch sequence of the same kernels (ka_affine_chain_raw), at
    m = 2^10 .. 2^24.  Per chain: device time in a back-to-back stream of
    chains, and latency of one chain waited for on the host (median)."""
    import ctypes

    import torch
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Session
    import oracle
    import workloads

    torch.cuda.set_device(0)
    sess = Session()
    a, b = workloads.chain_params()
    ca = np.ascontiguousarray(a, dtype=np.uint32)
    cb = np.ascontiguousarray(b, dtype=np.uint32)
    ref_actors = [sess.affine_actor(int(a[i]), int(b[i])) for i in range(8)]
    chain = ref_actors[0]
    composed = []
    for i in range(1, 8):
        chain = sess.compose(ref_actors[i], chain)
        composed.append(chain)
    val_actors = [sess.affine_actor(int(a[i]), int(b[i]), in_mode=ka.KA_VAL, out_mode=ka.KA_VAL) for i in range(8)]
    stream = torch.cuda.current_stream()
    o = oracle.default()
    rows = []
    for lg in (10, 14, 18, 22, 24):
        m = 1 << lg
        x0 = workloads.chain_input(seed=2, m=m)
        exp = o.affine_chain(x0, a, b)
        reps = max(5, min(200, (1 << 26) // m))

        def dev_ms(fn):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        def lat_us(fn, sync=True):
            ts = []
            for _ in range(min(reps, 50)):
                t0 = time.perf_counter()
                fn()
                if sync:
                    torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e6)
            return float(np.median(ts))

        dv = sess.upload(x0)
        vin = sess.wrap(dv)

        def refs_chain():
            (r,) = sess.request(chain, ka.ref(vin), n_out=1)
            sess.release_ref(r)

        def raw_chain():
            ka.check(ka.lib.ka_affine_chain_raw(sess.sys, ctypes.c_void_p(dv.data_ptr()), m, ca.ctypes.data,
                                                cb.ctypes.data, 8))

        def host_chain():
            x = x0
            for act in val_actors:
                (x,) = sess.request(act, ka.val(x.ctypes.data, x.size), n_out=1)
            return x

        # parity of each form, from the same input
        dv.copy_(torch.from_numpy(x0.view(np.int32)))
        refs_chain()
        ok = np.array_equal(sess.read(vin), exp)
        dv.copy_(torch.from_numpy(x0.view(np.int32)))
        raw_chain()
        torch.cuda.synchronize()
        ok &= np.array_equal(dv.cpu().numpy().view(np.uint32), exp)
        ok &= np.array_equal(host_chain(), exp)
        row = {"m": m, "parity": "bit-exact" if ok else "MISMATCH",
               "refs_device_ms": dev_ms(refs_chain), "raw_device_ms": dev_ms(raw_chain),
               "refs_latency_us": lat_us(refs_chain), "raw_latency_us": lat_us(raw_chain),
               "host_round_trip_latency_us": lat_us(host_chain, sync=False),
               "roofline_GBs_refs": 64.0 * m / 1e9 / 1e-3}
        row["roofline_GBs_refs"] = 64.0 * m / (row["refs_device_ms"] * 1e-3) / 1e9
        # The chain works in place on 4m bytes: at every size here that fits the
        # 256 MB Infinity Cache, so the rate above is not an HBM fraction.
        row["working_set_bytes"] = 4 * m
        row["cache_resident"] = 4 * m <= (256 << 20)
        row["refs_overhead_us"] = row["refs_latency_us"] - row["raw_latency_us"]
        row["refs_overhead_pct"] = 100.0 * row["refs_overhead_us"] / row["raw_latency_us"]
        log(f"[bench] chain m=2^{lg}: refs {row['refs_latency_us']:.1f} us, raw {row['raw_latency_us']:.1f} us, "
            f"host round trip {row['host_round_trip_latency_us']:.1f} us, device {row['refs_device_ms']:.4f} ms "
            f"({row['roofline_GBs_refs']:.0f} GB/s), {row['parity']}")
        rows.append(row)
        sess.release_ref(vin)
        del dv
    for act in composed + ref_actors + val_actors:
        sess.release_actor(act)
    sess.close()
    big = rows[-1]
    out = {"metric": METRIC, "value": big["m"] / (big["refs_device_ms"] * 1e-3), "unit": "elements/s",
           "n_gpus": 1, "steps": None, "warmup": 1, "ms_per_step": big["refs_device_ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "actor-overhead chain: 8 composed affine actors x <- a_i x + b_i over uint32[m], "
                                  "device-resident refs vs host round trip per stage vs raw launch sequence"},
           "chain": rows}
    print(json.dumps(out), flush=True)
    return 0 if all(r["parity"] == "bit-exact" for r in rows) else 1


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-log2", type=int, default=26)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--value-bits", type=int, default=16,
                    help="large: the index actor's value hint (every value below 2^bits; 0 = no hint)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the plain 2^16 request leg and the PCIe-inclusive leg of the default workload")
    ap.add_argument("--spawn-counts", default="1,10,100,1000,5000", help="spawn: actor counts")
    ap.add_argument("--spawn-runs", type=int, default=50, help="spawn: runs per count (the paper: mean of 50)")
    ap.add_argument("--workload", choices=("large", "batched", "served", "chain", "spawn"), default="large",
                    help="large: the 2^26 Zipf request (default); batched: 4096 requests of 2^10..2^20 values, "
                         "one batched pass against 4096 plain per-request pipelines; served: Poisson arrivals of "
                         "the 40/30/30 index/scan/chain mix at several rates, batched server against the plain "
                         "one-request-at-a-time server")
    ap.add_argument("--rates", default="1000,2000,5000,10000,20000,50000",
                    help="served: arrival rates in requests/s")
    ap.add_argument("--served-seconds", type=float, default=10.0,
                    help="served: seconds of arrivals per rate (at most --served-max requests)")
    ap.add_argument("--served-max", type=int, default=20000)
    ap.add_argument("--served-streams", type=int, default=2, help="served: streams of the batched server")
    ap.add_argument("--served-batch-mb", type=int, default=16, help="served: MiB of input per batch")
    ap.add_argument("--served-copy-threads", type=int, default=0,
                    help="served: threads copying a large payload into pinned memory (0: the library's 4)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run the in-place affine kernel over 2^n words 3 times "
                         "(a plain copy of known size, for scaling the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library runs the pipeline "
              "on a single GPU and has no multi-GPU sharding", file=sys.stderr)
        return 2
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "chain":
        return bench_chain(args)
    if args.workload == "spawn":
        return bench_spawn(args)

    import torch
    import paper_1709_07781_amd as ka
    from paper_1709_07781_amd.session import Session
    import workloads

    n = 1 << args.n_log2
    t0 = time.time()
    v = workloads.large_request(seed=args.seed, n=n)
    P, _ = active_passes(v)
    log(f"[bench] input ready: n=2^{args.n_log2} zipf(1.1) over 2^16 values, radix passes={P} "
        f"({time.time() - t0:.1f}s)")

    torch.cuda.set_device(0)
    sess = Session(profile=True)
    dv = sess.upload(v)
    torch.cuda.synchronize()

    # The index actor: wah_index with the value hint (sort of (value, row)
    # pairs, then the encoder, queued by one actor), refs in and out.
    import ctypes
    hint = (ctypes.c_uint32 * 2)(args.value_bits, 0)
    index_actor = sess.spawn("wah_index", [ka.arg(ka.KA_IN), ka.arg(ka.KA_PRIV, count=2, init=hint)]
                             + [ka.arg(ka.KA_OUT)] * 3)
    # The composition of the two stage actors (wah_encode_sorted (.)
    # radix_sort_rows_u32, no hint), timed beside it.
    sort = sess.spawn("radix_sort_rows_u32", [ka.arg(ka.KA_IN), ka.arg(ka.KA_OUT), ka.arg(ka.KA_OUT)])
    enc = sess.spawn("wah_encode_sorted", [ka.arg(ka.KA_IN), ka.arg(ka.KA_IN)] + [ka.arg(ka.KA_OUT)] * 3)
    pipe = sess.compose(enc, sort)
    vin = sess.wrap(dv)

    def step(keep=False, actor=index_actor):
        outs = sess.request(actor, ka.ref(vin), n_out=3)
        if keep:
            return outs
        for r in outs:
            sess.release_ref(r)
        return None

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()

    def finish(t, keep=False):
        outs = sess.receive(t, 3)
        sess.release_ticket(t)
        if keep:
            return outs
        for r in outs:
            sess.release_ref(r)
        return None

    def timed_region(profiled: bool, actor=index_actor):
        """K requests between two events on the library's stream, and an
        event after every request (the per-step times, for their median);
        with profiled, every launch is also bracketed by the library's own
        events.  Requests are pipelined: request k+1 is sent before request
        k is received (every request runs in full and is received), so the
        device never waits for the host's turnaround between requests."""
        ka.check(ka.lib.ka_profile_enable(sess.sys, 1 if profiled else 0))
        sess.profile_reset()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev0.record(stream)
        prev = None
        for k in range(args.steps):
            t = sess.send(actor, ka.ref(vin))
            evs[k].record(stream)
            if prev is not None:
                finish(prev)
            prev = t
            if k == args.steps - 1 or (k + 1) % 10 == 0:
                log(f"[bench] {'profiled ' if profiled else ''}step {k + 1}/{args.steps}")
        last_ = finish(prev, keep=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        per_step = [a.elapsed_time(b) for a, b in zip([ev0] + evs[:-1], evs)]
        return ev0.elapsed_time(ev1), time.perf_counter() - w0, last_, per_step

    # the reported value: no per-launch events in the timed region
    dev_ms, wall, last, per_step_ms = timed_region(False)
    ms_per_step = dev_ms / args.steps
    for r in last:
        sess.release_ref(r)
    # the composed two-actor pipeline, same input and timing
    for _ in range(args.warmup):
        step(actor=pipe)
    composed_dev_ms, _, last_c, _ = timed_region(False, actor=pipe)
    for r in last_c:
        sess.release_ref(r)
    composed_ms = composed_dev_ms / args.steps
    log(f"[bench] composed stage actors: {composed_ms:.4f} ms per request")
    # per-kernel device times for the roofline: a second region with the library's events
    prof_ms, _, last, _ = timed_region(True)
    prof = {k: sess.profile(k) for k in KERNELS}
    D = sess.length(last[0])
    W = sess.length(last[2])

    # ---- algorithmic bytes (what the method has to move) -----------------------------
    # The pipeline: P stable pair passes of 16 B per element each (the first
    # reads no rows but one 4 B histogram read of the keys is added), one read
    # of the sorted pairs by the encoder (8n), and the index it writes
    # (4W + 8D + 4).
    pipe_bytes = 16 * P * n + 8 * n + 4 * W + 8 * D + 4
    # What this implementation moves instead: with the 16-bit hint the sort
    # keys are stored as uint16 between passes (6 B per pair); every pass
    # counts its digits from the keys (upsweep: 4n, then 2n); the first pass
    # reads uint32 values and makes the rows; the encoder reads the sorted
    # pairs once.
    if 1 <= args.value_bits <= 16:
        moved_bytes = (4 * n + 10 * n) + (P - 1) * (2 * n + 12 * n) + 6 * n + 4 * W + 8 * D + 4
    else:
        moved_bytes = (4 * n + 12 * n) + (P - 1) * (4 * n + 16 * n) + 8 * n + 4 * W + 8 * D + 4
    # The dominant kernel, k_radix_scatter: per launch the bytes of the
    # method's pair pass (4-byte keys): the first pass reads keys (rows are
    # made from positions) and writes keys and rows, every later one reads
    # and writes both.  The uint16 sort keys move fewer bytes than these.
    scatter_bytes = 12 * n + 16 * n * (P - 1)
    launches, scatter_ms = prof["radix_scatter"]
    per_launch_bytes = scatter_bytes * args.steps / max(launches, 1)
    avg_launch_ms = scatter_ms / max(launches, 1)
    achieved = per_launch_bytes / (avg_launch_ms * 1e-3) / 1e9
    pipe_gbs = pipe_bytes / (ms_per_step * 1e-3) / 1e9
    traffic = measured_traffic(args.n_log2)

    if args.copy_calibration:
        buf = torch.zeros(n, dtype=torch.int32, device="cuda")
        cal = sess.affine_actor(1, 1)
        rb = sess.wrap(buf)
        for _ in range(3):
            (r,) = sess.request(cal, ka.ref(rb), n_out=1)
            sess.release_ref(r)
        torch.cuda.synchronize()
        sess.release_actor(cal)
        sess.release_ref(rb)
        del buf
        log("[bench] copy calibration: 3 in-place affine launches over 2^%d words" % args.n_log2)

    plain = None if args.no_extra_legs else plain_request_leg(sess, args)
    pcie = None if args.no_extra_legs else pcie_inclusive_leg(sess, v, args)

    parity = None
    cpu = None
    if not args.no_cpu_baseline or not args.no_parity:
        import oracle
        o = oracle.default()
        times, (ek, eo, ew) = timed_oracle(o, v, 1 if args.no_cpu_baseline else 3)
        log(f"[bench] oracle: {np.median(times):.2f}s per request (median of {len(times)}, one pinned core)")
        if not args.no_parity:
            ok = (np.array_equal(sess.read(last[0]), ek) and np.array_equal(sess.read(last[1]), eo)
                  and np.array_equal(sess.read(last[2]), ew))
            parity = "bit-exact" if ok else "MISMATCH"
        if not args.no_cpu_baseline:
            cpu = {"value": n / float(np.median(times)), "unit": "elements/s", "cores": 1, "kind": "oracle",
                   "sample": f"the full 2^{args.n_log2}-element request, median of {len(times)} runs on one core "
                             "(std::stable_sort + sequential six-part WAH encoder)",
                   "runs_s": times, "host": host_info()}
    for r in last:
        sess.release_ref(r)

    out = {
        "metric": METRIC,
        "value": n * args.steps / (dev_ms * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "large single request: 2^26 uint32 values Zipf(s=1.1) over 2^16 distinct values, "
                               "row ids 0..n-1, sort->WAH-encode pipeline (wah_index actor, 16-bit value hint), "
                               "per-stage launches, input resident in HBM",
                   "n": n, "D": D, "W": W, "radix_passes": P, "value_bits": args.value_bits, "seed": args.seed},
        "roofline": {"bound": "hbm", "kernel": "k_radix_scatter", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "launches": launches, "avg_launch_ms": avg_launch_ms,
                     "algorithmic_bytes_per_launch": per_launch_bytes},
        "pipeline": {"algorithmic_bytes": pipe_bytes, "moved_bytes": moved_bytes,
                     "bytes_formula": "16*P*n + 8*n + 4*W + 8*D + 4", "ms": ms_per_step, "achieved_GBs": pipe_gbs,
                     "moved_GBs": moved_bytes / (ms_per_step * 1e-3) / 1e9,
                     "frac": pipe_gbs / HBM_PEAK_GBS, "step_ms_median": float(np.median(per_step_ms)),
                     "step_ms_min": min(per_step_ms), "step_ms_max": max(per_step_ms),
                     "profiled_ms_per_step": prof_ms / args.steps,
                     "kernel_ms_per_step": {k: prof[k][1] / args.steps for k in prof},
                     "launches_per_step": {k: prof[k][0] / args.steps for k in prof},
                     "wall_s": wall},
        "composed_stage_actors": {"ms": composed_ms, "elements_per_s": n / (composed_ms * 1e-3),
                                  "frac": pipe_bytes / (composed_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "how": "wah_encode_sorted (.) radix_sort_rows_u32, no value hint, same input"},
        "cpu_baseline": cpu,
        "plain_request": plain,
        "pcie_inclusive": pcie,
        "parity": parity,
    }
    for a in (pipe, sort, enc, index_actor):
        sess.release_actor(a)
    sess.release_ref(vin)
    sess.close()
    print(json.dumps(out), flush=True)
    return 0 if parity in (None, "bit-exact") else 1


if __name__ == "__main__":
    sys.exit(main())
