#!/usr/bin/env python3
"""Throughput of the attestation check on one MI355X.

One step = one pass of the whole hot path over one batch resident in HBM:
HKDF-SHA256 key derivation and HMAC midstates for every identity of the
registry, binning of the transactions by message block count, HMAC-SHA256
recomputation of every credential with a constant-time compare, and the
validity bitmask plus count.  Default workload: the throughput sweep's
largest batch, 16M transactions over 1M identities (uniform), message lengths
lognormal (median 200 B, sigma 0.75) clipped to 64..1232 B, 0.5% invalid.
The same line carries two sections beside it: the batching workload (256
uneven blocks: one captured replay, one multi-block call and one plain call
per block) and a short serving run (continuous batching against one request
per launch: saturation, then p50/p99 latency at half load), every result
checked.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

I_REF = 1384                                   # VALU instructions per SHA-256 compression
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12      # 256 CU x 64 lanes x 2.4 GHz = 39.32 T lane-op/s
HBM_PEAK_GBS = 8000.0
METRIC = "verified HMAC attestations/sec on 1 GPU; %peak INT32 VALU; p99 batch latency"


def log(msg: str) -> None:
    print("[bench %7.1fs] %s" % (time.time() - T0, msg), file=sys.stderr, flush=True)


T0 = time.time()


def compressions(lengths: np.ndarray) -> int:
    """Inner blocks ceil((L + 9) / 64) after the cached ipad block, plus one outer block."""
    return int(((lengths + 9 + 63) // 64 + 1).sum())


COUNTERS = "profiles/k_verify_binned_sweep16M_hbm_counters.md"


def kernel_sources():
    """Every source compiled into libace.so: the files of csrc/ (one
    translation unit includes them all) and the public header."""
    import glob
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2603_10242_amd", "csrc", "*")))
    return [os.path.relpath(f, ROOT) for f in files] + ["include/ace.h"]


def kernel_sources_hash() -> str:
    import hashlib
    m = hashlib.sha256()
    for f in kernel_sources():
        with open(os.path.join(ROOT, f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def counter_traffic():
    """HBM bytes per launch of the verify kernel from the committed FETCH_SIZE and
    WRITE_SIZE summary, or None when the kernels changed after it was taken."""
    try:
        text = open(os.path.join(ROOT, COUNTERS)).read()
    except OSError:
        return None
    fields = dict(l.strip().split(": ", 1) for l in text.splitlines() if ": " in l.strip()
                  and l.strip().split(": ", 1)[0] in ("kernel_sources_sha256",
                                                       "traffic_bytes_per_launch"))
    if fields.get("kernel_sources_sha256") != kernel_sources_hash():
        return None
    return int(fields["traffic_bytes_per_launch"])


def host_cpu() -> dict:
    """The host's processor model and the threads the CPU oracle may use: the
    CPUs of this process's affinity set, capped by the cgroup's CPU quota and
    by OMP_NUM_THREADS where those are set (the share of the host's cores
    given to this job)."""
    import math
    import subprocess
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "cgroup_cpu_quota": None, "omp_num_threads": None, "model": "unknown"}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                info["model"] = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()
        if q != "max":
            info["cgroup_cpu_quota"] = math.ceil(int(q) / int(per))
    except (OSError, ValueError):
        pass
    try:
        info["omp_num_threads"] = int(os.environ["OMP_NUM_THREADS"])
    except (KeyError, ValueError):
        pass
    caps = [info["affinity"]] + [v for v in (info["cgroup_cpu_quota"], info["omp_num_threads"]) if v]
    info["threads"] = max(1, min(caps))
    return info


def cpu_baseline(w, seconds: float, runs: int = 5) -> dict:
    """The CPU oracle as it stands on this host, on the threads host_cpu()
    allows: key derivation for every identity, then the HMAC check of a
    prefix of the batch (the whole batch when `runs` passes over it fit in
    `seconds`), scaled to the batch; the median of `runs` runs.  Beside it the
    single-thread cost per transaction, also the median of `runs` runs."""
    import oracle
    host = host_cpu()
    threads = host["threads"]
    probe = min(w.n, 50_000)
    t = time.perf_counter()
    keys = oracle.derive_keys(w.rev, w.salt, w.info, threads)
    t_keys = time.perf_counter() - t
    t = time.perf_counter()
    oracle.verify_batch(keys, w.msg, w.off[: probe + 1], w.ids[:probe], w.tags[:probe], threads)
    per_tx = (time.perf_counter() - t) / probe
    # each run: all keys, then as many transactions as its share of `seconds` allows
    budget = max(seconds / runs - t_keys, 0.0)
    sample = int(min(w.n, max(probe, budget / max(per_tx, 1e-12))))
    sample -= sample % 32 if sample > 32 else 0
    truth = w.truth_bitmask()[: (sample + 31) // 32]
    steps, derive, verify = [], [], []
    for _ in range(runs):
        t = time.perf_counter()
        keys = oracle.derive_keys(w.rev, w.salt, w.info, threads)
        t_derive = time.perf_counter() - t
        t = time.perf_counter()
        mask, count = oracle.verify_batch(keys, w.msg, w.off[: sample + 1], w.ids[:sample],
                                          w.tags[:sample], threads)
        t_verify = time.perf_counter() - t
        if sample % 32 == 0 and not np.array_equal(mask, truth):
            raise SystemExit("oracle disagrees with the generator's truth mask")
        derive.append(t_derive)
        verify.append(t_verify)
        steps.append(t_derive + t_verify * (w.n / sample))
    # one thread, for the per-transaction cost the paper quotes for one core
    one = min(w.n, 50_000)
    single = []
    for _ in range(runs):
        t = time.perf_counter()
        oracle.verify_batch(keys, w.msg, w.off[: one + 1], w.ids[:one], w.tags[:one], 1)
        single.append((time.perf_counter() - t) / one * 1e6)
    step_s = float(np.median(steps))
    return {"value": w.n / step_s, "unit": "attestations/s", "cores": threads, "kind": "oracle",
            "sample": "HKDF for all %d identities (median %.2f s) + HMAC verify of the first %d "
                      "of %d txs (median %.2f s), verify time scaled to the whole batch; "
                      "median of %d runs" % (w.n_id, np.median(derive), sample, w.n,
                                             np.median(verify), runs),
            "runs": runs, "step_s_runs": steps,
            "single_thread_us_per_tx": float(np.median(single)),
            "single_thread_us_per_tx_runs": single,
            "paper_context_us_per_tx": "about 1 (text), 0.83 on one M3 Pro core (Table 10)",
            "host": host}


def openssl_context(w, threads: int, runs: int = 3) -> dict:
    """Context beside the oracle: the same step with OpenSSL (the workload
    generator's client library, which uses the CPU's SHA extensions where it
    has them): HKDF for every identity, then HMAC-SHA256 of every transaction,
    on `threads` threads (median of `runs`), and one thread's cost per
    transaction.  The recomputed tags are checked against the generator's
    truth mask once, outside the timing."""
    from paper_2603_10242_amd import workload as W
    steps = []
    for r in range(runs):
        t = time.perf_counter()
        keys = W.client_keys(w.rev, w.salt, w.info, threads)
        tags = W.client_sign(keys, w.msg, w.off, w.ids, threads)
        steps.append(time.perf_counter() - t)
        if r == 0:
            ok = np.all(tags == w.tags, axis=1)
            if not np.array_equal(ok, w.truth):
                raise RuntimeError("OpenSSL recomputation disagrees with the generator's truth mask")
        del tags
    one = min(w.n, 200_000)
    single = []
    for _ in range(runs):
        t = time.perf_counter()
        W.client_sign(keys, w.msg, w.off[: one + 1], w.ids[:one], 1)
        single.append((time.perf_counter() - t) / one * 1e6)
    step_s = float(np.median(steps))
    return {"value": w.n / step_s, "unit": "attestations/s", "cores": threads,
            "kind": "OpenSSL EVP HKDF + HMAC-SHA256 per call (context, not the oracle; its "
                    "threads share the library's internal locks)",
            "step_s_runs": steps, "single_thread_us_per_tx": float(np.median(single))}


def measured_valu_rate(ace, torch) -> dict:
    """The device's INT32 VALU issue rate from the library's probe kernel, beside
    the peak the roofline uses (the probe runs after the timed steps)."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    rates = [ace.valu_rate(iters=20000, wgs_per_cu=8) for _ in range(3)]
    best = max(rates) / 1e12
    log("VALU probe: %.2f T lane-instr/s measured (%d CUs, implied clock %.2f GHz), "
        "peak used %.2f" % (best, cus, best * 1e3 / (cus * 64), PEAK_INT32_TOPS))
    return {"measured": best, "unit": "T int32 lane-instr/s", "cus": cus,
            "implied_clock_ghz": best * 1e3 / (cus * 64), "peak_used": PEAK_INT32_TOPS,
            "probe": "8 WGs x 256 lanes per CU, 20000 x 192 alignbit/bitop3/add3 each, best of 3"}


def time_calls(fn, steps: int, warmup: int):
    """After warmup: the mean wall time (ms) of `steps` calls of fn() enqueued
    back to back between two synchronizations, and then, from a second run of
    max(steps, 50) calls with a stream event pair around each, every call's
    own time (the latency percentiles; the events between calls are kept out
    of the throughput run)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_lat = max(steps, 50)   # enough calls for a p99 that is not simply the maximum
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    for k in range(n_lat):
        starts[k].record(stream)
        fn()
        ends[k].record(stream)
    torch.cuda.synchronize()
    ev = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    return wall * 1e3 / steps, ev


def batching_section(steps: int, warmup: int) -> dict:
    """The batching workload: 256 blocks of lognormal sizes in one captured
    replay, in one eager multi-block call and in one plain call per block;
    every block's bitmask and count checked after each form's first call and
    after its timed calls."""
    from paper_2603_10242_amd import workload as W
    log("generating the batching workload (256 blocks)")
    w = W.config4()
    import torch
    from paper_2603_10242_amd import ace, autotune
    ace.load()
    torch.cuda.set_device(0)
    autotune.apply_saved()
    gflags = autotune.saved_graph_flags()
    edges = np.concatenate([[0], np.cumsum(w.block_sizes)])
    d_msg = ace.to_device(w.msg)
    blocks = [ace.upload_block(None, w.off[a:b + 1], w.ids[a:b], w.tags[a:b], msg_dev=d_msg)
              for a, b in zip(edges[:-1], edges[1:])]
    ks = ace.midstate_keyset(ace.to_device(w.rev), w.salt, w.info)
    L = w.lengths()
    comp = compressions(L)
    g = ace.Graph(ks, max_blocks=len(blocks), max_tx=w.n, flags=gflags)
    ws_multi = ace.workspace(ace.verify_workspace_size(ks, blocks, 0))
    ws_one = ace.workspace(max(ace.verify_workspace_size(ks, [b], 0) for b in blocks))
    torch.cuda.synchronize()
    log("uploaded %d txs in %d blocks (%.3f compressions/tx); graph flags %d" %
        (w.n, len(blocks), comp / w.n, gflags))
    packed = [W.pack_bits(w.truth[a:b]) for a, b in zip(edges[:-1], edges[1:])]

    def clear():
        for blk in blocks:
            blk.bitmask.fill_(-1)   # stale bits each form must overwrite

    def check(tag):
        torch.cuda.synchronize()
        for blk, a, b, want in zip(blocks, edges[:-1], edges[1:], packed):
            m, c = blk.result()
            if c != int(w.truth[a:b].sum()) or not np.array_equal(m, want):
                raise SystemExit("RESULT MISMATCH in %s" % tag)

    forms = {
        "graph": lambda: g.launch(blocks),
        "multi_block_call": lambda: ace.verify_batch(ks, blocks, ws_multi, 0),
        "per_block_calls": lambda: [ace.verify_batch(ks, [b], ws_one, 0) for b in blocks],
    }
    out = {}
    for name, fn in forms.items():
        clear()
        fn()
        check(name + ", first call")
        clear()
        ms, ev = time_calls(fn, steps, warmup)
        check(name + ", after the timed calls")
        out[name] = {"ms": ms, "p50_ms": float(np.percentile(ev, 50)),
                     "p99_ms": float(np.percentile(ev, 99)), "attestations_per_s": w.n / (ms / 1e3),
                     "pct_peak_int32_valu": 100.0 * comp * I_REF / (ms / 1e3) / 1e12 / PEAK_INT32_TOPS,
                     "checked": "every block's bitmask and count, after the first and the timed calls"}
        log("%-17s %.3f ms  (p99 %.3f)  %.3g tx/s" % (name, ms, out[name]["p99_ms"],
                                                      out[name]["attestations_per_s"]))
    g.close()
    return {
        "workload": "batching, 256 blocks lognormal(19,500, 1.0) in [1k, 200k]",
        "n_tx": w.n, "n_id": w.n_id, "ids": "zipf 1.1", "keys": "resident midstates",
        "block_sizes_min_max": [int(w.block_sizes.min()), int(w.block_sizes.max())],
        "graph_flags": gflags, "compressions": comp, "steps": steps, "warmup": warmup,
        "forms": out,
        "speedup_graph_vs_per_block": out["per_block_calls"]["ms"] / out["graph"]["ms"],
        "speedup_multi_block_vs_per_block": out["per_block_calls"]["ms"] / out["multi_block_call"]["ms"],
    }


def bench_batching(args) -> dict:
    import torch
    sec = batching_section(args.steps, args.warmup)
    return {
        "metric": METRIC,
        "value": sec["forms"]["graph"]["attestations_per_s"],
        "unit": "attestations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec["forms"]["graph"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {k: sec[k] for k in ("workload", "n_tx", "n_id", "ids", "keys",
                                       "block_sizes_min_max", "graph_flags")},
        "forms": sec["forms"],
        "speedup_graph_vs_per_block": sec["speedup_graph_vs_per_block"],
        "p99_ms": sec["forms"]["graph"]["p99_ms"],
        "device": torch.cuda.get_device_name(0),
    }


def drive(stream, pool, starts, sizes, arrivals, threads: int = 8):
    """Open-loop load: request k arrives at arrivals[k] (monotonic seconds) and is
    submitted then by one of `threads` native submitter threads (the load
    generator is C, so the interpreter's pauses stay out of the latencies).
    Returns the arrival, submit, admit and completion times of every request."""
    import ctypes
    from paper_2603_10242_amd import ace
    from paper_2603_10242_amd import workload as W
    fn = ctypes.cast(ace.load().ace_verify_stream, ctypes.c_void_p).value
    tickets, submit, masks, mask_words, counts = W.client_drive(
        fn, stream._h.value, pool, starts, sizes, arrivals, threads)
    n = len(sizes)
    done = np.zeros(n)
    admit = np.zeros(n)
    for k in range(n):
        t = ace.Ticket(int(tickets[k]), int(sizes[k]), None, None)
        stream.poll(t, True)
        _, admit[k], done[k] = stream.times(t)
        stream.release(t)
    # every request's count and whole bitmask against the generator's truth
    bad = 0
    for k in range(n):
        lo, hi = int(starts[k]), int(starts[k] + sizes[k])
        w0 = int(mask_words[k])
        if (int(counts[k]) != int(pool.truth[lo:hi].sum()) or
                not np.array_equal(masks[w0:w0 + (hi - lo + 31) // 32], W.pack_bits(pool.truth[lo:hi]))):
            bad += 1
    if bad:
        raise SystemExit("RESULT MISMATCH in %d of %d serving requests" % (bad, n))
    return np.asarray(arrivals), submit, admit, done


def serving_section(args, loads, sat_requests: int, sat_warmup: int, min_requests: int,
                    max_requests: int, point_seconds: float, plain_loads_own: bool) -> dict:
    """Poisson-arriving requests served by the continuous-batching engine and by
    the plain one-request-per-launch form: saturation of each (a backlog
    submitted at once, after an untimed one), then latency at the offered
    loads (fractions of the continuous form's saturation, or of each form's
    own when plain_loads_own).  Every request's bitmask and count is checked."""
    from paper_2603_10242_amd import workload as W
    log("generating the serving pool: %d txs over %d identities" % (args.pool, args.n_id_serving))
    pool = W.config5_pool(n_pool=args.pool, n_id=args.n_id_serving)
    import torch
    from paper_2603_10242_amd import ace, autotune
    ace.load()
    torch.cuda.set_device(0)
    autotune.apply_saved()
    ks = ace.midstate_keyset(ace.to_device(pool.rev), pool.salt, pool.info)
    torch.cuda.synchronize()
    log("midstate cache resident: %.0f MiB" % (ks.mid.numel() * 4 / 2**20))
    arena = torch.empty(args.arena_gib << 30, dtype=torch.uint8, device="cuda")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([W.SEED_BASE + 5, 3])))
    mean_size = float(W.serving_request_sizes(200_000).mean())
    bytes_per_tx = float(pool.lengths().mean()) + 32 + 4 + 8

    def requests(count, seed):
        sizes = W.serving_request_sizes(count, seed=W.SEED_BASE + 5 + seed)
        starts = rng.integers(0, pool.n - sizes)
        return sizes, starts

    out = {}
    for form, plain in (("continuous", False), ("plain", True)):
        st = ace.Stream.create(ks, arena, staging_bytes=args.staging_mib << 20,
                               max_inflight=args.inflight, plain=plain)
        # saturation: a backlog submitted as fast as the submitters can, after
        # an untimed backlog that brings the engine and its buffers up
        nsat = sat_requests if not plain else max(200, sat_requests // 4)
        nwarm = sat_warmup if not plain else sat_warmup // 4
        if nwarm:
            sizes, starts = requests(nwarm, 900 + plain)
            drive(st, pool, starts, sizes, np.full(nwarm, time.monotonic()))
        sizes, starts = requests(nsat, 1000 + plain)
        b0 = st.stats()["batches"]
        t0 = time.monotonic()
        arr, sub, adm, done = drive(st, pool, starts, sizes, np.full(nsat, t0))
        sat = float(sizes.sum()) / (done.max() - t0)
        out[form] = {"saturation_tx_per_s": sat, "saturation_requests": nsat, "warmup_requests": nwarm,
                     "batches": st.stats()["batches"] - b0}
        log("%-10s saturation %.3g tx/s (%d requests, %d batches; %d untimed before)" % (
            form, sat, nsat, out[form]["batches"], nwarm))
        st.close()
    for form, plain in (("continuous", False), ("plain", True)):
        st = ace.Stream.create(ks, arena, staging_bytes=args.staging_mib << 20,
                               max_inflight=args.inflight, plain=plain)
        ref = out[form if plain_loads_own else "continuous"]["saturation_tx_per_s"]
        points = []
        for frac in loads:
            rate_tx = frac * ref
            rate_req = rate_tx / mean_size
            # at least min_requests per point (the low loads would otherwise
            # see a few thousand), at most max_requests
            count = int(min(max_requests, max(min_requests, rate_req * point_seconds)))
            sizes, starts = requests(count, int(frac * 1000))
            gaps = rng.exponential(1.0 / rate_req, size=count)
            t0 = time.monotonic() + 0.05
            arr, sub, adm, done = drive(st, pool, starts, sizes, t0 + np.cumsum(gaps))
            lat = (done - arr) * 1e3
            late = (sub - arr) * 1e3       # the submitter thread's delay past the arrival
            span = done.max() - arr.min()
            points.append({"offered_frac": frac, "of": form if plain_loads_own else "continuous",
                           "offered_tx_per_s": rate_tx,
                           "achieved_tx_per_s": float(sizes.sum()) / span, "requests": count,
                           "p50_ms": float(np.percentile(lat, 50)),
                           "p99_ms": float(np.percentile(lat, 99)),
                           "p99_engine_ms": float(np.percentile((done - sub) * 1e3, 99)),
                           "p99_queue_ms": float(np.percentile((adm - sub) * 1e3, 99)),
                           "p99_submit_late_ms": float(np.percentile(late, 99)),
                           "max_ms": float(lat.max())})
            log("%-10s load %.2f: p50 %.3f ms, p99 %.3f ms (engine %.3f, queue %.3f, "
                "submitter late %.3f), %.3g tx/s" % (
                    form, frac, points[-1]["p50_ms"], points[-1]["p99_ms"],
                    points[-1]["p99_engine_ms"], points[-1]["p99_queue_ms"],
                    points[-1]["p99_submit_late_ms"], points[-1]["achieved_tx_per_s"]))
        out[form]["sweep"] = points
        out[form]["stats"] = st.stats()
        st.close()
    return {
        "workload": "serving: Poisson requests of lognormal(1,000, 1.5) txs in [1, 50,000], "
                    "requests cut from a %d-tx pool" % pool.n,
        "n_id": pool.n_id, "ids": "zipf 1.1", "keys": "resident midstates",
        "arena_gib": args.arena_gib, "staging_mib": args.staging_mib,
        "max_inflight": args.inflight, "mean_request_txs": mean_size,
        "latency": "scheduled arrival to bitmask in host memory",
        "checked": "every request's bitmask and count against the generator's truth mask",
        "forms": out,
        "saturation_speedup_vs_plain": out["continuous"]["saturation_tx_per_s"]
                                       / out["plain"]["saturation_tx_per_s"],
        "pcie_ceiling_tx_per_s": 64e9 / bytes_per_tx,
    }


def bench_serving(args) -> dict:
    import torch
    sec = serving_section(args, args.loads, args.sat_requests, args.sat_warmup, args.min_requests,
                          args.max_requests, args.point_seconds, plain_loads_own=False)
    half = [p for p in sec["forms"]["continuous"]["sweep"] if abs(p["offered_frac"] - 0.5) < 1e-9]
    return {
        "metric": METRIC,
        "value": sec["forms"]["continuous"]["saturation_tx_per_s"],
        "unit": "attestations/s",
        "n_gpus": 1, "steps": len(args.loads), "warmup": 0,
        "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {k: sec[k] for k in ("workload", "n_id", "ids", "keys", "arena_gib", "staging_mib",
                                       "max_inflight", "mean_request_txs", "latency")},
        "forms": sec["forms"],
        "saturation_speedup_vs_plain": sec["saturation_speedup_vs_plain"],
        "p99_ms": half[0]["p99_ms"] if half else None,
        "pcie_ceiling_tx_per_s": sec["pcie_ceiling_tx_per_s"],
        "device": torch.cuda.get_device_name(0),
    }


def bench_attest(args) -> dict:
    """Paper-form attestations (payload binding + credential over obj_hash || domain)
    at the throughput sweep's batch size, keys derived for the block's domain in
    the step."""
    from paper_2603_10242_amd import workload as W
    log("generating %d paper-form attestations over %d identities" % (args.n, args.n_id))
    w = W.paper_attestations(n=args.n, n_id=args.n_id, id_dist=args.ids, p_invalid=0.005)
    L = w.lengths()
    comp = int(((L + 9 + 63) // 64 + 2).sum())
    derive_comp = 8 * w.n_id + 2 if args.keys == "recomputed" else 0
    import torch
    from paper_2603_10242_amd import ace, autotune
    ace.load()
    torch.cuda.set_device(0)
    autotune.apply_saved()
    blk = ace.upload_block(w.payload, w.poff, w.ids, w.att, record_bytes=72)
    rev = ace.to_device(w.rev)
    ks = (ace.rev_keyset(rev, w.domain, w.info) if args.keys == "recomputed"
          else ace.midstate_keyset(rev, w.domain, w.info))
    flags = {"binned": ace.ACE_BUCKETED, "binned-persistent": ace.ACE_BUCKETED | ace.ACE_PERSISTENT,
             "ordered": ace.ACE_ORDERED}[args.mode]
    ws = ace.workspace(ace.verify_workspace_size(ks, [blk], flags))
    ace.verify_attestations(ks, [blk], ws, flags)
    torch.cuda.synchronize()
    mask, count = blk.result()
    if count != int(w.truth.sum()) or not np.array_equal(mask, w.truth_bitmask()):
        raise SystemExit("RESULT MISMATCH: count %d, expected %d" % (count, int(w.truth.sum())))
    log("first call bit-exact with the generator's truth mask (%d valid)" % count)
    ace.profile_read(reset=True)
    ace.profile_enable(True)
    ms, ev = time_calls(lambda: ace.verify_attestations(ks, [blk], ws, flags), args.steps,
                        args.warmup)
    ace.profile_enable(False)
    prof = ace.profile_read(reset=True)
    calls = max(1, prof["calls"])
    verify_s = prof["verify_ms"] / calls / 1e3
    achieved = comp * I_REF / verify_s / 1e12
    log("timed %d steps: %.3f ms/step, verify %.3f ms (%.1f%% of INT32 VALU peak)"
        % (args.steps, ms, verify_s * 1e3, 100 * achieved / PEAK_INT32_TOPS))
    result = {
        "metric": "verified paper-form attestations/sec on 1 GPU; %peak INT32 VALU",
        "value": w.n / (ms / 1e3), "unit": "attestations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "paper-form attestations, %dM txs, keys %s" % (w.n >> 20, args.keys),
                   "n_tx": w.n, "n_id": w.n_id, "ids": args.ids,
                   "payload": "uniform 130..154 B", "record": "obj_hash || domain || credential",
                   "mode": args.mode, "invalid": int(w.n - w.truth.sum())},
        "roofline": {"kernel": "k_verify_binned" if args.mode != "ordered" else "k_verify_ordered",
                     "bound": "alu", "achieved": achieved, "peak": PEAK_INT32_TOPS,
                     "unit": "T int32 lane-instr/s", "frac": achieved / PEAK_INT32_TOPS,
                     "traffic": None,
                     "per_launch": "%d compressions x %d VALU instr" % (comp, I_REF),
                     "avg_ms": verify_s * 1e3},
        "compressions_per_step": comp + derive_comp,
        "p50_ms": float(np.percentile(ev, 50)), "p99_ms": float(np.percentile(ev, 99)),
        "stages_ms": {k: prof[k] / calls for k in ("derive_ms", "bin_ms", "verify_ms",
                                                   "finalize_ms")},
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = host_cpu()["threads"]
        t = time.perf_counter()
        keys = oracle.derive_keys(w.rev, w.domain, w.info, threads)
        t_derive = time.perf_counter() - t
        sample = min(w.n, 1 << 20)
        t = time.perf_counter()
        oracle.verify_attest(keys, w.payload, w.poff[: sample + 1], w.ids[:sample],
                             w.att[:sample], threads)
        t_verify = time.perf_counter() - t
        step_s = t_derive + t_verify * w.n / sample
        result["cpu_baseline"] = {
            "value": w.n / step_s, "unit": "attestations/s", "cores": threads, "kind": "oracle",
            "sample": "HKDF for all %d identities (%.2f s) + the first %d of %d attestations "
                      "(%.2f s), scaled to the batch" % (w.n_id, t_derive, sample, w.n, t_verify)}
    return result


def bench_poh(args) -> dict:
    """Hash-chain segment verification: --poh-segments segments of --poh-steps
    hashes each, one compression per hash."""
    from paper_2603_10242_amd import workload as W
    n, T = args.poh_segments, args.poh_steps
    log("generating %d chain segments of %d hashes" % (n, T))
    w = W.poh_segments(n=n, steps=T, step_errors=False)
    import torch
    from paper_2603_10242_amd import ace
    ace.load()
    torch.cuda.set_device(0)
    s, e = ace.to_device(w.start), ace.to_device(w.end)
    mask = torch.zeros(((n + 31) // 32,), dtype=torch.int32, device="cuda")
    cnt = torch.zeros((1,), dtype=torch.int64, device="cuda")
    ace.poh_verify(s, e, T, mask, cnt)
    torch.cuda.synchronize()
    if int(cnt.item()) != int(w.truth.sum()) or not np.array_equal(
            mask.cpu().numpy().view(np.uint32), w.truth_bitmask()):
        raise SystemExit("RESULT MISMATCH")
    log("first call bit-exact with the generator's truth mask")
    ms, ev = time_calls(lambda: ace.poh_verify(s, e, T, mask, cnt), args.steps, args.warmup)
    comp = n * T
    achieved = comp * I_REF / (np.median(ev) / 1e3) / 1e12
    log("%.3f ms per call, %.2f G hashes/s, %.1f%% of INT32 VALU peak"
        % (np.median(ev), comp / np.median(ev) / 1e6, 100 * achieved / PEAK_INT32_TOPS))
    result = {
        "metric": "verified hash-chain steps/sec on 1 GPU; %peak INT32 VALU",
        "value": comp / (ms / 1e3), "unit": "hashes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "hash-chain segments: %d x %d hashes" % (n, T),
                   "segments": n, "hashes_per_segment": T},
        "roofline": {"kernel": "k_poh_verify", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_INT32_TOPS, "unit": "T int32 lane-instr/s",
                     "frac": achieved / PEAK_INT32_TOPS, "traffic": None,
                     "per_launch": "%d compressions x %d VALU instr" % (comp, I_REF),
                     "avg_ms": float(np.median(ev))},
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = host_cpu()["threads"]
        sample = min(n, 1 << 14)
        t = time.perf_counter()
        oracle.poh_verify(w.start[:sample], w.end[:sample], w.steps[:sample], threads)
        dt = time.perf_counter() - t
        result["cpu_baseline"] = {"value": sample * T / dt, "unit": "hashes/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": "the first %d of %d segments (%.2f s)" % (sample, n, dt)}
    return result


def bench_merkle(args) -> dict:
    """Attestation Merkle roots of the batching workload's 256 blocks: one root
    per block over its 72-byte attestation records."""
    from paper_2603_10242_amd import workload as W
    sizes = W.batching_block_sizes()
    n = int(sizes.sum())
    log("generating %d attestation records in %d blocks" % (n, sizes.size))
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([W.SEED_BASE + 8])))
    data = rng.integers(0, 256, size=72 * n, dtype=np.uint8)
    off = np.arange(n + 1, dtype=np.uint64) * 72
    import torch
    from paper_2603_10242_amd import ace
    ace.load()
    torch.cuda.set_device(0)
    d_data = ace.to_device(data)
    d_off = ace.to_device(off)
    roots = torch.zeros((sizes.size, 32), dtype=torch.uint8, device="cuda")
    trees, first = [], 0
    for b, m in enumerate(sizes):
        trees.append((d_data, d_off[first:first + int(m) + 1], int(m), roots[b]))
        first += int(m)
    ws = ace.merkle_roots(trees)
    torch.cuda.synchronize()
    check = [0, sizes.size // 2, sizes.size - 1]
    firsts = np.concatenate([[0], np.cumsum(sizes)])
    for b in check:
        lo, hi = int(firsts[b]), int(firsts[b + 1])
        want = W.client_merkle_root(data[72 * lo:72 * hi], off[lo:hi + 1] - off[lo])
        if roots[b].cpu().numpy().tobytes() != want:
            raise SystemExit("RESULT MISMATCH in block %d" % b)
    log("roots of blocks %s equal the client's" % check)
    ms, ev = time_calls(lambda: ace.merkle_roots(trees, ws), args.steps, args.warmup)
    comp = 2 * n + 2 * int(np.maximum(sizes - 1, 0).sum())   # 72-byte leaves: 2 blocks each
    achieved = comp * I_REF / (np.median(ev) / 1e3) / 1e12
    log("%.3f ms per call (%d roots), %.1f%% of INT32 VALU peak"
        % (np.median(ev), sizes.size, 100 * achieved / PEAK_INT32_TOPS))
    return {
        "metric": "attestation Merkle roots: leaves/sec on 1 GPU; %peak INT32 VALU",
        "value": n / (ms / 1e3), "unit": "leaves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "Merkle roots of 256 blocks (%d attestation records of 72 B)" % n,
                   "blocks": int(sizes.size), "leaves": n},
        "roofline": {"kernel": "k_merkle_leaves + k_merkle_level + k_merkle_top", "bound": "alu",
                     "achieved": achieved, "peak": PEAK_INT32_TOPS,
                     "unit": "T int32 lane-instr/s", "frac": achieved / PEAK_INT32_TOPS,
                     "traffic": None,
                     "per_launch": "%d compressions x %d VALU instr" % (comp, I_REF),
                     "avg_ms": float(np.median(ev))},
        "p50_ms": float(np.percentile(ev, 50)), "p99_ms": float(np.percentile(ev, 99)),
        "device": torch.cuda.get_device_name(0),
    }


def bench_derive(args) -> dict:
    """Key derivation: one stream (the attestation keys of 1M identities) and
    the seven purpose streams of Def. 2.1 plus the two validator streams for
    the same identities in one call."""
    from paper_2603_10242_amd import workload as W
    import torch
    from paper_2603_10242_amd import ace
    ace.load()
    torch.cuda.set_device(0)
    n = args.n_id
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([W.SEED_BASE + 9])))
    rev_h = rng.integers(0, 256, size=(n, 32), dtype=np.uint8)
    rev = ace.to_device(rev_h)
    salt = rng.integers(0, 256, size=32, dtype=np.uint8).tobytes()
    infos = [b"ACEGF-V1-ED25519-SOLANA", b"ACEGF-V1-ED25519-POLKADOT", b"ACEGF-V1-SECP256K1-EVM",
             b"ACEGF-V1-SECP256K1-BTC", b"ACEGF-V1-SECP256K1-COSMOS", b"ACEGF-V1-X25519-IDENTITY",
             b"ACEGF-V1-ML-DSA-44-PQC-IDENTITY", b"ACEGF-V1-VALIDATOR-CONSENSUS",
             b"ACEGF-V1-VALIDATOR-VOTE"]
    streams = [(salt, i) for i in infos]
    mid = torch.empty((n, 16), dtype=torch.int32, device="cuda")
    keys = torch.empty((len(streams), n, 32), dtype=torch.uint8, device="cuda")
    # correctness on a sample of identities against the client's OpenSSL HKDF
    ace.derive_keys_multi(rev, streams, key_out=keys)
    torch.cuda.synchronize()
    sample = np.arange(0, n, max(1, n // 512))
    for sidx, (sa, inf) in enumerate(streams):
        want = W.client_keys(rev_h[sample], sa, inf)
        if not np.array_equal(keys[sidx].cpu().numpy()[sample], want):
            raise SystemExit("RESULT MISMATCH in stream %d" % sidx)
    log("keys of %d sampled identities in %d streams equal OpenSSL's" % (sample.size, len(streams)))
    ms1, ev1 = time_calls(lambda: ace.derive_keys(rev, salt, W.INFO_ATTEST, mid_out=mid),
                          args.steps, args.warmup)
    msm, evm = time_calls(lambda: ace.derive_keys_multi(rev, streams, key_out=keys), args.steps,
                          args.warmup)
    c1 = 8 * n + 2
    cm = len(streams) * (8 * n + 2)
    f1 = c1 * I_REF / (np.median(ev1) / 1e3) / 1e12 / PEAK_INT32_TOPS
    fm = cm * I_REF / (np.median(evm) / 1e3) / 1e12 / PEAK_INT32_TOPS
    log("one stream: %.3f ms (%.1f%% of peak); %d streams: %.3f ms (%.1f%% of peak)"
        % (np.median(ev1), 100 * f1, len(streams), np.median(evm), 100 * fm))
    return {
        "metric": "derived HKDF keys/sec on 1 GPU; %peak INT32 VALU",
        "value": len(streams) * n / (msm / 1e3), "unit": "keys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": msm,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "HKDF keys: %d identities x %d purpose streams" % (n, len(streams)),
                   "identities": n, "streams": len(streams)},
        "roofline": {"kernel": "k_derive_multi", "bound": "alu", "achieved": fm * PEAK_INT32_TOPS,
                     "peak": PEAK_INT32_TOPS, "unit": "T int32 lane-instr/s", "frac": fm,
                     "traffic": None, "per_launch": "%d compressions x %d VALU instr" % (cm, I_REF),
                     "avg_ms": float(np.median(evm))},
        "one_stream": {"ms": float(np.median(ev1)), "keys_per_s": n / (np.median(ev1) / 1e3),
                       "frac": f1, "outputs": "midstates"},
        "per_identity_all_streams_ns": float(np.median(evm)) * 1e6 / n,
        "device": torch.cuda.get_device_name(0),
    }


def bench_sweep_table(args) -> dict:
    """The throughput sweep's grid: n = 1..16M transactions, resident midstates
    against keys derived in the step, the per-transaction derivation ablation,
    and Zipf-skewed identities."""
    from paper_2603_10242_amd import workload as W
    import torch
    from paper_2603_10242_amd import ace, autotune
    ace.load()
    torch.cuda.set_device(0)
    autotune.apply_saved()
    rows = []
    for ids in ("uniform", "zipf"):
        log("generating 16M txs (%s ids)" % ids)
        w = W.config3(n=16 << 20, n_id=1 << 20, id_dist=ids)
        d_msg = ace.to_device(w.msg)
        rev = ace.to_device(w.rev)
        kss = {"midstate": ace.midstate_keyset(rev, w.salt, w.info),
               "recomputed": ace.rev_keyset(rev, w.salt, w.info)}
        sizes = (1 << 20, 2 << 20, 4 << 20, 8 << 20, 16 << 20) if ids == "uniform" else (16 << 20,)
        for n in sizes:
            blk = ace.upload_block(None, w.off[: n + 1], w.ids[:n], w.tags[:n], msg_dev=d_msg)
            L = w.lengths()[:n]
            comp = compressions(L)
            variants = [("midstate", 0), ("recomputed", 0)]
            if n == 4 << 20 and ids == "uniform":
                variants.append(("recomputed", ace.ACE_PER_TX_KEYS))
            for keys, extra in variants:
                ks = kss[keys]
                flags = ace.ACE_BUCKETED | extra
                ws = ace.workspace(ace.verify_workspace_size(ks, [blk], flags))
                ms, ev = time_calls(lambda: ace.verify_batch(ks, [blk], ws, flags), args.steps,
                                    args.warmup)
                m, c = blk.result()
                if c != int(w.truth[:n].sum()):
                    raise SystemExit("RESULT MISMATCH in the sweep table")
                derive = 8 * w.n_id if keys == "recomputed" and not extra else 0
                per_tx = 8 * n if extra else 0
                total = comp + derive + per_tx
                rows.append({"ids": ids, "n_tx": n, "keys": keys + ("-per-tx" if extra else ""),
                             "ms": ms, "p99_ms": float(np.percentile(ev, 99)),
                             "attestations_per_s": n / (ms / 1e3),
                             "gcompressions_per_s": total / (ms / 1e3) / 1e9,
                             "pct_peak_int32_valu": 100.0 * total * I_REF / (ms / 1e3) / 1e12
                                                    / PEAK_INT32_TOPS})
                log("%-7s n=%8d %-18s %.3f ms  %.3g tx/s  %.1f%% peak" % (
                    ids, n, rows[-1]["keys"], ms, rows[-1]["attestations_per_s"],
                    rows[-1]["pct_peak_int32_valu"]))
            del blk
        del d_msg, rev, kss, w
        torch.cuda.empty_cache()
    best = max(rows, key=lambda r: r["attestations_per_s"])
    return {"metric": METRIC, "value": best["attestations_per_s"], "unit": "attestations/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
            "data": "synthetic",
            "config": {"workload": "throughput sweep grid", "n_id": 1 << 20,
                       "lengths": "lognormal median 200 B sigma 0.75 clipped 64..1232 B"},
            "rows": rows, "device": torch.cuda.get_device_name(0)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=16 << 20, help="transactions per batch")
    ap.add_argument("--n-id", type=int, default=1 << 20, help="identities in the registry")
    ap.add_argument("--ids", choices=["uniform", "zipf"], default="uniform")
    ap.add_argument("--keys", choices=["recomputed", "midstate"], default="recomputed",
                    help="derive every identity's key in the step, or use resident midstates")
    ap.add_argument("--mode", choices=["binned", "binned-persistent", "ordered"], default="binned")
    ap.add_argument("--workload", choices=["sweep", "batching", "serving", "sweep-table",
                                           "attest", "poh", "merkle", "derive"],
                    default="sweep",
                    help="sweep: the throughput sweep (default); batching: 256 uneven blocks; "
                         "serving: Poisson requests through the serving engine; "
                         "attest: paper-form attestations with payload binding; "
                         "poh: hash-chain segment verification; merkle: attestation roots; "
                         "derive: HKDF key streams")
    ap.add_argument("--poh-segments", type=int, default=1 << 18)
    ap.add_argument("--poh-steps", type=int, default=1024)
    ap.add_argument("--pool", type=int, default=4 << 20, help="serving: transactions in the pool")
    ap.add_argument("--n-id-serving", type=int, default=4 << 20, help="serving: identities")
    ap.add_argument("--arena-gib", type=int, default=8, help="serving: device arena")
    ap.add_argument("--staging-mib", type=int, default=2048, help="serving: pinned staging")
    ap.add_argument("--inflight", type=int, default=4, help="serving: batches in flight")
    ap.add_argument("--sat-requests", type=int, default=20000)
    ap.add_argument("--sat-warmup", type=int, default=4000,
                    help="serving: untimed backlog before the saturation run")
    ap.add_argument("--max-requests", type=int, default=20000)
    ap.add_argument("--min-requests", type=int, default=10000)
    ap.add_argument("--point-seconds", type=float, default=1.5)
    ap.add_argument("--loads", type=float, nargs="+",
                    default=[0.1, 0.18, 0.32, 0.5, 0.75, 0.9, 1.1, 1.5])
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run three plain device copies of this many bytes (a reference "
                         "for scaling hardware byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batching", action="store_true",
                    help="sweep: leave out the batching section of the line")
    ap.add_argument("--no-serving", action="store_true",
                    help="sweep: leave out the serving section of the line")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(asked for --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        return 2

    if args.workload == "batching":
        print(json.dumps(bench_batching(args)), flush=True)
        return 0
    if args.workload == "serving":
        print(json.dumps(bench_serving(args)), flush=True)
        return 0
    if args.workload == "derive":
        print(json.dumps(bench_derive(args)), flush=True)
        return 0
    if args.workload == "merkle":
        print(json.dumps(bench_merkle(args)), flush=True)
        return 0
    if args.workload == "poh":
        print(json.dumps(bench_poh(args)), flush=True)
        return 0
    if args.workload == "attest":
        print(json.dumps(bench_attest(args)), flush=True)
        return 0
    if args.workload == "sweep-table":
        print(json.dumps(bench_sweep_table(args)), flush=True)
        return 0

    from paper_2603_10242_amd import workload as W
    log("generating workload: %d txs, %d identities (%s ids)" % (args.n, args.n_id, args.ids))
    w = W.config3(n=args.n, n_id=args.n_id, id_dist=args.ids)
    L = w.lengths()
    verify_comp = compressions(L)
    derive_comp = 8 * w.n_id + 2 if args.keys == "recomputed" else 0
    log("workload ready: %.2f GB of messages, %.3f compressions/tx"
        % (L.sum() / 1e9, verify_comp / w.n))

    import torch
    from paper_2603_10242_amd import ace, autotune
    ace.load()
    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    tuned = autotune.apply_saved()
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("reference copies: 3 x %d bytes read and written" % args.copy_bytes)
        del src, dst
    blk = ace.upload_block(w.msg, w.off, w.ids, w.tags)
    rev = ace.to_device(w.rev)
    if args.keys == "recomputed":
        ks = ace.rev_keyset(rev, w.salt, w.info)
    else:
        ks = ace.midstate_keyset(rev, w.salt, w.info)
    flags = {"binned": ace.ACE_BUCKETED, "binned-persistent": ace.ACE_BUCKETED | ace.ACE_PERSISTENT,
             "ordered": ace.ACE_ORDERED}[args.mode]
    ws = ace.workspace(ace.verify_workspace_size(ks, [blk], flags))
    torch.cuda.synchronize()
    log("uploaded to %s; workspace %.1f MB" % (dev_name, ws.numel() / 1e6))

    # warm-up: the first step checked, the others back to back (with the GPU
    # idle between steps its clock had not settled when the timed run began)
    ace.verify_batch(ks, [blk], ws, flags)
    torch.cuda.synchronize()
    mask, count = blk.result()
    if count != int(w.truth.sum()) or not np.array_equal(mask, w.truth_bitmask()):
        log("RESULT MISMATCH: count %d, expected %d" % (count, int(w.truth.sum())))
        return 1
    log("warmup step 0 bit-exact with the generator's truth mask (%d valid)" % count)
    for _ in range(max(1, args.warmup) - 1):
        ace.verify_batch(ks, [blk], ws, flags)

    # value: K plain calls back to back between two synchronizations (no stage
    # events inside the library, no events between the calls); then, straight
    # after, more calls each between two stream events, for the step latency
    # percentiles (the results are checked after both)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ace.verify_batch(ks, [blk], ws, flags)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    n_lat = max(args.steps, 50)   # enough steps for a p99 that is not simply the maximum
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(n_lat)]
    for k in range(n_lat):
        starts[k].record(stream)
        ace.verify_batch(ks, [blk], ws, flags)
        ends[k].record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    log("timed %d steps: %.3f ms/step (events p50 %.3f, p99 %.3f)"
        % (args.steps, ms_per_step, np.percentile(step_ms, 50), np.percentile(step_ms, 99)))
    mask, count = blk.result()
    if count != int(w.truth.sum()) or not np.array_equal(mask, w.truth_bitmask()):
        log("RESULT MISMATCH after timing")
        return 1

    # stage and kernel durations: the same calls again with the library's stage
    # events on (HIP events on the stream each kernel is launched on)
    ace.profile_read(reset=True)
    ace.profile_enable(True)
    traced_ms, traced_ev = time_calls(lambda: ace.verify_batch(ks, [blk], ws, flags),
                                      args.steps, 0)
    ace.profile_enable(False)
    prof = ace.profile_read(reset=True)
    log("traced steps: %.3f ms/step (events p50 %.3f)" % (traced_ms, np.percentile(traced_ev, 50)))

    calls = max(1, prof["calls"])
    verify_s = prof["verify_ms"] / calls / 1e3
    derive_alone = None
    if derive_comp:
        # the derivation of the step on its own: every identity's key and
        # midstates into a buffer of the same layout, timed like the steps
        mid = torch.empty((w.n_id, 16), dtype=torch.int32, device="cuda")
        d_ms, d_ev = time_calls(lambda: ace.derive_keys(rev, w.salt, w.info, mid_out=mid),
                                args.steps, args.warmup)
        d_med = float(np.median(d_ev))
        derive_alone = {"kernel": "k_derive", "identities": w.n_id, "ms": d_med,
                        "compressions": derive_comp,
                        "pct_peak_int32_valu": 100.0 * derive_comp * I_REF / (d_med / 1e3) / 1e12
                                               / PEAK_INT32_TOPS}
        del mid
        log("standalone derivation of %d identities: %.3f ms (%.1f%% of INT32 VALU peak)"
            % (w.n_id, d_med, derive_alone["pct_peak_int32_valu"]))
    achieved = verify_comp * I_REF / verify_s / 1e12
    bytes_tx = L.astype(np.float64) + 32 + 4 + 8 + 64 + 1.0 / 8
    verify_bytes = float(bytes_tx.sum())
    step_comp = verify_comp + derive_comp
    traffic = counter_traffic() if (args.n == 16 << 20 and args.mode == "binned"
                                    and args.keys == "recomputed" and args.ids == "uniform") else None
    result = {
        "metric": METRIC,
        "value": w.n / (ms_per_step / 1e3),
        "unit": "attestations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "throughput sweep, %dM txs, keys %s" % (w.n >> 20, args.keys),
            "n_tx": w.n, "n_id": w.n_id, "ids": args.ids,
            "lengths": "lognormal median 200 B sigma 0.75 clipped 64..1232 B",
            "invalid": int(w.n - w.truth.sum()), "mode": args.mode,
            "keys": "HKDF + ipad/opad midstates for all identities inside the step"
                    if args.keys == "recomputed" else "resident midstates",
        },
        "roofline": {
            "kernel": "k_verify_binned" if args.mode != "ordered" else "k_verify_ordered",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_INT32_TOPS,
            "unit": "T int32 lane-instr/s",
            "frac": achieved / PEAK_INT32_TOPS,
            "traffic": traffic,
            "per_launch": "%d compressions x %d VALU instr" % (verify_comp, I_REF),
            "avg_ms": verify_s * 1e3,
            "gcompressions_per_s": verify_comp / verify_s / 1e9,
            # the counted HBM bytes over the live launch time, against the 8 TB/s peak
            "hbm_gbs": traffic / verify_s / 1e9 if traffic else None,
            "hbm_frac": traffic / verify_s / 1e9 / HBM_PEAK_GBS if traffic else None,
        },
        "pct_peak_int32_valu_step": 100.0 * step_comp * I_REF / (ms_per_step / 1e3) / 1e12
                                    / PEAK_INT32_TOPS,
        "compressions_per_step": step_comp,
        "gcompressions_per_s": step_comp / (ms_per_step / 1e3) / 1e9,
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "latency_steps": int(len(step_ms)),
        "latency_ms": [round(float(x), 3) for x in step_ms],
        "ms_per_step_traced": traced_ms,
        # in the binned form with keys derived in the call, the derivation runs
        # on a second stream beside the binning passes: bin_ms covers both and
        # derive_ms reads about 0; the derivation is priced from a standalone
        # ace_derive_keys call over the same identities (derive_standalone)
        "stages_ms": {k: prof[k] / calls for k in ("derive_ms", "bin_ms", "verify_ms",
                                                   "finalize_ms")},
        "derive_pct_peak": derive_alone["pct_peak_int32_valu"] if derive_alone else None,
        "derive_standalone": derive_alone,
        "hbm_gbs_algorithmic_verify": verify_bytes / verify_s / 1e9,
        "device": dev_name,
        "tuning": ace.get_tuning(),
        "tuning_source": "autotuned" if tuned else "library defaults",
    }
    result["valu_rate"] = measured_valu_rate(ace, torch)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (about %.0f s)" % args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        try:   # context only: a failure here must not cost the line
            result["cpu_baseline"]["openssl_context"] = openssl_context(w, result["cpu_baseline"]["cores"])
        except Exception as e:  # noqa: BLE001
            result["cpu_baseline"]["openssl_context"] = {"error": str(e)}
    del blk, rev, ks, ws, w
    torch.cuda.empty_cache()
    if not args.no_batching:
        # the batching workload's three forms, each checked
        result["batching"] = batching_section(args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_serving:
        # a short serving run: saturation of both forms, then latency at half
        # of each form's own saturation
        result["serving"] = serving_section(args, [0.5], sat_requests=10000, sat_warmup=2000,
                                            min_requests=10000, max_requests=10000,
                                            point_seconds=1.5, plain_loads_own=True)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
