#!/usr/bin/env python3
"""Throughput of the attestation check on one MI355X.

One step = one pass of the whole hot path over one batch resident in HBM:
HKDF-SHA256 key derivation and HMAC midstates for every identity of the
registry, binning of the transactions by message block count, HMAC-SHA256
recomputation of every credential with a constant-time compare, and the
validity bitmask plus count.  Default workload: the throughput sweep's
largest batch, 16M transactions over 1M identities (uniform), message lengths
lognormal (median 200 B, sigma 0.75) clipped to 64..1232 B, 0.5% invalid.

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


def cpu_baseline(w, seconds: float) -> dict:
    """The CPU oracle as it stands on this host: all keys, then a prefix sample of txs."""
    import oracle
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    t = time.perf_counter()
    keys = oracle.derive_keys(w.rev, w.salt, w.info, threads)
    t_derive = time.perf_counter() - t
    probe = min(w.n, 20_000)
    t = time.perf_counter()
    oracle.verify_batch(keys, w.msg, w.off[: probe + 1], w.ids[:probe], w.tags[:probe], threads)
    per_tx = (time.perf_counter() - t) / probe
    sample = int(min(w.n, max(probe, seconds / max(per_tx, 1e-9))))
    sample -= sample % 32 if sample > 32 else 0
    t = time.perf_counter()
    mask, count = oracle.verify_batch(keys, w.msg, w.off[: sample + 1], w.ids[:sample],
                                      w.tags[:sample], threads)
    t_verify = time.perf_counter() - t
    truth = w.truth_bitmask()[: (sample + 31) // 32]
    if sample % 32 == 0 and not np.array_equal(mask, truth):
        raise SystemExit("oracle disagrees with the generator's truth mask")
    step_s = t_derive + t_verify * (w.n / sample)
    return {"value": w.n / step_s, "unit": "attestations/s", "cores": threads, "kind": "oracle",
            "sample": "HKDF for all %d identities (%.2f s) + HMAC verify of the first %d of %d txs "
                      "(%.2f s), verify time scaled to the whole batch" %
                      (w.n_id, t_derive, sample, w.n, t_verify)}


def time_calls(fn, steps: int, warmup: int):
    """Per-call wall times (ms) of fn() bracketed by stream events, after warmup."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        fn()
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    return wall * 1e3 / steps, ev


def bench_batching(args) -> dict:
    """256 blocks of lognormal sizes in one captured replay, against one eager
    multi-block call and against one plain call per block."""
    from paper_2603_10242_amd import workload as W
    log("generating the batching workload (256 blocks)")
    w = W.config4()
    import torch
    from paper_2603_10242_amd import ace
    ace.load()
    torch.cuda.set_device(0)
    edges = np.concatenate([[0], np.cumsum(w.block_sizes)])
    d_msg = ace.to_device(w.msg)
    blocks = [ace.upload_block(None, w.off[a:b + 1], w.ids[a:b], w.tags[a:b], msg_dev=d_msg)
              for a, b in zip(edges[:-1], edges[1:])]
    ks = ace.midstate_keyset(ace.to_device(w.rev), w.salt, w.info)
    L = w.lengths()
    comp = compressions(L)
    g = ace.Graph(ks, max_blocks=len(blocks), max_tx=w.n)
    ws_multi = ace.workspace(ace.verify_workspace_size(ks, blocks, 0))
    ws_one = ace.workspace(max(ace.verify_workspace_size(ks, [b], 0) for b in blocks))
    torch.cuda.synchronize()
    log("uploaded %d txs in %d blocks (%.3f compressions/tx)" % (w.n, len(blocks), comp / w.n))

    def check(tag):
        for blk, a, b in zip(blocks, edges[:-1], edges[1:]):
            m, c = blk.result()
            if c != int(w.truth[a:b].sum()) or not np.array_equal(m, W.pack_bits(w.truth[a:b])):
                raise SystemExit("RESULT MISMATCH in %s" % tag)

    forms = {
        "graph": lambda: g.launch(blocks),
        "multi_block_call": lambda: ace.verify_batch(ks, blocks, ws_multi, 0),
        "per_block_calls": lambda: [ace.verify_batch(ks, [b], ws_one, 0) for b in blocks],
    }
    out = {}
    for name, fn in forms.items():
        fn()
        torch.cuda.synchronize()
        check(name)
        ms, ev = time_calls(fn, args.steps, args.warmup)
        check(name)
        out[name] = {"ms": ms, "p50_ms": float(np.percentile(ev, 50)),
                     "p99_ms": float(np.percentile(ev, 99)), "attestations_per_s": w.n / (ms / 1e3),
                     "pct_peak_int32_valu": 100.0 * comp * I_REF / (ms / 1e3) / 1e12 / PEAK_INT32_TOPS}
        log("%-17s %.3f ms  (p99 %.3f)  %.3g tx/s" % (name, ms, out[name]["p99_ms"],
                                                      out[name]["attestations_per_s"]))
    g.close()
    return {
        "metric": METRIC,
        "value": out["graph"]["attestations_per_s"],
        "unit": "attestations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": out["graph"]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "batching, 256 blocks lognormal(19,500, 1.0) in [1k, 200k]",
                   "n_tx": w.n, "n_id": w.n_id, "ids": "zipf 1.1", "keys": "resident midstates",
                   "block_sizes_min_max": [int(w.block_sizes.min()), int(w.block_sizes.max())]},
        "forms": out,
        "speedup_graph_vs_per_block": out["per_block_calls"]["ms"] / out["graph"]["ms"],
        "p99_ms": out["graph"]["p99_ms"],
        "device": torch.cuda.get_device_name(0),
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16 << 20, help="transactions per batch")
    ap.add_argument("--n-id", type=int, default=1 << 20, help="identities in the registry")
    ap.add_argument("--ids", choices=["uniform", "zipf"], default="uniform")
    ap.add_argument("--keys", choices=["recomputed", "midstate"], default="recomputed",
                    help="derive every identity's key in the step, or use resident midstates")
    ap.add_argument("--mode", choices=["binned", "binned-persistent", "ordered"], default="binned")
    ap.add_argument("--workload", choices=["sweep", "batching"], default="sweep",
                    help="sweep: the throughput sweep (default); batching: 256 uneven blocks")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run three plain device copies of this many bytes (a reference "
                         "for scaling hardware byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(asked for --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        return 2

    if args.workload == "batching":
        print(json.dumps(bench_batching(args)), flush=True)
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
    from paper_2603_10242_amd import ace
    ace.load()
    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
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

    for i in range(max(1, args.warmup)):
        ace.verify_batch(ks, [blk], ws, flags)
        torch.cuda.synchronize()
        if i == 0:
            mask, count = blk.result()
            if count != int(w.truth.sum()) or not np.array_equal(mask, w.truth_bitmask()):
                log("RESULT MISMATCH: count %d, expected %d" % (count, int(w.truth.sum())))
                return 1
            log("warmup step 0 bit-exact with the generator's truth mask (%d valid)" % count)

    ace.profile_read(reset=True)
    ace.profile_enable(True)
    stream = torch.cuda.current_stream()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        ace.verify_batch(ks, [blk], ws, flags)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ace.profile_enable(False)
    prof = ace.profile_read(reset=True)
    step_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ms_per_step = wall * 1e3 / args.steps
    log("timed %d steps: %.3f ms/step (events p50 %.3f, p99 %.3f)"
        % (args.steps, ms_per_step, np.percentile(step_ms, 50), np.percentile(step_ms, 99)))
    mask, count = blk.result()
    if count != int(w.truth.sum()) or not np.array_equal(mask, w.truth_bitmask()):
        log("RESULT MISMATCH after timing")
        return 1

    calls = max(1, prof["calls"])
    verify_s = prof["verify_ms"] / calls / 1e3
    derive_s = prof["derive_ms"] / calls / 1e3
    achieved = verify_comp * I_REF / verify_s / 1e12
    bytes_tx = L.astype(np.float64) + 32 + 4 + 8 + 64 + 1.0 / 8
    verify_bytes = float(bytes_tx.sum())
    step_comp = verify_comp + derive_comp
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
            "traffic": None,
            "per_launch": "%d compressions x %d VALU instr" % (verify_comp, I_REF),
            "avg_ms": verify_s * 1e3,
        },
        "pct_peak_int32_valu_step": 100.0 * step_comp * I_REF / (ms_per_step / 1e3) / 1e12
                                    / PEAK_INT32_TOPS,
        "compressions_per_step": step_comp,
        "gcompressions_per_s": step_comp / (ms_per_step / 1e3) / 1e9,
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "stages_ms": {k: prof[k] / calls for k in ("derive_ms", "bin_ms", "verify_ms",
                                                   "finalize_ms")},
        "derive_pct_peak": (100.0 * derive_comp * I_REF / derive_s / 1e12 / PEAK_INT32_TOPS
                            if derive_comp and derive_s > 0 else None),
        "hbm_gbs_algorithmic_verify": verify_bytes / verify_s / 1e9,
        "device": dev_name,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (about %.0f s)" % args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
