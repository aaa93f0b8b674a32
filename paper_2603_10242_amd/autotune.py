"""Autotuner for the launch shapes of libace.so.

Measures, on the device at hand, the candidates the library can run and
installs the fastest through ace_set_tuning:

* binned_min_tx: the batch size from which binning by block count beats the
  in-order kernel (the binning passes cost a few launches; below this size
  they do not pay);
* verify_wgs_per_cu ("tiles per CU"): workgroups per CU of the persistent
  verify kernel (and of the graph's in-order one), and whether the open mode
  should use the persistent kernel at all (auto_persistent);
* aux_wgs_per_cu: workgroups per CU of the binning and finalize passes;
* derive_wgs_per_cu: workgroups per CU of the key derivation while it runs on
  a second stream beside the binning passes (fewer leave room for them);
* grab_cap, per length bucket (inner block count ranges): wave tiles the
  persistent verify kernel takes per atomic grab while it works on that
  bucket, measured on batches drawn from the bucket alone, each against the
  dispatcher-scheduled kernel on the same batch;
* graph_flags: the launch form of the batching graph (the dispatcher-
  scheduled binned kernel, or the persistent one with the tuned caps),
  whichever replays the 256-block batching workload faster.

One transaction always owns one lane: SHA-256 is a Merkle-Damgard chain, so
the blocks of one message cannot be split across lanes; splitting one
compression's round and schedule work between lanes costs more lane
instructions than it saves in latency (the measured two-lane candidate is
described with the kernels' design).  The result is stored as JSON keyed by GPU architecture and CU count
(``tuning_<arch>_<cus>cu.json`` next to this file) and applied by
``apply_saved()``.

Run: python -m paper_2603_10242_amd.autotune
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def device_key() -> tuple[str, int]:
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return arch, int(p.multi_processor_count)


def tuning_path(arch: str, cus: int) -> str:
    return os.path.join(HERE, "tuning_%s_%dcu.json" % (arch, cus))


def apply_saved(verbose: bool = False) -> dict | None:
    """Installs the saved tuning for this device, if there is one."""
    from . import ace
    try:
        arch, cus = device_key()
    except Exception:
        return None
    path = tuning_path(arch, cus)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        saved = json.load(fh)
    ace.set_tuning(**saved["tuning"])
    if verbose:
        print("autotune: applied %s" % path, file=sys.stderr)
    return saved["tuning"]


def saved_graph_flags() -> int:
    """Launch form of the batching graph in the saved tuning (0: the open form,
    binned at the batching workload's size)."""
    try:
        arch, cus = device_key()
        with open(tuning_path(arch, cus)) as fh:
            return int(json.load(fh).get("graph_flags", 0))
    except Exception:
        return 0


def _time(fn, reps: int = 5) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        best = min(best, s.elapsed_time(e))
    return best


# Length buckets of the persistent kernel's sweep: ranges of the inner block
# count nb = ceil((L + 9) / 64); the throughput sweep's messages (64..1232 B)
# have nb 2..20.
BUCKETS = ((2, 2), (3, 3), (4, 4), (5, 5), (6, 7), (8, 11), (12, 20), (21, 64))


def _time_stream(fn, reps: int = 20) -> float:
    """Mean time of `reps` calls enqueued back to back on the current stream
    (launch latency hidden behind the previous call, as in a serving loop)."""
    import torch
    fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def run(sizes=(4096, 16384, 65536, 262144, 1 << 20, 4 << 20), big: int = 4 << 20,
        write: bool = True, log=print, out_dir: str | None = None,
        derive_n: int = 16 << 20, bucket_n: int = 1 << 20) -> dict:
    import torch

    from . import ace
    from . import workload as W

    ace.load()
    torch.cuda.set_device(0)
    arch, cus = device_key()
    default = ace.get_tuning()
    log("autotune on %s (%d CUs)" % (arch, cus))
    w = W.config3(n=max(max(sizes), big), n_id=1 << 18)
    ks = ace.midstate_keyset(ace.to_device(w.rev), w.salt, w.info)
    d_msg = ace.to_device(w.msg)
    meas = []

    def block(n):
        return ace.upload_block(None, w.off[: n + 1], w.ids[:n], w.tags[:n], msg_dev=d_msg)

    # 1. in-order vs binned by batch size
    crossover = None
    for n in sizes:
        blk = block(n)
        t_ord = _time(lambda: ace.verify_batch(ks, [blk], flags=ace.ACE_ORDERED))
        t_bin = _time(lambda: ace.verify_batch(ks, [blk], flags=ace.ACE_BUCKETED))
        meas.append({"n": n, "ordered_ms": t_ord, "binned_ms": t_bin})
        log("n=%8d ordered %.3f ms, binned %.3f ms" % (n, t_ord, t_bin))
        if crossover is None and t_bin < t_ord:
            crossover = n
    binned_min = crossover if crossover is not None else (1 << 62)

    # 2. persistent verify: workgroups per CU, against the dispatcher-scheduled
    # kernel, at three batch sizes; the open mode uses it only if it wins at all
    psizes = sorted({min(big, 1 << 18), min(big, 1 << 20), big})
    blks = {n: block(n) for n in psizes}
    t_plain = {n: _time(lambda: ace.verify_batch(ks, [blks[n]], flags=ace.ACE_BUCKETED))
               for n in psizes}
    best = (float("inf"), None, False)   # (sum of time ratios, wgs per CU, wins everywhere)
    for wpc in (1, 2, 4, 8, 16):
        ace.set_tuning(verify_wgs_per_cu=wpc)
        ratios = []
        for n in psizes:
            t = _time(lambda: ace.verify_batch(ks, [blks[n]],
                                               flags=ace.ACE_BUCKETED | ace.ACE_PERSISTENT))
            meas.append({"n": n, "persistent_wgs_per_cu": wpc, "ms": t,
                         "dispatcher_ms": t_plain[n]})
            ratios.append(t / t_plain[n])
        log("persistent %2d WG/CU: %s of the dispatcher-scheduled time" %
            (wpc, ", ".join("%.3f at n=%d" % (r, n) for r, n in zip(ratios, psizes))))
        if sum(ratios) < best[0]:
            best = (sum(ratios), wpc, all(r < 1.0 for r in ratios))
    # the persistent kernel's shape is kept even when the dispatcher-scheduled
    # kernel wins, for callers that ask for it (ACE_PERSISTENT) and for the
    # graph's grid-stride in-order kernel, which uses the same workgroups per CU
    best_wpc = best[1]
    blk = blks[big]

    # 3. binning and finalize passes: workgroups per CU
    ace.set_tuning(verify_wgs_per_cu=best_wpc)
    best_aux = (float("inf"), default["aux_wgs_per_cu"])
    for apc in (2, 4, 8, 16):
        ace.set_tuning(aux_wgs_per_cu=apc)
        t = _time(lambda: ace.verify_batch(ks, [blk], flags=ace.ACE_BUCKETED))
        meas.append({"n": big, "aux_wgs_per_cu": apc, "ms": t})
        log("aux %2d WG/CU: %.3f ms" % (apc, t))
        if t < best_aux[0]:
            best_aux = (t, apc)

    # 4. key derivation beside the binning passes (keys derived in the call):
    # workgroups per CU, 0 = as with the GPU to itself (at most four per CU,
    # lanes striding over the identities).  Measured on the
    # throughput sweep's batch (16M transactions, 1M identities): the best
    # share depends on how long the binning passes run beside the derivation,
    # and at 4M transactions they end well before it.
    ace.set_tuning(aux_wgs_per_cu=int(best_aux[1]))
    wd = W.config3(n=derive_n, n_id=1 << 20)
    dblk = ace.upload_block(wd.msg, wd.off, wd.ids, wd.tags)
    rks = ace.rev_keyset(ace.to_device(wd.rev), wd.salt, wd.info)
    best_der = (float("inf"), default.get("derive_wgs_per_cu", 1))
    for dpc in (0, 1, 2, 3, 4):
        ace.set_tuning(derive_wgs_per_cu=dpc)
        t = _time(lambda: ace.verify_batch(rks, [dblk], flags=ace.ACE_BUCKETED))
        meas.append({"n": derive_n, "n_id": int(wd.n_id), "derive_wgs_per_cu": dpc, "ms": t})
        log("derive %2d WG/CU beside binning: %.3f ms" % (dpc, t))
        if t < best_der[0]:
            best_der = (t, dpc)

    ace.set_tuning(derive_wgs_per_cu=int(best_der[1]))
    del dblk, rks, wd

    # 5. per length bucket: the persistent kernel's tiles per grab, on batches
    # whose messages all fall in the bucket, against the dispatcher-scheduled
    # kernel on the same batch
    caps = [0] * 64
    buckets = []
    for k, (lo, hi) in enumerate(BUCKETS):
        lmin, lmax = max(0, 64 * (lo - 1) - 8), 64 * hi - 9
        nb_n = bucket_n if hi <= 20 else bucket_n // 4   # long messages: fewer of them
        wb = W.generate("bucket-%d-%d" % (lo, hi), W.SEED_BASE + 40 + k, n=nb_n, n_id=1 << 18,
                        lengths=lambda r, n, a=lmin, b=lmax: r.integers(a, b + 1, size=n))
        kb = ace.midstate_keyset(ace.to_device(wb.rev), wb.salt, wb.info)
        bb = ace.upload_block(wb.msg, wb.off, wb.ids, wb.tags)
        ws = ace.workspace(ace.verify_workspace_size(kb, [bb], ace.ACE_BUCKETED))
        row = {"nb": [lo, hi], "n": nb_n,
               "dispatcher_ms": min(_time_stream(lambda: ace.verify_batch(kb, [bb], ws, ace.ACE_BUCKETED), 10)
                                    for _ in range(3))}
        best_cap = (float("inf"), 0)
        for cap in (1, 2, 4, 8):
            ace.set_tuning(grab_cap=[cap] * 64)
            t = min(_time_stream(lambda: ace.verify_batch(kb, [bb], ws,
                                                          ace.ACE_BUCKETED | ace.ACE_PERSISTENT), 10)
                    for _ in range(3))
            row["persistent_cap%d_ms" % cap] = t
            if t < best_cap[0]:
                best_cap = (t, cap)
        row["cap"] = best_cap[1]
        row["persistent_over_dispatcher"] = best_cap[0] / row["dispatcher_ms"]
        for nb in range(lo, hi + 1):
            caps[nb - 1] = best_cap[1]
        if hi == 64:
            caps[63] = best_cap[1]
        buckets.append(row)
        log("bucket nb %2d..%2d: dispatcher %.3f ms, persistent %s -> cap %d (%.3f of dispatcher)" % (
            lo, hi, row["dispatcher_ms"],
            ", ".join("%.3f" % row["persistent_cap%d_ms" % c] for c in (1, 2, 4, 8)), best_cap[1],
            row["persistent_over_dispatcher"]))
        del bb, kb, wb, ws
    ace.set_tuning(grab_cap=caps)

    # 6. the batching graph's launch form on the batching workload itself
    w4 = W.config4()
    edges = np.concatenate([[0], np.cumsum(w4.block_sizes)])
    d4 = ace.to_device(w4.msg)
    blocks = [ace.upload_block(None, w4.off[a:b + 1], w4.ids[a:b], w4.tags[a:b], msg_dev=d4)
              for a, b in zip(edges[:-1], edges[1:])]
    k4 = ace.midstate_keyset(ace.to_device(w4.rev), w4.salt, w4.info)
    graph_ms = {}
    for name, gflags in (("dispatcher", ace.ACE_BUCKETED),
                         ("persistent", ace.ACE_BUCKETED | ace.ACE_PERSISTENT)):
        g = ace.Graph(k4, max_blocks=len(blocks), max_tx=w4.n, flags=gflags)
        graph_ms[name] = min(_time_stream(lambda: g.launch(blocks)) for _ in range(3))
        g.close()
    graph_flags = (ace.ACE_BUCKETED | ace.ACE_PERSISTENT
                   if graph_ms["persistent"] < graph_ms["dispatcher"] else ace.ACE_BUCKETED)
    meas.append({"batching_graph_ms": graph_ms, "n": int(w4.n), "blocks": len(blocks)})
    log("batching graph: dispatcher-scheduled %.3f ms, persistent %.3f ms -> flags %d" % (
        graph_ms["dispatcher"], graph_ms["persistent"], graph_flags))

    tuning = {"binned_min_tx": int(binned_min), "verify_wgs_per_cu": int(best_wpc),
              "aux_wgs_per_cu": int(best_aux[1]), "auto_persistent": int(best[2]),
              "derive_wgs_per_cu": int(best_der[1]), "grab_cap": caps}
    ace.set_tuning(**tuning)
    result = {"arch": arch, "cus": cus, "tuning": tuning, "graph_flags": int(graph_flags),
              "lanes_per_message": 1, "buckets": buckets,
              "measured": meas, "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    if write:
        path = tuning_path(arch, cus)
        if out_dir:
            path = os.path.join(out_dir, os.path.basename(path))
        with open(path, "w") as fh:
            json.dump(result, fh, indent=1)
        log("wrote %s" % path)
    return result


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="measure and store the launch tuning")
    ap.add_argument("--out", default=None, help="directory for the JSON (default: the package)")
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    out = run(log=lambda m: print(m, file=sys.stderr, flush=True), out_dir=a.out)
    print(json.dumps(out["tuning"]))
