"""Parity at the benchmarks' full sizes, in the launch configuration bench.py
times (binned, keys derived in the call, the saved launch tuning): every
bitmask word, count and root against the CPU oracle, run multi-threaded over
the whole workload (the C oracle verifies the 16M batch in a few seconds on
the host's cores), and against the generator's truth mask.  Integer work:
tolerance 0."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2603_10242_amd import workload as W

pytestmark = pytest.mark.gpu

NT = max(1, min(16, os.cpu_count() or 1))  # oracle threads


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ace(need_gpu):
    import torch
    from paper_2603_10242_amd import ace as A
    from paper_2603_10242_amd import autotune
    A.load()
    torch.cuda.set_device(0)
    autotune.apply_saved()
    return A


def test_sweep_16M_keys_in_call(ace):
    import torch
    note("full size: 16M-tx sweep, 1M identities, binned, keys derived in the call")
    w = W.config3(n=16 << 20, n_id=1 << 20)
    rev = ace.to_device(w.rev)
    blk = ace.upload_block(w.msg, w.off, w.ids, w.tags)
    ks = ace.rev_keyset(rev, w.salt, w.info)
    ace.verify_batch(ks, [blk], flags=ace.ACE_BUCKETED)
    torch.cuda.synchronize()
    mask, count = blk.result()
    note("oracle on all %d transactions, %d threads" % (w.n, NT))
    keys = oracle.derive_keys(w.rev, w.salt, w.info, NT)
    omask, ocount = oracle.verify_batch(keys, w.msg, w.off, w.ids, w.tags, NT)
    assert count == ocount == int(w.truth.sum()) and ocount < w.n
    assert np.array_equal(mask, omask)
    assert np.array_equal(mask, w.truth_bitmask())


def test_paper_form_16M_keys_in_call(ace):
    import torch
    note("full size: 16M paper-form attestations, 1M identities, binned, keys in the call")
    a = W.paper_attestations(n=16 << 20, n_id=1 << 20, id_dist="uniform", p_invalid=0.005)
    rev = ace.to_device(a.rev)
    blk = ace.upload_block(a.payload, a.poff, a.ids, a.att, record_bytes=72)
    ks = ace.rev_keyset(rev, a.domain, a.info)
    ace.verify_attestations(ks, [blk], flags=ace.ACE_BUCKETED)
    torch.cuda.synchronize()
    mask, count = blk.result()
    note("oracle on all %d attestations, %d threads" % (a.n, NT))
    keys = oracle.derive_keys(a.rev, a.domain, a.info, NT)
    omask, ocount = oracle.verify_attest(keys, a.payload, a.poff, a.ids, a.att, NT)
    assert count == ocount == int(a.truth.sum()) and ocount < a.n
    assert np.array_equal(mask, omask)
    assert np.array_equal(mask, a.truth_bitmask())


def test_batching_256_blocks_graph_replay(ace):
    """The batching workload (256 blocks, 7.66M transactions, Zipf identities,
    resident midstates) in one captured replay and in one eager multi-block
    call: every block's bitmask and count against the oracle's for that
    block."""
    import torch
    note("full size: batching workload, 256 blocks in one graph replay")
    w = W.config4()
    edges = np.concatenate([[0], np.cumsum(w.block_sizes)])
    d_msg = ace.to_device(w.msg)
    ks = ace.midstate_keyset(ace.to_device(w.rev), w.salt, w.info)
    note("oracle on all %d transactions, %d threads" % (w.n, NT))
    keys = oracle.derive_keys(w.rev, w.salt, w.info, NT)
    want = []
    for a, b in zip(edges[:-1], edges[1:]):
        off = w.off[a:b + 1] - w.off[a]
        want.append(oracle.verify_batch(keys, w.msg[int(w.off[a]):int(w.off[b])], off, w.ids[a:b],
                                        w.tags[a:b], NT))
    g = ace.Graph(ks, max_blocks=len(edges) - 1, max_tx=w.n)
    try:
        for form in ("graph", "eager"):
            blocks = [ace.upload_block(None, w.off[a:b + 1], w.ids[a:b], w.tags[a:b], msg_dev=d_msg)
                      for a, b in zip(edges[:-1], edges[1:])]
            if form == "graph":
                g.launch(blocks)
            else:
                ace.verify_batch(ks, blocks)
            torch.cuda.synchronize()
            for k, (blk, (omask, ocount)) in enumerate(zip(blocks, want)):
                mask, count = blk.result()
                a, b = int(edges[k]), int(edges[k + 1])
                assert count == ocount == int(w.truth[a:b].sum()), (form, k)
                assert np.array_equal(mask, omask), (form, k)
    finally:
        g.close()


def test_serving_full_size_requests(ace):
    """Serving at the benchmark's scale: the 4M-identity midstate cache
    resident, 3,000 requests of lognormal(1,000, 1.5) sizes in [1, 50,000]
    cut from the 4M-transaction pool and submitted from 8 threads as a
    backlog (continuous batching, 4 batches in flight, the benchmark's arena
    and staging sizes): every request's bitmask and count against the
    oracle's for its range."""
    import threading
    import torch
    note("full size: serving, 3,000 requests from a 4M-transaction pool, 4M identities")
    pool = W.config5_pool()
    ks = ace.midstate_keyset(ace.to_device(pool.rev), pool.salt, pool.info)
    arena = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    st = ace.Stream.create(ks, arena, staging_bytes=2048 << 20, max_inflight=4)
    sizes = W.serving_request_sizes(3000)
    starts = np.random.Generator(np.random.PCG64(55)).integers(0, pool.n - sizes)
    reqs = [(int(a), int(a + z)) for a, z in zip(starts, sizes)]
    tickets = [None] * len(reqs)

    def client(t0):
        for k in range(t0, len(reqs), 8):
            lo, hi = reqs[k]
            tickets[k] = st.submit(pool.msg, pool.off[lo:hi + 1], pool.ids[lo:hi], pool.tags[lo:hi])

    threads = [threading.Thread(target=client, args=(t,)) for t in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert all(t is not None for t in tickets)
    note("oracle on all %d requests (%d transactions), %d threads" % (len(reqs), int(sizes.sum()), NT))
    keys = oracle.derive_keys(pool.rev, pool.salt, pool.info, NT)
    try:
        for (lo, hi), t in zip(reqs, tickets):
            mask, count = st.result(t)
            omask, ocount = oracle.verify_batch(keys, pool.msg, pool.off[lo:hi + 1], pool.ids[lo:hi],
                                                pool.tags[lo:hi], NT)
            assert count == ocount == int(pool.truth[lo:hi].sum()), (lo, hi)
            assert np.array_equal(mask, omask), (lo, hi)
        stats = st.stats()
        assert stats["completed"] == len(reqs) and stats["failed"] == 0
        assert stats["max_batch_requests"] > 1  # requests were merged into batches
    finally:
        st.close()


def test_merkle_256_blocks(ace):
    import torch
    note("full size: Merkle roots of the batching workload's 256 blocks of 72-byte records")
    sizes = W.batching_block_sizes()
    n = int(sizes.sum())
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([W.SEED_BASE + 8])))
    data = rng.integers(0, 256, size=72 * n, dtype=np.uint8)
    off = np.arange(n + 1, dtype=np.uint64) * 72
    d_data, d_off = ace.to_device(data), ace.to_device(off)
    roots = torch.zeros((sizes.size, 32), dtype=torch.uint8, device="cuda")
    trees, first = [], 0
    for b, m in enumerate(sizes):
        trees.append((d_data, d_off[first:first + int(m) + 1], int(m), roots[b]))
        first += int(m)
    ace.merkle_roots(trees)
    torch.cuda.synchronize()
    got = roots.cpu().numpy()
    note("oracle on all %d trees (%d leaves)" % (sizes.size, n))
    want = oracle.merkle_roots(data, off, sizes)
    assert np.array_equal(got, want)


def test_hash_chain_262144_segments(ace):
    import torch
    note("full size: 262,144 hash-chain segments of 1,024 hashes")
    w = W.poh_segments(n=1 << 18, steps=1024, step_errors=False)
    s, e = ace.to_device(w.start), ace.to_device(w.end)
    mask = torch.zeros((w.n + 31) // 32, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ace.poh_verify(s, e, 1024, mask, cnt)  # uniform steps, as the benchmark launches it
    torch.cuda.synchronize()
    m = mask.cpu().numpy().view(np.uint32)
    note("oracle on all %d segments, %d threads" % (w.n, NT))
    omask, ocount = oracle.poh_verify(w.start, w.end, w.steps, NT)
    assert int(cnt.item()) == ocount == int(w.truth.sum()) and ocount < w.n
    assert np.array_equal(m, omask)
    assert np.array_equal(m, w.truth_bitmask())
