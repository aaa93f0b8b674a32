"""Parity at the benchmarks' full sizes, in the launch configuration bench.py
times (binned, keys derived in the call, the saved launch tuning) and in the
other launch forms at those sizes (persistent verify, captured graphs of each
form, the in-order kernel), under the saved tuning and the library's default
one: every bitmask word, count and root against the CPU oracle, run
multi-threaded over the whole workload (the C oracle verifies the 16M batch
in a few seconds on the host's cores), and against the generator's truth
mask.  Integer work: tolerance 0."""
import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_2603_10242_amd import workload as W

from .conftest import TUNINGS, use_tuning

pytestmark = pytest.mark.gpu

NT = max(1, min(16, os.cpu_count() or 1))  # oracle threads
ORDERED, BUCKETED, PERSISTENT = 0x1, 0x2, 0x4


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def popcount(words: np.ndarray) -> int:
    return int(np.unpackbits(words.view(np.uint8)).sum())


@pytest.fixture(scope="module")
def ace(need_gpu):
    import torch
    from paper_2603_10242_amd import ace as A
    A.load()
    torch.cuda.set_device(0)
    use_tuning(A, "saved")
    yield A
    A.set_tuning(**A.default_tuning())


@pytest.fixture(scope="module")
def sweep16(ace):
    """The throughput sweep's 16M-transaction batch over 1M identities, resident,
    with the oracle's result for all of it."""
    note("generating the 16M-tx sweep workload")
    w = W.config3(n=16 << 20, n_id=1 << 20)
    note("oracle on all %d transactions, %d threads" % (w.n, NT))
    keys = oracle.derive_keys(w.rev, w.salt, w.info, NT)
    omask, ocount = oracle.verify_batch(keys, w.msg, w.off, w.ids, w.tags, NT)
    assert ocount == int(w.truth.sum()) and ocount < w.n
    assert np.array_equal(omask, w.truth_bitmask())
    rev = ace.to_device(w.rev)
    return SimpleNamespace(w=w, keys=keys, omask=omask, ocount=ocount, d_msg=ace.to_device(w.msg),
                           mid=ace.midstate_keyset(rev, w.salt, w.info),
                           rev=ace.rev_keyset(rev, w.salt, w.info))


def sweep_block(ace, s, n):
    w = s.w
    return ace.upload_block(None, w.off[: n + 1], w.ids[:n], w.tags[:n], msg_dev=s.d_msg)


def test_sweep_16M_keys_in_call(ace, sweep16):
    import torch
    note("full size: 16M-tx sweep, 1M identities, binned, keys derived in the call")
    s = sweep16
    blk = sweep_block(ace, s, s.w.n)
    ace.verify_batch(s.rev, [blk], flags=BUCKETED)
    torch.cuda.synchronize()
    mask, count = blk.result()
    assert count == s.ocount
    assert np.array_equal(mask, s.omask)


def expected_grab(ace, n: int) -> int:
    """Wave tiles per atomic grab of the persistent verify kernel for a batch
    of n transactions of the sweep (its bins pad to about n / 64 wave tiles):
    nwaves / (4 grabs x 4 waves x workgroups), clamped to 1..8."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    wgs = ace.get_tuning()["verify_wgs_per_cu"] * cus
    return max(1, min(8, (n // 64) // (wgs * 4 * 4)))


@pytest.mark.parametrize("tuning", TUNINGS)
def test_sweep_persistent_every_grab(ace, sweep16, tuning):
    """The persistent verify kernel on prefixes of the 16M sweep that make it
    take 1, 2, 3-4 and 8 wave tiles per atomic grab (library default: 8
    workgroups per CU; saved: 2), with resident midstates and with keys
    derived in the call; the open mode with auto_persistent set takes the
    same kernel.  Every bitmask word against the oracle."""
    import torch
    s = sweep16
    try:
        use_tuning(ace, tuning)
        grabs = set()
        for n in (1 << 20, 2 << 20, 6 << 20, 16 << 20):
            grabs.add(expected_grab(ace, n))
            note("persistent, tuning %s, n=%d, grab %d" % (tuning, n, expected_grab(ace, n)))
            blk = sweep_block(ace, s, n)
            want = s.omask[: n // 32]
            for kname, ks in (("midstate", s.mid), ("rev", s.rev)):
                for flags, auto in ((BUCKETED | PERSISTENT, 0), (0, 1)):
                    ace.set_tuning(auto_persistent=auto)
                    blk.bitmask.fill_(-1)
                    ace.verify_batch(ks, [blk], flags=flags)
                    torch.cuda.synchronize()
                    mask, count = blk.result()
                    assert count == popcount(want), (n, kname, flags)
                    assert np.array_equal(mask, want), (n, kname, flags)
            ace.set_tuning(auto_persistent=0)
            del blk
        assert 8 in grabs and len(grabs) >= 3, grabs
        # per-bucket caps on tiles per grab (1..8 by inner block count, and
        # one cap for every bucket) change no result
        blk = sweep_block(ace, s, s.w.n)
        for caps in ([1 + (b % 8) for b in range(64)], [1] * 64, [3] * 64):
            ace.set_tuning(grab_cap=caps)
            note("persistent, tuning %s, grab caps %s..." % (tuning, caps[:4]))
            blk.bitmask.fill_(-1)
            ace.verify_batch(s.rev, [blk], flags=BUCKETED | PERSISTENT)
            torch.cuda.synchronize()
            mask, count = blk.result()
            assert count == s.ocount and np.array_equal(mask, s.omask), caps[:4]
    finally:
        use_tuning(ace, "saved")


@pytest.mark.parametrize("tuning", TUNINGS)
def test_sweep_16M_graph_forms(ace, sweep16, tuning):
    """The 16M sweep split into three blocks, through graphs captured in each
    form with keys derived in the replay: the in-order grid-stride kernel (8
    to 32 passes over its grid), the binned dispatcher-scheduled kernel and
    the persistent one (8 tiles per grab); two replays each, every word
    against the oracle."""
    import torch
    s = sweep16
    w = s.w
    edges = [0, 5_000_000, 5_000_013, w.n]
    want = []
    for a, b in zip(edges[:-1], edges[1:]):
        if a % 32 == 0:
            # a block that starts on a word boundary: a slice of the whole
            # batch's result, bits past its end cleared
            m = s.omask[a // 32: (b + 31) // 32].copy()
            if b % 32:
                m[-1] &= np.uint32((1 << (b % 32)) - 1)
            want.append((m, popcount(m)))
        else:
            want.append(oracle.verify_batch(s.keys, w.msg, w.off[a:b + 1], w.ids[a:b],
                                            w.tags[a:b], NT))
    try:
        use_tuning(ace, tuning)
        for gflags in (ORDERED, BUCKETED, BUCKETED | PERSISTENT):
            note("16M graph, tuning %s, flags %d" % (tuning, gflags))
            g = ace.Graph(s.rev, max_blocks=4, max_tx=w.n, flags=gflags)
            try:
                for rep in range(2):
                    blocks = [ace.upload_block(None, w.off[a:b + 1], w.ids[a:b], w.tags[a:b],
                                               msg_dev=s.d_msg)
                              for a, b in zip(edges[:-1], edges[1:])]
                    for blk in blocks:
                        blk.bitmask.fill_(-1)
                    g.launch(blocks)
                    torch.cuda.synchronize()
                    for k, (blk, (omask, ocount)) in enumerate(zip(blocks, want)):
                        mask, count = blk.result()
                        assert count == ocount, (gflags, rep, k)
                        assert np.array_equal(mask, omask), (gflags, rep, k)
            finally:
                g.close()
    finally:
        use_tuning(ace, "saved")


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


@pytest.fixture(scope="module")
def batching(ace):
    """The batching workload (256 blocks of lognormal sizes, 7.66M transactions,
    Zipf identities, resident midstates) with the oracle's result per block."""
    note("generating the batching workload")
    w = W.config4()
    edges = np.concatenate([[0], np.cumsum(w.block_sizes)])
    note("oracle on all %d transactions, %d threads" % (w.n, NT))
    keys = oracle.derive_keys(w.rev, w.salt, w.info, NT)
    want = []
    for a, b in zip(edges[:-1], edges[1:]):
        off = w.off[a:b + 1] - w.off[a]
        want.append(oracle.verify_batch(keys, w.msg[int(w.off[a]):int(w.off[b])], off, w.ids[a:b],
                                        w.tags[a:b], NT))
    return SimpleNamespace(w=w, edges=edges, want=want, d_msg=ace.to_device(w.msg),
                           ks=ace.midstate_keyset(ace.to_device(w.rev), w.salt, w.info))


@pytest.mark.parametrize("tuning", TUNINGS)
@pytest.mark.parametrize("gflags", [0, BUCKETED | PERSISTENT, ORDERED])
def test_batching_256_blocks_graph_replay(ace, batching, tuning, gflags):
    """The batching workload in one captured replay (twice) and in one eager
    multi-block call, with the graph captured in the open form (binned at this
    size), as the persistent binned kernel (8 tiles per grab under the saved
    tuning) and as the in-order grid-stride kernel (15 to 59 passes over its
    grid): every block's bitmask and count against the oracle's for that
    block."""
    import torch
    note("full size: batching workload, 256 blocks, graph flags %d, tuning %s" % (gflags, tuning))
    bt = batching
    w, edges = bt.w, bt.edges
    try:
        use_tuning(ace, tuning)
        g = ace.Graph(bt.ks, max_blocks=len(edges) - 1, max_tx=w.n, flags=gflags)
        try:
            for form in ("graph", "graph", "eager"):
                blocks = [ace.upload_block(None, w.off[a:b + 1], w.ids[a:b], w.tags[a:b],
                                           msg_dev=bt.d_msg)
                          for a, b in zip(edges[:-1], edges[1:])]
                for blk in blocks:
                    blk.bitmask.fill_(-1)
                if form == "graph":
                    g.launch(blocks)
                else:
                    ace.verify_batch(bt.ks, blocks, flags=gflags)
                torch.cuda.synchronize()
                for k, (blk, (omask, ocount)) in enumerate(zip(blocks, bt.want)):
                    mask, count = blk.result()
                    a, b = int(edges[k]), int(edges[k + 1])
                    assert count == ocount == int(w.truth[a:b].sum()), (form, k)
                    assert np.array_equal(mask, omask), (form, k)
        finally:
            g.close()
    finally:
        use_tuning(ace, "saved")


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
