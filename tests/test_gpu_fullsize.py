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
