"""Parity at the benchmarks' full sizes, in the launch configuration bench.py
times (binned, keys derived in the call, the saved launch tuning): the whole
bitmask against the generator's truth mask, and a sample of transactions
checked one by one against the CPU oracle (which cannot verify 16M
transactions in a test's time).  Integer work: tolerance 0."""
import sys

import numpy as np
import pytest

import oracle
from paper_2603_10242_amd import workload as W

pytestmark = pytest.mark.gpu

N_SAMPLE = 20000


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


def gather(data, off, idx):
    """The records idx of a packed array, packed again (offsets from 0)."""
    lens = (off[idx + 1] - off[idx]).astype(np.int64)
    noff = np.zeros(idx.size + 1, dtype=np.uint64)
    noff[1:] = np.cumsum(lens)
    out = np.concatenate([data[int(off[i]):int(off[i + 1])] for i in idx]) if idx.size else data[:0]
    return out, noff


def sample(n, seed, invalid, k=N_SAMPLE):
    """About k indices: random ones, the first k // 4 invalid ones, and the
    last transaction (ragged tail)."""
    r = np.random.Generator(np.random.PCG64(seed))
    bad = np.flatnonzero(invalid)[: k // 4]
    idx = np.unique(np.concatenate([r.choice(n, k - bad.size - 1, replace=False), bad, [n - 1]]))
    return idx.astype(np.int64)


def bit(mask, i):
    return (mask[i >> 5] >> (i & 31)) & 1


def test_sweep_16M_keys_in_call_sampled(ace):
    import torch
    note("full size: 16M-tx sweep, 1M identities, binned, keys derived in the call")
    w = W.config3(n=16 << 20, n_id=1 << 20)
    rev = ace.to_device(w.rev)
    blk = ace.upload_block(w.msg, w.off, w.ids, w.tags)
    ks = ace.rev_keyset(rev, w.salt, w.info)
    ace.verify_batch(ks, [blk], flags=ace.ACE_BUCKETED)
    torch.cuda.synchronize()
    mask, count = blk.result()
    assert count == int(w.truth.sum())
    assert np.array_equal(mask, w.truth_bitmask())
    idx = sample(w.n, 71, ~w.truth)
    note("oracle on %d sampled transactions" % idx.size)
    ids = w.ids[idx]
    uid, local = np.unique(ids, return_inverse=True)
    keys = oracle.derive_keys(w.rev[uid], w.salt, w.info, 8)
    msg, off = gather(w.msg, w.off, idx)
    omask, ocount = oracle.verify_batch(keys, msg, off, local.astype(np.uint32), w.tags[idx], 8)
    got = np.array([bit(mask, int(i)) for i in idx], dtype=np.uint32)
    want = np.array([bit(omask, k) for k in range(idx.size)], dtype=np.uint32)
    assert np.array_equal(got, want)
    assert ocount == int(want.sum()) and ocount < idx.size  # the sample holds invalid ones


def test_paper_form_16M_keys_in_call_sampled(ace):
    import torch
    note("full size: 16M paper-form attestations, 1M identities, binned, keys in the call")
    a = W.paper_attestations(n=16 << 20, n_id=1 << 20, id_dist="uniform", p_invalid=0.005)
    rev = ace.to_device(a.rev)
    blk = ace.upload_block(a.payload, a.poff, a.ids, a.att, record_bytes=72)
    ks = ace.rev_keyset(rev, a.domain, a.info)
    ace.verify_attestations(ks, [blk], flags=ace.ACE_BUCKETED)
    torch.cuda.synchronize()
    mask, count = blk.result()
    assert count == int(a.truth.sum())
    assert np.array_equal(mask, a.truth_bitmask())
    idx = sample(a.n, 72, ~a.truth)
    note("oracle on %d sampled attestations" % idx.size)
    uid, local = np.unique(a.ids[idx], return_inverse=True)
    keys = oracle.derive_keys(a.rev[uid], a.domain, a.info, 8)
    payload, poff = gather(a.payload, a.poff, idx)
    omask, ocount = oracle.verify_attest(keys, payload, poff, local.astype(np.uint32), a.att[idx], 8)
    got = np.array([bit(mask, int(i)) for i in idx], dtype=np.uint32)
    want = np.array([bit(omask, k) for k in range(idx.size)], dtype=np.uint32)
    assert np.array_equal(got, want)
    assert ocount == int(want.sum()) and ocount < idx.size


def test_merkle_256_blocks_sampled_trees(ace):
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
    firsts = np.concatenate([[0], np.cumsum(sizes)])
    picks = sorted({0, 1, int(np.argmax(sizes)), int(np.argmin(sizes)), sizes.size // 2, sizes.size - 1})
    for b in picks:
        lo, hi = int(firsts[b]), int(firsts[b + 1])
        want = oracle.merkle_roots(data[72 * lo:72 * hi], off[lo:hi + 1] - off[lo], [hi - lo])
        assert np.array_equal(got[b], want[0]), b


def test_hash_chain_262144_segments_sampled(ace):
    import torch
    note("full size: 262,144 hash-chain segments of 1,024 hashes")
    w = W.poh_segments(n=1 << 18, steps=1024, step_errors=False)
    s, e = ace.to_device(w.start), ace.to_device(w.end)
    mask = torch.zeros((w.n + 31) // 32, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ace.poh_verify(s, e, 1024, mask, cnt)  # uniform steps, as the benchmark launches it
    torch.cuda.synchronize()
    m = mask.cpu().numpy().view(np.uint32)
    assert int(cnt.item()) == int(w.truth.sum())
    assert np.array_equal(m, w.truth_bitmask())
    idx = sample(w.n, 73, ~w.truth, 4096)
    omask, ocount = oracle.poh_verify(w.start[idx], w.end[idx], w.steps[idx], 8)
    got = np.array([bit(m, int(i)) for i in idx], dtype=np.uint32)
    want = np.array([bit(omask, k) for k in range(idx.size)], dtype=np.uint32)
    assert np.array_equal(got, want)
    assert ocount == int(want.sum()) and ocount < idx.size
