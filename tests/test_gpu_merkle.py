"""Parity of the Merkle roots on the GPU (ace_merkle_roots) with the CPU
oracle: every root byte identical (tolerance 0)."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ace(need_gpu):
    import torch
    from paper_2603_10242_amd import ace as A
    A.load()
    torch.cuda.set_device(0)
    return A


def forest(seed, sizes, lo=0, hi=200, lead=0):
    r = np.random.Generator(np.random.PCG64(seed))
    lens = r.integers(lo, hi + 1, size=int(np.sum(sizes)))
    off = np.zeros(lens.size + 1, np.uint64)
    np.cumsum(lens, out=off[1:])
    off += lead
    data = r.integers(0, 256, size=int(off[-1]) + 1, dtype=np.uint8)[: int(off[-1])]
    return data, off


def gpu_roots(ace, data, off, sizes, separate=False):
    """All trees over one data/offset array (shared), or each tree with its own."""
    import torch
    roots = torch.zeros((len(sizes), 32), dtype=torch.uint8, device="cuda")
    trees, first = [], 0
    d_data = ace.to_device(data if data.size else np.zeros(4, np.uint8))
    for b, n in enumerate(sizes):
        n = int(n)
        if separate:
            sub = off[first:first + n + 1]
            base = int(sub[0])
            dd = ace.to_device(data[base:int(sub[-1])] if n and sub[-1] > base
                               else np.zeros(4, np.uint8))
            do = ace.to_device((sub - base).astype(np.uint64))
        else:
            dd = d_data
            do = ace.to_device(off[first:first + n + 1] if n else off[:1])
        trees.append((dd, do, n, roots[b]))
        first += n
    ace.merkle_roots(trees)
    torch.cuda.synchronize()
    return roots.cpu().numpy()


@pytest.mark.parametrize("separate", [False, True])
def test_every_tree_size_0_to_300(ace, separate):
    note("merkle sizes 0..300 separate=%s" % separate)
    sizes = np.arange(0, 301)
    data, off = forest(61, sizes, lead=3)
    got = gpu_roots(ace, data, off, sizes, separate)
    want = oracle.merkle_roots(data, off, sizes)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("lead", [0, 1, 2, 3])
def test_record_leaves_every_alignment(ace, lead):
    """72-byte leaves (the check records of the paper form) starting at each
    byte alignment, in waves of 72-byte leaves only and in waves where a few
    leaves have other lengths (65, 71, 73, 119, 0), so that both leaf paths
    run; the last record ends the data (no bytes past it)."""
    note("merkle record leaves lead=%d" % lead)
    r = np.random.Generator(np.random.PCG64(720 + lead))
    sizes = [1, 2, 63, 64, 65, 127, 128, 129, 700, 1000]
    lens = np.full(int(np.sum(sizes)), 72, np.int64)
    odd = r.choice(lens.size, size=40, replace=False)
    lens[odd[odd > 1300]] = r.choice([65, 71, 73, 119, 0], size=int(np.sum(odd > 1300)))
    off = np.zeros(lens.size + 1, np.uint64)
    np.cumsum(lens, out=off[1:])
    off += lead
    data = r.integers(0, 256, size=int(off[-1]), dtype=np.uint8)
    for separate in (False, True):
        got = gpu_roots(ace, data, off, sizes, separate)
        assert np.array_equal(got, oracle.merkle_roots(data, off, sizes))


def test_leaf_lengths_0_to_300_misaligned(ace):
    """Leaves of every length 0..300 (each padding case) at every alignment."""
    note("merkle leaf lengths")
    lens = np.concatenate([np.arange(0, 301), np.arange(300, -1, -1)])
    off = np.zeros(lens.size + 1, np.uint64)
    np.cumsum(lens, out=off[1:])
    off += 1
    r = np.random.Generator(np.random.PCG64(62))
    data = r.integers(0, 256, size=int(off[-1]), dtype=np.uint8)
    sizes = [1, 2, 3, 5, 8, 13, 21, 34, 55, 89]
    sizes.append(lens.size - sum(sizes))
    assert np.array_equal(gpu_roots(ace, data, off, sizes), oracle.merkle_roots(data, off, sizes))


def test_large_trees_and_empty_trees(ace):
    note("merkle large")
    sizes = [0, 70_001, 1, 0, 65_536, 65_537, 2, 0]
    data, off = forest(63, sizes, lo=60, hi=160)
    assert np.array_equal(gpu_roots(ace, data, off, sizes), oracle.merkle_roots(data, off, sizes))


@pytest.mark.parametrize("sizes", [[1024], [1025], [2048], [2049], [1023, 1024, 1025, 2047, 2048, 2049, 3]])
def test_sizes_around_the_top_levels(ace, sizes):
    """Trees around the width at which the levels move into one launch (a
    workgroup per tree holding at most 1,024 nodes in LDS): exactly 1,024
    nodes at the first of those levels, one more, and mixes of both."""
    note("merkle top-level boundaries %s" % sizes)
    data, off = forest(64, sizes, lo=0, hi=90)
    assert np.array_equal(gpu_roots(ace, data, off, sizes), oracle.merkle_roots(data, off, sizes))


def test_decreasing_offsets_hash_as_empty(ace):
    note("merkle decreasing offsets")
    data = np.arange(40, dtype=np.uint8)
    off = np.array([0, 10, 4, 30, 40], np.uint64)
    assert np.array_equal(gpu_roots(ace, data, off, [4]), oracle.merkle_roots(data, off, [4]))
