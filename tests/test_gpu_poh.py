"""Parity of the hash-chain segment check on the GPU (ace_poh_verify) with the
CPU oracle and the generator's truth mask (tolerance 0)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2603_10242_amd import workload as W

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


def run(ace, start, end, steps, per_segment=True):
    import torch
    n = start.shape[0]
    s = ace.to_device(np.ascontiguousarray(start, np.uint8).reshape(-1, 32) if n
                      else np.zeros((1, 32), np.uint8))
    e = ace.to_device(np.ascontiguousarray(end, np.uint8).reshape(-1, 32) if n
                      else np.zeros((1, 32), np.uint8))
    if per_segment:
        st = ace.to_device(np.asarray(steps, np.uint32) if n else np.zeros(1, np.uint32))
    else:
        assert n == 0 or (np.asarray(steps) == steps[0]).all()
        st = int(steps[0]) if n else 0
    mask = torch.full((max(1, (n + 31) // 32),), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ace.poh_verify(s[:n], e[:n], st, mask, cnt)
    torch.cuda.synchronize()
    return mask.cpu().numpy().view(np.uint32)[: (n + 31) // 32], int(cnt.item())


@pytest.mark.parametrize("uniform", [True, False])
def test_segments(ace, uniform):
    note("poh segments uniform=%s" % uniform)
    r = np.random.Generator(np.random.PCG64(77))
    steps = 200 if uniform else r.integers(0, 400, size=20_000).astype(np.uint32)
    # one count for every segment cannot express a wrong claimed count: flips only
    w = W.poh_segments(n=20_000, steps=steps, n_invalid=300, seed=W.SEED_BASE + 500,
                       step_errors=not uniform)
    mask, count = run(ace, w.start, w.end, w.steps, per_segment=not uniform)
    omask, ocount = oracle.poh_verify(w.start, w.end, w.steps, nthreads=8)
    assert count == ocount == 19_700 == int(w.truth.sum())
    assert np.array_equal(mask, omask)
    assert np.array_equal(mask, w.truth_bitmask())


def test_one_chain_through_shared_checkpoints(ace):
    """One chain: start = C[0..n-1], end = C[1..n] as views of one array."""
    import torch
    note("poh chained")
    r = np.random.Generator(np.random.PCG64(78))
    steps = r.integers(0, 30, size=600).astype(np.uint32)
    w = W.poh_segments(n=600, steps=steps, chained=True, n_invalid=0, seed=W.SEED_BASE + 501)
    C = np.concatenate([w.start, w.end[-1:]])
    C[300, 5] ^= 4      # a broken checkpoint invalidates the segments on both sides of it
    d = ace.to_device(C)
    mask = torch.zeros(((600 + 31) // 32,), dtype=torch.int32, device="cuda")
    cnt = torch.zeros((1,), dtype=torch.int64, device="cuda")
    ace.poh_verify(d[:600], d[1:], ace.to_device(steps), mask, cnt)
    torch.cuda.synchronize()
    omask, ocount = oracle.poh_verify(C[:600], C[1:], steps)
    assert int(cnt.item()) == ocount
    assert np.array_equal(mask.cpu().numpy().view(np.uint32), omask)
    bits = np.unpackbits(omask.view(np.uint8), bitorder="little")[:600]
    assert bits[299] == 0 and bits[300] == 0 and bits.sum() == 598


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4097])
def test_sizes(ace, n):
    note("poh n=%d" % n)
    w = W.poh_segments(n=n, steps=17, n_invalid=n // 10, seed=W.SEED_BASE + 600 + n,
                       step_errors=False)
    for per_segment in (True, False):
        mask, count = run(ace, w.start, w.end, w.steps if n else np.zeros(0, np.uint32),
                          per_segment)
        assert count == int(w.truth.sum())
        assert np.array_equal(mask, w.truth_bitmask())
