"""Serving engine on the GPU: continuous batching of requests from host memory.
Every request's bitmask and count must equal the generator's truth mask, and a
request's result must be identical alone and inside a busy mix."""
import sys
import threading

import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def pool():
    return W.subset(W.config2(), 0, 60_000)


def requests(pool, count, seed, max_size=5000):
    r = np.random.Generator(np.random.PCG64(seed))
    sizes = np.clip(np.rint(np.exp(np.log(300) + 1.3 * r.standard_normal(count))), 0, max_size)
    out = []
    for s in sizes.astype(int):
        lo = int(r.integers(0, pool.n - s))
        out.append((lo, lo + s))
    return out


def submit(stream, pool, lo, hi, **kw):
    return stream.submit(pool.msg, pool.off[lo:hi + 1], pool.ids[lo:hi], pool.tags[lo:hi], **kw)


def check(stream, pool, reqs, tickets):
    for (lo, hi), t in zip(reqs, tickets):
        mask, count = stream.result(t)
        assert count == int(pool.truth[lo:hi].sum()), (lo, hi)
        assert np.array_equal(mask, W.pack_bits(pool.truth[lo:hi])), (lo, hi)


def make(ace, pool, keys="midstate", arena_mb=256, plain=False, inflight=4):
    import torch
    rev = ace.to_device(pool.rev)
    ks = ace.midstate_keyset(rev, pool.salt, pool.info) if keys == "midstate" else \
        ace.rev_keyset(rev, pool.salt, pool.info)
    torch.cuda.synchronize()
    arena = torch.empty(arena_mb << 20, dtype=torch.uint8, device="cuda")
    return ace.Stream.create(ks, arena, staging_bytes=64 << 20, max_inflight=inflight, plain=plain)


@pytest.mark.parametrize("keys", ["midstate", "rev"])
def test_many_requests_from_threads(ace, pool, keys):
    note("stream keys=%s" % keys)
    s = make(ace, pool, keys)
    reqs = requests(pool, 300, 11)
    tickets = [None] * len(reqs)

    def client(k0):
        for k in range(k0, len(reqs), 3):
            tickets[k] = submit(s, pool, *reqs[k])

    ths = [threading.Thread(target=client, args=(k,)) for k in range(3)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    check(s, pool, reqs, tickets)
    st = s.stats()
    assert st["completed"] == 300 and st["failed"] == 0
    s.close()


def test_alone_equals_in_mix(ace, pool):
    note("stream alone vs mix")
    reqs = requests(pool, 200, 12)
    probes = [3, 50, 199]
    alone = make(ace, pool, plain=True)
    ref = {p: alone.result(submit(alone, pool, *reqs[p])) for p in probes}
    alone.close()
    mix = make(ace, pool, inflight=4)
    tickets = [submit(mix, pool, lo, hi) for lo, hi in reqs]
    for p in probes:
        m, c = mix.result(tickets[p])
        assert c == ref[p][1] and np.array_equal(m, ref[p][0])
    check(mix, pool, reqs, tickets)
    assert mix.stats()["max_batch_requests"] > 1
    mix.close()


def test_small_arena_admission(ace, pool):
    note("stream small arena")
    s = make(ace, pool, arena_mb=4, inflight=8)
    reqs = requests(pool, 150, 13, max_size=3000)
    tickets = [submit(s, pool, lo, hi) for lo, hi in reqs]
    check(s, pool, reqs, tickets)
    st = s.stats()
    assert st["arena_peak_bytes"] <= st["arena_capacity_bytes"]
    with pytest.raises(ace.AceError) as e:
        submit(s, pool, 0, 50_000)
    assert e.value.code == ace.ACE_ERR_TOO_LARGE
    s.close()


def test_plain_form(ace, pool):
    s = make(ace, pool, plain=True)
    reqs = requests(pool, 40, 14)
    tickets = [submit(s, pool, lo, hi) for lo, hi in reqs]
    check(s, pool, reqs, tickets)
    st = s.stats()
    assert st["batches"] == 40 and st["max_batch_requests"] == 1
    s.close()
