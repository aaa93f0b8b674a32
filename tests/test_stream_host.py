"""The serving engine's queue, admission and retirement logic on the CPU.

The engine runs with its host backend: the arena is host memory and each
batch is verified by a callback -- here the CPU oracle.  Everything else
(staging, arena allocation, batching, out-of-order retirement, tickets,
error paths) is the same code the GPU engine runs."""
import threading

import numpy as np
import pytest

import oracle
from paper_2603_10242_amd import workload as W


@pytest.fixture(scope="module")
def ace():
    from paper_2603_10242_amd import ace as A
    A.load()
    return A


@pytest.fixture(scope="module")
def pool():
    return W.subset(W.config2(), 0, 30_000)


def oracle_verify(keys):
    def verify(msg, off, ids, tags):
        return oracle.verify_batch(keys, msg, off, ids, tags)
    return verify


def requests(pool, count, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    sizes = np.clip(np.rint(np.exp(np.log(200) + 1.2 * r.standard_normal(count))), 0, 3000)
    out = []
    for s in sizes.astype(int):
        lo = int(r.integers(0, pool.n - s))
        out.append((lo, lo + s))
    return out


def submit(stream, pool, lo, hi, **kw):
    return stream.submit(pool.msg, pool.off[lo:hi + 1], pool.ids[lo:hi], pool.tags[lo:hi], **kw)


def expect(pool, lo, hi):
    return W.pack_bits(pool.truth[lo:hi]), int(pool.truth[lo:hi].sum())


def test_requests_from_many_threads(ace, pool):
    s = ace.Stream.create_host(oracle_verify(pool.keys), arena_bytes=8 << 20,
                               staging_bytes=8 << 20, max_inflight=4)
    reqs = requests(pool, 200, 1)
    tickets = [None] * len(reqs)

    def client(k0):
        for k in range(k0, len(reqs), 4):
            tickets[k] = submit(s, pool, *reqs[k])

    ths = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    for (lo, hi), t in zip(reqs, tickets):
        mask, count = s.result(t)
        em, ec = expect(pool, lo, hi)
        assert count == ec and np.array_equal(mask, em)
        s.release(t)
    st = s.stats()
    assert st["completed"] == 200 and st["failed"] == 0
    assert st["batches"] <= 200 and st["max_batch_requests"] >= 1
    assert st["arena_peak_bytes"] <= st["arena_capacity_bytes"]
    s.close()


def test_alone_equals_in_mix(ace, pool):
    reqs = requests(pool, 60, 2)
    probe = reqs[7]
    alone = ace.Stream.create_host(oracle_verify(pool.keys), 4 << 20, 4 << 20, 1, plain=True)
    a = alone.result(submit(alone, pool, *probe))
    alone.close()
    import time

    def slow(msg, off, ids, tags):   # a busy device: requests pile up behind each batch
        time.sleep(0.02)
        return oracle.verify_batch(pool.keys, msg, off, ids, tags)

    mix = ace.Stream.create_host(slow, 4 << 20, 4 << 20, 1)
    ts = [submit(mix, pool, lo, hi) for lo, hi in reqs]
    b = mix.result(ts[7])
    assert a[1] == b[1] and np.array_equal(a[0], b[0])
    assert mix.stats()["max_batch_requests"] > 1   # the probe really shared batches
    mix.close()


def test_plain_form_is_one_request_per_launch(ace, pool):
    s = ace.Stream.create_host(oracle_verify(pool.keys), 4 << 20, 4 << 20, 4, plain=True)
    ts = [submit(s, pool, lo, hi) for lo, hi in requests(pool, 30, 3)]
    for t in ts:
        s.result(t)
    st = s.stats()
    assert st["batches"] == 30 and st["max_batch_requests"] == 1
    s.close()


def test_admission_respects_a_small_arena(ace, pool):
    # arena fits only a few requests at a time: admission must wait, never overflow
    s = ace.Stream.create_host(oracle_verify(pool.keys), arena_bytes=1 << 20,
                               staging_bytes=16 << 20, max_inflight=8)
    reqs = requests(pool, 80, 4)
    ts = [submit(s, pool, lo, hi) for lo, hi in reqs]
    for (lo, hi), t in zip(reqs, ts):
        mask, count = s.result(t)
        em, ec = expect(pool, lo, hi)
        assert count == ec and np.array_equal(mask, em)
    st = s.stats()
    assert st["arena_peak_bytes"] <= st["arena_capacity_bytes"] == 1 << 20
    s.close()


def test_too_large_and_nonblocking(ace, pool):
    s = ace.Stream.create_host(oracle_verify(pool.keys), arena_bytes=64 << 10,
                               staging_bytes=64 << 10, max_inflight=2)
    with pytest.raises(ace.AceError) as e:
        submit(s, pool, 0, 5000)
    assert e.value.code == ace.ACE_ERR_TOO_LARGE
    s.close()
    # staging that holds one request: a second non-blocking submit must say AGAIN
    # unless the first one already finished
    gate = threading.Event()

    def slow_verify(msg, off, ids, tags):
        gate.wait(5)
        return oracle.verify_batch(pool.keys, msg, off, ids, tags)

    s = ace.Stream.create_host(slow_verify, arena_bytes=1 << 20, staging_bytes=8 << 10,
                               max_inflight=1)
    t1 = submit(s, pool, 0, 20)
    with pytest.raises(ace.AceError) as e:
        submit(s, pool, 20, 40, nonblock=True)
    assert e.value.code == ace.ACE_ERR_AGAIN
    gate.set()
    assert s.result(t1)[1] == int(pool.truth[0:20].sum())
    s.close()


def test_injected_device_failure_fails_only_its_batch(ace, pool):
    s = ace.Stream.create_host(oracle_verify(pool.keys), 4 << 20, 4 << 20, 1, plain=True,
                               fail_after=3)
    reqs = requests(pool, 6, 5)
    ts = [submit(s, pool, lo, hi) for lo, hi in reqs]
    outcomes = []
    for (lo, hi), t in zip(reqs, ts):
        try:
            mask, count = s.result(t)
            em, ec = expect(pool, lo, hi)
            assert count == ec and np.array_equal(mask, em)
            outcomes.append("ok")
        except ace.AceError as e:
            assert e.code == ace.ACE_ERR_DEVICE
            outcomes.append("failed")
    assert outcomes == ["ok", "ok", "failed", "ok", "ok", "ok"]
    assert s.stats()["failed"] == 1
    s.close()


@pytest.mark.parametrize("plain", [True, False])
def test_failed_launch_call_fails_only_its_batch(ace, pool, plain):
    """The k-th batch's verify call itself fails after its input copies were
    queued: its requests get the device error, the slot is drained before the
    batch's arena and staging ranges are reused, and every other request --
    before and after, also those admitted into the memory it gave back --
    completes with the right result."""
    s = ace.Stream.create_host(oracle_verify(pool.keys), 1 << 20, 4 << 20, 2, plain=plain,
                               fail_after=2, fail_at_launch=True)
    reqs = requests(pool, 40, 8)
    ts = [submit(s, pool, lo, hi) for lo, hi in reqs]
    failed = 0
    for (lo, hi), t in zip(reqs, ts):
        try:
            mask, count = s.result(t)
        except ace.AceError as e:
            assert e.code == ace.ACE_ERR_DEVICE
            failed += 1
            continue
        em, ec = expect(pool, lo, hi)
        assert count == ec and np.array_equal(mask, em)
    st = s.stats()
    assert failed >= 1 and st["failed"] == failed and st["completed"] == len(reqs) - failed
    if plain:
        assert failed == 1
    # the failed batch's memory went back: a request that needs most of the
    # arena is still admitted
    lo, hi = 0, 2000
    mask, count = s.result(submit(s, pool, lo, hi))
    em, ec = expect(pool, lo, hi)
    assert count == ec and np.array_equal(mask, em)
    s.close()


def test_destroy_releases_blocked_submitter(ace, pool):
    """A submitter blocked for staging space while the stream is destroyed
    returns an error instead of touching the freed engine; destroy returns
    only after it has left."""
    gate = threading.Event()

    def slow(msg, off, ids, tags):
        gate.wait(5)
        return oracle.verify_batch(pool.keys, msg, off, ids, tags)

    s = ace.Stream.create_host(slow, arena_bytes=1 << 20, staging_bytes=8 << 10, max_inflight=1)
    t1 = submit(s, pool, 0, 20)
    outcome = []

    def blocked():
        try:
            submit(s, pool, 20, 40)   # waits: staging holds one request
            outcome.append("accepted")
        except ace.AceError as e:
            outcome.append(e.code)

    th = threading.Thread(target=blocked)
    th.start()
    import time
    time.sleep(0.1)
    closer = threading.Thread(target=s.close)
    closer.start()
    time.sleep(0.1)
    gate.set()
    closer.join(10)
    th.join(10)
    assert not closer.is_alive() and not th.is_alive()
    # the blocked submitter either got in before destroy began (then its
    # request was finished by the drain) or was turned away
    assert outcome in (["accepted"], [ace.ACE_ERR_INVALID_ARG])
    assert int(t1.count[0]) == int(pool.truth[0:20].sum())


def test_destroy_drains_queued_requests(ace, pool):
    s = ace.Stream.create_host(oracle_verify(pool.keys), 4 << 20, 4 << 20, 2)
    reqs = requests(pool, 40, 6)
    ts = [submit(s, pool, lo, hi) for lo, hi in reqs]
    s.close()  # returns only after every request finished
    for (lo, hi), t in zip(reqs, ts):
        em, ec = expect(pool, lo, hi)
        assert int(t.count[0]) == ec
        assert np.array_equal(t.mask[: (hi - lo + 31) // 32], em)


def test_empty_request_and_bad_ticket(ace, pool):
    s = ace.Stream.create_host(oracle_verify(pool.keys), 1 << 20, 1 << 20, 1)
    t = submit(s, pool, 5, 5)
    mask, count = s.result(t)
    assert count == 0 and mask.size == 0
    from paper_2603_10242_amd.ace import load
    assert load().ace_stream_poll(s._h, 999_999, 0) == ace.ACE_ERR_INVALID_ARG
    s.close()


def test_native_open_loop_driver(ace, pool):
    """The serving benchmark's native load generator submits every request at
    its arrival time through ace_verify_stream; each result matches the truth."""
    import ctypes
    import time
    st = ace.Stream.create_host(oracle_verify(pool.keys), 64 << 20, 16 << 20, max_inflight=4)
    try:
        r = np.random.Generator(np.random.PCG64(17))
        sizes = r.integers(1, 1500, size=120).astype(np.uint64)
        starts = r.integers(0, pool.n - 1500, size=120).astype(np.uint64)
        arrivals = time.monotonic() + 0.02 + np.cumsum(r.exponential(2e-4, size=120))
        fn = ctypes.cast(ace.load().ace_verify_stream, ctypes.c_void_p).value
        tickets, submit, masks, mask_words, counts = W.client_drive(
            fn, st._h.value, pool, starts, sizes, arrivals, threads=3)
        assert (submit >= arrivals - 1e-4).all()          # nobody submits before arrival
        for k in range(120):
            t = ace.Ticket(int(tickets[k]), int(sizes[k]), None, None)
            st.poll(t, True)
            lo, n = int(starts[k]), int(sizes[k])
            w0 = int(mask_words[k])
            assert int(counts[k]) == int(pool.truth[lo:lo + n].sum())
            assert np.array_equal(masks[w0:w0 + (n + 31) // 32], W.pack_bits(pool.truth[lo:lo + n]))
            st.release(t)
    finally:
        st.close()
