"""Parity of the HIP path (through the C ABI) with the CPU oracle and with the
generator's truth mask.  Integer work: every bitmask word and count must be
identical (tolerance 0).  Every test runs under the library's default launch
tuning and under the saved autotuned one."""
import sys

import numpy as np
import pytest

import oracle
from paper_2603_10242_amd import workload as W

from .conftest import TUNINGS, use_tuning

pytestmark = pytest.mark.gpu

MODES = {
    "ordered": 0x1,
    "binned": 0x2,
    "binned-persistent": 0x2 | 0x4,
}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=TUNINGS)
def ace(need_gpu, request):
    import torch
    from paper_2603_10242_amd import ace as A
    A.load()
    torch.cuda.set_device(0)
    note("launch tuning %s: %s" % (request.param, use_tuning(A, request.param)))
    yield A
    A.set_tuning(**A.default_tuning())


@pytest.fixture(scope="module")
def block_scale():
    """The block-scale workload with the oracle's keys and whole-batch result."""
    w = W.config2()
    keys = oracle.derive_keys(w.rev, w.salt, w.info, 8)
    return w, keys, oracle.verify_batch(keys, w.msg, w.off, w.ids, w.tags, 8)


def oracle_result(w, keys=None, nthreads=8, ids=None, off=None):
    keys = oracle.derive_keys(w.rev, w.salt, w.info, nthreads) if keys is None else keys
    return oracle.verify_batch(keys, w.msg, w.off if off is None else off,
                               w.ids if ids is None else ids, w.tags, nthreads)


def run(ace, w, keyset, flags, ids=None, off=None):
    import torch
    blk = ace.upload_block(w.msg, w.off if off is None else off, w.ids if ids is None else ids,
                           w.tags)
    ace.verify_batch(keyset, [blk], flags=flags)
    torch.cuda.synchronize()
    return blk.result()


def keysets(ace, w):
    rev = ace.to_device(w.rev)
    return {
        "midstate": ace.midstate_keyset(rev, w.salt, w.info),
        "rev": ace.rev_keyset(rev, w.salt, w.info),
    }


# ------------------------------------------------------------------ key derivation
@pytest.mark.parametrize("salt_len", [0, 1, 32, 64, 65, 200, 1024])
def test_derive_keys_salts(ace, salt_len):
    import torch
    note("derive_keys salt_len=%d" % salt_len)
    r = np.random.Generator(np.random.PCG64(salt_len + 7))
    n_id = 1000
    rev = r.integers(0, 256, size=(n_id, 32), dtype=np.uint8)
    salt = r.integers(0, 256, size=salt_len, dtype=np.uint8).tobytes()
    info = W.INFO_16
    d_rev = ace.to_device(rev)
    key = torch.zeros((n_id, 32), dtype=torch.uint8, device="cuda")
    mid = torch.zeros((n_id, 16), dtype=torch.int32, device="cuda")
    ace.derive_keys(d_rev, salt, info, key_out=key, mid_out=mid)
    torch.cuda.synchronize()
    okeys = oracle.derive_keys(rev, salt, info, 8)
    assert np.array_equal(key.cpu().numpy(), okeys)
    assert np.array_equal(mid.cpu().numpy().view(np.uint32), oracle.hmac_midstates(okeys))


@pytest.mark.parametrize("info", [b"", W.INFO_16, W.INFO_ATTEST, b"x" * 54, b"y" * 55,
                                  b"z" * 100, bytes(range(255))])
def test_derive_keys_infos(ace, info):
    import torch
    note("derive_keys info_len=%d" % len(info))
    r = np.random.Generator(np.random.PCG64(len(info) + 100))
    n_id = 333
    rev = r.integers(0, 256, size=(n_id, 32), dtype=np.uint8)
    salt = r.integers(0, 256, size=32, dtype=np.uint8).tobytes()
    key = torch.zeros((n_id, 32), dtype=torch.uint8, device="cuda")
    ace.derive_keys(ace.to_device(rev), salt, info, key_out=key)
    torch.cuda.synchronize()
    assert np.array_equal(key.cpu().numpy(), oracle.derive_keys(rev, salt, info, 8))


@pytest.mark.parametrize("n_id", [262143, 262145, 600001])
def test_derive_keys_strided_passes(ace, n_id):
    """More identities than the derivation's capped grid has lanes (four
    256-lane workgroups per CU, 262,144 lanes on 256 CUs): lanes take one,
    two or three identities, the last pass ragged.  Every key and midstate
    against the oracle."""
    import torch
    note("derive_keys strided n_id=%d" % n_id)
    r = np.random.Generator(np.random.PCG64(n_id))
    rev = r.integers(0, 256, size=(n_id, 32), dtype=np.uint8)
    salt = r.integers(0, 256, size=32, dtype=np.uint8).tobytes()
    key = torch.zeros((n_id, 32), dtype=torch.uint8, device="cuda")
    mid = torch.zeros((n_id, 16), dtype=torch.int32, device="cuda")
    ace.derive_keys(ace.to_device(rev), salt, W.INFO_ATTEST, key_out=key, mid_out=mid)
    torch.cuda.synchronize()
    okeys = oracle.derive_keys(rev, salt, W.INFO_ATTEST, 8)
    assert np.array_equal(key.cpu().numpy(), okeys)
    assert np.array_equal(mid.cpu().numpy().view(np.uint32), oracle.hmac_midstates(okeys))


def test_derive_keys_match_openssl_client_keys(ace):
    import torch
    w = W.config1()
    key = torch.zeros((w.n_id, 32), dtype=torch.uint8, device="cuda")
    ace.derive_keys(ace.to_device(w.rev), w.salt, w.info, key_out=key)
    torch.cuda.synchronize()
    assert np.array_equal(key.cpu().numpy(), w.keys)


def _info_strings():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "info_strings.tsv")
    return [l.split("\t")[1].encode() for l in open(path).read().splitlines()
            if l and not l.startswith("#")]


@pytest.mark.parametrize("n_id", [1, 300, 4097])
def test_derive_keys_multi(ace, n_id):
    """Keys and midstates of the paper's purpose streams, the validator streams
    and eleven slot domains (19 streams: two launches of up to 16)."""
    import torch
    note("derive multi n_id=%d" % n_id)
    r = np.random.Generator(np.random.PCG64(4242 + n_id))
    rev = r.integers(0, 256, size=(n_id, 32), dtype=np.uint8)
    streams = [(r.integers(0, 256, size=32, dtype=np.uint8).tobytes(), i) for i in _info_strings()]
    streams += [(r.integers(0, 256, size=8, dtype=np.uint8).tobytes(), W.INFO_ATTEST)
                for _ in range(8)]
    streams += [(b"", b""), (b"\x07" * 64, b"q" * 64), (b"s", b"i" * 54)]
    S = len(streams)
    key = torch.zeros((S, n_id, 32), dtype=torch.uint8, device="cuda")
    mid = torch.zeros((S, n_id, 16), dtype=torch.int32, device="cuda")
    ace.derive_keys_multi(ace.to_device(rev), streams, key_out=key, mid_out=mid)
    torch.cuda.synchronize()
    want = oracle.derive_keys_multi(rev, streams, nthreads=8)
    assert np.array_equal(key.cpu().numpy(), want)
    got_mid = mid.cpu().numpy().view(np.uint32)
    for s in (0, 7, 9, S - 1):
        assert np.array_equal(got_mid[s], oracle.hmac_midstates(want[s]))


def test_keys_in_call_from_short_lived_threads(ace):
    """Keys derived in the call (the derivation on a second stream per thread)
    from three rounds of eight threads that each verify one block and end:
    later threads reuse the second-stream contexts of ended ones."""
    import threading
    import torch
    note("keys in call from 24 short-lived threads")
    w = W.config2()
    rev = ace.to_device(w.rev)
    ks = ace.rev_keyset(rev, w.salt, w.info)
    step = w.n // 8
    parts = [W.subset(w, i * step, (i + 1) * step) for i in range(8)]
    errors = []

    def one(part):
        try:
            torch.cuda.set_device(0)
            blk = ace.upload_block(part.msg, part.off, part.ids, part.tags)
            ace.verify_batch(ks, [blk], flags=MODES["binned"])
            torch.cuda.synchronize()
            mask, count = blk.result()
            if count != int(part.truth.sum()) or not np.array_equal(mask, part.truth_bitmask()):
                errors.append(part.name)
        except Exception as e:  # reported below, in the test's thread
            errors.append("%s: %r" % (part.name, e))

    for _ in range(3):
        threads = [threading.Thread(target=one, args=(p,)) for p in parts]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
    assert not errors, errors


def test_binding_refuses_undersized_device_buffers(ace):
    """Outputs smaller than the call would write are refused before any launch."""
    import torch
    rev = torch.zeros((100, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError, match="mid_out"):
        ace.derive_keys(rev, b"s", b"i", mid_out=torch.zeros((99, 16), dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError, match="key_out"):
        ace.derive_keys_multi(rev, [(b"s", b"i"), (b"t", b"j")],
                              key_out=torch.zeros((1, 100, 32), dtype=torch.uint8, device="cuda"))
    w = W.config1()
    blk = ace.upload_block(w.msg, w.off, w.ids, w.tags)
    blk.bitmask = blk.bitmask[:-1].contiguous()
    with pytest.raises(ValueError, match="bitmask"):
        ace.verify_batch(ace.rev_keyset(ace.to_device(w.rev), w.salt, w.info), [blk])
    s = torch.zeros((64, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError, match="end"):
        ace.poh_verify(s, s[:63].contiguous(), 3, torch.zeros(2, dtype=torch.int32, device="cuda"),
                       torch.zeros(1, dtype=torch.int64, device="cuda"))


# ------------------------------------------------------------------ the tiny and block workloads
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("keys", ["midstate", "rev", "rev-per-tx"])
def test_tiny(ace, mode, keys):
    note("tiny mode=%s keys=%s" % (mode, keys))
    w = W.config1()
    ks = keysets(ace, w)["rev" if keys.startswith("rev") else "midstate"]
    flags = MODES[mode] | (0x8 if keys == "rev-per-tx" else 0)
    mask, count = run(ace, w, ks, flags)
    omask, ocount = oracle_result(w, keys=w.keys)
    assert count == ocount == 4096 - 205
    assert np.array_equal(mask, omask)
    assert np.array_equal(mask, w.truth_bitmask())


@pytest.mark.parametrize("mode", list(MODES))
def test_block_scale_keys_in_launch(ace, mode):
    note("block scale mode=%s" % mode)
    w = W.config2()
    mask, count = run(ace, w, keysets(ace, w)["rev"], MODES[mode])
    omask, ocount = oracle_result(w)
    assert count == ocount == 99_000
    assert np.array_equal(mask, omask)
    assert np.array_equal(mask, w.truth_bitmask())


def test_block_scale_per_tx_keys(ace):
    w = W.config2()
    mask, count = run(ace, w, keysets(ace, w)["rev"], MODES["binned"] | 0x8)
    assert count == 99_000 and np.array_equal(mask, w.truth_bitmask())


# ------------------------------------------------------------------ every padding case
@pytest.mark.parametrize("mode", list(MODES))
def test_every_length_0_to_1300_misaligned(ace, mode):
    """Every message length 0..1300 (each padding case), groups of 100 messages
    behind a random 0-3 byte lead so messages start at every alignment."""
    import torch
    note("lengths 0..1300 mode=%s" % mode)
    L = np.arange(0, 1301, dtype=np.int64)
    r = np.random.Generator(np.random.PCG64(1301))
    n_id = 64
    rev = r.integers(0, 256, size=(n_id, 32), dtype=np.uint8)
    salt = r.integers(0, 256, size=32, dtype=np.uint8).tobytes()
    keys = W.client_keys(rev, salt, W.INFO_16)
    ids = r.integers(0, n_id, size=L.size).astype(np.uint32)
    blocks, cases = [], []
    for lo in range(0, L.size, 100):
        hi = min(L.size, lo + 100)
        lead = int(r.integers(0, 4))
        off = np.zeros(hi - lo + 1, np.uint64)
        np.cumsum(L[lo:hi], out=off[1:])
        off += lead
        buf = r.integers(0, 256, size=int(off[-1]) + 1, dtype=np.uint8)[: int(off[-1])]
        tags = W.client_sign(keys, buf, off, ids[lo:hi])
        truth = np.ones(hi - lo, bool)
        flip = r.random(hi - lo) < 0.1
        tags[flip, 0] ^= 1
        truth[flip] = False
        blocks.append(ace.upload_block(buf, off, ids[lo:hi], tags))
        cases.append((truth, buf, off, ids[lo:hi], tags))
    ks = ace.midstate_keyset(ace.to_device(rev), salt, W.INFO_16)
    ace.verify_batch(ks, blocks, flags=MODES[mode])
    torch.cuda.synchronize()
    for blk, (truth, buf, off, ids_b, tags) in zip(blocks, cases):
        mask, count = blk.result()
        omask, ocount = oracle.verify_batch(keys, buf, off, ids_b, tags)
        assert count == ocount == int(truth.sum())
        assert np.array_equal(mask, omask)
        assert np.array_equal(mask, W.pack_bits(truth))


def test_long_messages_catch_all_bin(ace):
    import torch
    note("long messages")
    lengths = [4000, 4023, 4024, 4096, 5000, 9000, 20000, 63, 64, 1232] * 7
    w = W.generate("long", 99, n=len(lengths), n_id=16, lengths=np.array(lengths),
                   n_invalid=7, kinds=(W.KIND_TAG, W.KIND_MSG, W.KIND_KEY))
    for mode in MODES.values():
        mask, count = run(ace, w, keysets(ace, w)["midstate"], mode)
        assert count == w.n - 7 and np.array_equal(mask, w.truth_bitmask())


# ------------------------------------------------------------------ batch shapes, edge cases
@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 63, 64, 65, 4097])
def test_batch_sizes(ace, block_scale, n):
    note("batch size n=%d" % n)
    base, keys, _ = block_scale
    w = W.subset(base, 0, n)
    omask, ocount = oracle_result(w, keys=keys)
    ks = keysets(ace, w)
    for mode in [0] + list(MODES.values()):
        for name in ("midstate", "rev"):
            mask, count = run(ace, w, ks[name], mode)
            assert count == ocount == int(w.truth.sum())
            assert mask.shape[0] == (n + 31) // 32
            assert np.array_equal(mask, omask)
            assert np.array_equal(mask, w.truth_bitmask())


def test_unregistered_ids_and_bad_offsets(ace):
    note("unregistered ids, decreasing offsets")
    w = W.subset(W.config2(), 0, 5000)
    ids = w.ids.copy()
    off = w.off.copy()
    ids[[3, 100, 4999]] = [w.n_id, 0xFFFFFFFF, w.n_id + 5]
    off[200], off[201] = off[201], off[200]
    omask, ocount = oracle_result(w, ids=ids, off=off)
    for mode in MODES.values():
        for name, ks in keysets(ace, w).items():
            mask, count = run(ace, w, ks, mode, ids=ids, off=off)
            assert count == ocount and np.array_equal(mask, omask), (mode, name)


def test_every_single_bit_flip_is_rejected(ace):
    """Tamper invariants on the GPU: for three messages (55, 64 and 200 bytes,
    one padding case each), every single-bit flip of the message, of the
    credential and of the identity's root entropy is a transaction of one
    batch; only the three untouched transactions may pass, in every launch
    mode, with midstates and with keys derived in the call."""
    note("every single-bit flip")
    r = np.random.Generator(np.random.PCG64(2024))
    msgs = [r.integers(0, 256, size=L, dtype=np.uint8) for L in (55, 64, 200)]
    base_rev = r.integers(0, 256, size=(3, 32), dtype=np.uint8)
    rev = [base_rev]
    for j in range(3):                               # identity 3 + 256 j + b: REV_j, bit b flipped
        fl = np.repeat(base_rev[j:j + 1], 256, axis=0)
        fl[np.arange(256), np.arange(256) // 8] ^= (1 << (np.arange(256) % 8)).astype(np.uint8)
        rev.append(fl)
    rev = np.concatenate(rev)
    salt = r.integers(0, 256, size=32, dtype=np.uint8).tobytes()
    keys = W.client_keys(rev, salt, W.INFO_16)
    one_off = np.array([0, 0], np.uint64)
    tags = [W.client_sign(keys, m, one_off + np.array([0, m.size], np.uint64), np.array([j], np.uint32))[0]
            for j, m in enumerate(msgs)]
    parts, ids, tag_rows = [], [], []
    for j, m in enumerate(msgs):
        parts.append(m); ids.append(j); tag_rows.append(tags[j])                  # untouched
        for b in range(8 * m.size):                                                 # message flips
            f = m.copy(); f[b // 8] ^= 1 << (b % 8)
            parts.append(f); ids.append(j); tag_rows.append(tags[j])
        for b in range(256):                                                        # credential flips
            t = tags[j].copy(); t[b // 8] ^= 1 << (b % 8)
            parts.append(m); ids.append(j); tag_rows.append(t)
        for b in range(256):                                                        # root-entropy flips
            parts.append(m); ids.append(3 + 256 * j + b); tag_rows.append(tags[j])
    lead = 1                                                                        # misaligned start
    buf = np.concatenate([np.zeros(lead, np.uint8)] + parts)
    off = np.zeros(len(parts) + 1, np.uint64)
    off[1:] = np.cumsum([p.size for p in parts])
    off += lead
    ids = np.array(ids, np.uint32)
    tag_rows = np.stack(tag_rows)
    truth = np.zeros(len(parts), bool)
    firsts = np.cumsum([0] + [1 + 8 * m.size + 512 for m in msgs])[:3]
    truth[firsts] = True
    omask, ocount = oracle.verify_batch(oracle.derive_keys(rev, salt, W.INFO_16, 8), buf, off, ids,
                                        tag_rows, 8)
    assert ocount == 3 and np.array_equal(omask, W.pack_bits(truth))
    import torch
    devrev = ace.to_device(rev)
    for mode in MODES.values():
        for ks in (ace.midstate_keyset(devrev, salt, W.INFO_16), ace.rev_keyset(devrev, salt, W.INFO_16)):
            blk = ace.upload_block(buf, off, ids, tag_rows)
            ace.verify_batch(ks, [blk], flags=mode)
            torch.cuda.synchronize()
            mask, count = blk.result()
            assert count == 3 and np.array_equal(mask, omask), mode


@pytest.mark.parametrize("wide_min", [1, 150, 700])
def test_wide_records_read_offsets(ace, wide_min):
    """Binned calls verify a message of at least wide_min_len bytes from its
    block's offsets instead of its bin-order record (by default only messages
    of 2 GiB or more, whose length the record cannot hold).  Lowered, the
    tuning moves ordinary messages (96-512 bytes here) onto that path, which
    must change no result: unregistered identities and decreasing offsets
    included, both binned launch forms, midstates and keys derived in the
    call.  700 is the control with no wide message."""
    note("wide records, wide_min_len=%d" % wide_min)
    w = W.subset(W.config2(), 0, 5000)
    ids = w.ids.copy()
    off = w.off.copy()
    ids[[3, 100, 4999]] = [w.n_id, 0xFFFFFFFF, w.n_id + 5]
    off[200], off[201] = off[201], off[200]
    omask, ocount = oracle_result(w, ids=ids, off=off)
    old = ace.get_tuning()
    try:
        ace.set_tuning(wide_min_len=wide_min)
        for mode in ("binned", "binned-persistent"):
            for name, ks in keysets(ace, w).items():
                mask, count = run(ace, w, ks, MODES[mode], ids=ids, off=off)
                assert count == ocount and np.array_equal(mask, omask), (mode, name)
    finally:
        ace.set_tuning(**old)


def test_all_valid_and_all_invalid(ace):
    w = W.generate("clean", 5, n=3000, n_id=100, lengths=lambda r, n: r.integers(0, 700, size=n))
    for mode in MODES.values():
        mask, count = run(ace, w, keysets(ace, w)["midstate"], mode)
        assert count == 3000 and np.array_equal(mask, w.truth_bitmask())
    bad = W.generate("dirty", 6, n=3000, n_id=100, lengths=lambda r, n: r.integers(0, 700, size=n),
                     n_invalid=3000, kinds=(W.KIND_TAG, W.KIND_MSG, W.KIND_KEY))
    for mode in MODES.values():
        mask, count = run(ace, bad, keysets(ace, bad)["rev"], mode)
        assert count == 0 and not mask.any()


def test_empty_registry(ace):
    import torch
    w = W.subset(W.config1(), 0, 100)
    empty = ace.DeviceKeyset(ace.ACE_KEYS_MIDSTATE, 0,
                             mid=torch.zeros((1, 16), dtype=torch.int32, device="cuda"))
    for mode in MODES.values():
        mask, count = run(ace, w, empty, mode)
        assert count == 0 and not mask.any()


# ------------------------------------------------------------------ several blocks in one call
@pytest.mark.parametrize("mode", list(MODES))
def test_multi_block(ace, block_scale, mode):
    import torch
    note("multi-block mode=%s" % mode)
    w, keys, _ = block_scale
    sizes = [0, 1, 100, 3000, 64, 65, 5000, 0, 2048, 31, 20000, 7]
    ks = keysets(ace, w)["rev"]
    d_msg = ace.to_device(w.msg)
    blocks, parts = [], []
    lo = 0
    for s in sizes:
        hi = lo + s
        # every block addresses the shared message buffer with absolute offsets
        blocks.append(ace.upload_block(None, w.off[lo:hi + 1], w.ids[lo:hi], w.tags[lo:hi],
                                       msg_dev=d_msg))
        parts.append((lo, hi))
        lo = hi
    ace.verify_batch(ks, blocks, flags=MODES[mode])
    torch.cuda.synchronize()
    for blk, (lo, hi) in zip(blocks, parts):
        mask, count = blk.result()
        truth = w.truth[lo:hi]
        omask, ocount = oracle.verify_batch(keys, w.msg, w.off[lo:hi + 1], w.ids[lo:hi],
                                            w.tags[lo:hi], 8)
        assert count == ocount == int(truth.sum()), (lo, hi)
        assert np.array_equal(mask, omask), (lo, hi)
        assert np.array_equal(mask, W.pack_bits(truth)), (lo, hi)


def test_many_blocks_256(ace, block_scale):
    import torch
    note("256 blocks")
    base, keys, _ = block_scale
    w = W.subset(base, 0, 60_000)
    r = np.random.Generator(np.random.PCG64(256))
    cuts = np.sort(r.choice(np.arange(1, w.n), size=255, replace=False))
    edges = np.concatenate([[0], cuts, [w.n]])
    d_msg = ace.to_device(w.msg)
    blocks = [ace.upload_block(None, w.off[a:b + 1], w.ids[a:b], w.tags[a:b], msg_dev=d_msg)
              for a, b in zip(edges[:-1], edges[1:])]
    want = [oracle.verify_batch(keys, w.msg, w.off[a:b + 1], w.ids[a:b], w.tags[a:b], 8)
            for a, b in zip(edges[:-1], edges[1:])]
    for mode in [0] + list(MODES.values()):
        ace.verify_batch(keysets(ace, w)["midstate"], blocks, flags=mode)
        torch.cuda.synchronize()
        for blk, a, b, (omask, ocount) in zip(blocks, edges[:-1], edges[1:], want):
            mask, count = blk.result()
            assert count == ocount == int(w.truth[a:b].sum())
            assert np.array_equal(mask, omask)
            assert np.array_equal(mask, W.pack_bits(w.truth[a:b]))


def test_valu_probe_rate_is_plausible(ace):
    """The probe's measured INT32 VALU rate lies near the 39.32 T peak the
    roofline uses (256 CUs x 64 lanes x 2.4 GHz)."""
    note("valu probe")
    rate = ace.valu_rate(iters=2000, wgs_per_cu=8) / 1e12
    note("measured %.2f T lane-instr/s" % rate)
    assert 0.3 * 39.3216 < rate < 1.1 * 39.3216
