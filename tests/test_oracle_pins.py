"""Pins of the CPU oracle against things other than itself.

* SHA-256 / HMAC: Python's hashlib and hmac (OpenSSL) on seeded inputs,
  every length that exercises a different padding case.
* HKDF: the ``openssl kdf`` command line (RFC 5869 as OpenSSL implements it).
* Constants: FIPS 180-4 sec. 4.2.2 / 5.3.3 closed forms, with exact integer
  roots computed here in Python.
* Midstates: HMAC through two single-block computations equals hashlib's HMAC.
* Tamper invariants (Thm. attestation unforgeability): every single-bit flip
  of root entropy, key, message or credential is rejected.
* Context isolation (Def. 2.2): distinct salt or info gives distinct keys.
* The generator's truth mask (its corruption plan) on the tiny and block-scale
  workloads.
"""
import hashlib
import hmac
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2603_10242_amd import workload as W


def _rng(tag):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([0xACE0, tag])))


def _bytes(r, n):
    return r.integers(0, 256, size=n, dtype=np.uint8).tobytes()


# ---------------------------------------------------------------- constants
def _primes(k):
    out, p = [], 2
    while len(out) < k:
        if all(p % q for q in out if q * q <= p):
            out.append(p)
        p += 1
    return out


def _icbrt(x):
    lo, hi = 0, 1 << ((x.bit_length() + 2) // 3 + 1)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if mid ** 3 <= x:
            lo = mid
        else:
            hi = mid
    return lo


def closed_form_constants():
    import math
    ps = _primes(64)
    K = [(_icbrt(p << 96)) & 0xFFFFFFFF for p in ps]
    IV = [math.isqrt(p << 64) & 0xFFFFFFFF for p in ps[:8]]
    return np.array(K, np.uint32), np.array(IV, np.uint32)


def test_constants_closed_form():
    K, IV = oracle.constants()
    Kc, IVc = closed_form_constants()
    assert (K == Kc).all()
    assert (IV == IVc).all()
    # spot values that follow from the definition by hand: frac(sqrt 2) * 2^32
    assert IV[0] == int((2 ** 0.5 - 1) * 2 ** 32)


# ---------------------------------------------------------------- SHA-256
def test_sha256_every_length_to_4096():
    r = _rng(1)
    data = _bytes(r, 4096)
    for n in range(0, 4097):
        assert oracle.sha256(data[:n]) == hashlib.sha256(data[:n]).digest(), n


def test_sha256_large_random():
    r = _rng(2)
    for n in (65_537, 300_001, 1 << 20):
        d = _bytes(r, n)
        assert oracle.sha256(d) == hashlib.sha256(d).digest()


def test_compress_is_one_block_of_sha256():
    # F(H0, padded block) is SHA-256 of every message short enough for one block
    r = _rng(3)
    for n in range(0, 56):
        m = _bytes(r, n)
        blk = m + b"\x80" + b"\0" * (55 - n) + (8 * n).to_bytes(8, "big")
        st = oracle.sha256_compress(oracle.sha256_iv(), blk)
        assert st.astype(">u4").tobytes() == hashlib.sha256(m).digest()


# ---------------------------------------------------------------- HMAC
def test_hmac_key_lengths_0_to_200():
    r = _rng(4)
    msgs = [_bytes(r, n) for n in (0, 1, 40, 55, 56, 63, 64, 119, 120, 200, 1000, 2100)]
    for klen in range(0, 201):
        key = _bytes(r, klen)
        for m in msgs:
            assert oracle.hmac_sha256(key, m) == hmac.digest(key, m, "sha256"), (klen, len(m))


def test_hmac_every_message_length_to_1300():
    r = _rng(5)
    key = _bytes(r, 32)
    data = _bytes(r, 1300)
    for n in range(0, 1301):
        assert oracle.hmac_sha256(key, data[:n]) == hmac.digest(key, data[:n], "sha256"), n


def test_hmac_through_midstates_equals_hmac():
    # inner = F(ipad state, padded m) with bit length (64 + |m|) * 8,
    # outer = F(opad state, padded inner) with bit length (64 + 32) * 8.
    r = _rng(6)
    keys = r.integers(0, 256, size=(16, 32), dtype=np.uint8)
    mids = oracle.hmac_midstates(keys)
    for j in range(16):
        m = _bytes(r, 40)
        blk = m + b"\x80" + b"\0" * 15 + ((64 + 40) * 8).to_bytes(8, "big")
        inner = oracle.sha256_compress(mids[j, :8], blk).astype(">u4").tobytes()
        blk2 = inner + b"\x80" + b"\0" * 23 + ((64 + 32) * 8).to_bytes(8, "big")
        outer = oracle.sha256_compress(mids[j, 8:], blk2).astype(">u4").tobytes()
        assert outer == hmac.digest(keys[j].tobytes(), m, "sha256")


# ---------------------------------------------------------------- HKDF
def _openssl_hkdf(salt, ikm, info, length):
    cmd = ["openssl", "kdf", "-keylen", str(length), "-kdfopt", "digest:SHA256",
           "-kdfopt", "hexkey:" + ikm.hex()]
    if salt:
        cmd += ["-kdfopt", "hexsalt:" + salt.hex()]
    if info:
        cmd += ["-kdfopt", "hexinfo:" + info.hex()]
    out = subprocess.check_output(cmd + ["HKDF"], text=True).strip()
    return bytes.fromhex(out.replace(":", ""))


@pytest.mark.skipif(shutil.which("openssl") is None, reason="openssl CLI absent")
def test_hkdf_against_openssl_cli():
    r = _rng(7)
    cases = []
    for slen in (0, 1, 16, 32, 63, 64, 65, 80):
        for ilen in (0, 1, 16, 23, 54, 55, 80):
            cases.append((slen, ilen, 32))
    cases += [(32, 16, L) for L in (1, 31, 33, 64, 100, 255, 1000, 255 * 32)]
    for slen, ilen, L in cases:
        salt, ikm, info = _bytes(r, slen), _bytes(r, 32), _bytes(r, ilen)
        assert oracle.hkdf_sha256(salt, ikm, info, L) == _openssl_hkdf(salt, ikm, info, L), \
            (slen, ilen, L)


def test_hkdf_rejects_too_long_output():
    with pytest.raises(ValueError):
        oracle.hkdf_sha256(b"s", b"k", b"i", 255 * 32 + 1)


def test_hkdf_paper_info_strings_against_openssl():
    # the purpose strings named by Def. 2.1 and equation attestkey
    info_lines = [l.split("\t")[1].encode() for l in
                  open(__file__.replace("test_oracle_pins.py", "golden/info_strings.tsv"))
                  .read().splitlines() if l and not l.startswith("#")]
    r = _rng(8)
    rev, salt = _bytes(r, 32), _bytes(r, 32)
    keys = set()
    for info in info_lines:
        k = oracle.hkdf_sha256(salt, rev, info, 32)
        if shutil.which("openssl"):
            assert k == _openssl_hkdf(salt, rev, info, 32)
        keys.add(k)
    assert len(keys) == len(info_lines)


def test_context_isolation_distinct_keys():
    r = _rng(9)
    rev = r.integers(0, 256, size=(64, 32), dtype=np.uint8)
    a = oracle.derive_keys(rev, b"\x01" * 32, W.INFO_16)
    b = oracle.derive_keys(rev, b"\x02" * 32, W.INFO_16)
    c = oracle.derive_keys(rev, b"\x01" * 32, W.INFO_ATTEST)
    all_keys = {bytes(k) for k in np.concatenate([a, b, c])}
    assert len(all_keys) == 3 * 64


# ---------------------------------------------------------------- batch verdicts
def test_verify_matches_truth_tiny():
    w = W.config1()
    keys = oracle.derive_keys(w.rev, w.salt, w.info)
    assert (keys == w.keys).all()          # oracle HKDF == OpenSSL HKDF, per identity
    mask, count = oracle.verify_batch(keys, w.msg, w.off, w.ids, w.tags)
    assert count == 4096 - 205 == int(w.truth.sum())
    assert (mask == w.truth_bitmask()).all()


def test_verify_matches_truth_block_scale():
    w = W.config2()
    mask, count = oracle.verify_batch_rev(w.rev, w.salt, w.info, w.msg, w.off, w.ids, w.tags,
                                          nthreads=8)
    assert count == 100_000 - 1000
    assert (mask == w.truth_bitmask()).all()
    m1, c1 = oracle.verify_batch(w.keys, w.msg, w.off, w.ids, w.tags, nthreads=1)
    assert c1 == count and (m1 == mask).all()


def test_verify_special_cases():
    w = W.subset(W.config1(), 0, 100)
    ids = w.ids.copy()
    off = w.off.copy()
    ids[3] = w.n_id                 # identity outside the registry
    ids[4] = 0xFFFFFFFF
    off[10], off[11] = off[11], off[10]  # tx 9 and 10 get decreasing offsets
    mask, count = oracle.verify_batch(w.keys, w.msg, off, ids, w.tags)
    truth = w.truth.copy()
    truth[[3, 4]] = False
    bits = np.unpackbits(mask.view(np.uint8), bitorder="little")[:100].astype(bool)
    assert not bits[3] and not bits[4] and not bits[10]
    for i in range(100):
        if i in (3, 4, 9, 10, 11):
            continue
        assert bits[i] == truth[i]
    # empty batch
    m0, c0 = oracle.verify_batch(w.keys, w.msg[:0], np.zeros(1, np.uint64),
                                 np.zeros(0, np.uint32), np.zeros((0, 32), np.uint8))
    assert c0 == 0 and m0.size == 0


def test_empty_message_is_verifiable():
    key = bytes(range(32))
    tag = np.frombuffer(hmac.digest(key, b"", "sha256"), np.uint8).reshape(1, 32)
    mask, count = oracle.verify_batch(np.frombuffer(key, np.uint8).reshape(1, 32),
                                      np.zeros(0, np.uint8), np.zeros(2, np.uint64),
                                      np.zeros(1, np.uint32), tag)
    assert count == 1 and mask[0] == 1


def test_permuting_transactions_permutes_bits():
    w = W.subset(W.config2(), 0, 3000)
    r = _rng(10)
    p = r.permutation(w.n)
    L = w.lengths()[p]
    off = np.zeros(w.n + 1, np.uint64)
    np.cumsum(L, out=off[1:])
    msg = np.concatenate([w.msg[int(w.off[i]):int(w.off[i + 1])] for i in p])
    m0, c0 = oracle.verify_batch(w.keys, w.msg, w.off, w.ids, w.tags)
    m1, c1 = oracle.verify_batch(w.keys, msg, off, w.ids[p], w.tags[p])
    b0 = np.unpackbits(m0.view(np.uint8), bitorder="little")[: w.n]
    b1 = np.unpackbits(m1.view(np.uint8), bitorder="little")[: w.n]
    assert c0 == c1 and (b1 == b0[p]).all()


# ---------------------------------------------------------------- tamper invariants
def _paper_form_txs(count, seed):
    """Messages of the paper's form m = obj_hash || domain (32 + 8 = 40 bytes)."""
    r = _rng(seed)
    rev = r.integers(0, 256, size=(count, 32), dtype=np.uint8)
    salt = _bytes(r, 8)   # the domain c || s as an opaque 8-byte context
    keys = W.client_keys(rev, salt, W.INFO_ATTEST)
    msgs = [hashlib.sha256(_bytes(r, 200)).digest() + salt for _ in range(count)]
    return rev, salt, keys, msgs


def test_every_single_bit_flip_is_rejected():
    rev, salt, keys, msgs = _paper_form_txs(64, 11)
    ok_total = 0
    for j in range(64):
        key = keys[j].tobytes()
        m = msgs[j]
        tag = hmac.digest(key, m, "sha256")
        variants_m, variants_t = [m], [tag]
        for b in range(8 * len(m)):          # message flips
            mm = bytearray(m); mm[b // 8] ^= 1 << (b % 8)
            variants_m.append(bytes(mm)); variants_t.append(tag)
        for b in range(256):                 # credential flips
            tt = bytearray(tag); tt[b // 8] ^= 1 << (b % 8)
            variants_m.append(m); variants_t.append(bytes(tt))
        n = len(variants_m)
        off = np.arange(n + 1, dtype=np.uint64) * 40
        msg = np.frombuffer(b"".join(variants_m), np.uint8)
        tags = np.frombuffer(b"".join(variants_t), np.uint8).reshape(n, 32)
        mask, count = oracle.verify_batch(keys[j:j + 1], msg, off, np.zeros(n, np.uint32), tags)
        bits = np.unpackbits(mask.view(np.uint8), bitorder="little")[:n]
        assert bits[0] == 1 and count == 1, j
        ok_total += count
        # key flips: 256 flipped copies of the key, all checked against the true tag
        kf = np.repeat(keys[j:j + 1], 256, axis=0)
        kf[np.arange(256), np.arange(256) // 8] ^= (1 << (np.arange(256) % 8)).astype(np.uint8)
        off1 = np.arange(257, dtype=np.uint64) * 40
        mask, count = oracle.verify_batch(kf, np.frombuffer(m * 256, np.uint8), off1,
                                          np.arange(256, dtype=np.uint32),
                                          np.frombuffer(tag * 256, np.uint8).reshape(256, 32))
        assert count == 0, j
        # root-entropy flips: the derived key changes, so the credential fails
        rf = np.repeat(rev[j:j + 1], 256, axis=0)
        rf[np.arange(256), np.arange(256) // 8] ^= (1 << (np.arange(256) % 8)).astype(np.uint8)
        mask, count = oracle.verify_batch_rev(rf, salt, W.INFO_ATTEST,
                                              np.frombuffer(m * 256, np.uint8), off1,
                                              np.arange(256, dtype=np.uint32),
                                              np.frombuffer(tag * 256, np.uint8).reshape(256, 32))
        assert count == 0, j
    assert ok_total == 64


# ---------------------------------------------------------------- paper-form attestations
def _bits(mask, n):
    return np.unpackbits(np.asarray(mask, np.uint32).view(np.uint8), bitorder="little")[:n]


def _attest_by_hashlib(keys, payload, poff, ids, att):
    """Validity of each paper-form record from hashlib/hmac alone (no oracle code)."""
    out = np.zeros(ids.shape[0], bool)
    for i in range(ids.shape[0]):
        a, b = int(poff[i]), int(poff[i + 1])
        if ids[i] >= keys.shape[0] or b < a:
            continue
        rec = att[i].tobytes()
        bound = hashlib.sha256(payload[a:b].tobytes()).digest() == rec[:32]
        cred = hmac.digest(keys[ids[i]].tobytes(), rec[:40], "sha256") == rec[40:]
        out[i] = bound and cred
    return out


def test_attest_matches_truth_and_hashlib():
    w = W.paper_attestations(n=3000, n_id=512, n_invalid=300)
    keys = oracle.derive_keys(w.rev, w.domain, W.INFO_ATTEST, nthreads=4)
    assert (keys == w.keys).all()      # oracle HKDF == OpenSSL HKDF with the domain as salt
    mask, count = oracle.verify_attest(keys, w.payload, w.poff, w.ids, w.att, nthreads=4)
    assert count == 3000 - 300 == int(w.truth.sum())
    assert (mask == w.truth_bitmask()).all()
    ref = _attest_by_hashlib(keys, w.payload, w.poff, w.ids, w.att)
    assert (ref == w.truth).all()
    # every corruption kind occurred
    assert set(map(int, w.meta["bad_kind"])) == {W.P_PAYLOAD, W.P_OBJHASH, W.P_DOMAIN, W.P_CRED,
                                                 W.P_KEY}


def test_attest_single_bit_flips_and_special_cases():
    r = _rng(21)
    w = W.paper_attestations(n=8, n_id=8, n_invalid=0, seed=77)
    keys = w.keys
    for i in range(w.n):
        a, b = int(w.poff[i]), int(w.poff[i + 1])
        pl = w.payload[a:b]
        variants_p, variants_a = [pl], [w.att[i]]
        for bit in r.choice(8 * pl.size, size=64, replace=False):   # payload flips
            p2 = pl.copy(); p2[bit // 8] ^= 1 << (bit % 8)
            variants_p.append(p2); variants_a.append(w.att[i])
        for bit in range(8 * 72):                                  # every record bit
            a2 = w.att[i].copy(); a2[bit // 8] ^= 1 << (bit % 8)
            variants_p.append(pl); variants_a.append(a2)
        n = len(variants_p)
        poff = np.zeros(n + 1, np.uint64)
        np.cumsum([v.size for v in variants_p], out=poff[1:])
        mask, count = oracle.verify_attest(keys, np.concatenate(variants_p), poff,
                                           np.full(n, w.ids[i], np.uint32), np.stack(variants_a))
        bits = _bits(mask, n)
        assert bits[0] == 1 and count == 1, i
    # empty payload (binding to SHA-256 of the empty string), unregistered id, bad offsets
    dom = w.domain
    obj = hashlib.sha256(b"").digest()
    cred = hmac.digest(keys[0].tobytes(), obj + dom, "sha256")
    att = np.frombuffer((obj + dom + cred) * 3, np.uint8).reshape(3, 72)
    ids = np.array([0, 8, 0xFFFFFFFF], np.uint32)
    mask, count = oracle.verify_attest(keys, np.zeros(0, np.uint8), np.zeros(4, np.uint64), ids,
                                       att)
    assert count == 1 and mask[0] == 1
    poff = np.array([5, 5, 0, 0], np.uint64)            # record 1 has decreasing offsets
    mask, count = oracle.verify_attest(keys, np.zeros(8, np.uint8), poff,
                                       np.zeros(3, np.uint32), att)
    assert list(_bits(mask, 3)) == [1, 0, 1] and count == 2


# ---------------------------------------------------------------- several key streams
def _info_strings():
    return [l.split("\t")[1].encode() for l in
            open(__file__.replace("test_oracle_pins.py", "golden/info_strings.tsv"))
            .read().splitlines() if l and not l.startswith("#")]


def test_multi_stream_keys_against_openssl():
    """Every purpose string of the paper (golden file) and per-slot domains as
    salts: each stream's keys equal OpenSSL's HKDF, and no two keys coincide."""
    r = _rng(31)
    rev = r.integers(0, 256, size=(200, 32), dtype=np.uint8)
    streams = [(_bytes(r, 32), info) for info in _info_strings()]
    streams += [(_bytes(r, 8), W.INFO_ATTEST) for _ in range(3)]     # three slots' domains
    streams += [(b"", b""), (_bytes(r, 64), b"z" * 64)]
    out = oracle.derive_keys_multi(rev, streams, nthreads=4)
    assert out.shape == (len(streams), 200, 32)
    for s, (salt, info) in enumerate(streams):
        assert (out[s] == W.client_keys(rev, salt, info)).all(), s
    assert len({bytes(k) for k in out.reshape(-1, 32)}) == len(streams) * 200


# ---------------------------------------------------------------- hash-chain segments
def test_poh_segments_against_hashlib_chain():
    """One chain drawn with hashlib, cut at checkpoints of varying step counts
    (0 included): the oracle accepts exactly the uncorrupted segments, and a
    corrupted checkpoint shared by two segments breaks both."""
    r = _rng(41)
    steps = r.integers(0, 40, size=120).astype(np.uint32)
    w = W.poh_segments(n=120, steps=steps, chained=True, n_invalid=0, seed=41)
    assert (w.start[1:] == w.end[:-1]).all()
    h = w.start[0].tobytes()
    for i in range(120):           # the chain itself, independently of the generator's loop
        assert h == w.start[i].tobytes()
        for _ in range(int(steps[i])):
            h = hashlib.sha256(h).digest()
    mask, count = oracle.poh_verify(w.start, w.end, w.steps)
    assert count == 120 and (mask == W.pack_bits(np.ones(120, bool))).all()
    # corrupt checkpoint 50 (end of segment 49 = start of segment 50)
    start, end = w.start.copy(), w.end.copy()
    end[49, 3] ^= 0x10
    start[50] = end[49]
    mask, count = oracle.poh_verify(start, end, w.steps)
    bits = _bits(mask, 120)
    expect = np.ones(120, bool)
    expect[49] = False
    # segment 50 now starts from the corrupted value: broken unless it has no steps,
    # in which case its start and end are equal only if end[50] was corrupted alike
    expect[50] = (start[50] == end[50]).all() if w.steps[50] == 0 else False
    assert (bits.astype(bool) == expect).all()
    # a segment of zero steps is valid iff its ends are equal
    z = np.zeros((2, 32), np.uint8)
    z[1, 0] = 1
    mask, count = oracle.poh_verify(z[[0, 0]], z, np.zeros(2, np.uint32))
    assert list(_bits(mask, 2)) == [1, 0] and count == 1


def test_poh_segments_match_truth_and_openssl():
    w = W.poh_segments(n=2000, steps=97, n_invalid=40, seed=43)
    mask, count = oracle.poh_verify(w.start, w.end, w.steps, nthreads=4)
    assert count == 2000 - 40 == int(w.truth.sum())
    assert (mask == w.truth_bitmask()).all()
    # both corruption kinds occurred; one step too few is rejected like a flipped bit
    assert set(map(int, w.meta["bad_kind"])) == {0, 1}


# ---------------------------------------------------------------- Merkle roots
def _mth(leaves):
    """Merkle tree hash written the other way round: split at the largest power
    of two below n (the left-complete shape of RFC 6962, without its prefix
    bytes), leaf node = SHA-256(leaf)."""
    n = len(leaves)
    if n == 0:
        return hashlib.sha256(b"").digest()
    if n == 1:
        return hashlib.sha256(leaves[0]).digest()
    k = 1
    while 2 * k < n:
        k *= 2
    return hashlib.sha256(_mth(leaves[:k]) + _mth(leaves[k:])).digest()


def test_merkle_roots_against_recursive_split():
    """The level-by-level form with odd nodes moving up equals the recursive
    split form, for every tree size 0..70 and leaves of 0..200 bytes."""
    r = _rng(51)
    sizes = np.arange(0, 71)
    lens = r.integers(0, 201, size=int(sizes.sum()))
    off = np.zeros(lens.size + 1, np.uint64)
    np.cumsum(lens, out=off[1:])
    data = r.integers(0, 256, size=int(off[-1]), dtype=np.uint8)
    roots = oracle.merkle_roots(data, off, sizes)
    first = 0
    for b, n in enumerate(sizes):
        leaves = [data[int(off[i]):int(off[i + 1])].tobytes() for i in range(first, first + n)]
        assert roots[b].tobytes() == _mth(leaves), n
        first += n


def test_merkle_root_is_sensitive_to_every_leaf_bit_and_order():
    r = _rng(52)
    leaves = [_bytes(r, int(r.integers(1, 90))) for _ in range(13)]
    off = np.zeros(14, np.uint64)
    np.cumsum([len(x) for x in leaves], out=off[1:])
    base = oracle.merkle_roots(np.frombuffer(b"".join(leaves), np.uint8), off, [13])[0]
    seen = {base.tobytes()}
    for i in range(13):
        for bit in range(0, 8 * len(leaves[i]), 7):
            mod = [bytearray(x) for x in leaves]
            mod[i][bit // 8] ^= 1 << (bit % 8)
            root = oracle.merkle_roots(np.frombuffer(b"".join(mod), np.uint8), off, [13])[0]
            assert root.tobytes() not in seen
            seen.add(root.tobytes())
    swapped = leaves[:]
    swapped[3], swapped[4] = swapped[4], swapped[3]
    off2 = np.zeros(14, np.uint64)
    np.cumsum([len(x) for x in swapped], out=off2[1:])
    assert oracle.merkle_roots(np.frombuffer(b"".join(swapped), np.uint8), off2, [13])[0] \
        .tobytes() != base.tobytes()
    # decreasing offsets: the leaf is hashed as the empty string
    off3 = np.array([0, 5, 2, 9], np.uint64)
    data = np.frombuffer(_bytes(r, 9), np.uint8)
    got = oracle.merkle_roots(data, off3, [3])[0].tobytes()
    assert got == _mth([data[0:5].tobytes(), b"", data[2:9].tobytes()])
