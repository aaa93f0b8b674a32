"""Parity of the paper-form attestation check on the GPU (ace_verify_attestations)
with the CPU oracle and the generator's truth mask: payload binding
SHA-256(P) == obj_hash plus the credential HMAC(k, obj_hash || domain).
Integer work: every bitmask word and count identical (tolerance 0).  Every
test runs under the library's default launch tuning and the saved autotuned one."""
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
PER_TX_KEYS = 0x8


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


def upload(ace, w, poff=None, ids=None, payload_dev=None):
    return ace.upload_block(w.payload, w.poff if poff is None else poff,
                            w.ids if ids is None else ids, w.att, msg_dev=payload_dev,
                            record_bytes=72)


def keyset(ace, w, kind):
    rev = ace.to_device(w.rev)
    if kind == "midstate":
        return ace.midstate_keyset(rev, w.domain, w.info)
    return ace.rev_keyset(rev, w.domain, w.info)


def run(ace, w, kind, flags, poff=None, ids=None):
    import torch
    blk = upload(ace, w, poff, ids)
    ace.verify_attestations(keyset(ace, w, kind), [blk],
                            flags=flags | (PER_TX_KEYS if kind == "rev-per-tx" else 0))
    torch.cuda.synchronize()
    return blk.result()


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("kind", ["midstate", "rev", "rev-per-tx"])
def test_paper_form(ace, mode, kind):
    note("paper-form mode=%s keys=%s" % (mode, kind))
    w = W.paper_attestations(n=20_000, n_id=4096, n_invalid=500)
    mask, count = run(ace, w, kind, MODES[mode])
    omask, ocount = oracle.verify_attest(w.keys, w.payload, w.poff, w.ids, w.att, nthreads=8)
    assert count == ocount == 19_500 == int(w.truth.sum())
    assert np.array_equal(mask, omask)
    assert np.array_equal(mask, w.truth_bitmask())


@pytest.mark.parametrize("mode", list(MODES))
def test_every_payload_length_0_to_1300(ace, mode):
    """Payload lengths 0..1300 (every padding case of the digest chain), one
    record in ten corrupted, groups of 100 behind a 0-3 byte lead."""
    import torch
    note("paper-form lengths 0..1300 mode=%s" % mode)
    L = np.arange(0, 1301, dtype=np.int64)
    blocks, cases = [], []
    for g, lo in enumerate(range(0, L.size, 100)):
        hi = min(L.size, lo + 100)
        w = W.paper_attestations(n=hi - lo, n_id=64, lengths=L[lo:hi], id_dist="uniform",
                                 n_invalid=(hi - lo) // 10, seed=W.SEED_BASE + 100 + g)
        lead = g % 4
        poff = w.poff + lead
        buf = np.concatenate([np.zeros(lead, np.uint8), w.payload])
        payload_dev = ace.to_device(buf if buf.size else np.zeros(4, np.uint8))
        blocks.append(ace.upload_block(buf, poff, w.ids, w.att, msg_dev=payload_dev,
                                       record_bytes=72))
        cases.append((w, buf, poff))
    # each group draws its own registry and domain
    for blk, (w, buf, poff) in zip(blocks, cases):
        ace.verify_attestations(keyset(ace, w, "midstate"), [blk], flags=MODES[mode])
    torch.cuda.synchronize()
    for blk, (w, buf, poff) in zip(blocks, cases):
        mask, count = blk.result()
        omask, ocount = oracle.verify_attest(w.keys, buf, poff, w.ids, w.att)
        assert count == ocount == int(w.truth.sum())
        assert np.array_equal(mask, omask)
        assert np.array_equal(mask, w.truth_bitmask())


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4097])
def test_sizes(ace, n):
    note("paper-form n=%d" % n)
    w = W.paper_attestations(n=n, n_id=256, n_invalid=n // 10, seed=W.SEED_BASE + 200 + n)
    for mode in MODES.values():
        mask, count = run(ace, w, "midstate", mode)
        assert count == int(w.truth.sum())
        assert np.array_equal(mask, w.truth_bitmask())


def test_unregistered_ids_and_bad_offsets(ace):
    note("paper-form special cases")
    w = W.paper_attestations(n=300, n_id=128, n_invalid=0, seed=W.SEED_BASE + 300)
    ids = w.ids.copy()
    poff = w.poff.copy()
    ids[3] = w.n_id
    ids[4] = 0xFFFFFFFF
    poff[10], poff[11] = poff[11], poff[10]
    omask, ocount = oracle.verify_attest(w.keys, w.payload, poff, ids, w.att)
    for mode in MODES.values():
        mask, count = run(ace, w, "midstate", mode, poff=poff, ids=ids)
        assert count == ocount
        assert np.array_equal(mask, omask)


def test_every_single_bit_flip_is_rejected(ace):
    """Tamper invariants of the paper form on the GPU: for three attestations
    (payloads of 55, 64 and 200 bytes), every single-bit flip of the payload,
    of the 72-byte record (obj_hash, domain, credential) and of the identity's
    root entropy is a transaction of one batch; only the three untouched ones
    may pass, in every launch mode, with midstates and keys derived in the
    call."""
    import torch
    note("paper-form every single-bit flip")
    w = W.paper_attestations(n=3, n_id=3, lengths=np.array([55, 64, 200]), id_dist="uniform",
                             n_invalid=0, seed=W.SEED_BASE + 600)
    assert w.truth.all()
    rev = [w.rev]
    for j in range(3):                              # identity 3 + 256 j + b: REV_j, bit b flipped
        fl = np.repeat(w.rev[j:j + 1], 256, axis=0)
        fl[np.arange(256), np.arange(256) // 8] ^= (1 << (np.arange(256) % 8)).astype(np.uint8)
        rev.append(fl)
    rev = np.concatenate(rev)
    parts, ids, recs, truth = [], [], [], []
    for k in range(3):
        pl = w.payload[int(w.poff[k]):int(w.poff[k + 1])]
        j = int(w.ids[k])
        parts.append(pl); ids.append(j); recs.append(w.att[k]); truth.append(True)
        for b in range(8 * pl.size):                                                # payload flips
            f = pl.copy(); f[b // 8] ^= 1 << (b % 8)
            parts.append(f); ids.append(j); recs.append(w.att[k]); truth.append(False)
        for b in range(8 * 72):                                                     # record flips
            a = w.att[k].copy(); a[b // 8] ^= 1 << (b % 8)
            parts.append(pl); ids.append(j); recs.append(a); truth.append(False)
        for b in range(256):                                                        # root-entropy flips
            parts.append(pl); ids.append(3 + 256 * j + b); recs.append(w.att[k]); truth.append(False)
    lead = 3                                                                        # misaligned start
    buf = np.concatenate([np.zeros(lead, np.uint8)] + parts)
    poff = np.zeros(len(parts) + 1, np.uint64)
    poff[1:] = np.cumsum([p.size for p in parts])
    poff += lead
    ids = np.array(ids, np.uint32)
    recs = np.stack(recs)
    truth = np.array(truth)
    keys = oracle.derive_keys(rev, w.domain, w.info, 8)
    omask, ocount = oracle.verify_attest(keys, buf, poff, ids, recs, 8)
    assert ocount == 3 and np.array_equal(omask, W.pack_bits(truth))
    devrev = ace.to_device(rev)
    for mode in MODES.values():
        for ks in (ace.midstate_keyset(devrev, w.domain, w.info), ace.rev_keyset(devrev, w.domain, w.info)):
            blk = ace.upload_block(buf, poff, ids, recs, record_bytes=72)
            ace.verify_attestations(ks, [blk], flags=mode)
            torch.cuda.synchronize()
            mask, count = blk.result()
            assert count == 3 and np.array_equal(mask, omask), mode


@pytest.mark.parametrize("kind", ["midstate", "rev"])
def test_wide_records_read_offsets(ace, kind):
    """Paper form with wide_min_len lowered to 142 bytes (the median of these
    130-154 byte payloads): payloads of at least that length are read through
    their block's offsets, the rest through their bin-order records; results
    as the oracle's in both binned launch forms."""
    note("paper-form wide records keys=%s" % kind)
    w = W.paper_attestations(n=3000, n_id=256, n_invalid=300, seed=W.SEED_BASE + 500)
    ids = w.ids.copy()
    poff = w.poff.copy()
    ids[7] = w.n_id
    poff[20], poff[21] = poff[21], poff[20]
    omask, ocount = oracle.verify_attest(w.keys, w.payload, poff, ids, w.att)
    old = ace.get_tuning()
    try:
        ace.set_tuning(wide_min_len=142)
        for mode in ("binned", "binned-persistent"):
            mask, count = run(ace, w, kind, MODES[mode], poff=poff, ids=ids)
            assert count == ocount and np.array_equal(mask, omask), mode
    finally:
        ace.set_tuning(**old)


def test_multi_block(ace):
    """Several paper-form blocks in one call; bits land in their own blocks."""
    import torch
    note("paper-form multi-block")
    w = W.paper_attestations(n=9000, n_id=1024, n_invalid=90, seed=W.SEED_BASE + 400)
    cuts = [0, 1, 65, 4000, 4001, 9000]
    ks = keyset(ace, w, "midstate")
    for mode in MODES.values():
        blocks = []
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            poff = (w.poff[lo:hi + 1] - w.poff[lo]).astype(np.uint64)
            pl = w.payload[int(w.poff[lo]):int(w.poff[hi])]
            blocks.append(ace.upload_block(pl, poff, w.ids[lo:hi], w.att[lo:hi],
                                           record_bytes=72))
        ace.verify_attestations(ks, blocks, flags=mode)
        torch.cuda.synchronize()
        for blk, lo, hi in zip(blocks, cuts[:-1], cuts[1:]):
            mask, count = blk.result()
            assert count == int(w.truth[lo:hi].sum())
            assert np.array_equal(mask, W.pack_bits(w.truth[lo:hi]))
