"""Seeded synthetic workloads for the attestation check.

This module only draws random numbers (numpy PCG64) and lays them out the way
the verifier consumes them.  The credentials a client would attach (the
paper's Alg. 2, GenerateAttestation) are produced by the host's OpenSSL
through ``attest_client.c``; no hash arithmetic lives here.  The truth mask is
the corruption plan itself, so it is a witness independent of both the CPU
oracle and the GPU library.

Shapes follow the paper's workloads: 32-byte root entropy per identity
(Def. 2.1), a 32-byte credential per transaction (Def. 3.1), identities
chosen uniformly or Zipf-skewed, and message lengths fixed, uniform or
lognormal.  Every draw comes from ``SeedSequence(0xACE0 + config_no)``
spawned into independent child streams, one per quantity.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

INFO_16 = b"ACEGF-V1-MEMPOOL"            # 16-byte purpose string (first 16 bytes of the next)
INFO_ATTEST = b"ACEGF-V1-MEMPOOL-ATTEST"  # purpose string of equation attestkey

KIND_TAG, KIND_MSG, KIND_KEY = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_CLIENT_SRC = os.path.join(_HERE, "attest_client.c")
_DRIVER_SRC = os.path.join(_HERE, "serving_client.c")
_CLIENT_LIB = os.path.join(_HERE, "libace_client.so")
_client = None


def build_client(force: bool = True) -> str:
    if force or not os.path.exists(_CLIENT_LIB):
        tmp = _CLIENT_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp,
                               _CLIENT_SRC, _DRIVER_SRC, "-lcrypto", "-lpthread"])
        os.replace(tmp, _CLIENT_LIB)
    return _CLIENT_LIB


def _lib():
    global _client
    if _client is None:
        if not os.path.exists(_CLIENT_LIB):
            build_client(force=False)
        lib = ctypes.CDLL(_CLIENT_LIB)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        lib.client_derive_keys.argtypes = [vp, ctypes.c_uint64, vp, sz, vp, sz, vp, ctypes.c_int]
        lib.client_sign.argtypes = [vp, vp, vp, vp, ctypes.c_uint64, vp, ctypes.c_int]
        lib.client_digest.argtypes = [vp, vp, ctypes.c_uint64, vp, ctypes.c_int]
        lib.client_hash_chain.argtypes = [vp, vp, ctypes.c_uint64, vp, ctypes.c_int]
        lib.client_drive.argtypes = [vp] * 10 + [ctypes.c_uint64, ctypes.c_int] + [vp] * 4
        lib.client_drive.restype = ctypes.c_int
        _client = lib
    return _client


def host_threads() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, min(16, n or 1))


def client_keys(rev: np.ndarray, salt: bytes, info: bytes, nthreads: int | None = None) -> np.ndarray:
    """Client-side keys (OpenSSL HKDF-SHA256, 32 bytes) for every identity."""
    rev = np.ascontiguousarray(rev, dtype=np.uint8).reshape(-1, 32)
    keys = np.zeros_like(rev)
    sb, ib = (ctypes.c_char * max(1, len(salt))).from_buffer_copy(salt or b"\0"), \
        (ctypes.c_char * max(1, len(info))).from_buffer_copy(info or b"\0")
    rc = _lib().client_derive_keys(rev.ctypes.data, rev.shape[0], sb, len(salt), ib, len(info),
                                   keys.ctypes.data, nthreads or host_threads())
    if rc != 0:
        raise RuntimeError("OpenSSL HKDF failed (%d)" % rc)
    return keys


def client_sign(keys: np.ndarray, msg: np.ndarray, off: np.ndarray, key_index: np.ndarray,
                nthreads: int | None = None) -> np.ndarray:
    """Client-side credentials (OpenSSL HMAC-SHA256) for every transaction."""
    n = key_index.shape[0]
    tags = np.zeros((n, 32), np.uint8)
    if n == 0:
        return tags
    keys = np.ascontiguousarray(keys, dtype=np.uint8)
    msg_arg = msg if msg.size else np.zeros(1, np.uint8)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    key_index = np.ascontiguousarray(key_index, dtype=np.uint32)
    rc = _lib().client_sign(keys.ctypes.data, msg_arg.ctypes.data, off.ctypes.data,
                            key_index.ctypes.data, n, tags.ctypes.data,
                            nthreads or host_threads())
    if rc != 0:
        raise RuntimeError("OpenSSL HMAC failed (%d)" % rc)
    return tags


def client_digest(msg: np.ndarray, off: np.ndarray, nthreads: int | None = None) -> np.ndarray:
    """Client-side SHA-256 of every message (OpenSSL)."""
    n = off.shape[0] - 1
    out = np.zeros((n, 32), np.uint8)
    if n == 0:
        return out
    msg_arg = msg if msg.size else np.zeros(1, np.uint8)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    rc = _lib().client_digest(msg_arg.ctypes.data, off.ctypes.data, n, out.ctypes.data,
                              nthreads or host_threads())
    if rc != 0:
        raise RuntimeError("OpenSSL SHA-256 failed (%d)" % rc)
    return out


def client_hash_chain(start: np.ndarray, steps: np.ndarray, nthreads: int | None = None
                      ) -> np.ndarray:
    """end[i] = SHA-256 applied steps[i] times to start[i] (OpenSSL)."""
    start = np.ascontiguousarray(start, dtype=np.uint8).reshape(-1, 32)
    steps = np.ascontiguousarray(steps, dtype=np.uint32)
    out = np.zeros_like(start)
    if start.shape[0]:
        rc = _lib().client_hash_chain(start.ctypes.data, steps.ctypes.data, start.shape[0],
                                      out.ctypes.data, nthreads or host_threads())
        if rc != 0:
            raise RuntimeError("OpenSSL SHA-256 failed (%d)" % rc)
    return out


@dataclasses.dataclass
class Workload:
    """One batch of transactions plus the identity registry it refers to."""
    name: str
    rev: np.ndarray          # [n_id][32] u8 root entropy
    salt: bytes              # shared HKDF salt (the context)
    info: bytes              # HKDF purpose string
    msg: np.ndarray          # u8, all messages back to back
    off: np.ndarray          # u64 [n+1] byte offsets into msg
    ids: np.ndarray          # u32 [n] identity index of each tx
    tags: np.ndarray         # u8 [n][32] credential of each tx
    truth: np.ndarray        # bool [n] the generator's verdict (corruption plan)
    keys: np.ndarray         # u8 [n_id][32] client-side keys (OpenSSL)
    block_sizes: Optional[np.ndarray] = None   # for multi-block batches
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.ids.shape[0])

    @property
    def n_id(self) -> int:
        return int(self.rev.shape[0])

    def lengths(self) -> np.ndarray:
        return (self.off[1:] - self.off[:-1]).astype(np.int64)

    def truth_bitmask(self) -> np.ndarray:
        return pack_bits(self.truth)

    def block_ranges(self) -> list[tuple[int, int]]:
        if self.block_sizes is None:
            return [(0, self.n)]
        ends = np.cumsum(self.block_sizes)
        starts = ends - self.block_sizes
        return [(int(a), int(b)) for a, b in zip(starts, ends)]


def pack_bits(valid: np.ndarray) -> np.ndarray:
    """bool[n] -> u32[ceil(n/32)]: bit i%32 of word i/32, LSB first, tail bits 0."""
    n = valid.shape[0]
    words = (n + 31) // 32
    padded = np.zeros(words * 32, np.uint8)
    padded[:n] = valid.astype(np.uint8)
    by = np.packbits(padded.reshape(-1, 8), axis=1, bitorder="little").reshape(-1)
    return by.view(np.uint32).copy() if words else np.zeros(0, np.uint32)


def zipf_ids(rng_u: np.random.Generator, rng_perm: np.random.Generator, n: int, n_id: int,
             s: float) -> np.ndarray:
    """id = pi(rank), P(rank k) proportional to k^-s, inverse CDF on a float64 cumsum."""
    w = np.arange(1, n_id + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    u = rng_u.random(n) * cdf[-1]
    rank = np.minimum(np.searchsorted(cdf, u, side="right"), n_id - 1)
    perm = rng_perm.permutation(n_id).astype(np.uint32)
    return perm[rank]


def lognormal_lengths(rng: np.random.Generator, n: int, median: float = 200.0,
                      sigma: float = 0.75, lo: int = 64, hi: int = 1232) -> np.ndarray:
    z = rng.standard_normal(n)
    return np.clip(np.rint(np.exp(np.log(median) + sigma * z)), lo, hi).astype(np.int64)


def generate(name: str, seed: int, n: int, n_id: int, lengths, id_dist: str = "uniform",
             zipf_s: float = 1.1, n_invalid: int | None = None, p_invalid: float = 0.0,
             kinds: Sequence[int] = (KIND_TAG, KIND_MSG), info: bytes = INFO_16,
             block_sizes: np.ndarray | None = None, nthreads: int | None = None) -> Workload:
    """Draw one workload.  ``lengths`` is an int, an int array, or a callable(rng, n)."""
    ss = np.random.SeedSequence(seed)
    (r_rev, r_salt, r_idu, r_perm, r_len, r_msg, r_bad, r_kind, r_bit,
     r_wk) = [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(10)]

    rev = r_rev.integers(0, 256, size=(n_id, 32), dtype=np.uint8)
    salt = r_salt.integers(0, 256, size=32, dtype=np.uint8).tobytes()

    if id_dist == "uniform":
        ids = r_idu.integers(0, n_id, size=n, dtype=np.uint32) if n_id else np.zeros(n, np.uint32)
    elif id_dist == "zipf":
        ids = zipf_ids(r_idu, r_perm, n, n_id, zipf_s)
    else:
        raise ValueError(id_dist)

    if callable(lengths):
        L = np.asarray(lengths(r_len, n), dtype=np.int64)
    elif np.isscalar(lengths):
        L = np.full(n, int(lengths), np.int64)
    else:
        L = np.asarray(lengths, dtype=np.int64)
    off = np.zeros(n + 1, np.uint64)
    np.cumsum(L, out=off[1:])
    total = int(off[-1])
    msg = r_msg.integers(0, 256, size=total, dtype=np.uint8)

    if n_invalid is None:
        n_invalid = int(np.floor(p_invalid * n + 0.5))
    bad = r_bad.choice(n, size=n_invalid, replace=False) if n_invalid else np.zeros(0, np.int64)
    kind = np.asarray(kinds, np.int64)[r_kind.integers(0, len(kinds), size=n_invalid)]
    kind = np.where((kind == KIND_MSG) & (L[bad] == 0), KIND_TAG, kind)
    kind = np.where((kind == KIND_KEY) & (n_id < 2), KIND_TAG, kind)

    key_index = ids.copy()
    wk = bad[kind == KIND_KEY]
    if wk.size:
        other = r_wk.integers(0, n_id - 1, size=wk.size, dtype=np.int64)
        other = other + (other >= ids[wk])
        key_index[wk] = other.astype(np.uint32)

    keys = client_keys(rev, salt, info, nthreads)
    tags = client_sign(keys, msg, off, key_index, nthreads)

    # bit positions uniform within the chosen field
    field_bits = np.where(kind == KIND_MSG, 8 * L[bad], 256)
    bit = r_bit.integers(0, np.maximum(field_bits, 1), dtype=np.int64) if n_invalid else \
        np.zeros(0, np.int64)
    t_sel = kind == KIND_TAG
    tb = bad[t_sel]
    tags[tb, bit[t_sel] // 8] ^= (1 << (bit[t_sel] % 8)).astype(np.uint8)
    m_sel = kind == KIND_MSG
    mpos = off[bad[m_sel]].astype(np.int64) + bit[m_sel] // 8
    np.bitwise_xor.at(msg, mpos, (1 << (bit[m_sel] % 8)).astype(np.uint8))

    truth = np.ones(n, bool)
    truth[bad] = False
    meta = dict(seed=seed, n_invalid=int(n_invalid), kinds=list(map(int, kinds)),
                id_dist=id_dist, bad=bad, bad_kind=kind)
    return Workload(name, rev, salt, info, msg, off, ids.astype(np.uint32), tags, truth, keys,
                    block_sizes, meta)


# ----------------------------------------------------------------------------------------
# The five workloads: tiny, block scale, throughput sweep, batching, serving pool.
# ----------------------------------------------------------------------------------------
SEED_BASE = 0xACE0


def config1(nthreads=None) -> Workload:
    """1,024 identities, 4,096 txs, uniform ids, 128-byte messages, 205 bad (tag/msg flips)."""
    return generate("tiny", SEED_BASE + 1, n=4096, n_id=1024, lengths=128,
                    n_invalid=int(np.floor(0.05 * 4096 + 0.5)), kinds=(KIND_TAG, KIND_MSG),
                    nthreads=nthreads)


def config2(nthreads=None) -> Workload:
    """100,000 txs over 50,000 Zipf(1.1) identities, lengths U{96..512}, 1,000 bad."""
    return generate("block", SEED_BASE + 2, n=100_000, n_id=50_000,
                    lengths=lambda r, n: r.integers(96, 513, size=n),
                    id_dist="zipf", n_invalid=1000, kinds=(KIND_TAG, KIND_MSG, KIND_KEY),
                    nthreads=nthreads)


def config3(n: int = 16 << 20, n_id: int = 1 << 20, id_dist: str = "uniform",
            nthreads=None) -> Workload:
    """Throughput sweep: n txs, 1M identities, lognormal(200, 0.75) lengths in [64, 1232]."""
    return generate("sweep-%dM" % (n >> 20) if n >= (1 << 20) else "sweep-%d" % n,
                    SEED_BASE + 3, n=n, n_id=n_id, lengths=lognormal_lengths, id_dist=id_dist,
                    p_invalid=0.005, kinds=(KIND_TAG, KIND_MSG, KIND_KEY), nthreads=nthreads)


def batching_block_sizes(n_blocks: int = 256, seed: int = SEED_BASE + 4) -> np.ndarray:
    r = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
    z = r.standard_normal(n_blocks)
    return np.clip(np.rint(np.exp(np.log(19_500.0) + 1.0 * z)), 1_000, 200_000).astype(np.int64)


def config4(n_blocks: int = 256, n_id: int = 1 << 20, nthreads=None) -> Workload:
    """256 blocks of lognormal(19,500, 1.0) sizes in [1k, 200k]; lengths as the sweep; Zipf ids."""
    sizes = batching_block_sizes(n_blocks)
    return generate("batching-%d" % n_blocks, SEED_BASE + 4, n=int(sizes.sum()), n_id=n_id,
                    lengths=lognormal_lengths, id_dist="zipf", p_invalid=0.005,
                    kinds=(KIND_TAG, KIND_MSG, KIND_KEY), block_sizes=sizes, nthreads=nthreads)


def serving_request_sizes(n_req: int, seed: int = SEED_BASE + 5) -> np.ndarray:
    r = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
    z = r.standard_normal(n_req)
    return np.clip(np.rint(np.exp(np.log(1_000.0) + 1.5 * z)), 1, 50_000).astype(np.int64)


def serving_arrivals(n_req: int, rate_hz: float, seed: int = SEED_BASE + 5) -> np.ndarray:
    """Poisson arrivals: cumulative exponential gaps, seconds from t=0."""
    r = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2])))
    return np.cumsum(r.exponential(1.0 / rate_hz, size=n_req))


def config5_pool(n_pool: int = 4 << 20, n_id: int = 4 << 20, nthreads=None) -> Workload:
    """Transaction pool the serving requests are cut from: 4M Zipf identities, sweep lengths."""
    return generate("serving-pool", SEED_BASE + 5, n=n_pool, n_id=n_id,
                    lengths=lognormal_lengths, id_dist="zipf", p_invalid=0.005,
                    kinds=(KIND_TAG, KIND_MSG, KIND_KEY), nthreads=nthreads)


def subset(w: Workload, lo: int, hi: int, name: str | None = None) -> Workload:
    """Transactions [lo, hi) of a workload as a workload of their own (messages copied)."""
    a, b = int(w.off[lo]), int(w.off[hi])
    off = (w.off[lo:hi + 1] - w.off[lo]).astype(np.uint64)
    return Workload(name or "%s[%d:%d]" % (w.name, lo, hi), w.rev, w.salt, w.info,
                    w.msg[a:b].copy(), off, w.ids[lo:hi].copy(), w.tags[lo:hi].copy(),
                    w.truth[lo:hi].copy(), w.keys, None, dict(w.meta))


# ----------------------------------------------------------------------------------------
# Paper-form attestations (Def. 3.1): payload P, obj_hash = SHA-256(P), domain = c || s
# (8 bytes), key HKDF(REV, "ACEGF-V1-MEMPOOL-ATTEST", salt = domain), credential
# HMAC(k, obj_hash || domain).
# ----------------------------------------------------------------------------------------
P_PAYLOAD, P_OBJHASH, P_DOMAIN, P_CRED, P_KEY = 0, 1, 2, 3, 4


@dataclasses.dataclass
class AttestWorkload:
    name: str
    rev: np.ndarray       # [n_id][32]
    domain: bytes         # 8 bytes, the block's chain || slot; the HKDF salt
    info: bytes
    payload: np.ndarray   # u8, payloads back to back
    poff: np.ndarray      # u64 [n+1]
    ids: np.ndarray       # u32 [n]
    att: np.ndarray       # u8 [n][72]: obj_hash || domain || credential
    truth: np.ndarray
    keys: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.ids.shape[0])

    @property
    def n_id(self) -> int:
        return int(self.rev.shape[0])

    def lengths(self) -> np.ndarray:
        return (self.poff[1:] - self.poff[:-1]).astype(np.int64)

    def truth_bitmask(self) -> np.ndarray:
        return pack_bits(self.truth)


def paper_attestations(n: int = 2000, n_id: int = 1 << 16, seed: int = SEED_BASE + 6,
                       lengths=None, id_dist: str = "zipf", n_invalid: int | None = None,
                       p_invalid: float = 0.01, nthreads=None) -> AttestWorkload:
    """Paper-form transactions.  Payload lengths default to U{130..154}: the paper's
    220-244-byte transactions less the 90-byte attestation (Table 3)."""
    ss = np.random.SeedSequence(seed)
    (r_rev, r_dom, r_idu, r_perm, r_len, r_msg, r_bad, r_kind, r_bit,
     r_wk) = [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(10)]
    rev = r_rev.integers(0, 256, size=(n_id, 32), dtype=np.uint8)
    domain = r_dom.integers(0, 256, size=8, dtype=np.uint8).tobytes()
    if id_dist == "zipf":
        ids = zipf_ids(r_idu, r_perm, n, n_id, 1.1)
    else:
        ids = r_idu.integers(0, n_id, size=n, dtype=np.uint32)
    if lengths is None:
        L = r_len.integers(130, 155, size=n).astype(np.int64)
    elif callable(lengths):
        L = np.asarray(lengths(r_len, n), dtype=np.int64)
    else:
        L = np.full(n, int(lengths), np.int64) if np.isscalar(lengths) else np.asarray(lengths)
    poff = np.zeros(n + 1, np.uint64)
    np.cumsum(L, out=poff[1:])
    payload = r_msg.integers(0, 256, size=int(poff[-1]), dtype=np.uint8)
    keys = client_keys(rev, domain, INFO_ATTEST, nthreads)
    obj = client_digest(payload, poff, nthreads)
    dom = np.frombuffer(domain, np.uint8)
    msgs = np.concatenate([obj, np.repeat(dom[None, :], n, axis=0)], axis=1).reshape(-1)
    moff = np.arange(n + 1, dtype=np.uint64) * 40

    if n_invalid is None:
        n_invalid = int(np.floor(p_invalid * n + 0.5))
    bad = r_bad.choice(n, size=n_invalid, replace=False) if n_invalid else np.zeros(0, np.int64)
    kinds = (P_PAYLOAD, P_OBJHASH, P_DOMAIN, P_CRED, P_KEY)
    kind = np.asarray(kinds)[r_kind.integers(0, len(kinds), size=n_invalid)]
    kind = np.where((kind == P_PAYLOAD) & (L[bad] == 0), P_CRED, kind)
    key_index = ids.copy()
    wk = bad[kind == P_KEY]
    if wk.size:
        other = r_wk.integers(0, n_id - 1, size=wk.size, dtype=np.int64)
        other = other + (other >= ids[wk])
        key_index[wk] = other.astype(np.uint32)
    cred = client_sign(keys, msgs, moff, key_index, nthreads)
    att = np.concatenate([obj, np.repeat(dom[None, :], n, axis=0), cred], axis=1)
    # flips after signing: payload (binding fails), obj_hash, domain, credential
    field_bits = np.select([kind == P_PAYLOAD, kind == P_OBJHASH, kind == P_DOMAIN, kind == P_CRED],
                           [8 * L[bad], 256, 64, 256], 1)
    bit = r_bit.integers(0, np.maximum(field_bits, 1), dtype=np.int64) if n_invalid else \
        np.zeros(0, np.int64)
    for code, base in ((P_OBJHASH, 0), (P_DOMAIN, 32), (P_CRED, 40)):
        sel = kind == code
        att[bad[sel], base + bit[sel] // 8] ^= (1 << (bit[sel] % 8)).astype(np.uint8)
    sel = kind == P_PAYLOAD
    np.bitwise_xor.at(payload, poff[bad[sel]].astype(np.int64) + bit[sel] // 8,
                      (1 << (bit[sel] % 8)).astype(np.uint8))
    truth = np.ones(n, bool)
    truth[bad] = False
    return AttestWorkload("paper-form-%d" % n, rev, domain, INFO_ATTEST, payload, poff,
                          ids.astype(np.uint32), att, truth, keys,
                          dict(seed=seed, bad=bad, bad_kind=kind))


# ------------------------------------------------------------------ hash-chain segments
def client_merkle_root(data: np.ndarray, off: np.ndarray) -> bytes:
    """Root over the leaves data[off[i] .. off[i+1]) as a client builds it:
    leaf digests by OpenSSL, parents SHA-256(left || right) by hashlib, an
    unpaired last node moved up, SHA-256("") for no leaves."""
    import hashlib
    n = off.shape[0] - 1
    if n == 0:
        return hashlib.sha256(b"").digest()
    level = [bytes(x) for x in client_digest(data, off)]
    while len(level) > 1:
        nxt = [hashlib.sha256(level[i] + level[i + 1]).digest()
               for i in range(0, len(level) - 1, 2)]
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]


def client_drive(verify_stream_addr: int, stream_handle: int, pool, starts, sizes, arrivals,
                 threads: int = 8):
    """Open-loop submission of requests (starts[k], sizes[k]) of the pool at
    arrivals[k] (monotonic seconds) by native threads through the library's
    ace_verify_stream (its address).  Returns (tickets, submit times, masks,
    mask word offsets, counts); the caller polls and reads the tickets."""
    starts = np.ascontiguousarray(starts, np.uint64)
    sizes = np.ascontiguousarray(sizes, np.uint64)
    arrivals = np.ascontiguousarray(arrivals, np.float64)
    n = sizes.shape[0]
    words = (sizes + 31) // 32
    mask_words = np.zeros(n, np.uint64)
    np.cumsum(words[:-1], out=mask_words[1:])
    masks = np.zeros(max(1, int(words.sum())), np.uint32)
    counts = np.zeros(n, np.uint64)
    tickets = np.zeros(n, np.uint64)
    submit = np.zeros(n, np.float64)
    msg = np.ascontiguousarray(pool.msg, np.uint8)
    off = np.ascontiguousarray(pool.off, np.uint64)
    ids = np.ascontiguousarray(pool.ids, np.uint32)
    tags = np.ascontiguousarray(pool.tags, np.uint8)
    rc = _lib().client_drive(verify_stream_addr, stream_handle, msg.ctypes.data, off.ctypes.data,
                             ids.ctypes.data, tags.ctypes.data, starts.ctypes.data,
                             sizes.ctypes.data, mask_words.ctypes.data, arrivals.ctypes.data, n,
                             threads, masks.ctypes.data, counts.ctypes.data, tickets.ctypes.data,
                             submit.ctypes.data)
    if rc != 0:
        raise RuntimeError("ace_verify_stream failed (%d)" % rc)
    return tickets, submit, masks, mask_words, counts


@dataclasses.dataclass
class ChainWorkload:
    name: str
    start: np.ndarray     # [n][32]
    end: np.ndarray       # [n][32]
    steps: np.ndarray     # u32 [n]
    truth: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.steps.shape[0])

    def truth_bitmask(self) -> np.ndarray:
        return pack_bits(self.truth)


def poh_segments(n: int = 65536, steps=4096, seed: int = SEED_BASE + 7, chained: bool = False,
                 n_invalid: int | None = None, p_invalid: float = 0.005,
                 step_errors: bool = True, nthreads=None) -> ChainWorkload:
    """Segments of a SHA-256 hash chain (the clock of the consensus section):
    a checkpoint every `steps` hashes (an int, or one count per segment).
    chained=True draws one chain H_0 .. and cuts it at the checkpoints (end[i]
    == start[i+1]); otherwise every segment starts from its own random value,
    which has the same per-segment work and can be generated in parallel.
    Invalid segments: a bit of the end checkpoint flipped, or (step_errors) a
    claimed step count one more than the hashes that lead to the end."""
    ss = np.random.SeedSequence(seed)
    r_start, r_bad, r_kind, r_bit = [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(4)]
    st = (np.full(n, int(steps), np.uint32) if np.isscalar(steps)
          else np.asarray(steps, np.uint32).copy())
    if chained:
        import hashlib
        start = np.zeros((n, 32), np.uint8)
        end = np.zeros((n, 32), np.uint8)
        h = r_start.integers(0, 256, size=32, dtype=np.uint8).tobytes()
        for i in range(n):
            start[i] = np.frombuffer(h, np.uint8)
            for _ in range(int(st[i])):
                h = hashlib.sha256(h).digest()
            end[i] = np.frombuffer(h, np.uint8)
    else:
        start = r_start.integers(0, 256, size=(n, 32), dtype=np.uint8)
        end = client_hash_chain(start, st, nthreads)
    if n_invalid is None:
        n_invalid = int(np.floor(p_invalid * n + 0.5))
    bad = r_bad.choice(n, size=n_invalid, replace=False) if n_invalid else np.zeros(0, np.int64)
    kind = r_kind.integers(0, 2 if step_errors else 1, size=n_invalid)
    kind = np.where(st[bad] == 0, 0, kind)      # a zero-step segment cannot lose a step
    bit = r_bit.integers(0, 256, size=n_invalid)
    end = end.copy()
    flip = bad[kind == 0]
    end[flip, bit[kind == 0] // 8] ^= (1 << (bit[kind == 0] % 8)).astype(np.uint8)
    st[bad[kind == 1]] += 1    # the claimed count is one more than the hashes that lead there
    truth = np.ones(n, bool)
    truth[bad] = False
    return ChainWorkload("poh-%d" % n, start, end, st, truth,
                         dict(seed=seed, chained=chained, bad=bad, bad_kind=kind))
