"""ctypes wrapper over ``libace_oracle.so`` -- TEST INFRASTRUCTURE ONLY.

The C library is the plain definition of the attestation check (FIPS 180-4
SHA-256, RFC 2104 HMAC, RFC 5869 HKDF; the paper's Def. 2.1, Def. 3.1 and
Alg. 1 Phase 1a).  This module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ace_oracle.c")
_LIB = os.path.join(_HERE, "libace_oracle.so")
_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, pthreads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    sz = ctypes.c_size_t
    lib.oracle_constants.argtypes = [_u32p, _u32p]
    lib.oracle_sha256.argtypes = [_u8p, sz, _u8p]
    lib.oracle_sha256_compress.argtypes = [_u32p, _u8p]
    lib.oracle_sha256_iv.argtypes = [_u32p]
    lib.oracle_hmac_sha256.argtypes = [_u8p, sz, _u8p, sz, _u8p]
    lib.oracle_hmac_midstates.argtypes = [_u8p, sz, _u32p]
    lib.oracle_hkdf_sha256.argtypes = [_u8p, sz, _u8p, sz, _u8p, sz, _u8p, sz]
    lib.oracle_hkdf_sha256.restype = ctypes.c_int
    lib.oracle_derive_keys.argtypes = [_u8p, ctypes.c_uint32, _u8p, sz, _u8p, sz, _u8p,
                                       ctypes.c_int]
    lib.oracle_verify_batch.argtypes = [_u8p, ctypes.c_uint32, _u8p, _u64p, _u32p, _u8p,
                                        ctypes.c_uint64, _u32p, _u64p, ctypes.c_int]
    lib.oracle_verify_attest.argtypes = [_u8p, ctypes.c_uint32, _u8p, _u64p, _u32p, _u8p,
                                         ctypes.c_uint64, _u32p, _u64p, ctypes.c_int]
    lib.oracle_merkle_root.argtypes = [_u8p, _u64p, ctypes.c_uint64, _u8p]
    lib.oracle_merkle_root.restype = ctypes.c_int
    lib.oracle_poh_verify.argtypes = [_u8p, _u8p, _u32p, ctypes.c_uint64, _u32p, _u64p,
                                      ctypes.c_int]
    _lib = lib
    return lib


def _buf(b) -> ctypes.Array:
    b = bytes(b)
    return (ctypes.c_uint8 * max(1, len(b))).from_buffer_copy(b if b else b"\0")


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def constants() -> tuple[np.ndarray, np.ndarray]:
    """(K[64], H0[8]) as the oracle computes them from the primes."""
    k = np.zeros(64, np.uint32)
    iv = np.zeros(8, np.uint32)
    _load().oracle_constants(_ptr(k, _u32p), _ptr(iv, _u32p))
    return k, iv


def sha256(msg: bytes) -> bytes:
    out = (ctypes.c_uint8 * 32)()
    _load().oracle_sha256(_buf(msg), len(msg), out)
    return bytes(out)


def sha256_iv() -> np.ndarray:
    h = np.zeros(8, np.uint32)
    _load().oracle_sha256_iv(_ptr(h, _u32p))
    return h


def sha256_compress(state, block: bytes) -> np.ndarray:
    """One FIPS 180-4 block computation F(state, block); returns the new state."""
    if len(block) != 64:
        raise ValueError("a compression takes one 64-byte block")
    h = np.array(state, dtype=np.uint32).copy()
    _load().oracle_sha256_compress(_ptr(h, _u32p), _buf(block))
    return h


def hmac_sha256(key: bytes, msg: bytes) -> bytes:
    out = (ctypes.c_uint8 * 32)()
    _load().oracle_hmac_sha256(_buf(key), len(key), _buf(msg), len(msg), out)
    return bytes(out)


def hmac_midstates(keys: np.ndarray) -> np.ndarray:
    """[n][32] keys -> [n][16] u32: ipad state words 0-7, opad state 8-15."""
    keys = np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1, 32)
    out = np.zeros((keys.shape[0], 16), np.uint32)
    lib = _load()
    for j in range(keys.shape[0]):
        lib.oracle_hmac_midstates(_buf(keys[j].tobytes()), 32,
                                  out[j].ctypes.data_as(_u32p))
    return out


def hkdf_sha256(salt: bytes | None, ikm: bytes, info: bytes, length: int) -> bytes:
    out = (ctypes.c_uint8 * max(1, length))()
    s = b"" if salt is None else salt
    rc = _load().oracle_hkdf_sha256(_buf(s), len(s), _buf(ikm), len(ikm), _buf(info),
                                    len(info), out, length)
    if rc != 0:
        raise ValueError("HKDF output length exceeds 255 * 32")
    return bytes(out)[:length]


def derive_keys(rev: np.ndarray, salt: bytes, info: bytes, nthreads: int = 1) -> np.ndarray:
    """k_j = HKDF(salt, IKM = rev[j], info, 32) for every identity j."""
    rev = np.ascontiguousarray(rev, dtype=np.uint8).reshape(-1, 32)
    keys = np.zeros_like(rev)
    _load().oracle_derive_keys(_ptr(rev, _u8p), rev.shape[0], _buf(salt), len(salt),
                               _buf(info), len(info), _ptr(keys, _u8p), nthreads)
    return keys


def derive_keys_multi(rev: np.ndarray, streams, nthreads: int = 1) -> np.ndarray:
    """Keys of several HKDF streams (Def. 2.1: one root entropy, one key per
    (salt, info) purpose): out[s][j] = HKDF(salt_s, IKM = rev[j], info_s, 32)."""
    rev = np.ascontiguousarray(rev, dtype=np.uint8).reshape(-1, 32)
    out = np.zeros((len(streams), rev.shape[0], 32), np.uint8)
    for s, (salt, info) in enumerate(streams):
        out[s] = derive_keys(rev, salt, info, nthreads)
    return out


def verify_batch(keys: np.ndarray, msg: np.ndarray, off: np.ndarray, ids: np.ndarray,
                 tags: np.ndarray, nthreads: int = 1) -> tuple[np.ndarray, int]:
    """Bitmask (u32 words, LSB-first) and valid count for one block of txs."""
    keys = np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1, 32)
    msg = np.ascontiguousarray(msg, dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    tags = np.ascontiguousarray(tags, dtype=np.uint8).reshape(-1, 32)
    n = ids.shape[0]
    if off.shape[0] != n + 1 or tags.shape[0] != n:
        raise ValueError("off must hold n + 1 entries and tags n rows")
    mask = np.zeros(max(1, (n + 31) // 32), np.uint32)
    cnt = ctypes.c_uint64(0)
    msg_arg = msg if msg.size else np.zeros(1, np.uint8)
    _load().oracle_verify_batch(_ptr(keys, _u8p) if keys.size else None, keys.shape[0],
                                _ptr(msg_arg, _u8p), _ptr(off, _u64p), _ptr(ids, _u32p),
                                _ptr(tags, _u8p) if tags.size else None, n,
                                _ptr(mask, _u32p), ctypes.byref(cnt), nthreads)
    return mask[: (n + 31) // 32], int(cnt.value)


def verify_batch_rev(rev: np.ndarray, salt: bytes, info: bytes, msg, off, ids, tags,
                     nthreads: int = 1) -> tuple[np.ndarray, int]:
    """Keys derived from REV by HKDF first (Alg. 1 Phase 1a), then verified."""
    keys = derive_keys(rev, salt, info, nthreads)
    return verify_batch(keys, msg, off, ids, tags, nthreads)


def verify_attest(keys: np.ndarray, payload: np.ndarray, poff: np.ndarray, ids: np.ndarray,
                  att: np.ndarray, nthreads: int = 1) -> tuple[np.ndarray, int]:
    """Paper-form check: SHA-256(payload) == obj_hash and HMAC(k, obj_hash || domain) == cred."""
    keys = np.ascontiguousarray(keys, dtype=np.uint8).reshape(-1, 32)
    payload = np.ascontiguousarray(payload, dtype=np.uint8)
    poff = np.ascontiguousarray(poff, dtype=np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    att = np.ascontiguousarray(att, dtype=np.uint8).reshape(-1, 72)
    n = ids.shape[0]
    if poff.shape[0] != n + 1 or att.shape[0] != n:
        raise ValueError("poff must hold n + 1 entries and att n rows")
    mask = np.zeros(max(1, (n + 31) // 32), np.uint32)
    cnt = ctypes.c_uint64(0)
    p_arg = payload if payload.size else np.zeros(1, np.uint8)
    _load().oracle_verify_attest(_ptr(keys, _u8p) if keys.size else None, keys.shape[0],
                                 _ptr(p_arg, _u8p), _ptr(poff, _u64p), _ptr(ids, _u32p),
                                 _ptr(att, _u8p) if att.size else None, n, _ptr(mask, _u32p),
                                 ctypes.byref(cnt), nthreads)
    return mask[: (n + 31) // 32], int(cnt.value)


def poh_verify(start: np.ndarray, end: np.ndarray, steps: np.ndarray,
               nthreads: int = 1) -> tuple[np.ndarray, int]:
    """Hash-chain segments: bit i iff SHA-256^steps[i](start[i]) == end[i]."""
    start = np.ascontiguousarray(start, dtype=np.uint8).reshape(-1, 32)
    end = np.ascontiguousarray(end, dtype=np.uint8).reshape(-1, 32)
    steps = np.ascontiguousarray(steps, dtype=np.uint32)
    n = steps.shape[0]
    if start.shape[0] != n or end.shape[0] != n:
        raise ValueError("start and end must hold one row per segment")
    mask = np.zeros(max(1, (n + 31) // 32), np.uint32)
    cnt = ctypes.c_uint64(0)
    if n:
        _load().oracle_poh_verify(_ptr(start, _u8p), _ptr(end, _u8p), _ptr(steps, _u32p), n,
                                  _ptr(mask, _u32p), ctypes.byref(cnt), nthreads)
    return mask[: (n + 31) // 32], int(cnt.value)


def merkle_roots(data: np.ndarray, off: np.ndarray, tree_sizes) -> np.ndarray:
    """Roots [n_trees][32] of consecutive trees: tree b holds the next
    tree_sizes[b] leaves, leaf i being data[off[i] .. off[i+1])."""
    data = np.ascontiguousarray(data, dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    sizes = np.asarray(tree_sizes, dtype=np.int64)
    if off.shape[0] != int(sizes.sum()) + 1:
        raise ValueError("off must hold one entry per leaf plus one")
    d_arg = data if data.size else np.zeros(1, np.uint8)
    roots = np.zeros((sizes.shape[0], 32), np.uint8)
    lib = _load()
    first = 0
    for b, n in enumerate(sizes):
        sub = off[first:first + n + 1] if n else off[first:first + 1]
        out = (ctypes.c_uint8 * 32)()
        if lib.oracle_merkle_root(_ptr(d_arg, _u8p), _ptr(np.ascontiguousarray(sub), _u64p),
                                  int(n), out) != 0:
            raise MemoryError("oracle_merkle_root")
        roots[b] = np.frombuffer(bytes(out), np.uint8)
        first += int(n)
    return roots
