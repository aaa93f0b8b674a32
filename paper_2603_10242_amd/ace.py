"""Python binding of ``libace.so`` (include/ace.h): argument marshalling only.

Every step of the attestation check runs in the library's HIP kernels; this
module passes torch-allocated device pointers and the current HIP stream.
There is no fallback: if the library is missing or the GPU is absent, calls
raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime that libace.so then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libace.so")

ACE_OK = 0
ACE_ERR_INVALID_ARG = -1
ACE_ERR_RANGE = -2
ACE_ERR_NO_MEMORY = -3
ACE_ERR_DEVICE = -4
ACE_ERR_AGAIN = -5
ACE_ERR_TOO_LARGE = -6

ACE_ORDERED = 0x1
ACE_BUCKETED = 0x2
ACE_PERSISTENT = 0x4
ACE_PER_TX_KEYS = 0x8

ACE_KEYS_MIDSTATE = 0
ACE_KEYS_REV = 1

ACE_SCRATCH_BYTES = 64 << 20  # scratch array of ace_verify_batch_noalloc, per device


class AceError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("ace error %d: %s" % (code, msg))
        self.code = code


class ace_block(ctypes.Structure):
    _fields_ = [("d_msg", ctypes.c_void_p), ("d_off", ctypes.c_void_p),
                ("d_id", ctypes.c_void_p), ("d_tag", ctypes.c_void_p),
                ("n_tx", ctypes.c_uint64), ("d_bitmask_out", ctypes.c_void_p),
                ("d_count_out", ctypes.c_void_p)]


class ace_keyset(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("d_mid", ctypes.c_void_p), ("d_rev", ctypes.c_void_p),
                ("n_id", ctypes.c_uint32), ("h_salt", ctypes.c_void_p),
                ("salt_len", ctypes.c_size_t), ("h_info", ctypes.c_void_p),
                ("info_len", ctypes.c_size_t)]


class ace_hkdf_stream(ctypes.Structure):
    _fields_ = [("h_salt", ctypes.c_void_p), ("salt_len", ctypes.c_size_t),
                ("h_info", ctypes.c_void_p), ("info_len", ctypes.c_size_t)]


class ace_merkle_tree(ctypes.Structure):
    _fields_ = [("d_data", ctypes.c_void_p), ("d_off", ctypes.c_void_p),
                ("n_leaves", ctypes.c_uint64), ("d_root_out", ctypes.c_void_p)]


ACE_LENGTH_BUCKETS = 64


class ace_tuning(ctypes.Structure):
    _fields_ = [("binned_min_tx", ctypes.c_uint64), ("verify_wgs_per_cu", ctypes.c_uint32),
                ("aux_wgs_per_cu", ctypes.c_uint32), ("auto_persistent", ctypes.c_uint32),
                ("derive_wgs_per_cu", ctypes.c_uint32), ("wide_min_len", ctypes.c_uint64),
                ("grab_cap", ctypes.c_uint8 * ACE_LENGTH_BUCKETS)]


class ace_profile(ctypes.Structure):
    _fields_ = [("derive_ms", ctypes.c_double), ("bin_ms", ctypes.c_double),
                ("verify_ms", ctypes.c_double), ("finalize_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("calls", ctypes.c_uint64)]


_lib = None
_DEFAULT_TUNING: Optional[dict] = None


def load(path: str = LIB_PATH):
    """Load libace.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libace.so not built (%s): run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    vp, sz, u32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32
    lib.ace_last_error.restype = ctypes.c_char_p
    lib.ace_version.restype = ctypes.c_char_p
    lib.ace_derive_keys.argtypes = [vp, u32, vp, sz, vp, sz, vp, vp, vp]
    lib.ace_derive_keys.restype = ctypes.c_int
    lib.ace_verify_workspace_size.argtypes = [ctypes.POINTER(ace_keyset),
                                              ctypes.POINTER(ace_block), u32, u32]
    lib.ace_verify_workspace_size.restype = sz
    lib.ace_verify_batch.argtypes = [ctypes.POINTER(ace_keyset), ctypes.POINTER(ace_block), u32,
                                     vp, sz, u32, vp]
    lib.ace_verify_batch.restype = ctypes.c_int
    lib.ace_derive_keys_multi.argtypes = [vp, u32, ctypes.POINTER(ace_hkdf_stream), u32, vp, vp,
                                          vp]
    lib.ace_derive_keys_multi.restype = ctypes.c_int
    lib.ace_merkle_workspace_size.argtypes = [ctypes.POINTER(ace_merkle_tree), u32]
    lib.ace_merkle_workspace_size.restype = sz
    lib.ace_merkle_roots.argtypes = [ctypes.POINTER(ace_merkle_tree), u32, vp, sz, vp]
    lib.ace_merkle_roots.restype = ctypes.c_int
    lib.ace_poh_verify.argtypes = [vp, vp, vp, u32, ctypes.c_uint64, vp, vp, vp]
    lib.ace_poh_verify.restype = ctypes.c_int
    lib.ace_valu_rate.argtypes = [u32, u32, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.ace_valu_rate.restype = ctypes.c_int
    lib.ace_verify_attestations.argtypes = lib.ace_verify_batch.argtypes
    lib.ace_verify_batch_noalloc.argtypes = [ctypes.POINTER(ace_keyset), ctypes.POINTER(ace_block),
                                             u32, u32, vp]
    lib.ace_verify_batch_noalloc.restype = ctypes.c_int
    lib.ace_verify_attestations.restype = ctypes.c_int
    lib.ace_get_tuning.argtypes = [ctypes.POINTER(ace_tuning)]
    lib.ace_set_tuning.argtypes = [ctypes.POINTER(ace_tuning)]
    lib.ace_graph_workspace_size.argtypes = [ctypes.POINTER(ace_keyset), u32, ctypes.c_uint64, u32]
    lib.ace_graph_workspace_size.restype = sz
    lib.ace_graph_create.argtypes = [ctypes.POINTER(ace_keyset), u32, ctypes.c_uint64, vp, sz, u32,
                                     ctypes.POINTER(vp)]
    lib.ace_graph_launch.argtypes = [vp, ctypes.POINTER(ace_block), u32, vp]
    lib.ace_graph_destroy.argtypes = [vp]
    lib.ace_profile_enable.argtypes = [ctypes.c_int]
    lib.ace_profile_enable.restype = ctypes.c_int
    lib.ace_profile_read.argtypes = [ctypes.POINTER(ace_profile), ctypes.c_int]
    lib.ace_profile_read.restype = ctypes.c_int
    _lib = lib
    global _DEFAULT_TUNING
    _DEFAULT_TUNING = get_tuning()  # nothing can have changed it before the first load
    return lib


def _check(rc: int) -> None:
    if rc != ACE_OK:
        raise AceError(rc, load().ace_last_error().decode())


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(t: Optional[torch.Tensor], nbytes: int = 0, what: str = "tensor") -> Optional[int]:
    """Device pointer of t (None passes through), after checking that it is a
    contiguous device tensor of at least nbytes bytes: the library cannot see
    the size of a device buffer, so an undersized one must not reach it."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s: a contiguous device tensor is required" % what)
    _require_bytes(t.numel() * t.element_size(), nbytes, what)
    return t.data_ptr()


def _require_bytes(have: int, need: int, what: str) -> None:
    if have < need:
        raise ValueError("%s: %d bytes, %d needed" % (what, have, need))


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


# ------------------------------------------------------------------------------ containers
@dataclasses.dataclass
class DeviceBlock:
    """One block of transactions resident on the device, plus its outputs."""
    msg: torch.Tensor       # uint8 [total bytes] (may be a shared buffer)
    off: torch.Tensor       # int64 [n+1] (uint64 bits)
    ids: torch.Tensor       # int32 [n]   (uint32 bits)
    tags: torch.Tensor      # uint8 [n, 32]
    bitmask: torch.Tensor   # int32 [ceil(n/32)]
    count: torch.Tensor     # int64 [1]
    n: int

    def __setattr__(self, name, value):
        # a reassigned field invalidates the validated C descriptors below
        object.__setattr__(self, name, value)
        self.__dict__.pop("_structs", None)

    def struct(self, record_bytes: int = 32) -> ace_block:
        """The C descriptor (checked once per record width and kept until a field
        is reassigned; tensors must not be resized in place meanwhile)."""
        cache = self.__dict__.setdefault("_structs", {})
        s = cache.get(record_bytes)
        if s is None:
            n = self.n
            s = ace_block(_ptr(self.msg, 0, "msg"), _ptr(self.off, 8 * (n + 1), "off"),
                          _ptr(self.ids, 4 * n, "ids"), _ptr(self.tags, record_bytes * n, "tags"), n,
                          _ptr(self.bitmask, 4 * ((n + 31) // 32), "bitmask"),
                          _ptr(self.count, 8, "count"))
            cache[record_bytes] = s
        return s

    def result(self) -> tuple[np.ndarray, int]:
        m = self.bitmask.cpu().numpy().view(np.uint32).copy()
        return m, int(self.count.cpu().item())


@dataclasses.dataclass
class DeviceKeyset:
    kind: int
    n_id: int
    mid: Optional[torch.Tensor] = None   # int32 [n_id, 16]
    rev: Optional[torch.Tensor] = None   # uint8 [n_id, 32]
    salt: bytes = b""
    info: bytes = b""

    def struct(self) -> tuple[ace_keyset, list]:
        keep = [ctypes.create_string_buffer(self.salt, max(1, len(self.salt))),
                ctypes.create_string_buffer(self.info, max(1, len(self.info)))]
        ks = ace_keyset(self.kind, _ptr(self.mid, 64 * self.n_id, "midstates"),
                        _ptr(self.rev, 32 * self.n_id, "rev"), self.n_id,
                        ctypes.addressof(keep[0]), len(self.salt), ctypes.addressof(keep[1]),
                        len(self.info))
        return ks, keep


def to_device(a: np.ndarray, dtype=None, device="cuda") -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    elif a.dtype == np.uint32:
        a = a.view(np.int32)
    t = torch.from_numpy(a)
    return t.to(device) if dtype is None else t.to(device=device, dtype=dtype)


def upload_block(msg, off, ids, tags, device="cuda", msg_dev: Optional[torch.Tensor] = None,
                 record_bytes: int = 32) -> DeviceBlock:
    """Copies one block's arrays to the device and allocates its outputs.

    ``tags`` holds one check record per transaction: the 32-byte credential,
    or (record_bytes=72) the attestation obj_hash || domain || credential.
    """
    n = int(np.asarray(ids).shape[0])
    off = np.asarray(off, np.uint64)
    if off.shape[0] != n + 1:
        raise ValueError("off: %d entries for %d transactions" % (off.shape[0], n))
    if msg_dev is not None:
        m = msg_dev
        if n and _nbytes(m) < int(off[-1]):
            raise ValueError("msg_dev: %d bytes, offsets reach %d" % (_nbytes(m), int(off[-1])))
    else:
        host = np.asarray(msg, np.uint8).reshape(-1)
        # an all-empty batch still gets a real (4-byte) buffer to point at
        m = to_device(host if host.size else np.zeros(4, np.uint8), device=device)
    return DeviceBlock(m, to_device(off, device=device),
                       to_device(np.asarray(ids, np.uint32), device=device),
                       to_device(np.asarray(tags, np.uint8).reshape(-1, record_bytes),
                                 device=device),
                       torch.zeros((n + 31) // 32, dtype=torch.int32, device=device),
                       torch.zeros(1, dtype=torch.int64, device=device), n)


# ------------------------------------------------------------------------------ entry points
def derive_keys(rev: torch.Tensor, salt: bytes, info: bytes, key_out: Optional[torch.Tensor] = None,
                mid_out: Optional[torch.Tensor] = None, stream=None) -> None:
    """ace_derive_keys: HKDF-SHA256 keys and/or their HMAC midstates."""
    n_id = int(rev.shape[0]) if rev is not None else 0
    sb = ctypes.create_string_buffer(salt, max(1, len(salt)))
    ib = ctypes.create_string_buffer(info, max(1, len(info)))
    _check(load().ace_derive_keys(_ptr(rev, 32 * n_id, "rev") if n_id else None, n_id,
                                  ctypes.addressof(sb), len(salt), ctypes.addressof(ib), len(info),
                                  _ptr(key_out, 32 * n_id, "key_out"),
                                  _ptr(mid_out, 64 * n_id, "mid_out"), _stream(stream)))


def derive_keys_multi(rev: torch.Tensor, streams: Sequence[tuple[bytes, bytes]],
                      key_out: Optional[torch.Tensor] = None,
                      mid_out: Optional[torch.Tensor] = None, stream=None) -> None:
    """ace_derive_keys_multi: keys [S][n_id][32] and/or midstates [S][n_id][16]
    of S (salt, info) streams."""
    n_id = int(rev.shape[0]) if rev is not None else 0
    keep = []
    arr = (ace_hkdf_stream * max(1, len(streams)))()
    for k, (salt, info) in enumerate(streams):
        sb = ctypes.create_string_buffer(salt, max(1, len(salt)))
        ib = ctypes.create_string_buffer(info, max(1, len(info)))
        keep += [sb, ib]
        arr[k] = ace_hkdf_stream(ctypes.addressof(sb), len(salt), ctypes.addressof(ib), len(info))
    S = len(streams)
    _check(load().ace_derive_keys_multi(_ptr(rev, 32 * n_id, "rev") if n_id else None, n_id, arr, S,
                                        _ptr(key_out, 32 * n_id * S, "key_out"),
                                        _ptr(mid_out, 64 * n_id * S, "mid_out"), _stream(stream)))


def _blocks_array(blocks: Sequence[DeviceBlock], record_bytes: int = 32):
    arr = (ace_block * max(1, len(blocks)))()
    for i, b in enumerate(blocks):
        arr[i] = b.struct(record_bytes)
    return arr


def verify_workspace_size(keyset: DeviceKeyset, blocks: Sequence[DeviceBlock], flags: int = 0) -> int:
    ks, keep = keyset.struct()
    arr = _blocks_array(blocks)
    return int(load().ace_verify_workspace_size(ctypes.byref(ks), arr, len(blocks), flags))


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _verify(fn, keyset: DeviceKeyset, blocks: Sequence[DeviceBlock],
            ws: Optional[torch.Tensor], flags: int, stream, record_bytes: int = 32) -> torch.Tensor:
    ks, keep = keyset.struct()
    arr = _blocks_array(blocks, record_bytes)
    lib = load()
    need = int(lib.ace_verify_workspace_size(ctypes.byref(ks), arr, len(blocks), flags))
    if need == 0 and len(blocks):
        _check(fn(ctypes.byref(ks), arr, len(blocks), None, 0, flags, None))
    if ws is None or _nbytes(ws) < need:
        ws = workspace(need, device=blocks[0].bitmask.device if blocks else "cuda")
    _check(fn(ctypes.byref(ks), arr, len(blocks), _ptr(ws, need, "workspace"), _nbytes(ws), flags,
              _stream(stream)))
    return ws


def verify_batch(keyset: DeviceKeyset, blocks: Sequence[DeviceBlock],
                 ws: Optional[torch.Tensor] = None, flags: int = 0, stream=None) -> torch.Tensor:
    """ace_verify_batch over the given blocks; returns the workspace used."""
    return _verify(load().ace_verify_batch, keyset, blocks, ws, flags, stream)


def verify_attestations(keyset: DeviceKeyset, blocks: Sequence[DeviceBlock],
                        ws: Optional[torch.Tensor] = None, flags: int = 0,
                        stream=None) -> torch.Tensor:
    """ace_verify_attestations (blocks uploaded with record_bytes=72)."""
    return _verify(load().ace_verify_attestations, keyset, blocks, ws, flags, stream, 72)


def verify_batch_noalloc(keyset: DeviceKeyset, blocks: Sequence[DeviceBlock], flags: int = 0,
                         stream=None) -> None:
    """ace_verify_batch_noalloc: the library's static scratch array instead of
    a workspace (at most ACE_SCRATCH_BYTES; larger calls raise)."""
    ks, keep = keyset.struct()
    arr = _blocks_array(blocks)
    _check(load().ace_verify_batch_noalloc(ctypes.byref(ks), arr, len(blocks), flags,
                                           _stream(stream)))


def merkle_roots(trees: Sequence[tuple[torch.Tensor, torch.Tensor, int, torch.Tensor]],
                 ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """ace_merkle_roots over (data, off, n_leaves, root_out[32]) device tensors;
    returns the workspace used."""
    arr = (ace_merkle_tree * max(1, len(trees)))()
    for i, (data, off, n, root) in enumerate(trees):
        n = int(n)
        arr[i] = ace_merkle_tree(_ptr(data, 0, "data") if n else None,
                                 _ptr(off, 8 * (n + 1), "off") if n else None, n,
                                 _ptr(root, 32, "root"))
    lib = load()
    need = int(lib.ace_merkle_workspace_size(arr, len(trees)))
    if need == 0 and len(trees):
        _check(lib.ace_merkle_roots(arr, len(trees), None, 0, None))
    if ws is None or _nbytes(ws) < need:
        ws = workspace(need)
    _check(lib.ace_merkle_roots(arr, len(trees), _ptr(ws, need, "workspace"), _nbytes(ws),
                                _stream(stream)))
    return ws


def poh_verify(start: torch.Tensor, end: torch.Tensor, steps, bitmask: torch.Tensor,
               count: torch.Tensor, stream=None) -> None:
    """ace_poh_verify: `steps` is an int (every segment) or a uint32 tensor [n]."""
    n = int(start.shape[0])
    if isinstance(steps, torch.Tensor):
        d_steps, uni = _ptr(steps, 4 * n, "steps"), 0
    else:
        d_steps, uni = None, int(steps)
    _check(load().ace_poh_verify(_ptr(start, 32 * n, "start"), _ptr(end, 32 * n, "end"), d_steps, uni,
                                 n, _ptr(bitmask, 4 * ((n + 31) // 32), "bitmask"),
                                 _ptr(count, 8, "count"), _stream(stream)))


def valu_rate(iters: int = 20000, wgs_per_cu: int = 8, stream=None) -> float:
    """ace_valu_rate: measured INT32 VALU lane instructions per second."""
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = ctypes.c_double()
    _check(load().ace_valu_rate(iters, wgs_per_cu, _ptr(sink), ctypes.byref(out),
                                _stream(stream)))
    return out.value


def midstate_keyset(rev: torch.Tensor, salt: bytes, info: bytes, stream=None) -> DeviceKeyset:
    """Derives the resident midstate cache of a registry (ace_derive_keys)."""
    n_id = int(rev.shape[0])
    mid = torch.empty((max(n_id, 1), 16), dtype=torch.int32, device=rev.device)
    if n_id:
        derive_keys(rev, salt, info, mid_out=mid, stream=stream)
    return DeviceKeyset(ACE_KEYS_MIDSTATE, n_id, mid=mid)


def rev_keyset(rev: torch.Tensor, salt: bytes, info: bytes) -> DeviceKeyset:
    return DeviceKeyset(ACE_KEYS_REV, int(rev.shape[0]), rev=rev, salt=salt, info=info)


def profile_enable(on: bool = True) -> None:
    """ace_profile_enable: stage timing of ace_verify_batch on this thread."""
    _check(load().ace_profile_enable(1 if on else 0))


def profile_read(reset: bool = True) -> dict:
    """ace_profile_read: summed stage milliseconds of the profiled calls."""
    p = ace_profile()
    _check(load().ace_profile_read(ctypes.byref(p), 1 if reset else 0))
    return {k: getattr(p, k) for k, _ in ace_profile._fields_}


def get_tuning() -> dict:
    """ace_get_tuning as a dict (grab_cap as a list of 64 ints)."""
    t = ace_tuning()
    _check(load().ace_get_tuning(ctypes.byref(t)))
    out = {k: getattr(t, k) for k, _ in ace_tuning._fields_}
    out["grab_cap"] = list(out["grab_cap"])
    return out


def default_tuning() -> dict:
    """The library's own launch tuning (before any ace_set_tuning)."""
    load()
    return dict(_DEFAULT_TUNING)


def set_tuning(**kw) -> dict:
    """ace_set_tuning: updates the given fields, returns the previous tuning."""
    old = get_tuning()
    new = dict(old)
    new.update(kw)
    caps = [int(c) for c in new.pop("grab_cap")]
    if len(caps) != ACE_LENGTH_BUCKETS:
        raise ValueError("grab_cap needs %d entries" % ACE_LENGTH_BUCKETS)
    t = ace_tuning(*[int(new[k]) for k, _ in ace_tuning._fields_[:-1]],
                   (ctypes.c_uint8 * ACE_LENGTH_BUCKETS)(*caps))
    _check(load().ace_set_tuning(ctypes.byref(t)))
    return old


class Graph:
    """ace_graph_*: one capture of the whole pass, replayed for any block mix."""

    def __init__(self, keyset: DeviceKeyset, max_blocks: int, max_tx: int, flags: int = 0,
                 device="cuda"):
        lib = load()
        self._ks, self._keep = keyset.struct()
        self.keyset = keyset
        need = int(lib.ace_graph_workspace_size(ctypes.byref(self._ks), max_blocks, max_tx, flags))
        if need == 0:
            raise AceError(ACE_ERR_INVALID_ARG, "bad graph arguments")
        self.ws = workspace(need, device=device)
        h = ctypes.c_void_p()
        _check(lib.ace_graph_create(ctypes.byref(self._ks), max_blocks, max_tx,
                                    _ptr(self.ws, need, "workspace"), _nbytes(self.ws), flags,
                                    ctypes.byref(h)))
        self._h = h

    def launch(self, blocks: Sequence[DeviceBlock], stream=None) -> None:
        arr = _blocks_array(blocks)
        _check(load().ace_graph_launch(self._h, arr, len(blocks), _stream(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().ace_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------ serving
ACE_NONBLOCK = 0x1
ACE_STREAM_PLAIN = 0x1
ACE_STREAM_HOST_FAIL_LAUNCH = 0x100


class ace_stream_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "failed", "batches",
                                                "max_batch_requests", "pending",
                                                "arena_peak_bytes", "arena_capacity_bytes")]


HOST_VERIFY_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                  ctypes.c_void_p, ctypes.c_void_p)


def _stream_protos(lib):
    if getattr(lib, "_stream_protos", False):
        return
    vp, sz, u32, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint64
    lib.ace_stream_create.argtypes = [ctypes.POINTER(ace_keyset), vp, sz, sz, u32, u32,
                                      ctypes.POINTER(vp)]
    lib.ace_stream_create_host.argtypes = [HOST_VERIFY_FN, vp, sz, sz, u32, u32, u32,
                                           ctypes.POINTER(vp)]
    lib.ace_verify_stream.argtypes = [vp, vp, vp, vp, vp, u64, vp, vp, u32, ctypes.POINTER(u64)]
    lib.ace_stream_poll.argtypes = [vp, u64, ctypes.c_int]
    lib.ace_stream_ticket_times.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double)]
    lib.ace_stream_release.argtypes = [vp, u64]
    lib.ace_stream_get_stats.argtypes = [vp, ctypes.POINTER(ace_stream_stats)]
    lib.ace_stream_destroy.argtypes = [vp]
    lib._stream_protos = True


class Ticket:
    """One submitted request: its id and the host arrays its outputs land in."""

    def __init__(self, ticket: int, n: int, mask: np.ndarray, count: np.ndarray):
        self.id = ticket
        self.n = n
        self.mask = mask
        self.count = count


class Stream:
    """ace_stream_*: continuous-batching verification of requests from host memory."""

    def __init__(self, handle, keep=()):
        self._h = handle
        self._keep = list(keep)

    @classmethod
    def create(cls, keyset: DeviceKeyset, arena: torch.Tensor, staging_bytes: int,
               max_inflight: int = 4, plain: bool = False) -> "Stream":
        lib = load()
        _stream_protos(lib)
        ks, keep = keyset.struct()
        h = ctypes.c_void_p()
        _check(lib.ace_stream_create(ctypes.byref(ks), _ptr(arena, 0, "arena"), _nbytes(arena),
                                     staging_bytes,
                                     max_inflight, ACE_STREAM_PLAIN if plain else 0, ctypes.byref(h)))
        return cls(h, [keep, arena, keyset])

    @classmethod
    def create_host(cls, verify, arena_bytes: int, staging_bytes: int, max_inflight: int = 4,
                    plain: bool = False, fail_after: int = 0,
                    fail_at_launch: bool = False) -> "Stream":
        """Host backend for tests: verify(msg, off, ids, tags) -> (bitmask u32[], count).
        fail_after = k makes the k-th batch fail when it completes or, with
        fail_at_launch, in its launch call."""
        lib = load()
        _stream_protos(lib)

        def cb(user, msg, off, ids, tag, n, mask_out, count_out):
            try:
                n = int(n)
                o = np.ctypeslib.as_array(ctypes.cast(off, ctypes.POINTER(ctypes.c_uint64)),
                                          (n + 1,)).copy()
                span = int(o.max()) if n else 0
                m = (np.ctypeslib.as_array(ctypes.cast(msg, ctypes.POINTER(ctypes.c_uint8)),
                                           (span,)).copy() if span else np.zeros(0, np.uint8))
                i = (np.ctypeslib.as_array(ctypes.cast(ids, ctypes.POINTER(ctypes.c_uint32)),
                                           (n,)).copy() if n else np.zeros(0, np.uint32))
                t = (np.ctypeslib.as_array(ctypes.cast(tag, ctypes.POINTER(ctypes.c_uint8)),
                                           (n, 32)).copy() if n else np.zeros((0, 32), np.uint8))
                bm, c = verify(m, o, i, t)
                if n:
                    out = np.ctypeslib.as_array(ctypes.cast(mask_out, ctypes.POINTER(ctypes.c_uint32)),
                                                ((n + 31) // 32,))
                    out[:] = bm
                ctypes.cast(count_out, ctypes.POINTER(ctypes.c_uint64))[0] = int(c)
                return 0
            except Exception:  # reported to the engine as a device failure
                return -1

        fn = HOST_VERIFY_FN(cb)
        h = ctypes.c_void_p()
        flags = (ACE_STREAM_PLAIN if plain else 0) | (ACE_STREAM_HOST_FAIL_LAUNCH if fail_at_launch
                                                       else 0)
        _check(lib.ace_stream_create_host(fn, None, arena_bytes, staging_bytes, max_inflight, flags,
                                          fail_after, ctypes.byref(h)))
        return cls(h, [fn])

    def submit(self, msg: np.ndarray, off: np.ndarray, ids: np.ndarray, tags: np.ndarray,
               nonblock: bool = False) -> Ticket:
        n = int(ids.shape[0])
        msg = np.ascontiguousarray(msg, np.uint8)
        off = np.ascontiguousarray(off, np.uint64)
        ids = np.ascontiguousarray(ids, np.uint32)
        tags = np.ascontiguousarray(tags, np.uint8)
        mask = np.zeros(max(1, (n + 31) // 32), np.uint32)
        count = np.zeros(1, np.uint64)
        t = ctypes.c_uint64()
        _check(load().ace_verify_stream(self._h, msg.ctypes.data if msg.size else None,
                                        off.ctypes.data, ids.ctypes.data if n else None,
                                        tags.ctypes.data if n else None, n, mask.ctypes.data,
                                        count.ctypes.data, ACE_NONBLOCK if nonblock else 0,
                                        ctypes.byref(t)))
        return Ticket(t.value, n, mask, count)

    def poll(self, ticket: Ticket, wait: bool = True) -> bool:
        rc = load().ace_stream_poll(self._h, ticket.id, 1 if wait else 0)
        if rc == ACE_ERR_AGAIN:
            return False
        _check(rc)
        return True

    def result(self, ticket: Ticket) -> tuple[np.ndarray, int]:
        self.poll(ticket, True)
        return ticket.mask[: (ticket.n + 31) // 32].copy(), int(ticket.count[0])

    def times(self, ticket: Ticket) -> tuple[float, float, float]:
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        load().ace_stream_ticket_times(self._h, ticket.id, ctypes.byref(a), ctypes.byref(b),
                                       ctypes.byref(c))
        return a.value, b.value, c.value

    def release(self, ticket: Ticket) -> None:
        _check(load().ace_stream_release(self._h, ticket.id))

    def stats(self) -> dict:
        st = ace_stream_stats()
        _check(load().ace_stream_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ace_stream_stats._fields_}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(load().ace_stream_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
