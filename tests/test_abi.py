"""Host-only checks of libace.so: it loads, exports every entry point that
include/ace.h declares, rejects malformed calls before touching the GPU, and
its SHA-256 constant table equals the FIPS 180-4 closed form."""
import ctypes
import os
import re

import numpy as np
import pytest

from tests.test_oracle_pins import closed_form_constants

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ace.h")
DEVICE_SHA = os.path.join(ROOT, "paper_2603_10242_amd", "csrc", "sha256_gfx950.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"ACE_API\s+[^;(]*?\b(ace_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2603_10242_amd import ace
    return ace.load()


def test_header_declares_entry_points():
    syms = declared_symbols()
    for name in ("ace_derive_keys", "ace_verify_batch", "ace_verify_workspace_size",
                 "ace_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_device_constants_equal_closed_form():
    text = open(DEVICE_SHA).read()
    body = text[text.index("kRound[64]"):]
    k = [int(x, 16) for x in re.findall(r"0x([0-9a-f]{8})u", body[: body.index("};")])]
    body = text[text.index("kInit[8]"):]
    iv = [int(x, 16) for x in re.findall(r"0x([0-9a-f]{8})u", body[: body.index("};")])]
    K, IV = closed_form_constants()
    assert k == list(map(int, K)) and iv == list(map(int, IV))


def _keyset(ace, kind=0, n_id=4, mid=0x1000, rev=0, salt=b"", info=b""):
    sb = ctypes.create_string_buffer(salt or b"\0")
    ib = ctypes.create_string_buffer(info or b"\0")
    ks = ace.ace_keyset(kind, mid or None, rev or None, n_id, ctypes.addressof(sb), len(salt),
                        ctypes.addressof(ib), len(info))
    return ks, (sb, ib)


def _block(ace, n=100, **kw):
    f = dict(d_msg=0x10000, d_off=0x20000, d_id=0x30000, d_tag=0x40000, n_tx=n,
             d_bitmask_out=0x50000, d_count_out=0x60000)
    f.update(kw)
    return ace.ace_block(*[f[k] for k, _ in ace.ace_block._fields_])


def test_argument_errors_are_reported_before_any_launch(lib):
    from paper_2603_10242_amd import ace
    ks, keep = _keyset(ace)
    blk = (ace.ace_block * 1)(_block(ace))
    # no workspace
    assert lib.ace_verify_batch(ctypes.byref(ks), blk, 1, None, 0, 0, None) == ace.ACE_ERR_INVALID_ARG
    assert b"workspace" in lib.ace_last_error()
    # workspace too small
    need = lib.ace_verify_workspace_size(ctypes.byref(ks), blk, 1, 0)
    assert need > 0
    assert lib.ace_verify_batch(ctypes.byref(ks), blk, 1, 0x100000, need - 256, 0,
                                None) == ace.ACE_ERR_NO_MEMORY
    # misaligned workspace
    assert lib.ace_verify_batch(ctypes.byref(ks), blk, 1, 0x100010, need, 0,
                                None) == ace.ACE_ERR_INVALID_ARG
    # exclusive flags, unknown flags
    assert lib.ace_verify_batch(ctypes.byref(ks), blk, 1, 0x100000, need,
                                ace.ACE_ORDERED | ace.ACE_BUCKETED, None) == ace.ACE_ERR_INVALID_ARG
    assert lib.ace_verify_batch(ctypes.byref(ks), blk, 1, 0x100000, need, 0x100,
                                None) == ace.ACE_ERR_INVALID_ARG
    # per-transaction keys need root entropy
    assert lib.ace_verify_batch(ctypes.byref(ks), blk, 1, 0x100000, need, ace.ACE_PER_TX_KEYS,
                                None) == ace.ACE_ERR_INVALID_ARG
    # NULL arrays, misaligned arrays, NULL count
    for bad in (dict(d_off=0), dict(d_tag=0), dict(d_id=0x30001), dict(d_count_out=0),
                dict(d_off=0x20004)):
        b = (ace.ace_block * 1)(_block(ace, **bad))
        assert lib.ace_verify_batch(ctypes.byref(ks), b, 1, 0x100000, need, 0,
                                    None) == ace.ACE_ERR_INVALID_ARG, bad
    # too many transactions
    b = (ace.ace_block * 2)(_block(ace, n=1 << 31), _block(ace, n=1 << 31))
    assert lib.ace_verify_batch(ctypes.byref(ks), b, 2, 0x100000, need, 0,
                                None) == ace.ACE_ERR_RANGE
    # unknown keyset kind, missing keyset pointers
    ks2, k2 = _keyset(ace, kind=7)
    assert lib.ace_verify_batch(ctypes.byref(ks2), blk, 1, 0x100000, need, 0,
                                None) == ace.ACE_ERR_INVALID_ARG
    ks3, k3 = _keyset(ace, kind=1, rev=0)
    assert lib.ace_verify_batch(ctypes.byref(ks3), blk, 1, 0x100000, need, 0,
                                None) == ace.ACE_ERR_INVALID_ARG
    ks4, k4 = _keyset(ace, kind=1, rev=0x7000, salt=b"x" * 1025)
    assert lib.ace_verify_batch(ctypes.byref(ks4), blk, 1, 0x100000, need, 0,
                                None) == ace.ACE_ERR_INVALID_ARG


def test_noalloc_refuses_calls_beyond_its_scratch_array(lib):
    """ace_verify_batch_noalloc checks its arguments like ace_verify_batch and
    refuses a call whose workspace exceeds the static scratch array, before
    touching the GPU; the binding's constant is the header's."""
    from paper_2603_10242_amd import ace
    text = open(HEADER).read()
    m = re.search(r"#define ACE_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == ace.ACE_SCRATCH_BYTES
    ks, keep = _keyset(ace)
    blk = (ace.ace_block * 1)(_block(ace, n=3_000_000))
    assert lib.ace_verify_workspace_size(ctypes.byref(ks), blk, 1, ace.ACE_BUCKETED) > \
        ace.ACE_SCRATCH_BYTES
    assert lib.ace_verify_batch_noalloc(ctypes.byref(ks), blk, 1, ace.ACE_BUCKETED,
                                        None) == ace.ACE_ERR_TOO_LARGE
    assert b"scratch" in lib.ace_last_error()
    # keys derived in the call: 64 bytes per identity on top
    ks2, k2 = _keyset(ace, kind=1, rev=0x7000, n_id=1 << 20)
    small = (ace.ace_block * 1)(_block(ace, n=1000))
    assert lib.ace_verify_batch_noalloc(ctypes.byref(ks2), small, 1, ace.ACE_ORDERED,
                                        None) == ace.ACE_ERR_TOO_LARGE
    # the same argument errors as the workspace form
    assert lib.ace_verify_batch_noalloc(ctypes.byref(ks), small, 1, ace.ACE_ORDERED | ace.ACE_BUCKETED,
                                        None) == ace.ACE_ERR_INVALID_ARG
    bad = (ace.ace_block * 1)(_block(ace, n=1000, d_tag=0))
    assert lib.ace_verify_batch_noalloc(ctypes.byref(ks), bad, 1, 0, None) == ace.ACE_ERR_INVALID_ARG
    assert lib.ace_verify_batch_noalloc(None, small, 1, 0, None) == ace.ACE_ERR_INVALID_ARG
    # nothing to do
    assert lib.ace_verify_batch_noalloc(ctypes.byref(ks), small, 0, 0, None) == ace.ACE_OK


def test_tuning_grab_caps_round_trip_and_limits(lib):
    """The per-bucket grab caps of ace_tuning: set and read back, values above
    8 refused with the rest of the tuning left as it was."""
    from paper_2603_10242_amd import ace
    old = ace.get_tuning()
    try:
        caps = [b % 9 for b in range(ace.ACE_LENGTH_BUCKETS)]
        ace.set_tuning(grab_cap=caps, verify_wgs_per_cu=3)
        t = ace.get_tuning()
        assert t["grab_cap"] == caps and t["verify_wgs_per_cu"] == 3
        with pytest.raises(ace.AceError):
            ace.set_tuning(grab_cap=[0] * 63 + [9], verify_wgs_per_cu=5)
        assert ace.get_tuning() == t
        with pytest.raises(ValueError):
            ace.set_tuning(grab_cap=[1] * 10)
    finally:
        ace.set_tuning(**old)


def test_derive_argument_errors(lib):
    from paper_2603_10242_amd import ace
    salt = ctypes.create_string_buffer(b"s" * 32)
    info = ctypes.create_string_buffer(b"i" * 300)
    # both outputs NULL
    assert lib.ace_derive_keys(0x1000, 4, salt, 32, info, 16, None, None, None) == ace.ACE_ERR_INVALID_ARG
    # info too long, salt too long
    assert lib.ace_derive_keys(0x1000, 4, salt, 32, info, 256, 0x2000, None, None) == ace.ACE_ERR_INVALID_ARG
    assert lib.ace_derive_keys(0x1000, 4, salt, 1025, info, 16, 0x2000, None, None) == ace.ACE_ERR_INVALID_ARG
    # NULL root entropy
    assert lib.ace_derive_keys(None, 4, salt, 32, info, 16, 0x2000, None, None) == ace.ACE_ERR_INVALID_ARG
    # zero identities is a no-op that never launches
    assert lib.ace_derive_keys(None, 0, salt, 32, info, 16, 0x2000, None, None) == ace.ACE_OK


def test_derive_multi_argument_errors(lib):
    from paper_2603_10242_amd import ace
    salt = ctypes.create_string_buffer(b"s" * 80)
    info = ctypes.create_string_buffer(b"i" * 80)
    arr = (ace.ace_hkdf_stream * 2)()
    arr[0] = ace.ace_hkdf_stream(ctypes.addressof(salt), 32, ctypes.addressof(info), 23)
    arr[1] = ace.ace_hkdf_stream(ctypes.addressof(salt), 65, ctypes.addressof(info), 23)
    # second stream's salt too long: nothing launched for the first either
    assert lib.ace_derive_keys_multi(0x1000, 4, arr, 2, 0x2000, None, None) == ace.ACE_ERR_INVALID_ARG
    arr[1] = ace.ace_hkdf_stream(ctypes.addressof(salt), 8, ctypes.addressof(info), 65)
    assert lib.ace_derive_keys_multi(0x1000, 4, arr, 2, 0x2000, None, None) == ace.ACE_ERR_INVALID_ARG
    arr[1] = ace.ace_hkdf_stream(None, 8, ctypes.addressof(info), 8)
    assert lib.ace_derive_keys_multi(0x1000, 4, arr, 2, 0x2000, None, None) == ace.ACE_ERR_INVALID_ARG
    arr[1] = ace.ace_hkdf_stream(ctypes.addressof(salt), 64, ctypes.addressof(info), 64)
    assert lib.ace_derive_keys_multi(0x1000, 4, arr, 2, None, None, None) == ace.ACE_ERR_INVALID_ARG
    assert lib.ace_derive_keys_multi(0x1000, 4, None, 2, 0x2000, None, None) == ace.ACE_ERR_INVALID_ARG
    assert lib.ace_derive_keys_multi(None, 4, arr, 2, 0x2000, None, None) == ace.ACE_ERR_INVALID_ARG
    # nothing to do: no launch
    assert lib.ace_derive_keys_multi(None, 0, arr, 2, 0x2000, None, None) == ace.ACE_OK
    assert lib.ace_derive_keys_multi(None, 4, arr, 0, 0x2000, None, None) == ace.ACE_OK


def test_poh_argument_errors(lib):
    from paper_2603_10242_amd import ace
    E = ace.ACE_ERR_INVALID_ARG
    assert lib.ace_poh_verify(0x1000, 0x2000, None, 5, 10, 0x3000, None, None) == E
    assert lib.ace_poh_verify(0x1000, 0x2000, None, 5, 10, 0x3000, 0x4004, None) == E
    assert lib.ace_poh_verify(None, 0x2000, None, 5, 10, 0x3000, 0x4000, None) == E
    assert lib.ace_poh_verify(0x1000, None, None, 5, 10, 0x3000, 0x4000, None) == E
    assert lib.ace_poh_verify(0x1000, 0x2000, None, 5, 10, None, 0x4000, None) == E
    assert lib.ace_poh_verify(0x1001, 0x2000, None, 5, 10, 0x3000, 0x4000, None) == E
    assert lib.ace_poh_verify(0x1000, 0x2000, 0x5002, 5, 10, 0x3000, 0x4000, None) == E
    assert lib.ace_poh_verify(0x1000, 0x2000, None, 5, 2**33, 0x3000, 0x4000,
                              None) == ace.ACE_ERR_RANGE


def test_merkle_argument_errors_and_workspace(lib):
    from paper_2603_10242_amd import ace
    E = ace.ACE_ERR_INVALID_ARG
    arr = (ace.ace_merkle_tree * 3)()
    arr[0] = ace.ace_merkle_tree(0x1000, 0x2000, 10, 0x3000)
    arr[1] = ace.ace_merkle_tree(None, None, 0, 0x3020)
    arr[2] = ace.ace_merkle_tree(0x1000, 0x2000, 1000, 0x3040)
    # 32 bytes per leaf, the descriptor table and per-level prefixes (10 levels)
    need = lib.ace_merkle_workspace_size(arr, 3)
    assert need >= 32 * 1010 + 40 * 3 + 8 * 10 * 4 and need % 256 == 0
    assert lib.ace_merkle_roots(arr, 3, None, 0, None) == E
    assert lib.ace_merkle_roots(arr, 3, 0x100000, need - 1, None) == ace.ACE_ERR_NO_MEMORY
    assert lib.ace_merkle_roots(arr, 3, 0x100010, need, None) == E          # misaligned workspace
    arr[1] = ace.ace_merkle_tree(None, None, 0, None)                         # no root output
    assert lib.ace_merkle_roots(arr, 3, 0x100000, need, None) == E
    arr[1] = ace.ace_merkle_tree(None, None, 0, 0x3022)                       # misaligned root
    assert lib.ace_merkle_roots(arr, 3, 0x100000, need, None) == E
    arr[1] = ace.ace_merkle_tree(None, 0x2000, 5, 0x3020)                     # NULL data
    assert lib.ace_merkle_roots(arr, 3, 0x100000, need, None) == E
    arr[1] = ace.ace_merkle_tree(0x1000, 0x2004, 5, 0x3020)                   # misaligned offsets
    assert lib.ace_merkle_roots(arr, 3, 0x100000, need, None) == E
    assert lib.ace_merkle_workspace_size(None, 2) == 0
    assert lib.ace_merkle_roots(arr, 0, None, 0, None) == ace.ACE_OK           # nothing to do


def test_workspace_size_layout(lib):
    from paper_2603_10242_amd import ace
    ks, keep = _keyset(ace)
    one = (ace.ace_block * 1)(_block(ace, n=1_000_000))
    ordered = lib.ace_verify_workspace_size(ctypes.byref(ks), one, 1, ace.ACE_ORDERED)
    binned = lib.ace_verify_workspace_size(ctypes.byref(ks), one, 1, ace.ACE_BUCKETED)
    # ordered: the control words only (per-bin counters in 32 copies)
    assert 0 < ordered < 20 * 1024
    # binned: 8 B permutation + 16 B record + 4 B position + 1 bit per transaction,
    # plus 64 bins of padding
    assert binned >= ordered + 28 * 1_000_000
    assert binned < ordered + 29 * 1_000_000 + 128 * 1024
    rks, rkeep = _keyset(ace, kind=1, rev=0x7000, n_id=1000)
    with_mid = lib.ace_verify_workspace_size(ctypes.byref(rks), one, 1, ace.ACE_ORDERED)
    assert with_mid >= ordered + 64 * 1000
    assert lib.ace_verify_workspace_size(None, one, 1, 0) == 0


def test_tuning_roundtrip_and_limits(lib):
    from paper_2603_10242_amd import ace
    old = ace.get_tuning()
    assert old["verify_wgs_per_cu"] >= 1 and old["binned_min_tx"] > 0
    try:
        ace.set_tuning(verify_wgs_per_cu=4, binned_min_tx=1000)
        t = ace.get_tuning()
        assert t["verify_wgs_per_cu"] == 4 and t["binned_min_tx"] == 1000
        with pytest.raises(ace.AceError):
            ace.set_tuning(verify_wgs_per_cu=0)
        with pytest.raises(ace.AceError):
            ace.set_tuning(aux_wgs_per_cu=65)
        ace.set_tuning(derive_wgs_per_cu=0)          # 0: the library's own grid
        assert ace.get_tuning()["derive_wgs_per_cu"] == 0
        with pytest.raises(ace.AceError):
            ace.set_tuning(derive_wgs_per_cu=65)
        assert old["wide_min_len"] == 2**31 - 1     # only messages the record cannot hold
        ace.set_tuning(wide_min_len=1)
        assert ace.get_tuning()["wide_min_len"] == 1
        for bad in (0, 2**31, 2**40):
            with pytest.raises(ace.AceError):
                ace.set_tuning(wide_min_len=bad)
    finally:
        ace.set_tuning(**old)
    assert ace.get_tuning() == old


def test_graph_argument_errors(lib):
    from paper_2603_10242_amd import ace
    ks, keep = _keyset(ace)
    out = ctypes.c_void_p()
    assert lib.ace_graph_workspace_size(ctypes.byref(ks), 0, 1000, 0) == 0
    need = lib.ace_graph_workspace_size(ctypes.byref(ks), 16, 1 << 20, 0)
    assert need > 28 * (1 << 20)
    assert lib.ace_graph_create(ctypes.byref(ks), 16, 1 << 20, 0x100000, need - 256, 0,
                                ctypes.byref(out)) == ace.ACE_ERR_NO_MEMORY
    assert lib.ace_graph_create(ctypes.byref(ks), 0, 1 << 20, 0x100000, need, 0,
                                ctypes.byref(out)) == ace.ACE_ERR_INVALID_ARG
    assert lib.ace_graph_create(ctypes.byref(ks), 16, 1 << 20, 0x100008, need, 0,
                                ctypes.byref(out)) == ace.ACE_ERR_INVALID_ARG
    assert lib.ace_graph_launch(None, None, 0, None) == ace.ACE_ERR_INVALID_ARG
    assert lib.ace_graph_destroy(None) == ace.ACE_OK


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc absent")
def test_valu_probe_loop_is_192_valu_instructions(tmp_path):
    """The VALU-rate probe prices its launch at 192 lane instructions per loop
    iteration: the compiled loop body must hold exactly those."""
    import subprocess
    src = tmp_path / "probe.hip"
    src.write_text('#include "%s"\nvoid launch(uint32_t *s) { hipLaunchKernelGGL(ace::k_valu_rate, '
                   'dim3(1), dim3(256), 0, 0, 10u, 1u, s); }\n'
                   % os.path.join(ROOT, "paper_2603_10242_amd", "csrc", "valu_rate.hip"))
    asm = tmp_path / "probe.s"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "--cuda-device-only", "-S", "-o", str(asm), str(src)],
                          stderr=subprocess.DEVNULL)
    lines = asm.read_text().splitlines()
    head = next(i for i, l in enumerate(lines) if "Inner Loop Header" in l)
    tail = next(i for i in range(head, len(lines)) if "s_cbranch" in lines[i])
    ops = [l.split()[0] for l in lines[head + 1:tail] if l.strip().startswith("v_")]
    assert len(ops) == 192
    assert sorted(set(ops)) == ["v_add3_u32", "v_alignbit_b32", "v_bitop3_b32"]
