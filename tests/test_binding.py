"""The Python binding checks what the library cannot: that device arguments
are contiguous device tensors of at least the size the call will touch, and
that a block's offsets match its transactions.  No GPU needed: host tensors
and inconsistent host arrays must be refused before any library call."""
import numpy as np
import pytest
import torch

from paper_2603_10242_amd import ace


@pytest.fixture(scope="module")
def lib():
    return ace.load()


def test_host_tensors_are_refused(lib):
    rev = torch.zeros((4, 32), dtype=torch.uint8)
    with pytest.raises(ValueError, match="device tensor"):
        ace.derive_keys(rev, b"salt", b"info", mid_out=torch.zeros((4, 16), dtype=torch.int32))
    with pytest.raises(ValueError, match="device tensor"):
        ace.poh_verify(torch.zeros((3, 32), dtype=torch.uint8), torch.zeros((3, 32), dtype=torch.uint8),
                       5, torch.zeros(1, dtype=torch.int32), torch.zeros(1, dtype=torch.int64))


def test_offsets_must_match_transactions(lib):
    msg = np.zeros(10, np.uint8)
    with pytest.raises(ValueError, match="entries"):
        ace.upload_block(msg, np.array([0, 5, 10], np.uint64), np.array([0], np.uint32),
                         np.zeros((1, 32), np.uint8))


def test_size_rule():
    ace._require_bytes(32, 32, "x")
    with pytest.raises(ValueError, match="32 bytes, 33 needed"):
        ace._require_bytes(32, 33, "x")


def test_block_descriptor_checked_once_and_rechecked_after_reassignment(lib, monkeypatch):
    """A block's C descriptor is validated once and reused by later calls
    (256-block calls marshal in a fraction of a millisecond); reassigning a
    field drops it, so an undersized replacement is refused again."""
    calls = []

    def counting_ptr(t, nbytes=0, what="tensor"):
        calls.append(what)
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_contiguous():
            raise ValueError("%s: a contiguous device tensor is required" % what)
        ace._require_bytes(t.numel() * t.element_size(), nbytes, what)
        return t.data_ptr()

    monkeypatch.setattr(ace, "_ptr", counting_ptr)   # host tensors stand in for device ones
    n = 100
    blk = ace.DeviceBlock(torch.zeros(10, dtype=torch.uint8), torch.zeros(n + 1, dtype=torch.int64),
                          torch.zeros(n, dtype=torch.int32), torch.zeros((n, 72), dtype=torch.uint8),
                          torch.zeros(4, dtype=torch.int32), torch.zeros(1, dtype=torch.int64), n)
    s = blk.struct()
    assert len(calls) == 6 and blk.struct() is s and len(calls) == 6
    assert blk.struct(72) is not s          # another record width is checked on its own
    arr = ace._blocks_array([blk, blk])
    assert arr[0].n_tx == n and arr[1].d_bitmask_out == s.d_bitmask_out
    blk.bitmask = torch.zeros(3, dtype=torch.int32)   # 96 bits for 100 transactions
    with pytest.raises(ValueError, match="bitmask"):
        blk.struct()
    blk.bitmask = torch.zeros(4, dtype=torch.int32)
    assert blk.struct().d_bitmask_out == blk.bitmask.data_ptr()
