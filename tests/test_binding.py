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
