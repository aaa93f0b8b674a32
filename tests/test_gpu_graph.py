"""Captured batches (ace_graph_*): one capture replayed for different block
mixes must give exactly what the eager call gives and what the generator's
truth mask and the CPU oracle say, replay after replay, with eager work in
between, under the library's default launch tuning and the saved autotuned
one."""
import sys

import numpy as np
import pytest

import oracle
from paper_2603_10242_amd import workload as W

from .conftest import TUNINGS, use_tuning

pytestmark = pytest.mark.gpu


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
def data():
    return W.subset(W.config2(), 0, 80_000)


@pytest.fixture(scope="module")
def okeys(data):
    return oracle.derive_keys(data.rev, data.salt, data.info, 8)


def cut(ace, w, edges, d_msg):
    return [ace.upload_block(None, w.off[a:b + 1], w.ids[a:b], w.tags[a:b], msg_dev=d_msg)
            for a, b in zip(edges[:-1], edges[1:])]


def mixes(n):
    r = np.random.Generator(np.random.PCG64(4))
    out = []
    # 256 uneven blocks over everything
    cuts = np.sort(r.choice(np.arange(1, n), size=255, replace=False))
    out.append(np.concatenate([[0], cuts, [n]]))
    # a few blocks, some empty, over a prefix
    out.append(np.array([0, 0, 10, 10, 4097, 30000, 30001, 30001]))
    # one block
    out.append(np.array([0, 65]))
    # 40 blocks of a different prefix
    cuts = np.sort(r.choice(np.arange(1, 50_000), size=39, replace=False))
    out.append(np.concatenate([[0], cuts, [50_000]]))
    return out


def check(blocks, edges, w, keys):
    """Every block's bitmask and count against the oracle's for its range and
    against the generator's truth mask."""
    for blk, a, b in zip(blocks, edges[:-1], edges[1:]):
        mask, count = blk.result()
        omask, ocount = oracle.verify_batch(keys, w.msg, w.off[a:b + 1], w.ids[a:b], w.tags[a:b], 8)
        assert count == ocount == int(w.truth[a:b].sum()), (a, b)
        assert np.array_equal(mask, omask), (a, b)
        assert np.array_equal(mask, W.pack_bits(w.truth[a:b])), (a, b)


@pytest.mark.parametrize("keys", ["midstate", "rev"])
@pytest.mark.parametrize("flags", [0, 0x1, 0x2 | 0x4])
def test_graph_replays_match_eager(ace, data, okeys, keys, flags):
    import torch
    note("graph keys=%s flags=%d" % (keys, flags))
    w = data
    rev = ace.to_device(w.rev)
    ks = ace.midstate_keyset(rev, w.salt, w.info) if keys == "midstate" else \
        ace.rev_keyset(rev, w.salt, w.info)
    d_msg = ace.to_device(w.msg)
    g = ace.Graph(ks, max_blocks=300, max_tx=w.n, flags=flags)
    try:
        plan = mixes(w.n)
        for rep, edges in enumerate(plan + plan[::-1]):
            blocks = cut(ace, w, edges, d_msg)
            g.launch(blocks)
            torch.cuda.synchronize()
            check(blocks, edges, w, okeys)
            # eager pass over the same blocks, plus unrelated torch work
            eager = cut(ace, w, edges, d_msg)
            ace.verify_batch(ks, eager, flags=flags)
            junk = torch.arange(1 << 20, device="cuda", dtype=torch.int64).sum()
            torch.cuda.synchronize()
            assert int(junk.item()) == (1 << 20) * ((1 << 20) - 1) // 2
            for gb, eb in zip(blocks, eager):
                gm, gc = gb.result()
                em, ec = eb.result()
                assert gc == ec and np.array_equal(gm, em), rep
    finally:
        g.close()


@pytest.mark.parametrize("flags", [0, 0x1, 0x2 | 0x4])
def test_graph_back_to_back_replays(ace, data, okeys, flags):
    """Replays queued without a host sync in between (both pinned block lists in use)."""
    import torch
    note("graph back to back flags=%d" % flags)
    w = data
    ks = ace.midstate_keyset(ace.to_device(w.rev), w.salt, w.info)
    d_msg = ace.to_device(w.msg)
    g = ace.Graph(ks, max_blocks=300, max_tx=w.n, flags=flags)
    try:
        plan = mixes(w.n)
        sets = [cut(ace, w, e, d_msg) for e in plan]
        for blocks in sets:
            g.launch(blocks)
        torch.cuda.synchronize()
        for blocks, edges in zip(sets, plan):
            check(blocks, edges, w, okeys)
    finally:
        g.close()


def test_graph_rejects_oversize(ace, data):
    w = data
    ks = ace.midstate_keyset(ace.to_device(w.rev), w.salt, w.info)
    d_msg = ace.to_device(w.msg)
    g = ace.Graph(ks, max_blocks=4, max_tx=1000)
    try:
        with pytest.raises(ace.AceError):
            g.launch(cut(ace, w, np.array([0, 1, 2, 3, 4, 5]), d_msg))   # 5 blocks > 4
        with pytest.raises(ace.AceError):
            g.launch(cut(ace, w, np.array([0, 1001]), d_msg))            # 1001 txs > 1000
    finally:
        g.close()
