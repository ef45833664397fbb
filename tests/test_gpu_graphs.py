"""The scan replayed from captured hipGraphs: every replay is checked against
the oracle and against the eager path (graphs off, and timing on, which also
enqueues the launches one by one), with eager device work and
synchronisations between replays; graphs follow record updates, do not
outlive their database, and the cache's eviction keeps answers exact.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pir = pytest.importorskip("paper_2509_06514_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pir.Context(0)
    yield c
    c.graphs(True)
    c.close()


def _sel_rows(n, q, seed, stride):
    return synth.selections(n, q, seed=seed, stride=stride)


def test_replays_match_oracle_and_eager(ctx):
    n, r, q = 100003, 32, 5
    dbh = synth.database(n, r, seed=synth.S_DB + 80)
    db = ctx.load_db(dbh)
    stride = pir.sel_stride_for(n)
    d_sel = torch.zeros((q, stride), dtype=torch.uint8, device="cuda:0")
    d_out = torch.zeros((q, r), dtype=torch.uint8, device="cuda:0")
    d_eager = torch.zeros((q, r), dtype=torch.uint8, device="cuda:0")
    for rnd in range(6):
        sel = _sel_rows(n, q, synth.S_SEL + 80 + rnd, stride)
        d_sel.copy_(torch.from_numpy(sel))            # eager work between replays
        d_out.fill_(0xEE)
        ctx.graphs(True)
        db.dpxor_batch_async(d_sel, q, d_out)          # the same graph every round
        torch.cuda.synchronize()
        got = d_out.cpu().numpy()
        for i in range(q):
            assert np.array_equal(got[i], oracle.dpxor(dbh, sel[i])), (rnd, i)
        if rnd % 2 == 0:
            ctx.graphs(False)
        else:
            ctx.timing(True)
        d_eager.fill_(0x11)
        db.dpxor_batch_async(d_sel, q, d_eager)
        torch.cuda.synchronize()
        ctx.timing(False)
        ctx.graphs(True)
        assert np.array_equal(d_eager.cpu().numpy(), got), rnd
    db.free()


def test_graphs_follow_updates_and_reloads(ctx):
    n, r, q = 20000, 16, 3
    dbh = synth.database(n, r, seed=synth.S_DB + 81)
    db = ctx.load_db(dbh)
    stride = pir.sel_stride_for(n)
    sel = _sel_rows(n, q, synth.S_SEL + 81, stride)
    d_sel = torch.from_numpy(sel).to("cuda:0")
    d_out = torch.zeros((q, r), dtype=torch.uint8, device="cuda:0")
    db.dpxor_batch_async(d_sel, q, d_out)
    torch.cuda.synchronize()
    new = synth.database(500, r, seed=synth.S_DB + 82)
    db.update(1000, new)
    dbh2 = dbh.copy()
    dbh2[1000:1500] = new
    db.dpxor_batch_async(d_sel, q, d_out)               # replay after the update
    torch.cuda.synchronize()
    for i in range(q):
        assert np.array_equal(d_out[i].cpu().numpy(), oracle.dpxor(dbh2, sel[i])), i
    db.free()
    # a new database of the same shape must not meet the old one's graphs
    dbh3 = synth.database(n, r, seed=synth.S_DB + 83)
    db3 = ctx.load_db(dbh3)
    db3.dpxor_batch_async(d_sel, q, d_out)
    torch.cuda.synchronize()
    for i in range(q):
        assert np.array_equal(d_out[i].cpu().numpy(), oracle.dpxor(dbh3, sel[i])), i
    db3.free()


def test_eviction_keeps_answers_exact(ctx):
    # 300 distinct output pointers: more graphs than the cache holds
    n, r = 5000, 8
    dbh = synth.database(n, r, seed=synth.S_DB + 84)
    db = ctx.load_db(dbh)
    stride = pir.sel_stride_for(n)
    sel = _sel_rows(n, 1, synth.S_SEL + 84, stride)
    want = oracle.dpxor(dbh, sel[0])
    d_sel = torch.from_numpy(sel).to("cuda:0")
    big = torch.zeros((300, 256), dtype=torch.uint8, device="cuda:0")
    for k in range(300):
        db.dpxor_batch_async(d_sel, 1, big[k])
    torch.cuda.synchronize()
    out = big.cpu().numpy()
    for k in range(300):
        assert np.array_equal(out[k][:r], want), k
    # and replays of evicted-then-recaptured keys
    big.zero_()
    for k in (0, 1, 299):
        db.dpxor_batch_async(d_sel, 1, big[k])
    torch.cuda.synchronize()
    for k in (0, 1, 299):
        assert np.array_equal(big[k].cpu().numpy()[:r], want), k
    db.free()
