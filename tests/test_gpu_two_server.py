"""Two-server PIR end to end, and the serving loop's key requests and
idle-window updates, checked against the oracle.

- Key requests: a server's answer to a DPF key is the oracle's scan of the
  oracle's evaluation of that key.
- Updates are barriers in a database's request order: requests submitted
  before an update are answered from the old records, requests after it
  from the new ones, whatever the timing.
- The demo module: a client with two servers reconstructs every record
  before and after an update.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pir = pytest.importorskip("paper_2509_06514_amd")
from paper_2509_06514_amd import _native  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pir.Context(0)
    yield c
    c.close()


def _roots(seed):
    b = synth.stream_bytes(seed, 32)
    return b[:16], b[16:]


def _oracle_answer(dbh, key, n_bits):
    n = dbh.shape[0]
    bits = np.unpackbits(oracle.dpf_eval_full(key, n_bits), bitorder="little")[:n]
    return oracle.dpxor(dbh, np.packbits(bits, bitorder="little"))


def test_key_requests_match_oracle_and_reconstruct(ctx):
    n, r = 20011, 64
    dbh = synth.database(n, r, seed=synth.S_DB + 70)
    db = ctx.load_db(dbh)
    nb = pir.dpf_domain_bits(n)
    srv = pir.Server(ctx, q_max=16, max_wait_us=300, n_slots=3)
    i0 = srv.add_db(db)
    rng = np.random.default_rng(3)
    alphas = [0, n - 1] + [int(a) for a in rng.integers(0, n, 10)]
    keys, outs, ts = [], [], []
    for k, a in enumerate(alphas):
        k0, k1 = pir.dpf_gen(a, nb, *_roots(synth.S_KEY + 700 + k))
        for key in (k0, k1):
            out = np.zeros(r, np.uint8)
            keys.append(key)
            outs.append(out)
            ts.append(srv.submit_key(i0, key, out))
    # selection requests in the same stream
    sel = synth.selections(n, 5, seed=synth.S_SEL + 70)
    souts = [np.zeros(r, np.uint8) for _ in range(5)]
    sts = [srv.submit(i0, sel[q], souts[q]) for q in range(5)]
    for t in ts + sts:
        assert srv.wait(t, 120000) == _native.PIR_OK
    for k, a in enumerate(alphas):
        assert np.array_equal(pir.reconstruct(outs[2 * k], outs[2 * k + 1]), dbh[a]), a
    for j in (0, 1, 7):
        assert np.array_equal(outs[j], _oracle_answer(dbh, keys[j], nb)), j
    for q in range(5):
        assert np.array_equal(souts[q], oracle.dpxor(dbh, sel[q]))
    st = srv.stats()
    assert st["key_requests"] == 2 * len(alphas) and st["completed"] == 2 * len(alphas) + 5
    srv.close()
    db.free()


@pytest.mark.parametrize("wait_us", [0, 20000])
def test_update_is_a_barrier(ctx, wait_us):
    n, r = 50003, 32
    old = synth.database(n, r, seed=synth.S_DB + 71)
    db = ctx.load_db(old)
    srv = pir.Server(ctx, q_max=8, max_wait_us=wait_us, n_slots=2)
    i0 = srv.add_db(db)
    first, count = 1234, 3000
    new_recs = synth.database(count, r, seed=synth.S_DB + 72)
    new = old.copy()
    new[first:first + count] = new_recs
    sel = synth.selections(n, 12, seed=synth.S_SEL + 71)
    nb = pir.dpf_domain_bits(n)
    k0, _ = pir.dpf_gen(first + 17, nb, *_roots(synth.S_KEY + 800))
    before = [np.zeros(r, np.uint8) for _ in range(13)]
    after = [np.zeros(r, np.uint8) for _ in range(13)]
    tb = [srv.submit(i0, sel[q], before[q]) for q in range(12)] + [srv.submit_key(i0, k0, before[12])]
    tu = srv.update(i0, first, new_recs)
    ta = [srv.submit(i0, sel[q], after[q]) for q in range(12)] + [srv.submit_key(i0, k0, after[12])]
    for t in tb + [tu] + ta:
        assert srv.wait(t, 120000) == _native.PIR_OK
    for q in range(12):
        assert np.array_equal(before[q], oracle.dpxor(old, sel[q])), ("before", q)
        assert np.array_equal(after[q], oracle.dpxor(new, sel[q])), ("after", q)
    assert np.array_equal(before[12], _oracle_answer(old, k0, nb))
    assert np.array_equal(after[12], _oracle_answer(new, k0, nb))
    assert np.array_equal(db.read(first, count), new_recs)
    assert srv.stats()["updates_applied"] == 1
    srv.close()
    db.free()


def test_update_rejects_bad_range(ctx):
    n, r = 1000, 16
    db = ctx.load_db(synth.database(n, r, seed=synth.S_DB + 73))
    srv = pir.Server(ctx, q_max=4)
    i0 = srv.add_db(db)
    with pytest.raises(pir.PirError) as e:
        srv.update(i0, 990, np.zeros((20, r), np.uint8))
    assert e.value.code == _native.PIR_E_INVAL
    with pytest.raises(pir.PirError) as e:
        srv.update(5, 0, np.zeros((1, r), np.uint8))
    assert e.value.code == _native.PIR_E_NOTFOUND
    srv.close()
    db.free()


def test_two_server_demo():
    from paper_2509_06514_amd import two_server

    res = two_server.run(n_records=100003, record_bytes=32, n_queries=24, update_count=500, seed=5)
    assert res["before_update_ok"] and res["after_update_ok"] and res["replicas_updated"]
    for st in res["server_stats"]:
        assert st["key_requests"] == 48 and st["updates_applied"] == 1
