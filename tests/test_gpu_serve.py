"""Continuous-batching server: every answer in a concurrent mixed load is the
answer of that query alone (exact bytes), batches overlap on the device, and
the failure paths (admission, unknown database, full queue, timeout, shutdown
with requests in flight) report their codes."""
import threading

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


@pytest.fixture(scope="module")
def three_dbs(ctx):
    # three resident databases of different record sizes and ragged N
    shapes = [(100003, 32), (40001, 128), (9001, 1024)]
    hosts, dbs = [], []
    for k, (n, r) in enumerate(shapes):
        h = synth.database(n, r, seed=0x5E00 + k)
        hosts.append(h)
        dbs.append(ctx.load_db(h))
    yield hosts, dbs
    for d in dbs:
        d.free()


def test_mixed_concurrent_load_matches_alone(ctx, three_dbs):
    hosts, dbs = three_dbs
    srv = pir.Server(ctx, q_max=64, max_wait_us=200, n_slots=4)
    ids = [srv.add_db(d) for d in dbs]
    n_req = 600
    which = [synth.word(0x77, k) % 3 for k in range(n_req)]
    sels = [synth.selections(hosts[w].shape[0], 1, seed=0x9000 + k)[0] for k, w in enumerate(which)]
    outs = [np.zeros(hosts[w].shape[1], np.uint8) for w in which]
    tickets = [None] * n_req

    def client(lo, hi):
        for k in range(lo, hi):
            tickets[k] = srv.submit(ids[which[k]], sels[k], outs[k])

    threads = [threading.Thread(target=client, args=(i * 150, (i + 1) * 150)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for k in range(n_req):
        assert srv.wait(tickets[k], 60000) == _native.PIR_OK, k
    st = srv.stats()
    srv.close()
    for k, w in enumerate(which):
        alone = oracle.dpxor(hosts[w], sels[k])
        assert np.array_equal(outs[k], alone), k
        if k % 50 == 0:  # the library's own single-query path gives the same bytes
            assert np.array_equal(dbs[w].dpxor(sels[k]), alone)
    assert st["completed"] == n_req and st["submitted"] == n_req
    assert st["batches"] < n_req, "requests were coalesced into batches"
    assert st["max_inflight"] >= 2, "batches overlapped on the device"
    assert st["p99_us"] >= st["p50_us"] > 0


def test_admission_by_memory_budget(ctx, three_dbs):
    hosts, dbs = three_dbs
    # room for the first database and its slot buffers, not for the 9 MiB third one
    budget = dbs[0].device_bytes + (8 << 20)
    assert dbs[2].device_bytes > (8 << 20)
    srv = pir.Server(ctx, hbm_budget_bytes=budget, q_max=16, n_slots=2)
    srv.add_db(dbs[0])
    with pytest.raises(pir.PirError) as e:
        srv.add_db(dbs[2])
    assert e.value.code == _native.PIR_E_NOMEM
    # the admitted database still serves
    n, r = hosts[0].shape
    sel = synth.selections(n, 1, seed=0xADD)[0]
    out = np.zeros(r, np.uint8)
    assert srv.wait(srv.submit(0, sel, out), 60000) == _native.PIR_OK
    assert np.array_equal(out, oracle.dpxor(hosts[0], sel))
    srv.close()


def test_unknown_db_busy_and_timeout(ctx, three_dbs):
    hosts, dbs = three_dbs
    srv = pir.Server(ctx, q_max=64, max_wait_us=2_000_000, n_slots=2, queue_cap=4)
    i = srv.add_db(dbs[1])
    n, r = hosts[1].shape
    sel = synth.selections(n, 5, seed=0xAB)
    outs = [np.zeros(r, np.uint8) for _ in range(5)]
    rc, _ = srv.submit_raw(7, sel[0].ctypes.data, outs[0].ctypes.data)
    assert rc == _native.PIR_E_NOTFOUND
    tickets = [srv.submit(i, sel[k], outs[k]) for k in range(4)]
    rc, _ = srv.submit_raw(i, sel[4].ctypes.data, outs[4].ctypes.data)
    assert rc == _native.PIR_E_BUSY           # queue_cap = 4
    assert srv.wait(tickets[0], 10) == _native.PIR_E_TIMEOUT  # held for company (max_wait 2 s)
    for k in range(4):
        assert srv.wait(tickets[k], 60000) == _native.PIR_OK
        assert np.array_equal(outs[k], oracle.dpxor(hosts[1], sel[k]))
    assert srv.wait(tickets[0], 0) == _native.PIR_E_NOTFOUND  # already collected
    st = srv.stats()
    assert st["rejected"] == 1
    srv.close()


def test_shutdown_drains_in_flight_requests(ctx, three_dbs):
    hosts, dbs = three_dbs
    srv = pir.Server(ctx, q_max=32, max_wait_us=1000, n_slots=3)
    ids = [srv.add_db(d) for d in dbs]
    reqs = []
    for k in range(120):
        w = k % 3
        s = synth.selections(hosts[w].shape[0], 1, seed=0xD000 + k)[0]
        o = np.zeros(hosts[w].shape[1], np.uint8)
        srv.submit(ids[w], s, o)
        reqs.append((w, s, o))
    srv.close()  # stops accepting, finishes everything queued or running
    for w, s, o in reqs:
        assert np.array_equal(o, oracle.dpxor(hosts[w], s))


def test_poll_interface(ctx, three_dbs):
    hosts, dbs = three_dbs
    srv = pir.Server(ctx, q_max=8, n_slots=1)
    i = srv.add_db(dbs[0])
    n, r = hosts[0].shape
    sel = synth.selections(n, 1, seed=0xF00)[0]
    out = np.zeros(r, np.uint8)
    t = srv.submit(i, sel, out)
    import time
    for _ in range(20000):
        done, st = srv.poll(t)
        if done:
            break
        time.sleep(0.0005)
    assert done and st == _native.PIR_OK
    assert np.array_equal(out, oracle.dpxor(hosts[0], sel))
    srv.close()


# The serving configuration at its stated sizes: three resident databases of
# 2^23 x 32 B, 2^24 x 128 B and 2^22 x 1024 B (0.25, 2 and 4 GiB).
C5_SHAPES = [(1 << 23, 32), (1 << 24, 128), (1 << 22, 1024)]
C5_POOL = 64  # distinct selection vectors per database


@pytest.fixture(scope="module")
def c5(ctx):
    hosts, dbs, pools, wants = [], [], [], []
    for k, (n, r) in enumerate(C5_SHAPES):
        h = synth.database(n, r, seed=synth.S_DB + 5 + k)
        hosts.append(h)
        dbs.append(ctx.load_db(h))
        pool = synth.selections(n, C5_POOL, seed=synth.S_SEL + 60 + k)
        pools.append(pool)
        wants.append(oracle.dpxor_rows(h, pool))  # every pool row, answered alone by the oracle
    yield hosts, dbs, pools, wants
    for d in dbs:
        d.free()


def test_c5_poisson_mix_matches_oracle(ctx, c5):
    # Open-loop Poisson arrivals (8k q/s offered from 4 threads), each request
    # to a database drawn uniformly: every answer in the mix equals the
    # oracle's answer to that selection alone, batches form and overlap, and
    # no request is turned away.
    import time

    hosts, dbs, pools, wants = c5
    srv = pir.Server(ctx, q_max=64, max_wait_us=200, n_slots=4, queue_cap=1 << 20)
    ids = [srv.add_db(d) for d in dbs]
    rate, seconds, n_thr = 8000.0, 0.6, 4
    records = [[] for _ in range(n_thr)]  # (ticket, db, pool row, out)

    def submitter(tid):
        rng = np.random.default_rng(0xC5 + tid)
        t = time.perf_counter()
        stop = t + seconds
        while True:
            t += rng.exponential(n_thr / rate)
            if t > stop:
                break
            dt = t - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            w = int(rng.integers(0, 3))
            k = int(rng.integers(0, C5_POOL))
            out = np.zeros(C5_SHAPES[w][1], np.uint8)
            rc, tk = srv.submit_raw(ids[w], pools[w][k].ctypes.data, out.ctypes.data)
            records[tid].append((rc, tk, w, k, out))

    ths = [threading.Thread(target=submitter, args=(i,)) for i in range(n_thr)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    done = [r for lst in records for r in lst]
    assert all(rc == _native.PIR_OK for rc, *_ in done), "a submit was refused"
    for rc, tk, w, k, out in done:
        assert srv.wait(tk, 60000) == _native.PIR_OK
    st = srv.stats()
    srv.close()
    bad = [(w, k) for rc, tk, w, k, out in done if not np.array_equal(out, wants[w][k])]
    assert not bad, f"{len(bad)} of {len(done)} answers differ from the oracle, first {bad[:5]}"
    assert len(done) > 2000
    assert st["completed"] == len(done) and st["rejected"] == 0
    assert st["batches"] < len(done), "requests were coalesced into batches"
    assert st["max_inflight"] >= 2, "batches overlapped on the device"


def test_full_ring_blocks_instead_of_rejecting(ctx, c5):
    # One slot, single-request batches and the smallest ring ((n_slots + 1) *
    # q_max = 2 rows) on the 4 GiB database: submits wait for a batch to retire
    # instead of failing, and every answer is exact.
    hosts, dbs, pools, wants = c5
    srv = pir.Server(ctx, q_max=1, max_wait_us=0, n_slots=1, queue_cap=1000, ring_bytes=1)
    i = srv.add_db(dbs[2])
    outs = [np.zeros(C5_SHAPES[2][1], np.uint8) for _ in range(24)]
    tickets = [srv.submit(i, pools[2][k], outs[k]) for k in range(24)]
    for t in tickets:
        assert srv.wait(t, 60000) == _native.PIR_OK
    st = srv.stats()
    srv.close()
    for k in range(24):
        assert np.array_equal(outs[k], wants[2][k]), k
    assert st["rejected"] == 0
    assert st["blocked_submits"] > 0, "the two-row ring never filled"
