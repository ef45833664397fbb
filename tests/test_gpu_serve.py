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
