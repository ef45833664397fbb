"""GPU parity of the F_p inner-product form, r_q[l] = (sum_j v_q[j] D[j][l]) mod p,
through the C ABI, against the oracle element by element.

Shapes cover several tiles and ragged tails (records not a multiple of 64,
elements per record not a multiple of 16), query counts across row tiles
(1, 5, 16, 17, 64, 100), and primes from 2 to 127.  At the benchmark's size
(2^24 records x 32 elements, p = 127) and on a 5.4 GB database every row is
checked against the oracle.
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


def _db(n, L, p, seed):
    return (synth.stream_bytes(seed, n * L).reshape(n, L) % p).astype(np.uint8)


def _queries(q, stride, seed, top=128):
    # bytes below 128 (values past p act as their residues); junk past N
    rows = (synth.stream_bytes(seed, q * stride).reshape(q, stride) % top).astype(np.uint8)
    return rows


def _oracle_rows(D, rows, p):
    """The oracle's answer for every row, rows spread over the host threads
    (each row is one single-threaded oracle call; the C oracle releases the
    interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(min(16, oracle.host_threads())) as ex:
        return np.stack(list(ex.map(lambda v: oracle.fp_inner(D, v, p), rows)))


def _async(db, rows):
    q, stride = rows.shape
    pad = (max(stride, db.min_v_stride) + 15) // 16 * 16
    host = np.zeros((q, pad), np.uint8)
    host[:, :stride] = rows
    d_v = torch.from_numpy(host).to("cuda:0")
    d_out = torch.full((q, db.record_elems), 0xEE, dtype=torch.uint8, device="cuda:0")
    db.inner_async(d_v, q, d_out)
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


@pytest.mark.parametrize("p", [2, 3, 101, 127])
@pytest.mark.parametrize("n,L", [(1, 1), (63, 5), (64, 16), (1000, 32), (4097, 48), (20011, 100), (100003, 7)])
def test_matches_oracle(ctx, p, n, L):
    D = _db(n, L, p, synth.S_DB + 200 + 7 * p + L)
    db = ctx.load_fp_db(D, p)
    assert np.array_equal(db.read(0, n), D)
    for q in (1, 5, 17):
        rows = _queries(q, n + 70, synth.S_SEL + 300 + q + n, top=128 if q != 5 else p)
        got = _async(db, rows)
        for i in range(q):
            assert np.array_equal(got[i], oracle.fp_inner(D, rows[i][:n], p)), (p, n, L, q, i)
        assert np.array_equal(db.inner(rows[:, :n]), got)
    db.free()


@pytest.mark.parametrize("q", [16, 64, 100])
def test_query_tiles(ctx, q):
    n, L, p = 30001, 64, 127
    D = _db(n, L, p, synth.S_DB + 210)
    db = ctx.load_fp_db(D, p)
    rows = _queries(q, n, synth.S_SEL + 310 + q)
    got = _async(db, rows)
    for i in sorted({0, q // 2, q - 1}):
        assert np.array_equal(got[i], oracle.fp_inner(D, rows[i], p)), (q, i)
    want = (rows.astype(np.int64) @ D.astype(np.int64)) % p  # all rows, integer product
    assert np.array_equal(got, want.astype(np.uint8))
    db.free()


def test_largest_values_and_shares(ctx):
    # every element p - 1 and every query byte 127: the largest sums
    n, L, p = 1 << 22, 32, 127
    D = np.full((n, L), p - 1, np.uint8)
    db = ctx.load_fp_db(D, p)
    rows = np.full((2, n), 127, np.uint8)
    rows[0] = 126
    got = _async(db, rows)
    assert np.array_equal(got[0], np.full(L, (n * 126 * (p - 1)) % p, np.uint8))
    assert np.array_equal(got[1], np.full(L, (n * 127 * (p - 1)) % p, np.uint8))
    db.free()
    # additive shares of a unit vector reconstruct the record (mod p)
    D = _db(n, L, p, synth.S_DB + 220)
    db = ctx.load_fp_db(D, p)
    rng = np.random.default_rng(9)
    for i in (0, n - 1, int(rng.integers(0, n))):
        v1 = (synth.stream_bytes(synth.S_SEL + 320 + i % 1000, n) % p).astype(np.uint8)
        e = np.zeros(n, np.int64)
        e[i] = 1
        v2 = ((e - v1) % p).astype(np.uint8)
        r = _async(db, np.stack([v1, v2]))
        assert np.array_equal((r[0].astype(int) + r[1]) % p, D[i]), i
    db.free()


def test_benchmark_shape(ctx):
    # 2^24 records x 32 elements (512 MiB), p = 127, Q = 64: every row
    # against the oracle
    n, L, p, q = 1 << 24, 32, 127, 64
    D = _db(n, L, p, synth.S_DB + 230)
    db = ctx.load_fp_db(D, p)
    rows = _queries(q, n, synth.S_SEL + 330)
    got = _async(db, rows)
    want = _oracle_rows(D, rows, p)
    bad = [i for i in range(q) if not np.array_equal(got[i], want[i])]
    assert not bad, bad
    db.free()


def test_db_beyond_4_gib(ctx):
    # 2^27 + 77 records x 40 elements (5.4 GB): element offsets past 2^32,
    # ragged N and L, p = 127, Q = 64; every row against the oracle, and
    # read-back of the last records
    n, L, p, q = (1 << 27) + 77, 40, 127, 64
    D = _db(n, L, p, synth.S_DB + 240)
    db = ctx.load_fp_db(D, p)
    rows = _queries(q, n, synth.S_SEL + 340)
    got = _async(db, rows)
    want = _oracle_rows(D, rows, p)
    bad = [i for i in range(q) if not np.array_equal(got[i], want[i])]
    assert not bad, bad
    assert np.array_equal(db.read(n - 100, 100), D[n - 100:])
    db.free()


def test_rejects_bad_arguments(ctx):
    lib = pir.lib()
    D = np.zeros((100, 4), np.uint8)
    D[7, 2] = 5
    h = pir._native.ctypes.c_void_p()
    E = _native.PIR_E_INVAL
    assert lib.pir_fp_db_load(ctx.handle, D.ctypes.data, 100, 4, 5, pir._native.ctypes.byref(h)) == E  # 5 >= p
    assert lib.pir_fp_db_load(ctx.handle, D.ctypes.data, 100, 4, 1, pir._native.ctypes.byref(h)) == E
    assert lib.pir_fp_db_load(ctx.handle, D.ctypes.data, 100, 4, 128, pir._native.ctypes.byref(h)) == E
    assert lib.pir_fp_db_load(ctx.handle, D.ctypes.data, 0, 4, 7, pir._native.ctypes.byref(h)) == E
    db = ctx.load_fp_db(D, 7)
    v = torch.zeros((2, 128), dtype=torch.uint8, device="cuda:0")
    out = torch.zeros((2, 4), dtype=torch.uint8, device="cuda:0")
    assert db.min_v_stride == 128
    assert db.v_stride == 128
    assert lib.pir_fp_inner_async(db.handle, v.data_ptr(), 112, 2, out.data_ptr(), None) == E  # < 128
    assert lib.pir_fp_inner_async(db.handle, v.data_ptr(), 136, 1, out.data_ptr(), None) == E  # not x16
    assert lib.pir_fp_inner_async(db.handle, v.data_ptr() + 8, 128, 1, out.data_ptr(), None) == E
    assert lib.pir_fp_inner_async(db.handle, v.data_ptr(), 128, 0, out.data_ptr(), None) == E
    db.free()


@pytest.mark.parametrize("n", [64, 4097, 65536, 100003])
def test_recommended_pitch(ctx, n):
    # the recommended row pitch is the smallest odd multiple of 128 bytes that
    # holds a row, and the scan at that pitch gives the oracle's rows
    L, p, q = 16, 101, 17
    D = _db(n, L, p, synth.S_DB + 300 + n)
    db = ctx.load_fp_db(D, p)
    vs = db.v_stride
    assert vs >= db.min_v_stride and vs % 128 == 0 and (vs // 128) % 2 == 1
    assert vs - 256 < db.min_v_stride
    rows = _queries(q, vs, synth.S_SEL + 300 + n)
    rows[:, n:] = 0
    d_v = torch.from_numpy(rows).to("cuda:0")
    d_out = torch.full((q, L), 0xEE, dtype=torch.uint8, device="cuda:0")
    db.inner_async(d_v, q, d_out, v_stride=vs)
    torch.cuda.synchronize()
    want = np.stack([oracle.fp_inner(D, rows[i, :n], p) for i in range(q)])
    assert np.array_equal(d_out.cpu().numpy(), want)
    assert np.array_equal(db.inner(rows[:, :n]), want)  # synchronous call, staged at the same pitch
    db.free()


def test_sync_staging_pieces_and_pinned(ctx):
    # The synchronous call with more query bytes than the two 16 MiB staging
    # pieces (pageable rows: packed piece by piece, pieces reused), and with
    # pinned rows and answers (one pitched copy each way).  The pinned call
    # after a larger database's leaves older bytes in the device rows' tails
    # past N: they meet only the zero padding records and change nothing.
    L, p = 16, 101
    n_big, n_small, q = (1 << 21) + 37, 4097, 24   # 24 rows x ~2 MiB: four pieces
    D_big = _db(n_big, L, p, synth.S_DB + 400)
    D_small = _db(n_small, L, p, synth.S_DB + 401)
    big = ctx.load_fp_db(D_big, p)
    small = ctx.load_fp_db(D_small, p)
    rows = _queries(q, n_big + 3, synth.S_SEL + 400)
    want_async = _async(big, rows[:, :n_big])
    got = big.inner(rows)                            # pageable, 3 bytes of junk per row past N
    assert np.array_equal(got, want_async)
    for i in (0, 13, q - 1):
        assert np.array_equal(got[i], oracle.fp_inner(D_big, rows[i, :n_big], p)), i
    p_rows = pir.pinned_empty(rows.shape)
    p_rows[:] = rows
    p_out = pir.pinned_empty((q, L))
    assert big.inner(p_rows, out=p_out) is p_out
    assert np.array_equal(p_out, want_async)
    p_small = pir.pinned_empty((q, n_small))
    p_small[:] = rows[:, :n_small]
    got_small = small.inner(p_small, out=pir.pinned_empty((q, L)))
    for i in range(q):
        assert np.array_equal(got_small[i], oracle.fp_inner(D_small, rows[i, :n_small], p)), i
    small.free()
    big.free()
