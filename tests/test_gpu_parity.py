"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Every answer of dpXOR is unique (XOR over F_2 is exact), so the bar is
equality of bytes everywhere.  Inputs come from the seeded generator only.
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
    c.close()


def _dev_rows(sel_rows, n):
    """Copy host selection rows into a device buffer with the library's row pitch."""
    q = sel_rows.shape[0]
    stride = pir.sel_stride_for(n)
    host = np.zeros((q, stride), np.uint8)
    w = min(sel_rows.shape[1], stride)
    host[:, :w] = sel_rows[:, :w]
    return torch.from_numpy(host).to("cuda:0"), stride


def _flip(row, i):
    r = row.copy()
    r[i >> 3] ^= np.uint8(1 << (i & 7))
    return r


def test_c1_single_query_and_two_server_invariant(ctx):
    # 2^20 records of 32 B (32 MiB), one Bernoulli(0.5) query; the e_i check
    # for 16 random i: ans(b) XOR ans(b XOR e_i) = D[i].
    n, r = 1 << 20, 32
    dbh = synth.database(n, r, seed=synth.S_DB + 1)
    db = ctx.load_db(dbh)
    b = synth.selections(n, 1, seed=synth.S_SEL + 1)[0]
    got = db.dpxor(b)
    assert np.array_equal(got, oracle.dpxor(dbh, b))
    idx = synth.indices(n, 16, seed=synth.S_IDX + 1)
    rows = np.stack([b] + [_flip(b, i) for i in idx])
    ans = db.dpxor_batch(rows)
    assert np.array_equal(ans[0], got)
    for k, i in enumerate(idx):
        assert np.array_equal(ans[0] ^ ans[k + 1], dbh[i]), f"e_{i} reconstruction failed"
    db.free()


SHAPES = [(1, 1), (1, 32), (31, 3), (32, 32), (33, 1), (33, 33), (100, 2), (257, 4), (1000, 5),
          (1000, 8), (4097, 16), (4097, 17), (5000, 31), (65537, 32), (3001, 48), (2049, 64),
          (1234, 100), (777, 128), (10007, 256), (300, 1024), (65, 1000)]


@pytest.mark.parametrize("n,r", SHAPES)
def test_shape_grid_sync(ctx, n, r):
    dbh = synth.database(n, r, seed=1000 + n + r)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, 3, seed=2000 + n * 7 + r, tail_junk=True)
    got = db.dpxor_batch(sel)
    assert np.array_equal(got, oracle.dpxor_batch(dbh, sel))
    assert np.array_equal(db.dpxor(sel[1]), oracle.dpxor(dbh, sel[1]))
    db.free()


@pytest.mark.parametrize("n,r", [(70001, 32), (9000, 7), (5003, 256), (3000, 96)])
def test_special_selections(ctx, n, r):
    dbh = synth.database(n, r, seed=77 + r)
    db = ctx.load_db(dbh)
    nb = (n + 7) // 8
    zero = np.zeros(nb, np.uint8)
    ones = np.full(nb, 0xFF, np.uint8)
    assert not db.dpxor(zero).any()
    assert np.array_equal(db.dpxor(ones), np.bitwise_xor.reduce(dbh, axis=0))
    for i in (0, 31, 32, n - 1):
        e = zero.copy()
        e[i >> 3] = np.uint8(1 << (i & 7))
        assert np.array_equal(db.dpxor(e), dbh[i])
    db.free()


@pytest.mark.parametrize("q", [1, 2, 3, 8, 16, 17, 33, 64])
@pytest.mark.parametrize("n,r", [(50000, 32), (3333, 256), (20000, 8), (4000, 3)])
def test_batch_async_default(ctx, n, r, q):
    dbh = synth.database(n, r, seed=5 + n + r)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, q, seed=900 + q)
    want = oracle.dpxor_batch(dbh, sel)
    d_sel, stride = _dev_rows(sel, n)
    d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
    db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride)
    torch.cuda.synchronize()
    assert np.array_equal(d_out.cpu().numpy(), want)
    db.free()


VALU_CFGS = [(1, 4), (1, 8), (1, 16), (2, 4), (2, 8), (4, 2), (4, 4), (4, 8), (8, 1), (8, 2), (8, 4),
             (16, 1), (16, 2), (16, 4), (32, 1), (32, 2)]


@pytest.mark.parametrize("n,r,q", [(40000, 32, 21), (2500, 128, 9), (9000, 4, 5)])
def test_tile_invariance(ctx, n, r, q):
    # every compiled (q_tile, unroll) and several grid sizes give identical bytes
    dbh = synth.database(n, r, seed=31 * n + r)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, q, seed=4242 + q)
    want = oracle.dpxor_batch(dbh, sel)
    d_sel, stride = _dev_rows(sel, n)
    d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
    for qt, u in VALU_CFGS:
        for groups in (1, 7, 0):
            d_out.fill_(0xEE)
            db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride,
                                 cfg=pir.KernelCfg(pir.PIR_VARIANT_VALU, qt, u, groups))
            torch.cuda.synchronize()
            assert np.array_equal(d_out.cpu().numpy(), want), (qt, u, groups)
    db.free()


def test_update_and_read_back(ctx):
    n, r = 1000, 24
    dbh = synth.database(n, r, seed=3)
    db = ctx.load_db(dbh)
    assert np.array_equal(db.read(0, n), dbh)
    new = synth.database(77, r, seed=4)
    db.update(45, new)
    dbh2 = dbh.copy()
    dbh2[45:122] = new
    assert np.array_equal(db.read(0, n), dbh2)
    assert np.array_equal(db.read(40, 10), dbh2[40:50])
    sel = synth.selections(n, 4, seed=5)
    assert np.array_equal(db.dpxor_batch(sel), oracle.dpxor_batch(dbh2, sel))
    db.free()


def test_repeat_runs_deterministic(ctx):
    n, r, q = 200000, 32, 16
    dbh = synth.database(n, r, seed=8)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, q, seed=9)
    d_sel, stride = _dev_rows(sel, n)
    outs = []
    for _ in range(3):
        d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
        db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride)
        torch.cuda.synchronize()
        outs.append(d_out.cpu().numpy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    assert np.array_equal(outs[0], oracle.dpxor_batch(dbh, sel))
    db.free()


def test_invalid_arguments(ctx):
    n, r = 100, 32
    dbh = synth.database(n, r, seed=1)
    db = ctx.load_db(dbh)
    d_sel = torch.zeros(256, dtype=torch.uint8, device="cuda:0")
    d_out = torch.zeros(64, dtype=torch.uint8, device="cuda:0")
    from paper_2509_06514_amd import _native
    lib = pir.lib()
    import ctypes
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # stride not a multiple of 4, stride too small, q = 0, q too large
    assert lib.pir_dpxor_batch_async(db.handle, ctypes.c_void_p(d_sel.data_ptr()), 6, 1,
                                     ctypes.c_void_p(d_out.data_ptr()), s) == _native.PIR_E_INVAL
    assert lib.pir_dpxor_batch_async(db.handle, ctypes.c_void_p(d_sel.data_ptr()), 0, 1,
                                     ctypes.c_void_p(d_out.data_ptr()), s) == _native.PIR_E_INVAL
    assert lib.pir_dpxor_batch_async(db.handle, ctypes.c_void_p(d_sel.data_ptr()), 256, 0,
                                     ctypes.c_void_p(d_out.data_ptr()), s) == _native.PIR_E_INVAL
    assert lib.pir_dpxor_batch_async(db.handle, ctypes.c_void_p(d_sel.data_ptr()), 256, 5000,
                                     ctypes.c_void_p(d_out.data_ptr()), s) == _native.PIR_E_INVAL
    h = ctypes.c_void_p()
    assert lib.pir_db_load(ctx.handle, ctypes.c_void_p(dbh.ctypes.data), 0, 32,
                           ctypes.byref(h)) == _native.PIR_E_INVAL
    assert lib.pir_db_load(ctx.handle, ctypes.c_void_p(dbh.ctypes.data), 10, 0,
                           ctypes.byref(h)) == _native.PIR_E_INVAL
    assert lib.pir_db_update(db.handle, n - 1, 2, ctypes.c_void_p(dbh.ctypes.data)) == _native.PIR_E_INVAL
    db.free()


MFMA_VARIANTS = [pir.PIR_VARIANT_MFMA_F4, pir.PIR_VARIANT_MFMA_I8]


def _mfma_cfg_exists(variant, qt, unroll):
    """The matrix-core (q_tile, unroll) combinations the library compiles."""
    f4 = variant == pir.PIR_VARIANT_MFMA_F4
    if unroll in (2, 3, 4):
        return qt in (16, 32, 64)
    if unroll in (12, 15, 16, 17):
        return f4 and qt == 64
    return False


@pytest.mark.parametrize("variant", MFMA_VARIANTS)
@pytest.mark.parametrize("n,r", [(50000, 32), (4099, 64), (3333, 256), (1000, 1024), (70001, 128), (31, 32)])
def test_mfma_variants(ctx, variant, n, r):
    # the matrix-core forms (exact counts, then parity) give the oracle's bytes
    dbh = synth.database(n, r, seed=7 * n + r + variant)
    db = ctx.load_db(dbh)
    qs = (1, 5, 16, 17, 33, 64, 100)
    sel = synth.selections(n, max(qs), seed=600 + n + r)
    want = oracle.dpxor_batch(dbh, sel)
    d_sel, stride = _dev_rows(sel, n)
    for q in qs:
        d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
        for qt in (16, 32, 64):
            # LDS rings of 2/3/4 stages, split K on a 2-stage ring, split K with
            # selection words 4 K-steps at a time (shared and wave-private
            # database stages, database words straight into registers)
            for unroll in (2, 3, 4, 12, 15, 16, 17):
                if not _mfma_cfg_exists(variant, qt, unroll):
                    continue
                for groups in (0, 3, 1):
                    d_out.fill_(0xEE)
                    db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride,
                                         cfg=pir.KernelCfg(variant, qt, unroll, groups))
                    torch.cuda.synchronize()
                    assert np.array_equal(d_out.cpu().numpy(), want[:q]), (q, qt, unroll, groups)
    db.free()


@pytest.mark.parametrize("r", [32, 64])
def test_split_k_step_counts(ctx, r):
    # The split-K kernels move selection words in stages of four K-steps (16
    # blocks of 32 records each) and keep database stages one step ahead:
    # record groups of exactly 1 .. 9 K-steps (partial last stages), with and
    # without a ragged tail of fewer than 16 blocks, and a second, partial
    # 64-query tile, one record group each, all against the oracle.
    for steps in range(1, 10):
        for extra in (0, 37 + 32 * 5):
            n = 512 * steps + extra
            dbh = synth.database(n, r, seed=0x5C0 + 16 * steps + r + extra)
            db = ctx.load_db(dbh)
            sel = synth.selections(n, 70, seed=0x5C1 + steps + extra)
            want = oracle.dpxor_batch(dbh, sel)
            d_sel, stride = _dev_rows(sel, n)
            for q in (64, 70):
                d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
                for unroll in (12, 15, 16, 17):
                    d_out.fill_(0xEE)
                    db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride,
                                         cfg=pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 64, unroll, 1))
                    torch.cuda.synchronize()
                    assert np.array_equal(d_out.cpu().numpy(), want[:q]), (steps, extra, q, unroll)
            db.free()


@pytest.mark.parametrize("variant", MFMA_VARIANTS)
def test_mfma_counts_exact_on_large_group(ctx, variant):
    # 2^25 records: one requested record group would hold 2^25 > 2^24 records;
    # the planner splits it so fp32 counts stay exact.  All-ones selections
    # make every count maximal.
    n, r, q = 1 << 25, 32, 16
    dbh = synth.database(n, r, seed=0xACE + variant)
    db = ctx.load_db(dbh)
    stride = pir.sel_stride_for(n)
    host = np.full((q, stride), 0xFF, np.uint8)
    want_all = np.bitwise_xor.reduce(dbh, axis=0)
    rnd = synth.selections(n, 1, seed=0xBEE, stride=stride)
    host[3] = rnd[0]
    d_sel = torch.from_numpy(host).to("cuda:0")
    d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
    want3 = oracle.dpxor(dbh, rnd[0])
    cfgs = [(16, 2), (16, 3), (16, 4)]
    if variant == pir.PIR_VARIANT_MFMA_F4:
        cfgs += [(64, 12), (64, 15), (64, 16), (64, 17)]  # split K: each half's counts and their sum stay exact
    for qt, unroll in cfgs:
        d_out.fill_(0)
        db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride, cfg=pir.KernelCfg(variant, qt, unroll, 1))
        torch.cuda.synchronize()
        got = d_out.cpu().numpy()
        for i in range(q):
            if i != 3:
                assert np.array_equal(got[i], want_all), (unroll, i)
        assert np.array_equal(got[3], want3), unroll
    db.free()


def test_largest_batch(ctx):
    # Q = PIR_MAX_BATCH queries in one call: 64 query tiles of the matrix-core
    # form, the vector-ALU form and the synchronous host path give the oracle's rows
    n, r, q = 5003, 32, 4096
    dbh = synth.database(n, r, seed=0x4096)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, q, seed=0x4097)
    want = oracle.dpxor_batch(dbh, sel)
    d_sel, stride = _dev_rows(sel, n)
    d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
    for cfg in (None, pir.KernelCfg(pir.PIR_VARIANT_VALU, 32, 2, 0), pir.KernelCfg(pir.PIR_VARIANT_MFMA_I8, 64, 3, 0)):
        d_out.fill_(0xEE)
        db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride, cfg=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(d_out.cpu().numpy(), want), cfg
    assert np.array_equal(db.dpxor_batch(sel[:, : (n + 7) // 8]), want)
    db.free()


def test_largest_batch_of_large_records(ctx):
    # Q = PIR_MAX_BATCH answers of 20000-byte records: 2^24 words of
    # answers and more, which the cross-group fold covers in two launches of
    # whole rows; every row against the oracle
    n, r, q = 3001, 20000, 4096
    dbh = synth.database(n, r, seed=0x4098)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, q, seed=0x4099)
    want = oracle.dpxor_rows(dbh, sel)
    d_sel, stride = _dev_rows(sel, n)
    d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
    for cfg in (None, pir.KernelCfg(pir.PIR_VARIANT_VALU, 32, 2, 0)):
        d_out.fill_(0xEE)
        db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride, cfg=cfg)
        torch.cuda.synchronize()
        got = d_out.cpu().numpy()
        bad = [i for i in range(q) if not np.array_equal(got[i], want[i])]
        assert not bad, (cfg, len(bad), bad[:8])
    db.free()


def test_host_path_pinned_and_staged(ctx):
    # The synchronous call with pageable rows (packed into two pinned halves,
    # 4 rows of this database's 4 MiB device pitch per half, so 11 rows take
    # three chunks and reuse the first half) and with pinned rows and answers
    # (pitched copies straight to and from the device): same bytes as the
    # oracle, for an odd host stride and junk past N in every row.
    n, r, q = (1 << 25) + 77, 8, 11
    stride = (n + 7) // 8 + 3
    dbh = synth.database(n, r, seed=0x5717)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, q, seed=0x5718, stride=stride, tail_junk=True)
    want = oracle.dpxor_batch(dbh, sel)
    assert np.array_equal(db.dpxor_batch(sel), want)
    p_sel = pir.pinned_empty((q, stride))
    p_out = pir.pinned_empty((q, r))
    synth.selections(n, q, seed=0x5718, stride=stride, tail_junk=True, out=p_sel)
    p_out.fill(0xEE)
    assert db.dpxor_batch(p_sel, out=p_out) is p_out
    assert np.array_equal(p_out, want)
    assert np.array_equal(db.dpxor_batch(p_sel), want)  # pinned in, pageable out
    assert np.array_equal(db.dpxor_batch(sel, out=p_out), want)  # pageable in, pinned out
    assert np.array_equal(db.dpxor_batch(p_sel[:5]), want[:5])  # fewer rows on the same buffers
    p_one = pir.pinned_empty((r,))
    assert np.array_equal(db.dpxor(p_sel[3], out=p_one), want[3])
    assert np.array_equal(db.dpxor(sel[7]), want[7])
    db.free()


@pytest.mark.parametrize("n,r", [(50000, 32), (3333, 256)])
def test_wide_selection_kernel_unaligned_rows(ctx, n, r):
    # The split-K kernel with wide selection reads moves 16 bytes of a row per
    # lane.  At the minimum pitch (4 * ceil(N/32) bytes, not a multiple of 16
    # here) and at a base 4 bytes past an aligned address the launcher must
    # take the 4-byte selection loads instead; the answers stay the oracle's.
    dbh = synth.database(n, r, seed=0x16A + n + r)
    db = ctx.load_db(dbh)
    stride = db.min_sel_stride
    assert stride % 16 != 0
    q = 64
    sel = synth.selections(n, q, seed=0x16B + n, stride=stride)
    want = oracle.dpxor_batch(dbh, sel)
    cfgs = [pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 64, u, 0) for u in (15, 16, 17)]
    d_out = torch.empty((q, r), dtype=torch.uint8, device="cuda:0")
    for cfg in cfgs:
        for base in (0, 4):
            buf = torch.zeros(q * stride + 16, dtype=torch.uint8, device="cuda:0")
            buf[base:base + q * stride] = torch.from_numpy(sel.reshape(-1))
            d_sel = buf[base:]
            for qq in (q, 5):
                d_out.fill_(0xEE)
                db.dpxor_batch_async(d_sel, qq, d_out, sel_stride=stride, cfg=cfg)
                torch.cuda.synchronize()
                assert np.array_equal(d_out.cpu().numpy()[:qq], want[:qq]), (cfg, base, qq)
    # an aligned pitch (a multiple of 16 bytes) on the same rows
    stride16 = (stride + 15) // 16 * 16
    rows = np.zeros((q, stride16), np.uint8)
    rows[:, :stride] = sel
    d_rows = torch.from_numpy(rows).to("cuda:0")
    for cfg in cfgs:
        d_out.fill_(0xEE)
        db.dpxor_batch_async(d_rows, q, d_out, sel_stride=stride16, cfg=cfg)
        torch.cuda.synchronize()
        assert np.array_equal(d_out.cpu().numpy(), want), cfg
    db.free()
