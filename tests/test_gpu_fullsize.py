"""Parity at the full workload sizes, in the launch configurations the
benchmark times (tuned plans, same seeds as bench.py).

Every answer row is compared with the oracle's answer for that row alone
(IM-PIR Sec. 2, the server subresult r; Sec. 3.4, batched keys are
independent).  The oracle computes each row with one full database scan on
one host thread; rows run on every host thread of the process at once.  The
two-server identity ans(b) XOR ans(b XOR e_i) = D[i] is checked as well.
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


def _run(db, d_sel, stride, q, cfg=None):
    out = torch.empty((q, db.record_bytes), dtype=torch.uint8, device="cuda:0")
    out.fill_(0xEE)
    db.dpxor_batch_async(d_sel, q, out, sel_stride=stride, cfg=cfg)
    torch.cuda.synchronize()
    return out.cpu().numpy()


class OracleRows:
    """The oracle's answers for the first k selection rows, computed on demand."""

    def __init__(self, dbh, sel):
        self.dbh, self.sel = dbh, sel
        self.rows = np.empty((0, dbh.shape[1]), np.uint8)

    def first(self, k):
        have = self.rows.shape[0]
        if k > have:
            new = oracle.dpxor_rows(self.dbh, self.sel, range(have, k))
            self.rows = np.concatenate([self.rows, new])
        return self.rows[:k]


def _assert_rows(got, want, what):
    bad = [i for i in range(want.shape[0]) if not np.array_equal(got[i], want[i])]
    assert not bad, f"{what}: {len(bad)} of {want.shape[0]} rows differ from the oracle, first {bad[:8]}"


@pytest.fixture(scope="module")
def db_n28r32(ctx):
    # 2^28 records x 32 B = 8 GiB, the benchmark's database and selections
    n, r = 1 << 28, 32
    dbh = synth.database(n, r, seed=synth.S_DB + 3)
    db = ctx.load_db(dbh)
    stride = pir.sel_stride_for(n)
    sel = synth.selections(n, 512, seed=synth.S_SEL + 3, stride=stride)
    d_sel = torch.from_numpy(sel).to("cuda:0")
    yield dbh, db, sel, d_sel, stride, OracleRows(dbh, sel)
    del d_sel
    db.free()


@pytest.mark.parametrize("q", [1, 16, 64, 512])
def test_n28r32_tuned_plan_matches_oracle(db_n28r32, q):
    dbh, db, sel, d_sel, stride, orc = db_n28r32
    cfg = db.tune(q)  # what bench.py does before timing
    assert db.get_cfg(q).as_dict() == cfg.as_dict()
    got = _run(db, d_sel, stride, q)  # default path = the tuned plan
    _assert_rows(got, orc.first(q), f"q={q} {cfg}")


@pytest.mark.parametrize("q", [64, 512])
def test_n28r32_variants_match_oracle(db_n28r32, q):
    # bitwise select-XOR, int8 matrix cores and fp4 matrix cores, every row
    dbh, db, sel, d_sel, stride, orc = db_n28r32
    want = orc.first(q)
    for cfg in (pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 64, 4, 0),
                pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 64, 12, 0),
                pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 64, 15, 0),
                pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 64, 16, 0),
                pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 64, 17, 0),
                pir.KernelCfg(pir.PIR_VARIANT_MFMA_I8, 64, 4, 0),
                pir.KernelCfg(pir.PIR_VARIANT_MFMA_I8, 32, 2, 0),
                pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 32, 3, 0),
                pir.KernelCfg(pir.PIR_VARIANT_VALU, 16, 4, 0)):
        _assert_rows(_run(db, d_sel, stride, q, cfg), want, f"q={q} {cfg}")


def test_n28r32_two_server_identity(db_n28r32):
    # for random b and b XOR e_i (16 random i): ans(b) XOR ans(b XOR e_i) = D[i]
    dbh, db, sel, d_sel, stride, orc = db_n28r32
    n = dbh.shape[0]
    idx = synth.indices(n, 16, seed=synth.S_IDX + 3)
    pair = np.empty((1 + len(idx), stride), np.uint8)
    pair[0] = sel[0]
    for k, i in enumerate(idx):
        pair[k + 1] = sel[0]
        pair[k + 1, i >> 3] ^= np.uint8(1 << (i & 7))
    d_pair = torch.from_numpy(pair).to("cuda:0")
    ans = _run(db, d_pair, stride, pair.shape[0])
    assert np.array_equal(ans[0], orc.first(1)[0])
    for k, i in enumerate(idx):
        assert np.array_equal(ans[0] ^ ans[k + 1], dbh[i]), i


def test_n25r32_single_query_full_compare(ctx):
    # 2^25 records x 32 B (1 GiB): the single-query roofline configuration
    n, r = 1 << 25, 32
    dbh = synth.database(n, r, seed=synth.S_DB + 2)
    db = ctx.load_db(dbh)
    stride = pir.sel_stride_for(n)
    sel = synth.selections(n, 1, seed=synth.S_SEL + 2, stride=stride)
    db.tune(1)
    got = _run(db, torch.from_numpy(sel).to("cuda:0"), stride, 1)
    assert np.array_equal(got[0], oracle.dpxor(dbh, sel[0]))
    assert np.array_equal(db.dpxor(sel[0][: (n + 7) // 8]), got[0])
    db.free()


def test_n23r256_batched_rows(ctx):
    # 2^23 records x 256 B (2 GiB), Q in {8, 64, 256} in one pass each, every row
    n, r = 1 << 23, 256
    dbh = synth.database(n, r, seed=synth.S_DB + 4)
    db = ctx.load_db(dbh)
    stride = pir.sel_stride_for(n)
    sel = synth.selections(n, 256, seed=synth.S_SEL + 4, stride=stride)
    d_sel = torch.from_numpy(sel).to("cuda:0")
    want = oracle.dpxor_rows(dbh, sel)
    for q in (8, 64, 256):
        cfg = db.tune(q)
        _assert_rows(_run(db, d_sel, stride, q), want[:q], f"q={q} {cfg}")
        if q == 256:
            alt = _run(db, d_sel, stride, q, pir.KernelCfg(pir.PIR_VARIANT_VALU, 16, 4, 0))
            _assert_rows(alt, want, "q=256 VALU")
    db.free()


def test_db_beyond_2_32_words(ctx):
    # 5 * 2^27 + 77 records x 32 B (20 GiB): the bit-sliced database spans
    # about 5.4 * 10^9 32-bit words, past what a 32-bit word offset can
    # reach, and N is ragged (a partial last block, junk selection bits past
    # N).  Every scan form, every row against the oracle; read-back and an
    # update at the far end of the database.
    n, r, q = 5 * (1 << 27) + 77, 32, 64
    dbh = synth.database(n, r, seed=synth.S_DB + 5)
    db = ctx.load_db(dbh)
    assert db.device_bytes > 16 << 30
    stride = pir.sel_stride_for(n)
    sel = synth.selections(n, q, seed=synth.S_SEL + 5, stride=stride, tail_junk=True)
    d_sel = torch.from_numpy(sel).to("cuda:0")
    want = oracle.dpxor_rows(dbh, sel)
    F4, I8, VALU = pir.PIR_VARIANT_MFMA_F4, pir.PIR_VARIANT_MFMA_I8, pir.PIR_VARIANT_VALU
    for cfg in (None,  # the untuned default plan
                pir.KernelCfg(F4, 64, 17, 0), pir.KernelCfg(F4, 64, 16, 0), pir.KernelCfg(F4, 64, 12, 0),
                pir.KernelCfg(F4, 16, 3, 0), pir.KernelCfg(I8, 64, 4, 0), pir.KernelCfg(VALU, 16, 4, 0)):
        _assert_rows(_run(db, d_sel, stride, q, cfg), want, f"N={n} q={q} {cfg}")
    assert np.array_equal(_run(db, d_sel, stride, 1)[0], want[0])
    assert np.array_equal(db.read(n - 1000, 1000), dbh[n - 1000:])
    # flip the last record; every row that selects it changes by old ^ new
    new = np.bitwise_not(dbh[n - 1:])
    db.update(n - 1, new)
    picked = (sel[:, (n - 1) >> 3] >> ((n - 1) & 7)) & 1
    assert 0 < picked.sum() < q
    want2 = want ^ (picked[:, None].astype(np.uint8) * (dbh[n - 1] ^ new[0]))
    _assert_rows(_run(db, d_sel, stride, q), want2, "after the update")
    del d_sel
    db.free()


def test_register_load_kernel_group_past_4_gib(ctx):
    # 2^22 + 77 records x 1 KiB (4 GiB): with one record group the group's
    # database range is past the 32-bit buffer size of the register-load
    # split-K kernel, so the launcher takes the wave-private-stage kernel;
    # with two groups it runs itself.  Every row against the oracle.
    n, r, q = (1 << 22) + 77, 1024, 64
    dbh = synth.database(n, r, seed=synth.S_DB + 6)
    db = ctx.load_db(dbh)
    stride = pir.sel_stride_for(n)
    sel = synth.selections(n, q, seed=synth.S_SEL + 6, stride=stride)
    d_sel = torch.from_numpy(sel).to("cuda:0")
    want = oracle.dpxor_rows(dbh, sel)
    for groups in (1, 2):
        cfg = pir.KernelCfg(pir.PIR_VARIANT_MFMA_F4, 64, 17, groups)
        _assert_rows(_run(db, d_sel, stride, q, cfg), want, f"{cfg}")
    del d_sel
    db.free()
