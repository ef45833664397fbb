"""The autotuner through the C ABI: whatever it picks answers as the oracle
does, at the minimum selection pitch too, and its cache round-trips.

Shapes: ragged N (the minimum pitch 4 * ceil(N/32) bytes is then not a
multiple of 16, so the wide-selection kernels must fall back when handed
such rows), several record sizes and query counts on both sides of the
matrix-core threshold.
"""
import json

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


@pytest.mark.parametrize("n,r,q", [(50001, 32, 64), (3333, 256, 17), (100003, 64, 5), (40001, 128, 100)])
def test_tuned_plan_matches_oracle(ctx, n, r, q):
    dbh = synth.database(n, r, seed=0x7E0 + n + r)
    db = ctx.load_db(dbh)
    cfg = db.tune(q)
    assert cfg.variant in (pir.PIR_VARIANT_VALU, pir.PIR_VARIANT_MFMA_I8, pir.PIR_VARIANT_MFMA_F4), cfg
    assert db.get_cfg(q).as_dict() == cfg.as_dict()
    stride = db.min_sel_stride
    sel = synth.selections(n, q, seed=0x7E1 + n, stride=stride)
    want = oracle.dpxor_batch(dbh, sel)
    # synchronous call (rows repacked at the library's 256-byte pitch)
    assert np.array_equal(db.dpxor_batch(sel), want)
    # device rows at the minimum pitch, under the tuned plan
    d_sel = torch.from_numpy(sel).to("cuda:0")
    d_out = torch.full((q, r), 0xEE, dtype=torch.uint8, device="cuda:0")
    db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride)
    torch.cuda.synchronize()
    assert np.array_equal(d_out.cpu().numpy(), want), (cfg, stride)
    db.free()


def test_tune_cache_round_trip(tmp_path, monkeypatch):
    # pir_tune writes the file PIR_TUNE_CACHE names; a new context reads it
    # back and plans the same configuration without tuning
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n, r, q = 1 << 20, 32, 64
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PIR_TUNE_CACHE", str(cache))
    dbh = synth.database(n, r, seed=0x7E2)
    c1 = pir.Context(0)
    try:
        db1 = c1.load_db(dbh)
        cfg = db1.tune(q)
        db1.free()
    finally:
        c1.close()
    entries = json.loads(cache.read_text())
    nbits = ((n + 31) // 32).bit_length() - 1
    key = f"gfx950/R{r}/Q{q}/NB{nbits}"
    assert key in entries, entries
    assert entries[key] == cfg.as_dict()
    c2 = pir.Context(0)
    try:
        db2 = c2.load_db(dbh)
        assert db2.get_cfg(q).as_dict() == cfg.as_dict()
        db2.free()
    finally:
        c2.close()
