"""The scan entry point that allocates nothing, pir_dpxor_batch_async_noalloc
(partial answers in a fixed per-device scratch), against the entry point it
mirrors, pir_dpxor_batch_async, and the oracle: two calls in a row with the
second smaller, a plan whose partials must be regrouped to fit, and a batch
whose partials cannot fit at all."""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pir = pytest.importorskip("paper_2509_06514_amd")
from paper_2509_06514_amd import _native  # noqa: E402

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = _native.PIR_NOALLOC_SCRATCH_BYTES


def _noalloc(db, d_sel, stride, q, d_out):
    """The C-ABI call itself (argument types from the binding's signature table)."""
    return pir.lib().pir_dpxor_batch_async_noalloc(db.handle, ctypes.c_void_p(d_sel.data_ptr()), stride, q,
                                                    ctypes.c_void_p(d_out.data_ptr()),
                                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _both(db, sel, q):
    """Rows 0..q-1 of `sel` through the allocating entry point and through the
    no-allocation one (output buffers pre-filled with junk)."""
    stride = sel.shape[1]
    d_sel = torch.from_numpy(sel).to("cuda:0")
    r = db.record_bytes
    ref = torch.full((q, r), 0xEE, dtype=torch.uint8, device="cuda:0")
    got = torch.full((q, r), 0x11, dtype=torch.uint8, device="cuda:0")
    db.dpxor_batch_async(d_sel, q, ref, sel_stride=stride)
    assert _noalloc(db, d_sel, stride, q, got) == _native.PIR_OK, pir.lib().pir_last_error()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pir.Context(0)
    yield c
    c.close()


def test_two_calls_second_smaller(ctx):
    # first call: 2^20 + 77 records of 32 B, 64 queries (matrix-core plan)
    n, r, q = (1 << 20) + 77, 32, 64
    dbh = synth.database(n, r, seed=0x0A11)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, q, seed=0x0A12, stride=pir.sel_stride_for(n))
    ref, got = _both(db, sel, q)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.dpxor_rows(dbh, sel))
    db.free()
    # second call, smaller: 50001 records of 256 B, 7 queries (vector-ALU plan);
    # the scratch still holds the first call's partials
    n, r, q = 50001, 256, 7
    dbh = synth.database(n, r, seed=0x0A13)
    db = ctx.load_db(dbh)
    sel = synth.selections(n, q, seed=0x0A14, stride=pir.sel_stride_for(n))
    ref, got = _both(db, sel, q)
    assert np.array_equal(got, ref)
    assert np.array_equal(got, oracle.dpxor_rows(dbh, sel))
    # the binding's method of the same name
    d_out = torch.full((q, r), 0x33, dtype=torch.uint8, device="cuda:0")
    db.dpxor_batch_async_noalloc(torch.from_numpy(sel).to("cuda:0"), q, d_out, sel_stride=sel.shape[1])
    torch.cuda.synchronize()
    assert np.array_equal(d_out.cpu().numpy(), ref)
    db.free()


def test_plan_regrouped_to_fit_the_scratch(tmp_path, monkeypatch):
    # A cached plan with 4096 record groups: 256 queries x 256 B of partials
    # per group is 16x the scratch, so the no-allocation call folds the
    # records into fewer, longer groups; the answers are the same.
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n, r, q = 1 << 21, 256, 256
    nbits = ((n + 31) // 32).bit_length() - 1
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({f"gfx950/R{r}/Q{q}/NB{nbits}": {"variant": 3, "q_tile": 64, "unroll": 15,
                                                                  "groups": 4096}}))
    monkeypatch.setenv("PIR_TUNE_CACHE", str(cache))
    c = pir.Context(0)
    try:
        dbh = synth.database(n, r, seed=0x0A15)
        db = c.load_db(dbh)
        cfg = db.get_cfg(q)
        assert cfg.groups * q * r > SCRATCH_BYTES, cfg
        sel = synth.selections(n, q, seed=0x0A16, stride=pir.sel_stride_for(n))
        ref, got = _both(db, sel, q)
        assert np.array_equal(got, ref)
        rows = [0, 97, q - 1]
        assert np.array_equal(got[rows], oracle.dpxor_rows(dbh, sel, rows))
        db.free()
    finally:
        c.close()


def test_partials_beyond_the_scratch_are_refused(ctx):
    # 4096 queries of 16 KiB records need 64 MiB of partials even in one group
    n, r, q = 64, 16384, 4096
    db = ctx.load_db(synth.database(n, r, seed=0x0A17))
    stride = pir.sel_stride_for(n)
    d_sel = torch.zeros((q, stride), dtype=torch.uint8, device="cuda:0")
    d_out = torch.zeros((q, r), dtype=torch.uint8, device="cuda:0")
    assert _noalloc(db, d_sel, stride, q, d_out) == _native.PIR_E_INVAL
    assert b"fixed scratch" in pir.lib().pir_last_error()
    # the allocating entry point serves the same call
    db.dpxor_batch_async(d_sel, q, d_out, sel_stride=stride)
    torch.cuda.synchronize()
    assert not d_out.cpu().numpy().any()
    db.free()
