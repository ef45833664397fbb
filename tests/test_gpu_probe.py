"""The streaming-read probe (the measured HBM read roof) reads every 16-byte
chunk of its buffer exactly once: the XOR of its per-workgroup words equals
the XOR of all chunks, for every unroll and ragged workgroup counts."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pir = pytest.importorskip("paper_2509_06514_amd")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 1008, 1 << 20, (3 << 20) + 4080])
def test_read_probe_folds_every_chunk_once(nbytes):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    host = synth.stream_bytes(0x9E0B + nbytes, nbytes)
    want = np.bitwise_xor.reduce(host.view(np.uint32).reshape(-1, 4), axis=0)
    ctx = pir.Context(0)
    try:
        d_src = torch.from_numpy(host).to("cuda:0")
        for unroll in (4, 8, 16):
            for wgs in (1, 3, 257, 4096):
                sink = torch.full((wgs, 4), -1, dtype=torch.int32, device="cuda:0")
                ctx.read_probe_async(d_src, sink, unroll=unroll, workgroups=wgs)
                torch.cuda.synchronize()
                got = sink.cpu().numpy().view(np.uint32)
                chunks = nbytes // 16
                per = -(-chunks // wgs)
                used = -(-chunks // per)  # workgroups launched (each takes `per` chunks)
                assert np.array_equal(np.bitwise_xor.reduce(got[:used], axis=0), want), (unroll, wgs)
    finally:
        ctx.close()
