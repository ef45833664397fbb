"""Seeded input generator: pinned to SplitMix64's published outputs and to the
stated byte/bit layout."""
import numpy as np

import synth

MASK = (1 << 64) - 1


def test_splitmix64_published_vector():
    # First outputs of SplitMix64 seeded with 1234567 (the test vector shipped
    # with the reference C implementation by Vigna, and Java's SplittableRandom).
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [synth.word(1234567, k) for k in range(5)] == want


def test_bytes_are_little_endian_words():
    seed = 0xDEADBEEF
    b = synth.stream_bytes(seed, 40)
    for k in range(5):
        assert int.from_bytes(bytes(b[8 * k:8 * k + 8]), "little") == synth.word(seed, k)


def test_offset_and_threads_consistent():
    seed = 77
    whole = synth.stream_bytes(seed, (1 << 23) + 13)
    part = synth.stream_bytes(seed, 1001, offset=12345)
    assert np.array_equal(whole[12345:12345 + 1001], part)
    # the multi-threaded fill (large n) equals the per-word definition
    for k in (0, 1, 777, 524288, (1 << 20) - 1):
        assert int.from_bytes(bytes(whole[8 * k:8 * k + 8]), "little") == synth.word(seed, k)


def test_every_thread_count_fills_every_byte():
    # The fill splits n bytes into word-aligned pieces, one per thread.  Here
    # floor(n / t) is a multiple of 8 while t does not divide n (t = 16), the
    # split that must still reach the last bytes; unwritten bytes would keep
    # the 0x5A the buffer starts with.
    seed, n = 91, 16 * (1 << 19) + 10
    lib = synth._load()
    want = np.full(n, 0x5A, np.uint8)
    lib.synth_fill_bytes(seed, 0, want.ctypes.data, n, 1)
    last = n // 8
    tail = synth.word(seed, last).to_bytes(8, "little")[: n - 8 * last]
    assert bytes(want[8 * last:]) == tail
    for t in (2, 3, 5, 7, 8, 12, 16, 64):
        got = np.full(n, 0x5A, np.uint8)
        lib.synth_fill_bytes(seed, 0, got.ctypes.data, n, t)
        assert np.array_equal(got, want), t


def test_selection_bit_layout():
    n, q, seed = 200, 3, 0x2001
    rows = synth.selections(n, q, seed=seed, stride=32)
    for i in range(q):
        s = synth.mix64(seed + i)
        for j in range(n):
            bit_row = (rows[i, j >> 3] >> (j & 7)) & 1
            bit_stream = (synth.word(s, j >> 6) >> (j & 63)) & 1
            assert bit_row == bit_stream
        assert not rows[i, (n + 7) // 8:].any()


def test_selection_tail_zero_and_junk():
    n = 13
    z = synth.selections(n, 1, stride=8)
    j = synth.selections(n, 1, stride=8, tail_junk=True)
    assert z[0, 1] >> 5 == 0 and not z[0, 2:].any()
    assert (j[0, 2:] == 0xA5).all()
    assert z[0, 0] == j[0, 0] and (z[0, 1] & 0x1F) == (j[0, 1] & 0x1F)


def test_bernoulli_half():
    rows = synth.selections(1 << 16, 2)
    frac = np.unpackbits(rows).mean()
    assert abs(frac - 0.5) < 0.01
    db = synth.database(1 << 12, 32)
    assert abs(db.mean() - 127.5) < 2.0
