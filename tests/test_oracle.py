"""Pins for the CPU oracle against what the paper and the mathematics fix.

Each test would fail for a plausible mistake in the oracle: a dropped record
(first/last index), MSB-first instead of LSB-first selection bits, a
transposed database index, reading bits past N, or a non-zero empty sum.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def _pack(bits):
    bits = np.asarray(bits, dtype=np.uint8)
    return np.packbits(bits, bitorder="little")


def test_worked_example(golden):
    # IM-PIR Sec. 2 "Multi-Server PIR", Fig. 2 and its DPF restatement.
    g = golden("worked_example.txt")
    db = np.array(g["records"], dtype=np.uint8).reshape(-1, g["record_bytes"][0])
    r1 = oracle.dpxor(db, _pack(g["v1"]))
    r2 = oracle.dpxor(db, _pack(g["v2"]))
    assert r1.tolist() == g["r1"]
    assert r2.tolist() == g["r2"]
    rec = oracle.reconstruct(r1, r2)
    assert rec.tolist() == g["reconstructed"]
    i = g["target_index"][0]
    assert rec.tolist() == db[i].tolist()
    # v1 XOR v2 is the one-hot vector of the point function P_{i,1}
    onehot = [a ^ b for a, b in zip(g["v1"], g["v2"])]
    assert onehot == [1 if j == i else 0 for j in range(len(onehot))]


def _count_mod2(db, sel_bits):
    """Independent formulation: bit b of the answer is (sum_j v_j * bit_b(D[j])) mod 2."""
    dbits = np.unpackbits(db, axis=1, bitorder="little").astype(np.int64)  # (N, 8R)
    cnt = sel_bits.astype(np.int64) @ dbits                                 # (S, 8R)
    return np.packbits((cnt & 1).astype(np.uint8), axis=1, bitorder="little")


@pytest.mark.parametrize("n,r", [(1, 1), (5, 2), (8, 3), (11, 4), (12, 1), (12, 4)])
def test_brute_force_all_selections(n, r):
    db = synth.database(n, r, seed=0x51 + 7 * n + r)
    allsel = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.uint8)  # (2^n, n)
    rows = np.packbits(allsel, axis=1, bitorder="little")
    got = oracle.dpxor_batch(db, rows)
    want = _count_mod2(db, allsel)
    assert np.array_equal(got, want)


def test_two_server_reconstruction():
    # For random b1 and b2 = b1 XOR e_i: ans(b1) XOR ans(b2) = D[i] (Sec. 2;
    # the client step of Algorithm 1).
    n, r = 1000, 32
    db = synth.database(n, r, seed=0x77)
    b1 = synth.selections(n, 1, seed=0x78)[0]
    for i in synth.indices(n, 16, seed=0x79) + [0, n - 1]:
        b2 = b1.copy()
        b2[i >> 3] ^= 1 << (i & 7)
        rec = oracle.reconstruct(oracle.dpxor(db, b1), oracle.dpxor(db, b2))
        assert np.array_equal(rec, db[i])


def test_special_cases():
    n, r = 77, 5
    db = synth.database(n, r, seed=0x99)
    nb = (n + 7) // 8
    assert not oracle.dpxor(db, np.zeros(nb, np.uint8)).any()
    for i in (0, 1, 8, n - 1):
        e = np.zeros(nb, np.uint8)
        e[i >> 3] = 1 << (i & 7)
        assert np.array_equal(oracle.dpxor(db, e), db[i])
    ones = np.full(nb, 0xFF, np.uint8)           # bits past n are junk: ignored
    assert np.array_equal(oracle.dpxor(db, ones), np.bitwise_xor.reduce(db, axis=0))


def test_tail_bits_ignored():
    n, r = 45, 3
    db = synth.database(n, r, seed=5)
    clean = synth.selections(n, 4, seed=6, stride=12)
    junk = synth.selections(n, 4, seed=6, stride=12, tail_junk=True)
    assert not np.array_equal(clean, junk)
    assert np.array_equal(oracle.dpxor_batch(db, clean), oracle.dpxor_batch(db, junk))


def test_linearity_over_gf2():
    n, r = 300, 16
    db = synth.database(n, r, seed=11)
    a, b = synth.selections(n, 2, seed=12)
    lhs = oracle.dpxor(db, a ^ b)
    rhs = oracle.dpxor(db, a) ^ oracle.dpxor(db, b)
    assert np.array_equal(lhs, rhs)


def test_partition_identity():
    # Sec. 3.3: r = XOR_d s_d where s_d covers a contiguous chunk [dstart, dend].
    n, r = 1000, 8
    db = synth.database(n, r, seed=21)
    v = synth.selections(n, 1, seed=22)[0]
    bits = np.unpackbits(v, bitorder="little")[:n]
    acc = np.zeros(r, np.uint8)
    for start in range(0, n, 96):
        end = min(n, start + 96)
        acc ^= oracle.dpxor(db[start:end], _pack(bits[start:end]))
    assert np.array_equal(acc, oracle.dpxor(db, v))


def test_batch_rows_match_single():
    n, r, q = 129, 7, 5
    db = synth.database(n, r, seed=31)
    rows = synth.selections(n, q, seed=32, stride=20)
    out = oracle.dpxor_batch(db, rows)
    for i in range(q):
        assert np.array_equal(out[i], oracle.dpxor(db, rows[i]))
