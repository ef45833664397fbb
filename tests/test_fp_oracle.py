"""Pins for the F_p inner-product oracle: r[l] = (sum_j v[j] * D[j][l]) mod p
(IM-PIR Sec. 2 states the database over F_p; its XOR form is p = 2).

Each pin is fixed by something other than the oracle's own formula: the
record a unit query must return, the two-server reconstruction from additive
shares of a unit vector, the XOR oracle at p = 2, and an int64 matrix product
by numpy (a library primitive) with the reduction applied afterwards.
"""
import numpy as np
import pytest

import oracle
import synth

PRIMES = [2, 3, 5, 101, 127]


def _db(n, L, p, seed):
    return (synth.stream_bytes(seed, n * L).reshape(n, L) % p).astype(np.uint8)


def _query(n, p, seed):
    return (synth.stream_bytes(seed, n) % p).astype(np.uint8)


@pytest.mark.parametrize("p", PRIMES)
def test_unit_query_returns_the_record(p):
    n, L = 257, 13
    db = _db(n, L, p, synth.S_DB + p)
    for i in (0, 1, 100, n - 1):
        e = np.zeros(n, np.uint8)
        e[i] = 1
        assert np.array_equal(oracle.fp_inner(db, e, p), db[i])
        e[i] = 3 % p
        assert np.array_equal(oracle.fp_inner(db, e, p), (3 * db[i].astype(int)) % p)


@pytest.mark.parametrize("p", PRIMES)
def test_additive_shares_reconstruct(p):
    # two servers hold v1 and v2 = e_i - v1 (mod p): r1 + r2 = D[i] (mod p)
    n, L = 1000, 32
    db = _db(n, L, p, synth.S_DB + 10 + p)
    for k, i in enumerate((0, 517, n - 1)):
        v1 = _query(n, p, synth.S_SEL + 10 * p + k)
        e = np.zeros(n, np.int64)
        e[i] = 1
        v2 = ((e - v1.astype(np.int64)) % p).astype(np.uint8)
        r1, r2 = oracle.fp_inner(db, v1, p), oracle.fp_inner(db, v2, p)
        assert np.array_equal((r1.astype(int) + r2) % p, db[i])


def test_p2_equals_xor_oracle():
    # on 0/1 elements and 0/1 query values, the sum mod 2 of each byte is the XOR
    n, L = 3001, 24
    db = _db(n, L, 2, synth.S_DB + 30)
    v = _query(n, 2, synth.S_SEL + 30)
    bits = np.packbits(v, bitorder="little")
    assert np.array_equal(oracle.fp_inner(db, v, 2), oracle.dpxor(db, bits))


@pytest.mark.parametrize("p", PRIMES)
def test_matches_integer_matrix_product(p):
    rng = np.random.default_rng(p)
    for n, L in ((1, 1), (7, 3), (64, 16), (1000, 48)):
        db = rng.integers(0, p, (n, L), dtype=np.uint8)
        v = rng.integers(0, 128, n, dtype=np.uint8)  # values past p are integers too
        want = (v.astype(np.int64) @ db.astype(np.int64)) % p
        assert np.array_equal(oracle.fp_inner(db, v, p), want.astype(np.uint8))


def test_linearity():
    p, n, L = 127, 500, 9
    db = _db(n, L, p, synth.S_DB + 40)
    u, w = _query(n, p, synth.S_SEL + 41), _query(n, p, synth.S_SEL + 42)
    a, b = 5, 77
    comb = ((a * u.astype(int) + b * w.astype(int)) % p).astype(np.uint8)
    lhs = oracle.fp_inner(db, comb, p).astype(int)
    rhs = (a * oracle.fp_inner(db, u, p).astype(int) + b * oracle.fp_inner(db, w, p).astype(int)) % p
    assert np.array_equal(lhs, rhs)


def test_empty_query_and_large_sums():
    p, n, L = 127, 70000, 2
    db = np.full((n, L), 126, np.uint8)
    assert not oracle.fp_inner(db, np.zeros(n, np.uint8), p).any()
    # sums far past 2^31: 70000 * 127 * 126 = 1.12e9 per element, times 1 -> exact in 64 bits
    v = np.full(n, 127, np.uint8)
    assert np.array_equal(oracle.fp_inner(db, v, p), np.full(L, (n * 127 * 126) % p, np.uint8))
