"""Pins for the DPF oracle (the step before dpXOR): AES-128 known answers,
S-box values the standard prints, and the point-function identity."""
import os

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _kat():
    out = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "aes128_kat.txt")):
        line = line.split("#", 1)[0].strip()
        if line:
            k, v = (x.strip() for x in line.split("=", 1))
            out[k] = np.frombuffer(bytes.fromhex(v), np.uint8)
    return out


@pytest.mark.parametrize("name", ["fips197_B", "fips197_C1"])
def test_fips197_vectors(name):
    k = _kat()
    got = oracle.aes128_encrypt(k[name + "_key"], k[name + "_in"])
    assert got.tobytes().hex() == k[name + "_out"].tobytes().hex()


def test_sp800_38a_ecb_vectors():
    k = _kat()
    for i in (1, 2):
        got = oracle.aes128_encrypt(k["sp80038a_key"], k[f"sp80038a_in{i}"])
        assert np.array_equal(got, k[f"sp80038a_out{i}"])


def test_sbox_values_and_bijection():
    k = _kat()
    assert oracle.aes_sbox(0x53) == int(k["sbox_53"][0])
    assert oracle.aes_sbox(0x00) == int(k["sbox_00"][0])
    assert sorted(oracle.aes_sbox(x) for x in range(256)) == list(range(256))


def _roots(seed):
    b = synth.stream_bytes(seed, 32)
    return b[:16], b[16:]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_point_function_all_alpha(n):
    # Eval(k0, x) XOR Eval(k1, x) = [x = alpha] for every alpha and x
    for alpha in range(1 << n):
        r0, r1 = _roots(1000 * n + alpha)
        k0, k1 = oracle.dpf_gen(alpha, n, r0, r1)
        v0, v1 = oracle.dpf_eval_full(k0, n), oracle.dpf_eval_full(k1, n)
        bits = np.unpackbits(v0 ^ v1, bitorder="little")[: 1 << n]
        want = np.zeros(1 << n, np.uint8)
        want[alpha] = 1
        assert np.array_equal(bits, want), (n, alpha)


def test_off_path_leaves_equal_on_path_differs():
    # off the path to alpha both parties hold the same 128-bit node value
    n, alpha = 10, 0x2B5
    k0, k1 = oracle.dpf_gen(alpha, n, *_roots(7))
    for x in (0, 1, alpha - 1, alpha + 1, (1 << n) - 1, alpha ^ (1 << (n - 1))):
        assert np.array_equal(oracle.dpf_eval_block(k0, n, x), oracle.dpf_eval_block(k1, n, x))
    a, b = oracle.dpf_eval_block(k0, n, alpha), oracle.dpf_eval_block(k1, n, alpha)
    assert (a[0] ^ b[0]) & 1 == 1


def test_key_layout_and_share_density():
    # roots sit in C0[0][0] with the party index as low bit; C0 is zero elsewhere;
    # C1 is shared; each share alone looks like Bernoulli(1/2) bits
    n, alpha = 16, 12345
    k0, k1 = oracle.dpf_gen(alpha, n, *_roots(9))
    blocks = 2 * (n + 1)
    c0_0, c0_1 = k0[: blocks * 16], k1[: blocks * 16]
    assert c0_0[0] & 1 == 0 and c0_1[0] & 1 == 1
    assert not c0_0[16:].any() and not c0_1[16:].any()
    assert np.array_equal(k0[blocks * 16:], k1[blocks * 16:])
    v0 = oracle.dpf_eval_full(k0, n)
    frac = np.unpackbits(v0).mean()
    assert 0.48 < frac < 0.52


def _keysbox():
    out = []
    for line in open(os.path.join(ROOT, "tests", "golden", "aesavs_keysbox128.txt")):
        line = line.split("#", 1)[0].strip()
        if line:
            k, c = (x.strip() for x in line.split("=", 1))
            out.append((np.frombuffer(bytes.fromhex(k), np.uint8), np.frombuffer(bytes.fromhex(c), np.uint8)))
    return out


def test_aesavs_keysbox_vectors():
    z = np.zeros(16, np.uint8)
    for k, c in _keysbox():
        assert np.array_equal(oracle.aes128_encrypt(k, z), c)


def _blank_key(n):
    return np.zeros(oracle.dpf_key_bytes(n), np.uint8)


def _put(key, n, cw, x, d, block):
    o = ((2 * cw + x) * (n + 1) + d) * 16
    key[o:o + 16] = block


def test_eval_one_step_at_known_answers():
    # eq. 2-3 at n = 1, leaf 0: R(1, 0) = AES_{C0[0,0]}(0^128) XOR C_t[0][1],
    # t = bit 0 of the root; the AES value is a published known answer, the
    # codeword blocks are arbitrary
    cws = synth.stream_bytes(synth.S_KEY + 77, 4 * 16).reshape(4, 16)
    ts = set()
    for root, ct in _keysbox():
        key = _blank_key(1)
        _put(key, 1, 0, 0, 0, root)
        for i, (cw, x) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
            _put(key, 1, cw, x, 1, cws[i])
        t = int(root[0]) & 1
        ts.add(t)
        want = ct ^ cws[2 * t]  # C_t[0][1]
        assert np.array_equal(oracle.dpf_eval_block(key, 1, 0), want)
        assert oracle.dpf_eval_bit(key, 1, 0) == int(want[0]) & 1
    assert ts == {0, 1}


def test_eval_chain_through_known_answers():
    # n = 3, leaf 0: choose the correction words so that R(1, 0) and R(2, 0)
    # are themselves known-answer keys; then R(3, 0) is fixed by a third
    # known answer.  Pins that each node value keys the next PRF (eq. 3).
    ks = _keysbox()
    (k1, c1), (k2, c2), (k3, c3) = ks[0], ks[5], ks[9]
    n = 3
    key = _blank_key(n)
    _put(key, n, 0, 0, 0, k1)
    t1 = int(k1[0]) & 1
    _put(key, n, t1, 0, 1, c1 ^ k2)       # R(1,0) = c1 ^ (c1 ^ k2) = k2
    t2 = int(k2[0]) & 1
    _put(key, n, t2, 0, 2, c2 ^ k3)       # R(2,0) = k3
    t3 = int(k3[0]) & 1
    last = synth.stream_bytes(synth.S_KEY + 78, 16)
    _put(key, n, t3, 0, 3, last)
    assert np.array_equal(oracle.dpf_eval_block(key, n, 0), c3 ^ last)


def test_point_function_zero_and_large_domain():
    # n = 0: the two roots differ exactly in bit 0 (eq. 2)
    k0, k1 = oracle.dpf_gen(0, 0, *_roots(3))
    assert oracle.dpf_eval_bit(k0, 0, 0) ^ oracle.dpf_eval_bit(k1, 0, 0) == 1
    # n = 20: sampled leaves, alpha included
    n = 20
    rng = np.random.default_rng(20)
    for alpha in (0, (1 << n) - 1, int(rng.integers(0, 1 << n))):
        k0, k1 = oracle.dpf_gen(alpha, n, *_roots(4000 + alpha % 97))
        for x in [alpha] + [int(v) for v in rng.integers(0, 1 << n, 40)]:
            assert oracle.dpf_eval_bit(k0, n, x) ^ oracle.dpf_eval_bit(k1, n, x) == int(x == alpha), (alpha, x)
