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
