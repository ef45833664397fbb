"""GPU parity of the DPF evaluation (IM-PIR Sec. 3.2, eq. 1-3) and of the
key-to-answer path, through the C ABI, against the oracle.

Small domains are compared bit for bit over the whole domain, both for keys
from Gen and for keys whose codewords are arbitrary random blocks (eq. 3 for
any C0, C1); large domains on sampled leaves the oracle evaluates one by
one, plus the point-function identity over every leaf.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pir = pytest.importorskip("paper_2509_06514_amd")

pytestmark = pytest.mark.gpu

SENTINEL = 0x5A5A5A5A


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pir.Context(0)
    yield c
    c.close()


def _roots(seed):
    b = synth.stream_bytes(seed, 32)
    return b[:16], b[16:]


def _random_keys(n, count, seed):
    return synth.stream_bytes(seed, count * pir.dpf_key_bytes(n)).reshape(count, -1)


def _eval(ctx, keys, n, n_leaves, stride_words=None):
    keys = np.ascontiguousarray(keys, dtype=np.uint8).reshape(keys.shape[0], -1)
    words = (n_leaves + 31) // 32
    stride_words = stride_words or words
    d_keys = torch.from_numpy(keys).to("cuda:0")
    d_sel = torch.full((keys.shape[0], stride_words), SENTINEL, dtype=torch.int32, device="cuda:0")
    ctx.dpf_eval_async(d_keys, n, keys.shape[0], n_leaves, d_sel, sel_stride=4 * stride_words)
    torch.cuda.synchronize()
    return d_sel.cpu().numpy().view(np.uint32)


def _bits(words_row, count):
    return np.unpackbits(words_row.view(np.uint8), bitorder="little")[:count]


def _oracle_bits(key, n, count):
    full = np.unpackbits(oracle.dpf_eval_full(key, n), bitorder="little")
    out = np.zeros(count, np.uint8)
    m = min(count, 1 << n)
    out[:m] = full[:m]
    return out


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6, 7, 9, 12, 14, 15, 16])  # 15, 16: ten top levels in one launch
def test_eval_full_domain_matches_oracle(ctx, n):
    # two Gen keys and two keys with random codewords, whole domain
    r0, r1 = _roots(synth.S_KEY + n)
    alpha = (0x9E37 * (n + 1)) % (1 << n)
    k0, k1 = pir.dpf_gen(alpha, n, r0, r1)
    keys = np.stack([k0, k1, *_random_keys(n, 2, synth.S_KEY + 100 + n)])
    N = 1 << n
    got = _eval(ctx, keys, n, N)
    words = (N + 31) // 32
    for q in range(keys.shape[0]):
        assert np.array_equal(_bits(got[q], 32 * words), _oracle_bits(keys[q], n, 32 * words)), (n, q)
    x = _bits(got[0] ^ got[1], N)
    assert x.sum() == 1 and x[alpha] == 1


@pytest.mark.parametrize("n,n_leaves", [(10, 1000), (11, 1025), (13, 5000), (6, 33), (5, 7), (17, 100003)])
def test_eval_ragged_leaf_count(ctx, n, n_leaves):
    # words [0, ceil(n_leaves/32)) are written, the padding of the row is not touched
    keys = _random_keys(n, 3, synth.S_KEY + 200 + n)
    words = (n_leaves + 31) // 32
    got = _eval(ctx, keys, n, n_leaves, stride_words=words + 5)
    for q in range(3):
        want = _oracle_bits(keys[q], n, 32 * words)
        assert np.array_equal(_bits(got[q][:words], 32 * words), want), (n, n_leaves, q)
        assert (got[q][words:] == SENTINEL).all()


def test_eval_batch_rows_equal_single_key(ctx):
    # the launch chain depends on the number of keys; the rows may not
    n = 18
    keys = _random_keys(n, 37, synth.S_KEY + 300)
    batch = _eval(ctx, keys, n, 1 << n, stride_words=(1 << n) // 32 + 64)
    for q in (0, 17, 36):
        single = _eval(ctx, keys[q:q + 1], n, 1 << n)
        assert np.array_equal(batch[q][: (1 << n) // 32], single[0]), q
    rng = np.random.default_rng(5)
    for q in (0, 36):
        for j in rng.integers(0, 1 << n, 64):
            assert _bits(batch[q], 1 << n)[j] == oracle.dpf_eval_bit(keys[q], n, int(j))


@pytest.mark.parametrize("n", [22, 28])
def test_eval_point_function_large_domain(ctx, n):
    # Eval(k0) XOR Eval(k1) is the indicator of alpha over all 2^n leaves;
    # sampled leaves of each key against the oracle
    rng = np.random.default_rng(n)
    alphas = [0, (1 << n) - 1, int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))]
    keys = []
    for i, a in enumerate(alphas):
        k0, k1 = pir.dpf_gen(a, n, *_roots(synth.S_KEY + 400 + 8 * n + i))
        keys += [k0, k1]
    keys = np.stack(keys)
    d_keys = torch.from_numpy(keys).to("cuda:0")
    words = (1 << n) // 32
    d_sel = torch.zeros((len(keys), words), dtype=torch.int32, device="cuda:0")
    ctx.dpf_eval_async(d_keys, n, len(keys), 1 << n, d_sel)
    torch.cuda.synchronize()
    for i, a in enumerate(alphas):
        x = d_sel[2 * i] ^ d_sel[2 * i + 1]
        nz = torch.nonzero(x).flatten().cpu().numpy()
        assert list(nz) == [a // 32], (n, a, nz[:8])
        assert (int(x[a // 32].item()) & 0xFFFFFFFF) == 1 << (a % 32)
    host = d_sel.cpu().numpy().view(np.uint32)
    for q in range(len(keys)):
        js = list(rng.integers(0, 1 << n, 24)) + [alphas[q // 2]]
        for j in js:
            j = int(j)
            bit = (int(host[q][j >> 5]) >> (j & 31)) & 1
            assert bit == oracle.dpf_eval_bit(keys[q], n, j), (n, q, j)


def _load(ctx, n, r, seed):
    dbh = synth.database(n, r, seed=seed)
    return dbh, ctx.load_db(dbh)


@pytest.mark.parametrize("N,R", [(3000, 32), (1 << 12, 8), (777, 256), (1, 32), (70001, 13), (5000, 1000),
                                 (33, 3)])
def test_dpf_dpxor_two_server(ctx, N, R):
    # ans(k0) XOR ans(k1) = D[alpha]; ans(k0) = oracle scan of oracle-evaluated bits
    dbh, db = _load(ctx, N, R, synth.S_DB + 50 + R)
    n = pir.dpf_domain_bits(N)
    rng = np.random.default_rng(N)
    alphas = [int(a) for a in rng.integers(0, N, 6)] + [0, N - 1]
    k0s, k1s = [], []
    for i, a in enumerate(alphas):
        k0, k1 = pir.dpf_gen(a, n, *_roots(synth.S_KEY + 600 + i))
        k0s.append(k0)
        k1s.append(k1)
    keys = np.stack(k0s + k1s)
    d_keys = torch.from_numpy(keys).to("cuda:0")
    d_out = torch.empty((len(keys), R), dtype=torch.uint8, device="cuda:0")
    d_out.fill_(0xEE)
    db.dpf_dpxor_async(d_keys, len(keys), d_out)
    torch.cuda.synchronize()
    ans = d_out.cpu().numpy()
    m = len(alphas)
    for i, a in enumerate(alphas):
        assert np.array_equal(ans[i] ^ ans[m + i], dbh[a]), (N, R, a)
    for i in (0, m):
        sel = np.packbits(_oracle_bits(keys[i], n, N), bitorder="little")
        assert np.array_equal(ans[i], oracle.dpxor(dbh, sel)), i
    db.free()


def test_dpf_dpxor_large_in_key_groups(ctx):
    # 2^22 records x 32 B, 8 keys (4 pairs), in two calls with different key
    # counts: the same rows, and each pair reconstructs its record
    N, R = 1 << 22, 32
    dbh, db = _load(ctx, N, R, synth.S_DB + 57)
    n = pir.dpf_domain_bits(N)
    alphas = [0, N - 1, 123457, 3 * N // 4]
    ks = [pir.dpf_gen(a, n, *_roots(synth.S_KEY + 700 + i)) for i, a in enumerate(alphas)]
    keys = np.stack([k[0] for k in ks] + [k[1] for k in ks])
    d_keys = torch.from_numpy(keys).to("cuda:0")
    full = torch.full((8, R), 0xEE, dtype=torch.uint8, device="cuda:0")
    part = torch.full((3, R), 0x11, dtype=torch.uint8, device="cuda:0")
    db.dpf_dpxor_async(d_keys, 8, full)
    db.dpf_dpxor_async(d_keys, 3, part)
    torch.cuda.synchronize()
    ans = full.cpu().numpy()
    assert np.array_equal(part.cpu().numpy(), ans[:3])
    for i, al in enumerate(alphas):
        assert np.array_equal(ans[i] ^ ans[4 + i], dbh[al]), al
    db.free()


def test_dpf_eval_rejects_bad_arguments(ctx):
    n = 8
    keys = torch.zeros((2, pir.dpf_key_bytes(n)), dtype=torch.uint8, device="cuda:0")
    sel = torch.zeros((2, 8), dtype=torch.int32, device="cuda:0")
    lib = pir.lib()
    h = ctx.handle
    kp, sp = keys.data_ptr(), sel.data_ptr()
    E = pir._native.PIR_E_INVAL
    assert lib.pir_dpf_eval_async(h, kp, n, 2, 257, sp, 32, None) == E       # n_leaves > 2^n
    assert lib.pir_dpf_eval_async(h, kp, n, 2, 256, sp, 30, None) == E       # stride too small
    assert lib.pir_dpf_eval_async(h, kp, n, 0, 256, sp, 32, None) == E       # no keys
    assert lib.pir_dpf_eval_async(h, kp + 4, n, 1, 256, sp, 32, None) == E   # misaligned keys
    assert lib.pir_dpf_eval_async(h, kp, 37, 1, 256, sp, 32, None) == E      # domain too large
    assert lib.pir_dpf_eval_async(h, kp, n, 1, 0, sp, 32, None) == E         # no leaves
