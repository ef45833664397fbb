"""ORACLE for dpXOR and the DPF step before it -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never does, and shares
no code with it.

``dpxor_oracle.c`` is the plain single-threaded definition of the server
subresult (IM-PIR Sec. 2 "Multi-Server PIR", the equation for r; Sec. 3.3
"Inner products and XORing operations"):  r = XOR_j v[j] * D[j].  Its pins
(tests/test_oracle.py): the paper's worked example of the two-server scheme
(Fig. 2 and its DPF restatement, fixture tests/golden/), brute force over all
selections of tiny databases against an integer-count formulation, the
two-server reconstruction identity, special cases and linearity.

``dpf_oracle.c`` is AES-128 (FIPS-197) and the DPF of IM-PIR Sec. 3.1-3.2
(eq. 1-3; key generation after Boyle-Gilboa-Ishai 2016).  Its pins
(tests/test_dpf_oracle.py): FIPS-197 and SP 800-38A known answers, the
S-box values FIPS-197 prints, and the point-function identity
Eval(k0, x) XOR Eval(k1, x) = [x = alpha] by brute force.

``fp_oracle.c`` is the inner product over F_p (IM-PIR Sec. 2 states D in
F_p^{N x L}; the implemented XOR form is p = 2 on bits):
r[l] = (sum_j v[j] * D[j][l]) mod p.  Its pins (tests/test_fp_oracle.py):
unit queries return the record, additive shares of a unit vector
reconstruct the record, p = 2 on 0/1 elements equals the XOR oracle, brute
force against an int64 matrix product, and linearity.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "dpxor_oracle.c"), os.path.join(_HERE, "dpf_oracle.c"),
         os.path.join(_HERE, "fp_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared"]
_lib = None


def build():
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *_SRCS])
    os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        stale = not os.path.exists(_LIB) or any(
            os.path.getmtime(_LIB) < os.path.getmtime(src) for src in _SRCS)
        if stale:
            build()
        lib = ctypes.CDLL(_LIB)
        p, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
        i32 = ctypes.c_int
        lib.oracle_aes_sbox.restype = ctypes.c_uint8
        lib.oracle_aes_sbox.argtypes = [ctypes.c_uint8]
        lib.oracle_aes128_encrypt.restype = None
        lib.oracle_aes128_encrypt.argtypes = [p, p, p]
        lib.oracle_dpf_key_bytes.restype = u64
        lib.oracle_dpf_key_bytes.argtypes = [i32]
        lib.oracle_dpf_eval_block.restype = None
        lib.oracle_dpf_eval_block.argtypes = [p, i32, u64, p]
        lib.oracle_dpf_eval_bit.restype = i32
        lib.oracle_dpf_eval_bit.argtypes = [p, i32, u64]
        lib.oracle_dpf_eval_full.restype = None
        lib.oracle_dpf_eval_full.argtypes = [p, i32, p]
        lib.oracle_dpf_gen.restype = None
        lib.oracle_dpf_gen.argtypes = [u64, i32, p, p, p, p]
        lib.oracle_fp_inner.restype = i32
        lib.oracle_fp_inner.argtypes = [p, u64, u32, p, u32, p]
        lib.oracle_dpxor.restype = None
        lib.oracle_dpxor.argtypes = [p, u64, u32, p, p]
        lib.oracle_dpxor_batch.restype = None
        lib.oracle_dpxor_batch.argtypes = [p, u64, u32, p, u64, u32, p]
        lib.oracle_reconstruct.restype = None
        lib.oracle_reconstruct.argtypes = [p, p, u32, p]
        _lib = lib
    return _lib


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a


def dpxor(db, sel, n_records=None):
    """Answer r for one selection vector.  db: (N, R) uint8; sel: packed bits."""
    db = _u8(db)
    n, r = db.shape
    if n_records is not None:
        assert n_records <= n
        n = n_records
    sel = _u8(sel).reshape(-1)
    assert sel.size >= (n + 7) // 8
    out = np.empty(r, dtype=np.uint8)
    _load().oracle_dpxor(db.ctypes.data, n, r, sel.ctypes.data, out.ctypes.data)
    return out


def dpxor_batch(db, sel_rows):
    """Answers for Q selection rows: sel_rows is (Q, stride) uint8."""
    db = _u8(db)
    n, r = db.shape
    sel_rows = _u8(sel_rows)
    q, stride = sel_rows.shape
    assert stride >= (n + 7) // 8
    out = np.empty((q, r), dtype=np.uint8)
    _load().oracle_dpxor_batch(db.ctypes.data, n, r, sel_rows.ctypes.data, stride, q,
                               out.ctypes.data)
    return out


def host_threads():
    """Host threads this process may run on (its CPU affinity set)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


def dpxor_rows(db, sel_rows, rows=None, threads=None):
    """Answers of the selection rows `rows` (default: all) of a (Q, stride) array,
    each computed by the single-threaded oracle; rows run on up to `threads` host
    threads at once (the C oracle releases the interpreter lock).  Returns a
    (len(rows), R) array in the order of `rows`."""
    import threading

    db = _u8(db)
    sel_rows = _u8(sel_rows)
    rows = list(range(sel_rows.shape[0])) if rows is None else list(rows)
    out = np.empty((len(rows), db.shape[1]), dtype=np.uint8)
    nxt = [0]
    lock = threading.Lock()

    def work():
        while True:
            with lock:
                k = nxt[0]
                nxt[0] += 1
            if k >= len(rows):
                return
            out[k] = dpxor(db, sel_rows[rows[k]])

    t = min(len(rows), threads or host_threads())
    ths = [threading.Thread(target=work) for _ in range(t)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    return out


def reconstruct(r1, r2):
    """Client step of the two-server scheme: D[i] = r1 XOR r2."""
    r1, r2 = _u8(r1), _u8(r2)
    assert r1.shape == r2.shape
    out = np.empty_like(r1)
    _load().oracle_reconstruct(r1.ctypes.data, r2.ctypes.data, r1.size, out.ctypes.data)
    return out


# ---------------------------------------------------------------- AES / DPF

def aes_sbox(x):
    return int(_load().oracle_aes_sbox(x))


def aes128_encrypt(key, block):
    key = _u8(key).reshape(-1)
    block = _u8(block).reshape(-1)
    assert key.size == 16 and block.size == 16
    out = np.empty(16, np.uint8)
    _load().oracle_aes128_encrypt(key.ctypes.data, block.ctypes.data, out.ctypes.data)
    return out


def dpf_key_bytes(n):
    return int(_load().oracle_dpf_key_bytes(n))


def dpf_gen(alpha, n, root0, root1):
    """Keys (k0, k1) of P_{alpha,1} over 2^n points; roots are 16 random bytes each."""
    kb = dpf_key_bytes(n)
    k0, k1 = np.zeros(kb, np.uint8), np.zeros(kb, np.uint8)
    r0, r1 = _u8(root0).reshape(-1), _u8(root1).reshape(-1)
    _load().oracle_dpf_gen(alpha, n, r0.ctypes.data, r1.ctypes.data, k0.ctypes.data, k1.ctypes.data)
    return k0, k1


def dpf_eval_block(key, n, j):
    out = np.empty(16, np.uint8)
    key = _u8(key)
    _load().oracle_dpf_eval_block(key.ctypes.data, n, j, out.ctypes.data)
    return out


def dpf_eval_bit(key, n, j):
    key = _u8(key)
    return int(_load().oracle_dpf_eval_bit(key.ctypes.data, n, j))


def dpf_eval_full(key, n):
    """Packed selection vector of 2^n bits (LSB first)."""
    key = _u8(key)
    out = np.zeros(((1 << n) + 7) // 8, np.uint8)
    _load().oracle_dpf_eval_full(key.ctypes.data, n, out.ctypes.data)
    return out


def fp_inner(db, v, p):
    """r[l] = (sum_j v[j] * db[j][l]) mod p for a (N, L) uint8 database and N query bytes."""
    db = np.ascontiguousarray(db, dtype=np.uint8)
    n, L = db.shape
    v = np.ascontiguousarray(np.asarray(v, dtype=np.uint8).reshape(-1)[:n])
    if v.size < n:
        raise ValueError("query shorter than N")
    out = np.zeros(L, np.uint8)
    if _load().oracle_fp_inner(db.ctypes.data, n, L, v.ctypes.data, p, out.ctypes.data) != 0:
        raise MemoryError("oracle_fp_inner")
    return out
