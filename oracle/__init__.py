"""ORACLE for dpXOR -- test infrastructure only.

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
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpxor_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared"]
_lib = None


def build():
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC])
    os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        p, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
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


def reconstruct(r1, r2):
    """Client step of the two-server scheme: D[i] = r1 XOR r2."""
    r1, r2 = _u8(r1), _u8(r2)
    assert r1.shape == r2.shape
    out = np.empty_like(r1)
    _load().oracle_reconstruct(r1.ctypes.data, r2.ctypes.data, r1.size, out.ctypes.data)
    return out
