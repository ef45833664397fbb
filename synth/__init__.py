"""Seeded synthetic inputs (database records, selection bitvectors).

Holds no retrieval arithmetic: it only produces bytes, from a counter-based
SplitMix64 stream (Steele, Lea & Flood 2014).  The C source ``synth.c`` states
the byte and bit order.  Both the CPU oracle tests and the GPU path take their
inputs from here, so neither side depends on the other.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

# Seeds per workload: database stream, selection streams, point-index stream,
# DPF key material (root seeds, random codewords).
S_DB = 0x1000
S_SEL = 0x2000
S_IDX = 0x3000
S_KEY = 0x4000


def build():
    """Compile libsynth.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, u32, i32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
        lib.synth_mix64.restype = u64
        lib.synth_mix64.argtypes = [u64]
        lib.synth_word.restype = u64
        lib.synth_word.argtypes = [u64, u64]
        lib.synth_sel_seed.restype = u64
        lib.synth_sel_seed.argtypes = [u64, u64]
        lib.synth_fill_bytes.restype = None
        lib.synth_fill_bytes.argtypes = [u64, u64, p, u64, i32]
        lib.synth_selections.restype = None
        lib.synth_selections.argtypes = [u64, u64, u32, u64, p, u64, i32, i32]
        _lib = lib
    return _lib


def _threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except Exception:
        return 4


def mix64(z):
    return int(_load().synth_mix64(z & MASK64))


def word(seed, k):
    """Output word k of the stream with the given seed."""
    return int(_load().synth_word(seed & MASK64, k))


def stream_bytes(seed, n, offset=0, out=None):
    """Bytes [offset, offset+n) of stream `seed` as a uint8 array."""
    if out is None:
        out = np.empty(n, dtype=np.uint8)
    assert out.dtype == np.uint8 and out.flags.c_contiguous and out.size >= n
    _load().synth_fill_bytes(seed & MASK64, offset, out.ctypes.data, n, _threads())
    return out


def database(n_records, record_bytes, seed=S_DB, out=None):
    """N x R uint8 records of uniform bytes: record j is bytes [jR, (j+1)R)."""
    total = n_records * record_bytes
    if out is None:
        out = np.empty((n_records, record_bytes), dtype=np.uint8)
    assert out.dtype == np.uint8 and out.flags.c_contiguous and out.size == total
    _load().synth_fill_bytes(seed & MASK64, 0, out.ctypes.data, total, _threads())
    return out


def sel_row_bytes(n_records, align=4):
    """Smallest row stride holding n_records bits, rounded up to `align` bytes."""
    nb = (n_records + 7) // 8
    return max(align, (nb + align - 1) // align * align)


def selections(n_records, q, seed=S_SEL, q0=0, stride=None, tail_junk=False, out=None):
    """Q packed selection bitvectors (Bernoulli(0.5) bits), rows `stride` bytes apart.

    Bit j of row i is (row[j >> 3] >> (j & 7)) & 1.  With tail_junk the bits
    past n_records and the padding bytes hold junk instead of zeros.
    """
    if stride is None:
        stride = sel_row_bytes(n_records)
    assert stride >= (n_records + 7) // 8
    if out is None:
        out = np.empty((q, stride), dtype=np.uint8)
    assert out.dtype == np.uint8 and out.flags.c_contiguous and out.size >= q * stride
    _load().synth_selections(seed & MASK64, q0, q, n_records, out.ctypes.data, stride,
                             1 if tail_junk else 0, _threads())
    return out


def indices(n_records, count, seed=S_IDX):
    """`count` record indices drawn from stream `seed` (word k mod N)."""
    return [word(seed, k) % n_records for k in range(count)]
