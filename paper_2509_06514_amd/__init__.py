"""MI355X dpXOR: the server-side scan of DPF-based two-server PIR (IM-PIR).

A thin Python binding over libpir.so (include/pir.h).  Every step of the
scan runs in the library's HIP kernels; this module only marshals arguments.
torch supplies device buffers and streams for the asynchronous calls.
"""
import ctypes
import weakref

import numpy as np

from . import _native
from ._native import (PIR_MAX_BATCH, PIR_VARIANT_AUTO, PIR_VARIANT_MFMA_F4, PIR_VARIANT_MFMA_I8,
                      PIR_VARIANT_VALU, PirError, check, lib)

__all__ = ["Context", "Database", "FpDatabase", "Server", "KernelCfg", "PirError", "lib", "sel_stride_for",
           "dpf_key_bytes", "dpf_domain_bits", "dpf_gen", "reconstruct", "pinned_empty",
           "PIR_MAX_BATCH", "PIR_VARIANT_AUTO", "PIR_VARIANT_VALU", "PIR_VARIANT_MFMA_I8",
           "PIR_VARIANT_MFMA_F4"]


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _u8(a):
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), np.uint8).copy()
    a = np.asarray(a)
    if a.dtype != np.uint8:
        a = a.view(np.uint8) if a.dtype.itemsize == 1 else a.astype(np.uint8)
    return np.ascontiguousarray(a)


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class KernelCfg:
    """Explicit stage-1 configuration (variant, query tile, unroll, record groups)."""

    def __init__(self, variant=PIR_VARIANT_AUTO, q_tile=0, unroll=0, groups=0):
        self.variant, self.q_tile, self.unroll, self.groups = variant, q_tile, unroll, groups

    def _c(self):
        return _native.pir_kernel_cfg(self.variant, self.q_tile, self.unroll, self.groups)

    @classmethod
    def _from_c(cls, c):
        return cls(c.variant, c.q_tile, c.unroll, c.groups)

    def as_dict(self):
        return {"variant": self.variant, "q_tile": self.q_tile, "unroll": self.unroll,
                "groups": self.groups}

    def __repr__(self):
        return f"KernelCfg({self.as_dict()})"


def sel_stride_for(n_records, align=256):
    """Device selection-row pitch: whole 32-bit words for ceil(N/32) blocks, aligned."""
    words = (n_records + 31) // 32
    return (4 * words + align - 1) // align * align


def pinned_empty(shape, dtype=np.uint8):
    """A numpy array in pinned host memory (pir_host_alloc), freed with the array.

    The synchronous calls copy such buffers to and from the device without
    staging them.
    """
    dtype = np.dtype(dtype)
    count = int(np.prod(shape, dtype=np.int64))
    nbytes = max(count * dtype.itemsize, 1)
    p = lib().pir_host_alloc(nbytes)
    if not p:
        raise MemoryError(f"pir_host_alloc({nbytes}) failed")
    buf = (ctypes.c_uint8 * nbytes).from_address(p)
    weakref.finalize(buf, lib().pir_host_free, ctypes.c_void_p(p))
    return np.frombuffer(buf, dtype=dtype, count=count).reshape(shape)


def dpf_key_bytes(n):
    """Bytes of one DPF key over a 2^n domain: codewords C0, C1 of 2 x (n+1) 16-byte blocks."""
    return int(lib().pir_dpf_key_bytes(n))


def dpf_domain_bits(n_records):
    """Smallest n with 2^n >= n_records."""
    return int(lib().pir_dpf_domain_bits(n_records))


def reconstruct(ans0, ans1):
    """Client side: the record from the two servers' answers (XOR)."""
    a, b = _u8(ans0).reshape(-1), _u8(ans1).reshape(-1)
    if a.size != b.size:
        raise ValueError("answers differ in length")
    out = np.empty_like(a)
    check(lib().pir_reconstruct(_ptr(a), _ptr(b), a.size, _ptr(out)), "pir_reconstruct")
    return out


def dpf_gen(alpha, n, root0, root1):
    """Client-side key generation (host): the two parties' keys for the point at alpha.

    root0/root1: 16 random bytes each (bit 0 is replaced by the party index).
    """
    r0, r1 = _u8(root0).reshape(-1), _u8(root1).reshape(-1)
    if r0.size != 16 or r1.size != 16:
        raise ValueError("roots must be 16 bytes")
    kb = dpf_key_bytes(n)
    k0, k1 = np.empty(kb, np.uint8), np.empty(kb, np.uint8)
    check(lib().pir_dpf_gen(alpha, n, _ptr(r0), _ptr(r1), _ptr(k0), _ptr(k1)), "pir_dpf_gen")
    return k0, k1


class Context:
    """A device context (pir_ctx)."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        check(lib().pir_ctx_create(device, ctypes.byref(h)), "pir_ctx_create")
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def load_db(self, records, n_records=None):
        """Preload an (N, R) uint8 record array into HBM."""
        records = _u8(records)
        if records.ndim != 2:
            raise ValueError("records must be (N, R)")
        n, r = records.shape
        if n_records is not None:
            n = n_records
        h = ctypes.c_void_p()
        check(lib().pir_db_load(self._h, _ptr(records), n, r, ctypes.byref(h)), "pir_db_load")
        return Database(self, h)

    def graphs(self, on=True):
        """Replay the scan's launches from captured hipGraphs (default) or enqueue them one by one."""
        check(lib().pir_graphs_enable(self._h, 1 if on else 0), "pir_graphs_enable")

    def timing(self, on=True):
        check(lib().pir_timing_enable(self._h, 1 if on else 0), "pir_timing_enable")

    def timing_read(self, reset=True):
        t = _native.pir_timing()
        check(lib().pir_timing_read(self._h, ctypes.byref(t), 1 if reset else 0), "pir_timing_read")
        return {"stage1_launches": t.stage1_launches, "stage1_ms": t.stage1_ms,
                "stage2_launches": t.stage2_launches, "stage2_ms": t.stage2_ms,
                "dpf_evals": t.dpf_evals, "dpf_ms": t.dpf_ms,
                "fp_launches": t.fp_launches, "fp_ms": t.fp_ms}

    def load_fp_db(self, elements, p):
        """Load an (N, L) uint8 database over F_p (every element < p, 2 <= p <= 127)."""
        elements = _u8(elements)
        if elements.ndim != 2:
            raise ValueError("elements must be (N, L)")
        n, L = elements.shape
        h = ctypes.c_void_p()
        check(lib().pir_fp_db_load(self._h, _ptr(elements), n, L, p, ctypes.byref(h)), "pir_fp_db_load")
        return FpDatabase(self, h, n, L, p)

    def dpf_eval_async(self, d_keys, n, n_keys, n_leaves, d_sel, sel_stride=None, stream=None):
        """Full-domain DPF evaluation on the device (torch tensors), enqueued on `stream`.

        d_keys: n_keys consecutive keys of dpf_key_bytes(n) bytes; row q of d_sel
        (sel_stride bytes apart) receives the packed selection bits of key q.
        """
        if d_keys.device.type != "cuda" or d_sel.device.type != "cuda":
            raise ValueError("device tensors required")
        if d_keys.numel() * d_keys.element_size() < n_keys * dpf_key_bytes(n):
            raise ValueError("d_keys too small")
        words = (n_leaves + 31) // 32
        if sel_stride is None:
            sel_stride = d_sel.stride(0) * d_sel.element_size() if d_sel.dim() == 2 else 4 * words
        if d_sel.numel() * d_sel.element_size() < (n_keys - 1) * sel_stride + 4 * words:
            raise ValueError("d_sel too small")
        check(lib().pir_dpf_eval_async(self._h, ctypes.c_void_p(d_keys.data_ptr()), n, n_keys, n_leaves,
                                       ctypes.c_void_p(d_sel.data_ptr()), sel_stride, _stream_handle(stream)),
              "pir_dpf_eval_async")

    def read_probe_async(self, d_src, d_sink, unroll=8, workgroups=4096, stream=None):
        """Streaming-read probe over a device tensor (every 16-byte chunk read once);
        d_sink receives one 16-byte XOR word per workgroup."""
        nbytes = d_src.numel() * d_src.element_size()
        if d_src.device.type != "cuda" or d_sink.device.type != "cuda":
            raise ValueError("device tensors required")
        if d_sink.numel() * d_sink.element_size() < 16 * workgroups:
            raise ValueError("d_sink too small")
        check(lib().pir_read_probe_async(self._h, ctypes.c_void_p(d_src.data_ptr()), nbytes, unroll, workgroups,
                                         ctypes.c_void_p(d_sink.data_ptr()), _stream_handle(stream)),
              "pir_read_probe_async")

    def close(self):
        if self._h:
            check(lib().pir_ctx_destroy(self._h), "pir_ctx_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Database:
    """A resident database (pir_db)."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self._h = handle
        info = _native.pir_db_info()
        check(lib().pir_db_get_info(handle, ctypes.byref(info)), "pir_db_get_info")
        self.n_records = info.n_records
        self.record_bytes = info.record_bytes
        self.n_blocks = info.n_blocks
        self.device_bytes = info.device_bytes
        self.min_sel_stride = lib().pir_db_min_sel_stride(handle)

    @property
    def handle(self):
        return self._h

    @property
    def sel_row_bytes(self):
        return (self.n_records + 7) // 8

    def _host_out(self, out, shape):
        if out is None:
            return np.empty(shape, np.uint8)
        if out.dtype != np.uint8 or out.shape != shape or not out.flags.c_contiguous:
            raise ValueError(f"out must be a C-contiguous uint8 array of shape {shape}")
        return out

    def dpxor(self, sel, out=None):
        """One query, host in/out: sel packed bits (>= ceil(N/8) bytes) -> R-byte answer.

        Arrays from pinned_empty (for sel and out) skip the library's staging copies.
        """
        sel = _u8(sel).reshape(-1)
        if sel.size < self.sel_row_bytes:
            raise ValueError("selection shorter than ceil(N/8) bytes")
        out = self._host_out(out, (self.record_bytes,))
        check(lib().pir_dpxor(self._h, _ptr(sel), _ptr(out)), "pir_dpxor")
        return out

    def dpxor_batch(self, sel_rows, out=None):
        """Q queries, host in/out: sel_rows (Q, stride) uint8 -> (Q, R) answers.

        Arrays from pinned_empty (for sel_rows and out) skip the library's staging copies.
        """
        sel_rows = _u8(sel_rows)
        q, stride = sel_rows.shape
        if stride < self.sel_row_bytes:
            raise ValueError("selection rows shorter than ceil(N/8) bytes")
        out = self._host_out(out, (q, self.record_bytes))
        check(lib().pir_dpxor_batch(self._h, _ptr(sel_rows), stride, q, _ptr(out)), "pir_dpxor_batch")
        return out

    def dpxor_batch_async(self, d_sel, q, d_out, sel_stride=None, stream=None, cfg=None):
        """Q queries on device buffers (torch tensors), enqueued on `stream`.

        d_sel: q rows of sel_stride bytes (a multiple of 4, >= min_sel_stride);
        d_out: q*R bytes.
        """
        if sel_stride is None:
            sel_stride = d_sel.stride(0) * d_sel.element_size() if d_sel.dim() == 2 else self.min_sel_stride
        if d_sel.device.type != "cuda" or d_out.device.type != "cuda":
            raise ValueError("device tensors required")
        if d_sel.numel() * d_sel.element_size() < (q - 1) * sel_stride + self.min_sel_stride:
            raise ValueError("d_sel too small")
        if d_out.numel() * d_out.element_size() < q * self.record_bytes:
            raise ValueError("d_out too small")
        s = _stream_handle(stream)
        if cfg is None:
            rc = lib().pir_dpxor_batch_async(self._h, ctypes.c_void_p(d_sel.data_ptr()), sel_stride, q,
                                             ctypes.c_void_p(d_out.data_ptr()), s)
        else:
            c = cfg._c()
            rc = lib().pir_dpxor_batch_async_cfg(self._h, ctypes.c_void_p(d_sel.data_ptr()), sel_stride, q,
                                                 ctypes.c_void_p(d_out.data_ptr()), s, ctypes.byref(c))
        check(rc, "pir_dpxor_batch_async")

    def dpxor_batch_async_noalloc(self, d_sel, q, d_out, sel_stride=None, stream=None):
        """As dpxor_batch_async, with the partial answers in the library's fixed
        per-device scratch (no allocation; calls that overlap on one GPU race)."""
        if sel_stride is None:
            sel_stride = d_sel.stride(0) * d_sel.element_size() if d_sel.dim() == 2 else self.min_sel_stride
        if d_sel.device.type != "cuda" or d_out.device.type != "cuda":
            raise ValueError("device tensors required")
        if d_sel.numel() * d_sel.element_size() < (q - 1) * sel_stride + self.min_sel_stride:
            raise ValueError("d_sel too small")
        if d_out.numel() * d_out.element_size() < q * self.record_bytes:
            raise ValueError("d_out too small")
        check(lib().pir_dpxor_batch_async_noalloc(self._h, ctypes.c_void_p(d_sel.data_ptr()), sel_stride, q,
                                                  ctypes.c_void_p(d_out.data_ptr()), _stream_handle(stream)),
              "pir_dpxor_batch_async_noalloc")

    def dpf_dpxor_async(self, d_keys, n_keys, d_out, stream=None):
        """Answers from DPF keys: row q of d_out = XOR_j Eval(k_q, j) * D[j] (device tensors)."""
        n = dpf_domain_bits(self.n_records)
        if d_keys.device.type != "cuda" or d_out.device.type != "cuda":
            raise ValueError("device tensors required")
        if d_keys.numel() * d_keys.element_size() < n_keys * dpf_key_bytes(n):
            raise ValueError("d_keys too small")
        if d_out.numel() * d_out.element_size() < n_keys * self.record_bytes:
            raise ValueError("d_out too small")
        check(lib().pir_dpf_dpxor_async(self._h, ctypes.c_void_p(d_keys.data_ptr()), n_keys,
                                        ctypes.c_void_p(d_out.data_ptr()), _stream_handle(stream)),
              "pir_dpf_dpxor_async")

    def get_cfg(self, q):
        c = _native.pir_kernel_cfg()
        check(lib().pir_get_cfg(self._h, q, ctypes.byref(c)), "pir_get_cfg")
        return KernelCfg._from_c(c)

    def tune(self, q):
        c = _native.pir_kernel_cfg()
        check(lib().pir_tune(self._h, q, ctypes.byref(c)), "pir_tune")
        return KernelCfg._from_c(c)

    def update(self, first, records):
        records = _u8(records)
        n = records.shape[0]
        check(lib().pir_db_update(self._h, first, n, _ptr(records)), "pir_db_update")

    def read(self, first, count):
        out = np.empty((count, self.record_bytes), np.uint8)
        check(lib().pir_db_read(self._h, first, count, _ptr(out)), "pir_db_read")
        return out

    def free(self):
        if self._h:
            check(lib().pir_db_free(self._h), "pir_db_free")
            self._h = None


class FpDatabase:
    """A resident database over F_p (pir_fpdb): answers r_q = (v_q . D) mod p."""

    def __init__(self, ctx, handle, n_records, record_elems, p):
        self.ctx = ctx
        self._h = handle
        self.n_records, self.record_elems, self.p = n_records, record_elems, p
        self.min_v_stride = lib().pir_fp_min_v_stride(handle)
        self.v_stride = lib().pir_fp_v_stride(handle)  # recommended row pitch (odd multiple of 128)

    @property
    def handle(self):
        return self._h

    def inner(self, v_rows, out=None):
        """Q queries, host in/out: v_rows (Q, >= N) uint8 (< 128) -> (Q, L) answers.

        Arrays from pinned_empty (for v_rows and out) skip the library's staging copies.
        """
        v_rows = _u8(v_rows)
        if v_rows.ndim == 1:
            v_rows = v_rows.reshape(1, -1)
        q, stride = v_rows.shape
        shape = (q, self.record_elems)
        if out is None:
            out = np.empty(shape, np.uint8)
        elif out.dtype != np.uint8 or out.shape != shape or not out.flags.c_contiguous:
            raise ValueError(f"out must be a C-contiguous uint8 array of shape {shape}")
        check(lib().pir_fp_inner(self._h, _ptr(v_rows), stride, q, _ptr(out)), "pir_fp_inner")
        return out

    def inner_async(self, d_v, q, d_out, v_stride=None, stream=None):
        """Q queries on device buffers (torch tensors) on `stream`; rows v_stride bytes apart."""
        if v_stride is None:
            v_stride = d_v.stride(0) * d_v.element_size() if d_v.dim() == 2 else self.min_v_stride
        if d_v.device.type != "cuda" or d_out.device.type != "cuda":
            raise ValueError("device tensors required")
        if d_v.numel() * d_v.element_size() < (q - 1) * v_stride + self.min_v_stride:
            raise ValueError("d_v too small")
        if d_out.numel() * d_out.element_size() < q * self.record_elems:
            raise ValueError("d_out too small")
        check(lib().pir_fp_inner_async(self._h, ctypes.c_void_p(d_v.data_ptr()), v_stride, q,
                                       ctypes.c_void_p(d_out.data_ptr()), _stream_handle(stream)),
              "pir_fp_inner_async")

    def read(self, first, count):
        out = np.empty((count, self.record_elems), np.uint8)
        check(lib().pir_fp_db_read(self._h, first, count, _ptr(out)), "pir_fp_db_read")
        return out

    def free(self):
        if self._h:
            check(lib().pir_fp_db_free(self._h), "pir_fp_db_free")
            self._h = None


class Server:
    """Continuous-batching server (pir_server)."""

    def __init__(self, ctx, hbm_budget_bytes=0, q_max=64, max_wait_us=0, n_slots=4, queue_cap=0,
                 submit_wait_ms=0, ring_bytes=0):
        cfg = _native.pir_serve_config(hbm_budget_bytes, q_max, max_wait_us, n_slots, queue_cap, submit_wait_ms,
                                       ring_bytes)
        h = ctypes.c_void_p()
        check(lib().pir_serve_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), "pir_serve_create")
        self._h = h
        self._dbs = {}

    def add_db(self, db):
        i = ctypes.c_uint32()
        check(lib().pir_serve_add_db(self._h, db.handle, ctypes.byref(i)), "pir_serve_add_db")
        self._dbs[i.value] = db
        return i.value

    def submit(self, db_id, sel, out):
        """Queue a query; `out` (R-byte uint8 array) is filled on completion."""
        sel = _u8(sel)
        t = ctypes.c_uint64()
        check(lib().pir_serve_submit(self._h, db_id, _ptr(sel), _ptr(out), ctypes.byref(t)),
              "pir_serve_submit")
        return t.value

    def submit_key(self, db_id, key, out):
        """Queue a query as a DPF key (the server evaluates it); `out` is filled on completion."""
        key = _u8(key).reshape(-1)
        n = dpf_domain_bits(self._dbs[db_id].n_records)
        if key.size < dpf_key_bytes(n):
            raise ValueError("key shorter than pir_dpf_key_bytes(n)")
        t = ctypes.c_uint64()
        check(lib().pir_serve_submit_key(self._h, db_id, _ptr(key), _ptr(out), ctypes.byref(t)),
              "pir_serve_submit_key")
        return t.value

    def update(self, db_id, first, records):
        """Queue a record update, ordered with the database's requests; returns its ticket."""
        records = _u8(records)
        t = ctypes.c_uint64()
        check(lib().pir_serve_update(self._h, db_id, first, records.shape[0], _ptr(records), ctypes.byref(t)),
              "pir_serve_update")
        return t.value

    def submit_key_raw(self, db_id, key_ptr, out_ptr):
        t = ctypes.c_uint64()
        rc = lib().pir_serve_submit_key(self._h, db_id, ctypes.c_void_p(key_ptr), ctypes.c_void_p(out_ptr),
                                        ctypes.byref(t))
        return rc, t.value

    def submit_raw(self, db_id, sel_ptr, out_ptr):
        t = ctypes.c_uint64()
        rc = lib().pir_serve_submit(self._h, db_id, ctypes.c_void_p(sel_ptr), ctypes.c_void_p(out_ptr),
                                    ctypes.byref(t))
        return rc, t.value

    def wait(self, ticket, timeout_ms=-1):
        return lib().pir_serve_wait(self._h, ticket, timeout_ms)

    def poll(self, ticket):
        st = ctypes.c_int()
        r = lib().pir_serve_poll(self._h, ticket, ctypes.byref(st))
        if r < 0:
            check(r, "pir_serve_poll")
        return (r == 1), st.value

    def stats(self, reset=False):
        s = _native.pir_serve_stats()
        check(lib().pir_serve_stats_get(self._h, ctypes.byref(s), 1 if reset else 0), "pir_serve_stats_get")
        d = {k: getattr(s, k) for k, _ in s._fields_ if k != "batch_hist"}
        d["batch_hist"] = list(s.batch_hist)
        return d

    def close(self):
        if self._h:
            check(lib().pir_serve_destroy(self._h), "pir_serve_destroy")
            self._h = None
