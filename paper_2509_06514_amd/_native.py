"""ctypes declarations for libpir.so (the C ABI in include/pir.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any call.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpir.so")

PIR_OK = 0
PIR_E_INVAL = -1
PIR_E_NOMEM = -2
PIR_E_DEVICE = -3
PIR_E_BUSY = -4
PIR_E_NOTFOUND = -5
PIR_E_SHUTDOWN = -6
PIR_E_TIMEOUT = -7

STATUS_NAMES = {
    PIR_OK: "PIR_OK", PIR_E_INVAL: "PIR_E_INVAL", PIR_E_NOMEM: "PIR_E_NOMEM",
    PIR_E_DEVICE: "PIR_E_DEVICE", PIR_E_BUSY: "PIR_E_BUSY", PIR_E_NOTFOUND: "PIR_E_NOTFOUND",
    PIR_E_SHUTDOWN: "PIR_E_SHUTDOWN", PIR_E_TIMEOUT: "PIR_E_TIMEOUT",
}

PIR_MAX_BATCH = 4096
PIR_VARIANT_AUTO = 0
PIR_VARIANT_VALU = 1
PIR_VARIANT_MFMA_I8 = 2
PIR_VARIANT_MFMA_F4 = 3


class pir_db_info(ctypes.Structure):
    _fields_ = [("n_records", ctypes.c_uint64), ("record_bytes", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("n_blocks", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("sel_words", ctypes.c_uint64)]


class pir_kernel_cfg(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_uint32), ("q_tile", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32), ("groups", ctypes.c_uint32)]


class pir_timing(ctypes.Structure):
    _fields_ = [("stage1_launches", ctypes.c_uint64), ("stage1_ms", ctypes.c_double),
                ("stage2_launches", ctypes.c_uint64), ("stage2_ms", ctypes.c_double),
                ("dpf_evals", ctypes.c_uint64), ("dpf_ms", ctypes.c_double),
                ("fp_launches", ctypes.c_uint64), ("fp_ms", ctypes.c_double)]


class pir_serve_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("q_max", ctypes.c_uint32),
                ("max_wait_us", ctypes.c_uint32), ("n_slots", ctypes.c_uint32),
                ("queue_cap", ctypes.c_uint32), ("submit_wait_ms", ctypes.c_uint32),
                ("ring_bytes", ctypes.c_uint64)]


class pir_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("elapsed_s", ctypes.c_double), ("qps", ctypes.c_double),
                ("batch_hist", ctypes.c_uint64 * 13), ("h2d_bytes", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint32), ("n_slots", ctypes.c_uint32),
                ("key_requests", ctypes.c_uint64), ("updates_applied", ctypes.c_uint64),
                ("blocked_submits", ctypes.c_uint64)]


PIR_NOALLOC_SCRATCH_BYTES = 32 << 20  # fixed scratch of pir_dpxor_batch_async_noalloc, per device

_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32
_I = ctypes.c_int

# name -> (restype, argtypes); every function declared in include/pir.h
SIGNATURES = {
    "pir_last_error": (ctypes.c_char_p, []),
    "pir_version": (ctypes.c_char_p, []),
    "pir_ctx_create": (_I, [_I, _PP]),
    "pir_ctx_destroy": (_I, [_P]),
    "pir_db_load": (_I, [_P, _P, _U64, _U32, _PP]),
    "pir_db_update": (_I, [_P, _U64, _U64, _P]),
    "pir_db_read": (_I, [_P, _U64, _U64, _P]),
    "pir_db_free": (_I, [_P]),
    "pir_db_get_info": (_I, [_P, ctypes.POINTER(pir_db_info)]),
    "pir_db_min_sel_stride": (_U64, [_P]),
    "pir_dpxor": (_I, [_P, _P, _P]),
    "pir_dpxor_batch": (_I, [_P, _P, _U64, _U32, _P]),
    "pir_dpxor_batch_async": (_I, [_P, _P, _U64, _U32, _P, _P]),
    "pir_dpxor_batch_async_cfg": (_I, [_P, _P, _U64, _U32, _P, _P, ctypes.POINTER(pir_kernel_cfg)]),
    "pir_dpxor_batch_async_noalloc": (_I, [_P, _P, _U64, _U32, _P, _P]),
    "pir_get_cfg": (_I, [_P, _U32, ctypes.POINTER(pir_kernel_cfg)]),
    "pir_tune": (_I, [_P, _U32, ctypes.POINTER(pir_kernel_cfg)]),
    "pir_graphs_enable": (_I, [_P, _I]),
    "pir_timing_enable": (_I, [_P, _I]),
    "pir_timing_read": (_I, [_P, ctypes.POINTER(pir_timing), _I]),
    "pir_serve_create": (_I, [_P, ctypes.POINTER(pir_serve_config), _PP]),
    "pir_serve_add_db": (_I, [_P, _P, ctypes.POINTER(_U32)]),
    "pir_serve_submit": (_I, [_P, _U32, _P, _P, ctypes.POINTER(_U64)]),
    "pir_serve_submit_key": (_I, [_P, _U32, _P, _P, ctypes.POINTER(_U64)]),
    "pir_serve_update": (_I, [_P, _U32, _U64, _U64, _P, ctypes.POINTER(_U64)]),
    "pir_serve_wait": (_I, [_P, _U64, _I]),
    "pir_serve_poll": (_I, [_P, _U64, ctypes.POINTER(_I)]),
    "pir_serve_stats_get": (_I, [_P, ctypes.POINTER(pir_serve_stats), _I]),
    "pir_serve_destroy": (_I, [_P]),
    "pir_dpf_key_bytes": (_U64, [_U32]),
    "pir_dpf_domain_bits": (_U32, [_U64]),
    "pir_dpf_gen": (_I, [_U64, _U32, _P, _P, _P, _P]),
    "pir_dpf_eval_async": (_I, [_P, _P, _U32, _U32, _U64, _P, _U64, _P]),
    "pir_dpf_dpxor_async": (_I, [_P, _P, _U32, _P, _P]),
    "pir_reconstruct": (_I, [_P, _P, _U64, _P]),
    "pir_fp_db_load": (_I, [_P, _P, _U64, _U32, _U32, _PP]),
    "pir_fp_db_free": (_I, [_P]),
    "pir_fp_db_read": (_I, [_P, _U64, _U64, _P]),
    "pir_fp_min_v_stride": (_U64, [_P]),
    "pir_fp_v_stride": (_U64, [_P]),
    "pir_fp_inner_async": (_I, [_P, _P, _U64, _U32, _P, _P]),
    "pir_fp_inner": (_I, [_P, _P, _U64, _U32, _P]),
    "pir_read_probe_async": (_I, [_P, _P, _U64, _U32, _U32, _P, _P]),
    "pir_host_alloc": (_P, [ctypes.c_size_t]),
    "pir_host_free": (None, [_P]),
}

_lib = None


def lib():
    """The loaded libpir.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2509_06514_amd.build` "
                "(there is no CPU fallback)")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


class PirError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().pir_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, where):
    if code != PIR_OK:
        raise PirError(code, where)
    return code
