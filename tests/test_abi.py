"""The C-ABI library loads and exports every function include/pir.h declares.
No compute calls are made here (the CPU suite runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2509_06514_amd as pir
from paper_2509_06514_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "pir.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(pir_[a-z0-9_]+)\s*\(", text))


def test_library_exports_every_declared_function():
    lib = pir.lib()
    declared = _header_functions()
    assert len(declared) >= 25
    for name in declared:
        assert hasattr(lib, name), f"libpir.so does not export {name}"
    assert declared == set(_native.SIGNATURES), "binding table and header disagree"


def test_version_and_error_strings():
    lib = pir.lib()
    assert b"gfx950" in lib.pir_version()
    assert lib.pir_last_error() is not None


def test_null_arguments_rejected_without_device_work():
    lib = pir.lib()
    out = ctypes.c_void_p()
    assert lib.pir_db_load(None, None, 1, 1, ctypes.byref(out)) == _native.PIR_E_INVAL
    assert b"NULL" in lib.pir_last_error()
    assert lib.pir_dpxor(None, None, None) == _native.PIR_E_INVAL
    assert lib.pir_dpxor_batch(None, None, 0, 1, None) == _native.PIR_E_INVAL
    assert lib.pir_dpxor_batch_async(None, None, 0, 1, None, None) == _native.PIR_E_INVAL
    assert lib.pir_serve_create(None, None, ctypes.byref(out)) == _native.PIR_E_INVAL
    assert lib.pir_serve_submit(None, 0, None, None, None) == _native.PIR_E_INVAL
    assert lib.pir_db_min_sel_stride(None) == 0
    assert lib.pir_fp_min_v_stride(None) == 0
    assert lib.pir_fp_v_stride(None) == 0
    assert lib.pir_host_alloc(0) is None


def test_sel_stride_helper():
    assert pir.sel_stride_for(1) == 256
    assert pir.sel_stride_for(32 * 64) == 256
    assert pir.sel_stride_for(32 * 64 + 1) == 512
    assert pir.sel_stride_for(1 << 28, align=4) == (1 << 28) // 8


def _gpu_may_be_present():
    hvd = os.environ.get("HIP_VISIBLE_DEVICES")
    if hvd is not None and hvd.strip() in ("", "-1"):
        return False  # every device hidden
    return os.path.exists("/dev/kfd")


@pytest.mark.skipif(_gpu_may_be_present(),
                    reason="a GPU may be present; the no-device path is checked where there is none")
def test_no_device_fails_loudly():
    lib = pir.lib()
    h = ctypes.c_void_p()
    rc = lib.pir_ctx_create(0, ctypes.byref(h))
    assert rc == _native.PIR_E_DEVICE
    assert lib.pir_last_error()


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors have the size and field offsets of the C structs in
    # include/pir.h, as gcc lays them out
    import subprocess
    structs = {"pir_db_info": _native.pir_db_info, "pir_kernel_cfg": _native.pir_kernel_cfg,
               "pir_timing": _native.pir_timing, "pir_serve_config": _native.pir_serve_config,
               "pir_serve_stats": _native.pir_serve_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pir.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("  return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for name, cls in structs.items():
        assert got[(name, "sizeof")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
