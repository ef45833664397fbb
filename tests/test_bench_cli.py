"""bench.py's host-side contract (no GPU): the one-GPU limit and the names it
reports for the kernel a plan launches."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import paper_2509_06514_amd as pir  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)


@pytest.mark.parametrize("cfg,r,q,name", [
    ((1, 1, 8, 0), 32, 1, "k_stage1_valu<1, 8, false>"),
    ((1, 8, 2, 0), 16, 8, "k_stage1_valu<8, 2, true>"),
    ((3, 64, 3, 0), 32, 64, "k_stage1_mfma_lds<4, true, 3>"),
    ((2, 16, 4, 0), 32, 16, "k_stage1_mfma_lds<1, false, 4>"),
    ((3, 64, 12, 0), 32, 64, "k_stage1_mfma_ks<2, 2>"),
    ((3, 64, 15, 0), 32, 64, "k_stage1_mfma_ksw<2>"),
    ((3, 64, 16, 0), 32, 64, "k_stage1_mfma_ksp<2>"),
    ((3, 64, 15, 0), 32, 512, "k_stage1_mfma_ksw<0>"),
    ((3, 64, 16, 0), 256, 256, "k_stage1_mfma_ksp<0>"),
    ((3, 64, 17, 0), 32, 64, "k_stage1_mfma_ksv<2>"),
    ((3, 64, 17, 0), 32, 512, "k_stage1_mfma_ksv<0>"),
    ((3, 64, 12, 0), 32, 65, "k_stage1_mfma_ks<2, 0>"),
])
def test_kernel_names_follow_the_plan(cfg, r, q, name):
    assert bench.kernel_name(pir.KernelCfg(*cfg), r, q) == name


def test_kernel_names_exist_in_the_source():
    src = open(os.path.join(ROOT, "paper_2509_06514_amd", "csrc", "pir_kernels.hip")).read()
    for kernel in ("k_stage1_valu", "k_stage1_mfma_lds", "k_stage1_mfma_ks", "k_stage1_mfma_ksw", "k_stage1_mfma_ksp",
                   "k_stage1_mfma_ksv"):
        assert f"\n{kernel}(" in src, kernel


def test_engine_clock_sampler_reads_the_starred_level(tmp_path, monkeypatch):
    # the serving sweep's optional clock samples come from sysfs pp_dpm_sclk,
    # whose current level carries a trailing '*'
    import threading
    f = tmp_path / "pp_dpm_sclk"
    f.write_text("S: 96Mhz\n0: 500Mhz\n1: 2243Mhz *\n2: 2400Mhz\n")
    import glob as glob_mod
    monkeypatch.setattr(glob_mod, "glob", lambda pattern: [str(f)])
    stop, out = threading.Event(), []
    th = threading.Thread(target=bench.sample_engine_clock, args=(0.001, stop, out))
    th.start()
    import time
    deadline = time.time() + 10
    while len(out) < 3 and time.time() < deadline:
        time.sleep(0.001)
    stop.set()
    th.join(timeout=10)
    assert not th.is_alive()
    assert set(out) == {2243}


def test_traffic_is_taken_only_for_the_profiled_kernel(monkeypatch):
    # roofline.traffic comes from the committed counter runs only for the
    # kernel instance and sources they were taken on; otherwise it is null
    import json
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_dpxor_n28r32.json")))
    n = 1 << 28
    ksv = pir.KernelCfg(3, 64, 17, 2048)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda *a: t["kernel_source_sha256_16"])
    assert bench.load_traffic(n, 32, 64, ksv) == t["q64"]["hbm_bytes_per_launch"]
    assert bench.load_traffic(n, 32, 64, pir.KernelCfg(3, 64, 16, 2048)) is None   # another kernel
    assert bench.load_traffic(n, 32, 512, ksv) is None                             # no counters at Q = 512
    monkeypatch.setattr(bench, "kernel_source_hash", lambda *a: "0" * 16)
    assert bench.load_traffic(n, 32, 64, ksv) is None                              # sources changed since
