"""Build libpir.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2509_06514_amd.build
"""
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpir.so")
ARCH = "gfx950"

SOURCES = ["pir_kernels.hip", "pir_dpf.hip", "pir_fp.hip", "pir_probe.hip", "pir_noalloc.hip",
           "pir_runtime.cpp", "pir_dpf_api.cpp", "pir_fp_api.cpp", "pir_serve.cpp"]

# Sources whose matrix-core accumulators may live in the accumulation
# registers (AGPRs); everywhere else they live in ordinary VGPRs (no AGPR
# copies per step).
AGPR_SOURCES = set()
VGPR_FORM = ["-mllvm", "-amdgpu-mfma-vgpr-form"]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    # packed fp32 VALU forms are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}",
    f"-I{CSRC}",
]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def build(verbose=False):
    """Compile every HIP/C++ source and link libpir.so (always rebuilds)."""
    hipcc = _hipcc()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        flags = HIPCC_FLAGS if src in AGPR_SOURCES else HIPCC_FLAGS + VGPR_FORM
        cmd = [hipcc, *flags, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature flag: harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
        if lines and (verbose or p.returncode):
            print("\n".join(lines), file=sys.stderr)
        if p.returncode:
            failed.append(src)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-pthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t = time.time()
    build(verbose="-v" in sys.argv)
    print(f"built {LIB} in {time.time() - t:.1f}s")
