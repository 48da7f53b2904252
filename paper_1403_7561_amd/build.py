"""Builds the HIP library in place: ``python -m paper_1403_7561_amd.build``.

Every HIP source is compiled for gfx950 with hipcc into
``paper_1403_7561_amd/libqe.so`` (the C ABI declared in include/qe.h).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqe.so")
SOURCES = ["qe_kernels.hip", "qe_sheets.hip", "qe_runtime.hip", "qe_batch.hip", "qe_schrod.hip", "qe_seq.hip", "qe_mg.hip"]
ARCH = os.environ.get("QE_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


LIBS = []


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def build(verbose=False, out=None):
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    lib = out or LIB
    tmp = lib + ".tmp"
    extra = os.environ.get("QE_EXTRA_FLAGS", "").split()
    cmd = [hipcc(), *FLAGS, *extra, "-shared", "-o", tmp, *srcs, f"-I{os.path.join(ROOT, 'include')}", *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines()
            if ln.strip() and "packed-fp32-ops" not in ln and "unknown target feature" not in ln]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
